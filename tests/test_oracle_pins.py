"""Pins for the CPU oracle: facts fixed by the paper and by the mathematics.

The oracle is checked against things other than itself: a hand-worked EC
example, explicit unfolding times explicit Khatri-Rao products in both column
conventions, the Gram closed form of a fully stored exact rank-R tensor, the
order-2 reduction to a sparse-dense matrix product, invariants, central finite
differences of the loss, and a brute-force sort for the layout order.
"""
import itertools
import os

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _random_sparse(rng, dims, nnz, distinct=True):
    total = int(np.prod(dims))
    if distinct:
        lin = rng.choice(total, size=nnz, replace=False)
    else:
        lin = rng.integers(0, total, size=nnz)
    idx = np.stack(np.unravel_index(lin, dims)).astype(np.int32)
    val = rng.uniform(-1, 1, size=nnz)
    return idx, val


def _factors(rng, dims, R):
    return [rng.uniform(-1, 1, size=(d, R)) for d in dims]


def _read_golden(name):
    rec = {"nz": []}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            key, *vals = line.split()
            nums = [float(v) for v in vals]
            if key == "nz":
                rec["nz"].append(nums)
            else:
                rec[key] = nums
    return rec


def test_worked_example_golden():
    g = _read_golden("ec_worked_example.txt")
    dims = [int(x) for x in g["dims"]]
    R = int(g["rank"][0])
    nz = np.array(g["nz"])
    idx = nz[:, :3].T.astype(np.int32)
    val = nz[:, 3]
    A = [np.array(g["factor%d" % w]).reshape(dims[w], R) for w in range(3)]
    for d in range(3):
        Y = oracle.mttkrp(idx, val, dims, A, d)
        np.testing.assert_array_equal(Y, np.array(g["mttkrp%d" % d]).reshape(dims[d], R))
    loss, _ = oracle.cp_loss(idx, val, A)
    assert loss == g["loss"][0]
    G0 = oracle.cp_grad(idx, val, dims, A, 0)
    np.testing.assert_array_equal(G0, np.array(g["grad0"]).reshape(dims[0], R))


@pytest.mark.parametrize("dims,nnz", [((5, 4, 3), 23), ((4, 3, 3, 2), 31), ((3, 2, 2, 2, 3), 40)])
@pytest.mark.parametrize("convention", ["first_fastest", "cyclic"])
def test_brute_force_unfold_times_khatri_rao(dims, nnz, convention):
    rng = np.random.default_rng(11)
    idx, val = _random_sparse(rng, dims, nnz)
    A = _factors(rng, dims, 3)
    X = oracle.to_dense(idx, val, dims)
    for d in range(len(dims)):
        ref = oracle.mttkrp_dense(X, A, d, convention)
        got = oracle.mttkrp(idx, val, dims, A, d)
        assert np.max(np.abs(got - ref)) <= 1e-12 * max(1.0, np.max(np.abs(ref)))


def test_cyclic_pairing_matches_eq1_for_order3():
    # Eq. 1 pairs X_(0) with B kr C, X_(1) with C kr A, X_(2) with A kr B.
    rng = np.random.default_rng(3)
    dims = (4, 5, 3)
    idx, val = _random_sparse(rng, dims, 30)
    A, B, C = _factors(rng, dims, 2)
    X = oracle.to_dense(idx, val, dims)
    pairs = [(B, C), (C, A), (A, B)]
    for d in range(3):
        ref = oracle.unfold(X, d, "cyclic") @ oracle.khatri_rao(list(pairs[d]))
        np.testing.assert_allclose(oracle.mttkrp(idx, val, dims, [A, B, C], d), ref,
                                   rtol=0, atol=1e-12)


def test_khatri_rao_column_is_kronecker():
    rng = np.random.default_rng(5)
    B = rng.normal(size=(3, 4))
    C = rng.normal(size=(5, 4))
    K = oracle.khatri_rao([B, C])
    for r in range(4):
        np.testing.assert_allclose(K[:, r], np.kron(B[:, r], C[:, r]), rtol=0, atol=1e-14)


@pytest.mark.parametrize("dims,R", [((9, 7, 5), 4), ((6, 5, 4, 3), 3)])
def test_closed_form_full_exact_rank_R(dims, R):
    # X = [[A_0, ..., A_{N-1}]] stored densely as a "sparse" tensor with every
    # entry a nonzero.  Then MTTKRP_d = A_d * (Hadamard of A_w^T A_w, w != d),
    # by the Khatri-Rao Gram identity.
    rng = np.random.default_rng(7)
    A = _factors(rng, dims, R)
    lin = np.arange(int(np.prod(dims)))
    idx = np.stack(np.unravel_index(lin, dims)).astype(np.int32)
    val = np.zeros(lin.size)
    for r in range(R):
        prod = np.ones(lin.size)
        for w in range(len(dims)):
            prod = prod * A[w][idx[w], r]
        val = val + prod
    for d in range(len(dims)):
        gram = np.ones((R, R))
        for w in range(len(dims)):
            if w != d:
                gram = gram * (A[w].T @ A[w])
        ref = A[d] @ gram
        np.testing.assert_allclose(oracle.mttkrp(idx, val, dims, A, d), ref, rtol=1e-11, atol=1e-11)
    # The CP model at every entry reproduces the stored values exactly enough.
    loss, _ = oracle.cp_loss(idx, val, A)
    assert loss < 1e-24 * lin.size


def test_order2_is_spmm():
    rng = np.random.default_rng(9)
    dims = (13, 11)
    idx, val = _random_sparse(rng, dims, 40)
    A = _factors(rng, dims, 5)
    X = oracle.to_dense(idx, val, dims)
    np.testing.assert_allclose(oracle.mttkrp(idx, val, dims, A, 0), X @ A[1], rtol=0, atol=1e-13)
    np.testing.assert_allclose(oracle.mttkrp(idx, val, dims, A, 1), X.T @ A[0], rtol=0, atol=1e-13)


def test_single_nonzero_and_empty():
    rng = np.random.default_rng(1)
    dims = (6, 5, 4)
    A = _factors(rng, dims, 3)
    idx = np.array([[2], [4], [1]], dtype=np.int32)
    val = np.array([1.5])
    Y = oracle.mttkrp(idx, val, dims, A, 1)
    ref = np.zeros((5, 3))
    ref[4] = 1.5 * A[0][2] * A[2][1]
    np.testing.assert_array_equal(Y, ref)
    empty = np.zeros((3, 0), dtype=np.int32)
    for d in range(3):
        assert not oracle.mttkrp(empty, np.zeros(0), dims, A, d).any()


def test_invariants_linearity_permutation_relabel_scaling():
    rng = np.random.default_rng(21)
    dims = (7, 6, 5, 4)
    idx, val = _random_sparse(rng, dims, 60)
    val2 = rng.uniform(-1, 1, size=val.size)
    A = _factors(rng, dims, 4)
    for d in range(4):
        Y1 = oracle.mttkrp(idx, val, dims, A, d)
        Y2 = oracle.mttkrp(idx, val2, dims, A, d)
        np.testing.assert_allclose(oracle.mttkrp(idx, 2 * val - 3 * val2, dims, A, d),
                                   2 * Y1 - 3 * Y2, rtol=0, atol=1e-13)
        p = rng.permutation(val.size)
        np.testing.assert_allclose(oracle.mttkrp(idx[:, p], val[p], dims, A, d), Y1,
                                   rtol=0, atol=1e-13)
    # relabelling modes permutes outputs
    sigma = [2, 0, 3, 1]
    idx_s = idx[sigma]
    dims_s = [dims[s] for s in sigma]
    A_s = [A[s] for s in sigma]
    for d in range(4):
        np.testing.assert_allclose(oracle.mttkrp(idx_s, val, dims_s, A_s, d),
                                   oracle.mttkrp(idx, val, dims, A, sigma[d]), rtol=0, atol=1e-13)
    # scaling factor w by 2^3 scales every other mode's output by exactly 2^3
    # and leaves mode w's own output unchanged
    A8 = list(A)
    A8[1] = A[1] * 8.0
    for d in range(4):
        Y = oracle.mttkrp(idx, val, dims, A, d)
        Ys = oracle.mttkrp(idx, val, dims, A8, d)
        np.testing.assert_array_equal(Ys, Y if d == 1 else 8.0 * Y)


def test_duplicates_add_up():
    rng = np.random.default_rng(4)
    dims = (4, 4, 4)
    A = _factors(rng, dims, 2)
    idx = np.array([[1, 1], [2, 2], [3, 3]], dtype=np.int32)
    val = np.array([0.25, 0.5])
    Y = oracle.mttkrp(idx, val, dims, A, 0)
    Y1 = oracle.mttkrp(idx[:, :1], np.array([0.75]), dims, A, 0)
    np.testing.assert_allclose(Y, Y1, rtol=0, atol=1e-15)


def test_gradient_central_differences():
    # L(A) = sum (x - CP(A))^2; dL/dA_d from the oracle against central
    # differences of the float64 loss.
    rng = np.random.default_rng(13)
    dims = (6, 5, 4, 3)
    R = 3
    idx, val = _random_sparse(rng, dims, 50)
    A = _factors(rng, dims, R)
    h = 1e-6
    for d in range(4):
        G = oracle.cp_grad(idx, val, dims, A, d)
        fd = np.zeros_like(A[d])
        for i in range(dims[d]):
            for r in range(R):
                Ap = [a.copy() for a in A]
                Am = [a.copy() for a in A]
                Ap[d][i, r] += h
                Am[d][i, r] -= h
                fd[i, r] = (oracle.cp_loss(idx, val, Ap)[0] - oracle.cp_loss(idx, val, Am)[0]) / (2 * h)
        assert oracle.rel_fro(G, fd) < 1e-6


def test_zero_residual_gives_zero_loss_and_gradient():
    rng = np.random.default_rng(17)
    dims = (8, 6, 5)
    idx, _ = _random_sparse(rng, dims, 70)
    A = _factors(rng, dims, 4)
    val = oracle.cp_model(idx, A)
    loss, resid = oracle.cp_loss(idx, val, A)
    assert loss == 0.0 and not resid.any()
    for d in range(3):
        assert not oracle.cp_grad(idx, val, dims, A, d).any()


def test_cp_model_brute_force():
    rng = np.random.default_rng(19)
    dims = (4, 3, 5)
    idx, _ = _random_sparse(rng, dims, 12)
    A = _factors(rng, dims, 3)
    full = np.einsum("ir,jr,kr->ijk", *A)
    np.testing.assert_allclose(oracle.cp_model(idx, A), full[tuple(idx.astype(np.int64))],
                               rtol=0, atol=1e-14)


# ---------------------------------------------------------------- layout oracle

@pytest.mark.parametrize("ch", [1, 7, 64, 4096])
def test_layout_oracle_matches_brute_force_sort(ch):
    rng = np.random.default_rng(23)
    dims = (6, 5, 7, 3)
    nnz = 300
    idx = np.stack([rng.integers(0, d, size=nnz) for d in dims]).astype(np.int32)  # duplicates
    for mode in range(4):
        lay = oracle.layout(idx, mode, ch)
        others = [w for w in range(4) if w != mode]
        key = lambda k: (idx[mode, k],) + tuple(idx[w, k] for w in others) + (k,)
        expect = sorted(range(nnz), key=key)  # input position breaks ties -> stable
        np.testing.assert_array_equal(lay["perm"], expect)
        np.testing.assert_array_equal(lay["out_idx"], idx[mode][expect])
        assert np.all(np.diff(lay["out_idx"].astype(np.int64)) >= 0)
        n_chunks = -(-nnz // ch)
        assert lay["n_chunks"] == n_chunks
        for k in range(n_chunks):
            s, e = k * ch, min(k * ch + ch, nnz)
            o = lay["out_idx"]
            head = k > 0 and o[s - 1] == o[s]
            tail = e < nnz and o[e - 1] == o[e]
            assert lay["flags"][k] == (int(head) | (int(tail) << 1))


def test_layout_oracle_mode0_of_lexicographic_input_is_identity():
    rng = np.random.default_rng(29)
    dims = (5, 5, 5)
    lin = np.sort(rng.choice(125, size=40, replace=False))
    idx = np.stack(np.unravel_index(lin, dims)).astype(np.int32)
    lay = oracle.layout(idx, 0, 8)
    np.testing.assert_array_equal(lay["perm"], np.arange(40))


# ---------------------------------------------------------------- bfloat16 RNE

def test_bf16_rne_known_bit_patterns():
    cases = {
        0x3F800000: 0x3F80,   # 1.0
        0x3F808000: 0x3F80,   # tie, even stays
        0x3F818000: 0x3F82,   # tie, odd rounds up
        0x3F808001: 0x3F81,   # just above half
        0x3F807FFF: 0x3F80,   # just below half
        0xBF818000: 0xBF82,   # negative tie, odd
        0x00000000: 0x0000,
        0x80000000: 0x8000,
        0x7F7FFFFF: 0x7F80,   # largest float rounds to +inf in bf16
    }
    x = np.array(list(cases.keys()), dtype=np.uint32).view(np.float32)
    np.testing.assert_array_equal(oracle.bf16_rne(x), np.array(list(cases.values()), dtype=np.uint16))


def test_bf16_rne_matches_torch_cpu_cast():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(31)
    x = (2 * rng.random(100000, dtype=np.float32) - 1)
    t = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    np.testing.assert_array_equal(oracle.bf16_rne(x), t)


def test_rel_fro_definition():
    a = np.array([[3.0, 4.0]])
    assert oracle.rel_fro(a, a) == 0.0
    assert oracle.rel_fro(np.zeros((1, 2)), a) == 1.0
    assert oracle.rel_fro(np.zeros(3), np.zeros(3)) == 0.0
    assert oracle.rel_fro(np.ones(3), np.zeros(3)) == float("inf")
