"""GPU checks against facts that hold without any reference implementation:
the closed form on a fully stored exact rank-R tensor, and invariants of
MTTKRP (Eq. 1) under scaling, mode relabelling and linear combinations of the
values.  Integer-valued data keeps every fp32 sum exact in any order, so the
invariants are asserted bit for bit."""
import numpy as np
import pytest

from gpu_util import dev_factors, hip_mttkrp, log

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2507_15121_amd import api, synth  # noqa: E402


@pytest.mark.parametrize("dims,rank", [((64, 48, 40), 16), ((30, 20, 12, 10), 8)])
def test_closed_form_on_fully_stored_rank_r_tensor(dims, rank):
    """X = sum_r a_r o b_r o ... stored entry by entry: MTTKRP_d(X) equals
    A_d times the Hadamard product of the other factors' Gram matrices (the
    Khatri-Rao Gram identity), computed here in fp64."""
    rng = np.random.default_rng(len(dims))
    A = [rng.uniform(-1, 1, (d, rank)).astype(np.float32) for d in dims]
    A64 = [a.astype(np.float64) for a in A]
    X = np.zeros(dims)
    for r in range(rank):
        t = np.array(1.0)
        for a in A64:
            t = np.multiply.outer(t, a[:, r])
        X += t
    idx = np.array(np.unravel_index(np.arange(X.size), dims), dtype=np.int32)
    val = X.ravel().astype(np.float32)
    t = api.Tensor(idx, val, dims)
    dfac = dev_factors(A)
    for d in range(len(dims)):
        H = np.ones((rank, rank))
        for w in range(len(dims)):
            if w != d:
                H *= A64[w].T @ A64[w]
        ref = A64[d] @ H
        got = hip_mttkrp(t, d, dfac)
        # val is X rounded to fp32 (relative 6e-8), then fp32 products and sums
        e = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        log("closed form order %d mode %d rel %.2e" % (len(dims), d, e))
        assert e <= 1e-5
    t.close()


def _int_tensor(seed, dims=(3000, 1500, 700), nnz=40000, rank=32):
    rng = np.random.default_rng(seed)
    st = synth.tensor(dims, nnz, "zipf", 1.2, 0.05, seed=seed)
    val = rng.integers(1, 5, size=st.nnz).astype(np.float32)
    F = [rng.integers(-2, 3, size=(d, rank)).astype(np.float32) for d in dims]
    return st.idx, val, dims, F, rng


def test_power_of_two_scaling_is_exact():
    idx, val, dims, F, _ = _int_tensor(1)
    t = api.Tensor(idx, val, dims, chunk_nnz=64)
    base = [hip_mttkrp(t, d, dev_factors(F)) for d in range(3)]
    G = [f.copy() for f in F]
    G[1] *= 8.0
    scaled = [hip_mttkrp(t, d, dev_factors(G)) for d in range(3)]
    for d in (0, 2):
        np.testing.assert_array_equal(scaled[d], 8.0 * base[d])
    np.testing.assert_array_equal(scaled[1], base[1])   # mode 1 does not read its own factor
    t.close()


def test_mode_relabelling_permutes_outputs():
    idx, val, dims, F, _ = _int_tensor(2)
    perm = (2, 0, 1)                                    # new mode j is old mode perm[j]
    t = api.Tensor(idx, val, dims, chunk_nnz=128)
    tp = api.Tensor(idx[list(perm)], val, tuple(dims[p] for p in perm), chunk_nnz=128)
    out = [hip_mttkrp(t, d, dev_factors(F)) for d in range(3)]
    Fp = [F[p] for p in perm]
    for j in range(3):
        np.testing.assert_array_equal(hip_mttkrp(tp, j, dev_factors(Fp)), out[perm[j]])
    t.close()
    tp.close()


def test_linearity_in_the_values():
    idx, val, dims, F, rng = _int_tensor(3)
    val2 = rng.integers(-3, 4, size=val.size).astype(np.float32)
    comb = (2.0 * val - 3.0 * val2).astype(np.float32)
    outs = []
    for v in (val, val2, comb):
        t = api.Tensor(idx, v, dims, chunk_nnz=256)
        outs.append([hip_mttkrp(t, d, dev_factors(F)) for d in range(3)])
        t.close()
    for d in range(3):
        np.testing.assert_array_equal(outs[2][d], 2.0 * outs[0][d] - 3.0 * outs[1][d])
