"""GPU checks of the two forms beside plain fp32 MTTKRP: bf16 factor
gathers with fp32 accumulation, and the differentiable sparse CP loss with the
fused residual + MTTKRP backward."""
import numpy as np
import pytest

import oracle
from gpu_util import dev_factors, hip_mttkrp, log, oracle_mttkrp, rel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2507_15121_amd import api, synth  # noqa: E402
from paper_2507_15121_amd.autograd import SparseCPLoss, SparseCPLossFused, sparse_cp_loss  # noqa: E402


# ------------------------------------------------------------------ bfloat16

@pytest.mark.parametrize("rank", [32, 64, 128, 5, 40, 16, 8])
def test_bf16_factors(rank):
    """16 and 32: 8-byte lanes (rows of up to 64 bytes); 64 and 128: 16-byte
    lanes; 5, 8 and 40: the column-tile path."""
    dims = (20000, 5000, 3000)
    st = synth.tensor(dims, 80000, "zipf", 1.1, 0.05, seed=21)
    factors = synth.factors(dims, rank, seed=21)
    t = api.Tensor(st.idx, st.val, dims, chunk_nnz=512)
    dbf = dev_factors(factors, torch.bfloat16)
    for w, f in enumerate(factors):
        bits = dbf[w].view(torch.int16).cpu().numpy().view(np.uint16)
        np.testing.assert_array_equal(bits, oracle.bf16_rne(f))  # torch RNE == oracle RNE
    rounded = [oracle.bf16_to_f32(oracle.bf16_rne(f)) for f in factors]
    for d in range(3):
        got = hip_mttkrp(t, d, dbf, bf16=True)
        assert not np.isnan(got).any()
        e_round = rel(got, oracle_mttkrp(st.idx, st.val, dims, rounded, d))
        e_full = rel(got, oracle_mttkrp(st.idx, st.val, dims, factors, d))
        log("bf16 R=%d mode %d: vs rounded %.2e, vs fp32 factors %.2e" % (rank, d, e_round, e_full))
        assert e_round <= 1e-5   # fp32 accumulation kept
        assert e_full <= 1e-2    # bf16 gather error bar
    t.close()


@pytest.mark.parametrize("dims,rank", [((3000, 2000, 500, 100), 32), ((3000, 2000, 500, 100), 16),
                                       ((3000, 2000, 500, 100), 64), ((1500, 800, 300, 200, 100), 32)])
def test_bf16_factors_three_or_more_inputs(dims, rank):
    """Orders 4 and 5.  At rank 32 the 64-byte rows are gathered with 16-byte
    lanes (16 rows per instruction) when three or more factors are gathered;
    rank 16 keeps 8-byte lanes, rank 64 has 16-byte lanes anyway."""
    st = synth.tensor(dims, 60000, "zipf", 1.2, 0.05, seed=len(dims) * 100 + rank)
    factors = synth.factors(dims, rank, seed=rank)
    t = api.Tensor(st.idx, st.val, dims, chunk_nnz=256)
    dbf = dev_factors(factors, torch.bfloat16)
    rounded = [oracle.bf16_to_f32(oracle.bf16_rne(f)) for f in factors]
    for d in range(len(dims)):
        got = hip_mttkrp(t, d, dbf, bf16=True)
        assert not np.isnan(got).any()
        e_round = rel(got, oracle_mttkrp(st.idx, st.val, dims, rounded, d))
        e_full = rel(got, oracle_mttkrp(st.idx, st.val, dims, factors, d))
        log("bf16 order %d R=%d mode %d: vs rounded %.2e, vs fp32 factors %.2e" % (len(dims), rank, d, e_round, e_full))
        assert e_round <= 1e-5 and e_full <= 1e-2
    t.close()
    # integer inputs: every sum exact, so bit-equal to the oracle
    rng = np.random.default_rng(rank)
    val = rng.integers(1, 5, st.nnz).astype(np.float32)
    ifac = [rng.integers(-2, 3, (n, rank)).astype(np.float32) for n in dims]
    t = api.Tensor(st.idx, val, dims, chunk_nnz=64)
    dbi = dev_factors(ifac, torch.bfloat16)
    for d in range(len(dims)):
        np.testing.assert_array_equal(hip_mttkrp(t, d, dbi, bf16=True),
                                      oracle_mttkrp(st.idx, val, dims, ifac, d).astype(np.float32))
    t.close()


def test_bf16_integer_exact():
    rng = np.random.default_rng(3)
    dims = (3000, 1500, 700)
    st = synth.tensor(dims, 40000, "zipf", 1.2, 0.1, seed=3)
    val = rng.integers(1, 5, st.nnz).astype(np.float32)
    factors = [rng.integers(-2, 3, (d, 64)).astype(np.float32) for d in dims]
    t = api.Tensor(st.idx, val, dims, chunk_nnz=64)
    dbf = dev_factors(factors, torch.bfloat16)
    for d in range(3):
        np.testing.assert_array_equal(hip_mttkrp(t, d, dbf, bf16=True),
                                      oracle_mttkrp(st.idx, val, dims, factors, d).astype(np.float32))
    t.close()


# ------------------------------------------------------------ CP loss / grad

def _problem(dims, nnz, rank, seed, hot=0.0):
    st = synth.tensor(dims, nnz, "zipf", 1.2, hot, seed=seed)
    rng = np.random.default_rng(seed)
    factors = [(rng.uniform(-1, 1, (d, rank)) * 0.5).astype(np.float32) for d in dims]
    return st, factors


@pytest.mark.parametrize("dims,rank", [((3000, 2000, 500, 100), 32), ((2000, 1500, 800), 16),
                                       ((500, 400, 300), 64), ((400, 300, 200), 5)])
def test_cp_loss_and_grad_vs_oracle(dims, rank):
    st, factors = _problem(dims, 40000, rank, seed=rank, hot=0.05)
    t = api.Tensor(st.idx, st.val, dims, chunk_nnz=256)
    dfac = dev_factors(factors)
    loss = api.cp_loss(t, dfac)
    ref_loss, _ = oracle.cp_loss(st.idx, st.val, factors)
    log("loss %.9e ref %.9e" % (float(loss), ref_loss))
    assert abs(float(loss) - ref_loss) <= 1e-5 * abs(ref_loss)
    for d in range(len(dims)):
        g = api.cp_grad(t, d, dfac, -2.0 * 0.75).cpu().numpy()
        ref = oracle.cp_grad(st.idx, st.val, dims, factors, d, grad_out=0.75)
        e = rel(g, ref)
        log("  grad mode %d rel %.2e" % (d, e))
        assert e <= 1e-5
    t.close()


def test_autograd_function_matches_oracle_and_skips_unneeded_grads():
    dims = (2000, 1000, 300, 50)
    st, factors = _problem(dims, 30000, 32, seed=5)
    t = api.Tensor(st.idx, st.val, dims)
    dfac = [f.requires_grad_(w != 2) for w, f in enumerate(dev_factors(factors))]
    L = SparseCPLoss.apply(t, *dfac)
    assert L.dtype == torch.float64 and L.dim() == 0
    (3.0 * L).backward()
    assert dfac[2].grad is None
    for d in (0, 1, 3):
        ref = oracle.cp_grad(st.idx, st.val, dims, factors, d, grad_out=3.0)
        assert rel(dfac[d].grad.cpu().numpy(), ref) <= 1e-5
    t.close()


def test_zero_residual_gives_zero_loss_and_grad():
    dims = (500, 300, 200)
    rng = np.random.default_rng(7)
    idx, _ = synth.coords(dims, 20000, "zipf", 1.1, seed=7)
    factors = [rng.integers(-2, 3, (d, 16)).astype(np.float32) for d in dims]
    val = oracle.cp_model(idx, factors).astype(np.float32)  # exact small integers
    t = api.Tensor(idx, val, dims)
    dfac = dev_factors(factors)
    assert float(api.cp_loss(t, dfac)) == 0.0
    for d in range(3):
        assert not api.cp_grad(t, d, dfac, -2.0).cpu().numpy().any()
    t.close()


def test_directional_finite_difference():
    # [L(A + eps V) - L(A - eps V)] / (2 eps) against <grad L, V>, loss summed in fp64
    dims = (5000, 2000, 500, 100)
    st, factors = _problem(dims, 100000, 32, seed=9)
    t = api.Tensor(st.idx, st.val, dims)
    rng = np.random.default_rng(10)
    V = [rng.uniform(-1, 1, f.shape).astype(np.float32) for f in factors]
    dfac = [f.requires_grad_() for f in dev_factors(factors)]
    L = SparseCPLoss.apply(t, *dfac)
    L.backward()
    dirderiv = sum(float((f.grad * torch.from_numpy(v).cuda()).sum(dtype=torch.float64))
                   for f, v in zip(dfac, V))
    eps = 1e-3
    plus = dev_factors([f + eps * v for f, v in zip(factors, V)])
    minus = dev_factors([f - eps * v for f, v in zip(factors, V)])
    fd = (float(api.cp_loss(t, plus)) - float(api.cp_loss(t, minus))) / (2 * eps)
    log("directional derivative %.6e, central difference %.6e" % (dirderiv, fd))
    assert abs(fd - dirderiv) <= 1e-3 * abs(dirderiv)
    t.close()


@pytest.mark.parametrize("dims,rank", [((3000, 2000, 500, 100), 32), ((2000, 1500, 800), 16),
                                       ((500, 400, 300), 64), ((400, 300, 200), 5)])
def test_cp_loss_grad_one_pass_vs_oracle(dims, rank):
    """amped_cp_loss_grad for every mode (vector path at 16, 32 and 64, the
    column-tile path at 5): the gradient against the FP64 oracle gradient and
    the loss, summed in that mode's order, against the oracle loss, both at
    1e-5 relative."""
    st, factors = _problem(dims, 40000, rank, seed=rank + 100, hot=0.05)
    t = api.Tensor(st.idx, st.val, dims, chunk_nnz=256)
    dfac = dev_factors(factors)
    ref_loss, _ = oracle.cp_loss(st.idx, st.val, factors)
    for d in range(len(dims)):
        loss, g = api.cp_loss_grad(t, d, dfac, -2.0 * 0.75)
        ref = oracle.cp_grad(st.idx, st.val, dims, factors, d, grad_out=0.75)
        e, el = rel(g.cpu().numpy(), ref), abs(float(loss) - ref_loss) / abs(ref_loss)
        log("loss+grad mode %d: grad rel %.2e, loss rel %.2e" % (d, e, el))
        assert e <= 1e-5 and el <= 1e-5
    t.close()


@pytest.mark.parametrize("dims,rank", [((60, 50), 32), ((14, 12, 10, 9, 8), 16), ((10, 9, 8, 7, 6, 5), 8),
                                       ((6, 6, 5, 5, 4, 4, 3, 3), 4), ((9, 8, 7, 6, 5, 4), 40)])
def test_cp_loss_and_gradients_at_orders_2_to_8(dims, rank):
    """The loss, every mode's gradient and the one-pass loss + gradient at
    orders 2, 5, 6 and 8 (more than four input modes take the column-tile
    path) against the FP64 oracle, at 1e-5."""
    rng = np.random.default_rng(len(dims) * 100 + rank)
    nnz = min(3000, int(np.prod(dims)) // 2)
    idx, _ = synth.coords(dims, nnz, "uniform", seed=len(dims))
    val = rng.uniform(0, 1, nnz).astype(np.float32)
    factors = [(rng.uniform(-1, 1, (d, rank)) * 0.7).astype(np.float32) for d in dims]
    t = api.Tensor(idx, val, dims, chunk_nnz=64)
    dfac = dev_factors(factors)
    ref_loss, _ = oracle.cp_loss(idx, val, factors)
    assert abs(float(api.cp_loss(t, dfac)) - ref_loss) <= 1e-5 * abs(ref_loss)
    for d in range(len(dims)):
        ref = oracle.cp_grad(idx, val, dims, factors, d)
        e = rel(api.cp_grad(t, d, dfac, -2.0).cpu().numpy(), ref)
        loss, g = api.cp_loss_grad(t, d, dfac, -2.0)
        ef, el = rel(g.cpu().numpy(), ref), abs(float(loss) - ref_loss) / abs(ref_loss)
        log("order %d R=%d mode %d: grad rel %.2e, one pass %.2e, loss rel %.2e" % (len(dims), rank, d, e, ef, el))
        assert e <= 1e-5 and ef <= 1e-5 and el <= 1e-5
    t.close()


def test_cp_loss_grad_integer_exact_equals_separate_calls():
    """Small integers (values 1..4, factors -2..2): every residual, product and
    partial sum is exact, so the one-pass gradient equals amped_cp_grad's and
    the oracle's bit for bit, and the loss equals amped_cp_loss's and the
    oracle's exactly, for every mode, also when called again on the same
    outputs."""
    rng = np.random.default_rng(31)
    dims = (3000, 1500, 700)
    st = synth.tensor(dims, 40000, "zipf", 1.2, 0.1, seed=31)
    val = rng.integers(1, 5, st.nnz).astype(np.float32)
    factors = [rng.integers(-2, 3, (d, 32)).astype(np.float32) for d in dims]
    t = api.Tensor(st.idx, val, dims, chunk_nnz=64)
    dfac = dev_factors(factors)
    ref_loss, _ = oracle.cp_loss(st.idx, val, factors)
    sep_loss = float(api.cp_loss(t, dfac))
    assert sep_loss == ref_loss
    loss = torch.full((), float("nan"), dtype=torch.float64, device="cuda")
    for d in range(3):
        g = torch.full((dims[d], 32), float("nan"), device="cuda")
        for _ in range(2):
            api.cp_loss_grad(t, d, dfac, -2.0, out=g, loss=loss)
            torch.cuda.synchronize()
            assert float(loss) == ref_loss
            ref = oracle.cp_grad(st.idx, val, dims, factors, d).astype(np.float32)
            np.testing.assert_array_equal(g.cpu().numpy(), ref)
            np.testing.assert_array_equal(g.cpu().numpy(), api.cp_grad(t, d, dfac, -2.0).cpu().numpy())
    t.close()


def test_fused_autograd_forward_keeps_one_gradient():
    """sparse_cp_loss with factors that need gradients takes the one-pass
    forward (loss and the first needed mode's gradient); the backward pass
    scales that gradient by dL_out on the device and computes the others.
    Mode 0 needs no gradient here, so the early gradient is mode 1's; under
    torch.no_grad() the loss-only form runs."""
    dims = (2000, 1000, 300, 50)
    st, factors = _problem(dims, 30000, 32, seed=15)
    t = api.Tensor(st.idx, st.val, dims)
    dfac = [f.requires_grad_(w != 0) for w, f in enumerate(dev_factors(factors))]
    L = sparse_cp_loss(t, *dfac)
    assert isinstance(L.grad_fn, SparseCPLossFused._backward_cls)
    ref_loss, _ = oracle.cp_loss(st.idx, st.val, factors)
    assert abs(float(L.detach()) - ref_loss) <= 1e-5 * ref_loss
    (2.5 * L).backward()
    assert dfac[0].grad is None
    for d in (1, 2, 3):
        ref = oracle.cp_grad(st.idx, st.val, dims, factors, d, grad_out=2.5)
        e = rel(dfac[d].grad.cpu().numpy(), ref)
        log("fused autograd grad mode %d rel %.2e" % (d, e))
        assert e <= 1e-5
    with torch.no_grad():
        L2 = sparse_cp_loss(t, *dfac)
    assert L2.grad_fn is None and abs(float(L2) - ref_loss) <= 1e-5 * ref_loss
    # a second backward through the same graph: the kept gradient was used up
    # by the first, so every gradient is computed again, with the same values
    L3 = sparse_cp_loss(t, *dfac)
    for f in dfac:
        f.grad = None
    L3.backward(retain_graph=True)
    first = [None if f.grad is None else f.grad.clone() for f in dfac]
    for f in dfac:
        f.grad = None
    L3.backward()
    for d in (1, 2, 3):
        assert rel(dfac[d].grad.cpu().numpy(), first[d].cpu().numpy()) <= 1e-6
    t.close()


# ------------------------------------------------------------- hot-row cache

_CHILD_RUN = r"""
import sys, numpy as np, torch
sys.path.insert(0, sys.argv[1]); sys.path.insert(0, sys.argv[1] + "/tests")
from paper_2507_15121_amd import api
from gpu_util import dev_factors, hip_mttkrp
z = np.load(sys.argv[2])
dims = tuple(int(x) for x in z["dims"])
factors = [z["f%d" % w] for w in range(3)]
t = api.Tensor(z["idx"], z["val"], dims, chunk_nnz=256)
out = {}
for bf in (False, True):
    dfac = dev_factors(factors, torch.bfloat16 if bf else None)
    for d in range(3):
        out["%s%d" % ("b" if bf else "f", d)] = hip_mttkrp(t, d, dfac, bf16=bf)
np.savez(sys.argv[3], **out)
"""


@pytest.mark.parametrize("var,value", [("AMPED_HOT_MAX", "0"), ("AMPED_QUEUE_STRIPES", "1"),
                                       ("AMPED_QUEUE_STRIPES", "3")])
def test_hot_row_cache_and_queue_stripes_are_bit_exact(tmp_path, var, value):
    """The same launches with the LDS row cache off (AMPED_HOT_MAX=0), or with
    one global work-queue counter or three stripes instead of the default
    eight (AMPED_QUEUE_STRIPES; each read once per process, so in a child
    process) give bit-identical outputs.  Values and factors are small
    integers, so every sum is exact in fp32 and the order in which chunks are
    taken and chunk-boundary atomics land cannot change a bit."""
    import os
    import subprocess
    import sys
    from gpu_util import hip_mttkrp as hm
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    dims = (30000, 4000, 2500)
    st = synth.tensor(dims, 120000, "zipf", 1.3, 0.05, seed=33)
    rng = np.random.default_rng(33)
    val = rng.integers(1, 5, size=st.nnz).astype(np.float32)
    factors = [rng.integers(-2, 3, size=(d, 32)).astype(np.float32) for d in dims]
    t = api.Tensor(st.idx, val, dims, chunk_nnz=256)
    mine = {}
    for bf in (False, True):
        dfac = dev_factors(factors, torch.bfloat16 if bf else None)
        for d in range(3):
            mine["%s%d" % ("b" if bf else "f", d)] = hm(t, d, dfac, bf16=bf)
    inp = str(tmp_path / "inputs.npz")
    np.savez(inp, dims=np.array(dims), idx=st.idx, val=val, **{"f%d" % w: f for w, f in enumerate(factors)})
    path = str(tmp_path / "child.npz")
    env = dict(os.environ, **{var: value})
    log("child run with %s=%s" % (var, value))
    r = subprocess.run([sys.executable, "-c", _CHILD_RUN, root, inp, path], env=env, capture_output=True,
                       text=True, timeout=240)
    assert r.returncode == 0, r.stderr[-2000:]
    other = np.load(path)
    for k, v in mine.items():
        np.testing.assert_array_equal(v.view(np.uint32), other[k].view(np.uint32), err_msg=k)
