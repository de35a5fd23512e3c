"""GPU checks of host-resident layouts streamed to the device in shards
(out-of-core shard streaming, Sec. 4.8), through the C ABI.

Bars, as for device-resident tensors: relative Frobenius error <= 1e-5 against
the FP64 oracle for fp32 MTTKRP, loss and gradients; bit-exact for integer
inputs, where a streamed and a device-resident tensor must agree bit for bit;
bit-exact layouts.  Tiny shards (a few chunks) put hundreds of shard edges
inside the tensor, including inside one giant output row.
"""
import numpy as np
import pytest

import oracle
from oracle import als
from gpu_util import dev_factors, hip_mttkrp, log, oracle_mttkrp, rel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2507_15121_amd import api, synth  # noqa: E402


def _zipf(dims, nnz, seed, hot=0.05):
    return synth.tensor(dims, nnz, "zipf", 1.1, hot, seed=seed)


@pytest.mark.parametrize("chunk,shard", [(64, 192), (256, 1000), (4096, 0)])
def test_streamed_mttkrp_vs_oracle(chunk, shard):
    dims = (20000, 5000, 3000)
    st = _zipf(dims, 60000, seed=21)
    factors = synth.factors(dims, 32, seed=21)
    t = api.Tensor(st.idx, st.val, dims, chunk_nnz=chunk, host_layout=True, shard_nnz=shard)
    dfac = dev_factors(factors)
    for d in range(3):
        got = hip_mttkrp(t, d, dfac)
        assert not np.isnan(got).any(), "mode %d left rows unwritten" % d
        e = rel(got, oracle_mttkrp(st.idx, st.val, dims, factors, d))
        log("streamed chunk=%d shard=%d mode %d rel %.2e" % (chunk, shard, d, e))
        assert e <= 1e-5
    t.close()


def test_streamed_bf16_vs_oracle_on_rounded_factors():
    dims = (8000, 3000, 2000)
    st = _zipf(dims, 40000, seed=22)
    factors = synth.factors(dims, 64, seed=22)
    rounded = [oracle.bf16_to_f32(oracle.bf16_rne(f)) for f in factors]
    t = api.Tensor(st.idx, st.val, dims, chunk_nnz=128, host_layout=True, shard_nnz=512)
    dfac = dev_factors(factors, torch.bfloat16)
    for d in range(3):
        e = rel(hip_mttkrp(t, d, dfac, bf16=True), oracle_mttkrp(st.idx, st.val, dims, rounded, d))
        log("streamed bf16 mode %d rel %.2e" % (d, e))
        assert e <= 1e-5
    t.close()


@pytest.mark.parametrize("rank", [32, 5, 100])
def test_streamed_integer_inputs_equal_resident_bit_for_bit(rank):
    """R = 32: vector path; 5 and 100: scalar column tiles (100 takes two
    tiles, each streaming every shard)."""
    rng = np.random.default_rng(rank)
    dims = (3000, 1500, 700)
    st = synth.tensor(dims, 50000, "zipf", 1.2, 0.1, seed=rank)
    val = rng.integers(1, 5, size=st.nnz).astype(np.float32)
    factors = [rng.integers(-2, 3, size=(d, rank)).astype(np.float32) for d in dims]
    res = api.Tensor(st.idx, val, dims, chunk_nnz=64)
    strm = api.Tensor(st.idx, val, dims, chunk_nnz=64, host_layout=True, shard_nnz=320)
    dfac = dev_factors(factors)
    for d in range(3):
        ref = oracle_mttkrp(st.idx, val, dims, factors, d)
        assert np.abs(ref).max() < 2 ** 24
        a = hip_mttkrp(res, d, dfac)
        b = hip_mttkrp(strm, d, dfac)
        np.testing.assert_array_equal(b, ref.astype(np.float32))
        assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
    res.close()
    strm.close()


def test_streamed_loss_and_grad_vs_oracle():
    dims = (3000, 2000, 500, 100)
    st = synth.tensor(dims, 40000, "zipf", 1.2, 0.05, seed=23)
    factors = synth.factors(dims, 32, seed=23)
    t = api.Tensor(st.idx, st.val, dims, chunk_nnz=256, host_layout=True, shard_nnz=1024)
    dfac = dev_factors(factors)
    loss = float(api.cp_loss(t, dfac))
    ref_loss, _ = oracle.cp_loss(st.idx, st.val, factors)
    log("streamed loss %.9e ref %.9e" % (loss, ref_loss))
    assert abs(loss - ref_loss) <= 1e-5 * abs(ref_loss)
    for d in range(4):
        g = api.cp_grad(t, d, dfac, -2.0).cpu().numpy()
        ref = oracle.cp_grad(st.idx, st.val, dims, factors, d)
        e = rel(g, ref)
        # the one-pass form: the loss adds up over the 40 shards of the mode
        lf, gf = api.cp_loss_grad(t, d, dfac, -2.0)
        ef, elf = rel(gf.cpu().numpy(), ref), abs(float(lf) - ref_loss) / abs(ref_loss)
        log("  streamed grad mode %d rel %.2e; one pass: grad rel %.2e, loss rel %.2e" % (d, e, ef, elf))
        assert e <= 1e-5 and ef <= 1e-5 and elf <= 1e-5
    t.close()


def test_streamed_layouts_equal_resident_ones():
    dims = (900, 700, 500)
    st = _zipf(dims, 30000, seed=24)
    perm_order = np.random.default_rng(24).permutation(st.nnz)   # not lexicographic: both builders sort
    idx, val = st.idx[:, perm_order], st.val[perm_order]
    res = api.Tensor(idx, val, dims, chunk_nnz=100, keep_perm=True)
    strm = api.Tensor(idx, val, dims, chunk_nnz=100, keep_perm=True, host_layout=True, shard_nnz=700)
    for d in range(3):
        a, b = res.layout(d, perm=True), strm.layout(d, perm=True)
        ref = oracle.layout(idx, d, 100)
        np.testing.assert_array_equal(b["perm"], ref["perm"])
        for k in a:
            np.testing.assert_array_equal(a[k], b[k])
    res.close()
    strm.close()


def test_streamed_als_sweep_vs_oracle_with_duplicates():
    """Exact duplicates (summed before squaring in ||X||^2) end up adjacent in
    the mode-0 layout; the norm pass cuts its shards between such runs."""
    dims = (500, 400, 300)
    st = _zipf(dims, 20000, seed=25, hot=0.0)
    idx = np.concatenate([st.idx, st.idx[:, :3000], st.idx[:, :500]], axis=1)
    val = np.concatenate([st.val, st.val[:3000] * 0.5, st.val[:500] * 0.25])
    rng = np.random.default_rng(25)
    F0 = [rng.uniform(-1, 1, (d, 16)).astype(np.float32) for d in dims]
    t = api.Tensor(idx, val, dims, chunk_nnz=64, host_layout=True, shard_nnz=256)
    dF = dev_factors(F0)
    lam, fit = api.cp_als_sweep(t, dF)
    torch.cuda.synchronize()
    Fo, lo, fo = als.cp_als_sweep(idx, val, dims, [f.astype(np.float64) for f in F0])
    errs = [oracle.rel_fro(dF[d].cpu().numpy(), Fo[d]) for d in range(3)]
    log("streamed ALS errs %s fit %.6f vs %.6f" % (["%.1e" % e for e in errs], float(fit.item()), fo))
    assert max(errs) <= 1e-4
    assert oracle.rel_fro(lam.cpu().numpy(), lo) <= 1e-4
    assert abs(float(fit.item()) - fo) <= 1e-5
    t.close()


def test_run_of_duplicates_longer_than_a_shard():
    """MTTKRP splits such a run over shards like any row; the ALS norm pass,
    which must see a run whole, reports it as unsupported."""
    dims = (50, 40, 30)
    rng = np.random.default_rng(26)
    idx = np.concatenate([np.array([[7], [8], [9]], np.int32).repeat(300, axis=1),
                          np.stack([rng.integers(0, d, 2000) for d in dims]).astype(np.int32)], axis=1)
    val = rng.uniform(0, 1, idx.shape[1]).astype(np.float32)
    factors = synth.factors(dims, 8, seed=26)
    t = api.Tensor(idx, val, dims, chunk_nnz=16, host_layout=True, shard_nnz=64)
    dfac = dev_factors(factors)
    for d in range(3):
        assert rel(hip_mttkrp(t, d, dfac), oracle_mttkrp(idx, val, dims, factors, d)) <= 1e-5
    with pytest.raises(api.AmpedError) as ei:
        api.cp_als_sweep(t, dfac)
    assert ei.value.status == api.ERR_UNSUPPORTED
    torch.cuda.synchronize()
    t.close()


def test_streamed_empty_tensor_zeroes_outputs():
    dims = (30, 20, 10)
    t = api.Tensor(np.zeros((3, 0), np.int32), np.zeros(0, np.float32), dims, host_layout=True, shard_nnz=64)
    dfac = dev_factors(synth.factors(dims, 16, seed=27))
    for d in range(3):
        assert not hip_mttkrp(t, d, dfac).any()
    assert float(api.cp_loss(t, dfac)) == 0.0
    t.close()


@pytest.mark.parametrize("dims,rank", [((40, 30), 32), ((12, 10, 8, 6, 5), 16), ((6, 5, 5, 4, 4, 3, 3, 2), 4)])
def test_streamed_orders_2_5_8(dims, rank):
    rng = np.random.default_rng(len(dims) + 40)
    nnz = min(2000, int(np.prod(dims)) // 2)
    idx, _ = synth.coords(dims, nnz, "uniform", seed=len(dims) + 40)
    val = rng.uniform(0, 1, nnz).astype(np.float32)
    factors = [rng.uniform(-1, 1, (d, rank)).astype(np.float32) for d in dims]
    t = api.Tensor(idx, val, dims, chunk_nnz=16, host_layout=True, shard_nnz=48)
    dfac = dev_factors(factors)
    for d in range(len(dims)):
        e = rel(hip_mttkrp(t, d, dfac), oracle_mttkrp(idx, val, dims, factors, d))
        assert e <= 1e-5, "order %d mode %d rel %.2e" % (len(dims), d, e)
    loss = float(api.cp_loss(t, dfac))
    ref_loss, _ = oracle.cp_loss(idx, val, factors)
    assert abs(loss - ref_loss) <= 1e-5 * abs(ref_loss)
    t.close()


def test_streamed_chained_als_sweeps_reuse_grams():
    """Three chained sweeps on a streamed tensor, the later ones reusing the
    Gram matrices the previous sweep left, each against the oracle's sweep
    from the same factors."""
    dims = (900, 700, 500)
    st = _zipf(dims, 30000, seed=28, hot=0.0)
    rng = np.random.default_rng(28)
    F0 = [rng.uniform(-1, 1, (d, 12)).astype(np.float32) for d in dims]
    t = api.Tensor(st.idx, st.val, dims, chunk_nnz=128, host_layout=True, shard_nnz=2048)
    dF = dev_factors(F0)
    for s in range(3):
        start = [f.cpu().numpy().astype(np.float64) for f in dF]
        lam, fit = api.cp_als_sweep(t, dF, reuse_grams=s > 0)
        Fo, lo, fo = als.cp_als_sweep(st.idx, st.val, dims, start)
        errs = [oracle.rel_fro(dF[d].cpu().numpy(), Fo[d]) for d in range(3)]
        log("streamed chained sweep %d: errs %s fit %.6f vs %.6f" % (s, ["%.1e" % e for e in errs],
                                                                     float(fit.item()), fo))
        assert max(errs) <= 1e-4 and abs(float(fit.item()) - fo) <= 1e-5
    t.close()
