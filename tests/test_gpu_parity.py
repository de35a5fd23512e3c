"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Bars: bit-exact for layouts and chunk flags; relative Frobenius error
<= 1e-5 for fp32 MTTKRP; bit-exact for integer-valued inputs, whose sums are
exact in fp32 in any order.
"""
import numpy as np
import pytest

import oracle
from gpu_util import dev_factors, hip_mttkrp, log, oracle_mttkrp, rel, torch_mod

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2507_15121_amd import api, synth  # noqa: E402

TOL = 1e-5


def _tensor(idx, val, dims, **kw):
    return api.Tensor(idx, val, dims, **kw)


def _check_all_modes(idx, val, dims, factors, tol=TOL, **kw):
    t = _tensor(idx, val, dims, **kw)
    dfac = dev_factors(factors)
    errs = []
    for d in range(len(dims)):
        got = hip_mttkrp(t, d, dfac)
        ref = oracle_mttkrp(idx, val, dims, factors, d)
        assert not np.isnan(got).any(), "mode %d left rows unwritten" % d
        e = rel(got, ref)
        errs.append(e)
        assert e <= tol, "mode %d rel err %.3e" % (d, e)
    t.close()
    return errs


@pytest.mark.parametrize("rank", [16, 32, 64])
def test_uniform_1000x800x600_all_modes(rank):
    w = synth.WORKLOADS["uniform3-1000x800x600-100k"]
    st = synth.workload(w.name)
    factors = synth.factors(st.dims, rank)
    log("uniform 100k R=%d" % rank)
    errs = _check_all_modes(st.idx, st.val, st.dims, factors)
    log("  rel errs %s" % errs)


@pytest.mark.parametrize("chunk", [1, 7, 64, 4096])
def test_zipf_small_with_hot_slice(chunk):
    dims = (20000, 5000, 3000)
    st = synth.tensor(dims, 60000, "zipf", 1.1, 0.05, seed=11)
    factors = synth.factors(dims, 32, seed=11)
    log("zipf 60k hot chunk=%d" % chunk)
    _check_all_modes(st.idx, st.val, dims, factors, chunk_nnz=chunk)


def _int_problem(rng, dims, nnz, rank, hot=0.0):
    st = synth.tensor(dims, nnz, "zipf", 1.2, hot, seed=int(rng.integers(1 << 30)))
    val = rng.integers(1, 5, size=nnz).astype(np.float32)
    factors = [rng.integers(-2, 3, size=(d, rank)).astype(np.float32) for d in dims]
    return st.idx, val, factors


@pytest.mark.parametrize("chunk", [7, 64, 4096])
def test_integer_inputs_bit_exact_and_stable(chunk):
    rng = np.random.default_rng(chunk)
    dims = (3000, 1500, 700)
    idx, val, factors = _int_problem(rng, dims, 50000, 32, hot=0.1)
    t = _tensor(idx, val, dims, chunk_nnz=chunk)
    dfac = dev_factors(factors)
    for d in range(3):
        ref = oracle_mttkrp(idx, val, dims, factors, d)
        assert np.abs(ref).max() < 2 ** 24
        first = hip_mttkrp(t, d, dfac)
        np.testing.assert_array_equal(first, ref.astype(np.float32))
        for _ in range(9):
            again = hip_mttkrp(t, d, dfac)
            assert np.array_equal(again.view(np.uint32), first.view(np.uint32))
    t.close()


@pytest.mark.parametrize("dims,rank", [((40, 30), 32), ((30, 20, 10, 8), 32), ((12, 10, 8, 6, 5), 16),
                                       ((9, 8, 7, 6, 5, 4), 8), ((6, 5, 5, 4, 4, 3, 3, 2), 4)])
def test_orders_2_to_8(dims, rank):
    rng = np.random.default_rng(len(dims))
    nnz = min(2000, int(np.prod(dims)) // 2)
    idx, _ = synth.coords(dims, nnz, "uniform", seed=len(dims))
    val = rng.uniform(0, 1, nnz).astype(np.float32)
    factors = [rng.uniform(-1, 1, (d, rank)).astype(np.float32) for d in dims]
    log("order %d rank %d" % (len(dims), rank))
    _check_all_modes(idx, val, dims, factors, chunk_nnz=64)


@pytest.mark.parametrize("rank", [1, 3, 5, 8, 20, 48, 100, 128, 200])
def test_ranks_vector_and_column_tile_paths(rank):
    dims = (500, 400, 300)
    st = synth.tensor(dims, 20000, "zipf", 1.1, 0.0, seed=rank)
    factors = synth.factors(dims, rank, seed=rank)
    log("rank %d" % rank)
    _check_all_modes(st.idx, st.val, dims, factors, chunk_nnz=256)


def test_single_nonzero_and_single_row_modes():
    dims = (7, 1, 5)
    idx = np.array([[3], [0], [4]], np.int32)
    val = np.array([1.5], np.float32)
    rng = np.random.default_rng(2)
    factors = [rng.uniform(-1, 1, (d, 32)).astype(np.float32) for d in dims]
    _check_all_modes(idx, val, dims, factors)


def test_all_nonzeros_in_one_slice_many_chunks():
    rng = np.random.default_rng(3)
    dims = (50, 4000, 3000)
    nnz = 30000
    lin = np.sort(rng.choice(4000 * 3000, size=nnz, replace=False))
    idx = np.stack([np.full(nnz, 17), lin // 3000, lin % 3000]).astype(np.int32)
    val = rng.uniform(0, 1, nnz).astype(np.float32)
    factors = [rng.uniform(-1, 1, (d, 32)).astype(np.float32) for d in dims]
    for ch in (1, 7, 100):
        log("one slice chunk=%d" % ch)
        _check_all_modes(idx, val, dims, factors, chunk_nnz=ch)


def test_empty_tensor_zeroes_output():
    dims = (100, 70, 3)
    idx = np.zeros((3, 0), np.int32)
    val = np.zeros(0, np.float32)
    t = _tensor(idx, val, dims)
    dfac = dev_factors([np.ones((d, 16), np.float32) for d in dims])
    for d in range(3):
        out = hip_mttkrp(t, d, dfac)
        assert out.shape == (dims[d], 16) and not out.any() and not np.isnan(out).any()
    t.close()


def test_long_untouched_row_runs():
    # few nonzeros in huge modes: most output rows are zero, in long runs
    rng = np.random.default_rng(4)
    dims = (200000, 64, 100000)
    nnz = 500
    idx = np.stack([rng.integers(0, d, nnz) for d in dims]).astype(np.int32)
    val = rng.uniform(0, 1, nnz).astype(np.float32)
    factors = [rng.uniform(-1, 1, (d, 16)).astype(np.float32) for d in dims]
    _check_all_modes(idx, val, dims, factors, chunk_nnz=32)


@pytest.mark.parametrize("chunk", [1, 7, 64])
def test_untouched_runs_of_every_length_near_the_kernel_threshold(chunk):
    """Touched mode-0 rows separated by runs of 1..40 untouched rows (every
    length on both sides of 16, below which the init kernel zeroes a run row
    by row from its list and above which as one range), with 1-3 nonzeros per
    touched row, so runs start at chunk starts, lane-group run starts and
    inside runs; also a short run before the first and after the last touched
    row.  Every output
    starts as NaN: mode 0 must equal the oracle bit for bit on integer inputs
    (untouched rows exactly 0), resident and streamed in shards of 50
    nonzeros, for MTTKRP and for the fused gradient (with and without the
    loss)."""
    rng = np.random.default_rng(1600 + chunk)
    rows0, gaps = [5], []
    while len(rows0) < 400:
        gaps.append(1 + (len(rows0) * 7) % 40)
        rows0.append(rows0[-1] + gaps[-1] + 1)
    I0 = rows0[-1] + 9
    per = rng.integers(1, 4, len(rows0))
    i0 = np.repeat(np.asarray(rows0, dtype=np.int32), per)
    nnz = i0.size
    dims = (I0, 50, 30)
    i1 = rng.integers(0, dims[1], nnz).astype(np.int32)
    i2 = rng.integers(0, dims[2], nnz).astype(np.int32)
    idx = np.stack([i0, i1, i2])
    o = np.lexsort(idx[::-1])
    idx = np.ascontiguousarray(idx[:, o])
    val = rng.integers(1, 5, nnz).astype(np.float32)
    factors = [rng.integers(-2, 3, (d, 16)).astype(np.float32) for d in dims]
    ref = oracle_mttkrp(idx, val, dims, factors, 0).astype(np.float32)
    gref = oracle.cp_grad(idx, val, dims, factors, 0).astype(np.float32)
    dfac = dev_factors(factors)
    for kw in ({}, {"host_layout": True, "shard_nnz": 50}):
        t = _tensor(idx, val, dims, chunk_nnz=chunk, **kw)
        np.testing.assert_array_equal(hip_mttkrp(t, 0, dfac), ref)
        g = torch.full((I0, 16), float("nan"), device="cuda")
        api.cp_grad(t, 0, dfac, -2.0, out=g)
        np.testing.assert_array_equal(g.cpu().numpy(), gref)
        g.fill_(float("nan"))
        api.cp_loss_grad(t, 0, dfac, -2.0, out=g)
        np.testing.assert_array_equal(g.cpu().numpy(), gref)
        t.close()


@pytest.mark.parametrize("where", ["head", "tail", "middle"])
def test_millions_of_untouched_rows_in_one_run(where):
    """All nonzeros of mode 0 within 1000 consecutive rows of a 3M-row mode,
    so the rest of the output is one or two untouched runs of millions of
    rows, which the init kernel zeroes as ranges of about 2048 rows spread
    over its grid; every output starts as NaN and must match the oracle with
    the untouched rows exactly 0 (also for the fused gradient)."""
    rng = np.random.default_rng({"head": 1, "tail": 2, "middle": 3}[where])
    dims = (3_000_000, 64, 32)
    lo = {"head": 2_990_000, "tail": 0, "middle": 1_500_000}[where]
    nnz = 20000
    idx = np.stack([rng.integers(lo, lo + 1000, nnz), rng.integers(0, dims[1], nnz),
                    rng.integers(0, dims[2], nnz)]).astype(np.int32)
    val = rng.integers(1, 5, nnz).astype(np.float32)
    factors = [rng.integers(-2, 3, (d, 16)).astype(np.float32) for d in dims]
    t = _tensor(idx, val, dims)
    dfac = dev_factors(factors)
    for d in range(3):
        np.testing.assert_array_equal(hip_mttkrp(t, d, dfac),
                                      oracle_mttkrp(idx, val, dims, factors, d).astype(np.float32))
    g = torch.full((dims[0], 16), float("nan"), device="cuda")
    api.cp_grad(t, 0, dfac, -2.0, out=g)
    np.testing.assert_array_equal(g.cpu().numpy(), oracle.cp_grad(idx, val, dims, factors, 0).astype(np.float32))
    t.close()


def test_duplicates_and_unsorted_input():
    rng = np.random.default_rng(5)
    dims = (300, 200, 100)
    nnz = 20000
    idx = np.stack([rng.integers(0, d, nnz) for d in dims]).astype(np.int32)  # duplicates, unsorted
    val = rng.uniform(0, 1, nnz).astype(np.float32)
    factors = [rng.uniform(-1, 1, (d, 32)).astype(np.float32) for d in dims]
    _check_all_modes(idx, val, dims, factors, chunk_nnz=128)


@pytest.mark.parametrize("chunk", [7, 4096])
def test_device_layout_bit_exact(chunk):
    st = synth.tensor((2000, 900, 400), 30000, "zipf", 1.1, 0.05, seed=6)
    rng = np.random.default_rng(6)
    p = rng.permutation(st.nnz)
    idx, val = st.idx[:, p], st.val[p]  # shuffled input
    t = _tensor(idx, val, st.dims, chunk_nnz=chunk, keep_perm=True)
    for d in range(3):
        lay = t.layout(d, perm=True)
        ref = oracle.layout(idx, d, chunk)
        np.testing.assert_array_equal(lay["perm"], ref["perm"])
        np.testing.assert_array_equal(lay["out_idx"], ref["out_idx"])
        np.testing.assert_array_equal(lay["in_idx"], ref["in_idx"])
        np.testing.assert_array_equal(lay["values"].view(np.uint32), val[ref["perm"]].view(np.uint32))
        np.testing.assert_array_equal(lay["flags"], ref["flags"])
    assert t.touched == tuple(len(np.unique(idx[w])) for w in range(3))
    t.close()


@pytest.mark.parametrize("shuffle", [False, True])
def test_device_layout_wide_keys_matches_host_builder(shuffle):
    """Index ranges that need 4 radix passes (up to 27 bits), many equal keys
    and, when shuffled, a device-built lexicographic order: the device layout's
    permutation and chunk flags equal the host builder's, bit for bit."""
    dims = (100_000_000, 3, 70_000_000)
    rng = np.random.default_rng(12)
    nnz = 300_000
    idx = np.stack([rng.integers(0, d, nnz) for d in dims]).astype(np.int32)
    idx[0, : nnz // 3] = 12_345_678          # a long run of one key
    val = rng.uniform(0, 1, nnz).astype(np.float32)
    if not shuffle:
        o = np.lexsort(idx[::-1])
        idx, val = idx[:, o], val[o]
    log("wide keys, shuffled=%s" % shuffle)
    t = _tensor(idx, val, dims, chunk_nnz=1000, keep_perm=True)
    for d in range(3):
        lay = t.layout(d, perm=True)
        perm, flags = api.layout_host(idx, dims, d, 1000)
        np.testing.assert_array_equal(lay["perm"], perm)
        np.testing.assert_array_equal(lay["flags"], flags)
        np.testing.assert_array_equal(lay["out_idx"], idx[d][perm])
    t.close()


def test_device_layout_bit_exact_above_256_scan_tiles():
    """24M nonzeros: each radix pass scans 256 x 24M / 4096 digit counts in
    tiles of 4096, i.e. 366 scan tiles, so the tile totals are scanned in two
    carried rounds (more than 256 tiles appear from about 16.7M nonzeros on).
    Shuffled input with 2M exact duplicates copied from other positions, a run
    of 2M nonzeros with one mode-0 index and 300k identical coordinates: the
    device layout of every mode (perm, out_idx, in_idx, values, chunk flags)
    equals the host builder's, which the CPU tests pin to the oracle's
    ordering, bit for bit."""
    rng = np.random.default_rng(24)
    dims = (5000, 300_000, 70_000)
    nnz = 24_000_000
    idx = np.stack([rng.integers(0, d, nnz, dtype=np.int32) for d in dims])
    idx[0, :2_000_000] = 4321
    idx[:, 2_000_000:2_300_000] = np.array([[17], [123_456], [65_432]], dtype=np.int32)
    src = rng.integers(0, nnz, 2_000_000)
    dst = rng.integers(0, nnz, 2_000_000)
    idx[:, dst] = idx[:, src]
    p = rng.permutation(nnz)
    idx = np.ascontiguousarray(idx[:, p])
    val = rng.uniform(0, 1, nnz).astype(np.float32)
    log("layout 24M: building on the device")
    t = _tensor(idx, val, dims, keep_perm=True)
    for d in range(3):
        lay = t.layout(d, perm=True)
        perm, flags = api.layout_host(idx, dims, d, 4096)
        np.testing.assert_array_equal(lay["perm"], perm)
        np.testing.assert_array_equal(lay["flags"], flags)
        np.testing.assert_array_equal(lay["out_idx"], idx[d][perm])
        others = [w for w in range(3) if w != d]
        for j, w in enumerate(others):
            np.testing.assert_array_equal(lay["in_idx"][j], idx[w][perm])
        np.testing.assert_array_equal(lay["values"].view(np.uint32), val[perm].view(np.uint32))
        log("layout 24M: mode %d equal to the host builder" % d)
    t.close()


def test_non_default_stream_and_reuse_of_output():
    st = synth.tensor((3000, 2000, 1000), 40000, "zipf", 1.1, 0.0, seed=8)
    factors = synth.factors(st.dims, 32, seed=8)
    t = _tensor(st.idx, st.val, st.dims)
    dfac = dev_factors(factors)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        got = hip_mttkrp(t, 1, dfac, stream=s)
    ref = oracle_mttkrp(st.idx, st.val, st.dims, factors, 1)
    assert rel(got, ref) <= TOL
    t.close()


def test_modes_on_concurrent_streams():
    """Different modes of one tensor have their own work queues, so their
    calls may overlap on different streams (default priority); five rounds of
    all three modes at once, each output against the oracle."""
    st = synth.tensor((5000, 3000, 2000), 80000, "zipf", 1.1, 0.05, seed=12)
    factors = synth.factors(st.dims, 32, seed=12)
    t = _tensor(st.idx, st.val, st.dims, chunk_nnz=256)
    dfac = dev_factors(factors)
    refs = [oracle_mttkrp(st.idx, st.val, st.dims, factors, d) for d in range(3)]
    streams = [torch.cuda.Stream() for _ in range(3)]
    outs = [torch.empty((st.dims[d], 32), dtype=torch.float32, device="cuda") for d in range(3)]
    torch.cuda.synchronize()
    for _ in range(5):
        for o in outs:
            o.fill_(float("nan"))
        torch.cuda.synchronize()
        for d, s in enumerate(streams):
            with torch.cuda.stream(s):
                f = [None if w == d else x for w, x in enumerate(dfac)]
                api.mttkrp(t, d, f, out=outs[d], stream=s)
        torch.cuda.synchronize()
        for d in range(3):
            assert rel(outs[d].cpu().numpy(), refs[d]) <= TOL
    t.close()


def test_all_mode_step_replayed_from_a_hip_graph():
    """The library's launches (init kernel + MTTKRP kernel per mode, the fused
    loss + gradient, bf16 MTTKRP) captured once into a HIP graph (torch's
    CUDAGraph) and replayed five times, with eager work between the replays
    that overwrites every output: each replay must give the eager results bit
    for bit (integer inputs, so any summation order is exact).  The queue
    counters and the loss are reset by the init kernel inside the graph, with
    no memset node."""
    rng = np.random.default_rng(77)
    dims = (3000, 2000, 1000)
    st = synth.tensor(dims, 60000, "zipf", 1.2, 0.05, seed=77)
    val = rng.integers(1, 5, st.nnz).astype(np.float32)
    factors = [rng.integers(-2, 3, (d, 32)).astype(np.float32) for d in dims]
    t = _tensor(st.idx, val, dims, chunk_nnz=256)
    dfac = dev_factors(factors)
    dbf = [f.to(torch.bfloat16) for f in dfac]
    outs = [torch.empty((d, 32), device="cuda") for d in dims]
    outs_b = [torch.empty((d, 32), device="cuda") for d in dims]
    grad0 = torch.empty((dims[0], 32), device="cuda")
    loss = torch.empty((), dtype=torch.float64, device="cuda")

    def step():
        for d in range(3):
            api.mttkrp(t, d, [None if w == d else f for w, f in enumerate(dfac)], out=outs[d])
            api.mttkrp_bf16(t, d, [None if w == d else f for w, f in enumerate(dbf)], out=outs_b[d])
        api.cp_loss_grad(t, 0, dfac, -2.0, out=grad0, loss=loss)

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step()   # eager: first-call set-up happens outside the capture
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    ref = [o.clone() for o in outs] + [o.clone() for o in outs_b] + [grad0.clone(), loss.clone()]
    ref_y = [oracle_mttkrp(st.idx, val, dims, factors, d).astype(np.float32) for d in range(3)]
    for d in range(3):
        np.testing.assert_array_equal(ref[d].cpu().numpy(), ref_y[d])
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        step()
    for rep in range(5):
        for o in outs + outs_b + [grad0]:
            o.fill_(float("nan"))
        loss.fill_(-1.0)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for a, b in zip(outs + outs_b + [grad0, loss], ref):
            np.testing.assert_array_equal(a.cpu().numpy(), b.cpu().numpy())
        log("graph replay %d equal to the eager step" % rep)
    t.close()


def test_call_errors_on_device():
    from ctypes import c_void_p
    st = synth.tensor((300, 200, 100), 2000, "zipf", 1.1, 0.0, seed=9)
    t = _tensor(st.idx, st.val, st.dims)
    dfac = dev_factors(synth.factors(st.dims, 32, seed=9))
    out = torch.empty((300, 32), device="cuda")
    with pytest.raises(ValueError):
        api.mttkrp(t, 0, [None, dfac[1][1:], dfac[2]], out=out)  # wrong shape, caught in python
    L = api.lib()
    ptrs = (c_void_p * 3)(None, dfac[1].data_ptr() + 4, dfac[2].data_ptr())
    assert L.amped_mttkrp(t.handle, 0, 32, ptrs, c_void_p(out.data_ptr()), None) == api.ERR_INVALID
    ptrs = (c_void_p * 3)(None, dfac[1].data_ptr(), dfac[2].data_ptr())
    assert L.amped_mttkrp(t.handle, 3, 32, ptrs, c_void_p(out.data_ptr()), None) == api.ERR_INVALID
    assert L.amped_mttkrp(t.handle, 0, 0, ptrs, c_void_p(out.data_ptr()), None) == api.ERR_INVALID
    assert L.amped_mttkrp(t.handle, 0, 32, ptrs, None, None) == api.ERR_INVALID
    ptrs = (c_void_p * 3)(None, None, dfac[2].data_ptr())
    assert L.amped_mttkrp(t.handle, 0, 32, ptrs, c_void_p(out.data_ptr()), None) == api.ERR_INVALID
    # the fused gradient needs the output mode's factor too
    ptrs = (c_void_p * 3)(None, dfac[1].data_ptr(), dfac[2].data_ptr())
    assert L.amped_cp_grad(t.handle, 0, 32, ptrs, 1.0, c_void_p(out.data_ptr()), None) == api.ERR_INVALID
    assert "factors[0]" in L.amped_last_error().decode()
    t.close()
