"""Full-size parity: the 200M-nonzero Zipf tensor (10M x 5M x 2M, R=32) in the
launch configuration the benchmark times, checked on sampled output rows that
the oracle computes one by one (the heaviest row of each mode plus random
touched rows), and on whole-output properties that hold at any size."""
import numpy as np
import pytest

import oracle
from gpu_util import log, oracle_rows, sample_rows

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2507_15121_amd import api, synth  # noqa: E402


def _sample_rows(st, d, rng, n):
    counts = np.bincount(st.idx[d], minlength=st.dims[d])
    touched = np.flatnonzero(counts)
    rows = rng.choice(touched, size=min(n, touched.size), replace=False)
    rows = np.unique(np.concatenate([rows, [int(np.argmax(counts))]]))
    untouched = np.flatnonzero(counts == 0)
    return rows, counts, untouched


def _oracle_rows(st, factors64, d, rows, R):
    lut = np.full(st.dims[d], -1, dtype=np.int64)
    lut[rows] = np.arange(rows.size)
    m = lut[st.idx[d]] >= 0
    sub = st.idx[:, m].copy()
    sub[d] = lut[sub[d]]
    dims = list(st.dims)
    dims[d] = rows.size
    fs = list(factors64)
    fs[d] = np.zeros((rows.size, R))
    return oracle.mttkrp(sub, st.val[m], dims, fs, d)


@pytest.fixture(scope="module")
def big():
    w = synth.WORKLOADS["zipf3-10Mx5Mx2M-200M"]
    log("generating %s" % w.name)
    st = synth.workload(w.name)
    factors = synth.factors(st.dims, w.rank)
    log("building layouts")
    T = api.Tensor(st.idx, st.val, st.dims)
    yield st, factors, T, w.rank
    T.close()


def test_fullsize_fp32_sampled_rows(big):
    st, factors, T, R = big
    dfac = [torch.from_numpy(f).cuda() for f in factors]
    f64 = [f.astype(np.float64) for f in factors]
    rng = np.random.default_rng(1)
    for d in range(3):
        out = torch.full((st.dims[d], R), float("nan"), device="cuda")
        api.mttkrp(T, d, [None if w == d else f for w, f in enumerate(dfac)], out=out)
        torch.cuda.synchronize()
        assert not torch.isnan(out).any().item(), "mode %d left rows unwritten" % d
        rows, counts, untouched = _sample_rows(st, d, rng, 300)
        got = out[torch.from_numpy(rows).cuda()].cpu().numpy()
        e = oracle.rel_fro(got, _oracle_rows(st, f64, d, rows, R))
        heavy = int(np.argmax(counts))
        k = int(np.searchsorted(rows, heavy))
        eh = oracle.rel_fro(got[k:k + 1], _oracle_rows(st, f64, d, np.array([heavy]), R))
        log("mode %d: sampled rel %.2e, heaviest row (%d nnz) rel %.2e" % (d, e, counts[heavy], eh))
        assert e <= 1e-5 and eh <= 1e-5
        if untouched.size:
            z = out[torch.from_numpy(untouched[:100000]).cuda()]
            assert not z.any().item()
        # whole-output property: sum_i Y_d[i,r] A_d[i,r] = sum_k val_k prod_w A_w[i_w(k),r]
        # does not depend on d
        prod = out.double() * dfac[d].double()
        inv, scale = prod.sum(0).cpu().numpy(), prod.abs().sum(0).cpu().numpy()
        if d == 0:
            inv0, scale0 = inv, scale
        else:
            assert np.all(np.abs(inv - inv0) <= 1e-5 * (scale + scale0))


def test_fullsize_bf16_sampled_rows(big):
    st, factors, T, R = big
    dbf = [torch.from_numpy(f).cuda().to(torch.bfloat16) for f in factors]
    f64 = [f.astype(np.float64) for f in factors]
    rng = np.random.default_rng(2)
    for d in range(3):
        out = api.mttkrp_bf16(T, d, [None if w == d else f for w, f in enumerate(dbf)])
        rows, _, _ = _sample_rows(st, d, rng, 200)
        got = out[torch.from_numpy(rows).cuda()].cpu().numpy()
        e = oracle.rel_fro(got, _oracle_rows(st, f64, d, rows, R))
        log("bf16 mode %d: sampled rel %.2e vs fp64 oracle on fp32 factors" % (d, e))
        assert e <= 1e-2


def test_fullsize_r64_fp32_and_bf16(big):
    """The same 200M-nonzero tensor at R = 64 (256-byte fp32 rows, 16 lanes per
    row; 128-byte bf16 rows): fp32 against the FP64 oracle at 1e-5; bf16
    against the oracle on the bf16-rounded factors at 1e-5 (fp32 accumulation)
    and against the oracle on the fp32 factors at 1e-2, per mode."""
    st, _, T, _ = big
    R = 64
    factors = synth.factors(st.dims, R)
    dfac = [torch.from_numpy(f).cuda() for f in factors]
    dbf = [f.to(torch.bfloat16) for f in dfac]
    rng = np.random.default_rng(64)

    def bf16_round(f):
        return oracle.bf16_to_f32(oracle.bf16_rne(f))
    for d in range(3):
        rows, counts, _ = sample_rows(st.idx[d], st.dims[d], rng, 200)
        sel = torch.from_numpy(rows).cuda()
        out = torch.full((st.dims[d], R), float("nan"), device="cuda")
        api.mttkrp(T, d, [None if w == d else f for w, f in enumerate(dfac)], out=out)
        torch.cuda.synchronize()
        assert not torch.isnan(out).any().item()
        got = out[sel].cpu().numpy()
        out.fill_(float("nan"))
        api.mttkrp_bf16(T, d, [None if w == d else f for w, f in enumerate(dbf)], out=out)
        torch.cuda.synchronize()
        assert not torch.isnan(out).any().item()
        got_b = out[sel].cpu().numpy()
        del out
        ref, _ = oracle_rows(st.idx, st.val, st.dims, factors, d, rows)
        ref_b, _ = oracle_rows(st.idx, st.val, st.dims, factors, d, rows, transform=bf16_round)
        e, eb, ebf = oracle.rel_fro(got, ref), oracle.rel_fro(got_b, ref_b), oracle.rel_fro(got_b, ref)
        log("R=64 mode %d: fp32 rel %.2e; bf16 rel %.2e vs oracle on bf16-rounded factors, %.2e vs fp32 factors" %
            (d, e, eb, ebf))
        assert e <= 1e-5 and eb <= 1e-5 and ebf <= 1e-2


def test_factor_above_4GiB_uses_64bit_gathers():
    # mode-0 factor: 40M rows x 32 fp32 = 5.1 GB, beyond 32-bit buffer offsets;
    # modes 1 and 2 gather from it (64-bit addresses), mode 0 does not
    dims = (40_000_000, 1000, 500)
    R = 32
    st = synth.tensor(dims, 2_000_000, "zipf", 1.1, 0.0, seed=12)
    T = api.Tensor(st.idx, st.val, dims)
    rng = np.random.default_rng(12)
    dfac = [torch.empty((d, R), device="cuda").uniform_(-1, 1) for d in dims]
    f64 = [f.double().cpu().numpy() for f in dfac]
    for d in range(3):
        out = torch.full((dims[d], R), float("nan"), device="cuda")
        api.mttkrp(T, d, [None if w == d else f for w, f in enumerate(dfac)], out=out)
        torch.cuda.synchronize()
        rows, _, _ = _sample_rows(st, d, rng, 300)
        got = out[torch.from_numpy(rows).cuda()].cpu().numpy()
        e = oracle.rel_fro(got, _oracle_rows(st, f64, d, rows, R))
        log("5 GB factor, mode %d: sampled rel %.2e" % (d, e))
        assert e <= 1e-5
        assert not torch.isnan(out).any().item()
    T.close()


def test_bf16_factor_above_4GiB_narrow_lanes():
    """bf16 factors at rank 32 (64-byte rows, 8-byte lanes): a 72M-row factor is
    4.6 GB, past 32-bit buffer offsets, so modes 1 and 2 gather it with 64-bit
    addresses.  The oracle sees the same bf16 values (exactly widened) on the
    rows the sampled outputs use."""
    dims = (72_000_000, 1000, 500)
    R = 32
    st = synth.tensor(dims, 2_000_000, "zipf", 1.1, 0.0, seed=13)
    T = api.Tensor(st.idx, st.val, dims)
    rng = np.random.default_rng(13)
    dbf = []
    for d in dims:
        f = torch.empty((d, R), device="cuda").uniform_(-1, 1)
        dbf.append(f.to(torch.bfloat16))
        del f
    for d in (1, 2):
        out = torch.full((dims[d], R), float("nan"), device="cuda")
        api.mttkrp_bf16(T, d, [None if w == d else f for w, f in enumerate(dbf)], out=out)
        torch.cuda.synchronize()
        rows, _, _ = _sample_rows(st, d, rng, 200)
        got = out[torch.from_numpy(rows).cuda()].cpu().numpy()
        m = np.isin(st.idx[d], rows)
        sub = st.idx[:, m].astype(np.int64)
        fs, cdims = [], []
        for w in range(3):
            if w == d:
                sub[w] = np.searchsorted(rows, sub[w])
                fs.append(np.zeros((rows.size, R)))
                cdims.append(rows.size)
            else:
                used = np.unique(sub[w])
                fs.append(dbf[w][torch.from_numpy(used).cuda()].float().double().cpu().numpy())
                sub[w] = np.searchsorted(used, sub[w])
                cdims.append(used.size)
        ref = oracle.mttkrp(sub.astype(np.int32), st.val[m], cdims, fs, d)
        e = oracle.rel_fro(got, ref)
        log("4.6 GB bf16 factor, mode %d: sampled rel %.2e" % (d, e))
        assert e <= 1e-5
        assert not torch.isnan(out).any().item()
    T.close()


def test_index_space_at_the_int32_limit():
    """Mode 0 spans the largest index space the ABI accepts (2^31 - 1 rows).
    At rank 8 its factor and its output are 68.7 GB each, and rows near the top of
    the index space sit 68 GB into them.  Nearly all 2^31 output rows are
    untouched, which gives the init kernel about a million gap ranges.  Checked:
    - every output row is written (NaN prefill);
    - exactly the touched rows are nonzero;
    - sampled rows match the oracle on the factor rows they use: the first and
      last indices, rows from the dense top 5M of the index space, and random ones."""
    torch.cuda.empty_cache()
    free, _ = torch.cuda.mem_get_info()
    if free < 200e9:
        pytest.skip("needs about 160 GB of free device memory")
    I0 = 2**31 - 1
    dims = (I0, 3000, 2000)
    R = 8
    rng = np.random.default_rng(31)
    n = 200_000
    i0 = np.concatenate([[0, 1, I0 - 2, I0 - 1], rng.integers(I0 - 5_000_000, I0, 100_000),
                         rng.integers(0, I0, n - 100_004)])
    idx = np.stack([i0, rng.integers(0, dims[1], n), rng.integers(0, dims[2], n)]).astype(np.int32)
    val = rng.random(n).astype(np.float32) + 0.5
    log("int32-limit index space: building layouts")
    T = api.Tensor(idx, val, dims)
    dfac = [torch.empty((d, R), device="cuda").uniform_(-1, 1) for d in dims]
    block = 1 << 28
    for d in range(3):
        out = torch.full((dims[d], R), float("nan"), device="cuda")
        api.mttkrp(T, d, [None if w == d else f for w, f in enumerate(dfac)], out=out)
        torch.cuda.synchronize()
        nan_rows = nonzero_rows = 0
        for a in range(0, dims[d], block):
            part = out[a:a + block]
            nan_rows += int(torch.isnan(part).any(dim=1).sum().item())
            nonzero_rows += int((part != 0).any(dim=1).sum().item())
        touched = np.unique(idx[d])
        log("int32-limit mode %d: %d rows, %d touched, %d nonzero rows, %d NaN rows" %
            (d, dims[d], touched.size, nonzero_rows, nan_rows))
        assert nan_rows == 0
        assert nonzero_rows == touched.size
        pick = rng.choice(touched, size=min(300, touched.size), replace=False)
        rows = np.unique(np.concatenate([pick, touched[:2], touched[-2:]]))
        got = out[torch.from_numpy(rows.astype(np.int64)).cuda()].cpu().numpy()
        del out
        m = np.isin(idx[d], rows)
        sub = idx[:, m].astype(np.int64)
        fs, cdims = [], []
        for w in range(3):
            if w == d:
                sub[w] = np.searchsorted(rows, sub[w])
                fs.append(np.zeros((rows.size, R)))
                cdims.append(rows.size)
            else:
                used = np.unique(sub[w])
                fs.append(dfac[w][torch.from_numpy(used).cuda()].double().cpu().numpy())
                sub[w] = np.searchsorted(used, sub[w])
                cdims.append(used.size)
        e = oracle.rel_fro(got, oracle.mttkrp(sub.astype(np.int32), val[m], cdims, fs, d))
        log("int32-limit mode %d: sampled rel %.2e (rows %d..%d)" % (d, e, rows[0], rows[-1]))
        assert e <= 1e-5
        torch.cuda.empty_cache()
    T.close()
    del dfac
    torch.cuda.empty_cache()


def test_largest_nonzero_count_in_chunks_of_one():
    """2^31 - 1 nonzeros, the most the ABI accepts, in chunks of one nonzero:
    2^31 - 1 work-queue chunks, the largest count the queue counters meet.
    Mode 0 has 2^31 - 1 rows with one nonzero each, so each chunk stores one
    whole row.  Only mode 0 is computed here.  In modes 1 and 2 every row has
    thousands of one-nonzero chunks, all added atomically into the same row.
    The inputs are integers, so every output value is exact.  Checked:
    - no row is left unwritten (NaN prefill);
    - the column sums of the whole output equal int64 sums of the per-nonzero
      terms;
    - sampled rows equal the oracle bit for bit."""
    torch.cuda.empty_cache()
    free, _ = torch.cuda.mem_get_info()
    if free < 240e9:
        pytest.skip("needs about 200 GB of free device memory")
    nnz = 2**31 - 1
    dims = (nnz, 1 << 19, 1 << 14)
    R = 8
    idx = np.empty((3, nnz), np.int32)
    val = np.empty(nnz, np.float32)
    step = 1 << 27
    for a in range(0, nnz, step):
        k = np.arange(a, min(a + step, nnz), dtype=np.int64)
        idx[0, a:a + k.size] = k
        idx[1, a:a + k.size] = (k * 40503 + k // 977) % dims[1]
        idx[2, a:a + k.size] = (k * 69069 + 12345) % dims[2]
        val[a:a + k.size] = (k % 3 + 1).astype(np.float32)
    rng = np.random.default_rng(7)
    fac = [None] + [rng.integers(-2, 3, (d, R)).astype(np.float32) for d in dims[1:]]
    log("2^31 - 1 nonzeros, chunks of one: building layouts")
    T = api.Tensor(idx, val, dims, chunk_nnz=1)
    assert T.n_chunks == nnz
    dfac = [None] + [torch.from_numpy(f).cuda() for f in fac[1:]]
    out = torch.full((nnz, R), float("nan"), device="cuda")
    api.mttkrp(T, 0, dfac, out=out)
    torch.cuda.synchronize()
    log("mode 0 done; checking")
    # column sums: output (exact integers in fp32, summed in fp64) against int64 terms
    got_sum = torch.zeros(R, dtype=torch.float64, device="cuda")
    nan_rows = 0
    for a in range(0, nnz, step):
        part = out[a:a + step]
        nan_rows += int(torch.isnan(part).any(dim=1).sum().item())
        got_sum += part.double().sum(dim=0)
    assert nan_rows == 0
    f1 = dfac[1].long()
    f2 = dfac[2].long()
    ref_sum = torch.zeros(R, dtype=torch.int64, device="cuda")
    for a in range(0, nnz, 1 << 25):
        b = min(a + (1 << 25), nnz)
        i1 = torch.from_numpy(idx[1, a:b]).cuda().long()
        i2 = torch.from_numpy(idx[2, a:b]).cuda().long()
        v = torch.from_numpy(val[a:b]).cuda().long()
        ref_sum += (v[:, None] * f1[i1] * f2[i2]).sum(dim=0)
    log("column sums %s (int64 terms %s)" % (got_sum.cpu().numpy(), ref_sum.cpu().numpy()))
    assert torch.equal(got_sum, ref_sum.double())
    rows = np.unique(np.concatenate([[0, 1, nnz - 2, nnz - 1], rng.integers(0, nnz, 300)]))
    got = out[torch.from_numpy(rows).cuda()].cpu().numpy()
    del out
    sub = idx[:, rows].astype(np.int64)
    fs, cdims = [np.zeros((rows.size, R))], [rows.size]
    sub[0] = np.arange(rows.size)
    for w in (1, 2):
        used = np.unique(sub[w])
        fs.append(fac[w][used].astype(np.float64))
        sub[w] = np.searchsorted(used, sub[w])
        cdims.append(used.size)
    ref = oracle.mttkrp(sub.astype(np.int32), val[rows], cdims, fs, 0).astype(np.float32)
    np.testing.assert_array_equal(got, ref)
    T.close()
    torch.cuda.empty_cache()


def test_bf16_factor_above_4GiB_order_4_wide_lanes():
    """bf16 factors at rank 32 with three gathered factors (order 4): 64-byte rows
    gathered with 16-byte lanes.  A 72M-row factor is 4.6 GB, past 32-bit buffer
    offsets, so modes 1-3 gather it with 64-bit addresses.  The oracle sees the
    same bf16 values (exactly widened) on the rows the sampled outputs use."""
    dims = (72_000_000, 1000, 500, 300)
    R = 32
    st = synth.tensor(dims, 2_000_000, "zipf", 1.1, 0.0, seed=14)
    T = api.Tensor(st.idx, st.val, dims)
    rng = np.random.default_rng(14)
    dbf = []
    for d in dims:
        f = torch.empty((d, R), device="cuda").uniform_(-1, 1)
        dbf.append(f.to(torch.bfloat16))
        del f
    for d in (1, 2, 3):
        out = torch.full((dims[d], R), float("nan"), device="cuda")
        api.mttkrp_bf16(T, d, [None if w == d else f for w, f in enumerate(dbf)], out=out)
        torch.cuda.synchronize()
        rows, _, _ = _sample_rows(st, d, rng, 200)
        got = out[torch.from_numpy(rows).cuda()].cpu().numpy()
        m = np.isin(st.idx[d], rows)
        sub = st.idx[:, m].astype(np.int64)
        fs, cdims = [], []
        for w in range(4):
            if w == d:
                sub[w] = np.searchsorted(rows, sub[w])
                fs.append(np.zeros((rows.size, R)))
                cdims.append(rows.size)
            else:
                used = np.unique(sub[w])
                fs.append(dbf[w][torch.from_numpy(used).cuda()].float().double().cpu().numpy())
                sub[w] = np.searchsorted(used, sub[w])
                cdims.append(used.size)
        ref = oracle.mttkrp(sub.astype(np.int32), st.val[m], cdims, fs, d)
        e = oracle.rel_fro(got, ref)
        log("4.6 GB bf16 factor, order 4, mode %d: sampled rel %.2e" % (d, e))
        assert e <= 1e-5
        assert not torch.isnan(out).any().item()
    T.close()
