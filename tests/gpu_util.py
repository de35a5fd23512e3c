"""Shared helpers for the GPU tests: run the HIP path through the C ABI and
the oracle on the same seeded inputs."""
import sys

import numpy as np

import oracle


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def torch_mod():
    import torch
    return torch


def dev_factors(factors, dtype=None):
    torch = torch_mod()
    out = []
    for f in factors:
        t = torch.from_numpy(np.ascontiguousarray(f, dtype=np.float32)).cuda()
        if dtype is not None:
            t = t.to(dtype)
        out.append(t.contiguous())
    return out


def nan_out(rows, rank):
    torch = torch_mod()
    return torch.full((rows, rank), float("nan"), dtype=torch.float32, device="cuda")


def hip_mttkrp(t, mode, dfac, bf16=False, stream=None):
    from paper_2507_15121_amd import api
    torch = torch_mod()
    rank = dfac[0].shape[1]
    out = nan_out(t.dims[mode], rank)
    f = [None if w == mode else x for w, x in enumerate(dfac)]
    if bf16:
        api.mttkrp_bf16(t, mode, f, out=out, stream=stream)
    else:
        api.mttkrp(t, mode, f, out=out, stream=stream)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def oracle_mttkrp(idx, val, dims, factors, mode):
    return oracle.mttkrp(idx, np.asarray(val, np.float64), dims,
                         [np.asarray(f, np.float64) for f in factors], mode)


def rel(a, b):
    return oracle.rel_fro(a, b)


def _compact_inputs(idx, dims, factors, d, rows, transform):
    """The nonzeros whose mode-d index is in `rows` (sorted, unique), with the
    mode-d index relabelled to its position in `rows` and every other mode's
    index relabelled to the rows of a compacted factor that holds only the rows
    those nonzeros use (passed through `transform`, then upcast to float64).
    The compacted problem has the same per-nonzero terms as the full one."""
    sel = np.zeros(int(dims[d]), dtype=bool)
    sel[rows] = True
    m = np.flatnonzero(sel[idx[d]])
    sub = idx[:, m].astype(np.int32)
    sub[d] = np.searchsorted(rows, sub[d]).astype(np.int32)
    cdims = list(dims)
    cdims[d] = rows.size
    R = factors[0].shape[1]
    fs = []
    for w in range(len(dims)):
        if w == d:
            fs.append(None)
            continue
        used = np.zeros(int(dims[w]), dtype=bool)
        used[sub[w]] = True
        keep = np.flatnonzero(used)
        lut = np.zeros(int(dims[w]), dtype=np.int32)
        lut[keep] = np.arange(keep.size, dtype=np.int32)
        sub[w] = lut[sub[w]]
        cdims[w] = max(1, keep.size)
        f = np.asarray(factors[w][keep])
        fs.append((transform(f) if transform else f).astype(np.float64) if keep.size else np.zeros((1, R)))
    return m, sub, cdims, fs


def oracle_rows(idx, val, dims, factors, d, rows, transform=None, own=None, threads=16):
    """FP64 oracle MTTKRP of mode d on the output rows `rows` only (sorted,
    unique): returns a rows.size x R array.  The nonzeros of those rows are
    split into `threads` pieces by position, each runs through the unchanged
    sequential oracle on its own thread, and the pieces are added in fp64
    (MTTKRP is linear in the tensor's values, so only the fp64 summation order
    changes).  `transform` maps factor rows before the upcast (e.g. bf16
    rounding by the oracle's own routine)."""
    import concurrent.futures
    rows = np.asarray(rows, dtype=np.int64)
    m, sub, cdims, fs = _compact_inputs(idx, dims, factors, d, rows, transform)
    R = factors[0].shape[1]
    fs[d] = np.zeros((rows.size, R))
    v = np.asarray(val)[m]
    bounds = np.linspace(0, m.size, threads + 1).astype(np.int64)
    with concurrent.futures.ThreadPoolExecutor(threads) as pool:
        parts = list(pool.map(lambda i: oracle.mttkrp(sub[:, bounds[i]:bounds[i + 1]], v[bounds[i]:bounds[i + 1]],
                                                      cdims, fs, d), range(threads)))
    return np.sum(parts, axis=0), int(m.size)


def oracle_grad_rows(idx, val, dims, factors, d, rows, threads=16):
    """FP64 oracle gradient -2 MTTKRP_d(E) of the CP loss on the output rows
    `rows` only: the residuals e_k = x_k - sum_r prod_w A_w[i_w(k), r] of those
    rows' nonzeros (each depends on its own coordinates only) and their MTTKRP,
    pieces by position on threads, added in fp64."""
    import concurrent.futures
    rows = np.asarray(rows, dtype=np.int64)
    m, sub, cdims, fs = _compact_inputs(idx, dims, factors, d, rows, None)
    fs[d] = np.asarray(factors[d][rows], dtype=np.float64)
    v = np.asarray(val)[m]
    bounds = np.linspace(0, m.size, threads + 1).astype(np.int64)

    def piece(i):
        a, b = bounds[i], bounds[i + 1]
        return oracle.cp_grad(sub[:, a:b], v[a:b], cdims, fs, d)
    with concurrent.futures.ThreadPoolExecutor(threads) as pool:
        parts = list(pool.map(piece, range(threads)))
    return np.sum(parts, axis=0)


def oracle_loss(idx, val, factors, threads=16):
    """FP64 oracle CP loss, pieces of the nonzeros by position on threads, the
    piece losses added in fp64 (only the fp64 summation order changes)."""
    import concurrent.futures
    nnz = idx.shape[1]
    bounds = np.linspace(0, nnz, threads + 1).astype(np.int64)
    f64 = [np.asarray(f, dtype=np.float64) for f in factors]

    def piece(i):
        a, b = bounds[i], bounds[i + 1]
        return oracle.cp_loss(idx[:, a:b], val[a:b], f64)[0]
    with concurrent.futures.ThreadPoolExecutor(threads) as pool:
        return float(sum(pool.map(piece, range(threads))))


def sample_rows(idx_d, dim, rng, n, extra=()):
    """n random touched rows of one mode plus its heaviest row and `extra`,
    sorted; also the per-row counts and the untouched rows."""
    counts = np.bincount(idx_d, minlength=dim)
    touched = np.flatnonzero(counts)
    rows = rng.choice(touched, size=min(n, touched.size), replace=False)
    rows = np.unique(np.concatenate([rows, [int(np.argmax(counts))], np.asarray(extra, dtype=np.int64)]))
    return rows, counts, np.flatnonzero(counts == 0)
