"""CPU oracle for sparse MTTKRP, the sparse CP loss and its gradient.

TEST INFRASTRUCTURE.  Only the tests, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It shares no code
with the HIP path and never imports the product package.

Everything is computed in float64 from exactly upcast inputs:

* ``mttkrp``       -- the per-nonzero definition in ``mttkrp_ref.c``
                      (Eq. 1, Sec. 2.1, accumulated as the elementwise
                      computation "EC" of Sec. 3 into a zeroed output).
* ``cp_loss``      -- sum over nonzeros of (x - CP model)^2 (CP model, Sec. 2.1).
* ``cp_grad``      -- dL/dA_d = -2 * MTTKRP_d(E), E the sparse residual tensor
                      on the same pattern (differentiate the loss above; the
                      inner sum over nonzeros is Eq. 1 with values e_k).
* ``layout``       -- per-mode order of the nonzeros (all nonzeros of one
                      output index together, Sec. 3.1 tensor sharding), keyed by
                      (i_d, then the other indices in ascending mode order),
                      stable for exact duplicates; fixed-size chunks stand for
                      the equal-size inter-shard partitions of Sec. 3.1/3.2.
* ``bf16_rne``     -- IEEE round-to-nearest-even to bfloat16, on bit patterns.
* dense helpers    -- explicit unfolding and Khatri-Rao product (Table 1
                      notation, Sec. 2.1 matricization) for brute-force pins.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        _lib = _configure(ctypes.CDLL(_LIB_PATH))
    return _lib


def _configure(lib):
    """Declare the C signatures on a loaded oracle library."""
    pp = ctypes.POINTER(ctypes.c_void_p)
    lib.oracle_mttkrp.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_int64,
                                  ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                  ctypes.c_int, pp, ctypes.c_void_p]
    lib.oracle_mttkrp.restype = None
    lib.oracle_cp_model.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_void_p,
                                    ctypes.c_int, pp, ctypes.c_void_p]
    lib.oracle_cp_model.restype = None
    lib.oracle_cp_loss.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_void_p,
                                   ctypes.c_void_p, ctypes.c_int, pp, ctypes.c_void_p]
    lib.oracle_cp_loss.restype = ctypes.c_double
    return lib


def _prep(idx, val, factors):
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    if idx.ndim != 2:
        raise ValueError("idx must be [order][nnz]")
    val = np.ascontiguousarray(val, dtype=np.float64)
    fs = [np.ascontiguousarray(f, dtype=np.float64) for f in factors]
    R = fs[0].shape[1]
    for f in fs:
        if f.ndim != 2 or f.shape[1] != R:
            raise ValueError("factors must all be [I_w][R]")
    ptrs = (ctypes.c_void_p * len(fs))(*[f.ctypes.data for f in fs])
    return idx, val, fs, R, ptrs


def mttkrp(idx, val, dims, factors, mode):
    """float64 MTTKRP along ``mode``; returns a dims[mode] x R array."""
    lib = _load()
    idx, val, fs, R, ptrs = _prep(idx, val, factors)
    order, nnz = idx.shape
    d = np.ascontiguousarray(dims, dtype=np.int64)
    out = np.empty((int(d[mode]), R), dtype=np.float64)
    lib.oracle_mttkrp(order, d.ctypes.data, nnz, idx.ctypes.data, val.ctypes.data,
                      int(mode), R, ctypes.cast(ptrs, ctypes.POINTER(ctypes.c_void_p)),
                      out.ctypes.data)
    return out


def cp_model(idx, factors):
    """float64 CP model value at every stored coordinate."""
    lib = _load()
    idx, _, fs, R, ptrs = _prep(idx, np.zeros(1), factors)
    order, nnz = idx.shape
    out = np.empty(nnz, dtype=np.float64)
    lib.oracle_cp_model(order, nnz, idx.ctypes.data, R,
                        ctypes.cast(ptrs, ctypes.POINTER(ctypes.c_void_p)), out.ctypes.data)
    return out


def cp_loss(idx, val, factors):
    """Return (L, residuals) with L = sum_k (x_k - xhat_k)^2 in float64."""
    lib = _load()
    idx, val, fs, R, ptrs = _prep(idx, val, factors)
    order, nnz = idx.shape
    resid = np.empty(nnz, dtype=np.float64)
    loss = lib.oracle_cp_loss(order, nnz, idx.ctypes.data, val.ctypes.data, R,
                              ctypes.cast(ptrs, ctypes.POINTER(ctypes.c_void_p)),
                              resid.ctypes.data)
    return float(loss), resid


def cp_grad(idx, val, dims, factors, mode, grad_out=1.0):
    """dL/dA_mode times grad_out, i.e. -2 * grad_out * MTTKRP_mode(residuals)."""
    _, resid = cp_loss(idx, val, factors)
    return -2.0 * float(grad_out) * mttkrp(idx, resid, dims, factors, mode)


# ----------------------------------------------------------------------------
# layout oracle

def layout(idx, mode, chunk_nnz):
    """Per-mode nonzero order and chunk table.

    Returns a dict with ``perm`` (int64, position -> input nonzero),
    ``out_idx``, ``in_idx`` ([order-1][nnz], other modes ascending),
    ``flags`` (uint8 per chunk: bit0 = chunk's first row continues from the
    previous chunk, bit1 = chunk's last row continues into the next chunk) and
    ``n_chunks``.
    """
    idx = np.asarray(idx)
    order, nnz = idx.shape
    others = [w for w in range(order) if w != mode]
    # np.lexsort: the LAST key is the primary key; it is a stable sort, so
    # exact duplicates keep their input order.
    keys = [idx[w] for w in reversed(others)] + [idx[mode]]
    perm = np.lexsort(keys).astype(np.int64) if nnz else np.zeros(0, np.int64)
    out_idx = idx[mode][perm]
    in_idx = np.stack([idx[w][perm] for w in others]) if others else np.zeros((0, nnz), idx.dtype)
    CH = int(chunk_nnz)
    n_chunks = (nnz + CH - 1) // CH
    flags = np.zeros(n_chunks, dtype=np.uint8)
    for k in range(n_chunks):
        s = k * CH
        e = min(s + CH, nnz)
        if k > 0 and out_idx[s - 1] == out_idx[s]:
            flags[k] |= 1
        if e < nnz and out_idx[e - 1] == out_idx[e]:
            flags[k] |= 2
    return {"perm": perm, "out_idx": out_idx, "in_idx": in_idx, "flags": flags,
            "n_chunks": n_chunks}


# ----------------------------------------------------------------------------
# bfloat16 rounding (IEEE round-to-nearest, ties to even, on the fp32 bits)

def bf16_rne(x):
    """float32 array -> uint16 bfloat16 bit patterns (finite inputs)."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    return ((u + 0x7FFF + lsb) >> 16).astype(np.uint16)


def bf16_to_f32(bits):
    return (np.asarray(bits, dtype=np.uint16).astype(np.uint32) << 16).view(np.float32)


# ----------------------------------------------------------------------------
# dense helpers for brute-force pins

def to_dense(idx, val, dims):
    X = np.zeros(tuple(int(d) for d in dims), dtype=np.float64)
    np.add.at(X, tuple(np.asarray(i, dtype=np.int64) for i in idx), np.asarray(val, np.float64))
    return X


def unfold(X, n, convention):
    """Mode-n matricization X_(n) (Sec. 2.1).

    The paper leaves the column order open.  ``"first_fastest"`` (Kolda and
    Bader): the lowest remaining mode varies fastest along the columns.
    ``"cyclic"``: the other modes taken in the order n+1, ..., N-1, 0, ..., n-1
    with the LAST of them varying fastest, which is the pairing of Eq. 1
    (X_(0) with B kr C, X_(1) with C kr A, X_(2) with A kr B).
    """
    N = X.ndim
    if convention == "first_fastest":
        rest = [w for w in range(N) if w != n]
        # row-major reshape makes the last axis fastest, so reverse.
        Y = np.transpose(X, [n] + rest[::-1])
    elif convention == "cyclic":
        rest = [(n + j) % N for j in range(1, N)]
        Y = np.transpose(X, [n] + rest)
    else:
        raise ValueError(convention)
    return Y.reshape(X.shape[n], -1)


def khatri_rao(mats):
    """Column-wise Kronecker product; the LAST matrix's row index is fastest."""
    R = mats[0].shape[1]
    out = np.ones((1, R))
    for M in mats:
        out = (out[:, None, :] * M[None, :, :]).reshape(-1, R)
    return out


def kr_operands(factors, n, convention):
    N = len(factors)
    if convention == "first_fastest":
        rest = [w for w in range(N) if w != n]
        return [factors[w] for w in rest[::-1]]
    rest = [(n + j) % N for j in range(1, N)]
    return [factors[w] for w in rest]


def mttkrp_dense(X, factors, n, convention):
    """Explicit X_(n) @ (Khatri-Rao of the other factors)."""
    return unfold(X, n, convention) @ khatri_rao(kr_operands(factors, n, convention))


def rel_fro(Y, Yref):
    """||Y - Yref||_F / ||Yref||_F in float64 (0 when both are exactly zero)."""
    Y = np.asarray(Y, dtype=np.float64)
    Yref = np.asarray(Yref, dtype=np.float64)
    den = np.linalg.norm(Yref)
    num = np.linalg.norm(Y - Yref)
    if den == 0.0:
        return 0.0 if num == 0.0 else float("inf")
    return float(num / den)
