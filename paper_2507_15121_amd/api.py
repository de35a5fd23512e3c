"""Thin Python binding of the C ABI in ``include/amped.h`` (ctypes).

Argument marshalling only: every step of MTTKRP, the bf16 form, the CP loss
and the fused gradient runs in ``libamped.so``'s HIP kernels.  PyTorch
provides device memory (tensors) and streams.  If the library is not built,
every call raises; there is no fallback.
"""
import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# AMPED_LIB selects another build of the same library (e.g. a tuning variant)
LIB_PATH = os.environ.get("AMPED_LIB") or os.path.join(_HERE, "libamped.so")

OK, ERR_INVALID, ERR_RANGE, ERR_NOMEM, ERR_HIP, ERR_UNSUPPORTED = range(6)
STATUS_NAMES = {0: "OK", 1: "INVALID", 2: "RANGE", 3: "NOMEM", 4: "HIP", 5: "UNSUPPORTED"}

# every symbol declared in include/amped.h
EXPORTED = ["amped_tensor_create", "amped_tensor_destroy", "amped_tensor_info", "amped_tensor_layout",
            "amped_layout_host", "amped_mttkrp", "amped_mttkrp_bf16", "amped_cp_loss", "amped_cp_grad",
            "amped_cp_loss_grad", "amped_gram", "amped_gram_noalloc", "amped_cp_als_sweep", "amped_last_error", "amped_version"]


class AmpedError(RuntimeError):
    def __init__(self, status, message):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), message))
        self.status = status
        self.message = message


class _Options(ctypes.Structure):
    _fields_ = [("chunk_nnz", ctypes.c_int64), ("device_byte_cap", ctypes.c_int64),
                ("keep_perm", ctypes.c_int32), ("host_layout", ctypes.c_int32), ("shard_nnz", ctypes.c_int64)]


_lib = None


def lib():
    """The loaded C library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libamped.so is not built (run __graft_entry__.build()); "
                               "there is no fallback path")
        L = ctypes.CDLL(LIB_PATH)
        vp, i64, i32, pvp = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.POINTER(ctypes.c_void_p)
        L.amped_tensor_create.argtypes = [i32, vp, i64, vp, vp, ctypes.POINTER(_Options), ctypes.POINTER(vp)]
        L.amped_tensor_destroy.argtypes = [vp]
        L.amped_tensor_info.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp]
        L.amped_tensor_layout.argtypes = [vp, i32, vp, vp, vp, vp, vp]
        L.amped_layout_host.argtypes = [i32, vp, i64, vp, i32, i64, vp, vp]
        L.amped_mttkrp.argtypes = [vp, i32, i32, pvp, vp, vp]
        L.amped_mttkrp_bf16.argtypes = [vp, i32, i32, pvp, vp, vp]
        L.amped_cp_loss.argtypes = [vp, i32, pvp, vp, vp]
        L.amped_cp_grad.argtypes = [vp, i32, i32, pvp, ctypes.c_float, vp, vp]
        L.amped_cp_loss_grad.argtypes = [vp, i32, i32, pvp, ctypes.c_float, vp, vp, vp]
        L.amped_gram.argtypes = [vp, i64, i32, vp, vp]
        L.amped_gram_noalloc.argtypes = [vp, i64, i32, vp, vp]
        L.amped_cp_als_sweep.argtypes = [vp, i32, pvp, vp, vp, ctypes.c_uint, vp]
        for name in EXPORTED:
            if name not in ("amped_last_error", "amped_version"):
                getattr(L, name).restype = ctypes.c_int
        L.amped_last_error.restype = ctypes.c_char_p
        L.amped_last_error.argtypes = []
        L.amped_version.restype = ctypes.c_char_p
        L.amped_version.argtypes = []
        _lib = L
    return _lib


def _check(status):
    if status != OK:
        raise AmpedError(status, lib().amped_last_error().decode())


def version():
    return lib().amped_version().decode()


def _host_coo(indices, values, dims):
    idx = indices
    if hasattr(idx, "detach"):
        idx = idx.detach().cpu().numpy()
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    if idx.ndim != 2:
        raise ValueError("indices must be [order][nnz]")
    val = values
    if val is not None and hasattr(val, "detach"):
        val = val.detach().cpu().numpy()
    val = np.ascontiguousarray(val, dtype=np.float32) if val is not None else None
    d = np.ascontiguousarray(dims, dtype=np.int64)
    return idx, val, d


def layout_host(indices, dims, mode, chunk_nnz):
    """Host-only layout build: (perm int32 [nnz], chunk flags uint8)."""
    idx, _, d = _host_coo(indices, None, dims)
    order, nnz = idx.shape
    perm = np.empty(nnz, dtype=np.int32)
    flags = np.empty((nnz + chunk_nnz - 1) // chunk_nnz, dtype=np.uint8)
    _check(lib().amped_layout_host(order, d.ctypes.data, nnz, idx.ctypes.data if nnz else None,
                                   int(mode), int(chunk_nnz), perm.ctypes.data, flags.ctypes.data))
    return perm, flags


class Tensor:
    """A sparse tensor whose per-mode layouts live on the current HIP device,
    or (host_layout=True) in pinned host memory, streamed to the device in
    shards of shard_nnz nonzeros on every call."""

    def __init__(self, indices, values, dims, chunk_nnz=0, keep_perm=False, device_byte_cap=0,
                 host_layout=False, shard_nnz=0):
        idx, val, d = _host_coo(indices, values, dims)
        order, nnz = idx.shape
        if val.shape != (nnz,):
            raise ValueError("values must have one entry per nonzero")
        opts = _Options(int(chunk_nnz), int(device_byte_cap), 1 if keep_perm else 0, 1 if host_layout else 0,
                        int(shard_nnz))
        h = ctypes.c_void_p()
        self._h = None
        _check(lib().amped_tensor_create(order, d.ctypes.data, nnz, idx.ctypes.data if nnz else None,
                                         val.ctypes.data if nnz else None, ctypes.byref(opts),
                                         ctypes.byref(h)))
        self._h = h
        self.order = order
        self.dims = tuple(int(x) for x in d)
        self.nnz = nnz
        o = ctypes.c_int()
        ch, nc, dev_bytes = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        touched = np.zeros(order, dtype=np.int64)
        _check(lib().amped_tensor_info(self._h, ctypes.byref(o), None, None, ctypes.byref(ch), ctypes.byref(nc),
                                       touched.ctypes.data, ctypes.byref(dev_bytes)))
        self.chunk_nnz = ch.value
        self.n_chunks = nc.value
        self.touched = tuple(int(x) for x in touched)
        self.device_bytes = dev_bytes.value

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("tensor is closed")
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None:
            h, self._h = self._h, None
            _check(lib().amped_tensor_destroy(h))

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def layout(self, mode, perm=False):
        """Copy a mode's device layout to host numpy arrays."""
        n = self.nnz
        out = {"out_idx": np.empty(n, np.int32), "in_idx": np.empty((self.order - 1, n), np.int32),
               "values": np.empty(n, np.float32), "flags": np.empty(self.n_chunks, np.uint8)}
        p = np.empty(n, np.int32) if perm else None
        _check(lib().amped_tensor_layout(self.handle, int(mode), p.ctypes.data if perm else None,
                                         out["out_idx"].ctypes.data, out["in_idx"].ctypes.data,
                                         out["values"].ctypes.data, out["flags"].ctypes.data))
        if perm:
            out["perm"] = p
        return out


# ------------------------------------------------------------------ device calls

def _torch():
    import torch
    return torch


def _stream_ptr(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr_array(t: Tensor, factors: Sequence, dtype, skip: Optional[int]):
    torch = _torch()
    if len(factors) != t.order:
        raise ValueError("need one factor per mode (%d), got %d" % (t.order, len(factors)))
    ptrs = (ctypes.c_void_p * t.order)()
    rank = None
    for w, f in enumerate(factors):
        if w == skip and f is None:
            ptrs[w] = None
            continue
        if not isinstance(f, torch.Tensor) or not f.is_cuda:
            raise TypeError("factor %d must be a CUDA/HIP torch tensor" % w)
        if f.dtype != dtype or f.dim() != 2 or not f.is_contiguous():
            raise ValueError("factor %d must be a contiguous 2-D %s tensor" % (w, dtype))
        if f.shape[0] != t.dims[w]:
            raise ValueError("factor %d has %d rows, mode size is %d" % (w, f.shape[0], t.dims[w]))
        if rank is None:
            rank = int(f.shape[1])
        elif f.shape[1] != rank:
            raise ValueError("factors disagree on the rank")
        ptrs[w] = f.data_ptr()
    return ptrs, rank


def _out(t, mode, rank, out, like):
    torch = _torch()
    if out is None:
        out = torch.empty((t.dims[mode], rank), dtype=torch.float32, device=like.device)
    if out.dtype != torch.float32 or not out.is_contiguous() or tuple(out.shape) != (t.dims[mode], rank):
        raise ValueError("output must be a contiguous float32 tensor of shape %s" % ((t.dims[mode], rank),))
    return out


def _first(factors, skip):
    return next(f for w, f in enumerate(factors) if w != skip or f is not None)


def mttkrp(t: Tensor, mode: int, factors, out=None, stream=None):
    """fp32 MTTKRP along ``mode``; factors[mode] may be None."""
    torch = _torch()
    ptrs, rank = _ptr_array(t, factors, torch.float32, mode)
    out = _out(t, mode, rank, out, _first(factors, mode))
    _check(lib().amped_mttkrp(t.handle, int(mode), rank, ptrs, ctypes.c_void_p(out.data_ptr()),
                              _stream_ptr(stream)))
    return out


def mttkrp_bf16(t: Tensor, mode: int, factors, out=None, stream=None):
    """MTTKRP with bfloat16 factors (torch.bfloat16 tensors), fp32 output."""
    torch = _torch()
    ptrs, rank = _ptr_array(t, factors, torch.bfloat16, mode)
    out = _out(t, mode, rank, out, _first(factors, mode))
    _check(lib().amped_mttkrp_bf16(t.handle, int(mode), rank, ptrs, ctypes.c_void_p(out.data_ptr()),
                                   _stream_ptr(stream)))
    return out


def cp_loss(t: Tensor, factors, out=None, stream=None):
    """Sparse CP loss as a 0-dim float64 device tensor."""
    torch = _torch()
    ptrs, rank = _ptr_array(t, factors, torch.float32, None)
    if out is None:
        out = torch.empty((), dtype=torch.float64, device=factors[0].device)
    if out.dtype != torch.float64 or out.numel() != 1:
        raise ValueError("loss output must be one float64")
    _check(lib().amped_cp_loss(t.handle, rank, ptrs, ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)))
    return out


def cp_grad(t: Tensor, mode: int, factors, scale: float, out=None, stream=None):
    """scale * MTTKRP_mode(residuals); scale = -2 * dL gives dL * dLoss/dA_mode."""
    torch = _torch()
    ptrs, rank = _ptr_array(t, factors, torch.float32, None)
    out = _out(t, mode, rank, out, factors[0])
    _check(lib().amped_cp_grad(t.handle, int(mode), rank, ptrs, ctypes.c_float(scale),
                               ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)))
    return out


def cp_loss_grad(t: Tensor, mode: int, factors, scale: float, out=None, loss=None, stream=None):
    """cp_grad() and cp_loss() in one pass over the mode's layout: returns
    (loss as a 0-dim float64 device tensor, scale * MTTKRP_mode(residuals))."""
    torch = _torch()
    ptrs, rank = _ptr_array(t, factors, torch.float32, None)
    out = _out(t, mode, rank, out, factors[0])
    if loss is None:
        loss = torch.empty((), dtype=torch.float64, device=factors[0].device)
    if loss.dtype != torch.float64 or loss.numel() != 1:
        raise ValueError("loss output must be one float64")
    _check(lib().amped_cp_loss_grad(t.handle, int(mode), rank, ptrs, ctypes.c_float(scale),
                                    ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(loss.data_ptr()),
                                    _stream_ptr(stream)))
    return loss, out


def gram(A, out=None, stream=None):
    """A^T A (float64, rank x rank) of a contiguous 2-D float32 device tensor."""
    torch = _torch()
    if not isinstance(A, torch.Tensor) or not A.is_cuda or A.dtype != torch.float32 or A.dim() != 2 \
            or not A.is_contiguous():
        raise ValueError("A must be a contiguous 2-D float32 CUDA/HIP tensor")
    rank = int(A.shape[1])
    if out is None:
        out = torch.empty((rank, rank), dtype=torch.float64, device=A.device)
    if out.dtype != torch.float64 or tuple(out.shape) != (rank, rank) or not out.is_contiguous():
        raise ValueError("out must be a contiguous (rank, rank) float64 tensor")
    _check(lib().amped_gram(ctypes.c_void_p(A.data_ptr()), int(A.shape[0]), rank, ctypes.c_void_p(out.data_ptr()),
                            _stream_ptr(stream)))
    return out


def gram_noalloc(A, out, stream=None):
    """A^T A like gram(), through the entry point that allocates nothing (its
    partial sums use the library's fixed device array); `out` is required."""
    torch = _torch()
    if not isinstance(A, torch.Tensor) or not A.is_cuda or A.dtype != torch.float32 or A.dim() != 2 \
            or not A.is_contiguous():
        raise ValueError("A must be a contiguous 2-D float32 CUDA/HIP tensor")
    rank = int(A.shape[1])
    if out.dtype != torch.float64 or tuple(out.shape) != (rank, rank) or not out.is_contiguous():
        raise ValueError("out must be a contiguous (rank, rank) float64 tensor")
    _check(lib().amped_gram_noalloc(ctypes.c_void_p(A.data_ptr()), int(A.shape[0]), rank,
                                    ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)))
    return out


ALS_REUSE_GRAMS = 1


def cp_als_sweep(t: Tensor, factors, lam=None, fit=None, reuse_grams=False, stream=None):
    """One CP-ALS sweep over all modes; factors (float32 device tensors) are
    updated in place.  Returns (lambda, fit) as float64 device tensors.
    reuse_grams: the factors are exactly what the previous sweep on this
    tensor left, so its Gram matrices are reused."""
    torch = _torch()
    ptrs, rank = _ptr_array(t, factors, torch.float32, None)
    dev = factors[0].device
    if lam is None:
        lam = torch.empty(rank, dtype=torch.float64, device=dev)
    if fit is None:
        fit = torch.empty((), dtype=torch.float64, device=dev)
    if lam.dtype != torch.float64 or lam.numel() != rank or fit.dtype != torch.float64 or fit.numel() != 1:
        raise ValueError("lambda must hold rank float64 values and fit one float64")
    _check(lib().amped_cp_als_sweep(t.handle, rank, ptrs, ctypes.c_void_p(lam.data_ptr()),
                                    ctypes.c_void_p(fit.data_ptr()), ALS_REUSE_GRAMS if reuse_grams else 0,
                                    _stream_ptr(stream)))
    return lam, fit
