"""Seeded synthetic sparse tensors and factor matrices (input generation only).

The paper measures on FROSTT Amazon / Patents / Reddit-2015 and on Twitch
(Table 3).  None of them is used here; these generators stand in for them with
the same order (3-4 modes), index-space sizes (10^5-10^8 per mode), nonzero
counts (10^8-10^9) and power-law index popularity.  The native part is
``csrc/synth.c``; this module only marshals arrays and names the workloads.

This module holds none of the MTTKRP arithmetic; both the HIP path's tests
and benchmark and the oracle's tests take their inputs from it.
"""
import ctypes
import os
from dataclasses import dataclass, field
from typing import Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libamped_synth.so")
_lib = None

DEFAULT_SEED = 250715121


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError("libamped_synth.so is not built; run __graft_entry__.build()")
        lib = ctypes.CDLL(_LIB_PATH)
        lib.synth_coords.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int,
                                     ctypes.c_double, ctypes.c_double, ctypes.c_uint64,
                                     ctypes.c_void_p, ctypes.c_void_p]
        lib.synth_coords.restype = ctypes.c_int
        lib.synth_values.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_void_p]
        lib.synth_values.restype = None
        lib.synth_factor.argtypes = [ctypes.c_uint64, ctypes.c_int, ctypes.c_int64, ctypes.c_int64,
                                     ctypes.c_void_p]
        lib.synth_factor.restype = None
        lib.synth_rank_perm.argtypes = [ctypes.c_uint64, ctypes.c_int, ctypes.c_int64, ctypes.c_void_p]
        lib.synth_rank_perm.restype = None
        lib.synth_zipf_ranks.argtypes = [ctypes.c_int64, ctypes.c_double, ctypes.c_uint64,
                                         ctypes.c_uint64, ctypes.c_int64, ctypes.c_void_p]
        lib.synth_zipf_ranks.restype = ctypes.c_int64
        _lib = lib
    return _lib


@dataclass
class Workload:
    """A named synthetic tensor recipe."""
    name: str
    dims: Tuple[int, ...]
    nnz: int
    dist: str                 # "uniform" or "zipf"
    zipf_s: float = 0.0
    hot_frac: float = 0.0     # share of nnz forced into one mode-0 slice
    rank: int = 32
    description: str = ""


WORKLOADS = {
    w.name: w for w in [
        Workload("uniform3-1000x800x600-100k", (1000, 800, 600), 100_000, "uniform", rank=16,
                 description="order 3, 100k distinct uniform coordinates, R=16"),
        Workload("zipf3-10Mx5Mx2M-200M", (10_000_000, 5_000_000, 2_000_000), 200_000_000, "zipf",
                 zipf_s=1.1, rank=32,
                 description="order 3, 200M nnz, Zipf(1.1) per mode, duplicates merged, R=32"),
        Workload("zipf3-10Mx5Mx2M-200M-R64", (10_000_000, 5_000_000, 2_000_000), 200_000_000, "zipf",
                 zipf_s=1.1, rank=64,
                 description="same tensor, R=64 (fp32 and bf16 factors)"),
        Workload("zipf4-50Mx20Mx1Mx100k-500M", (50_000_000, 20_000_000, 1_000_000, 100_000),
                 500_000_000, "zipf", zipf_s=1.2, rank=32,
                 description="order 4, 500M nnz, Zipf(1.2) per mode, R=32 (sparse CP loss)"),
        Workload("skew3-100Mx50Mx10M-1B", (100_000_000, 50_000_000, 10_000_000), 1_000_000_000,
                 "zipf", zipf_s=1.1, hot_frac=0.05, rank=32,
                 description="order 3, 1B nnz, Zipf(1.1) per mode plus one mode-0 slice with 5% of nnz"),
    ]
}


@dataclass
class SparseTensor:
    dims: Tuple[int, ...]
    idx: np.ndarray           # int32 [order][nnz], lexicographically sorted
    val: np.ndarray           # float32 [nnz]
    info: dict = field(default_factory=dict)

    @property
    def order(self):
        return len(self.dims)

    @property
    def nnz(self):
        return int(self.idx.shape[1])


def coords(dims, nnz, dist="zipf", zipf_s=1.1, hot_frac=0.0, seed=DEFAULT_SEED):
    """int32 [order][nnz] distinct coordinates, lexicographically sorted."""
    lib = _load()
    dims = np.ascontiguousarray(dims, dtype=np.int64)
    order = int(dims.size)
    idx = np.empty((order, int(nnz)), dtype=np.int32)
    info = np.zeros(4, dtype=np.int64)
    rc = lib.synth_coords(order, dims.ctypes.data, int(nnz), 1 if dist == "zipf" else 0,
                          float(zipf_s), float(hot_frac), int(seed), idx.ctypes.data,
                          info.ctypes.data)
    if rc != 0:
        raise RuntimeError("synth_coords failed with code %d" % rc)
    return idx, {"draws_main": int(info[0]), "draws_hot": int(info[1]),
                 "hot_index": int(info[2]), "hot_nnz": int(info[3])}


def values(nnz, seed=DEFAULT_SEED):
    """float32 U(0,1) values, one per nonzero in final order."""
    lib = _load()
    out = np.empty(int(nnz), dtype=np.float32)
    lib.synth_values(int(seed), int(nnz), out.ctypes.data)
    return out


def factor(mode, rows, rank, seed=DEFAULT_SEED):
    """float32 U(-1,1) factor matrix rows x rank, row-major."""
    lib = _load()
    out = np.empty((int(rows), int(rank)), dtype=np.float32)
    lib.synth_factor(int(seed), int(mode), int(rows), int(rank), out.ctypes.data)
    return out


def factors(dims, rank, seed=DEFAULT_SEED):
    return [factor(w, d, rank, seed) for w, d in enumerate(dims)]


def tensor(dims, nnz, dist="zipf", zipf_s=1.1, hot_frac=0.0, seed=DEFAULT_SEED):
    idx, info = coords(dims, nnz, dist, zipf_s, hot_frac, seed)
    return SparseTensor(tuple(int(d) for d in dims), idx, values(nnz, seed), info)


def workload(name, seed=DEFAULT_SEED, nnz: Optional[int] = None):
    """Generate a named workload (optionally with a reduced nonzero count)."""
    w = WORKLOADS[name]
    n = w.nnz if nnz is None else int(nnz)
    return tensor(w.dims, n, w.dist, w.zipf_s, w.hot_frac, seed)


def rank_perm(mode, I, seed=DEFAULT_SEED):
    lib = _load()
    out = np.empty(int(I), dtype=np.int32)
    lib.synth_rank_perm(int(seed), int(mode), int(I), out.ctypes.data)
    return out


def zipf_ranks(I, s, n, seed=DEFAULT_SEED, stream=999):
    """0-based Zipf ranks from the generator's own sampler (for tests)."""
    lib = _load()
    out = np.empty(int(n), dtype=np.int64)
    lib.synth_zipf_ranks(int(I), float(s), int(seed), int(stream), int(n), out.ctypes.data)
    return out


def slice_stats(idx, dims):
    """Per mode: distinct indices used, largest slice, top-10 slice share."""
    out = []
    nnz = idx.shape[1]
    for w, d in enumerate(dims):
        c = np.bincount(idx[w], minlength=int(d))
        top = np.sort(c)[::-1][:10]
        out.append({"distinct": int(np.count_nonzero(c)), "largest": int(top[0]) if nnz else 0,
                    "top10_share": float(top.sum() / max(nnz, 1))})
    return out
