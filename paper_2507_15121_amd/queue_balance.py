"""Work-queue load balance of the MTTKRP kernel on one GPU.

The paper reports that its load-balancing scheme keeps the compute time of its
GPUs within 1% of the total (Sec. 5.5, Workload Distribution among GPUs).  On
one GPU the partitions go to compute units instead (the dynamic mapping of
Sec. 4.2, here a work queue of equal-size chunks), so the question becomes how
evenly the chunks, their nonzeros and the busy time spread over the
workgroups of the persistent grid (one 512-thread workgroup per compute unit
for MTTKRP).  This script runs the diagnostic build of the library
(``libamped_qstats.so``, built by ``build.build_qstats``), in which every wave
records the chunks and nonzeros it took and the wall-clock times of its first
pop and its exit, and prints a Markdown summary per mode.

    python -m paper_2507_15121_amd.queue_balance --workload skew3-100Mx50Mx10M-1B
"""
import argparse
import ctypes
import os
import sys
import time

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))


def _records(lib):
    n = ctypes.c_int64()
    wpb = ctypes.c_int32()
    hz = ctypes.c_double()
    lib.amped_queue_stats.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.c_void_p]
    lib.amped_queue_stats.restype = ctypes.c_int
    st = lib.amped_queue_stats(None, 0, ctypes.byref(n), ctypes.byref(wpb), ctypes.byref(hz))
    if st != 0:
        raise RuntimeError(lib.amped_last_error().decode())
    rec = np.zeros((n.value, 4), dtype=np.uint64)
    st = lib.amped_queue_stats(rec.ctypes.data, n.value, ctypes.byref(n), ctypes.byref(wpb), ctypes.byref(hz))
    if st != 0:
        raise RuntimeError(lib.amped_last_error().decode())
    return rec, wpb.value, hz.value


def summarize(rec, waves_per_block, hz):
    """Per-workgroup totals and spreads of one launch's per-wave records."""
    blocks = rec.shape[0] // waves_per_block
    r = rec[: blocks * waves_per_block].reshape(blocks, waves_per_block, 4)
    chunks = r[:, :, 0].sum(1).astype(np.int64)
    nnz = r[:, :, 1].sum(1).astype(np.int64)
    took = r[:, :, 0] > 0
    first = np.where(took, r[:, :, 2], np.iinfo(np.uint64).max).min(1).astype(np.float64)
    exit_ = r[:, :, 3].max(1).astype(np.float64)
    t0 = first.min()
    span = exit_.max() - t0
    busy = exit_ - first
    return {
        "blocks": blocks, "waves_per_block": waves_per_block,
        "span_us": span / hz * 1e6,
        "chunks": (int(chunks.min()), float(chunks.mean()), int(chunks.max())),
        "nnz": (int(nnz.min()), float(nnz.mean()), int(nnz.max())),
        "nnz_spread": float((nnz.max() - nnz.min()) / nnz.mean()) if nnz.mean() else 0.0,
        # when the workgroups finish, relative to the whole launch
        "exit_spread": float((exit_.max() - exit_.min()) / span) if span > 0 else 0.0,
        "start_spread": float((first.max() - first.min()) / span) if span > 0 else 0.0,
        "busy_spread": float((busy.max() - busy.min()) / span) if span > 0 else 0.0,
        "idle_share": float(1.0 - busy.sum() / (blocks * span)) if span > 0 else 0.0,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="skew3-100Mx50Mx10M-1B")
    ap.add_argument("--nnz", type=int, default=None)
    ap.add_argument("--repeats", type=int, default=3, help="recorded launches per mode (after one warm-up)")
    args = ap.parse_args()
    lib_path = os.path.join(_HERE, "libamped_qstats.so")
    if not os.path.exists(lib_path):
        sys.exit("libamped_qstats.so is not built (paper_2507_15121_amd.build.build_qstats)")
    import torch

    from paper_2507_15121_amd import api, synth
    # the package import has already read AMPED_LIB; point the binding at the
    # diagnostic build before its first call loads a library
    if api._lib is not None:
        sys.exit("the C library is already loaded")
    api.LIB_PATH = lib_path
    torch.cuda.set_device(0)
    wl = synth.WORKLOADS[args.workload]
    t0 = time.time()
    st = synth.workload(wl.name, nnz=args.nnz)
    print("<!-- generated in %.0fs -->" % (time.time() - t0), flush=True)
    T = api.Tensor(st.idx, st.val, st.dims)
    fac = [torch.from_numpy(f).cuda() for f in synth.factors(st.dims, wl.rank)]
    L = api.lib()
    print("| mode | launch | workgroups x waves | span us | chunks per workgroup min / mean / max | "
          "nonzeros per workgroup min / mean / max | nonzero spread | first-pop spread | exit spread | "
          "busy spread | idle share |")
    print("|---|---|---|---|---|---|---|---|---|---|---|")
    for d in range(st.order):
        f = [None if w == d else x for w, x in enumerate(fac)]
        out = torch.empty((st.dims[d], wl.rank), device="cuda")
        api.mttkrp(T, d, f, out=out)
        for k in range(args.repeats):
            api.mttkrp(T, d, f, out=out)
            torch.cuda.synchronize()
            s = summarize(*_records(L))
            print("| %d | %d | %d x %d | %.0f | %d / %.1f / %d | %d / %.0f / %d | %.4f | %.4f | %.4f | %.4f | %.4f |" % (
                d, k, s["blocks"], s["waves_per_block"], s["span_us"], *s["chunks"], *s["nnz"], s["nnz_spread"],
                s["start_spread"], s["exit_spread"], s["busy_spread"], s["idle_share"]), flush=True)
        del out
    T.close()


if __name__ == "__main__":
    main()
