"""All-mode sparse MTTKRP benchmark on one MI355X.

One step = MTTKRP along every mode of the tensor (each mode into its own
output, all from the same factors), the paper's metric "time to compute
MTTKRP across all modes in one iteration" (Sec. 5.1).  Inputs are resident in
HBM before the timed region; the layout build is excluded (as preprocessing is
in the paper).  Printed as one JSON line; beside the fp32 value it reports the
bf16-factor form, the sparse CP loss forward + fused backward, the dominant
kernel's roofline figures and the CPU oracle's rate on a bounded sample.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MTTKRP nnz/s + achieved HBM TB/s per mode; FP32 vs BF16-factor at stated tol"
HBM_PEAK_GBS = 8000.0
PROFILES = os.path.join(ROOT, "profiles")


def measured_traffic(workload, lib_path):
    """HBM-side bytes per launch of the fp32 kernel from a committed counter
    summary (profiles/mttkrp_<workload>_R*_traffic.md), used only while the
    loaded library is the build those counters were taken on."""
    import glob
    import hashlib
    sha = hashlib.sha256(open(lib_path, "rb").read()).hexdigest()
    for path in glob.glob(os.path.join(PROFILES, "mttkrp_%s_R*_traffic.md" % workload)):
        fields = {}
        for line in open(path):
            if ":" in line and line.split(":", 1)[0] in ("traffic_bytes_per_launch", "library_sha256"):
                k, v = line.split(":", 1)
                fields[k.strip()] = v.strip()
        if fields.get("library_sha256") == sha and "traffic_bytes_per_launch" in fields:
            return float(fields["traffic_bytes_per_launch"]), os.path.basename(path)
    return None, None


def gather_ceiling(key="ceiling_GBps"):
    """A measured row-gather rate of the GPU from the committed summary
    profiles/gather_ceiling_mi355x.md, or None.  `ceiling_GBps`: random
    128-byte rows that miss the L2 but hit the Infinity Cache (the fastest an
    L2 miss returns); `row_request_ceiling_GBps`: random rows that hit the L2
    (the fastest the CUs issue row loads of the kernel's shape)."""
    path = os.path.join(PROFILES, "gather_ceiling_mi355x.md")
    try:
        for line in open(path):
            if line.startswith(key + ":"):
                return float(line.split(":", 1)[1])
    except OSError:
        pass
    return None


T0 = time.time()


def log(msg):
    print("[bench +%.0fs] %s" % (time.time() - T0, msg), file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="skew3-100Mx50Mx10M-1B")
    ap.add_argument("--nnz", type=int, default=None, help="override the workload's nonzero count")
    ap.add_argument("--rank", type=int, default=None, help="override the workload's rank")
    ap.add_argument("--chunk", type=int, default=0)
    ap.add_argument("--seed", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true", help="skip the bf16 and CP loss/grad forms")
    ap.add_argument("--no-accuracy", action="store_true",
                    help="skip the sampled-row checks against the oracle (part of the CPU-baseline leg)")
    ap.add_argument("--no-out-of-core", action="store_true",
                    help="skip timing the all-mode fp32 step with host-resident layouts streamed in shards")
    ap.add_argument("--shard-nnz", type=int, default=0, help="nonzeros per streamed shard (0 = library default)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target oracle time for the CPU baseline")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain device copy of known size (for counter scaling)")
    return ap.parse_args()


def slice_stats(st):
    """Per mode: distinct indices, and the shares of nonzeros in the largest
    slice and in the 10 largest slices."""
    out = {"distinct": [], "largest_slice_share": [], "top10_slice_share": []}
    for w in range(st.order):
        c = np.bincount(st.idx[w], minlength=st.dims[w])
        top = np.partition(c, -10)[-10:] if c.size >= 10 else c
        out["distinct"].append(int(np.count_nonzero(c)))
        out["largest_slice_share"].append(float(top.max()) / max(st.nnz, 1))
        out["top10_slice_share"].append(float(top.sum()) / max(st.nnz, 1))
    return out


def host_info():
    """Cores this process may run on, the CPU model name and the host RAM."""
    cores = len(os.sched_getaffinity(0))
    model = ""
    try:
        import subprocess
        for line in subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
                break
    except (OSError, subprocess.SubprocessError):
        pass
    ram_gb = None
    try:
        for line in open("/proc/meminfo"):
            if line.startswith("MemTotal:"):
                ram_gb = int(line.split()[1]) * 1024 / 1e9
                break
    except OSError:
        pass
    return cores, model, ram_gb


def oracle_rows(st, factors64, d, rows, R, pool, parts):
    """FP64 oracle MTTKRP of mode d on the given output rows only.

    The nonzeros of those rows are split into `parts` pieces by position and
    each piece runs through the unchanged sequential oracle on its own thread;
    the per-piece outputs are added in fp64 (MTTKRP is linear in the tensor
    values, so this changes only the fp64 summation order).  Called from the
    CPU-baseline leg only."""
    import oracle
    lut = np.full(st.dims[d], -1, dtype=np.int64)
    lut[rows] = np.arange(rows.size)
    m = np.flatnonzero(lut[st.idx[d]] >= 0)
    dims = list(st.dims)
    dims[d] = rows.size
    fs = list(factors64)
    fs[d] = np.zeros((rows.size, R))

    def piece(sl):
        sub = st.idx[:, m[sl]].copy()
        sub[d] = lut[sub[d]]
        return oracle.mttkrp(sub, st.val[m[sl]], dims, fs, d)
    bounds = np.linspace(0, m.size, parts + 1).astype(np.int64)
    outs = list(pool.map(piece, [slice(bounds[i], bounds[i + 1]) for i in range(parts)]))
    return np.sum(outs, axis=0)


def sampled_rel_errors(st, factors64, outs, rank, rng, pool, parts, n_rows=200):
    """Relative Frobenius error of each mode's output on sampled rows (the
    heaviest row plus random touched rows) against the FP64 oracle.  Called
    from the CPU-baseline leg only."""
    import oracle
    errs = []
    for d, out in enumerate(outs):
        counts = np.bincount(st.idx[d], minlength=st.dims[d])
        touched = np.flatnonzero(counts)
        pick = rng.choice(touched, size=min(n_rows, touched.size), replace=False)
        rows = np.unique(np.concatenate([pick, [int(np.argmax(counts))]]))
        ref = oracle_rows(st, factors64, d, rows, rank, pool, parts)
        errs.append(oracle.rel_fro(out[rows], ref))
    return errs


def row_block_jobs(idx, val, dims, factors64, d, parts):
    """Split mode d's MTTKRP into at most `parts` blocks of output rows,
    balanced by nonzero count and cut at row boundaries (equal row ranges when
    there are no nonzeros).  Returns the row bounds and, per block, the
    arguments of one oracle call with the block's rows relabelled to start at
    0; the blocks' outputs stacked in order are the full mode-d output."""
    S = val.size
    R = factors64[0].shape[1]
    key = idx[d]
    if S:
        cum = np.cumsum(np.bincount(key, minlength=dims[d]))
        cuts = np.searchsorted(cum, np.arange(1, parts) * (S / parts), side="left") + 1
    else:
        cuts = np.arange(1, parts) * (dims[d] // parts)
    bounds = np.unique(np.concatenate([[0], np.minimum(cuts, dims[d]), [dims[d]]])).astype(np.int64)
    blk = (np.searchsorted(bounds, key, side="right") - 1).astype(np.int16)
    order = np.argsort(blk, kind="stable")
    starts = np.searchsorted(blk[order], np.arange(bounds.size - 1), side="left")
    ends = np.append(starts[1:], S)
    jobs = []
    for b in range(bounds.size - 1):
        o = order[starts[b]:ends[b]]
        sub = idx[:, o]
        sub[d] -= int(bounds[b])
        bdims = list(dims)
        bdims[d] = int(bounds[b + 1] - bounds[b])
        fs = list(factors64)
        fs[d] = np.zeros((1, R))
        jobs.append((np.ascontiguousarray(sub), val[o], bdims, fs, d))
    return bounds, jobs


def cpu_baseline(st, factors64, pool, cores, target_s):
    """The FP64 oracle timed on every core of this process's affinity set.

    A strided sample of the tensor's nonzeros (every k-th one, so it spans the
    whole tensor) is split, per mode, into one block of output rows per core,
    balanced by nonzero count and cut at row boundaries; each block runs
    through the unchanged sequential oracle on its own thread with its rows
    relabelled to start at 0, so the blocks' outputs together are the
    full-size output, zeroed as in the sequential oracle.  The timed wall clock
    covers those per-mode block runs; the sample size follows the model
    t(S) = a + b S fitted on a zero-nonzero and a pilot run."""
    import oracle
    N = st.order

    def sample(S):
        stride = max(1, st.nnz // max(S, 1))
        sel = np.arange(stride // 2, st.nnz, stride, dtype=np.int64)[:S] if S else np.zeros(0, np.int64)
        return st.idx[:, sel], st.val[sel].astype(np.float64)

    def run(S):
        idx, val = sample(S)
        t = 0.0
        for d in range(N):
            _, jobs = row_block_jobs(idx, val, st.dims, factors64, d, cores)
            t0 = time.perf_counter()
            list(pool.map(lambda j: oracle.mttkrp(*j).shape, jobs))
            t += time.perf_counter() - t0
            del jobs
        return t

    t_zero = run(0)
    S0 = int(min(st.nnz, 2_000_000 * cores))
    b_per = max(run(S0) - t_zero, 1e-9) / S0
    S = int(min(st.nnz, max(S0, (target_s - t_zero) / b_per)))
    return S, run(S), t_zero


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2507_15121_amd import api, synth

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    torch.cuda.set_device(0)
    wl = synth.WORKLOADS[args.workload]
    seed = synth.DEFAULT_SEED if args.seed is None else args.seed
    R = args.rank or wl.rank
    nnz = wl.nnz if args.nnz is None else args.nnz

    t0 = time.time()
    st = synth.workload(wl.name, seed=seed, nnz=nnz)
    factors = synth.factors(st.dims, R, seed=seed)
    gen_s = time.time() - t0
    log("generated %s nnz=%d in %.1fs (%s)" % (wl.name, st.nnz, gen_s, st.info))
    index_stats = slice_stats(st)
    log("index stats %s" % index_stats)

    t0 = time.time()
    T = api.Tensor(st.idx, st.val, st.dims, chunk_nnz=args.chunk)
    torch.cuda.synchronize()
    build_s = time.time() - t0
    log("layouts built in %.1fs, device bytes %.2f GB, touched %s" % (build_s, T.device_bytes / 1e9, T.touched))

    N = st.order
    dfac = [torch.from_numpy(f).cuda() for f in factors]
    outs = [torch.empty((st.dims[d], R), dtype=torch.float32, device="cuda") for d in range(N)]
    stream = torch.cuda.current_stream()

    def step(fac, bf16=False, ev=None):
        for d in range(N):
            f = [None if w == d else x for w, x in enumerate(fac)]
            if ev is not None:
                ev[d][0].record(stream)
            if bf16:
                api.mttkrp_bf16(T, d, f, out=outs[d], stream=stream)
            else:
                api.mttkrp(T, d, f, out=outs[d], stream=stream)
            if ev is not None:
                ev[d][1].record(stream)

    def timed(fac, bf16=False):
        for _ in range(args.warmup):
            step(fac, bf16)
        torch.cuda.synchronize()
        evs = [[[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(N)]
               for _ in range(args.steps)]
        start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        start.record(stream)
        for k in range(args.steps):
            step(fac, bf16, evs[k])
        end.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - w0
        times = [[evs[k][d][0].elapsed_time(evs[k][d][1]) for k in range(args.steps)] for d in range(N)]
        per_mode = [float(np.mean(x)) for x in times]
        timed.medians = [float(np.median(x)) for x in times]
        return start.elapsed_time(end) / args.steps, per_mode, wall

    ms_step, per_mode_ms, wall = timed(dfac)
    per_mode_median_ms = timed.medians
    log("fp32: %.3f ms/step, per mode %s ms, wall %.3fs" % (ms_step, ["%.3f" % x for x in per_mode_ms], wall))

    # algorithmic bytes per mode: nonzero stream + each distinct input row once + output once
    def mode_bytes(d, fbytes):
        stream_b = st.nnz * (4 * N + 4)
        gather_b = sum(T.touched[w] * R * fbytes for w in range(N) if w != d)
        out_b = st.dims[d] * R * 4
        return stream_b + gather_b + out_b
    bytes32 = [mode_bytes(d, 4) for d in range(N)]
    achieved = sum(bytes32) / (sum(per_mode_ms) * 1e-3) / 1e9
    per_mode = [{"mode": d, "rows": st.dims[d], "touched": T.touched[d], "ms": per_mode_ms[d],
                 "ms_median": per_mode_median_ms[d],
                 "nnz_per_s": st.nnz / (per_mode_ms[d] * 1e-3),
                 "algorithmic_GBps": bytes32[d] / (per_mode_ms[d] * 1e-3) / 1e9} for d in range(N)]

    acc = {}
    forms = {}
    if not args.no_forms:
        dbf = [f.to(torch.bfloat16) for f in dfac]
        ms_bf, pm_bf, _ = timed(dbf, bf16=True)
        bytes16 = [mode_bytes(d, 2) for d in range(N)]
        forms["bf16"] = {"ms_per_step": ms_bf, "per_mode_ms": pm_bf,
                         "nnz_per_s": N * st.nnz / (ms_bf * 1e-3),
                         "algorithmic_GBps": sum(bytes16) / (sum(pm_bf) * 1e-3) / 1e9}
        log("bf16: %s" % forms["bf16"])
        # sparse CP loss forward + fused residual/MTTKRP backward for every mode
        grads = [torch.empty_like(f) for f in dfac]
        loss = torch.empty((), dtype=torch.float64, device="cuda")

        def cp_step_separate():   # loss pass, then one gradient pass per mode (N + 1 passes)
            api.cp_loss(T, dfac, out=loss, stream=stream)
            for d in range(N):
                api.cp_grad(T, d, dfac, -2.0, out=grads[d], stream=stream)

        def cp_step():   # loss with mode 0's gradient in one pass, then the other modes (N passes)
            api.cp_loss_grad(T, 0, dfac, -2.0, out=grads[0], loss=loss, stream=stream)
            for d in range(1, N):
                api.cp_grad(T, d, dfac, -2.0, out=grads[d], stream=stream)

        def time_cp(fn):
            for _ in range(args.warmup):
                fn()
            torch.cuda.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            for _ in range(args.steps):
                fn()
            b.record(stream)
            torch.cuda.synchronize()
            return a.elapsed_time(b) / args.steps
        ms_sep = time_cp(cp_step_separate)
        loss_sep = float(loss)
        ms_cp = time_cp(cp_step)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        forms["cp_loss_and_grad"] = {"ms_per_step": ms_cp, "loss": float(loss),
                                     "nnz_per_s": N * st.nnz / (ms_cp * 1e-3),
                                     "passes": N, "ms_per_step_separate_loss_pass": ms_sep,
                                     "loss_separate_pass": loss_sep}
        # directional finite difference at full size: [L(A + eps V) - L(A - eps V)] / (2 eps)
        # against <grad L, V> for a seeded random direction V (losses summed in fp64)
        gen = torch.Generator(device="cuda").manual_seed(1234)
        Vd = [torch.rand(f.shape, generator=gen, device="cuda") * 2 - 1 for f in dfac]
        def dot64(x, y, chunk=1 << 24):   # float64 inner product in chunks (bounded temporaries)
            x, y = x.reshape(-1), y.reshape(-1)
            return sum(float((x[i:i + chunk].double() * y[i:i + chunk].double()).sum())
                       for i in range(0, x.numel(), chunk))
        dirderiv = sum(dot64(grads[d], Vd[d]) for d in range(N))
        eps = 1e-3
        lp = torch.empty((), dtype=torch.float64, device="cuda")
        lm = torch.empty((), dtype=torch.float64, device="cuda")
        api.cp_loss(T, [f + eps * v for f, v in zip(dfac, Vd)], out=lp, stream=stream)
        api.cp_loss(T, [f - eps * v for f, v in zip(dfac, Vd)], out=lm, stream=stream)
        torch.cuda.synchronize()
        fd = (float(lp) - float(lm)) / (2 * eps)
        forms["cp_loss_and_grad"]["fd_check"] = {"directional_derivative": dirderiv, "central_difference": fd,
                                                 "eps": eps, "rel_diff": abs(fd - dirderiv) / abs(dirderiv)}
        del Vd
        log("cp loss+grad: %s" % forms["cp_loss_and_grad"])
        if R <= 128:
            # CP-ALS sweeps (MTTKRP + Gram + R x R algebra + update per mode)
            # on copies of the factors, and the Gram kernel on its own
            als_fac = [f.clone() for f in dfac]
            lam = torch.empty(R, dtype=torch.float64, device="cuda")
            fitv = torch.empty((), dtype=torch.float64, device="cuda")
            api.cp_als_sweep(T, als_fac, lam, fitv, stream=stream)
            torch.cuda.synchronize()
            n_sw = max(1, min(args.steps, 5))
            a.record(stream)
            for _ in range(n_sw):   # chained sweeps reuse the Gram matrices the last one left
                api.cp_als_sweep(T, als_fac, lam, fitv, reuse_grams=True, stream=stream)
            b.record(stream)
            torch.cuda.synchronize()
            ms_als = a.elapsed_time(b) / n_sw
            big = max(range(N), key=lambda d: st.dims[d])
            G = torch.empty((R, R), dtype=torch.float64, device="cuda")
            for _ in range(3):
                api.gram(dfac[big], out=G, stream=stream)
            torch.cuda.synchronize()
            a.record(stream)
            for _ in range(10):
                api.gram(dfac[big], out=G, stream=stream)
            b.record(stream)
            torch.cuda.synchronize()
            ms_gram = a.elapsed_time(b) / 10
            rows = st.dims[big]
            forms["cp_als_sweep"] = {"ms_per_sweep": ms_als, "fit_after": float(fitv), "sweeps": n_sw + 1,
                                     "gram_ms": ms_gram, "gram_rows": rows,
                                     "gram_TFLOPs": 2.0 * rows * R * R / (ms_gram * 1e-3) / 1e12,
                                     "gram_GBps": rows * R * 4 / (ms_gram * 1e-3) / 1e9}
            log("cp-als sweep: %s" % forms["cp_als_sweep"])
            del als_fac

    if not args.no_out_of_core:
        # host-resident layouts (pinned host memory, host order builder),
        # streamed to the device in shards on every call
        t0 = time.time()
        TH = api.Tensor(st.idx, st.val, st.dims, chunk_nnz=args.chunk, host_layout=True, shard_nnz=args.shard_nnz)
        host_build_s = time.time() - t0
        log("host-resident layouts built in %.1fs, device bytes %.3f GB" % (host_build_s, TH.device_bytes / 1e9))
        step(dfac)
        ref = [o.clone() for o in outs]
        outs_h = [torch.empty_like(o) for o in outs]

        def step_h():
            for d in range(N):
                f = [None if w == d else x for w, x in enumerate(dfac)]
                api.mttkrp(TH, d, f, out=outs_h[d], stream=stream)
        step_h()
        torch.cuda.synchronize()
        diff = [float(torch.linalg.norm(outs_h[d] - ref[d]) / torch.linalg.norm(ref[d])) for d in range(N)]
        n_h = max(1, min(args.steps, 3))
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(n_h):
            step_h()
        b.record(stream)
        torch.cuda.synchronize()
        ms_h = a.elapsed_time(b) / n_h
        streamed = N * st.nnz * (4 * N + 4)
        # reference: plain pinned host -> device copies of 1 GiB
        hbuf = torch.empty(1 << 28, dtype=torch.float32, pin_memory=True)
        dbuf = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
        for _ in range(2):
            dbuf.copy_(hbuf, non_blocking=True)
        torch.cuda.synchronize()
        a.record(stream)
        for _ in range(5):
            dbuf.copy_(hbuf, non_blocking=True)
        b.record(stream)
        torch.cuda.synchronize()
        h2d = 5 * (1 << 30) / (a.elapsed_time(b) * 1e-3) / 1e9
        forms["out_of_core"] = {"ms_per_step": ms_h, "steps": n_h, "host_build_s": host_build_s,
                                "device_bytes": TH.device_bytes, "shard_nnz": args.shard_nnz or (1 << 25),
                                "streamed_GB_per_step": streamed / 1e9,
                                "stream_GBps": streamed / (ms_h * 1e-3) / 1e9, "pinned_h2d_GBps": h2d,
                                "rel_diff_vs_resident": diff, "slowdown_vs_resident": ms_h / ms_step}
        log("out-of-core: %s" % forms["out_of_core"])
        TH.close()
        del ref, outs_h, hbuf, dbuf

    if args.copy_calibration:
        n = 1 << 30  # 4 GiB of fp32 read, 4 GiB written
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    cpu = None
    if not args.no_cpu_baseline:
        # the CPU-baseline leg: the only place the bench runs the oracle.  It checks
        # sampled output rows of the GPU runs, then times the oracle on a sample,
        # on every core of this process's affinity set.
        import concurrent.futures
        import oracle
        cores, cpu_model, ram_gb = host_info()
        pool = concurrent.futures.ThreadPoolExecutor(cores)
        factors64 = [f.astype(np.float64) for f in factors]
        if not args.no_accuracy:
            step(dfac)
            torch.cuda.synchronize()
            host_outs = [o.cpu().numpy() for o in outs]
            acc["fp32_rel_err_sampled"] = sampled_rel_errors(st, factors64, host_outs, R,
                                                             np.random.default_rng(7), pool, cores)
            log("fp32 sampled rel errors %s" % acc["fp32_rel_err_sampled"])
            if "bf16" in forms:
                step(dbf, bf16=True)
                torch.cuda.synchronize()
                host_outs = [o.cpu().numpy() for o in outs]
                # against the oracle on the fp32 factors (the bf16 error), and on the
                # bf16-rounded factors (shows the accumulation stayed fp32); same rows
                forms["bf16"]["rel_err_vs_fp64_sampled"] = sampled_rel_errors(
                    st, factors64, host_outs, R, np.random.default_rng(8), pool, cores)
                rounded = [oracle.bf16_to_f32(oracle.bf16_rne(f)).astype(np.float64) for f in factors]
                forms["bf16"]["rel_err_vs_fp64_on_bf16_factors_sampled"] = sampled_rel_errors(
                    st, rounded, host_outs, R, np.random.default_rng(8), pool, cores)
                del rounded
                log("bf16 sampled rel errors %s / on bf16 factors %s" % (
                    forms["bf16"]["rel_err_vs_fp64_sampled"],
                    forms["bf16"]["rel_err_vs_fp64_on_bf16_factors_sampled"]))
            del host_outs
        S, t_cpu, t_zero = cpu_baseline(st, factors64, pool, cores, args.cpu_seconds)
        pool.shutdown()
        cpu_value = N * S / t_cpu
        cpu = {"value": cpu_value, "unit": "nnz/s", "cores": cores, "kind": "oracle",
               "sample": "every %d-th nonzero of the same tensor (%d nonzeros), all %d modes; per mode one "
                         "block of output rows per core (balanced by nonzeros), each through the sequential "
                         "float64 oracle on its own thread; full-size factors, outputs zeroed (%.1fs of the "
                         "%.1fs); wall clock" % (max(1, st.nnz // max(S, 1)), S, N, t_zero, t_cpu),
               "cpu_model": cpu_model, "host_ram_GB": ram_gb, "seconds": t_cpu}
        log("cpu baseline %s" % cpu)

    traffic, traffic_src = measured_traffic(wl.name, api.LIB_PATH)
    # the measured traffic per launch over the mean launch time of this run: the rate the
    # kernel really moves between L2 and the fabric (Infinity Cache hits included)
    mean_launch_s = float(np.mean(per_mode_ms)) * 1e-3
    fabric_gbps = traffic / mean_launch_s / 1e9 if traffic is not None else None
    ceiling = gather_ceiling()
    issue_ceiling = gather_ceiling("row_request_ceiling_GBps")
    # factor rows the kernel asks for per launch (every gathered row, also those the
    # L1 or the LDS hot-row cache then serve), over the mean launch time
    rows_gbps = st.nnz * (N - 1) * R * 4 / mean_launch_s / 1e9
    value = N * st.nnz / (ms_step * 1e-3)
    if cpu is not None:
        cpu["gpu_over_cpu"] = value / cpu["value"]
    res = {
        "metric": METRIC, "value": value, "unit": "nnz/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": wl.name, "dims": list(st.dims), "nnz": st.nnz, "rank": R,
                   "dist": wl.dist, "zipf_s": wl.zipf_s, "hot_frac": wl.hot_frac,
                   "chunk_nnz": T.chunk_nnz, "seed": seed,
                   "value_is": "modes x nnz / all-mode step time"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                     "traffic_source": traffic_src,
                     "traffic_GBps": fabric_gbps,
                     "traffic_frac": fabric_gbps / HBM_PEAK_GBS if fabric_gbps is not None else None,
                     "l2_miss_ceiling_GBps": ceiling,
                     "traffic_over_l2_miss_ceiling": (fabric_gbps / ceiling
                                                      if fabric_gbps is not None and ceiling else None),
                     "rows_requested_GBps": rows_gbps,
                     "row_request_ceiling_GBps": issue_ceiling,
                     "rows_requested_over_ceiling": rows_gbps / issue_ceiling if issue_ceiling else None,
                     "kernel": "mttkrp_kernel (fp32)",
                     "bytes_model": "per mode: nnz*(4N+4) + sum_{w!=d} touched_w*R*4 + I_d*R*4"},
        "per_mode": per_mode,
        "forms": forms,
        "accuracy": acc,
        "layout_build_s": build_s, "generate_s": gen_s, "index_stats": index_stats,
        "cpu_baseline": cpu,
    }
    T.close()
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
