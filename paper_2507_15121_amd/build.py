"""Build the native parts of the package in-tree.

* ``libamped.so``       -- the C-ABI library: host layout builder (g++/OpenMP)
                           and the gfx950 HIP kernels (hipcc).
* ``libamped_synth.so`` -- the seeded input generator (gcc/OpenMP), host only.
* ``libamped_qstats.so`` -- libamped.so built with AMPED_QUEUE_STATS=1: the
                           load-balance diagnostic (per-wave work-queue records).
* ``gather_ceiling``    -- a program that times random 128-byte row gathers from a
                           table of a given size (the GPU's row-gather ceiling).

Every call recompiles.  ``python -m paper_2507_15121_amd.build`` runs it.
"""
import concurrent.futures
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
INCLUDE = os.path.join(ROOT, "include")
BUILD_DIR = os.path.join(HERE, "_build")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
ARCH = "gfx950"

LIB = os.path.join(HERE, "libamped.so")
SYNTH_LIB = os.path.join(HERE, "libamped_synth.so")
# load-balance diagnostic build: per-wave work-queue records (include/amped_diag.h)
QSTATS_LIB = os.path.join(HERE, "libamped_qstats.so")
# row-gather ceiling of the GPU (a program, not part of the library)
CEILING_BIN = os.path.join(HERE, "gather_ceiling")

HIP_SOURCES = ["kernels.hip", "k_mttkrp_f32.hip", "k_mttkrp_bf16.hip", "k_grad.hip", "k_grad_loss.hip", "k_loss.hip",
               "sort.hip", "als.hip"]
HOST_SOURCES = ["api.cpp", "layout.cpp"]

HIPCC_FLAGS = [
    "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC",
    # CDNA packed-fp32 instructions stay off; plain fp32 code only.
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # fp32/fp64 atomic adds as hardware atomics, not CAS loops.
    "-munsafe-fp-atomics",
    "-Wall", "-Wno-unused-function",
]
HOST_FLAGS = ["-O3", "-std=c++17", "-fPIC", "-fopenmp", "-Wall", "-Wextra",
              "-D__HIP_PLATFORM_AMD__", "-I" + os.path.join(ROCM, "include")]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build_synth(verbose=False):
    tmp = SYNTH_LIB + ".tmp"
    _run(["gcc", "-O3", "-std=c99", "-fopenmp", "-fPIC", "-shared", "-Wall",
          "-o", tmp, os.path.join(CSRC, "synth.c"), "-lm"], verbose)
    os.replace(tmp, SYNTH_LIB)
    return SYNTH_LIB


def build_amped(verbose=False, extra_hip_flags=(), out=None, build_dir=None, extra_host_flags=()):
    """Build libamped.so (or, with `out`, a variant with extra compiler flags)."""
    hipcc = shutil.which("hipcc") or os.path.join(ROCM, "bin", "hipcc")
    lib_path = out or LIB
    bdir = build_dir or BUILD_DIR
    os.makedirs(bdir, exist_ok=True)
    jobs = []
    for src in HIP_SOURCES:
        obj = os.path.join(bdir, src + ".o")
        jobs.append(([hipcc] + HIPCC_FLAGS + list(extra_hip_flags) +
                     ["-I" + INCLUDE, "-I" + CSRC, "-c", os.path.join(CSRC, src), "-o", obj], obj))
    for src in HOST_SOURCES:
        obj = os.path.join(bdir, src + ".o")
        jobs.append((["g++"] + HOST_FLAGS + list(extra_host_flags) + ["-I" + INCLUDE, "-I" + CSRC, "-c",
                                            os.path.join(CSRC, src), "-o", obj], obj))
    workers = max(1, min(len(jobs), os.cpu_count() or 1, 8))
    with concurrent.futures.ThreadPoolExecutor(workers) as ex:
        list(ex.map(lambda j: _run(j[0], verbose), jobs))
    objs = [j[1] for j in jobs]
    tmp = lib_path + ".tmp"
    _run(["g++", "-shared", "-fopenmp", "-o", tmp] + objs +
         ["-L" + os.path.join(ROCM, "lib"), "-lamdhip64",
          "-Wl,-rpath," + os.path.join(ROCM, "lib"), "-Wl,--no-undefined"], verbose)
    os.replace(tmp, lib_path)
    return lib_path


def build_gather_ceiling(verbose=False):
    """The row-gather ceiling program (csrc/gather_ceiling.hip): the rate at
    which the GPU returns random 128-byte rows from a table of a given size."""
    hipcc = shutil.which("hipcc") or os.path.join(ROCM, "bin", "hipcc")
    tmp = CEILING_BIN + ".tmp"
    _run([hipcc] + HIPCC_FLAGS + ["-o", tmp, os.path.join(CSRC, "gather_ceiling.hip")], verbose)
    os.replace(tmp, CEILING_BIN)
    return CEILING_BIN


def build_qstats(verbose=False):
    """The load-balance diagnostic variant of libamped.so."""
    flag = ["-DAMPED_QUEUE_STATS=1"]
    return build_amped(verbose, extra_hip_flags=flag, extra_host_flags=flag, out=QSTATS_LIB,
                       build_dir=os.path.join(BUILD_DIR, "qstats"))


def build(verbose=False):
    build_synth(verbose)
    build_amped(verbose)
    build_qstats(verbose)
    build_gather_ceiling(verbose)


if __name__ == "__main__":
    build(verbose="-q" not in sys.argv)
