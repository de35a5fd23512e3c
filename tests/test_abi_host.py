"""Host-side checks of the C ABI (no GPU needed): the library loads and exports
every declared symbol, the host layout builder is bit-exact against the
oracle's ordering, and argument errors come back as status codes."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from paper_2507_15121_amd import api, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    text = open(os.path.join(ROOT, "include", "amped.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(amped_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = api.lib()
    decl = _declared_symbols()
    assert decl, "no declarations found"
    for name in decl:
        assert hasattr(L, name), name
    assert sorted(api.EXPORTED) == decl
    assert "gfx950" in api.version()


def _random_coo(rng, dims, nnz, dup=True):
    return np.stack([rng.integers(0, d, size=nnz) for d in dims]).astype(np.int32)


@pytest.mark.parametrize("dims", [(5, 4), (9, 8, 7), (6, 5, 4, 3), (4, 3, 3, 2, 2)])
@pytest.mark.parametrize("ch", [1, 7, 64, 4096])
def test_layout_host_bitexact_vs_oracle(dims, ch):
    rng = np.random.default_rng(sum(dims) * 31 + ch)
    nnz = 500
    idx = _random_coo(rng, dims, nnz)  # with duplicates, unsorted
    for mode in range(len(dims)):
        perm, flags = api.layout_host(idx, dims, mode, ch)
        ref = oracle.layout(idx, mode, ch)
        np.testing.assert_array_equal(perm, ref["perm"])
        np.testing.assert_array_equal(flags, ref["flags"])


def test_layout_host_sorted_input_and_permutation_invariance():
    idx, _ = synth.coords((300, 200, 100), 20_000, "zipf", 1.1, seed=3)
    rng = np.random.default_rng(1)
    p = rng.permutation(idx.shape[1])
    shuffled = idx[:, p]
    for mode in range(3):
        a, fa = api.layout_host(idx, (300, 200, 100), mode, 64)
        b, fb = api.layout_host(shuffled, (300, 200, 100), mode, 64)
        # distinct coordinates: the sorted coordinates are identical
        np.testing.assert_array_equal(idx[:, a], shuffled[:, b])
        np.testing.assert_array_equal(fa, fb)
        ref = oracle.layout(shuffled, mode, 64)
        np.testing.assert_array_equal(b, ref["perm"])


def test_layout_host_large_radix_paths():
    # mode sizes that need 1, 2 and 3 radix passes; input not sorted
    dims = (70_000, 3_000_000, 100)
    rng = np.random.default_rng(5)
    idx = _random_coo(rng, dims, 200_000)
    for mode in range(3):
        perm, flags = api.layout_host(idx, dims, mode, 1000)
        ref = oracle.layout(idx, mode, 1000)
        np.testing.assert_array_equal(perm, ref["perm"])
        np.testing.assert_array_equal(flags, ref["flags"])


def test_layout_host_edge_cases():
    # nnz = 0, a single nonzero, all nonzeros in one slice
    perm, flags = api.layout_host(np.zeros((3, 0), np.int32), (4, 4, 4), 1, 8)
    assert perm.size == 0 and flags.size == 0
    perm, flags = api.layout_host(np.array([[1], [2], [3]], np.int32), (4, 4, 4), 2, 8)
    assert perm.tolist() == [0] and flags.tolist() == [0]
    idx = np.stack([np.full(100, 3), np.arange(100) % 7, np.arange(100) % 11]).astype(np.int32)
    perm, flags = api.layout_host(idx, (5, 7, 11), 0, 10)
    ref = oracle.layout(idx, 0, 10)
    np.testing.assert_array_equal(perm, ref["perm"])
    assert flags.tolist() == [2] + [3] * 8 + [1]


def _create_status(order, dims, nnz, idx, val, opts=None):
    L = api.lib()
    h = ctypes.c_void_p()
    d = np.ascontiguousarray(dims, dtype=np.int64)
    o = api._Options(*opts) if opts else None
    st = L.amped_tensor_create(order, d.ctypes.data, nnz, idx, val,
                               ctypes.byref(o) if o is not None else None, ctypes.byref(h))
    if st == api.OK:
        L.amped_tensor_destroy(h)
    else:
        assert h.value is None
        assert L.amped_last_error().decode()
    return st


def test_create_argument_errors():
    idx = np.zeros((3, 4), np.int32)
    val = np.zeros(4, np.float32)
    ip, vp = idx.ctypes.data, val.ctypes.data
    assert _create_status(1, [4], 4, ip, vp) == api.ERR_INVALID
    assert _create_status(9, [4] * 9, 4, ip, vp) == api.ERR_INVALID
    assert _create_status(3, [4, 0, 4], 4, ip, vp) == api.ERR_INVALID
    assert _create_status(3, [4, 4, 2 ** 31], 4, ip, vp) == api.ERR_INVALID
    assert _create_status(3, [4, 4, 4], -1, ip, vp) == api.ERR_INVALID
    assert _create_status(3, [4, 4, 4], 4, None, vp) == api.ERR_INVALID
    assert _create_status(3, [4, 4, 4], 4, ip, None) == api.ERR_INVALID
    assert _create_status(3, [4, 4, 4], 4, ip, vp, (-5, 0, 0, 0, 0)) == api.ERR_INVALID
    assert _create_status(3, [4, 4, 4], 4, ip, vp, (0, 0, 2, 0, 0)) == api.ERR_INVALID
    assert _create_status(3, [4, 4, 4], 4, ip, vp, (0, 0, 0, 2, 0)) == api.ERR_INVALID
    assert _create_status(3, [4, 4, 4], 4, ip, vp, (0, 0, 0, 1, -1)) == api.ERR_INVALID
    bad = idx.copy()
    bad[1, 2] = 4
    assert _create_status(3, [4, 4, 4], 4, bad.ctypes.data, vp) == api.ERR_RANGE
    bad[1, 2] = -1
    assert _create_status(3, [4, 4, 4], 4, bad.ctypes.data, vp) == api.ERR_RANGE
    # device byte cap: refused before the device is touched
    assert _create_status(3, [4, 4, 4], 4, ip, vp, (0, 64, 0, 0, 0)) == api.ERR_NOMEM
    assert _create_status(3, [4, 4, 4], 4, ip, vp, (0, 64, 0, 1, 0)) == api.ERR_NOMEM
    L = api.lib()
    assert L.amped_tensor_create(3, np.array([4, 4, 4], np.int64).ctypes.data, 4, ip, vp, None,
                                 None) == api.ERR_INVALID


def test_calls_with_null_handle_are_rejected():
    L = api.lib()
    ptrs = (ctypes.c_void_p * 3)()
    assert L.amped_mttkrp(None, 0, 32, ptrs, None, None) == api.ERR_INVALID
    assert L.amped_mttkrp_bf16(None, 0, 32, ptrs, None, None) == api.ERR_INVALID
    assert L.amped_cp_loss(None, 32, ptrs, None, None) == api.ERR_INVALID
    assert L.amped_cp_grad(None, 0, 32, ptrs, ctypes.c_float(1.0), None, None) == api.ERR_INVALID
    assert L.amped_cp_als_sweep(None, 32, ptrs, None, None, 0, None) == api.ERR_INVALID
    assert L.amped_gram(None, 10, 32, None, None) == api.ERR_INVALID
    fake = ctypes.c_void_p(16)   # never dereferenced: the size checks come first
    assert L.amped_gram(fake, 0, 32, fake, None) == api.ERR_INVALID
    assert L.amped_gram(fake, 10, 129, fake, None) == api.ERR_INVALID
    assert L.amped_tensor_info(None, None, None, None, None, None, None, None) == api.ERR_INVALID
    assert L.amped_tensor_layout(None, 0, None, None, None, None, None) == api.ERR_INVALID
    assert L.amped_tensor_destroy(None) == api.OK
    assert L.amped_layout_host(3, np.array([4, 4, 4], np.int64).ctypes.data, 0, None, 5, 8, None,
                               None) == api.ERR_INVALID


def test_create_without_gpu_reports_unsupported():
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    idx = np.zeros((3, 4), np.int32)
    val = np.zeros(4, np.float32)
    assert _create_status(3, [4, 4, 4], 4, idx.ctypes.data, val.ctypes.data) == api.ERR_UNSUPPORTED


def test_host_layout_needs_only_two_shards_of_device_memory():
    """A byte cap that refuses the device-resident layouts of 100k nonzeros
    (about 5 MB) admits the same tensor with host-resident layouts streamed in
    8192-nonzero shards (two staging buffers of about 130 KB); without a GPU
    the call then stops at the device check."""
    rng = np.random.default_rng(3)
    nnz = 100_000
    dims = [500, 400, 300]
    idx = np.stack([rng.integers(0, d, nnz) for d in dims]).astype(np.int32)
    val = rng.random(nnz, dtype=np.float32)
    ip, vp = idx.ctypes.data, val.ctypes.data
    cap = 1 << 20
    assert _create_status(3, dims, nnz, ip, vp, (0, cap, 0, 0, 0)) == api.ERR_NOMEM
    assert _create_status(3, dims, nnz, ip, vp, (0, cap, 0, 1, 8192)) in (api.OK, api.ERR_UNSUPPORTED)
    # the default shard (2^25 nonzeros) is clipped to the tensor: one chunk-rounded shard
    assert _create_status(3, dims, nnz, ip, vp, (0, cap, 0, 1, 0)) == api.ERR_NOMEM


def test_bench_refuses_more_than_one_gpu():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and not r.stdout.strip()
