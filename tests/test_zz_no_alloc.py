"""amped_gram_noalloc (the Gram entry point that allocates nothing) through the
C ABI against amped_gram on the same inputs, on consecutive calls that share
the library's fixed device scratch: a large call, then a smaller one, so that
stale partial sums of the first would show in the second."""
import numpy as np
import pytest

from oracle import als
from gpu_util import log

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2507_15121_amd import api  # noqa: E402


def _pair(rows, rank, seed):
    g = torch.Generator(device="cuda").manual_seed(seed)
    A = torch.rand((rows, rank), generator=g, device="cuda") * 2 - 1
    ref = api.gram(A)
    got = torch.full((rank, rank), float("nan"), dtype=torch.float64, device="cuda")
    api.gram_noalloc(A, out=got)
    torch.cuda.synchronize()
    return A, ref.cpu().numpy(), got.cpu().numpy()


@pytest.mark.parametrize("big,small", [((3_000_000, 64), (100_000, 16)), ((5_000_000, 128), (40_000, 128)),
                                       ((2_000_000, 32), (7, 32))])
def test_noalloc_matches_gram_on_two_calls_in_a_row(big, small):
    for k, (rows, rank) in enumerate((big, small)):
        A, ref, got = _pair(rows, rank, seed=rows + rank + k)
        assert np.isfinite(got).all()
        rel = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        oracle_rel = np.linalg.norm(got - als.gram(A.cpu().numpy())) / np.linalg.norm(ref)
        log("gram_noalloc call %d: %d x %d, rel %.2e to amped_gram, %.2e to the oracle" % (k, rows, rank, rel,
                                                                                            oracle_rel))
        if rank <= 64:
            # same slabs, same deterministic summation: the same bits
            np.testing.assert_array_equal(got, ref)
        assert rel <= 1e-6 and oracle_rel <= 1e-6
        np.testing.assert_array_equal(got, got.T)


def test_noalloc_allocates_no_device_memory():
    A = torch.rand((1_000_000, 32), device="cuda")
    out = torch.empty((32, 32), dtype=torch.float64, device="cuda")
    api.gram_noalloc(A, out=out)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for _ in range(3):
        api.gram_noalloc(A, out=out)
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free0


def test_noalloc_argument_errors():
    from ctypes import c_void_p
    L = api.lib()
    A = torch.rand((100, 129), device="cuda")
    G = torch.empty((129, 129), dtype=torch.float64, device="cuda")
    assert L.amped_gram_noalloc(c_void_p(A.data_ptr()), 100, 129, c_void_p(G.data_ptr()), None) == api.ERR_INVALID
    assert "128" in L.amped_last_error().decode()
    assert L.amped_gram_noalloc(c_void_p(A.data_ptr()), 0, 32, c_void_p(G.data_ptr()), None) == api.ERR_INVALID
    assert L.amped_gram_noalloc(None, 100, 32, c_void_p(G.data_ptr()), None) == api.ERR_INVALID
