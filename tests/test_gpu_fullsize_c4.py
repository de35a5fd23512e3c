"""Full-size checks of the differentiable sparse CP model on the order-4
tensor (50M x 20M x 1M x 100k, 500M nonzeros, Zipf 1.2 per mode, R=32): the
loss against the FP64 oracle over all nonzeros, the fused residual + MTTKRP
gradient of every mode on sampled rows against the oracle gradient restricted
to those rows' nonzeros, and the directional finite difference of the GPU
loss against the GPU gradients, all in the launch configuration the benchmark
times."""
import numpy as np
import pytest

import oracle
from gpu_util import log, oracle_grad_rows, oracle_loss, sample_rows

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2507_15121_amd import api, autograd, synth  # noqa: E402

WORKLOAD = "zipf4-50Mx20Mx1Mx100k-500M"


@pytest.fixture(scope="module")
def c4():
    w = synth.WORKLOADS[WORKLOAD]
    log("generating %s" % w.name)
    st = synth.workload(w.name)
    factors = synth.factors(st.dims, w.rank)
    log("building layouts")
    T = api.Tensor(st.idx, st.val, st.dims)
    dfac = [torch.from_numpy(f).cuda() for f in factors]
    torch.cuda.synchronize()
    yield st, factors, T, dfac
    T.close()


def test_c4_loss_vs_oracle(c4):
    st, factors, T, dfac = c4
    loss = float(api.cp_loss(T, dfac))
    ref = oracle_loss(st.idx, st.val, factors)
    log("loss %.10e, oracle %.10e, rel %.2e" % (loss, ref, abs(loss - ref) / ref))
    assert abs(loss - ref) <= 1e-5 * abs(ref)


def test_c4_gradient_sampled_rows(c4):
    st, factors, T, dfac = c4
    rng = np.random.default_rng(41)
    for d in range(4):
        g = torch.full(tuple(dfac[d].shape), float("nan"), dtype=torch.float32, device="cuda")
        api.cp_grad(T, d, dfac, -2.0, out=g)
        torch.cuda.synchronize()
        assert not torch.isnan(g).any().item(), "mode %d gradient left elements unwritten" % d
        rows, counts, untouched = sample_rows(st.idx[d], st.dims[d], rng, 100)
        if untouched.size:
            assert not g[torch.from_numpy(untouched).cuda()].any().item()
        got = g[torch.from_numpy(rows).cuda()].cpu().numpy()
        del g
        ref = oracle_grad_rows(st.idx, st.val, st.dims, factors, d, rows)
        e = oracle.rel_fro(got, ref)
        k = int(np.searchsorted(rows, int(np.argmax(counts))))
        eh = oracle.rel_fro(got[k][None], ref[k][None])
        log("grad mode %d: %d sampled rows rel %.2e, heaviest row (%d nnz) rel %.2e" %
            (d, rows.size, e, int(counts.max()), eh))
        assert e <= 1e-5 and eh <= 1e-5


def test_c4_directional_finite_difference(c4):
    """[L(A + eps V) - L(A - eps V)] / (2 eps) against <grad L, V> for a seeded
    random direction V over all four factors, with the gradients from the
    autograd function's backward (the fused kernels) and the losses summed in
    fp64; the central difference of a quartic loss has a truncation error of
    order eps^2, far below the 1e-3 bar at eps = 1e-3."""
    st, factors, T, dfac = c4
    A = [f.clone().requires_grad_(True) for f in dfac]
    L = autograd.SparseCPLoss.apply(T, *A)
    L.backward()
    gen = torch.Generator(device="cuda").manual_seed(4321)
    V = [torch.rand(f.shape, generator=gen, device="cuda") * 2 - 1 for f in dfac]

    def dot64(x, y, chunk=1 << 24):
        x, y = x.reshape(-1), y.reshape(-1)
        return sum(float((x[i:i + chunk].double() * y[i:i + chunk].double()).sum())
                   for i in range(0, x.numel(), chunk))
    dd = sum(dot64(a.grad, v) for a, v in zip(A, V))
    eps = 1e-3
    lp = float(api.cp_loss(T, [f + eps * v for f, v in zip(dfac, V)]))
    lm = float(api.cp_loss(T, [f - eps * v for f, v in zip(dfac, V)]))
    fd = (lp - lm) / (2 * eps)
    rel = abs(fd - dd) / abs(dd)
    log("directional derivative %.8e, central difference %.8e, rel %.2e" % (dd, fd, rel))
    assert rel <= 1e-3
