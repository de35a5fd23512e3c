"""GPU checks of the CP-ALS building blocks through the C ABI against the
oracle (oracle/als.py): the Gram matrix on the matrix cores and whole sweeps.

Tolerances.  The MTTKRP and Gram matrices are fp32 products with errors of
about 1e-6 relative (fp32 rounding over sums the oracle does in fp64); the
R x R algebra is fp64.  The update A_d = M V^{-1} amplifies relative errors
of M and V by at most cond(V), which is O(1) for the well-spread random
factors used here, so factors and lambda are compared at 1e-4 relative
(Frobenius).  The fit, 1 - sqrt(||X||^2 - 2<X, Xhat> + ||Xhat||^2) / ||X||,
carries an absolute error of about e / (2 (1 - fit)) for a relative error e
of about 2e-6 in <X, Xhat>: 1e-5 absolute for the fits below 0.9 tested
against the oracle, and at most sqrt(2 e) = 2e-3 as the fit nears 1."""
import numpy as np
import pytest

import oracle
from oracle import als
from gpu_util import log

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2507_15121_amd import api, synth  # noqa: E402


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


@pytest.mark.parametrize("rows,rank", [(1, 5), (7, 16), (4097, 32), (100_003, 32), (20_000, 48), (9_000, 64),
                                       (30_001, 100), (5_000, 128)])
def test_gram_vs_oracle(rows, rank):
    rng = np.random.default_rng(rows + rank)
    A = rng.uniform(-1, 1, (rows, rank)).astype(np.float32)
    G = api.gram(_dev(A)).cpu().numpy()
    ref = als.gram(A)
    e = oracle.rel_fro(G, ref)
    log("gram rows=%d R=%d rel %.2e" % (rows, rank, e))
    assert e <= 1e-6
    np.testing.assert_array_equal(G, G.T)


def _sweep_pair(idx, val, dims, rank, seed, sweeps=1, chunk=0):
    rng = np.random.default_rng(seed)
    F0 = [rng.uniform(-1, 1, (d, rank)).astype(np.float32) for d in dims]
    t = api.Tensor(idx, val, dims, chunk_nnz=chunk)
    dF = [_dev(f) for f in F0]
    Fo = [f.astype(np.float64) for f in F0]
    out = []
    for s in range(sweeps):
        lam, fit = api.cp_als_sweep(t, dF)
        torch.cuda.synchronize()
        Fo, lo, fo = als.cp_als_sweep(idx, val, dims, Fo)
        out.append(([f.cpu().numpy() for f in dF], lam.cpu().numpy(), float(fit.item()), Fo, lo, fo))
        # continue both from their own iterates (each step is compared above)
    t.close()
    return out


@pytest.mark.parametrize("rank", [8, 16, 32, 5, 12, 100, 128])
def test_one_sweep_vs_oracle(rank):
    """R = 8/16/32: vector paths; 5 and 12: scalar solve loads and stores;
    100: four-tile Gram groups; 128: the R x R algebra in global memory (its
    4 R^2 doubles exceed the LDS it may use)."""
    dims = (3000, 2000, 1500)
    st = synth.tensor(dims, 60000, "zipf", 1.1, 0.05, seed=40 + rank)
    (F, lam, fit, Fo, lo, fo), = _sweep_pair(st.idx, st.val, dims, rank, seed=rank)
    errs = [oracle.rel_fro(F[d], Fo[d]) for d in range(3)]
    log("ALS R=%d factor errs %s lambda %.2e fit %.6f vs %.6f" %
        (rank, ["%.1e" % e for e in errs], oracle.rel_fro(lam, lo), fit, fo))
    assert max(errs) <= 1e-4
    assert oracle.rel_fro(lam, lo) <= 1e-4
    assert abs(fit - fo) <= 1e-5


@pytest.mark.parametrize("reuse", [False, True])
def test_sweeps_track_oracle_and_fit_rises(reuse):
    """A sparse sample of an exact rank-4 model plus 1% noise: 8 sweeps from a
    random start, each compared with the oracle's sweep from the same start.
    reuse: every sweep after the first takes the Gram matrices the one before
    left (computed from M and the update, not from the stored factors)."""
    dims = (800, 600, 500)
    rng = np.random.default_rng(50)
    U = [rng.uniform(0.1, 1.0, (d, 4)) for d in dims]
    lin = rng.choice(dims[0] * dims[1] * dims[2], size=40000, replace=False)
    idx = np.array(np.unravel_index(lin, dims), dtype=np.int32)
    val = np.sum(U[0][idx[0]] * U[1][idx[1]] * U[2][idx[2]], axis=1)
    val = (val * (1 + 0.01 * rng.standard_normal(val.size))).astype(np.float32)
    t = api.Tensor(idx, val, dims)
    F0 = [rng.uniform(-1, 1, (d, 4)).astype(np.float32) for d in dims]
    dF = [_dev(f) for f in F0]
    fits = []
    for s in range(8):
        start = [f.cpu().numpy().astype(np.float64) for f in dF]
        lam, fit = api.cp_als_sweep(t, dF, reuse_grams=reuse and s > 0)
        Fo, lo, fo = als.cp_als_sweep(idx, val, dims, start)
        f = float(fit.item())
        log("sweep %d fit %.6f oracle %.6f" % (s, f, fo))
        assert abs(f - fo) <= 1e-5
        for d in range(3):
            assert oracle.rel_fro(dF[d].cpu().numpy(), Fo[d]) <= 1e-4
        fits.append(f)
    assert all(b >= a - 1e-6 for a, b in zip(fits, fits[1:]))
    t.close()


def test_exact_factors_are_a_fixed_point():
    """From the exact factors of a fully stored rank-4 tensor, one sweep
    reproduces the tensor (checked on the reconstruction, 1e-5 relative).  The
    reported fit comes from ||X||^2 - 2<X, Xhat> + ||Xhat||^2, which cancels
    as the fit nears 1: an error e of about 2e-6 relative in <X, Xhat> (fp32
    MTTKRP and Gram products) leaves a fit error of at most sqrt(2 e) = 2e-3."""
    dims = (40, 30, 20)
    rng = np.random.default_rng(60)
    U = [rng.uniform(-1, 1, (d, 4)) for d in dims]
    X = np.einsum("ir,jr,kr->ijk", U[0], U[1], U[2])
    idx = np.array(np.unravel_index(np.arange(X.size), dims), dtype=np.int32)
    val = X.ravel().astype(np.float32)
    t = api.Tensor(idx, val, dims)
    dF = [_dev(u) for u in U]
    lam, fit = api.cp_als_sweep(t, dF)
    F = [f.cpu().numpy().astype(np.float64) for f in dF]
    Xhat = np.einsum("r,ir,jr,kr->ijk", lam.cpu().numpy(), F[0], F[1], F[2])
    e = oracle.rel_fro(Xhat, X)
    log("fixed point: reconstruction rel %.2e, fit %.8f" % (e, fit.item()))
    assert e <= 1e-5
    assert fit.item() >= 1 - 2e-3
    t.close()


def test_duplicates_add_up_in_the_fit():
    dims = (500, 400, 300)
    st = synth.tensor(dims, 20000, "zipf", 1.1, 0.0, seed=70)
    idx = np.concatenate([st.idx, st.idx[:, :3000]], axis=1)        # 3000 exact duplicates
    val = np.concatenate([st.val, st.val[:3000] * 0.5])
    (F, lam, fit, Fo, lo, fo), = _sweep_pair(idx, val, dims, 8, seed=7, chunk=512)
    log("duplicates: fit %.6f oracle %.6f" % (fit, fo))
    assert abs(fit - fo) <= 1e-5
    assert max(oracle.rel_fro(F[d], Fo[d]) for d in range(3)) <= 1e-4


def test_order_four():
    dims = (600, 500, 400, 50)
    st = synth.tensor(dims, 30000, "zipf", 1.2, 0.0, seed=80)
    (F, lam, fit, Fo, lo, fo), = _sweep_pair(st.idx, st.val, dims, 16, seed=8)
    errs = [oracle.rel_fro(F[d], Fo[d]) for d in range(4)]
    log("order 4: errs %s fit %.6f vs %.6f" % (["%.1e" % e for e in errs], fit, fo))
    assert max(errs) <= 1e-4 and abs(fit - fo) <= 1e-5


def test_reuse_needs_a_previous_sweep_at_that_rank():
    dims = (300, 200, 100)
    st = synth.tensor(dims, 5000, "zipf", 1.1, 0.0, seed=90)
    t = api.Tensor(st.idx, st.val, dims)
    rng = np.random.default_rng(9)
    dF = [_dev(rng.uniform(-1, 1, (d, 8))) for d in dims]
    with pytest.raises(api.AmpedError):
        api.cp_als_sweep(t, dF, reuse_grams=True)          # no sweep yet
    api.cp_als_sweep(t, dF)
    api.cp_als_sweep(t, dF, reuse_grams=True)
    dG = [_dev(rng.uniform(-1, 1, (d, 16))) for d in dims]
    with pytest.raises(api.AmpedError):
        api.cp_als_sweep(t, dG, reuse_grams=True)          # another rank
    torch.cuda.synchronize()
    t.close()


@pytest.mark.parametrize("dims,rank", [((3000, 2000), 16), ((300, 250, 200, 150, 40), 8)])
def test_orders_two_and_five(dims, rank):
    """Order 2 (V is a single Gram matrix) and order 5 (V the Hadamard of four)."""
    st = synth.tensor(dims, 20000, "zipf", 1.1, 0.0, seed=len(dims) + 90)
    (F, lam, fit, Fo, lo, fo), = _sweep_pair(st.idx, st.val, dims, rank, seed=len(dims))
    errs = [oracle.rel_fro(F[d], Fo[d]) for d in range(len(dims))]
    log("order %d: errs %s fit %.6f vs %.6f" % (len(dims), ["%.1e" % e for e in errs], fit, fo))
    assert max(errs) <= 1e-4 and abs(fit - fo) <= 1e-5
    assert oracle.rel_fro(lam, lo) <= 1e-4


def test_zero_factor_column_stays_zero():
    """A zero column in factor 1 makes V singular for the other modes (its
    pivot is replaced by a tiny one on the GPU): column 2 of every factor ends
    zero with lambda 0, and the rest follows the oracle's restricted solve."""
    dims = (2000, 1500, 1000)
    st = synth.tensor(dims, 40000, "zipf", 1.1, 0.0, seed=95)
    rng = np.random.default_rng(95)
    F0 = [rng.uniform(-1, 1, (d, 8)).astype(np.float32) for d in dims]
    F0[1][:, 2] = 0.0
    t = api.Tensor(st.idx, st.val, dims)
    dF = [_dev(f) for f in F0]
    lam, fit = api.cp_als_sweep(t, dF)
    torch.cuda.synchronize()
    Fo, lo, fo = als.cp_als_sweep(st.idx, st.val, dims, [f.astype(np.float64) for f in F0])
    F = [f.cpu().numpy() for f in dF]
    lam = lam.cpu().numpy()
    log("zero column: lambda %s, fit %.6f vs %.6f" % (lam, float(fit.item()), fo))
    for d in range(3):
        assert not F[d][:, 2].any()
        assert oracle.rel_fro(F[d], Fo[d]) <= 1e-4
    assert lam[2] == 0.0 and lo[2] == 0.0
    assert oracle.rel_fro(lam, lo) <= 1e-4
    assert abs(float(fit.item()) - fo) <= 1e-5
    t.close()


def _backward_error(A, V, M):
    """Normwise backward error of A as a solution of A V = M up to a scale per
    column of A (the update's columns are normalised): the scales s minimise
    ||A diag(s) V - M||_F (a small least-squares problem), and the residual is
    taken relative to ||A diag(s)||_F ||V||_2 + ||M||_F."""
    R = A.shape[1]
    D = np.stack([np.outer(A[:, r], V[r, :]).ravel() for r in range(R)], axis=1)
    s, *_ = np.linalg.lstsq(D, M.ravel(), rcond=None)
    As = A * s
    return float(np.linalg.norm(As @ V - M) / (np.linalg.norm(As) * np.linalg.norm(V, 2) + np.linalg.norm(M)))


@pytest.mark.parametrize("delta", [1e-1, 1e-2, 1e-3])
def test_nearly_collinear_columns_tolerance_scaled_by_condition(delta):
    """Modes 1 and 2 start with column 1 = column 0 + delta * noise, so the
    mode-0 system V = (A_1^T A_1) * (A_2^T A_2) is ill-conditioned (cond(V)
    about 2e2, 2e4 and 2e6; the update sums M W in fp32 at the first and in
    fp64 at the other two, whose 1-norm condition exceeds 1e4).  The update A_0 = M V^{-1} amplifies the fp32 errors of
    M and V (about 1e-6 relative) by up to cond(V), so the GPU's mode-0 factor
    is compared with the oracle's at max(1e-4, 1e-6 cond(V)) where that bound
    says something (below 0.5).  Whatever the conditioning, a backward-stable
    solve leaves a normwise backward error near the data's own error: the GPU
    factor must solve the oracle's system A V = M (fp64 M and V from the same
    starting factors) to 1e-5.  The GPU inverts V by Gauss-Jordan elimination
    without pivoting, which is stable for symmetric positive definite V."""
    dims = (3000, 2000, 1500)
    R = 16
    st = synth.tensor(dims, 60000, "zipf", 1.1, 0.05, seed=77)
    rng = np.random.default_rng(77)
    F0 = [rng.uniform(-1, 1, (d, R)) for d in dims]
    for w in (1, 2):
        F0[w][:, 1] = F0[w][:, 0] + delta * rng.uniform(-1, 1, dims[w])
    F0 = [f.astype(np.float32) for f in F0]
    trace = []
    Fo, lo, fo = als.cp_als_sweep(st.idx, st.val, dims, [f.astype(np.float64) for f in F0], trace=trace)
    V, M = trace[0]["V"], trace[0]["M"]
    cond = float(np.linalg.cond(V))
    t = api.Tensor(st.idx, st.val, dims)
    dF = [_dev(f) for f in F0]
    lam, fit = api.cp_als_sweep(t, dF)
    torch.cuda.synchronize()
    F = [f.cpu().numpy() for f in dF]
    t.close()
    e0 = oracle.rel_fro(F[0], Fo[0])
    tol = max(1e-4, 1e-6 * cond)
    eta = _backward_error(F[0].astype(np.float64), V, M)
    eta_ref = _backward_error(Fo[0], V, M)
    log("ALS delta=%g: cond(V_0) %.2e (1-norm %.2e), mode-0 factor rel %.2e (bound %.2e), backward error %.2e "
        "(oracle's own %.2e), fit %.6f vs %.6f" % (delta, cond, np.linalg.cond(V, 1), e0, tol, eta, eta_ref,
                                                 float(fit.item()), fo))
    assert cond > 1e2, "the test must exercise an ill-conditioned V"
    assert all(np.isfinite(f).all() for f in F) and np.isfinite(lam.cpu().numpy()).all()
    if tol < 0.5:
        assert e0 <= tol
    assert eta <= 1e-5
