"""Pins of the CP-ALS oracle (oracle/als.py) against facts that do not come
from the oracle itself: the normal equations checked through an explicit
unfolding times Khatri-Rao product, the fit against a dense reconstruction,
the fixed point at exact factors, recovery of a low-rank tensor, the
non-decreasing fit of ALS, and Gram matrices of orthonormal columns.  A few
plausible mistakes (inline mutants) must each fail one of these checks."""
import numpy as np
import pytest

import oracle
from oracle import als


def _cp_tensor(dims, U, lam=None):
    R = U[0].shape[1]
    lam = np.ones(R) if lam is None else lam
    X = np.zeros(dims)
    for r in range(R):
        t = np.array(lam[r])
        for f in U:
            t = np.multiply.outer(t, f[:, r])
        X += t
    return X


def _all_entries(X):
    idx = np.array(np.unravel_index(np.arange(X.size), X.shape), dtype=np.int32)
    return idx, X.ravel().astype(np.float64)


def _sparse(dims, nnz, seed, dup=0):
    rng = np.random.default_rng(seed)
    lin = rng.choice(int(np.prod(dims)), size=nnz, replace=False)
    idx = np.array(np.unravel_index(lin, dims), dtype=np.int32)
    if dup:
        idx = np.concatenate([idx, idx[:, :dup]], axis=1)   # exact duplicates add up
    val = rng.uniform(0.5, 1.5, idx.shape[1])
    return idx, val


def test_gram_of_orthonormal_columns_is_identity():
    rng = np.random.default_rng(1)
    Q, _ = np.linalg.qr(rng.standard_normal((50, 7)))
    np.testing.assert_allclose(als.gram(Q), np.eye(7), atol=1e-12)
    A = rng.standard_normal((40, 5))
    G = als.gram(A)
    assert abs(np.trace(G) - np.sum(A * A)) < 1e-10
    assert np.linalg.eigvalsh(G).min() > -1e-10


def test_tensor_norm_sums_duplicates_first():
    dims = (5, 4, 3)
    idx, val = _sparse(dims, 20, 2, dup=6)
    X = oracle.to_dense(idx, val, dims)        # np.add.at sums duplicates
    assert abs(als.tensor_norm2(idx, val) - np.sum(X * X)) < 1e-10


@pytest.mark.parametrize("convention", ["first_fastest", "cyclic"])
def test_each_update_solves_its_normal_equations(convention):
    """M = X_(d) KR(others) through an explicit unfolding, and the new A_d
    satisfies A_d diag(lambda) V = M with V the Hadamard of the other Grams."""
    dims = (6, 5, 4)
    idx, val = _sparse(dims, 50, 3, dup=4)
    X = oracle.to_dense(idx, val, dims)
    rng = np.random.default_rng(3)
    F0 = [rng.standard_normal((d, 3)) for d in dims]
    trace = []
    F, lam, fit = als.cp_als_sweep(idx, val, dims, F0, trace=trace)
    for step in trace:
        d = step["mode"]
        before = step["factors_before"]
        M_dense = oracle.mttkrp_dense(X, before, d, convention)
        np.testing.assert_allclose(step["M"], M_dense, rtol=1e-12, atol=1e-12)
        V = np.ones((3, 3))
        for w in range(3):
            if w != d:
                V = V * (before[w].T @ before[w])
        A = (F[d] if d == 2 else trace[d + 1]["factors_before"][d])
        np.testing.assert_allclose(A @ np.diag(step["lam"]) @ V, M_dense, rtol=1e-9, atol=1e-10)
        # unit columns
        np.testing.assert_allclose(np.linalg.norm(A, axis=0), 1.0, rtol=1e-12)


def test_fit_matches_dense_reconstruction():
    dims = (5, 4, 6)
    idx, val = _sparse(dims, 40, 4, dup=5)
    X = oracle.to_dense(idx, val, dims)
    rng = np.random.default_rng(4)
    F0 = [rng.standard_normal((d, 2)) for d in dims]
    F, lam, fit = als.cp_als_sweep(idx, val, dims, F0)
    assert abs(fit - als.dense_fit(X, F, lam)) < 1e-10


def test_exact_factors_are_a_fixed_point():
    dims = (6, 5, 4)
    rng = np.random.default_rng(5)
    U = [rng.standard_normal((d, 2)) for d in dims]
    X = _cp_tensor(dims, U)
    idx, val = _all_entries(X)
    F, lam, fit = als.cp_als_sweep(idx, val, dims, U)
    assert fit > 1 - 1e-10
    np.testing.assert_allclose(_cp_tensor(dims, F, lam), X, atol=1e-10)


def test_recovers_a_low_rank_tensor():
    dims = (8, 7, 6)
    rng = np.random.default_rng(6)
    U = [rng.standard_normal((d, 3)) for d in dims]
    X = _cp_tensor(dims, U)
    idx, val = _all_entries(X)
    F = [rng.standard_normal((d, 3)) for d in dims]
    fits = []
    for _ in range(100):
        F, lam, fit = als.cp_als_sweep(idx, val, dims, F)
        fits.append(fit)
    assert fits[-1] > 0.9999, fits[-5:]


def test_fit_never_decreases():
    dims = (9, 8, 7)
    idx, val = _sparse(dims, 120, 7)
    rng = np.random.default_rng(7)
    F = [rng.standard_normal((d, 4)) for d in dims]
    last = -np.inf
    for _ in range(8):
        F, lam, fit = als.cp_als_sweep(idx, val, dims, F)
        assert fit >= last - 1e-12
        last = fit


# ----------------------------------------------------------------- mutants

def _mutant_sweeps():
    """Each returns (factors, lambda, fit) with one plausible mistake."""
    def all_grams(idx, val, dims, factors, trace=None):   # V includes mode d's own Gram
        F = [np.array(f, float) for f in factors]
        G = [f.T @ f for f in F]
        for d in range(3):
            M = oracle.mttkrp(idx, val, dims, F, d)
            V = G[0] * G[1] * G[2]
            A = np.linalg.solve(V, M.T).T
            lam = np.linalg.norm(A, axis=0)
            F[d] = A / lam
            G[d] = F[d].T @ F[d]
        return F, lam, _fit(idx, val, F, lam, M, G)

    def no_norm(idx, val, dims, factors, trace=None):     # lambda kept, columns not scaled
        F = [np.array(f, float) for f in factors]
        G = [f.T @ f for f in F]
        for d in range(3):
            M = oracle.mttkrp(idx, val, dims, F, d)
            V = np.prod([G[w] for w in range(3) if w != d], axis=0)
            F[d] = np.linalg.solve(V, M.T).T
            lam = np.linalg.norm(F[d], axis=0)
            G[d] = F[d].T @ F[d]
        return F, lam, _fit(idx, val, F, lam, M, G)

    def stale_gram(idx, val, dims, factors, trace=None):   # Grams not refreshed after each update
        F = [np.array(f, float) for f in factors]
        G = [f.T @ f for f in F]
        for d in range(3):
            M = oracle.mttkrp(idx, val, dims, F, d)
            V = np.prod([G[w] for w in range(3) if w != d], axis=0)
            A = np.linalg.solve(V, M.T).T
            lam = np.linalg.norm(A, axis=0)
            F[d] = A / lam
        G = [f.T @ f for f in F]
        return F, lam, _fit(idx, val, F, lam, M, G)

    def _fit(idx, val, F, lam, M, G):
        x2 = als.tensor_norm2(idx, val)
        inner = float(np.sum(lam * np.sum(M * F[2], axis=0)))
        xhat2 = float(lam @ (G[0] * G[1] * G[2]) @ lam)
        return 1 - np.sqrt(max(0, x2 - 2 * inner + xhat2)) / np.sqrt(x2)

    return {"all_grams": all_grams, "no_norm": no_norm, "stale_gram": stale_gram}


@pytest.mark.parametrize("name", ["all_grams", "no_norm", "stale_gram"])
def test_mutants_fail_a_pin(name):
    sweep = _mutant_sweeps()[name]
    dims = (8, 7, 6)
    rng = np.random.default_rng(8)
    U = [rng.standard_normal((d, 3)) for d in dims]
    X = _cp_tensor(dims, U)
    idx, val = _all_entries(X)
    failed = []
    # dense fit vs reported fit
    F0 = [rng.standard_normal((d, 3)) for d in dims]
    F, lam, fit = sweep(idx, val, dims, F0)
    if abs(fit - als.dense_fit(X, F, lam)) > 1e-8:
        failed.append("fit")
    # exact factors stay a fixed point
    F, lam, fit = sweep(idx, val, dims, U)
    if not np.allclose(_cp_tensor(dims, F, lam), X, atol=1e-8):
        failed.append("fixed point")
    # unit columns
    if not np.allclose(np.linalg.norm(F[0], axis=0), 1.0):
        failed.append("normalisation")
    assert failed, "mutant %s passed every pin" % name


def test_zero_factor_column_gives_the_smaller_rank_sweep():
    """A zero column r in factor 1 zeroes row and column r of V for the other
    modes: the update leaves column r zero in every mode with lambda_r = 0, and
    the other columns, lambda and the fit are those of the rank R-1 sweep
    without column r."""
    dims = (8, 7, 6)
    idx, val = _sparse(dims, 150, 11)
    rng = np.random.default_rng(11)
    F = [rng.standard_normal((d, 4)) for d in dims]
    F[1][:, 2] = 0.0
    G, lam, fit = als.cp_als_sweep(idx, val, dims, F)
    keep = [0, 1, 3]
    Gs, lams, fits = als.cp_als_sweep(idx, val, dims, [f[:, keep] for f in F])
    for d in range(3):
        assert not G[d][:, 2].any()
        np.testing.assert_allclose(G[d][:, keep], Gs[d], rtol=1e-9, atol=1e-12)
    assert lam[2] == 0.0
    np.testing.assert_allclose(lam[keep], lams, rtol=1e-9)
    assert abs(fit - fits) < 1e-10
