"""CPU oracle for one CP-ALS sweep around sparse MTTKRP.

TEST INFRASTRUCTURE (same rules as the rest of ``oracle/``): only the tests,
``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may use
it; it shares no code with the HIP path.

CPD by alternating least squares (Sec. 2.1; Alg. 1's mode loop) computes, for
each mode d in turn, the MTTKRP of Eq. 2 with the current factors.  The paper
does not spell out what is done with that MTTKRP; the standard CP-ALS update
is taken here (the reading is listed with the others in the design notes):

    M   = X_(d) (Khatri-Rao product of the other factors)      (Eq. 1/2)
    V   = Hadamard product over w != d of  A_w^T A_w             (R x R)
    A_d = M V^{-1}                      (least-squares solution for mode d)
          V_rr = prod_{w != d} ||A_w(:, r)||^2 is zero exactly when some other
          factor's column r is zero; then row and column r of V are zero, the
          system is solved on the other indices and A_d(:, r) = 0 (the
          minimum-norm solution)
    lambda_r = ||A_d(:, r)||_2,  A_d(:, r) /= lambda_r   (0-norm columns stay 0)

and after the last mode the fit of the CP model to the full tensor (missing
entries are zeros):

    ||X - Xhat||^2 = ||X||^2 - 2 <X, Xhat> + ||Xhat||^2
    <X, Xhat>      = sum_r lambda_r sum_i M(i, r) A_d(i, r)        (last mode)
    ||Xhat||^2     = lambda^T (Hadamard over all w of A_w^T A_w) lambda
    fit            = 1 - ||X - Xhat|| / ||X||

All in float64; the MTTKRP is the oracle's per-nonzero definition.  ||X||^2 is
taken over distinct coordinates (duplicates add up first).
"""
import numpy as np

from . import mttkrp as _mttkrp


def gram(A):
    """A^T A in float64 (a matmul as a library step)."""
    A = np.asarray(A, dtype=np.float64)
    return A.T @ A


def tensor_norm2(idx, val):
    """||X||^2 with exact duplicates summed before squaring."""
    idx = np.asarray(idx)
    val = np.asarray(val, dtype=np.float64)
    if val.size == 0:
        return 0.0
    order = np.lexsort(idx[::-1])
    s = idx[:, order]
    v = val[order]
    new = np.ones(v.size, dtype=bool)
    new[1:] = np.any(s[:, 1:] != s[:, :-1], axis=0)
    sums = np.add.reduceat(v, np.flatnonzero(new))
    return float(np.sum(sums * sums))


def cp_als_sweep(idx, val, dims, factors, trace=None):
    """One sweep over the modes 0..N-1.  Returns (factors, lambda, fit).

    ``trace``: if a list, per-mode dicts {mode, M, V, lam, factors_before}
    are appended (for the pins)."""
    N = len(dims)
    F = [np.array(f, dtype=np.float64) for f in factors]
    R = F[0].shape[1]
    G = [gram(f) for f in F]
    lam = np.ones(R)
    M = None
    for d in range(N):
        before = [f.copy() for f in F]
        M = _mttkrp(idx, val, dims, F, d)
        V = np.ones((R, R))
        for w in range(N):
            if w != d:
                V = V * G[w]
        live = np.diag(V) > 0
        if live.all():
            A = np.linalg.solve(V, M.T).T      # M V^{-1}; V is symmetric
        else:
            A = np.zeros_like(M)
            if live.any():
                A[:, live] = np.linalg.solve(V[np.ix_(live, live)], M[:, live].T).T
        lam = np.sqrt(np.sum(A * A, axis=0))
        nz = lam > 0
        A[:, nz] = A[:, nz] / lam[nz]
        A[:, ~nz] = 0.0
        F[d] = A
        G[d] = gram(A)
        if trace is not None:
            trace.append({"mode": d, "M": M, "V": V, "lam": lam.copy(), "factors_before": before})
    x2 = tensor_norm2(idx, val)
    inner = float(np.sum(lam * np.sum(M * F[N - 1], axis=0)))
    H = np.ones((R, R))
    for w in range(N):
        H = H * G[w]
    xhat2 = float(lam @ H @ lam)
    fit = 1.0 - np.sqrt(max(0.0, x2 - 2.0 * inner + xhat2)) / np.sqrt(x2) if x2 > 0 else 0.0
    return F, lam, fit


def dense_fit(X, factors, lam):
    """Brute-force fit on a dense tensor: Xhat built from outer products."""
    N = X.ndim
    R = factors[0].shape[1]
    Xhat = np.zeros(X.shape)
    for r in range(R):
        t = np.array(lam[r])
        for w in range(N):
            t = np.multiply.outer(t, factors[w][:, r])
        Xhat += t
    return 1.0 - np.linalg.norm(X - Xhat) / np.linalg.norm(X)
