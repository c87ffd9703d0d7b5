"""Exact solvers for the 1-D TV prox, independent of the oracle's FGP.

  taut_string(v, lam)   -- the taut-string characterisation (Davies & Kovac
                           2001): with prefix sums S_k = v_0 + ... + v_{k-1},
                           the solution's prefix sums F are the shortest path
                           from (0, 0) to (N, S_N) inside the tube |F - S| <=
                           lam; z_i = F_{i+1} - F_i.
  dual_bvls(v, lam)     -- the dual box-constrained least squares
                           min_{|w_i| <= lam} |v - D^T w|^2, z = v - D^T w,
                           solved by scipy's bounded-variable least squares.
  active_set(v, lam)    -- brute force over all 3^(N-1) active sets of that
                           dual (N <= 8): each set fixes some w_i = +-lam and
                           solves the rest as an equality system; the one
                           meeting every KKT condition is the solution.
  nonneg_qp(v, lam)     -- the non-negative 1-D prox from its dual,
                           solved by scipy's L-BFGS-B.

D is the 1-D forward difference (N-1 x N): (D z)_i = z_{i+1} - z_i.
"""

from __future__ import annotations

import itertools

import numpy as np
from scipy.optimize import lsq_linear, minimize


def _dmat(N):
    D = np.zeros((N - 1, N))
    for i in range(N - 1):
        D[i, i] = -1.0
        D[i, i + 1] = 1.0
    return D


def taut_string(v, lam):
    v = np.asarray(v, dtype=np.float64)
    N = len(v)
    S = np.concatenate([[0.0], np.cumsum(v)])
    lo = S - lam
    hi = S + lam
    lo[0] = hi[0] = S[0]
    lo[N] = hi[N] = S[N]
    F = np.empty(N + 1)
    F[0] = S[0]
    k0, y0 = 0, S[0]
    while k0 < N:
        # extend the segment from (k0, y0) as far as a straight line fits the tube
        smax, jmax = -np.inf, -1   # tightest lower slope bound and where
        smin, jmin = np.inf, -1    # tightest upper slope bound and where
        j = k0 + 1
        bend = None
        while j <= N:
            sl = (lo[j] - y0) / (j - k0)
            su = (hi[j] - y0) / (j - k0)
            if sl > smin:
                # the lower tube wall at j rises above the steepest feasible
                # line: the string bends down at the upper-wall contact jmin
                bend = (jmin, hi[jmin])
                break
            if su < smax:
                bend = (jmax, lo[jmax])
                break
            if sl >= smax:
                smax, jmax = sl, j
            if su <= smin:
                smin, jmin = su, j
            j += 1
        if bend is None:
            # the whole rest fits; the endpoint is pinned (lo = hi there)
            slope = (S[N] - y0) / (N - k0)
            for k in range(k0 + 1, N + 1):
                F[k] = y0 + slope * (k - k0)
            break
        jb, yb = bend
        slope = (yb - y0) / (jb - k0)
        for k in range(k0 + 1, jb + 1):
            F[k] = y0 + slope * (k - k0)
        k0, y0 = jb, yb
    return np.diff(F)


def dual_bvls(v, lam):
    v = np.asarray(v, dtype=np.float64)
    N = len(v)
    D = _dmat(N)
    res = lsq_linear(D.T, v, bounds=(-lam * np.ones(N - 1), lam * np.ones(N - 1)),
                     method="bvls", tol=1e-15, max_iter=10000)
    return v - D.T @ res.x


def active_set(v, lam):
    v = np.asarray(v, dtype=np.float64)
    N = len(v)
    assert N <= 8
    D = _dmat(N)
    M = D @ D.T          # Hessian of the dual objective
    c = D @ v            # dual gradient is M w - c
    best = None
    for pattern in itertools.product((-1, 0, 1), repeat=N - 1):
        pat = np.array(pattern)
        free = pat == 0
        w = lam * pat.astype(np.float64)
        if free.any():
            Mf = M[np.ix_(free, free)]
            rhs = c[free] - M[np.ix_(free, ~free)] @ w[~free]
            try:
                w[free] = np.linalg.solve(Mf, rhs)
            except np.linalg.LinAlgError:
                continue
        if np.any(np.abs(w[free]) > lam + 1e-12):
            continue
        grad = M @ w - c
        # KKT: w_i = +lam needs grad_i <= 0, w_i = -lam needs grad_i >= 0
        ok = np.all(grad[pat == 1] <= 1e-10) and np.all(grad[pat == -1] >= -1e-10)
        if ok:
            z = v - D.T @ w
            if best is not None:
                assert np.allclose(best, z, atol=1e-10)
            best = z
    assert best is not None
    return best


def nonneg_qp(v, lam):
    """Non-negative 1-D TV prox from its dual.  For z >= 0 the inner minimum
    over z of 1/2|z - v|^2 + <Dz, w> is attained at z = max(c, 0) with
    c = v - D^T w, and the dual problem becomes
        min_{|w_i| <= lam}  1/2 |max(v - D^T w, 0)|^2,
    a smooth bound-constrained problem solved by scipy's L-BFGS-B."""
    v = np.asarray(v, dtype=np.float64)
    N = len(v)
    D = _dmat(N)

    def f(w):
        c = np.maximum(v - D.T @ w, 0.0)
        return 0.5 * c @ c, -(D @ c)

    r = minimize(f, np.zeros(N - 1), jac=True, method="L-BFGS-B",
                 bounds=[(-lam, lam)] * (N - 1),
                 options=dict(ftol=1e-20, gtol=1e-14, maxiter=100000, maxcor=50))
    return np.maximum(v - D.T @ r.x, 0.0)
