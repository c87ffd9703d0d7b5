"""Pins of the oracle's stochastic-angle method (SPDHG over angle subsets
with the prox skipped as in PDHGSkip-2, the paper's "Discussion and Future
work"): the subset draw, the subset operators, the bookkeeping of the dual
blocks, and convergence to the minimiser that the deterministic solvers
reach on the same problem."""
import math

import numpy as np
import pytest

import oracle as O
import synth


def test_subset_draw_uniform_and_pure():
    n, K = 7, 21000
    draws = np.array([O.subset(11, 3, k, n) for k in range(K)])
    assert draws.min() == 0 and draws.max() == n - 1
    counts = np.bincount(draws, minlength=n)
    sd = math.sqrt(K * (1 / n) * (1 - 1 / n))
    assert np.all(np.abs(counts - K / n) < 4.5 * sd)
    # a pure function of (seed, stream, k); other streams and seeds differ
    assert all(O.subset(11, 3, k, n) == draws[k] for k in range(0, K, 997))
    other = np.array([O.subset(11, 4, k, n) for k in range(2000)])
    assert 0.05 < np.mean(other == draws[:2000]) < 0.25
    # independent of the coin on the same (seed, stream): joint frequencies
    # of (theta, subset) factorise
    th = np.array([O.coin(11, 3, k, 0.5) for k in range(K)])
    for j in range(n):
        both = np.sum((th == 1) & (draws == j))
        e = K * 0.5 / n
        assert abs(both - e) < 4.5 * math.sqrt(e)
    assert O.subset(1, 1, 0, 1) == 0 and O.subset(1, 1, -1, 3) == -1 and O.subset(1, 1, 0, 0) == -1


def small_ct(N=24, na=20, nd=35, seed=5):
    ang = synth.parallel_beam_angles(na)
    A = O.joseph(N, N, ang, nd, 2.0 / N, 2.0 / N)
    u, eta = synth.phantom_and_noise(N, N, 6, seed, (na, nd))
    Au = A.apply(u)
    b = synth.to_f32_exact(Au + 0.01 * Au.max() * eta)
    return A, b, ang


@pytest.mark.parametrize("n", [1, 3, 4, 20])
def test_subset_operators_are_rows_of_A(n):
    A, _, ang = small_ct()
    rng = np.random.default_rng(1)
    x = rng.standard_normal((24, 24))
    full = A.apply(x)
    y = rng.standard_normal(full.shape)
    for j in range(n):
        rows = O.subset_rows(len(ang), n, j)
        assert np.array_equal(O.subset_apply(A, n, j, x), full[rows])
        ym = np.zeros_like(y)
        ym[rows] = y[rows]
        assert np.array_equal(O.subset_adjoint(A, n, j, y[rows]), A.adjoint(ym))


def steps(A, na, n, rho=0.99):
    norms = []
    for j in range(n):
        Aj = O.joseph(A.H, A.W, synth.parallel_beam_angles(na)[j::n], A.out_shape[1],
                      2.0 / A.H, 2.0 / A.H)
        norms.append(Aj.norm(300))
    m = max(norms)
    return rho / (n * m), rho / m


def test_one_iteration_touches_only_the_drawn_subset():
    A, b, ang = small_ct()
    n = 4
    sigma, tau = steps(A, len(ang), n)
    rng = np.random.default_rng(2)
    y0 = rng.standard_normal(A.out_shape)
    r = O.spdhgskip(A, b, n, 0.05, sigma, tau, 0.5, 1, 10, nonneg=1, seed=9, y=y0.copy())
    j = int(r["subset"][0])
    assert j == O.subset(9, 0, 0, n)
    others = np.setdiff1d(np.arange(len(ang)), O.subset_rows(len(ang), n, j))
    assert np.array_equal(r["y"][others], y0[others])
    assert not np.array_equal(r["y"][O.subset_rows(len(ang), n, j)],
                              y0[O.subset_rows(len(ang), n, j)])
    assert int(r["theta"][0]) == O.coin(9, 0, 0, 0.5)


@pytest.mark.slow
@pytest.mark.parametrize("n,p", [(1, 1.0), (4, 1.0), (4, 0.3), (10, 0.5)])
def test_converges_to_the_deterministic_minimiser(n, p):
    """Both methods minimise 1/2|Au - b|^2 + alpha TV(u), u >= 0: after
    enough iterations SPDHG with skipped prox reaches the objective of a long
    PDHG run (FGP prox of 200 iterations, warm started) to 1e-6."""
    A, b, ang = small_ct()
    alpha = 0.05
    L = A.norm(300)
    ref = O.pdhg(A, b, alpha, 1 / L, 1 / L, 4000, 200, nonneg=1)
    phi_star = O.objective(A, b, ref["x"], alpha)
    sigma, tau = steps(A, len(ang), n)
    r = O.spdhgskip(A, b, n, alpha, sigma, tau, p, 30000 if n > 1 else 8000, 50, nonneg=1,
                    seed=21, want_obj=True)
    phi = r["obj"][-1]
    assert abs(phi - phi_star) <= 1e-6 * phi_star, (phi, phi_star)
    assert r["x"].min() >= 0
    assert abs(r["nprox"] - p * len(r["theta"])) <= 5 * math.sqrt(len(r["theta"]) * p * (1 - p) + 1)
