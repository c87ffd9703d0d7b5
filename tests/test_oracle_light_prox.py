"""Pins of the oracle's ProxSkip on the light-prox problems of Sec. 2.1-2.2
(Dual-ROF, Dual-Huber-ROF).

- p = 1 equals the separately written ProjGD bit for bit (reading: the prox
  argument is formed as w + (gamma - gamma / p) h).
- A two-pixel image has a one-dimensional dual: q* = clip((b2 - b1) / (2 +
  eps / alpha), -alpha, alpha), closed form for both problems.
- Without eps the primal iterate b + div q solves TV denoising: on a 1 x N
  image it matches the exact taut-string solver, in 2-D the TV-prox duality
  gap goes to zero.
- With eps > 0 the problem is strongly convex (mu = eps / alpha) and the
  distance to the minimiser shrinks linearly.
"""
import numpy as np
import pytest

import oracle as O
from exact1d import taut_string


@pytest.mark.parametrize("eps", [0.0, 0.05])
def test_p1_is_projgd_bitwise(eps):
    b = np.random.default_rng(1).random((9, 11))
    r = O.dual_rof_proxskip(b, 0.3, eps, 1 / 8, 1.0, 120, seed=3)
    g = O.dual_rof_projgd(b, 0.3, eps, 1 / 8, 120)
    assert r["nprox"] == 120
    assert np.array_equal(r["q"], g["q"])


@pytest.mark.parametrize("b1,b2,alpha,eps", [(0.2, 0.9, 0.5, 0.0), (0.2, 0.9, 0.1, 0.0),
                                             (0.7, 0.1, 0.5, 0.3), (0.7, 0.1, 0.05, 0.3)])
def test_two_pixel_closed_form(b1, b2, alpha, eps):
    b = np.array([[b1, b2]])
    mu = eps / alpha
    q_star = np.clip((b2 - b1) / (2.0 + mu), -alpha, alpha)
    r = O.dual_rof_proxskip(b, alpha, eps, 1.0 / (4.0 + mu), 0.3, 3000, seed=5)
    assert abs(r["q"][1, 0, 0] - q_star) < 1e-12          # the x component at pixel 0
    assert np.all(r["q"][0] == 0)                          # no vertical differences
    np.testing.assert_allclose(r["u"], [[b1 + q_star, b2 - q_star]], atol=1e-12)


def test_rows_match_the_taut_string():
    r = np.random.default_rng(2)
    v = np.repeat([0.1, 0.8, 0.3, 0.6], 8) + 0.05 * r.standard_normal(32)
    b = v[None, :]
    res = O.dual_rof_proxskip(b, 0.2, 0.0, 1 / 8, 0.3, 60000, seed=9)
    z = taut_string(v, 0.2)
    assert np.abs(res["u"][0] - z).max() < 1e-8


def test_duality_gap_vanishes_in_2d():
    r = np.random.default_rng(4)
    b = r.random((24, 20))
    gaps = []
    q = h = None
    for k0 in (0, 5000, 10000, 15000):
        res = O.dual_rof_proxskip(b, 0.15, 0.0, 1 / 8, 0.2, 5000, seed=11, k0=k0, q=q, h=h)
        q, h = res["q"], res["h"]
        gap, primal = O.tv_gap(b, 0.15, q)
        gaps.append(gap / primal)
    assert all(g1 < g0 for g0, g1 in zip(gaps, gaps[1:])), gaps
    assert gaps[-1] < 1e-7
    # skipped steps leave q slightly outside the ball; near the solution the
    # excursion is tiny
    assert np.hypot(res["q"][0], res["q"][1]).max() <= 0.15 * (1 + 1e-6)


def test_huber_linear_convergence():
    r = np.random.default_rng(6)
    b = r.random((16, 18))
    alpha, eps = 0.3, 0.03
    mu = eps / alpha
    gamma = 1 / (8 + mu)
    ref = O.dual_rof_projgd(b, alpha, eps, gamma, 40000)["q"]
    errs = []
    q = h = None
    for k0 in range(0, 1000, 200):
        res = O.dual_rof_proxskip(b, alpha, eps, gamma, np.sqrt(mu / 8), 200, seed=13, k0=k0,
                                  q=q, h=h)
        q, h = res["q"], res["h"]
        errs.append(np.linalg.norm(q - ref))
    # each block of 200 iterations shrinks the error by a sizeable factor
    assert all(e1 < 0.5 * e0 for e0, e1 in zip(errs, errs[1:])), errs
    res = O.dual_rof_proxskip(b, alpha, eps, gamma, np.sqrt(mu / 8), 5000, seed=13, k0=1000,
                              q=q, h=h)
    assert np.linalg.norm(res["q"] - ref) < 1e-12
