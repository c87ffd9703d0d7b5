"""Pins of the oracle's inner-solver skip (the paper's "Discussion and Future
work": skipping inside the inner solver): the TV prox solved by ProxSkip on
its dual, and ProxSkip / PDHGSkip-2 that call it.

- Without the constraint the inner solver is ProxSkip on Dual-ROF: it equals
  the separately written Dual-ROF routine bit for bit, and ProjGD at p = 1.
- On a 1 x N image it reaches the exact taut-string solution; with z >= 0 it
  reaches max(taut string, 0) (for TV on a chain and a box constraint the
  prox of the sum is the clipped TV prox, Yu 2013, "On decomposing the
  proximal map").
- In 2-D the constrained TV-prox duality gap of its dual iterate goes to
  zero; where the constraint is inactive the constrained run equals the
  unconstrained one bit for bit.
- The outer methods: one ProxSkip step at p = 1 on A = I, gamma = 1 is the
  TV prox of b; long runs reach the minimiser of the independent reference
  solvers; resuming at k0 with the carried state is bitwise.
"""
import math

import numpy as np
import pytest

import oracle as O
import synth
from exact1d import taut_string


def _rows(seed=3, n=32, lo=-0.3):
    r = np.random.default_rng(seed)
    return np.repeat([lo, 0.5, -0.1, 0.4], n // 4) + 0.05 * r.standard_normal(n)


def test_unconstrained_is_dual_rof_proxskip_bitwise():
    v = np.random.default_rng(1).random((9, 13))
    a = O.tv_prox_skip(v, 0.2, 150, 0.3, nonneg=0, seed=4, stream=6, k0=17)
    b = O.dual_rof_proxskip(v, 0.2, 0.0, 1 / 8, 0.3, 150, seed=4, stream=6, k0=17)
    assert a["nproj"] == b["nprox"]
    assert np.array_equal(a["q"], b["q"]) and np.array_equal(a["h"], b["h"])
    np.testing.assert_array_equal(a["z"], v + O.div(a["q"]))


def test_p1_is_projgd():
    v = np.random.default_rng(2).random((10, 7))
    a = O.tv_prox_skip(v, 0.25, 90, 1.0, seed=1)
    g = O.dual_rof_projgd(v, 0.25, 0.0, 1 / 8, 90)
    assert a["nproj"] == 90
    assert np.array_equal(a["q"], g["q"])


@pytest.mark.parametrize("nonneg", [0, 1])
def test_rows_match_the_taut_string(nonneg):
    v = _rows()
    z = taut_string(v, 0.15)
    if nonneg:
        z = np.maximum(z, 0.0)
    res = O.tv_prox_skip(v[None, :], 0.15, 60000, 0.3, nonneg=nonneg, seed=2)
    assert np.abs(res["z"][0] - z).max() < 1e-10
    assert 0.25 * 60000 < res["nproj"] < 0.35 * 60000


def test_nonneg_gap_vanishes_in_2d():
    b = np.random.default_rng(5).random((20, 18)) - 0.3
    q = h = None
    gaps = []
    for k0 in (0, 4000, 8000, 12000):
        r = O.tv_prox_skip(b, 0.1, 4000, 0.25, nonneg=1, seed=7, k0=k0, q=q, h=h)
        q, h = r["q"], r["h"]
        gap, primal = O.tv_gap(b, 0.1, q, nonneg=1)
        gaps.append(gap / primal)
    assert all(g1 < g0 for g0, g1 in zip(gaps, gaps[1:])), gaps
    assert gaps[-1] < 1e-11
    assert r["z"].min() >= 0.0 and (r["z"] == 0).sum() > 0
    # the unconstrained prox of the same b goes negative: the constraint binds
    assert O.tv_prox_skip(b, 0.1, 4000, 0.25, seed=7)["z"].min() < 0


def test_inactive_constraint_changes_nothing():
    v = 1.0 + np.random.default_rng(5).random((12, 11))
    a = O.tv_prox_skip(v, 0.05, 300, 0.2, nonneg=1, seed=3)
    b = O.tv_prox_skip(v, 0.05, 300, 0.2, nonneg=0, seed=3)
    assert np.array_equal(a["q"], b["q"]) and np.array_equal(a["z"], b["z"])


# ---------------------------------------------------------------- outer methods
@pytest.mark.parametrize("nonneg", [0, 1])
def test_one_denoising_step_is_the_tv_prox(nonneg):
    """A = I, gamma = 1, p = 1: w = x - (x - b) = b and the step returns
    prox_{alpha TV}(b) (clipped at 0 with the constraint)."""
    v = _rows(7)
    A = O.identity(1, v.size)
    r = O.proxskip_inner(A, v[None, :], 0.15, 1.0, 1.0, 1, 60000, 0.3, nonneg=nonneg, seed=5)
    z = taut_string(v, 0.15)
    if nonneg:
        z = np.maximum(z, 0.0)
    assert r["nprox"] == 1
    assert np.abs(r["x"][0] - z).max() < 1e-10
    # the outer control variate: h = (p / gamma) (z - xhat) with xhat = b
    assert np.abs(r["h"][0] - (z - v)).max() < 1e-10


def test_proxskip_inner_reaches_the_denoising_minimiser():
    u, eta = synth.phantom_and_noise(24, 24, 5, 3, (24, 24))
    b = u + 0.05 * eta
    alpha = 0.1
    ustar, qs = O.fgp(b, alpha, 40000)
    gap, _ = O.tv_gap(b, alpha, qs)
    A = O.identity(24, 24)
    # an inexact prox: the objective error shrinks like 1/k, not linearly
    # (1.7e-7 after 3000 iterations, 3.0e-8 after 12000)
    r = O.proxskip_inner(A, b, alpha, 1.0, 0.3, 3000, 100, 0.3, seed=11)
    phi, phis = O.objective(A, b, r["x"], alpha), O.objective(A, b, ustar, alpha)
    assert phi - (phis - gap) <= 3e-7 * phis
    bound = math.sqrt(2 * max(phi - phis + gap, 0)) + math.sqrt(2 * gap)
    assert np.linalg.norm(r["x"] - ustar) <= bound + 1e-9
    assert 0.2 * 100 * r["nprox"] < r["nproj"] < 0.4 * 100 * r["nprox"]


def test_pdhgskip_inner_ct_reaches_the_reference_minimiser(ct24_reference):
    A, b, alpha, ref = ct24_reference
    L = A.norm(200)
    r = O.pdhgskip_inner(A, b, alpha, 1 / L, 1 / L, 0.3, 8000, 30, 0.3, nonneg=1, seed=8)
    phis = [O.objective(A, b, x, alpha) for x in (ref["x"], r["x"])]
    assert abs(phis[1] - phis[0]) <= 1e-6 * phis[0]
    assert r["x"].min() >= 0
    assert np.max(np.abs(r["x"] - ref["x"])) < 1e-3 * np.max(np.abs(ref["x"]))


def test_inner_resume_is_bitwise():
    u, eta = synth.phantom_and_noise(16, 16, 5, 2, (16, 16))
    b = u + 0.05 * eta
    A = O.identity(16, 16)
    kw = dict(seed=77, stream=3, nonneg=1)
    full = O.pdhgskip_inner(A, b, 0.1, 1.0, 1.0, 0.4, 30, 6, 0.3, **kw)
    a = O.pdhgskip_inner(A, b, 0.1, 1.0, 1.0, 0.4, 13, 6, 0.3, **kw)
    c = O.pdhgskip_inner(A, b, 0.1, 1.0, 1.0, 0.4, 17, 6, 0.3, k0=13, x=a["x"], h=a["h"],
                         y=a["y"], q=a["q"], h_in=a["h_in"], **kw)
    for key in ("x", "h", "y", "q", "h_in"):
        assert np.array_equal(full[key], c[key]), key
    assert full["nproj"] == a["nproj"] + c["nproj"]


def test_inner_coins_come_from_their_own_stream():
    """The prox call at outer iteration k draws inner coins on stream
    stream xor 2^62 at indices k K_in + i."""
    b = np.random.default_rng(9).random((8, 8))
    A = O.identity(8, 8)
    K_in, p, p_in, seed, stream = 7, 0.5, 0.3, 21, 5
    r = O.proxskip_inner(A, b, 0.1, 1.0, p, 40, K_in, p_in, seed=seed, stream=stream)
    want = sum(O.coin(seed, stream ^ O.INNER_STREAM, k * K_in + i, p_in)
               for k in range(40) if r["theta"][k] for i in range(K_in))
    assert r["nproj"] == want
    assert r["nprox"] == int(r["theta"].sum())
