"""Pins of the oracle's TV prox (FGP) and its duality gap.

Independent exact solutions: the 1-D taut string, the dual bounded least
squares (scipy BVLS), brute force over the dual's active sets, a generic QP
solver for the non-negative case, the 2-pixel closed form; invariants the
prox must keep (alpha = 0, constants, mean, shifts); the duality gap as a
certificate that goes to zero.
"""

import math

import numpy as np
import pytest

import oracle as O
import synth
from exact1d import active_set, dual_bvls, nonneg_qp, taut_string


def rng(seed=0):
    return np.random.default_rng(seed)


def test_taut_string_agrees_with_bvls_and_active_set():
    """The three exact 1-D solvers agree with each other (checks the checkers)."""
    r = rng(10)
    for N in (2, 3, 5, 8):
        for _ in range(6):
            v = r.standard_normal(N) * 2
            lam = r.uniform(0.05, 1.5)
            z1 = taut_string(v, lam)
            z2 = dual_bvls(v, lam)
            z3 = active_set(v, lam)
            assert np.allclose(z1, z3, atol=1e-10)
            assert np.allclose(z2, z3, atol=1e-9)
    for N in (40, 97):
        v = r.standard_normal(N)
        lam = 0.4
        assert np.allclose(taut_string(v, lam), dual_bvls(v, lam), atol=1e-9)


@pytest.mark.parametrize("orient", ["row", "col"])
def test_fgp_1d_matches_taut_string(orient):
    r = rng(11)
    N = 24
    v = np.round(r.standard_normal(N), 2) + np.repeat(r.uniform(-1, 1, 4), N // 4)
    lam = 0.3
    ref = taut_string(v, lam)
    img = v[None, :] if orient == "row" else v[:, None]
    z, q = O.fgp(img, lam, 20000)
    assert np.max(np.abs(z.ravel() - ref)) < 1e-8
    g, primal = O.tv_gap(img, lam, q)
    assert 0 <= g < 1e-10 * primal


def test_fgp_column_constant_image_reduces_to_1d():
    """v constant down each column: the 2-D isotropic prox is the 1-D prox
    of one row, repeated (D_y z = 0 at the solution)."""
    r = rng(12)
    W, H = 20, 6
    a = r.standard_normal(W)
    v = np.tile(a, (H, 1))
    lam = 0.25
    z, _ = O.fgp(v, lam, 20000)
    ref = taut_string(a, lam)
    assert np.max(np.abs(z - ref[None, :])) < 1e-8


def test_fgp_two_pixel_closed_form():
    """1x2 image: z = (v1 - lam s, v2 + lam s), s = sign(v1 - v2), if
    |v1 - v2| > 2 lam; otherwise both equal the mean."""
    for v1, v2, lam in [(1.0, 0.0, 0.2), (0.3, 2.0, 0.5), (0.4, 0.5, 0.2), (-1.0, 1.0, 1.0)]:
        z, _ = O.fgp(np.array([[v1, v2]]), lam, 400)
        if abs(v1 - v2) > 2 * lam:
            s = math.copysign(1.0, v1 - v2)
            ref = [v1 - lam * s, v2 + lam * s]
        else:
            ref = [(v1 + v2) / 2] * 2
        assert np.allclose(z.ravel(), ref, atol=1e-12)


def test_fgp_momentum_first_iterations_two_pixels():
    """Worked case of the first three FGP iterations on a 1x2 image with the
    projection inactive (lam large): the dual is one number q (q_x at the
    first pixel), div q = (q, -q), D z = v2 - v1 - 2 q, so one projected
    gradient step from r is q' = r + (v2 - v1 - 2 r) / 8 = 3/4 r + (v2-v1)/8.
    With e = q - q*, q* = (v2 - v1)/2: e' = 3/4 e_r.  Momentum: t_1 = 1,
    t_2 = (1 + sqrt 5)/2, t_3 = (1 + sqrt(1 + 4 t_2^2))/2; r_1 = q_0,
    r_2 = q_1 (coefficient (t_1 - 1)/t_2 = 0), r_3 = q_2 + (t_2 - 1)/t_3 (q_2 - q_1)."""
    v1, v2 = 0.7, -0.4
    qs = (v2 - v1) / 2
    e0 = -qs          # start from q = 0
    e1 = 0.75 * e0
    e2 = 0.75 * e1
    t2 = (1 + math.sqrt(5)) / 2
    t3 = (1 + math.sqrt(1 + 4 * t2 * t2)) / 2
    e3 = 0.75 * (e2 + (t2 - 1) / t3 * (e2 - e1))
    for k, e in [(1, e1), (2, e2), (3, e3)]:
        _, q = O.fgp(np.array([[v1, v2]]), 100.0, k)
        assert abs(q[1, 0, 0] - (qs + e)) < 1e-15
        assert q[1, 0, 1] == 0.0 and np.all(q[0] == 0.0)


def test_fgp_nonneg_1d_matches_qp():
    r = rng(13)
    for _ in range(3):
        N = 12
        v = r.standard_normal(N) * 0.8 + 0.2
        lam = 0.3
        z, q = O.fgp(v[None, :], lam, 30000, nonneg=1)
        ref = nonneg_qp(v, lam)
        assert np.all(z >= 0)
        assert np.max(np.abs(z.ravel() - ref)) < 1e-6
        g, primal = O.tv_gap(v[None, :], lam, q, nonneg=1)
        assert 0 <= g < 1e-9 * primal


def test_fgp_invariants():
    r = rng(14)
    H, W = 17, 23
    v = r.standard_normal((H, W))
    # alpha = 0: identity, bitwise
    z, q = O.fgp(v, 0.0, 50)
    assert np.array_equal(z, v) and np.all(q == 0.0)
    # constant image: fixed point, bitwise
    c = np.full((H, W), 0.37)
    z, q = O.fgp(c, 0.8, 50)
    assert np.array_equal(z, c) and np.all(q == 0.0)
    # mean preserved (sum of a divergence is zero)
    z, _ = O.fgp(v, 0.3, 50)
    assert abs(z.mean() - v.mean()) < 1e-14
    # shift equivariance
    z2, _ = O.fgp(v + 2.5, 0.3, 50)
    assert np.allclose(z2, z + 2.5, atol=1e-12)
    # the dual stays in the ball
    _, q = O.fgp(v, 0.3, 50)
    assert np.all(np.sqrt(q[0] ** 2 + q[1] ** 2) <= 0.3 * (1 + 1e-14))
    # zero iterations: z = v + div(warm q)
    qw = r.standard_normal((2, H, W)) * 0.1
    z, qn = O.fgp(v, 0.3, 0, q=qw)
    assert np.array_equal(qn, qw)
    assert np.allclose(z, v + O.div(qw), atol=0)


def test_fgp_gap_goes_to_zero_and_warm_start_continues():
    """On a crop of the 128x128 denoising phantom: the gap is >= 0, falls as
    iterations grow, reaches a tiny relative value, and warm-starting with
    the returned dual continues the descent."""
    w = synth.WORKLOADS["denoise128"]
    u, eta = synth.make_inputs(w)
    b = (u + w.noise * eta)[40:72, 40:72]
    lam = w.alpha
    gaps = []
    for k in (10, 100, 1000, 10000):
        z, q = O.fgp(b, lam, k)
        g, primal = O.tv_gap(b, lam, q)
        assert g >= 0
        gaps.append(g / primal)
    assert gaps[0] > gaps[1] > gaps[2] > gaps[3]
    assert gaps[3] < 5e-8
    # warm start: 100 more iterations from the 1000-iteration dual beat 1000
    _, q1 = O.fgp(b, lam, 1000)
    _, q2 = O.fgp(b, lam, 100, q=q1)
    assert O.tv_gap(b, lam, q2)[0] < O.tv_gap(b, lam, q1)[0]


def test_gap_is_zero_at_exact_1d_solution_dual():
    """Certificate check of the gap formula: the exact 1-D solution's dual
    (from BVLS) gives gap ~ 0, a perturbed feasible dual gives gap > 0."""
    r = rng(15)
    N = 16
    v = r.standard_normal(N)
    lam = 0.35
    from scipy.optimize import lsq_linear
    D = np.zeros((N - 1, N))
    for i in range(N - 1):
        D[i, i], D[i, i + 1] = -1, 1
    w = lsq_linear(D.T, v, bounds=(-lam, lam), method="bvls", tol=1e-15).x
    q = np.zeros((2, 1, N))
    q[1, 0, :N - 1] = w
    g, primal = O.tv_gap(v[None, :], lam, q)
    assert abs(g) < 1e-12 * primal
    q2 = q.copy()
    q2[1, 0, 3] *= 0.5
    assert O.tv_gap(v[None, :], lam, q2)[0] > 1e-6
