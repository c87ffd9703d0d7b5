"""Pins of the oracle's comparison methods of the paper: FISTA with the FGP
prox (Alg. "FISTA", Beck-Teboulle momentum) and PDHGSkip-1 (Alg.
"PDHGSkip-1", omega + 1 = 1/p)."""
import math

import numpy as np
import pytest

import oracle as O
import synth


def blur_problem(N=40, seed=3, noise=0.01):
    k = synth.gaussian_blur_kernel(9, 2.0)
    A = O.blur(N, N, k)
    u, eta = synth.phantom_and_noise(N, N, 6, seed, (N, N))
    return A, u, A.apply(u) + noise * eta


def test_fista_first_step_is_a_pgd_step():
    A, _, b = blur_problem()
    x0 = np.random.default_rng(0).standard_normal(b.shape)
    q0 = 0.01 * np.random.default_rng(1).standard_normal((2,) + b.shape)
    f = O.fista(A, b, 0.02, 1.0, 1, 20, x=x0.copy(), q=q0.copy())
    g = O.pgd(A, b, 0.02, 1.0, 1, 20, x=x0.copy(), q=q0.copy())
    assert np.array_equal(f["x"], g["x"]) and np.array_equal(f["q"], g["q"])


def test_fista_rate_bound_with_exact_prox():
    """alpha = 0 makes the prox the identity exactly (FGP with lambda = 0
    returns v bit for bit), so Beck and Teboulle's bound applies:
    Phi(x_k) - Phi* <= 2 L |x_0 - x*|^2 / (k + 1)^2 with b = A u, Phi* = 0,
    x* = u, L = |A|^2 = 1 (step 1/L).  Plain PGD only has the O(1/k) bound
    and is well above the FISTA bound on this ill-conditioned blur."""
    A, u, _ = blur_problem()
    b = A.apply(u)
    K = 400
    f = O.fista(A, b, 0.0, 1.0, K, 1, want_obj=True)
    bound = 2 * np.sum(u ** 2) / (np.arange(1, K + 1) + 1) ** 2
    assert np.all(f["obj"] <= bound)
    g = O.pgd(A, b, 0.0, 1.0, K, 1, want_obj=True)
    assert g["obj"][-1] > 3 * f["obj"][-1]


@pytest.mark.slow
def test_fista_reaches_the_pgd_minimum():
    A, _, b = blur_problem(N=32)
    ref = O.pgd(A, b, 0.02, 1.0, 3000, 100)
    phi_star = O.objective(A, b, ref["x"], 0.02)
    f = O.fista(A, b, 0.02, 1.0, 1500, 100, want_obj=True)
    assert abs(f["obj"][-1] - phi_star) <= 1e-6 * phi_star


def ct(N=24, na=20, nd=35, seed=5):
    ang = synth.parallel_beam_angles(na)
    A = O.joseph(N, N, ang, nd, 2.0 / N, 2.0 / N)
    u, eta = synth.phantom_and_noise(N, N, 6, seed, (na, nd))
    Au = A.apply(u)
    return A, synth.to_f32_exact(Au + 0.01 * Au.max() * eta)


def test_pdhgskip1_at_p1_is_pdhg_bitwise():
    A, b = ct()
    L = A.norm(200)
    r1 = O.pdhgskip1(A, b, 0.05, 1 / L, 1 / L, 1.0, 25, 20, nonneg=1, seed=4)
    r2 = O.pdhg(A, b, 0.05, 1 / L, 1 / L, 25, 20, nonneg=1)
    assert np.all(r1["theta"] == 1)
    for k in ("x", "y", "q"):
        assert np.array_equal(r1[k], r2[k]), k


def test_pdhgskip1_skipped_iterations_keep_x():
    A, b = ct()
    L = A.norm(200)
    rng = np.random.default_rng(3)
    x0 = np.abs(rng.standard_normal((24, 24)))
    y0 = rng.standard_normal(A.out_shape)
    # find an iteration index with theta = 0 for this stream
    k0 = next(k for k in range(100) if O.coin(8, 0, k, 0.3) == 0)
    r = O.pdhgskip1(A, b, 0.05, 0.5 / L, 0.5 / L, 0.3, 1, 20, nonneg=1, seed=8, k0=k0,
                    x=x0.copy(), y=y0.copy())
    assert r["theta"][0] == 0 and r["nprox"] == 0
    assert np.array_equal(r["x"], x0)
    tau = 0.5 / L
    assert np.allclose(r["y"], (y0 + tau * (A.apply(x0) - b)) / (1 + tau), rtol=0, atol=1e-14)


@pytest.mark.slow
def test_pdhgskip1_reaches_the_pdhg_minimum():
    A, b = ct()
    L = A.norm(300)
    ref = O.pdhg(A, b, 0.05, 1 / L, 1 / L, 4000, 200, nonneg=1)
    phi_star = O.objective(A, b, ref["x"], 0.05)
    p = 0.5
    s = 0.99 * math.sqrt(p) / L   # sigma tau (1 + omega) |A|^2 = 0.98 < 1
    r = O.pdhgskip1(A, b, 0.05, s, s, p, 20000, 50, nonneg=1, seed=2, want_obj=True)
    assert abs(r["obj"][-1] - phi_star) <= 1e-6 * phi_star, (r["obj"][-1], phi_star)
