"""Checks of the stored reference minima Phi* (tests/golden/phi_star_*.json,
written by tests/golden/make_phi_star.py from the CPU oracle only).

- denoise128: Phi is the TV prox objective of b (lambda = alpha), so weak
  duality brackets the true minimum with any dual point: a short FGP run
  from zero gives D(q) = P(z_q) - gap(q) <= Phi* <= P(z_q).  The stored value
  must sit in that bracket, and its own certificate must be tight.
- ct512 / deblur512: Phi* is a minimum, so it cannot exceed the objective at
  the zero image; the stored trajectory must be non-increasing at its end
  and its last chunk must have changed by less than the stopping tolerance.
  A second float64 method (the oracle's explicit diagonally preconditioned
  PDHG, no inner solver) must agree to 1e-7 relative after meeting its own
  stopping rule, and the stored value must lie inside the weak-duality
  bracket written beside it (a dual point made exactly feasible).
- The bracket itself (make_phi_star.certificate) on a small CT problem: it
  contains the objective of a long run and is tight there, and at a
  perturbed point its width is at least the perturbation's excess.
"""
import json
import os
import sys

import numpy as np
import pytest

import oracle as O
import synth

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
if HERE not in sys.path:
    sys.path.insert(0, HERE)


def load(name):
    path = os.path.join(HERE, f"phi_star_{name}.json")
    if not os.path.exists(path):
        pytest.skip(f"{path} not generated")
    return json.load(open(path))


def test_denoise128_bracketed_by_weak_duality():
    d = load("denoise128")
    w = synth.WORKLOADS["denoise128"]
    u, eta = synth.make_inputs(w)
    b = u + w.noise * eta
    _, q = O.fgp(b, w.alpha, 300, 0)
    gap, primal = O.tv_gap(b, w.alpha, q)
    phi = d["phi_star"]
    assert primal - gap <= phi <= primal
    lo, hi = d["certificate"]
    assert lo <= phi <= hi and hi - lo <= 1e-9 * phi
    # the workload's objective at the primal point of q is the prox primal
    # value (the identity that makes the prox minimum the workload's Phi*)
    z, _ = O.fgp(b, w.alpha, 0, 0, q=q)
    assert abs(O.objective(O.identity(w.H, w.W), b, z, w.alpha) - primal) <= 1e-12 * primal


@pytest.mark.parametrize("name", ["ct512", "deblur512"])
def test_minimum_below_zero_image_and_converged(name):
    d = load(name)
    w = synth.WORKLOADS[name]
    u, eta = synth.make_inputs(w)
    if name == "ct512":
        A = O.joseph(w.H, w.W, synth.parallel_beam_angles(w.n_ang), w.n_det, w.pixel,
                     w.det_spacing)
        Au = A.apply(u)
        b = synth.to_f32_exact(Au + w.noise * Au.max() * eta)
    else:
        A = O.blur(w.H, w.W, synth.gaussian_blur_kernel(w.blur_size, w.blur_sigma))
        b = synth.to_f32_exact(A.apply(u) + w.noise * eta)
    phi = d["phi_star"]
    assert phi < O.objective(A, b, np.zeros((w.H, w.W)), w.alpha)
    tail = [v for _, v in d["trajectory"]]
    assert tail[-1] == phi and all(a >= b_ for a, b_ in zip(tail, tail[1:]))
    assert d["last_chunk_rel_change"] < 1e-6


@pytest.mark.parametrize("name", ["ct512", "deblur512"])
def test_second_method_agrees_and_bracket_holds(name):
    d = load(name)
    if "cross_check" not in d:
        pytest.skip("cross-check not generated")
    cc = d["cross_check"]
    phi = d["phi_star"]
    assert cc["last_chunk_rel_change"] <= 1e-10
    assert abs(cc["phi_star"] - phi) <= 1e-7 * phi
    assert cc["rel_diff_to_first_method"] == pytest.approx(abs(cc["phi_star"] - phi) / cc["phi_star"])
    cert = cc["certificate"]
    # the bracket's upper end is the objective at the second method's end point
    assert cert["upper"] == pytest.approx(cc["phi_star"], rel=1e-12)
    # both stored minima are objective values at feasible points, so the
    # smaller is the better upper bound; the bracket's lower end is below it
    assert cert["lower"] <= min(phi, cc["phi_star"])


@pytest.mark.slow
def test_certificate_brackets_and_detects_a_perturbation():
    from make_phi_star import certificate
    N, na, nd = 24, 20, 35
    ang = synth.parallel_beam_angles(na)
    A = O.joseph(N, N, ang, nd, 2.0 / N, 2.0 / N)
    u, eta = synth.phantom_and_noise(N, N, 6, 5, (na, nd))
    Au = A.apply(u)
    b = synth.to_f32_exact(Au + 0.01 * Au.max() * eta)
    alpha = 0.05
    L = A.norm(300)
    r = O.pdhg(A, b, alpha, 1 / L, 1 / L, 4000, 200, nonneg=1)
    x, y, q = r["x"], r["y"], r["q"]
    r2 = O.pdhg_explicit(A, b, alpha, 1, 20000, x=x.copy(), y1=y.copy(),
                         y2=O.proj_ball(q * L, alpha))
    c = certificate(A, b, alpha, r2["x"], r2["y2"])
    phi_long = O.objective(A, b, x, alpha)
    assert c["lower"] <= phi_long + 1e-12 and c["lower"] <= c["upper"]
    assert c["upper"] - c["lower"] <= 1e-7 * c["upper"]
    # a perturbed point: the bracket's upper end rises by the excess, the
    # lower end stays below the minimum
    xp = np.maximum(r2["x"] + 0.01 * np.random.default_rng(0).standard_normal(x.shape), 0)
    cp = certificate(A, b, alpha, xp, r2["y2"])
    assert cp["lower"] <= phi_long + 1e-12
    assert cp["upper"] - cp["lower"] >= O.objective(A, b, xp, alpha) - phi_long - 1e-9
