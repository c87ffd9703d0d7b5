"""Checks of the stored reference minima Phi* (tests/golden/phi_star_*.json,
written by tests/golden/make_phi_star.py from the CPU oracle only).

- denoise128: Phi is the TV prox objective of b (lambda = alpha), so weak
  duality brackets the true minimum with any dual point: a short FGP run
  from zero gives D(q) = P(z_q) - gap(q) <= Phi* <= P(z_q).  The stored value
  must sit in that bracket, and its own certificate must be tight.
- ct512 / deblur512: Phi* is a minimum, so it cannot exceed the objective at
  the zero image; the stored trajectory must be non-increasing at its end
  and its last chunk must have changed by less than the stopping tolerance.
"""
import json
import os

import numpy as np
import pytest

import oracle as O
import synth

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


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
