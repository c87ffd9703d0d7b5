#!/usr/bin/env python3
"""Writes the reference minima Phi* of the time-to-accuracy workloads, from
the CPU oracle only:

- phi_star_ct512.json: the 512x512 CT workload (min 1/2|Au - b|^2 + 0.05
  TV(u), u >= 0).  Inputs: the workload's seeded phantom and noise (synth),
  b = A u + 0.01 max(Au) eta with the oracle's Joseph A in float64, rounded to
  float32 (the values the GPU run sees).  Method: PDHG (PDHGSkip-2 at p = 1,
  which the paper states recovers PDHG) with a warm-started FGP prox of 100
  iterations, sigma = tau = 1/|A|, run in chunks until the objective changes
  by less than `tol` (relative) over the last chunk; Phi* is the last value.
- phi_star_denoise128.json: the 128x128 float64 denoising workload (A = I,
  min 1/2|u - b|^2 + 0.1 TV(u), b = u + 0.05 eta).  Phi is then the TV prox
  objective of b with lambda = alpha, so FGP on it, run until the relative
  duality gap is below 1e-12 (or 400000 iterations), gives Phi* with a
  certificate: Phi* lies in [P - gap, P].
- phi_star_deblur512.json: the 512x512 deblurring workload (periodic 9x9
  Gaussian blur, sigma 2, b = A u + 0.01 eta rounded to float32, alpha
  0.02).  Method: PGD (ProxSkip at p = 1), step 1 = 1/|A|^2, warm-started
  FGP prox of 100 iterations, in chunks until the objective changes by less
  than `tol` over the last chunk.

The trajectory tail is stored so a reader can judge the convergence.

Cross-check (--cross-check, ct512 and deblur512): a second float64 method and
a duality certificate, both stored under "cross_check":

- the oracle's explicit diagonally preconditioned PDHG on K = [A; D] with
  closed-form proxes (the reference method of the paper's CT section), no
  inner solver, started from the first method's end point and its duals
  (y1 = the data dual, y2 = the prox dual divided by the prox step: the
  saddle point of the first method's fixed point), run in chunks of 1000
  iterations until Phi changes by less than 1e-10 relative over a chunk;
- a certificate of the unconstrained problem min 1/2|Au - b|^2 + alpha TV(u)
  (a lower bound of the u >= 0 problem too): y1 = A x - b shifted so that
  A^T y1 sums to zero (the range of div), y2 = the explicit method's dual
  plus D phi with div D phi = A^T y1 - div y2 solved exactly by the DCT-II
  (which diagonalises the Neumann Laplacian D^T D), then both scaled by
  s = min(1, alpha / max|y2_i|) so that |y2_i| <= alpha.  Weak duality:
  Phi* >= -s^2 |y1|^2 / 2 - s <y1, b> + <r, u*>, r the rounding residual of
  A^T y1 - div y2 (bounded by |r| |x| (1 + 1e-3)); Phi* <= Phi(x) for the
  feasible end point x.

  OMP_NUM_THREADS=6 python tests/golden/make_phi_star.py [--workload ct512] [--cross-check]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402
import scipy.fft  # noqa: E402

import oracle as O  # noqa: E402
import synth  # noqa: E402


HERE = os.path.dirname(os.path.abspath(__file__))


def denoise128(a):
    w = synth.WORKLOADS["denoise128"]
    u, eta = synth.make_inputs(w)
    b = u + w.noise * eta  # a float64 workload: no rounding
    q = np.zeros((2, w.H, w.W))
    traj = []
    done = 0
    t0 = time.time()
    while done < a.max_fgp:
        _, q = O.fgp(b, w.alpha, a.fgp_chunk, 0, q)
        done += a.fgp_chunk
        gap, primal = O.tv_gap(b, w.alpha, q)
        traj.append((done, primal, gap))
        print(f"{done} FGP iterations, {time.time() - t0:.0f} s: P = {primal:.15e}, "
              f"gap = {gap:.3e}", flush=True)
        if gap <= 1e-12 * primal:
            break
    return {
        "phi_star": traj[-1][1],
        "workload": "denoise128",
        "method": "oracle FGP on the prox problem of b with lambda = alpha (Phi is that "
                  "problem's primal objective), float64, until relative gap <= 1e-12 or "
                  f"{a.max_fgp} iterations",
        "fgp_iterations": done,
        "gap": traj[-1][2],
        "certificate": [traj[-1][1] - traj[-1][2], traj[-1][1]],
        "trajectory": traj[-8:],
    }


def deblur512(a):
    w = synth.WORKLOADS["deblur512"]
    A = O.blur(w.H, w.W, synth.gaussian_blur_kernel(w.blur_size, w.blur_sigma))
    u, eta = synth.make_inputs(w)
    b = synth.to_f32_exact(A.apply(u) + w.noise * eta)
    x = np.zeros((w.H, w.W))
    q = np.zeros((2, w.H, w.W))
    traj = []
    done = 0
    t0 = time.time()
    while done < a.max:
        r = O.pgd(A, b, w.alpha, 1.0, a.chunk, a.inner, x=x, q=q)
        x, q = r["x"], r["q"]
        done += a.chunk
        phi = O.objective(A, b, x, w.alpha)
        traj.append((done, phi))
        print(f"{done} iterations, {time.time() - t0:.0f} s: Phi = {phi:.12e}", flush=True)
        if len(traj) >= 2 and abs(traj[-2][1] - phi) <= a.tol * phi:
            break
    out = {
        "phi_star": traj[-1][1],
        "workload": "deblur512",
        "method": f"oracle PGD (ProxSkip at p=1), step 1, FGP {a.inner} inner iterations, "
                  "float64",
        "iterations": done,
        "last_chunk_rel_change": abs(traj[-2][1] - traj[-1][1]) / traj[-1][1] if len(traj) > 1 else None,
        "trajectory": traj[-12:],
    }
    if a.cross_check:
        # PGD's fixed point: x = prox(x - A^T(Ax - b)) = x - A^T(Ax - b) + div q,
        # so y1 = Ax - b, y2 = q / step (step 1) is its saddle point
        out["certificate_first_method"] = certificate(A, b, w.alpha, x, O.proj_ball(q, w.alpha))
        cross_check(out, A, b, w.alpha, 0, x, A.apply(x) - b, q, a, "deblur512")
    return out


def neumann_poisson(e):
    """phi with D^T D phi = e (e of zero sum; the zero mode of phi is 0):
    the DCT-II diagonalises D^T D with eigenvalues 4 sin^2(pi k / 2H) +
    4 sin^2(pi l / 2W)."""
    H, W = e.shape
    k = np.arange(H)[:, None]
    l_ = np.arange(W)[None, :]
    lam = 4 * np.sin(np.pi * k / (2 * H)) ** 2 + 4 * np.sin(np.pi * l_ / (2 * W)) ** 2
    ehat = scipy.fft.dctn(e, type=2, norm="ortho")
    lam[0, 0] = 1.0
    ph = ehat / lam
    ph[0, 0] = 0.0
    return scipy.fft.idctn(ph, type=2, norm="ortho")


def certificate(A, b, alpha, x, y2):
    """[lower, upper] bracket of the minimum of 1/2|Au - b|^2 + alpha TV(u)
    (u >= 0 or not) from a feasible point x (>= 0 where the problem asks it)
    and a dual estimate y2 of the TV term (|y2_i| <= alpha)."""
    y1 = A.apply(x) - b
    w = A.apply(np.ones_like(x))
    y1 = y1 - (np.vdot(y1, w) / np.vdot(w, w)) * w     # sum of A^T y1 = <y1, A 1> = 0
    g = A.adjoint(y1)
    e = g - O.div(y2)
    e = e - e.mean()                                   # rounding only: both sides sum to 0
    phi = neumann_poisson(-e)                          # div D phi = -D^T D phi = e
    y2c = y2 + O.grad(phi)
    nrm = np.sqrt(y2c[0] ** 2 + y2c[1] ** 2).max()
    s = min(1.0, alpha / nrm)
    y1s, y2s = s * y1, s * y2c
    r = A.adjoint(y1s) - O.div(y2s)
    dual = -0.5 * np.vdot(y1s, y1s) - np.vdot(y1s, b)
    slack = np.linalg.norm(r) * np.linalg.norm(x) * (1 + 1e-3)
    upper = O.objective(A, b, x, alpha)
    return {"lower": float(dual - slack), "upper": float(upper), "scale": float(s),
            "residual_norm": float(np.linalg.norm(r)), "dual_value": float(dual)}


def explicit_cross_check(A, b, alpha, nonneg, x, y1, y2, max_iters, label):
    """Explicit preconditioned PDHG from (x, y1, y2) in chunks of 1000
    iterations until Phi changes by less than 1e-10 relative over a chunk."""
    traj = [(0, O.objective(A, b, x, alpha))]
    done = 0
    t0 = time.time()
    while done < max_iters:
        r = O.pdhg_explicit(A, b, alpha, nonneg, 1000, x=x, y1=y1, y2=y2)
        x, y1, y2 = r["x"], r["y1"], r["y2"]
        done += 1000
        traj.append((done, O.objective(A, b, x, alpha)))
        print(f"{label}: explicit PDHG {done} iterations, {time.time() - t0:.0f} s: "
              f"Phi = {traj[-1][1]:.12e}", flush=True)
        if abs(traj[-2][1] - traj[-1][1]) <= 1e-10 * traj[-1][1]:
            break
    return x, y1, y2, traj


def cross_check(out, A, b, alpha, nonneg, x, y1, y2, a, label):
    x2, y1e, y2e, traj = explicit_cross_check(A, b, alpha, nonneg, x.copy(), y1.copy(),
                                              O.proj_ball(y2, alpha), a.max_explicit, label)
    cert = certificate(A, b, alpha, x2, y2e)
    phi1, phi2 = out["phi_star"], traj[-1][1]
    print(f"{label}: Phi1 = {phi1:.12e}, explicit Phi2 = {phi2:.12e} "
          f"(rel {abs(phi1 - phi2) / phi2:.2e}); certificate [{cert['lower']:.12e}, "
          f"{cert['upper']:.12e}] (width {(cert['upper'] - cert['lower']) / phi2:.2e} rel, "
          f"scale {cert['scale']:.12f})", flush=True)
    out["cross_check"] = {
        "method": "oracle explicit diagonally preconditioned PDHG on K = [A; D] "
                  "(closed-form proxes, no inner solver), float64, started from the "
                  "first method's end point and duals, chunks of 1000 iterations until "
                  "Phi changes by less than 1e-10 relative over a chunk",
        "phi_star": phi2,
        "iterations": traj[-1][0],
        "last_chunk_rel_change": abs(traj[-2][1] - traj[-1][1]) / traj[-1][1],
        "rel_diff_to_first_method": abs(phi1 - phi2) / phi2,
        "min_x": float(x2.min()),
        "trajectory": traj[-12:],
        "certificate": cert,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="ct512", choices=["ct512", "denoise128", "deblur512"])
    ap.add_argument("--chunk", type=int, default=250)
    ap.add_argument("--max", type=int, default=8000)
    ap.add_argument("--inner", type=int, default=100)
    ap.add_argument("--tol", type=float, default=2e-9)
    ap.add_argument("--fgp-chunk", type=int, default=2000)
    ap.add_argument("--max-fgp", type=int, default=400000)
    ap.add_argument("--out", default=None)
    ap.add_argument("--cross-check", action="store_true")
    ap.add_argument("--max-explicit", type=int, default=40000)
    a = ap.parse_args()
    out_path = a.out or os.path.join(HERE, f"phi_star_{a.workload}.json")
    if a.workload != "ct512":
        out = denoise128(a) if a.workload == "denoise128" else deblur512(a)
        flag = " --cross-check" if a.cross_check else ""
        out["generated_by"] = (f"tests/golden/make_phi_star.py --workload {a.workload}{flag} "
                               "(calls only oracle/ and synth/)")
        json.dump(out, open(out_path, "w"), indent=1)
        print("wrote", out_path, flush=True)
        return
    w = synth.WORKLOADS["ct512"]
    ang = synth.parallel_beam_angles(w.n_ang)
    A = O.joseph(w.H, w.W, ang, w.n_det, w.pixel, w.det_spacing)
    u, eta = synth.make_inputs(w)
    Au = A.apply(u)
    b = synth.to_f32_exact(Au + w.noise * Au.max() * eta)
    L = A.norm(50)
    x = np.zeros((w.H, w.W))
    y = np.zeros((w.n_ang, w.n_det))
    q = np.zeros((2, w.H, w.W))
    traj = []
    done = 0
    t0 = time.time()
    while done < a.max:
        r = O.pdhg(A, b, w.alpha, 1 / L, 1 / L, a.chunk, a.inner, nonneg=1, x=x, y=y, q=q)
        x, y, q = r["x"], r["y"], r["q"]
        done += a.chunk
        phi = O.objective(A, b, x, w.alpha)
        traj.append((done, phi))
        print(f"{done} iterations, {time.time() - t0:.0f} s: Phi = {phi:.12e}", flush=True)
        if len(traj) >= 2 and abs(traj[-2][1] - phi) <= a.tol * phi:
            break
    out = {
        "phi_star": traj[-1][1],
        "workload": "ct512",
        "method": f"oracle PDHG (PDHGSkip-2 at p=1), FGP {a.inner} inner iterations, "
                  f"sigma = tau = 1/|A| (|A| = {L:.12f}), float64",
        "iterations": done,
        "last_chunk_rel_change": abs(traj[-2][1] - traj[-1][1]) / traj[-1][1] if len(traj) > 1 else None,
        "min_x": float(x.min()),
        "trajectory": traj[-12:],
        "generated_by": "tests/golden/make_phi_star.py (calls only oracle/ and synth/)",
    }
    if a.cross_check:
        # PDHG's fixed point: div q = sigma A^T y, so y2 = q / sigma = L q
        y2 = O.proj_ball(q * L, w.alpha)
        out["certificate_first_method"] = certificate(A, b, w.alpha, x, y2)
        cross_check(out, A, b, w.alpha, 1, x, y, y2, a, "ct512")
        out["generated_by"] = ("tests/golden/make_phi_star.py --cross-check "
                               "(calls only oracle/ and synth/)")
    json.dump(out, open(out_path, "w"), indent=1)
    print("wrote", out_path, flush=True)


if __name__ == "__main__":
    main()
