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

  OMP_NUM_THREADS=6 python tests/golden/make_phi_star.py [--workload ct512]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

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
    return {
        "phi_star": traj[-1][1],
        "workload": "deblur512",
        "method": f"oracle PGD (ProxSkip at p=1), step 1, FGP {a.inner} inner iterations, "
                  "float64",
        "iterations": done,
        "last_chunk_rel_change": abs(traj[-2][1] - traj[-1][1]) / traj[-1][1] if len(traj) > 1 else None,
        "trajectory": traj[-12:],
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
    a = ap.parse_args()
    out_path = a.out or os.path.join(HERE, f"phi_star_{a.workload}.json")
    if a.workload != "ct512":
        out = denoise128(a) if a.workload == "denoise128" else deblur512(a)
        out["generated_by"] = (f"tests/golden/make_phi_star.py --workload {a.workload} "
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
    json.dump(out, open(out_path, "w"), indent=1)
    print("wrote", out_path, flush=True)


if __name__ == "__main__":
    main()
