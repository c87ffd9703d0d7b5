#!/usr/bin/env python3
"""Writes phi_star_ct512.json: the reference minimum Phi* of the 512x512 CT
workload (min 1/2|Au - b|^2 + 0.05 TV(u), u >= 0), from the CPU oracle only.

Inputs: the workload's seeded phantom and noise (synth), b = A u + 0.01
max(Au) eta with the oracle's Joseph A in float64, rounded to float32 (the
values the GPU run sees).  Method: PDHG (PDHGSkip-2 at p = 1, which the paper
states recovers PDHG) with a warm-started FGP prox of 100 iterations, sigma =
tau = 1/|A|, run in chunks until the objective changes by less than `tol`
(relative) over the last chunk; Phi* is the last value.  The trajectory
tail is stored so a reader can judge the convergence.

  OMP_NUM_THREADS=6 python tests/golden/make_phi_star.py [--chunk 250] [--max 8000]
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--chunk", type=int, default=250)
    ap.add_argument("--max", type=int, default=8000)
    ap.add_argument("--inner", type=int, default=100)
    ap.add_argument("--tol", type=float, default=2e-9)
    ap.add_argument("--out", default=os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                                  "phi_star_ct512.json"))
    a = ap.parse_args()
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
    json.dump(out, open(a.out, "w"), indent=1)
    print("wrote", a.out, flush=True)


if __name__ == "__main__":
    main()
