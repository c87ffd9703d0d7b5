#!/usr/bin/env python3
"""Writes the oracle's long full-size runs that the GPU parity tests compare
against, from the CPU oracle only (calls oracle/ and synth/, nothing else):

- parity_ct512_pdhgskip.npz: the 512x512 CT workload (Joseph, 180 angles,
  725 bins, alpha 0.05, u >= 0), PDHGSkip-2 at p = 0.1 with 50 FGP
  iterations per prox, sigma = tau = 1/|A| (|A| from 50 oracle power
  iterations, stored), float64, 3000 outer iterations: the iterate x (stored
  as float32) after 1000 and 3000 iterations, the objective after every
  iteration and the coin trace.
- parity_ct512_pdhgskip_inner.npz: the same CT problem and steps, PDHGSkip-2
  at p = 0.3 with the TV prox solved by 50 steps of ProxSkip on its dual
  (projection probability 0.3, the skipping inner solver), 1000 outer
  iterations: x (float32) after 500 and 1000 iterations, the objective and
  coin traces and the number of inner projections.
- parity_deblur512_proxskip.npz: the 512x512 deblurring workload (periodic
  9x9 Gaussian blur, alpha 0.02), ProxSkip at p = 0.1, step 1, 50 FGP
  iterations, 2000 outer iterations: x after 1000 and 2000 iterations, the
  objective trace and the coin trace.

Inputs are the workloads' seeded phantoms and noise, b rounded to float32 as
the GPU runs see it.

  OMP_NUM_THREADS=8 python tests/golden/make_parity_runs.py [--workload ct512|ct512_inner|deblur512]
"""
import argparse
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle as O  # noqa: E402
import synth  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def ct512():
    w = synth.WORKLOADS["ct512"]
    ang = synth.parallel_beam_angles(w.n_ang)
    A = O.joseph(w.H, w.W, ang, w.n_det, w.pixel, w.det_spacing)
    u, eta = synth.make_inputs(w)
    Au = A.apply(u)
    b = synth.to_f32_exact(Au + w.noise * Au.max() * eta)
    L = A.norm(50)
    seed = synth.coin_seed(w.index)
    x = np.zeros((w.H, w.W))
    h = np.zeros((w.H, w.W))
    q = np.zeros((2, w.H, w.W))
    y = np.zeros((w.n_ang, w.n_det))
    out = {"sigma": 1 / L, "tau": 1 / L, "p": w.p, "seed": seed, "inner_iters": w.inner_iters}
    objs, thetas = [], []
    t0 = time.time()
    for k0, K in ((0, 1000), (1000, 2000)):
        r = O.pdhgskip(A, b, w.alpha, 1 / L, 1 / L, w.p, K, w.inner_iters, nonneg=1, seed=seed,
                       k0=k0, x=x, h=h, y=y, q=q, want_obj=True)
        x, h, y, q = r["x"], r["h"], r["y"], r["q"]
        objs.append(r["obj"])
        thetas.append(r["theta"])
        out[f"x_{k0 + K}"] = x.astype(np.float32)
        print(f"ct512: {k0 + K} iterations, {time.time() - t0:.0f} s", flush=True)
    out["obj"] = np.concatenate(objs)
    out["theta"] = np.concatenate(thetas)
    return out


def ct512_inner():
    w = synth.WORKLOADS["ct512"]
    ang = synth.parallel_beam_angles(w.n_ang)
    A = O.joseph(w.H, w.W, ang, w.n_det, w.pixel, w.det_spacing)
    u, eta = synth.make_inputs(w)
    Au = A.apply(u)
    b = synth.to_f32_exact(Au + w.noise * Au.max() * eta)
    L = A.norm(50)
    seed = synth.coin_seed(w.index)
    p, p_in = 0.3, 0.3
    x = np.zeros((w.H, w.W))
    h = np.zeros((w.H, w.W))
    q = np.zeros((2, w.H, w.W))
    h_in = np.zeros((2, w.H, w.W))
    y = np.zeros((w.n_ang, w.n_det))
    out = {"sigma": 1 / L, "tau": 1 / L, "p": p, "p_in": p_in, "seed": seed,
           "inner_iters": w.inner_iters}
    objs, thetas, nproj = [], [], 0
    t0 = time.time()
    for k0, K in ((0, 500), (500, 500)):
        r = O.pdhgskip_inner(A, b, w.alpha, 1 / L, 1 / L, p, K, w.inner_iters, p_in, nonneg=1,
                             seed=seed, k0=k0, x=x, h=h, y=y, q=q, h_in=h_in, want_obj=True)
        x, h, y, q, h_in = r["x"], r["h"], r["y"], r["q"], r["h_in"]
        objs.append(r["obj"])
        thetas.append(r["theta"])
        nproj += r["nproj"]
        out[f"x_{k0 + K}"] = x.astype(np.float32)
        print(f"ct512 inner skip: {k0 + K} iterations, {time.time() - t0:.0f} s", flush=True)
    out["obj"] = np.concatenate(objs)
    out["theta"] = np.concatenate(thetas)
    out["n_inner_proj"] = nproj
    return out


def deblur512():
    w = synth.WORKLOADS["deblur512"]
    A = O.blur(w.H, w.W, synth.gaussian_blur_kernel(w.blur_size, w.blur_sigma))
    u, eta = synth.make_inputs(w)
    b = synth.to_f32_exact(A.apply(u) + w.noise * eta)
    seed = synth.coin_seed(w.index)
    x = np.zeros((w.H, w.W))
    h = np.zeros((w.H, w.W))
    q = np.zeros((2, w.H, w.W))
    out = {"step": 1.0, "p": w.p, "seed": seed, "inner_iters": w.inner_iters}
    objs, thetas = [], []
    t0 = time.time()
    for k0, K in ((0, 1000), (1000, 1000)):
        r = O.proxskip(A, b, w.alpha, 1.0, w.p, K, w.inner_iters, seed=seed, k0=k0, x=x, h=h,
                       q=q, want_obj=True)
        x, h, q = r["x"], r["h"], r["q"]
        objs.append(r["obj"])
        thetas.append(r["theta"])
        out[f"x_{k0 + K}"] = x.astype(np.float32)
        print(f"deblur512: {k0 + K} iterations, {time.time() - t0:.0f} s", flush=True)
    out["obj"] = np.concatenate(objs)
    out["theta"] = np.concatenate(thetas)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="ct512", choices=["ct512", "ct512_inner", "deblur512"])
    ap.add_argument("--out", default=None)
    a = ap.parse_args()
    run, name = {"ct512": (ct512, "parity_ct512_pdhgskip"),
                 "ct512_inner": (ct512_inner, "parity_ct512_pdhgskip_inner"),
                 "deblur512": (deblur512, "parity_deblur512_proxskip")}[a.workload]
    out = run()
    path = a.out or os.path.join(HERE, f"{name}.npz")
    np.savez_compressed(path, **out)
    print("wrote", path, flush=True)


if __name__ == "__main__":
    main()
