#!/usr/bin/env python3
"""Benchmark: PDHGSkip-2 on the 512x512 parallel-beam CT workload (MI355X).

Workload (synthetic stand-in for the paper's catalyst CT slice): a 512x512
float32 ellipse phantom (30 seeded ellipses), 180 angles over [0, pi), 725
detector bins, Joseph projector with its exact-transpose backprojector,
Gaussian noise of 1 % of the sinogram maximum; min 1/2|Au - b|^2 + 0.05 TV(u)
with u >= 0, PDHGSkip-2 with p = 0.1, sigma = tau = 1/|A|, 50 FGP iterations
per prox, 3000 outer iterations, seeded coin.

One step = one full solve (3000 outer iterations from a zero state) with all
inputs resident in HBM.  value = outer iterations per second over the timed
steps.  Also reported: time to 1e-4 relative objective for PDHGSkip-2 (p =
0.1) and PDHG (p = 1), the dominant kernel's roofline, the FGP kernel's HBM
rate on a large image, and the CPU oracle timed on this host.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0          # MI355X HBM3E, GB/s
PEAK_FP32_TFLOPS = 157.3       # MI355X vector fp32
PEAK_BF16_TFLOPS = 2500.0      # MI355X dense bf16 MFMA
CNN_FLOP_PER_PX = 2 * 9 * (2 * 32 + 32 * 32 + 32 * 32 + 32 * 2)  # 3x3 convs 2-32-32-32-2


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-tta", action="store_true", help="skip time-to-accuracy runs")
    ap.add_argument("--fgp-size", type=int, default=8192)
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-form comparison")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-prox training and runs")
    ap.add_argument("--no-light", action="store_true", help="skip the Dual-ROF / Huber runs")
    ap.add_argument("--batched-only", action="store_true",
                    help="only the batched-form run (one warm and one timed batched solve, no "
                         "per-slice comparison): the program to profile for the batched FGP "
                         "kernels; prints a batched record, not the benchmark line")
    ap.add_argument("--batched-outer", type=int, default=500,
                    help="with --batched-only: outer iterations of the batched solve")
    ap.add_argument("--tune-save", default=None,
                    help="with --batched-only: write the run's FGP tuning table to this file")
    ap.add_argument("--tune-load", default=None,
                    help="with --batched-only: take the FGP tuning table from this file (no "
                         "tuning sweeps in the run)")
    ap.add_argument("--kernels-only", action="store_true",
                    help="only the per-kernel launches (event times, FGP HBM rate, the copy that "
                         "calibrates byte counters): the short program to run under rocprofv3 "
                         "--pmc; prints a kernels record, not the benchmark line")
    return ap.parse_args()


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on exactly one GPU (asked for --gpus {args.gpus}, WORLD_SIZE "
              f"{world}); the library has no multi-GPU path.", flush=True)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2411_00688_amd as T
    import synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.init()
    if args.batched_only:
        res = batched_bench(T, K=args.batched_outer, plain=False, tune_load=args.tune_load,
                            tune_save=args.tune_save)
        print(json.dumps({"record": "batched", **res}), flush=True)
        return
    w = synth.WORKLOADS["ct512"]
    N, na, nd = w.H, w.n_ang, w.n_det
    ang = synth.parallel_beam_angles(na)
    K, Kin, p, alpha = w.outer_iters, w.inner_iters, w.p, w.alpha
    seed = synth.coin_seed(w.index)

    ctx = T.tvs_ctx_create(0)
    op = T.tvs_op_ct_joseph(ctx, N, N, ang, nd, w.pixel, w.det_spacing)

    # ---- inputs (untimed): b = A u + 0.01 max(Au) eta, rounded to float32
    u, eta = synth.make_inputs(w)
    Au = torch.empty(na, nd, dtype=torch.float64, device=dev)
    T.tvs_op_apply(op, torch.tensor(u, device=dev), Au)
    b = (Au + w.noise * Au.max() * torch.tensor(eta, device=dev)).float().contiguous()
    Lnorm = T.tvs_op_norm(op, 100, 1)
    sigma = tau = 1.0 / Lnorm
    best, _ = T.tvs_fgp_autotune(ctx, T.TVS_F32, N, N, Kin, 3)
    log(f"|A| = {Lnorm:.10f}; FGP tile variant {T.tvs_fgp_variant(best)}")

    if args.kernels_only:
        kern = kernel_times(T, ctx, op, N, na, nd, Kin, 0, K)
        fgp_big = fgp_hbm(T, ctx, args.fgp_size, Kin)
        cnn_fwd = cnn_forward_rate(T, ctx)
        print(json.dumps({"record": "kernels", "launch_ms": kern["launch_ms"],
                          "copy_calibration_bytes": COPY_CAL_BYTES, "tv_prox_hbm": fgp_big,
                          "cnn_forward": cnn_fwd}), flush=True)
        T.tvs_op_destroy(op)
        T.tvs_ctx_destroy(ctx)
        return

    x = torch.zeros(N, N, device=dev)
    h = torch.zeros_like(x)
    q = torch.zeros(2, N, N, device=dev)
    y = torch.zeros(na, nd, device=dev)

    def solve(pp=p, iters=K, obj=False, graph=True):
        for t in (x, h, q, y):
            t.zero_()
        return T.tvs_pdhgskip(op, b, x, h, q, y, alpha, sigma, tau, pp, iters, Kin, nonneg=1,
                              seed=seed, graph=graph and not obj, want_obj=obj, want_theta=obj)

    # ---- headline: full solves
    for _ in range(args.warmup):
        solve()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record()
    rep = None
    for _ in range(args.steps):
        rep = solve()
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = ev0.elapsed_time(ev1) / args.steps
    value = K / (ms_step / 1e3)
    log(f"{args.steps} solves: {ms_step:.2f} ms each ({wall:.3f} s wall), {value:.1f} outer it/s, "
        f"{rep['n_prox']} prox per solve")

    # ---- time to 1e-4 relative objective (deterministic replay for Phi)
    tta = small = spdhg = None
    if not args.no_tta:
        tta = time_to_accuracy(solve, w, K, extra=ct_comparisons(T, op, w, b, Lnorm, seed, K))
        spdhg = spdhg_tta(T, ctx, w, b, seed)
        small = small_tta(T, ctx)

    # ---- per-kernel timing with HIP events on the context's stream
    kern = kernel_times(T, ctx, op, N, na, nd, Kin, rep["n_prox"], K)
    # A standalone A call pads its input first; the solver does not (Aᵀ's
    # epilogue writes the padded copies), and its A kernel is shorter than
    # the backprojector pair, so the pair stands for the Joseph operators.
    ps_ms = kern["per_step_ms"]
    dom = "joseph_adj" if ps_ms["joseph_adj"] >= ps_ms["fgp_prox"] else "fgp_prox"
    roof = roofline(dom, kern, N, na, nd, Kin)

    # ---- FGP on a large image: true HBM rate of the TV-prox kernel; and at the
    # workload's own 512^2 (working set resident in the last-level cache), in
    # a context of its own so that the run's tuning table stays as it is
    fgp_big = fgp_hbm(T, ctx, args.fgp_size, Kin)
    ctx512 = T.tvs_ctx_create(0)
    fgp_512 = fgp_hbm(T, ctx512, N, Kin, resident=True)
    T.tvs_ctx_destroy(ctx512)

    # ---- batched form: 256 uneven denoising slices in one graph vs one solve per slice
    batched = None
    if not args.no_batched:
        batched = batched_bench(T)

    # ---- light-prox problems (Dual-ROF / Dual-Huber-ROF, 200 x 300)
    light = None
    if not args.no_light:
        light = light_prox_bench(T, ctx)

    # ---- learned prox: trained here on the method's own prox inputs
    learned_res = None
    if not args.no_learned:
        learned_res = learned_bench(T, ctx, op, w, b, sigma, tau, seed, tta)

    # ---- CPU oracle baseline on this host
    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(b.double().cpu().numpy(), w, ang, sigma, tau, seed)

    T.tvs_op_destroy(op)
    T.tvs_ctx_destroy(ctx)

    out = {
        "metric": "outer iterations/s, PDHGSkip-2 (p=0.1) on 512^2 CT; time to 1e-4 rel. objective; TV-prox HBM GB/s",
        "value": round(value, 2),
        "unit": "outer_iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "ct512: PDHGSkip-2, 512x512 Joseph CT, 180 angles, 725 bins, "
                               "alpha 0.05, p 0.1, 50 FGP iters, 3000 outer iters, u >= 0",
                   "outer_iters_per_step": K, "prox_per_step": rep["n_prox"],
                   "fgp_variant": list(T.tvs_fgp_variant(best)), "norm_A": Lnorm},
        "time_to_1e-4": tta,
        "time_to_1e-4_angle_subsets": spdhg,
        "time_to_1e-4_denoise_deblur": small,
        "kernels_ms_per_step": trace_per_step(K),
        "roofline": roof,
        "tv_prox_hbm": fgp_big,
        "tv_prox_512": fgp_512,
        "batched": batched,
        "learned": learned_res,
        "light_prox": light,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def tta_entry(run, K, phis, name):
    """Time to 1e-4 of one method: k* = first outer iteration after which
    |Phi(x_k) - Phi*| / Phi* stays <= 1e-4, Phi from an instrumented replay
    of the same deterministic run (run(iters, obj=True)); the time is the
    median HIP-event time of three un-instrumented graph runs of exactly k*
    iterations (run(iters))."""
    import numpy as np
    import torch
    r = run(K, obj=True)
    rel = np.abs(r["obj"] - phis) / phis
    bad = np.nonzero(rel > 1e-4)[0]
    kstar = int(bad[-1] + 2) if len(bad) else 1
    if kstar > K:
        return {"iters": None, "note": f"not reached in {K} iterations",
                "final_rel": float(rel[-1])}
    times = []
    for _ in range(3):
        run(kstar)  # capture / warm
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        run(kstar)
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    out = {"iters": kstar, "ms": round(float(np.median(times)), 3),
           "prox_calls": int(np.sum(r["theta"][:kstar])), "final_rel": float(rel[-1])}
    log(f"time to 1e-4 ({name}): {kstar} iterations, {out['ms']:.2f} ms")
    return out


def time_to_accuracy(solve, w, K, p_sweep=(0.1, 0.3, 0.5, 0.7), extra=None):
    """Time to 1e-4 on the CT workload: PDHGSkip-2 at the workload's p, the
    p sweep, and PDHG (p = 1)."""
    path = os.path.join(ROOT, "tests", "golden", "phi_star_ct512.json")
    if not os.path.exists(path):
        return {"note": "reference minimum Phi* not available"}
    phis = json.load(open(path))["phi_star"]
    res = {"phi_star": phis}
    for pp in sorted(set(p_sweep) | {w.p}) + [1.0]:
        name = "pdhg_p1" if pp == 1.0 else f"pdhgskip_p{pp}"
        res[name] = tta_entry(lambda iters, obj=False: solve(pp=pp, iters=iters, obj=obj), K,
                              phis, name)
    key = f"pdhgskip_p{w.p}"
    if res.get(key, {}).get("ms") and res.get("pdhg_p1", {}).get("ms"):
        res["speedup_pdhgskip_vs_pdhg"] = round(res["pdhg_p1"]["ms"] / res[key]["ms"], 3)
    if extra is not None:
        res.update(extra(phis))
    return res


def ct_comparisons(T, op, w, b, L, seed, K):
    """The paper's comparison methods on the CT workload: PDHGSkip-1 at p in
    {0.3, 0.7} (sigma = tau = 0.99 sqrt(p) / |A|, so that sigma tau (1 +
    omega) |A|^2 < 1) and FISTA (step 1 / |A|^2), 50 inner iterations; and
    PDHGSkip-2 with skipping inside the inner solver (the TV prox by ProxSkip
    on its dual, projection probability p_in = 0.3, K_in inner steps per
    call) at (p, K_in) in {(0.1, 100), (0.3, 50), (0.3, 100)}."""
    import math
    import numpy as np
    import torch
    dev = torch.device("cuda:0")
    N, na, nd = w.H, w.n_ang, w.n_det
    x = torch.zeros(N, N, device=dev)
    h = torch.zeros_like(x)
    q = torch.zeros(2, N, N, device=dev)
    hin = torch.zeros_like(q)
    y = torch.zeros(na, nd, device=dev)

    def entries(phis):
        out = {}
        for pp, kin in ((0.1, 100), (0.3, 50), (0.3, 100)):
            def run_in(iters, obj=False, pp=pp, kin=kin):
                for t in (x, h, q, y, hin):
                    t.zero_()
                return T.tvs_pdhgskip_ex(op, b, x, h, q, y, w.alpha, 1.0 / L, 1.0 / L, pp, iters,
                                         kin, nonneg=1, seed=seed, graph=not obj, want_obj=obj,
                                         want_theta=obj, inner_p=0.3, inner_h=hin)
            name = f"pdhgskip_p{pp}_inner_skip_k{kin}_p0.3"
            out[name] = tta_entry(run_in, K, phis, name)
        for pp in (0.3, 0.7):
            s = 0.99 * math.sqrt(pp) / L

            def run(iters, obj=False, pp=pp, s=s):
                for t in (x, q, y):
                    t.zero_()
                return T.tvs_pdhgskip1(op, b, x, q, y, w.alpha, s, s, pp, iters, w.inner_iters,
                                       nonneg=1, seed=seed, graph=not obj, want_obj=obj,
                                       want_theta=obj)
            out[f"pdhgskip1_p{pp}"] = tta_entry(run, K, phis, f"pdhgskip1_p{pp}")

        def run_f(iters, obj=False):
            for t in (x, q):
                t.zero_()
            r = T.tvs_fista(op, b, x, q, w.alpha, 1.0 / L ** 2, iters, w.inner_iters, nonneg=1,
                            graph=not obj, want_obj=obj)
            r["theta"] = np.ones(iters, dtype=np.uint8)
            return r
        out["fista"] = tta_entry(run_f, K, phis, "fista")
        return out
    return entries


def spdhg_tta(T, ctx, w, b, seed, K=6000, configs=((4, 0.1), (4, 0.3), (10, 0.1), (10, 0.3),
                                                      (10, 1.0))):
    """Time to 1e-4 on the CT workload with random angle subsets (SPDHG over
    n interleaved subsets with the skipped prox): per (n, p), step sizes
    sigma = 0.99 / (n max_j |A_j|), tau = 0.99 / max_j |A_j| (SPDHG's
    condition sigma tau |A_j|^2 < 1/n), norms of the subset operators by 100
    power iterations on the GPU."""
    import torch
    import synth
    path = os.path.join(ROOT, "tests", "golden", "phi_star_ct512.json")
    if not os.path.exists(path):
        return {"note": "reference minimum Phi* not available"}
    phis = json.load(open(path))["phi_star"]
    dev = torch.device("cuda:0")
    N, na, nd = w.H, w.n_ang, w.n_det
    ang = synth.parallel_beam_angles(na)
    op = T.tvs_op_ct_joseph(ctx, N, N, ang, nd, w.pixel, w.det_spacing)
    x = torch.zeros(N, N, device=dev)
    h = torch.zeros_like(x)
    q = torch.zeros(2, N, N, device=dev)
    y = torch.zeros(na, nd, device=dev)
    res = {"phi_star": phis, "outer_iters_budget": K}
    norms = {}
    for n, pp in configs:
        if n not in norms:
            m = 0.0
            for j in range(n):
                sop = T.tvs_op_ct_joseph(ctx, N, N, ang[j::n], nd, w.pixel, w.det_spacing)
                m = max(m, T.tvs_op_norm(sop, 100, 1))
                T.tvs_op_destroy(sop)
            norms[n] = m
        m = norms[n]
        sigma, tau = 0.99 / (n * m), 0.99 / m

        def run(iters, obj=False, n=n, pp=pp, sigma=sigma, tau=tau):
            for t in (x, h, q, y):
                t.zero_()
            return T.tvs_spdhgskip(op, b, x, h, q, y, n, w.alpha, sigma, tau, pp, iters,
                                   w.inner_iters, nonneg=1, seed=seed, graph=not obj,
                                   want_obj=obj, want_theta=obj)

        name = f"subsets{n}_p{pp}"
        res[name] = tta_entry(run, K, phis, name)
        res[name].update({"sigma": sigma, "tau": tau, "max_subset_norm": m})
    T.tvs_op_destroy(op)
    return res


def small_tta(T, ctx):
    """Time to 1e-4 relative objective on the denoising workload (128^2
    float64, A = I, alpha 0.1, ProxSkip p = 0.1 vs PGD, 500 outer x 100 FGP)
    and the deblurring workload (512^2 float32, periodic 9x9 Gaussian blur,
    alpha 0.02, ProxSkip p in {0.05, 0.1, 0.3} vs PGD, 2000 outer x 50 FGP),
    step 1, same protocol as time_to_accuracy (k* from an instrumented
    replay, HIP-event time of a graph run of k* iterations).  Phi* from
    tests/golden/phi_star_<workload>.json (CPU oracle)."""
    import numpy as np
    import torch
    import synth
    dev = torch.device("cuda:0")
    res = {}
    for name in ("denoise128", "deblur512"):
        path = os.path.join(ROOT, "tests", "golden", f"phi_star_{name}.json")
        if not os.path.exists(path):
            res[name] = {"note": "reference minimum Phi* not available"}
            continue
        phis = json.load(open(path))["phi_star"]
        w = synth.WORKLOADS[name]
        dt = torch.float64 if w.dtype == "f64" else torch.float32
        T.tvs_fgp_autotune(ctx, T.TVS_F64 if w.dtype == "f64" else T.TVS_F32, w.H, w.W,
                           w.inner_iters, 2)  # both methods run on the tuned variant
        u, eta = synth.make_inputs(w)
        if w.operator == "identity":
            op = T.tvs_op_identity(ctx, w.H, w.W)
            b = torch.tensor(u + w.noise * eta, dtype=torch.float64, device=dev).to(dt)
        else:
            op = T.tvs_op_blur_periodic(ctx, w.H, w.W,
                                        synth.gaussian_blur_kernel(w.blur_size, w.blur_sigma))
            Au = torch.empty(w.H, w.W, dtype=torch.float64, device=dev)
            T.tvs_op_apply(op, torch.tensor(u, device=dev), Au)
            b = (Au + w.noise * torch.tensor(eta, device=dev)).to(dt).contiguous()
        x = torch.zeros(w.H, w.W, dtype=dt, device=dev)
        h, q = torch.zeros_like(x), torch.zeros(2, w.H, w.W, dtype=dt, device=dev)
        K, Kin, seed = w.outer_iters, w.inner_iters, synth.coin_seed(w.index)

        def solve(pp, iters, obj=False):
            for t in (x, h, q):
                t.zero_()
            return T.tvs_proxskip(op, b, x, h, q, w.alpha, 1.0, pp, iters, Kin, nonneg=w.nonneg,
                                  seed=seed, graph=not obj, want_obj=obj, want_theta=obj)

        out = {"phi_star": phis, "dtype": w.dtype}
        for pp in tuple(w.p_sweep or (w.p,)) + (1.0,):
            key = "pgd_p1" if pp == 1.0 else f"proxskip_p{pp}"
            out[key] = tta_entry(lambda iters, obj=False: solve(pp, iters, obj), K, phis,
                                 f"{name} {key}")
        if name == "deblur512":
            # the paper's table of the deblurring comparison, on this workload:
            # ProxSkip (p = 0.5, 10 inner; p = 0.05, 100 inner), ISTA (10
            # inner) and FISTA (100 and 10 inner), to 1e-4, 3000 iterations
            def psk(pp, kin):
                def run(iters, obj=False):
                    for t in (x, h, q):
                        t.zero_()
                    return T.tvs_proxskip(op, b, x, h, q, w.alpha, 1.0, pp, iters, kin, seed=seed,
                                          graph=not obj, want_obj=obj, want_theta=obj)
                return run

            def fista(kin):
                def run(iters, obj=False):
                    for t in (x, q):
                        t.zero_()
                    r = T.tvs_fista(op, b, x, q, w.alpha, 1.0, iters, kin, graph=not obj,
                                    want_obj=obj)
                    r["theta"] = np.ones(iters, dtype=np.uint8)
                    return r
                return run

            table = {}
            for key, run in (("proxskip_p0.5_inner10", psk(0.5, 10)),
                             ("proxskip_p0.05_inner100", psk(0.05, 100)),
                             ("ista_inner10", psk(1.0, 10)),
                             ("fista_inner100", fista(100)), ("fista_inner10", fista(10))):
                table[key] = tta_entry(run, 3000, phis, f"deblur512 {key}")
            out["paper_table"] = table
        T.tvs_op_destroy(op)
        res[name] = out
        log(f"time to 1e-4 ({name}): {out}")
    return res


def _evtime(fn, reps):
    import torch
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def kernel_times(T, ctx, op, N, na, nd, Kin, n_prox, K):
    """Average launch duration of the hot kernels, timed with HIP events on
    the stream the library launches on (torch's current stream)."""
    import torch
    dev = torch.device("cuda:0")
    g = torch.Generator(device=dev).manual_seed(0)
    xi = torch.rand(N, N, device=dev, generator=g)
    yi = torch.rand(na, nd, device=dev, generator=g)
    xo = torch.empty(N, N, device=dev)
    yo = torch.empty(na, nd, device=dev)
    qq = torch.zeros(2, N, N, device=dev)
    bp = _evtime(lambda: T.tvs_op_adjoint(op, yi, xo), 50)        # one joseph_adj launch
    fp = _evtime(lambda: T.tvs_op_apply(op, xi, yo), 50)          # transpose + joseph_fwd
    prox = _evtime(lambda: T.tvs_tv_prox(ctx, xi, 0.05, Kin, 1, qq, xo), 20)
    # a plain device copy of known size (256 MiB each way): the reference that
    # scales rocprofv3's FETCH_SIZE / WRITE_SIZE counters to bytes
    cal_src = torch.zeros(COPY_CAL_BYTES // 4, device=dev)
    cal_dst = torch.empty_like(cal_src)
    cal_dst.copy_(cal_src)
    torch.cuda.synchronize()
    del cal_src, cal_dst
    per_step = {"joseph_adj": bp * K, "joseph_fwd": fp * K, "fgp_prox": prox * n_prox}
    log("kernel ms: " + ", ".join(f"{k} {v:.4f}" for k, v in
                                  (("joseph_adj", bp), ("joseph_fwd", fp), ("fgp_prox", prox))))
    return {"launch_ms": {"joseph_adj": bp, "joseph_fwd": fp, "fgp_prox": prox},
            "per_step_ms": per_step}


COPY_CAL_BYTES = 256 << 20
PMC_SUMMARY = os.path.join(ROOT, "profiles", "joseph_adj_ct512_pmc.md")
TRACE_SUMMARY = os.path.join(ROOT, "profiles", "ct512_bench_kernels.md")


def trace_per_step(K):
    """Milliseconds per 3000-iteration solve spent in each hot kernel, from
    the committed rocprofv3 kernel trace of the solve (average duration in
    the solve x launches per solve), or None when a kernel source changed
    since the trace was taken."""
    import hashlib
    import re
    try:
        text = open(TRACE_SUMMARY).read()
        rec = json.loads(re.search(r"```json\n(.*?)\n```", text, re.S).group(1))
        for src, want in rec["source_sha256"].items():
            if hashlib.sha256(open(os.path.join(ROOT, src), "rb").read()).hexdigest() != want:
                return None
    except (OSError, AttributeError, ValueError, KeyError):
        return None
    if rec.get("outer_iters") != K:
        return None
    return {k: round(v["avg_us"] * v["launches_per_solve"] / 1e3, 3)
            for k, v in rec["kernels"].items()}


def measured_traffic(kernel_source, hash_key="source_sha256"):
    """Bytes per launch from the committed rocprofv3 counter summary, or None
    when the kernel source changed since the counters were taken."""
    import hashlib
    import re
    try:
        text = open(PMC_SUMMARY).read()
        m = re.search(r"```json\n(.*?)\n```", text, re.S)
        rec = json.loads(m.group(1))
        src = open(os.path.join(ROOT, kernel_source), "rb").read()
    except (OSError, AttributeError, ValueError):
        return None
    if rec.get(hash_key) != hashlib.sha256(src).hexdigest():
        return None
    return rec


def joseph_nnz(N, na, nd):
    """Number of nonzero weights of the 512^2 Joseph matrix (two per sample
    inside the image), counted from the geometry on the host."""
    import numpy as np
    px = 2.0 / N
    ang = np.arange(na) * math.pi / na
    total = 0
    for a in ang:
        c, s = math.cos(a), math.sin(a)
        sb = (np.arange(nd) - (nd - 1) / 2) * px
        steps = (np.arange(N) - (N - 1) / 2) * px
        if abs(c) >= abs(s):
            u = (sb[:, None] - (-steps[None, :]) * s) / c / px + (N - 1) / 2
        else:
            u = (N - 1) / 2 - (sb[:, None] - steps[None, :] * c) / s / px
        fl = np.floor(u)
        total += int(np.sum((fl >= 0) & (fl < N)) + np.sum((fl + 1 >= 0) & (fl + 1 < N)))
    return total


def roofline(dom, kern, N, na, nd, Kin):
    ms = kern["launch_ms"][dom]
    if dom in ("joseph_adj", "joseph_fwd"):
        nnz = joseph_nnz(N, na, nd)
        flops = 2.0 * nnz                     # one multiply-add per matrix weight
        ach = flops / (ms * 1e-3) / 1e12
        rec = measured_traffic("paper_2411_00688_amd/csrc/kernels_ops.hip")
        key = "joseph_adj_bytes_per_launch" if dom == "joseph_adj" else "joseph_fwd_bytes_per_launch"
        traffic = rec.get(key) if rec else None
        return {"kernel": dom, "bound": "alu", "achieved": round(ach, 3),
                "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                "frac": round(ach / PEAK_FP32_TFLOPS, 5), "traffic": traffic,
                "launch_ms": round(ms, 5), "work": f"2 flop per weight, {nnz} weights"}
    # FGP prox call: Kin iterations of 28 B/px algorithmic traffic
    byts = 28.0 * N * N * Kin
    ach = byts / (ms * 1e-3) / 1e9
    return {"kernel": dom, "bound": "hbm", "achieved": round(ach, 1), "peak": PEAK_HBM_GBS,
            "unit": "GB/s", "frac": round(ach / PEAK_HBM_GBS, 4), "traffic": None,
            "launch_ms": round(ms, 5)}


def fgp_hbm(T, ctx, n, Kin, resident=False):
    """FGP at n x n float32 (working set far beyond the 256 MB last-level
    cache): a one-iteration-per-launch variant moves exactly the algorithmic
    28 B/px (read q_{k-1}, q_{k-2}, v; write q_k), so its GB/s is an HBM rate
    (the fastest such variant, tiles or row-walking strips, is reported next
    to torch's 1 GiB device copy on the same GPU); the tuned temporally
    blocked variant is reported as an effective rate.  resident: an image
    whose working set stays in the last-level cache (512^2: 7.3 MB), where
    every rate is an effective one (algorithmic bytes over time), not HBM
    traffic."""
    import torch
    dev = torch.device("cuda:0")
    g = torch.Generator(device=dev).manual_seed(1)
    v = torch.rand(n, n, device=dev, generator=g)
    q = torch.zeros(2, n, n, device=dev)
    z = torch.empty(n, n, device=dev)
    res = {"size": n}
    iters = 40  # a multiple of every depth in the variant table: every launch is a full one

    def rate(vi):
        T.tvs_fgp_set_variant(ctx, T.TVS_F32, n, n, vi)
        ms_all = _evtime(lambda: T.tvs_tv_prox(ctx, v, 0.05, iters, 0, q, z), 3)
        # the call ends with one finalize pass (z = v + div q); time it alone
        ms_fin = _evtime(lambda: T.tvs_tv_prox(ctx, v, 0.05, 0, 0, q, z), 3)
        ms = ms_all - ms_fin
        gbs = 28.0 * n * n * iters / (ms * 1e-3) / 1e9
        log(f"  FGP {n}^2 variant {T.tvs_fgp_variant(vi)}: {ms / iters:.4f} ms per iteration")
        return {"variant": list(T.tvs_fgp_variant(vi)), "ms_per_iter": round(ms / iters, 4),
                "GB/s": round(gbs, 1), "frac_of_hbm_peak": round(gbs / PEAK_HBM_GBS, 4)}

    ts1 = [rate(vi) for vi in range(T.tvs_fgp_variant_count()) if T.tvs_fgp_variant(vi)[2] == 1]
    res["one_iter_per_launch"] = max(ts1, key=lambda r: r["GB/s"])
    vi, _ = T.tvs_fgp_autotune(ctx, T.TVS_F32, n, n, iters, 1)
    res["tuned"] = rate(vi)
    if resident:
        for key in ("one_iter_per_launch", "tuned"):
            r = res[key]
            r["effective_GB/s"] = r.pop("GB/s")
            r["effective_frac_of_hbm_peak"] = r.pop("frac_of_hbm_peak")
        res["note"] = ("working set resident in the last-level cache: effective rates "
                       "(28 B/px per iteration over time), not HBM traffic")
        T.tvs_fgp_set_variant(ctx, T.TVS_F32, n, n, -1)
        log(f"FGP {n}^2 (cache-resident): {res}")
        return res
    # a plain device copy of 1 GiB: the rate this GPU reaches on pure streaming
    a = torch.empty(1 << 28, device=dev)
    b = torch.empty_like(a)
    t = _evtime(lambda: b.copy_(a), 10)
    copy_gbs = 2.0 * (1 << 30) / (t * 1e-3) / 1e9
    res["device_copy_GB/s"] = round(copy_gbs, 1)
    res["one_iter_per_launch"]["frac_of_device_copy"] = round(
        res["one_iter_per_launch"]["GB/s"] / copy_gbs, 4)
    del a, b
    # the tuned variant's rate counts algorithmic bytes per iteration: effective
    t = res["tuned"]
    t["effective_GB/s"] = t.pop("GB/s")
    t["effective_frac_of_hbm_peak"] = t.pop("frac_of_hbm_peak")
    # measured bytes per launch (rocprofv3 counters, while the kernel source is
    # unchanged) and the HBM rate they give at the launch's duration
    rec = measured_traffic("paper_2411_00688_amd/csrc/kernels_fgp.hip", "fgp_source_sha256")
    if rec and n == 8192:
        by = rec.get("fgp_8192_bytes_per_launch", {})
        for key in ("one_iter_per_launch", "tuned"):
            name = "x".join(str(x) for x in res[key]["variant"])
            if name in by:
                r = res[key]
                r["traffic_per_launch"] = by[name]
                launch_s = r["ms_per_iter"] * r["variant"][2] * 1e-3
                r["measured_hbm_GB/s"] = round(by[name] / launch_s / 1e9, 1)
    T.tvs_fgp_set_variant(ctx, T.TVS_F32, n, n, -1)
    del v, q, z
    torch.cuda.empty_cache()
    log(f"FGP {n}^2: {res}")
    return res


def cnn_forward_rate(T, ctx, N=512, reps=20):
    """The learned prox's network forward on one N x N image, both operand
    modes: time per call (HIP events) and the MFMA rate.  Useful work is
    CNN_FLOP_PER_PX per pixel; the two-part BF16 mode issues three MFMAs per
    product (hi*hi, hi*lo, lo*hi), so its issued rate is three times that."""
    import torch
    dev = torch.device("cuda:0")
    cnn = T.tvs_cnn_create(ctx, 7)
    v = torch.rand(N, N, device=dev, generator=torch.Generator(device=dev).manual_seed(2))
    qt = torch.empty(1, 2, N, N, device=dev)
    res = {"size": N, "flop_per_px": CNN_FLOP_PER_PX}
    for fast, name, mult in ((False, "bf16x3", 3), (True, "bf16x1", 1)):
        T.tvs_cnn_set_fast_forward(cnn, fast)
        ms = _evtime(lambda: T.tvs_cnn_forward(cnn, v, 0.43, 1, qt, None), reps)
        tf = CNN_FLOP_PER_PX * N * N / (ms * 1e-3) / 1e12
        res[name] = {"ms": round(ms, 4), "useful_TFLOP/s": round(tf, 1),
                     "mfma_issued_TFLOP/s": round(mult * tf, 1),
                     "frac_of_bf16_peak": round(mult * tf / PEAK_BF16_TFLOPS, 4)}
    T.tvs_cnn_destroy(cnn)
    return res


def light_prox_bench(T, ctx):
    """ProxSkip on the light-prox problems (Sec. 2.1-2.2) on a 200 x 300
    shapes-like phantom with noise 0.05, float64, the paper's protocol:
    Dual-ROF (alpha 0.5, step 1/8), p in {1 (ProjGD), 0.5, 0.3, 0.1, 0.01},
    50000 iterations each, the l2 error of u_K = b + div q_K against u*
    (ProjGD, 200000 iterations); Dual-Huber-ROF (alpha 0.55, eps 0.01, step
    1/(8 + eps/alpha), p 0.04767), 5000 iterations, the iteration at which the
    relative error first drops below 1e-6 (u* from 50000 ProjGD iterations)
    and the mean projection count over 30 coin streams."""
    import numpy as np
    import torch
    import synth
    dev = torch.device("cuda:0")
    H, W = 200, 300
    u, eta = synth.phantom_and_noise(H, W, 12, synth.phantom_seed(5), (H, W))
    b = torch.tensor(u + 0.05 * eta, dtype=torch.float64, device=dev)
    q = torch.zeros(2, H, W, dtype=torch.float64, device=dev)
    hh = torch.zeros_like(q)
    dq = torch.empty(H, W, dtype=torch.float64, device=dev)

    def reset():
        q.zero_()
        hh.zero_()

    def primal():
        T.tvs_div(ctx, q, dq)
        return b + dq

    def timed(fn):
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        r = fn()
        e1.record()
        torch.cuda.synchronize()
        return r, e0.elapsed_time(e1)

    res = {"image": [H, W], "dtype": "f64"}
    # Dual-ROF
    reset()
    T.tvs_dual_rof_proxskip(ctx, b, q, hh, 0.5, 0.0, 0.125, 1.0, 200000, graph=True)
    u_star = primal().clone()
    nrm = torch.linalg.norm(u_star).item()
    rof = {}
    for p in (1.0, 0.5, 0.3, 0.1, 0.01):
        K = 50000
        reset()
        T.tvs_dual_rof_proxskip(ctx, b, q, hh, 0.5, 0.0, 0.125, p, K, seed=17, graph=True)
        reset()
        r, ms = timed(lambda: T.tvs_dual_rof_proxskip(ctx, b, q, hh, 0.5, 0.0, 0.125, p, K,
                                                      seed=17, graph=True))
        err = torch.linalg.norm(primal() - u_star).item() / nrm
        rof[f"p={p}"] = {"iters": K, "prox_calls": r["n_prox"], "ms": round(ms, 3),
                         "us_per_iter": round(1e3 * ms / K, 4), "rel_l2_err": err}
        log(f"Dual-ROF p={p}: {rof[f'p={p}']}")
    res["dual_rof"] = {"alpha": 0.5, "step": 0.125, "u_star": "ProjGD, 200000 iterations",
                       "runs": rof}
    # Dual-Huber-ROF
    alpha, eps, p, K = 0.55, 0.01, 0.04767, 5000
    step = 1.0 / (8.0 + eps / alpha)
    reset()
    T.tvs_dual_rof_proxskip(ctx, b, q, hh, alpha, eps, step, 1.0, 50000, graph=True)
    u_star = primal().clone()
    nrm = torch.linalg.norm(u_star).item()
    reset()
    hit = None
    for k0 in range(0, K, 50):
        T.tvs_dual_rof_proxskip(ctx, b, q, hh, alpha, eps, step, p, 50, seed=19, k0=k0)
        if hit is None and torch.linalg.norm(primal() - u_star).item() / nrm < 1e-6:
            hit = k0 + 50
    reset()
    T.tvs_dual_rof_proxskip(ctx, b, q, hh, alpha, eps, step, p, K, seed=19, graph=True)
    reset()
    r, ms = timed(lambda: T.tvs_dual_rof_proxskip(ctx, b, q, hh, alpha, eps, step, p, K,
                                                  seed=19, graph=True))
    err = torch.linalg.norm(primal() - u_star).item() / nrm
    counts = []
    for sd in range(30):
        reset()
        counts.append(T.tvs_dual_rof_proxskip(ctx, b, q, hh, alpha, eps, step, p, K,
                                              seed=1000 + sd)["n_prox"])
    res["dual_huber_rof"] = {"alpha": alpha, "eps": eps, "step": step, "p": p, "iters": K,
                             "prox_calls": r["n_prox"], "mean_prox_calls_30_streams":
                             float(np.mean(counts)), "ms": round(ms, 3),
                             "iters_per_s": round(K / (ms * 1e-3), 1), "rel_l2_err": err,
                             "iters_to_1e-6": hit,
                             "ms_to_1e-6": round(ms * hit / K, 3) if hit else None}
    log(f"Dual-Huber-ROF: {res['dual_huber_rof']}")
    # the fused kernel against the HBM roofline: float32 Dual-Huber-ROF at
    # 8192^2, where the library fuses 6 steps per launch (32 x 32 tiles);
    # one launch reads b, q, h and writes q, h once (36 B/px), so its bytes
    # per launch are 36 N^2
    N2, K2, TS2 = 8192, 96, 6
    b2 = torch.rand(N2, N2, device=dev, generator=torch.Generator(device=dev).manual_seed(3))
    q2 = torch.zeros(2, N2, N2, device=dev)
    h2 = torch.zeros_like(q2)
    T.tvs_dual_rof_proxskip(ctx, b2, q2, h2, alpha, eps, step, p, K2, seed=23, graph=True)
    _, ms2 = timed(lambda: T.tvs_dual_rof_proxskip(ctx, b2, q2, h2, alpha, eps, step, p, K2,
                                                   seed=23, graph=True))
    launch_ms = ms2 / (K2 // TS2)
    gbs = 36.0 * N2 * N2 / (launch_ms * 1e-3) / 1e9
    res["kernel_roofline"] = {"image": [N2, N2], "dtype": "f32", "steps_per_launch": TS2,
                              "launch_ms": round(launch_ms, 4), "us_per_step": round(ms2 / K2 * 1e3, 2),
                              "bytes_per_launch": 36 * N2 * N2,
                              "GB/s": round(gbs, 1), "frac_of_hbm_peak": round(gbs / 8000.0, 4),
                              "step_equivalent_GB/s": round(TS2 * gbs, 1)}
    log(f"light-prox kernel 8192^2: {res['kernel_roofline']}")
    del b2, q2, h2
    return res


def learned_bench(T, ctx, op, w, b, sigma, tau, seed, tta, steps=6000, per_source=6700):
    """The learned prox at its training configuration: a 4-layer 3x3 CNN
    trained on about 20k 128^2 pairs from the three single-image workloads
    and used inside PDHGSkip-2 on the CT workload.
    Pairs: prox inputs recorded from runs on phantoms other than the timed
    run's (denoising 128^2: ProxSkip p 0.1, lam 1; deblurring 512^2: ProxSkip
    p 0.1 and 0.3, lam 0.2 and 0.067; CT 512^2: PDHGSkip-2 p 0.1, lam =
    alpha sigma / p, u >= 0), the 512^2 ones cut into 128^2 crops,
    per_source pairs drawn from each workload.  Targets: the prox of each
    crop to a relative duality gap <= 1e-4 (batched FGP with warm duals; a
    crop that does not get there in 6000 iterations is dropped).  Training:
    Adam on mini-batches of 32 crops of one workload, dual-target weight 0.1.
    Held out: the prox inputs of the timed CT run (512^2).  Reports (i) cold
    prox calls: duality gap after the method's 50 FGP iterations from the
    zero dual and from the network's dual, and the FGP iterations the
    network's start needs to match the zero start; (ii) PDHGSkip-2 with the
    gap-gated learned prox (gate 1e-3: the previous call's dual first, then
    the network's single-part BF16 forward, then FGP from the better of the
    two) to 1e-4: iterations from an instrumented run, the time of an
    un-instrumented one (HIP graph) of exactly that many, against the plain
    run."""
    import numpy as np
    import torch
    import synth
    from paper_2411_00688_amd import learned
    dev = torch.device("cuda:0")
    N, na, nd, Kin, p = w.H, w.n_ang, w.n_det, w.inner_iters, w.p
    lam = w.alpha * sigma / p
    rng = np.random.default_rng(11)
    t0 = time.perf_counter()
    groups, info = [], {}

    def take(V, lams, name, nonneg):
        Vc = learned.crops(V, 128)
        lc = np.repeat(np.asarray(lams, dtype=np.float64), Vc.shape[0] // V.shape[0])
        sel = np.sort(rng.choice(Vc.shape[0], min(per_source, Vc.shape[0]), replace=False))
        Vc = Vc[torch.as_tensor(sel, device=dev)].contiguous()
        lc = lc[sel]
        Z, Q, rel, its = learned.prox_targets(ctx, Vc, lc, nonneg=nonneg, tol=1e-4, chunk=250,
                                              max_iters=6000, log=log)
        ok = np.flatnonzero(rel <= 1e-4)
        okt = torch.as_tensor(ok, device=dev)
        groups.append((Vc[okt].contiguous(), Z[okt].contiguous(), Q[okt].contiguous(), lc[ok],
                       nonneg))
        info[name] = {"pairs": int(len(ok)), "drawn": int(len(sel)),
                      "lam": sorted({round(float(x), 4) for x in lc}),
                      "target_fgp_iters": its, "target_rel_gap_max": float(rel[ok].max())}
        log(f"learned prox pairs, {name}: {info[name]}")

    # denoising 128^2 (float32 runs of the workload's configuration)
    wd = synth.WORKLOADS["denoise128"]
    opd = T.tvs_op_identity(ctx, wd.H, wd.W)
    Vs, i = [], 1
    while sum(v.shape[0] for v in Vs) < per_source:
        u, eta = synth.make_inputs(wd, seed_index=i)
        bd = torch.tensor(u + wd.noise * eta, dtype=torch.float32, device=dev)
        Vs.append(learned.record_prox_inputs(opd, bd, wd.alpha, 1.0, wd.p, wd.outer_iters,
                                             wd.inner_iters, 80, seed=synth.coin_seed(wd.index, i),
                                             H=wd.H, W=wd.W))
        i += 1
    T.tvs_op_destroy(opd)
    V = torch.cat(Vs)
    take(V, [wd.alpha / wd.p] * V.shape[0], "denoise128", 0)
    del Vs, V
    # deblurring 512^2, p 0.1 and 0.3
    wb = synth.WORKLOADS["deblur512"]
    opb = T.tvs_op_blur_periodic(ctx, wb.H, wb.W, synth.gaussian_blur_kernel(wb.blur_size, wb.blur_sigma))
    Vs, ls = [], []
    for i, pp in ((1, 0.1), (2, 0.3)):
        u, eta = synth.make_inputs(wb, seed_index=i)
        Au = torch.empty(wb.H, wb.W, dtype=torch.float64, device=dev)
        T.tvs_op_apply(opb, torch.tensor(u, device=dev), Au)
        bb = (Au + wb.noise * torch.tensor(eta, device=dev)).float().contiguous()
        v = learned.record_prox_inputs(opb, bb, wb.alpha, 1.0, pp, wb.outer_iters, wb.inner_iters,
                                       240, seed=synth.coin_seed(wb.index, i), H=wb.H, W=wb.W)
        Vs.append(v)
        ls += [wb.alpha / pp] * v.shape[0]
    T.tvs_op_destroy(opb)
    take(torch.cat(Vs), ls, "deblur512", 0)
    del Vs

    # CT 512^2 (the workload of the timed run, other phantoms)
    def problem(i):
        u, eta = synth.make_inputs(w, seed_index=i)
        Au = torch.empty(na, nd, dtype=torch.float64, device=dev)
        T.tvs_op_apply(op, torch.tensor(u, device=dev), Au)
        return (Au + w.noise * Au.max() * torch.tensor(eta, device=dev)).float().contiguous()

    def record(bb, i, m=340):
        return learned.record_prox_inputs(op, bb, w.alpha, sigma, p, w.outer_iters, Kin, m,
                                          nonneg=1, seed=synth.coin_seed(w.index, i),
                                          dual_step=tau, H=N, W=N)

    V = torch.cat([record(problem(i), i) for i in (1, 2)])
    take(V, [lam] * V.shape[0], "ct512", 1)
    del V
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    cnn = T.tvs_cnn_create(ctx, 7)
    secs, loss = learned.train_groups(cnn, groups, steps, batch=32, lr=1e-3, mu=0.1, seed=3,
                                      log_every=1000, log=log)
    n_pairs = sum(g[0].shape[0] for g in groups)
    log(f"learned prox: {n_pairs} pairs ({t_data:.1f} s), {steps} steps in {secs:.1f} s")
    del groups
    torch.cuda.empty_cache()
    Vt = record(b, 0, 320)[::8].contiguous()
    res = {"config": "4-layer 3x3 CNN (2-32-32-32-2), BF16 MFMA with FP32 accumulation; pairs "
                     "from the denoising, deblurring and CT workloads in 128^2 crops; targets to "
                     "relative gap 1e-4; gate 1e-3",
           "pairs": n_pairs, "sources": info, "data_s": round(t_data, 2),
           "train_steps": steps, "train_batch": 32, "train_s": round(secs, 2),
           "train_ms_per_step": round(1e3 * secs / steps, 3), "final_loss": loss, "lam": lam}
    g50 = learned.cold_start_gaps(ctx, cnn, Vt, lam, Kin, nonneg=1)
    zero50 = float(np.median(g50["zero"]))
    res["cold_gap_after_50"] = {"zero_start": zero50, "network_start": float(np.median(g50["cnn"]))}
    g0 = learned.cold_start_gaps(ctx, cnn, Vt, lam, 0, nonneg=1)
    res["cold_gap_network_alone"] = float(np.median(g0["cnn"]))
    match = None
    for k in range(5, Kin + 1, 5):
        if np.median(learned.cold_start_gaps(ctx, cnn, Vt, lam, k, nonneg=1)["cnn"]) <= zero50:
            match = k
            break
    res["network_start_iters_to_match_zero_start_50"] = match
    # times of the pieces
    qb = torch.empty(2, N, N, device=dev)
    zb = torch.empty(N, N, device=dev)
    t_fgp = _evtime(lambda: T.tvs_tv_prox(ctx, Vt[0], lam, Kin, 1, qb, zb), 5)
    t_fin = _evtime(lambda: T.tvs_tv_prox(ctx, Vt[0], lam, 0, 1, qb, zb), 5)
    qt = torch.empty(1, 2, N, N, device=dev)
    fwd = {}
    for fast in (False, True):
        T.tvs_cnn_set_fast_forward(cnn, fast)
        fwd["bf16x1" if fast else "bf16x3"] = round(
            _evtime(lambda: T.tvs_cnn_forward(cnn, Vt[0], lam, 1, qt, None), 10), 4)
    per_it = (t_fgp - t_fin) / Kin
    res["ms"] = {"fgp_50": round(t_fgp, 4), "fgp_per_iter": round(per_it, 5),
                 "network_forward": fwd}
    # MFMA rate of the forward (two-part mode issues three MFMAs per product)
    res["network_forward_mfma_frac_of_bf16_peak"] = {
        k: round((3 if k == "bf16x3" else 1) * CNN_FLOP_PER_PX * N * N / (ms * 1e-3) / 1e12
                 / PEAK_BF16_TFLOPS, 4) for k, ms in fwd.items()}
    # the solver with the gap-gated learned prox, single-part forward
    T.tvs_cnn_set_fast_forward(cnn, True)
    phis = (tta or {}).get("phi_star")
    if phis:
        x = torch.zeros(N, N, device=dev)
        h, q, y = torch.zeros_like(x), torch.zeros(2, N, N, device=dev), torch.zeros(na, nd, device=dev)

        def solve(iters, gate, obj=False):
            for t in (x, h, q, y):
                t.zero_()
            return T.tvs_pdhgskip_ex(op, b, x, h, q, y, w.alpha, sigma, tau, p, iters, Kin,
                                     nonneg=1, seed=seed, want_obj=obj, graph=not obj,
                                     cnn=cnn, gap_tol=gate)

        plain = (tta or {}).get(f"pdhgskip_p{p}") or {}
        # the configuration's gate (1e-3), and a gate at the target accuracy
        for gate in (1e-3, 1e-4):
            r = solve(w.outer_iters, gate, obj=True)
            rel = np.abs(r["obj"] - phis) / phis
            bad = np.nonzero(rel > 1e-4)[0]
            kstar = int(bad[-1] + 2) if len(bad) else 1
            out = {"iters_to_1e-4": kstar if kstar <= w.outer_iters else None,
                   "final_rel": float(rel[-1]), "prox_calls": int(r["n_prox"]),
                   "fgp_fallbacks": int(r["n_fallback"]), "forward": "bf16x1"}
            if kstar <= w.outer_iters:
                times = []
                for _ in range(3):
                    solve(kstar, gate)  # capture / warm
                    torch.cuda.synchronize()
                    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    e0.record()
                    solve(kstar, gate)
                    e1.record()
                    torch.cuda.synchronize()
                    times.append(e0.elapsed_time(e1))
                out["ms_to_1e-4"] = round(float(np.median(times)), 3)
            if plain.get("ms") and out.get("ms_to_1e-4"):
                out["plain_pdhgskip_ms_to_1e-4"] = plain["ms"]
                out["plain_pdhgskip_iters_to_1e-4"] = plain["iters"]
                out["speedup_vs_plain"] = round(plain["ms"] / out["ms_to_1e-4"], 3)
            res[f"pdhgskip_learned_gate_{gate:g}"] = out
            log(f"learned PDHGSkip-2, gate {gate:g}: {out}")
    T.tvs_cnn_destroy(cnn)
    return res


BATCHED_SUMMARY = os.path.join(ROOT, "profiles", "fgp_batched_c4.md")


def batched_fgp_record():
    """The committed rocprofv3 record of the batched FGP kernels in one
    batched solve (kernel time and counter bytes), or None when a source it
    depends on changed since it was taken."""
    import hashlib
    import re
    try:
        text = open(BATCHED_SUMMARY).read()
        rec = json.loads(re.search(r"```json\n(.*?)\n```", text, re.S).group(1))
        for src, want in rec["source_sha256"].items():
            if hashlib.sha256(open(os.path.join(ROOT, src), "rb").read()).hexdigest() != want:
                return None
    except (OSError, AttributeError, ValueError, KeyError):
        return None
    return rec


def batched_bench(T, K=500, Kin=50, plain=True, tune_load=None, tune_save=None):
    """The batched workload (256 slices, sizes 128..1024 squared, per-slice
    alpha and p, A = I, gamma = 1, 500 outer iterations, 50 FGP iterations):
    one batched run captured in a HIP graph, against the plain method, one
    single-image solve per slice.  Both produce identical iterates (tested),
    so any time-to-accuracy target is reached at the same iteration counts
    and the ratio of run times is the ratio of times to that accuracy.  Both
    sides run on FGP variants picked by the autotuner, in a context of their
    own: the batched run's for the batch, the plain run's per slice size."""
    import numpy as np
    import torch
    import synth
    dev = torch.device("cuda:0")
    sp = synth.batched_slices()
    slices, off = [], 0
    for s in sp:
        slices.append(dict(H=s["H"], W=s["W"], offset=off, alpha=s["alpha"], p=s["p"],
                           seed=s["seed"], stream_id=s["stream"]))
        off += s["H"] * s["W"]
    total = off
    b = torch.empty(total, dtype=torch.float32, device=dev)
    for sl, s in zip(slices, sp):
        u, eta = synth.batched_slice_inputs(s)
        b[sl["offset"]:sl["offset"] + sl["H"] * sl["W"]] = torch.tensor(
            (u + s["sigma"] * eta).ravel(), dtype=torch.float32)
    x = torch.zeros(total, device=dev)
    h = torch.zeros_like(x)
    q = torch.zeros(2 * total, device=dev)
    ctx = T.tvs_ctx_create(0)  # its own tuning table
    tuned = {}
    if tune_load:
        T.tvs_tune_load(ctx, tune_load)
        for n in sorted({s["H"] for s in sp}):
            tuned[str(n)] = list(T.tvs_fgp_variant(T.tvs_fgp_query(ctx, T.TVS_F32, n, n)[0]))
        vb = T.tvs_fgp_query_batched(ctx, T.TVS_F32, len(slices))[0]
    else:
        for n in sorted({s["H"] for s in sp}):
            vi, _ = T.tvs_fgp_autotune(ctx, T.TVS_F32, n, n, Kin, 2)
            tuned[str(n)] = list(T.tvs_fgp_variant(vi))
        vb, _ = T.tvs_fgp_autotune_batched(ctx, T.TVS_F32, slices, Kin, 2)
    if tune_save:
        T.tvs_tune_save(ctx, tune_save)

    def run_batched():
        for t in (x, h, q):
            t.zero_()
        return T.tvs_proxskip_batched(ctx, slices, b, x, h, q, 1.0, K, Kin, graph=True)

    log(f"batched: {len(slices)} slices, {K} outer iterations: warm run")
    nprox = run_batched()                       # capture + warm
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    run_batched()
    e1.record()
    torch.cuda.synchronize()
    ms_b = e0.elapsed_time(e1)
    # algorithmic FGP bytes of the solve: 28 B/px per FGP iteration (read two
    # dual iterates and v, write one) over every slice's prox calls
    nprox = np.asarray(nprox)
    alg = 28.0 * Kin * float(sum(int(c) * s["H"] * s["W"] for c, s in zip(nprox, sp)))
    if not plain:
        res = {"slices": len(slices), "outer_iters": K, "inner_iters": Kin,
               "prox_calls": int(np.sum(nprox)), "batched_ms": round(ms_b, 2),
               "fgp_algorithmic_bytes_per_solve": alg,
               "fgp_variant_batched": list(T.tvs_fgp_variant(vb))}
        log(f"batched: {res}")
        del x, h, q, b
        T.tvs_ctx_destroy(ctx)
        torch.cuda.empty_cache()
        return res
    # plain method: one solve per slice (stream launches, the faster of the two
    # single-image modes for short runs; a graph per slice pays its capture)
    ops = {}
    for sl in slices:
        key = (sl["H"], sl["W"])
        if key not in ops:
            ops[key] = T.tvs_op_identity(ctx, *key)
    views = []
    for sl in slices:
        n = sl["H"] * sl["W"]
        o = sl["offset"]
        views.append((b[o:o + n].view(sl["H"], sl["W"]), x[o:o + n].view(sl["H"], sl["W"]),
                      h[o:o + n].view(sl["H"], sl["W"]),
                      q[2 * o:2 * o + 2 * n].view(2, sl["H"], sl["W"])))

    def run_plain():
        for t in (x, h, q):
            t.zero_()
        for sl, (bv, xv, hv, qv) in zip(slices, views):
            T.tvs_proxskip(ops[(sl["H"], sl["W"])], bv, xv, hv, qv, sl["alpha"], 1.0, sl["p"], K,
                           Kin, seed=sl["seed"], stream_id=sl["stream_id"])

    run_plain()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record()
    run_plain()
    e1.record()
    torch.cuda.synchronize()
    ms_p = max(e0.elapsed_time(e1), (time.perf_counter() - t0) * 1e3)
    for op in ops.values():
        T.tvs_op_destroy(op)
    px = float(total)
    res = {"slices": len(slices), "pixels": int(total), "outer_iters": K, "inner_iters": Kin,
           "prox_calls": int(np.sum(nprox)),
           "batched_ms": round(ms_b, 2), "plain_per_slice_ms": round(ms_p, 2),
           "speedup": round(ms_p / ms_b, 3),
           "batched_Gpx_iters_per_s": round(px * K / (ms_b * 1e-3) / 1e9, 3),
           "fgp_variant_batched": list(T.tvs_fgp_variant(vb)), "fgp_variant_per_size": tuned,
           "fgp_algorithmic_bytes_per_solve": alg}
    # roofline of the batched FGP kernels: their time in one solve and their
    # counter bytes (FETCH_SIZE + WRITE_SIZE, copy-calibrated) from the
    # committed rocprofv3 record of the same solve
    # (profiled on a shorter batched solve of the same slices and variants:
    # counter collection serialises every launch)
    rec = batched_fgp_record()
    if rec and rec.get("slices") == len(slices) and rec.get("inner_iters") == Kin:
        t = rec["fgp_kernel_ms_per_solve"] * 1e-3
        a = rec["algorithmic_bytes_per_solve"]
        meas = rec["fetch_bytes_per_solve"] + rec["write_bytes_per_solve"]
        res["fgp_roofline"] = {
            "bound": "hbm", "unit": "GB/s", "peak": PEAK_HBM_GBS,
            "profiled_solve_outer_iters": rec["outer_iters"],
            "profiled_variant": rec["fgp_variant"],
            "same_variant_as_this_run": rec["fgp_variant"] == list(T.tvs_fgp_variant(vb)),
            "kernel_ms_per_solve": rec["fgp_kernel_ms_per_solve"],
            "algorithmic_bytes_per_solve": a,
            "achieved": round(a / t / 1e9, 1),
            "frac": round(a / t / 1e9 / PEAK_HBM_GBS, 4),
            "traffic_per_solve": meas,
            "measured_hbm_GB/s": round(meas / t / 1e9, 1),
            "measured_frac_of_hbm_peak": round(meas / t / 1e9 / PEAK_HBM_GBS, 4)}
    log(f"batched: {res}")
    del x, h, q, b
    T.tvs_ctx_destroy(ctx)
    torch.cuda.empty_cache()
    return res


def cpu_baseline(b, w, ang, sigma, tau, seed, target_s=12.0):
    """The CPU oracle (float64, OpenMP) on the same inputs, timed on this
    host's cores over the first outer iterations of the same run."""
    import oracle as O
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    A = O.joseph(w.H, w.W, ang, w.n_det, w.pixel, w.det_spacing)
    t0 = time.perf_counter()
    O.pdhgskip(A, b, w.alpha, sigma, tau, w.p, 2, w.inner_iters, nonneg=1, seed=seed)
    per = (time.perf_counter() - t0) / 2
    n = max(4, min(200, int(target_s / max(per, 1e-3))))
    t0 = time.perf_counter()
    r = O.pdhgskip(A, b, w.alpha, sigma, tau, w.p, n, w.inner_iters, nonneg=1, seed=seed)
    el = time.perf_counter() - t0
    log(f"CPU oracle: {n} iterations in {el:.2f} s on {threads} threads ({r['nprox']} prox)")
    out = {"value": round(n / el, 4), "unit": "outer_iters/s", "cores": threads, "kind": "oracle",
           "sample": f"first {n} of the {w.outer_iters} outer iterations of the same run "
                     f"({r['nprox']} prox calls, float64)", "seconds": round(el, 2)}
    # the same on one thread (OpenMP runtime of the oracle library), shorter sample
    try:
        import ctypes
        gomp = ctypes.CDLL("libgomp.so.1")
    except OSError:
        gomp = None
    if gomp is not None and threads > 1:
        # a window whose prox rate is the run's: the first n >= 10 iterations
        # with a coin count within 30 % of p n
        theta = [O.coin(seed, 0, k, w.p) for k in range(200)]
        n1, cnt = 10, sum(theta[:10])
        while n1 < 200 and abs(cnt - w.p * n1) > 0.3 * w.p * n1:
            cnt += theta[n1]
            n1 += 1
        gomp.omp_set_num_threads(1)
        try:
            t0 = time.perf_counter()
            r1 = O.pdhgskip(A, b, w.alpha, sigma, tau, w.p, n1, w.inner_iters, nonneg=1, seed=seed)
            el1 = time.perf_counter() - t0
        finally:
            gomp.omp_set_num_threads(threads)
        out["single_thread"] = {"value": round(n1 / el1, 4),
                                "sample": f"first {n1} outer iterations ({r1['nprox']} prox calls, "
                                          f"the run's prox rate {w.p})",
                                "seconds": round(el1, 2)}
        log(f"CPU oracle, one thread: {n1} iterations in {el1:.2f} s ({r1['nprox']} prox)")
    out["host_cpu"] = host_cpu()
    return out


def host_cpu():
    """CPU model and the cores this process may use (from /proc/cpuinfo and
    the scheduler affinity)."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = os.cpu_count()
    return {"model": model, "logical_cpus": os.cpu_count(), "usable_cpus": usable}


if __name__ == "__main__":
    main()
