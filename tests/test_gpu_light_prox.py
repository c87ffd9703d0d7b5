"""GPU parity of ProxSkip on Dual-ROF / Dual-Huber-ROF (Sec. 2.1-2.2).

Bars as for the other solvers: the coin schedule is bit-exact; float64 runs
agree with the oracle to 1e-10 relative L2 (FMA contraction on the GPU side
only); float32 runs to 1e-4 after 100 iterations; graph replays, resumed
runs and the fused-step boundaries (8 steps per launch) change nothing.
"""
import numpy as np
import pytest
import torch

import oracle as O
import paper_2411_00688_amd as T
import synth
from gpu_util import F32, F64, as_input, dev, host, rel_l2

pytestmark = pytest.mark.gpu


def noisy(H, W, seed, sigma=0.05):
    u, eta = synth.phantom_and_noise(H, W, 12, seed, (H, W))
    return u + sigma * eta


def run_gpu(ctx, b, alpha, eps, step, p, K, dt, seed=3, k0=0, q=None, h=None, graph=False):
    H, W = b.shape
    qd = torch.zeros(2, H, W, dtype=dt, device="cuda") if q is None else q
    hd = torch.zeros(2, H, W, dtype=dt, device="cuda") if h is None else h
    r = T.tvs_dual_rof_proxskip(ctx, dev(b, dt), qd, hd, alpha, eps, step, p, K, seed=seed,
                                k0=k0, graph=graph, want_theta=True)
    return qd, hd, r


@pytest.mark.parametrize("H,W", [(37, 45), (1, 60), (50, 1), (200, 300)])
@pytest.mark.parametrize("eps", [0.0, 0.05])
def test_f64_matches_oracle(ctx, H, W, eps):
    b = as_input(noisy(H, W, H + W), F64)
    alpha, p, K = 0.3, 0.2, 53          # K not a multiple of the fused depth
    step = 1.0 / (8.0 + eps / alpha)
    ref = O.dual_rof_proxskip(b, alpha, eps, step, p, K, seed=3)
    q, h, r = run_gpu(ctx, b, alpha, eps, step, p, K, F64)
    assert np.array_equal(r["theta"], ref["theta"]) and r["n_prox"] == ref["nprox"]
    assert rel_l2(host(q), ref["q"]) < 1e-10
    assert rel_l2(host(h), ref["h"]) < 1e-9


@pytest.mark.parametrize("eps,p", [(0.0, 0.1), (0.01, 0.04767), (0.0, 1.0)])
def test_f32_workload_100_iterations(ctx, eps, p):
    """The 200 x 300 shapes-like workload, alpha 0.5 (Dual-ROF) / 0.55
    (Dual-Huber-ROF), first 100 iterations in float32."""
    b = as_input(noisy(200, 300, 7), F32)
    alpha = 0.5 if eps == 0 else 0.55
    step = 1.0 / (8.0 + eps / alpha)
    ref = O.dual_rof_proxskip(b, alpha, eps, step, p, 100, seed=21)
    q, h, r = run_gpu(ctx, b, alpha, eps, step, p, 100, F32, seed=21)
    assert np.array_equal(r["theta"], ref["theta"])
    assert rel_l2(host(q), ref["q"]) < 1e-4
    u = dev(b, F32) + torch.zeros(200, 300, device="cuda")
    dq = torch.empty(200, 300, device="cuda")
    T.tvs_div(ctx, q, dq)
    assert rel_l2(host(u + dq), ref["u"]) < 1e-5


@pytest.mark.parametrize("eps", [0.0, 0.05])
def test_f64_large_image_matches_oracle(ctx, eps):
    """An image large enough for the 32 x 32-tile path (>= 2 tiles per CU)."""
    b = as_input(noisy(768, 800, 41), F64)
    alpha, p, K = 0.3, 0.3, 21
    step = 1.0 / (8.0 + eps / alpha)
    ref = O.dual_rof_proxskip(b, alpha, eps, step, p, K, seed=9)
    q, h, r = run_gpu(ctx, b, alpha, eps, step, p, K, F64, seed=9)
    assert np.array_equal(r["theta"], ref["theta"])
    assert rel_l2(host(q), ref["q"]) < 1e-10
    assert rel_l2(host(h), ref["h"]) < 1e-9


@pytest.mark.parametrize("eps", [0.0, 0.05])
def test_f64_one_tile_per_cu_path_matches_oracle(ctx, eps):
    """520 x 500 has between one and two 32 x 32 tiles per CU: the path with
    32 x 32 tiles, 8 steps per launch and 1024-thread workgroups."""
    b = as_input(noisy(520, 500, 17), F64)
    alpha, p, K = 0.3, 0.3, 21
    step = 1.0 / (8.0 + eps / alpha)
    ref = O.dual_rof_proxskip(b, alpha, eps, step, p, K, seed=12)
    q, h, r = run_gpu(ctx, b, alpha, eps, step, p, K, F64, seed=12)
    assert np.array_equal(r["theta"], ref["theta"])
    assert rel_l2(host(q), ref["q"]) < 1e-10
    assert rel_l2(host(h), ref["h"]) < 1e-9


def test_f32_8192_sampled_windows(ctx):
    """The 8192^2 float32 run the benchmark times (32 x 32 tiles, 8 steps per
    launch), checked on sampled windows: after K steps a pixel depends only
    on inputs within distance K, so the oracle on a window with a margin of
    K + 2 pixels is exact in the window's middle; the coin is the same
    stream (the window run uses the same seed)."""
    n, K = 8192, 16
    alpha, eps, p = 0.55, 0.01, 0.3
    step = 1.0 / (8.0 + eps / alpha)
    g = torch.Generator(device="cuda").manual_seed(6)
    b = torch.rand(n, n, device="cuda", generator=g)
    q = torch.zeros(2, n, n, device="cuda")
    h = torch.zeros_like(q)
    T.tvs_dual_rof_proxskip(ctx, b, q, h, alpha, eps, step, p, K, seed=13)
    m = K + 2
    for (i, j) in [(0, 0), (n - 24, n - 24), (31, 33), (4095, 5000), (0, 4000)]:
        i0, j0 = max(i - m, 0), max(j - m, 0)
        i1, j1 = min(i + 24 + m, n), min(j + 24 + m, n)
        bw = host(b[i0:i1, j0:j1]).astype(np.float64)
        ref = O.dual_rof_proxskip(bw, alpha, eps, step, p, K, seed=13)
        sl = (slice(None), slice(i - i0, i - i0 + 24), slice(j - j0, j - j0 + 24))
        assert np.abs(host(q[:, i:i + 24, j:j + 24]) - ref["q"][sl]).max() <= 1e-5, (i, j)
        assert np.abs(host(h[:, i:i + 24, j:j + 24]) - ref["h"][sl]).max() <= 1e-3, (i, j)


def test_p1_is_projgd(ctx):
    b = as_input(noisy(40, 33, 5), F64)
    ref = O.dual_rof_projgd(b, 0.25, 0.0, 1 / 8, 40)
    q, _, r = run_gpu(ctx, b, 0.25, 0.0, 1 / 8, 1.0, 40, F64)
    assert r["n_prox"] == 40
    assert rel_l2(host(q), ref["q"]) < 1e-12


def test_graph_resume_and_fusion_boundaries_bitwise(ctx):
    b = as_input(noisy(64, 70, 9), F32)
    args = (0.4, 0.02, 1 / 8.05, 0.3)
    q1, h1, _ = run_gpu(ctx, b, *args, 45, F32)
    for rep in range(2):
        q2, h2, _ = run_gpu(ctx, b, *args, 45, F32, graph=True)
        assert torch.equal(q1, q2) and torch.equal(h1, h2), rep
    # 45 = 13 + 32: a resumed run crosses the fused-step boundaries elsewhere
    q3, h3, _ = run_gpu(ctx, b, *args, 13, F32)
    q3, h3, _ = run_gpu(ctx, b, *args, 32, F32, k0=13, q=q3, h=h3)
    assert torch.equal(q1, q3) and torch.equal(h1, h3)


def test_invalid_arguments(ctx):
    b = torch.zeros(4, 4, device="cuda")
    q = torch.zeros(2, 4, 4, device="cuda")
    for bad in (dict(p=0.0), dict(p=1.2), dict(step=0.0), dict(alpha=-1.0), dict(eps=-0.1)):
        kw = dict(alpha=0.1, eps=0.0, step=0.125, p=0.5)
        kw.update(bad)
        with pytest.raises(T.TvsError):
            T.tvs_dual_rof_proxskip(ctx, b, q, q.clone(), kw["alpha"], kw["eps"], kw["step"],
                                    kw["p"], 4)
