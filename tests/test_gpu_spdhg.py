"""GPU parity of the stochastic-angle method (SPDHG over interleaved angle
subsets with the prox skipped as in PDHGSkip-2, the paper's "Discussion and
Future work") against the oracle: coin and subset schedules bitwise, float64
iterates to rounding, float32 to the workload tolerances, graph replays equal
stream runs."""
import numpy as np
import pytest
import torch

import oracle as O
import paper_2411_00688_amd as T
import synth
from gpu_util import F32, F64, as_input, ct_problem, dev, host, rel_l2

pytestmark = pytest.mark.gpu


def zeros(shape, dt):
    return torch.zeros(shape, dtype=dt, device="cuda")


def subset_steps(A, ang, nd, N, n, rho=0.99):
    """SPDHG step sizes: sigma tau |A_j|^2 = rho^2 / n max-norm ratio < 1 / n."""
    m = max(O.joseph(N, N, ang[j::n], nd, 2.0 / N, 2.0 / N).norm(100) for j in range(n))
    return rho / (n * m), rho / m


@pytest.mark.parametrize("n,p", [(4, 0.3), (1, 1.0), (24, 0.5)])
def test_spdhgskip_f64_matches_oracle(ctx, n, p):
    N, na, nd = 32, 24, 47
    ang, A, _, b = ct_problem(N, na, nd, dtype=F64)
    sigma, tau = subset_steps(A, ang, nd, N, n)
    K, Kin = 60, 20
    ref = O.spdhgskip(A, b, n, 0.05, sigma, tau, p, K, Kin, nonneg=1, seed=6, want_obj=True)
    op = T.tvs_op_ct_joseph(ctx, N, N, ang, nd, 2.0 / N, 2.0 / N)
    try:
        x, h, q, y = zeros((N, N), F64), zeros((N, N), F64), zeros((2, N, N), F64), zeros((na, nd), F64)
        r = T.tvs_spdhgskip(op, dev(b, F64), x, h, q, y, n, 0.05, sigma, tau, p, K, Kin, nonneg=1,
                            seed=6, want_obj=True, want_theta=True, want_subsets=True)
        assert np.array_equal(r["theta"], ref["theta"])
        assert np.array_equal(r["subsets"], ref["subset"])
        assert r["n_prox"] == ref["nprox"]
        assert rel_l2(host(x), ref["x"]) < 1e-10
        assert rel_l2(host(y), ref["y"]) < 1e-10
        assert rel_l2(host(q), ref["q"]) < 1e-10
        assert np.max(np.abs(r["obj"] - ref["obj"]) / ref["obj"]) < 1e-12
    finally:
        T.tvs_op_destroy(op)


def test_spdhgskip_f32_graph_equals_stream_and_oracle(ctx):
    N, na, nd = 64, 45, 93
    ang, A, _, b = ct_problem(N, na, nd, dtype=F32)
    n, p, K, Kin = 5, 0.3, 120, 20
    sigma, tau = subset_steps(A, ang, nd, N, n)
    ref = O.spdhgskip(A, b, n, 0.05, sigma, tau, p, K, Kin, nonneg=1, seed=8)
    op = T.tvs_op_ct_joseph(ctx, N, N, ang, nd, 2.0 / N, 2.0 / N)
    try:
        outs = []
        for graph in (False, True, True):
            x, h, q, y = zeros((N, N), F32), zeros((N, N), F32), zeros((2, N, N), F32), zeros((na, nd), F32)
            T.tvs_spdhgskip(op, dev(b, F32), x, h, q, y, n, 0.05, sigma, tau, p, K, Kin, nonneg=1,
                            seed=8, graph=graph)
            torch.cuda.synchronize()
            outs.append([t.clone() for t in (x, h, q, y)])
        for o in outs[1:]:
            assert all(torch.equal(a, c) for a, c in zip(outs[0], o))
        x, h, q, y = outs[0]
        assert rel_l2(host(x), ref["x"]) < 1e-4
        assert rel_l2(host(y), ref["y"]) < 1e-4
    finally:
        T.tvs_op_destroy(op)


def test_spdhgskip_ct512_f32_100_iters(ctx):
    """The 512x512 CT workload (180 angles, 725 bins, alpha 0.05, u >= 0)
    with 10 angle subsets of 18 angles and p = 0.1, first 100 iterations."""
    w = synth.WORKLOADS["ct512"]
    ang = synth.parallel_beam_angles(w.n_ang)
    A = O.joseph(w.H, w.W, ang, w.n_det, w.pixel, w.det_spacing)
    u, eta = synth.make_inputs(w)
    Au = A.apply(u)
    b = as_input(Au + w.noise * Au.max() * eta, F32)
    n = 10
    m = max(O.joseph(w.H, w.W, ang[j::n], w.n_det, w.pixel, w.det_spacing).norm(30)
            for j in range(n))
    sigma, tau = 0.99 / (n * m), 0.99 / m
    K = 100
    seed = synth.coin_seed(w.index)
    ref = O.spdhgskip(A, b, n, w.alpha, sigma, tau, w.p, K, w.inner_iters, nonneg=1, seed=seed,
                      want_obj=True)
    op = T.tvs_op_ct_joseph(ctx, w.H, w.W, ang, w.n_det, w.pixel, w.det_spacing)
    try:
        x, h = zeros((w.H, w.W), F32), zeros((w.H, w.W), F32)
        q, y = zeros((2, w.H, w.W), F32), zeros((w.n_ang, w.n_det), F32)
        r = T.tvs_spdhgskip(op, dev(b, F32), x, h, q, y, n, w.alpha, sigma, tau, w.p, K,
                            w.inner_iters, nonneg=1, seed=seed, want_obj=True, want_theta=True,
                            want_subsets=True)
        assert np.array_equal(r["theta"], ref["theta"])
        assert np.array_equal(r["subsets"], ref["subset"])
        assert rel_l2(host(x), ref["x"]) < 1e-4
        assert rel_l2(host(y), ref["y"]) < 1e-4
        assert np.max(np.abs(r["obj"] - ref["obj"]) / ref["obj"]) < 1e-5
    finally:
        T.tvs_op_destroy(op)


def test_spdhgskip_argument_errors(ctx):
    op = T.tvs_op_identity(ctx, 8, 8)
    try:
        x, h, q = zeros((8, 8), F32), zeros((8, 8), F32), zeros((2, 8, 8), F32)
        y = zeros((8, 8), F32)
        with pytest.raises(T.TvsError) as e:
            T.tvs_spdhgskip(op, dev(np.zeros((8, 8)), F32), x, h, q, y, 2, 0.1, 0.1, 0.1, 0.5, 3, 2)
        assert e.value.status == 6
    finally:
        T.tvs_op_destroy(op)
    N, na, nd = 16, 6, 23
    ang = synth.parallel_beam_angles(na)
    op = T.tvs_op_ct_joseph(ctx, N, N, ang, nd, 2.0 / N, 2.0 / N)
    try:
        x, h, q = zeros((N, N), F32), zeros((N, N), F32), zeros((2, N, N), F32)
        y = zeros((na, nd), F32)
        for bad in (0, na + 1):
            with pytest.raises(T.TvsError):
                T.tvs_spdhgskip(op, zeros((na, nd), F32), x, h, q, y, bad, 0.1, 0.1, 0.1, 0.5, 3, 2)
    finally:
        T.tvs_op_destroy(op)
