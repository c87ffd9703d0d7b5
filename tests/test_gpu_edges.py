"""GPU edge cases: degenerate and extreme shapes, single angles and bins,
one-pixel problems, batches of one-pixel slices, and sizes at the documented
limits; each against the oracle or against an exact property.
"""
import numpy as np
import pytest
import torch

import oracle as O
import paper_2411_00688_amd as T
import synth
from gpu_util import F32, F64, as_input, dev, host, rel_l2

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("H,W", [(1, 32768), (32768, 1), (2, 20001), (3, 3)])
@pytest.mark.parametrize("dt", [F32, F64])
def test_fgp_extreme_aspect_ratios(ctx, H, W, dt):
    r = np.random.default_rng(H + W)
    v = as_input(r.random((H, W)), dt)
    z_ref, q_ref = O.fgp(v, 0.07, 25)
    q = torch.zeros(2, H, W, dtype=dt, device="cuda")
    z = torch.empty(H, W, dtype=dt, device="cuda")
    T.tvs_tv_prox(ctx, dev(v, dt), 0.07, 25, 0, q, z)
    tol = 1e-12 if dt == F64 else 1e-5
    assert rel_l2(host(z), z_ref) < tol
    assert rel_l2(host(q), q_ref) < tol * 10


@pytest.mark.parametrize("dt", [F32, F64])
def test_one_pixel_problem(ctx, dt):
    """One pixel: D = 0, so the prox is the identity (P_X aside) and ProxSkip
    is gradient descent on 1/2 (x - b)^2: x_k = b (1 - (1 - gamma)^k)."""
    b = torch.tensor([[0.75]], dtype=dt, device="cuda")
    q = torch.zeros(2, 1, 1, dtype=dt, device="cuda")
    z = torch.empty(1, 1, dtype=dt, device="cuda")
    T.tvs_tv_prox(ctx, b, 0.3, 10, 0, q, z)
    assert z.item() == 0.75 and torch.count_nonzero(q) == 0
    op = T.tvs_op_identity(ctx, 1, 1)
    try:
        x, h = torch.zeros(1, 1, dtype=dt, device="cuda"), torch.zeros(1, 1, dtype=dt, device="cuda")
        T.tvs_proxskip(op, b, x, h, q, 0.3, 0.5, 0.4, 30, 5, seed=2)
        ref = O.proxskip(O.identity(1, 1), np.array([[0.75]]), 0.3, 0.5, 0.4, 30, 5, seed=2)
        assert abs(x.item() - ref["x"][0, 0]) < (1e-15 if dt == F64 else 1e-6)
        assert abs(x.item() - 0.75 * (1 - 0.5 ** 30)) < 1e-6
    finally:
        T.tvs_op_destroy(op)


@pytest.mark.parametrize("n_ang,n_det", [(1, 1), (1, 40), (3, 1)])
def test_joseph_single_angle_or_bin(ctx, n_ang, n_det):
    N = 24
    ang = np.array([0.3, 1.2, 2.5])[:n_ang]
    A = O.joseph(N, N, ang, n_det, 2 / N, 2 / N)
    op = T.tvs_op_ct_joseph(ctx, N, N, ang, n_det, 2 / N, 2 / N)
    try:
        r = np.random.default_rng(3)
        for dt, tol in ((F64, 1e-13), (F32, 1e-6)):
            x = as_input(r.random((N, N)), dt)
            y = torch.empty(n_ang, n_det, dtype=dt, device="cuda")
            T.tvs_op_apply(op, dev(x, dt), y)
            yref = A.apply(x)
            assert np.abs(host(y) - yref).max() <= tol * max(1.0, np.abs(yref).max())
            yy = as_input(r.random((n_ang, n_det)), dt)
            xb = torch.empty(N, N, dtype=dt, device="cuda")
            T.tvs_op_adjoint(op, dev(yy, dt), xb)
            xref = A.adjoint(yy)
            assert np.abs(host(xb) - xref).max() <= tol * max(1.0, np.abs(xref).max())
    finally:
        T.tvs_op_destroy(op)


def test_batched_many_one_pixel_slices(ctx):
    n = 300
    slices = [dict(H=1, W=1, offset=s, alpha=0.1, p=0.3 + 0.002 * s, seed=s, stream_id=s)
              for s in range(n)]
    b = torch.tensor(np.linspace(0.0, 1.0, n), dtype=F64, device="cuda")
    x, h = torch.zeros(n, dtype=F64, device="cuda"), torch.zeros(n, dtype=F64, device="cuda")
    q = torch.zeros(2 * n, dtype=F64, device="cuda")
    T.tvs_proxskip_batched(ctx, slices, b, x, h, q, 0.5, 25, 3)
    for s in (0, 17, 299):
        ref = O.proxskip(O.identity(1, 1), b[s:s + 1].cpu().numpy().reshape(1, 1), 0.1, 0.5,
                         slices[s]["p"], 25, 3, seed=s, stream=s)
        assert abs(x[s].item() - ref["x"][0, 0]) < 1e-15


def test_size_limits_rejected(ctx):
    with pytest.raises(T.TvsError):
        T.tvs_op_identity(ctx, 0, 5)
    with pytest.raises(T.TvsError):
        T.tvs_op_identity(ctx, 65536, 32769)  # more than 2^31 pixels
    v = torch.zeros(1, 1, device="cuda")
    with pytest.raises((T.TvsError, ValueError)):
        T.tvs_tv_prox(ctx, v, -1.0, 3, 0, torch.zeros(2, 1, 1, device="cuda"),
                      torch.zeros(1, 1, device="cuda"))


@pytest.mark.parametrize("graph", [False, True])
def test_zero_outer_iterations_change_nothing(ctx, graph):
    """outer_iters = 0 is a valid empty run for every solver entry point: the
    state comes back bit for bit and no prox call is counted."""
    N, na, nd = 24, 12, 35
    ang = synth.parallel_beam_angles(na)
    op = T.tvs_op_ct_joseph(ctx, N, N, ang, nd, 2 / N, 2 / N)
    try:
        r = np.random.default_rng(5)
        b = dev(r.random((na, nd)), F32)
        st = [dev(r.random(s), F32) for s in ((N, N), (N, N), (2, N, N), (na, nd), (2, N, N))]
        before = [t.clone() for t in st]
        x, h, q, y, hin = st
        outs = [
            T.tvs_proxskip(op, b, x, h, q, 0.05, 0.1, 0.3, 0, 5, graph=graph),
            T.tvs_pdhgskip(op, b, x, h, q, y, 0.05, 0.3, 0.3, 0.3, 0, 5, graph=graph),
            T.tvs_pdhgskip_ex(op, b, x, h, q, y, 0.05, 0.3, 0.3, 0.3, 0, 5, graph=graph,
                              inner_p=0.3, inner_h=hin),
            T.tvs_spdhgskip(op, b, x, h, q, y, 3, 0.05, 0.1, 0.3, 0.3, 0, 5, graph=graph),
        ]
        torch.cuda.synchronize()
        for o in outs:
            assert o["n_prox"] == 0 and o["iters"] == 0
        assert outs[2]["n_inner_proj"] == 0
        for a, c in zip(before, st):
            assert torch.equal(a, c)
    finally:
        T.tvs_op_destroy(op)
