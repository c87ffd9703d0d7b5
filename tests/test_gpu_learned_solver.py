"""GPU checks of solver runs with the learned prox and with prox-input
recording (tvs_proxskip_ex / tvs_pdhgskip_ex).

- Recording leaves the run bitwise unchanged, and the recorded prox inputs
  equal the prox argument of the algorithm formed from the oracle's state
  (v = x_k - step * grad + (step - step / p) h_k) after the same iterations.
- A network whose parameters are all zero predicts q = 0, so with the gate
  always open every prox call returns P_X(v): the run equals the plain run
  with alpha = 0 bit for bit.
- With the gate always closed, every call runs inner_iters FGP iterations
  from the zero network dual or the previous call's dual, whichever has the
  smaller relative gap: the run equals the oracle stepped one iteration at a
  time with that choice made in float64 before each prox call.
- The previous call's dual is checked before the network: a network whose
  output is NaN never matters when that dual passes the gate (no call falls
  back, the run equals the alpha = 0 run), and always falls back when it
  does not (the run equals the plain run).
"""
import numpy as np
import pytest
import torch

import oracle as O
import paper_2411_00688_amd as T
import synth
from gpu_util import F32, as_input, ct_problem, denoise_problem, dev, host, rel_l2

pytestmark = pytest.mark.gpu


def zeros(shape, dt=F32):
    return torch.zeros(shape, dtype=dt, device="cuda")


@pytest.fixture
def zero_cnn(ctx):
    c = T.tvs_cnn_create(ctx, 1)
    T.tvs_cnn_set_params(c, np.zeros(T.tvs_cnn_param_count(), dtype=np.float32))
    yield c
    T.tvs_cnn_destroy(c)


def ct_setup(ctx, N=48, na=36, nd=69):
    ang, A, _, b = ct_problem(N, na, nd, dtype=F32)
    L = A.norm(60)
    op = T.tvs_op_ct_joseph(ctx, N, N, ang, nd, 2 / N, 2 / N)
    return A, b, L, op


def test_recording_is_passive_and_matches_prox_argument(ctx):
    A, b, L, op = ct_setup(ctx)
    N, (na, nd) = A.H, A.out_shape
    K, Kin, p, seed, alpha = 60, 20, 0.2, 31, 0.05
    sig = tau = 1.0 / L
    try:
        plain = [zeros((N, N)), zeros((N, N)), zeros((2, N, N)), zeros((na, nd))]
        r0 = T.tvs_pdhgskip(op, dev(b, F32), *plain, alpha, sig, tau, p, K, Kin, nonneg=1,
                            seed=seed, want_theta=True)
        st = [zeros((N, N)), zeros((N, N)), zeros((2, N, N)), zeros((na, nd))]
        rec = zeros((5, N, N))
        r1 = T.tvs_pdhgskip_ex(op, dev(b, F32), *st, alpha, sig, tau, p, K, Kin, nonneg=1,
                               seed=seed, v_record=rec)
        for a0, a1 in zip(plain, st):
            assert torch.equal(a0, a1)
        assert r1["n_recorded"] == min(5, r0["n_prox"]) and r1["n_fallback"] == 0
        # the oracle's state just before each recorded prox call
        calls = np.flatnonzero(r0["theta"])[:5]
        x = h = y = q = None
        k_done = 0
        for c, k in enumerate(calls):
            if k > k_done:
                ref = O.pdhgskip(A, b, alpha, sig, tau, p, int(k - k_done), Kin, nonneg=1,
                                 seed=seed, k0=k_done, x=x, h=h, y=y, q=q)
                x, h, y, q = ref["x"], ref["h"], ref["y"], ref["q"]
                k_done = int(k)
            if x is None:
                x, h, y, q = np.zeros((N, N)), np.zeros((N, N)), np.zeros((na, nd)), np.zeros((2, N, N))
            v = x - sig * A.adjoint(y) + (sig - sig / p) * h
            assert rel_l2(host(rec[c]), v) < 1e-4, c
    finally:
        T.tvs_op_destroy(op)


@pytest.mark.parametrize("graph", [False, True])
def test_zero_network_gate_open_equals_alpha_zero(ctx, zero_cnn, graph):
    A, b, L, op = ct_setup(ctx)
    N, (na, nd) = A.H, A.out_shape
    K, Kin, p, seed = 80, 10, 0.3, 5
    try:
        ref = [zeros((N, N)), zeros((N, N)), zeros((2, N, N)), zeros((na, nd))]
        T.tvs_pdhgskip(op, dev(b, F32), *ref, 0.0, 1 / L, 1 / L, p, K, Kin, nonneg=1, seed=seed)
        for rep in range(2 if graph else 1):
            st = [zeros((N, N)), zeros((N, N)), zeros((2, N, N)), zeros((na, nd))]
            r = T.tvs_pdhgskip_ex(op, dev(b, F32), *st, 0.05, 1 / L, 1 / L, p, K, Kin, nonneg=1,
                                  seed=seed, graph=graph, cnn=zero_cnn, gap_tol=float("inf"))
            assert r["n_fallback"] == 0
            for k in (0, 1, 3):  # x, h, y (q differs: alpha = 0 keeps q = 0 too)
                assert torch.equal(st[k], ref[k]), (rep, k)
            assert torch.count_nonzero(st[2]) == 0
    finally:
        T.tvs_op_destroy(op)


def test_zero_network_gate_closed_starts_from_better_dual(ctx, zero_cnn):
    N = 40
    _, b = denoise_problem(N, dtype=F32)
    K, Kin, p, seed, alpha = 30, 15, 0.4, 8, 0.1
    lam = alpha / p  # step 1
    # a poor initial dual: the first call must start from the network's zero
    q0 = as_input(np.random.default_rng(4).uniform(-lam, lam, (2, N, N)), F32)
    op = T.tvs_op_identity(ctx, N, N)
    try:
        x, h, q = zeros((N, N)), zeros((N, N)), dev(q0, F32)
        r = T.tvs_proxskip_ex(op, dev(b, F32), x, h, q, alpha, 1.0, p, K, Kin, seed=seed,
                              cnn=zero_cnn, gap_tol=-1.0, want_theta=True)
        assert r["n_fallback"] == r["n_prox"] > 0
        A = O.identity(N, N)
        xo, ho, qo = np.zeros((N, N)), np.zeros((N, N)), q0.astype(np.float64)
        starts = []
        for k in range(K):
            start = qo
            if r["theta"][k]:
                v = (xo - (xo - b)) + (1.0 - 1.0 / p) * ho  # the prox argument at step 1
                rel = []
                for cand in (np.zeros((2, N, N)), qo):
                    g, pr = O.tv_gap(v, lam, cand)
                    rel.append(g / pr if pr > 0 else g)
                # a clear margin, so float32 gaps take the same decision
                assert abs(rel[0] - rel[1]) > 1e-3 * max(rel), (k, rel)
                start = np.zeros((2, N, N)) if rel[0] < rel[1] else qo
                starts.append(rel[0] < rel[1])
            ref = O.proxskip(A, b, alpha, 1.0, p, 1, Kin, seed=seed, k0=k, x=xo, h=ho, q=start)
            xo, ho, qo = ref["x"], ref["h"], ref["q"]
        assert starts[0] and not all(starts)  # both starts are exercised
        assert rel_l2(host(x), xo) < 1e-4
        assert rel_l2(host(h), ho) < 1e-3
        assert rel_l2(host(q), qo) < 1e-3
    finally:
        T.tvs_op_destroy(op)


def test_nan_network_always_falls_back(ctx):
    """A network whose float32 activations overflow (all parameters 1e30, as
    after diverged training) yields NaN duals (inf scaled by 0 in the ball
    projection) and a NaN gap: with a gate no previous dual passes, every
    call falls back, inside a solver run from the previous call's dual, so
    the run equals the plain run bit for bit (graph and stream), and the
    standalone prox runs FGP from the zero dual."""
    cnn = T.tvs_cnn_create(ctx, 1)
    T.tvs_cnn_set_params(cnn, np.full(T.tvs_cnn_param_count(), 1e30, dtype=np.float32))
    A, b, L, op = ct_setup(ctx)
    N, (na, nd) = A.H, A.out_shape
    K, Kin, p, seed = 40, 10, 0.3, 12
    try:
        ref = [zeros((N, N)), zeros((N, N)), zeros((2, N, N)), zeros((na, nd))]
        r0 = T.tvs_pdhgskip(op, dev(b, F32), *ref, 0.05, 1 / L, 1 / L, p, K, Kin, nonneg=1,
                            seed=seed)
        for graph in (False, True):
            st = [zeros((N, N)), zeros((N, N)), zeros((2, N, N)), zeros((na, nd))]
            r = T.tvs_pdhgskip_ex(op, dev(b, F32), *st, 0.05, 1 / L, 1 / L, p, K, Kin, nonneg=1,
                                  seed=seed, graph=graph, cnn=cnn, gap_tol=1e-12)
            assert r["n_fallback"] == r["n_prox"] == r0["n_prox"] > 0
            for k in range(4):
                assert torch.equal(st[k], ref[k]), (graph, k)
        v = dev(A.adjoint(b) / N, F32)  # some image
        q = torch.empty(2, N, N, dtype=F32, device="cuda")
        z = torch.empty(N, N, dtype=F32, device="cuda")
        fb, rg = T.tvs_cnn_prox(cnn, v, 0.2, 1, 1.0, 15, q, z)
        assert fb and not np.isfinite(rg)
        q0, z0 = zeros((2, N, N)), torch.empty(N, N, dtype=F32, device="cuda")
        T.tvs_tv_prox(ctx, v, 0.2, 15, 1, q0, z0)
        assert torch.equal(q, q0) and torch.equal(z, z0)
    finally:
        T.tvs_op_destroy(op)
        T.tvs_cnn_destroy(cnn)


def test_previous_dual_that_passes_the_gate_skips_the_network(ctx):
    """Gate 1: the zero dual of the first call passes (its relative gap,
    TV(z) lam / P(z), is at most 1), so does every later call's (still zero):
    the NaN network is never consulted, no call falls back, and the run
    equals the alpha = 0 run (z = P_X(v) at every call) bit for bit."""
    cnn = T.tvs_cnn_create(ctx, 1)
    T.tvs_cnn_set_params(cnn, np.full(T.tvs_cnn_param_count(), 1e30, dtype=np.float32))
    A, b, L, op = ct_setup(ctx)
    N, (na, nd) = A.H, A.out_shape
    K, Kin, p, seed = 40, 10, 0.3, 12
    try:
        ref = [zeros((N, N)), zeros((N, N)), zeros((2, N, N)), zeros((na, nd))]
        T.tvs_pdhgskip(op, dev(b, F32), *ref, 0.0, 1 / L, 1 / L, p, K, Kin, nonneg=1, seed=seed)
        for graph in (False, True):
            st = [zeros((N, N)), zeros((N, N)), zeros((2, N, N)), zeros((na, nd))]
            r = T.tvs_pdhgskip_ex(op, dev(b, F32), *st, 0.05, 1 / L, 1 / L, p, K, Kin, nonneg=1,
                                  seed=seed, graph=graph, cnn=cnn, gap_tol=1.0)
            assert r["n_prox"] > 0 and r["n_fallback"] == 0
            for k in (0, 1, 3):
                assert torch.equal(st[k], ref[k]), (graph, k)
            assert torch.count_nonzero(st[2]) == 0
    finally:
        T.tvs_op_destroy(op)
        T.tvs_cnn_destroy(cnn)


def test_learned_solver_rejects_float64(ctx, zero_cnn):
    N = 16
    _, b = denoise_problem(N, dtype=torch.float64)
    op = T.tvs_op_identity(ctx, N, N)
    try:
        x = torch.zeros(N, N, dtype=torch.float64, device="cuda")
        with pytest.raises(T.TvsError):
            T.tvs_proxskip_ex(op, dev(b, torch.float64), x, x.clone(), torch.zeros(2, N, N,
                              dtype=torch.float64, device="cuda"), 0.1, 1.0, 0.5, 4, 4,
                              cnn=zero_cnn)
    finally:
        T.tvs_op_destroy(op)
