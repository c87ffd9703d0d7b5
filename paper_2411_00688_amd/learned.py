"""Training pipeline of the learned TV prox, over the C ABI.

The network is trained on pairs the method itself produces: the prox inputs
v recorded during ProxSkip / PDHGSkip-2 runs (tvs_*_ex with v_record), with
targets from a long FGP solve of the same prox (z_target, q_target).  Every
computation runs in the library; this module only batches tensors.
"""
from __future__ import annotations

import time

from . import (tvs_cnn_prox, tvs_cnn_train_step, tvs_op_out_size, tvs_pdhgskip_ex,
               tvs_proxskip_ex, tvs_tv_prox)


def record_prox_inputs(op, b, alpha, step, p, outer_iters, inner_iters, max_record, nonneg=0,
                       seed=0, stream_id=0, dual_step=None, H=None, W=None):
    """Runs the solver once (PDHGSkip-2 if dual_step is given, else ProxSkip)
    from zero state and returns the prox inputs of its first max_record prox
    calls as an (m, H, W) float32 tensor."""
    import torch
    dev = b.device
    x = torch.zeros(H, W, device=dev)
    h = torch.zeros_like(x)
    q = torch.zeros(2, H, W, device=dev)
    rec = torch.zeros(max_record, H, W, device=dev)
    if dual_step is None:
        r = tvs_proxskip_ex(op, b, x, h, q, alpha, step, p, outer_iters, inner_iters,
                            nonneg=nonneg, seed=seed, stream_id=stream_id, v_record=rec)
    else:
        y = torch.zeros(tvs_op_out_size(op), device=dev)
        r = tvs_pdhgskip_ex(op, b, x, h, q, y, alpha, step, dual_step, p, outer_iters,
                            inner_iters, nonneg=nonneg, seed=seed, stream_id=stream_id,
                            v_record=rec)
    return rec[:r["n_recorded"]].contiguous()


def fgp_targets(ctx, V, lam, iters, nonneg=0):
    """(z_target, q_target) of every prox input: `iters` FGP iterations from
    a zero dual."""
    import torch
    n, H, W = V.shape
    Z = torch.empty_like(V)
    Q = torch.zeros(n, 2, H, W, device=V.device)
    for k in range(n):
        tvs_tv_prox(ctx, V[k], lam, iters, nonneg, Q[k], Z[k])
    return Z, Q


def train(cnn, V, Z, Q, lam, steps, batch=2, lr=1e-3, mu=0.1, nonneg=0, seed=0,
          lr_drop_at=0.8, log_every=0, log=print):
    """Adam on random mini-batches of the pairs (lr divided by 10 after the
    fraction lr_drop_at of the steps).  Returns (seconds, last loss)."""
    import numpy as np
    import torch
    rng = np.random.default_rng(seed)
    n = V.shape[0]
    lam_b = [float(lam)] * batch
    t0 = time.perf_counter()
    loss = None
    for s in range(steps):
        idx = torch.as_tensor(rng.choice(n, batch, replace=n < batch), device=V.device)
        want = s == steps - 1 or (bool(log_every) and s % log_every == 0)
        cur = lr * (0.1 if s >= lr_drop_at * steps else 1.0)
        loss = tvs_cnn_train_step(cnn, V[idx].contiguous(), lam_b, Z[idx].contiguous(), cur,
                                  nonneg=nonneg, want_loss=want, q_target=Q[idx].contiguous(),
                                  mu=mu)
        if want:
            log(f"  step {s}: loss {loss:.4e}")
    torch.cuda.synchronize()
    return time.perf_counter() - t0, loss


def cold_start_gaps(ctx, cnn, V, lam, iters, nonneg=0):
    """Relative duality gaps after `iters` FGP iterations on each prox input,
    starting from the zero dual and from the network's dual."""
    import torch
    H, W = V.shape[1:]
    out = {"zero": [], "cnn": []}
    for k in range(V.shape[0]):
        for name in ("zero", "cnn"):
            q = torch.zeros(2, H, W, device=V.device)
            z = torch.empty(H, W, device=V.device)
            if name == "cnn":
                tvs_cnn_prox(cnn, V[k], lam, nonneg, float("inf"), 0, q, z)
            out[name].append(tvs_tv_prox(ctx, V[k], lam, iters, nonneg, q, z, want_gap=True))
    return out
