"""Training pipeline of the learned TV prox, over the C ABI.

The network is trained on pairs the method itself produces: the prox inputs
v recorded during ProxSkip / PDHGSkip-2 runs (tvs_*_ex with v_record), with
targets from a long FGP solve of the same prox (z_target, q_target).  Every
computation runs in the library; this module only batches tensors.
"""
from __future__ import annotations

import time

from . import (tvs_cnn_prox, tvs_cnn_train_step, tvs_op_out_size, tvs_pdhgskip_ex,
               tvs_proxskip_batched, tvs_proxskip_ex, tvs_tv_gap, tvs_tv_prox)


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


def crops(V, size):
    """The non-overlapping size x size crops of every image of V (m, H, W),
    image by image in row-major tile order, as an (m k, size, size) tensor."""
    m, H, W = V.shape
    a, b = H // size, W // size
    if a == 0 or b == 0:
        raise ValueError(f"images of {H} x {W} have no {size} x {size} crop")
    C = V[:, :a * size, :b * size].reshape(m, a, size, b, size).permute(0, 1, 3, 2, 4)
    return C.reshape(m * a * b, size, size).contiguous()


def prox_targets(ctx, V, lams, nonneg=0, tol=1e-4, chunk=200, max_iters=6000, log=None):
    """The TV prox of every image of V (n, h, w, float32) at its own weight
    lams[i], to a relative duality gap of at most tol where max_iters FGP
    iterations reach it.  One batched call (A = I, step 1, p = 1, one outer
    iteration, whose prox argument is b itself) runs `chunk` FGP iterations
    on every image not yet converged, from its dual of the previous call;
    the relative gap gap(q) / P(z_q) of each image is checked between calls.
    Returns (Z, Q, relative gaps as a numpy array, FGP iterations run)."""
    import numpy as np
    import torch
    n, h, w = V.shape
    npx = h * w
    dev = V.device
    b = V.reshape(-1).contiguous()
    x = torch.zeros_like(b)
    hh = torch.zeros_like(b)
    q = torch.zeros(2 * b.numel(), device=dev)
    rel = np.full(n, np.inf)
    todo = np.arange(n)
    done_iters = 0
    while len(todo) and done_iters < max_iters:
        slices = [dict(H=h, W=w, offset=int(i) * npx, alpha=float(lams[i]), p=1.0, seed=0,
                       stream_id=int(i)) for i in todo]
        hh.zero_()  # the prox argument of the one outer iteration is b + h = b
        tvs_proxskip_batched(ctx, slices, b, x, hh, q, 1.0, 1, chunk, nonneg=nonneg)
        done_iters += chunk
        for i in todo:
            o = int(i) * npx
            g, pr = tvs_tv_gap(ctx, V[i], float(lams[i]), nonneg, q[2 * o:2 * o + 2 * npx].view(2, h, w))
            rel[i] = g / pr if pr > 0 else g
        todo = todo[rel[todo] > tol]
        if log:
            log(f"  prox targets: {done_iters} FGP iterations, {len(todo)} of {n} above {tol:g}")
    return x.view(n, h, w), q.view(n, 2, h, w), rel, done_iters


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


def train_groups(cnn, groups, steps, batch=32, lr=1e-3, mu=0.1, seed=0, lr_drop_at=0.8,
                 log_every=0, log=print):
    """Adam on pairs of several sources: groups is a list of (V, Z, Q, lams,
    nonneg), lams one weight per pair.  Each step draws a source (with
    probability proportional to its size) and a mini-batch from it, so that
    a batch shares the output constraint of its source.  The lr is divided
    by 10 after the fraction lr_drop_at of the steps.  Returns (seconds, last
    loss)."""
    import numpy as np
    import torch
    rng = np.random.default_rng(seed)
    sizes = np.array([g[0].shape[0] for g in groups], dtype=np.float64)
    t0 = time.perf_counter()
    loss = None
    for s in range(steps):
        V, Z, Q, lams, nonneg = groups[rng.choice(len(groups), p=sizes / sizes.sum())]
        n = V.shape[0]
        sel = rng.choice(n, batch, replace=n < batch)
        idx = torch.as_tensor(sel, device=V.device)
        want = s == steps - 1 or (bool(log_every) and s % log_every == 0)
        cur = lr * (0.1 if s >= lr_drop_at * steps else 1.0)
        loss = tvs_cnn_train_step(cnn, V[idx].contiguous(), [float(lams[i]) for i in sel],
                                  Z[idx].contiguous(), cur, nonneg=nonneg, want_loss=want,
                                  q_target=Q[idx].contiguous(), mu=mu)
        if want and log:
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
