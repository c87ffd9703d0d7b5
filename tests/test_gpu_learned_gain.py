"""What the trained network gains over the method without it.

The network is trained on the GPU (its own forward and backward kernels) on
prox inputs recorded from ProxSkip runs of TV denoising, with targets from
long FGP solves.  On prox inputs of held-out runs, a cold prox call (no warm
dual) started from the trained network's dual reaches a smaller duality gap
after the same number of FGP iterations than the method's zero start; the
untrained network gives no such head start.
"""
import numpy as np
import pytest
import torch

import paper_2411_00688_amd as T
import synth
from paper_2411_00688_amd import learned

pytestmark = pytest.mark.gpu

N, ALPHA, P, K, KIN = 96, 0.1, 0.5, 60, 30
LAM = ALPHA * 1.0 / P


def runs(ctx, op, seeds):
    vs = []
    for s in seeds:
        u, eta = synth.phantom_and_noise(N, N, 12, 5000 + s, (N, N))
        b = torch.tensor(synth.to_f32_exact(u + 0.05 * eta), dtype=torch.float32, device="cuda")
        vs.append(learned.record_prox_inputs(op, b, ALPHA, 1.0, P, K, KIN, 40, seed=s,
                                             stream_id=s, H=N, W=N))
    return torch.cat(vs)


def test_trained_network_warm_start_beats_zero_start(ctx):
    op = T.tvs_op_identity(ctx, N, N)
    cnn = T.tvs_cnn_create(ctx, 3)
    try:
        V = runs(ctx, op, range(6))
        Vt = runs(ctx, op, (100, 101))[::4].contiguous()
        Z, Q = learned.fgp_targets(ctx, V, LAM, 200)
        before = learned.cold_start_gaps(ctx, cnn, Vt, LAM, 10)
        secs, loss = learned.train(cnn, V, Z, Q, LAM, steps=800, batch=8, lr=1e-3, mu=1.0)
        print(f"{V.shape[0]} pairs, 800 steps in {secs:.2f} s, loss {loss}")
        for iters in (0, 10, 30):
            g = learned.cold_start_gaps(ctx, cnn, Vt, LAM, iters)
            zero, net = np.median(g["zero"]), np.median(g["cnn"])
            print(f"FGP iterations {iters}: median relative gap zero {zero:.4f} network {net:.4f}")
            assert net < 0.8 * zero, iters
        assert np.median(before["cnn"]) > 0.9 * np.median(before["zero"])
    finally:
        T.tvs_cnn_destroy(cnn)
        T.tvs_op_destroy(op)
