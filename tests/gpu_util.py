"""Helpers shared by the GPU parity tests (inputs to both sides, comparisons)."""
import numpy as np
import torch

import oracle as O
import synth

DEV = torch.device("cuda:0")
F32, F64 = torch.float32, torch.float64


def dev(a, dtype):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


def host(x):
    torch.cuda.synchronize()
    return x.detach().double().cpu().numpy()


def rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300))


def as_input(a, dtype):
    """The values both sides see: float32 inputs are rounded once, and the
    oracle gets the rounded values in float64."""
    return synth.to_f32_exact(a) if dtype == F32 else np.asarray(a, dtype=np.float64)


def ct_problem(N, n_ang, n_det, n_ell=8, seed=21, dtype=F32, noise=0.01):
    ang = synth.parallel_beam_angles(n_ang)
    u, eta = synth.phantom_and_noise(N, N, n_ell, seed, (n_ang, n_det))
    A = O.joseph(N, N, ang, n_det, 2.0 / N, 2.0 / N)
    Au = A.apply(u)
    b = as_input(Au + noise * Au.max() * eta, dtype)
    return ang, A, u, b


def blur_problem(N, seed=22, dtype=F32, noise=0.01, n_ell=8):
    k = synth.gaussian_blur_kernel(9, 2.0)
    u, eta = synth.phantom_and_noise(N, N, n_ell, seed, (N, N))
    A = O.blur(N, N, k)
    b = as_input(A.apply(u) + noise * eta, dtype)
    return k, A, u, b


def denoise_problem(N, seed=23, dtype=F64, noise=0.05, n_ell=8):
    u, eta = synth.phantom_and_noise(N, N, n_ell, seed, (N, N))
    return u, as_input(u + noise * eta, dtype)
