"""Seeded synthetic inputs for the TV-regularised imaging workloads.

This module is shared by the CPU oracle side (tests, the CPU baseline) and the
GPU path (tests, bench).  It draws random numbers and paints phantoms; it holds
none of the method's arithmetic: no forward operator, no gradient, no prox, no
objective.  Where a workload needs ``b = A u + noise`` the caller applies its
own ``A`` to the phantom returned here and adds the noise field scaled as the
workload states.

The paper's own images (a 200x300 "shapes" image, a real catalyst CT slice)
are not available; these piecewise-constant ellipse phantoms with Gaussian
noise stand in for them, sized as the workloads below state.

Recipe (every draw from ``numpy.random.Generator(PCG64(seed))``, float64):
  for each ellipse, in draw order: centre row ~ U[0.1H, 0.9H], centre column
  ~ U[0.1W, 0.9W], semi-axes a, b ~ U[0.03M, 0.25M] with M = min(H, W),
  rotation ~ U[0, pi), intensity ~ U[0, 1].  A pixel (i, j) is tested at its
  centre (i + 0.5, j + 0.5); later ellipses overwrite earlier ones; the
  background is 0.  The noise field is standard normal, drawn from the same
  generator after the phantom.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "ellipse_phantom",
    "noise_field",
    "gaussian_blur_kernel",
    "parallel_beam_angles",
    "Workload",
    "WORKLOADS",
    "phantom_seed",
    "coin_seed",
    "batched_slices",
    "to_f32_exact",
]


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def ellipse_phantom(H: int, W: int, n_ellipses: int, seed: int,
                    rng: np.random.Generator | None = None) -> np.ndarray:
    """Piecewise-constant phantom in [0, 1], float64, shape (H, W)."""
    if rng is None:
        rng = _rng(seed)
    M = min(H, W)
    ii = np.arange(H, dtype=np.float64)[:, None] + 0.5
    jj = np.arange(W, dtype=np.float64)[None, :] + 0.5
    u = np.zeros((H, W), dtype=np.float64)
    for _ in range(n_ellipses):
        cy = rng.uniform(0.1 * H, 0.9 * H)
        cx = rng.uniform(0.1 * W, 0.9 * W)
        a = rng.uniform(0.03 * M, 0.25 * M)
        b = rng.uniform(0.03 * M, 0.25 * M)
        phi = rng.uniform(0.0, math.pi)
        val = rng.uniform(0.0, 1.0)
        dy = ii - cy
        dx = jj - cx
        c, s = math.cos(phi), math.sin(phi)
        e1 = (dx * c + dy * s) / a
        e2 = (-dx * s + dy * c) / b
        u[e1 * e1 + e2 * e2 <= 1.0] = val
    return u


def noise_field(shape, rng: np.random.Generator) -> np.ndarray:
    """Standard normal field drawn from ``rng`` (continue the phantom's rng)."""
    return rng.standard_normal(shape)


def phantom_and_noise(H: int, W: int, n_ellipses: int, seed: int, noise_shape):
    """Phantom, then a standard-normal noise field from the same generator."""
    rng = _rng(seed)
    u = ellipse_phantom(H, W, n_ellipses, seed, rng=rng)
    eta = noise_field(noise_shape, rng)
    return u, eta


def gaussian_blur_kernel(size: int = 9, sigma: float = 2.0) -> np.ndarray:
    """Centred size x size Gaussian, exp(-(m^2+n^2)/(2 sigma^2)), summing to 1.

    This is the definition of the blur operator's point-spread function (an
    input of the operator, like the CT angles), not part of the method.
    """
    r = size // 2
    m = np.arange(-r, r + 1, dtype=np.float64)
    g = np.exp(-(m[:, None] ** 2 + m[None, :] ** 2) / (2.0 * sigma * sigma))
    return g / g.sum()


def parallel_beam_angles(n_ang: int) -> np.ndarray:
    """theta_a = a * pi / n_ang, a = 0..n_ang-1 (float64)."""
    return np.arange(n_ang, dtype=np.float64) * (math.pi / n_ang)


def to_f32_exact(a: np.ndarray) -> np.ndarray:
    """Round to float32 and return the rounded values as float64.

    Both sides are fed the same rounded values so that input quantisation is
    not counted as error.
    """
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def phantom_seed(workload_index: int, i: int = 0) -> int:
    return 1000 * workload_index + i


def coin_seed(workload_index: int, i: int = 0) -> int:
    return 7000 + 1000 * workload_index + i


@dataclass(frozen=True)
class Workload:
    """One workload shape (sizes, weights, iteration counts)."""
    name: str
    index: int
    H: int
    W: int
    n_ellipses: int
    dtype: str            # "f64" or "f32"
    operator: str         # "identity" | "blur" | "ct"
    alpha: float
    p: float
    outer_iters: int
    inner_iters: int
    nonneg: int
    noise: float          # sigma (identity, blur) or fraction of max sinogram (ct)
    p_sweep: tuple = ()
    blur_size: int = 9
    blur_sigma: float = 2.0
    n_ang: int = 0
    n_det: int = 0
    extra: dict = field(default_factory=dict)

    @property
    def pixel(self) -> float:
        """CT pixel size: the image covers [-1, 1]^2."""
        return 2.0 / self.W

    @property
    def det_spacing(self) -> float:
        return 2.0 / self.W


WORKLOADS = {
    "denoise128": Workload(
        name="denoise128", index=1, H=128, W=128, n_ellipses=10, dtype="f64",
        operator="identity", alpha=0.1, p=0.1, outer_iters=500, inner_iters=100,
        nonneg=0, noise=0.05),
    "deblur512": Workload(
        name="deblur512", index=2, H=512, W=512, n_ellipses=30, dtype="f32",
        operator="blur", alpha=0.02, p=0.1, outer_iters=2000, inner_iters=50,
        nonneg=0, noise=0.01, p_sweep=(0.05, 0.1, 0.3)),
    "ct512": Workload(
        name="ct512", index=3, H=512, W=512, n_ellipses=30, dtype="f32",
        operator="ct", alpha=0.05, p=0.1, outer_iters=3000, inner_iters=50,
        nonneg=1, noise=0.01, n_ang=180, n_det=725),
}


def make_inputs(w: Workload, seed_index: int = 0, H: int | None = None,
                W: int | None = None, n_ang: int | None = None,
                n_det: int | None = None):
    """Phantom and the unscaled noise field for a workload (optionally resized).

    Returns (u_true, eta) as float64; eta has the data-space shape (image shape
    for identity/blur, (n_ang, n_det) for CT).
    """
    H = H or w.H
    W = W or w.W
    if w.operator == "ct":
        shape = (n_ang or w.n_ang, n_det or w.n_det)
    else:
        shape = (H, W)
    return phantom_and_noise(H, W, w.n_ellipses, phantom_seed(w.index, seed_index), shape)


BATCH_SIZES = (128, 256, 384, 512, 768, 1024)


def batched_slices(n: int = 256, seed: int = 4000, sizes=BATCH_SIZES):
    """Per-slice parameters of the batched denoising workload.

    Each slice: N ~ U{sizes}, ellipse count 10 + N // 64 capped at 30,
    sigma ~ U[0.02, 0.1], alpha = 2 sigma, p ~ U[0.05, 0.3], phantom seed
    4000000 + slice index, coin stream = slice index.
    """
    rng = _rng(seed)
    out = []
    for s in range(n):
        N = int(sizes[int(rng.integers(0, len(sizes)))])
        sigma = float(rng.uniform(0.02, 0.1))
        p = float(rng.uniform(0.05, 0.3))
        out.append(dict(index=s, H=N, W=N, n_ellipses=min(30, 10 + N // 64),
                        sigma=sigma, alpha=2.0 * sigma, p=p,
                        seed=4_000_000 + s, stream=s))
    return out


def batched_slice_inputs(sl: dict):
    """Phantom and noise field of one batched slice (float64)."""
    return phantom_and_noise(sl["H"], sl["W"], sl["n_ellipses"], sl["seed"],
                             (sl["H"], sl["W"]))


# ---------------------------------------------------------------- learned prox
CNN_LAYERS = ((2, 32), (32, 32), (32, 32), (32, 2))  # (in, out) channels, 3x3 kernels


def cnn_params(seed: int, scale: float = 1.0, bias_sd: float = 0.05) -> np.ndarray:
    """Seeded parameter vector of the learned-prox network (per layer
    W[9][in][out] then b[out]): He-scaled normal weights, small normal biases."""
    rng = _rng(seed)
    parts = []
    for ci, co in CNN_LAYERS:
        parts.append(rng.standard_normal(9 * ci * co) * scale * np.sqrt(2.0 / (9 * ci)))
        parts.append(rng.standard_normal(co) * bias_sd)
    return np.concatenate(parts)


def prox_training_inputs(n: int, H: int, W: int, seed: int, sigma=(0.02, 0.15),
                         lam=(0.02, 1.0), n_ellipses=(10, 30)):
    """n noisy phantoms v = u + sigma * noise and their prox weights lam
    (log-uniform), the inputs of the learned prox's training pairs."""
    rng = _rng(seed)
    vs = np.empty((n, H, W))
    lams = np.exp(rng.uniform(np.log(lam[0]), np.log(lam[1]), n))
    for k in range(n):
        s = int(rng.integers(0, 2**31 - 1))
        ne = int(rng.integers(n_ellipses[0], n_ellipses[1] + 1))
        u, eta = phantom_and_noise(H, W, ne, s, (H, W))
        vs[k] = u + rng.uniform(sigma[0], sigma[1]) * eta
    return vs, lams
