"""Pins of the oracle's discrete operators against facts the mathematics fixes.

D / div: adjoint identity, the closed-form spectrum of the Neumann Laplacian
(DCT-II), hand-computed special cases.  TV: closed form on a rectangle.
P_lam: the variational inequality that characterises a Euclidean projection.
Blur: numpy's FFT (circular convolution theorem).  Joseph: brute-force dense
transpose, cardinal angles (column / row sums), disk chord lengths.
"""

import math

import numpy as np
import pytest

import oracle as O
import synth


def rng(seed=0):
    return np.random.default_rng(seed)


# ----------------------------------------------------------------- D, div
@pytest.mark.parametrize("H,W", [(1, 7), (6, 1), (5, 7), (32, 17)])
def test_div_is_minus_grad_adjoint(H, W):
    r = rng(1)
    u = r.standard_normal((H, W))
    q = r.standard_normal((2, H, W))
    lhs = np.sum(O.grad(u) * q)
    rhs = -np.sum(u * O.div(q))
    assert abs(lhs - rhs) <= 1e-13 * (abs(lhs) + np.abs(u).sum())


@pytest.mark.parametrize("H,W", [(4, 6), (5, 7), (1, 9)])
def test_neumann_laplacian_spectrum(H, W):
    """-div grad is the Neumann Laplacian; its eigenvalues are
    4 sin^2(pi k / 2H) + 4 sin^2(pi l / 2W) (diagonalised by the DCT-II)."""
    n = H * W
    M = np.zeros((n, n))
    for c in range(n):
        e = np.zeros(n)
        e[c] = 1.0
        M[:, c] = -O.div(O.grad(e.reshape(H, W))).ravel()
    ev = np.sort(np.linalg.eigvalsh(M))
    ky = 4 * np.sin(np.pi * np.arange(H) / (2 * H)) ** 2
    kx = 4 * np.sin(np.pi * np.arange(W) / (2 * W)) ** 2
    ref = np.sort((ky[:, None] + kx[None, :]).ravel())
    assert np.allclose(ev, ref, atol=1e-12)
    # |D|^2 < 8, the bound behind the step 1/8
    assert ev[-1] < 8.0


def test_grad_special_cases():
    H, W = 4, 5
    ramp_x = np.tile(np.arange(W, dtype=float), (H, 1))
    g = O.grad(ramp_x)
    assert np.all(g[0] == 0.0)
    assert np.all(g[1][:, :-1] == 1.0) and np.all(g[1][:, -1] == 0.0)
    ramp_y = np.tile(np.arange(H, dtype=float)[:, None], (1, W))
    g = O.grad(ramp_y)
    assert np.all(g[1] == 0.0)
    assert np.all(g[0][:-1] == 1.0) and np.all(g[0][-1] == 0.0)
    # div of a single unit dual entry: +1 at the pixel, -1 at its successor
    q = np.zeros((2, H, W))
    q[1, 1, 2] = 1.0
    d = O.div(q)
    ref = np.zeros((H, W))
    ref[1, 2] = 1.0
    ref[1, 3] = -1.0
    assert np.array_equal(d, ref)
    # an entry in the last column has no difference behind it: div ignores it
    q = np.zeros((2, H, W))
    q[1, 2, W - 1] = 5.0
    q[0, H - 1, 1] = 7.0
    assert np.array_equal(O.div(q), np.zeros((H, W)))


def test_tv_rectangle_closed_form():
    """Indicator of [i0,i1) x [j0,j1) away from the border: every boundary
    pixel contributes 1, except the bottom-right inner corner whose two unit
    differences give sqrt(2):  TV = 2 w + 2 h - 2 + sqrt(2)."""
    H, W = 20, 30
    i0, i1, j0, j1 = 3, 11, 5, 19
    u = np.zeros((H, W))
    u[i0:i1, j0:j1] = 1.0
    ref = 2 * (j1 - j0) + 2 * (i1 - i0) - 2 + math.sqrt(2.0)
    assert abs(O.tv(u) - ref) < 1e-12
    assert O.tv(3.7 * np.ones((H, W))) == 0.0


# ----------------------------------------------------------------- P_lam
def test_projection_characterisation():
    r = rng(2)
    n = 4000
    lam = 0.7
    w = r.standard_normal((2, 1, n)) * 1.5
    P = O.proj_ball(w, lam)
    norms = np.sqrt(P[0] ** 2 + P[1] ** 2)
    assert np.all(norms <= lam * (1 + 1e-15))
    # identity inside the ball, idempotent
    inside = np.sqrt(w[0] ** 2 + w[1] ** 2) <= lam
    assert np.array_equal(P[:, inside], w[:, inside])
    assert np.allclose(O.proj_ball(P, lam), P, rtol=0, atol=1e-15)
    # <w - Pw, c - Pw> <= 0 for every c in the ball (Euclidean projection)
    for _ in range(20):
        ang = r.uniform(0, 2 * np.pi, n)
        rad = lam * np.sqrt(r.uniform(0, 1, n))
        c = np.stack([rad * np.sin(ang), rad * np.cos(ang)])[:, None, :]
        ip = np.sum((w - P) * (c - P), axis=0)
        assert np.all(ip <= 1e-12)


def test_projection_lambda_zero():
    w = rng(3).standard_normal((2, 3, 5))
    w[:, 0, 0] = 0.0
    P = O.proj_ball(w, 0.0)
    assert np.all(P == 0.0)


# ----------------------------------------------------------------- blur
@pytest.mark.parametrize("H,W,kh,kw", [(16, 20, 9, 9), (12, 9, 3, 5), (7, 11, 9, 9)])
def test_blur_matches_fft(H, W, kh, kw):
    r = rng(4)
    k = r.uniform(-0.2, 1.0, (kh, kw))
    x = r.standard_normal((H, W))
    A = O.blur(H, W, k)
    # circular convolution theorem with the kernel centred at (0, 0)
    kc = np.zeros((H, W))
    for a in range(kh):
        for c in range(kw):
            kc[(a - kh // 2) % H, (c - kw // 2) % W] += k[a, c]
    ref = np.real(np.fft.ifft2(np.fft.fft2(x) * np.fft.fft2(kc)))
    assert np.allclose(A.apply(x), ref, atol=1e-12)
    refT = np.real(np.fft.ifft2(np.fft.fft2(x) * np.conj(np.fft.fft2(kc))))
    assert np.allclose(A.adjoint(x), refT, atol=1e-12)


def test_blur_gaussian_properties():
    k = synth.gaussian_blur_kernel(9, 2.0)
    assert abs(k.sum() - 1.0) < 1e-15
    A = O.blur(32, 32, k)
    assert np.allclose(A.apply(np.ones((32, 32))), 1.0, atol=1e-14)
    assert abs(A.norm(300) - 1.0) < 1e-6


# ----------------------------------------------------------------- Joseph
def _dense(apply, n_in, in_shape):
    cols = []
    for c in range(n_in):
        e = np.zeros(n_in)
        e[c] = 1.0
        cols.append(apply(e.reshape(in_shape)).ravel())
    return np.stack(cols, axis=1)


def test_joseph_dense_transpose_exact():
    H, W, nd = 8, 8, 13
    ang = synth.parallel_beam_angles(6)
    A = O.joseph(H, W, ang, nd, 2.0 / W, 2.0 / W)
    M = _dense(A.apply, H * W, (H, W))
    MT = _dense(A.adjoint, len(ang) * nd, (len(ang), nd))
    assert np.array_equal(MT, M.T)
    assert np.all(M >= 0)


def test_joseph_dense_transpose_rect_and_odd_angles():
    H, W, nd = 5, 9, 11
    ang = np.array([0.1, 0.7, 1.2, 2.0, 2.9, np.pi / 4, 3 * np.pi / 4])
    A = O.joseph(H, W, ang, nd, 0.3, 0.21)
    M = _dense(A.apply, H * W, (H, W))
    MT = _dense(A.adjoint, len(ang) * nd, (len(ang), nd))
    assert np.array_equal(MT, M.T)


def test_joseph_adjoint_identity_larger():
    H = W = 64
    ang = synth.parallel_beam_angles(45)
    A = O.joseph(H, W, ang, 93, 2.0 / W, 2.0 / W)
    r = rng(5)
    x = r.standard_normal((H, W))
    y = r.standard_normal((45, 93))
    lhs = np.sum(A.apply(x) * y)
    rhs = np.sum(x * A.adjoint(y))
    assert abs(lhs - rhs) <= 1e-13 * np.sum(np.abs(A.apply(np.abs(x))) * np.abs(y))


def test_joseph_cardinal_angles():
    """theta = 0: rays are vertical lines x = s; with 13 bins over 8 columns at
    equal spacing every bin centre falls half-way between two pixel centres,
    so each bin is the mean of two adjacent column sums times the pixel size.
    theta = pi/2: the same with row sums (rows run the other way)."""
    H, W, nd = 8, 8, 13
    px = 0.25
    x = rng(6).standard_normal((H, W))
    A = O.joseph(H, W, np.array([0.0, np.pi / 2]), nd, px, px)
    y = A.apply(x)
    col = np.concatenate([[0.0] * 3, x.sum(axis=0), [0.0] * 3])  # col(j) at index j+3
    row = np.concatenate([[0.0] * 3, x.sum(axis=1), [0.0] * 3])
    for b in range(nd):
        # theta = 0: continuous column = b - 6 + 3.5 = b - 2.5
        j0 = b - 3
        ref0 = px * 0.5 * ((col[j0 + 3] if 0 <= j0 + 3 < len(col) else 0.0)
                           + (col[j0 + 4] if 0 <= j0 + 4 < len(col) else 0.0))
        assert abs(y[0, b] - ref0) < 1e-13
        # theta = pi/2: continuous row = 3.5 - (b - 6) = 9.5 - b
        i0 = 9 - b
        ref1 = px * 0.5 * ((row[i0 + 3] if 0 <= i0 + 3 < len(row) else 0.0)
                           + (row[i0 + 4] if 0 <= i0 + 4 < len(row) else 0.0))
        assert abs(y[1, b] - ref1) < 1e-12


def test_joseph_disk_chord_lengths():
    """A uniform disk of radius R projects to the chord length 2 sqrt(R^2 - s^2)
    at every angle.  The pixelated disk and the interpolation make the error
    first order in the pixel size: it stays within a few pixels, has no bias,
    and halves when the resolution doubles."""
    R = 0.6
    rms = []
    for N in (128, 256):
        px = 2.0 / N
        c = (np.arange(N) - (N - 1) / 2) * px
        X, Y = np.meshgrid(c, -c)
        disk = (X ** 2 + Y ** 2 <= R ** 2).astype(float)
        nd = int(np.ceil(N * 1.42)) | 1
        ang = synth.parallel_beam_angles(12)
        y = O.joseph(N, N, ang, nd, px, px).apply(disk)
        s = (np.arange(nd) - (nd - 1) / 2) * px
        chord = 2 * np.sqrt(np.maximum(R ** 2 - s ** 2, 0))
        e = (y - chord)[:, np.abs(s) < 0.9 * R]
        assert np.max(np.abs(e)) < 2 * px
        assert np.mean(np.abs(e)) < 0.6 * px
        assert abs(np.mean(e)) < 0.2 * px
        rms.append(np.sqrt(np.mean(e ** 2)))
    assert 0.35 < rms[1] / rms[0] < 0.65


def test_joseph_norm_matches_svd():
    H = W = 10
    ang = synth.parallel_beam_angles(8)
    A = O.joseph(H, W, ang, 15, 0.2, 0.2)
    M = _dense(A.apply, H * W, (H, W))
    smax = np.linalg.svd(M, compute_uv=False)[0]
    assert abs(A.norm(2000) - smax) < 1e-8 * smax


def test_identity_norm():
    assert abs(O.identity(8, 9).norm(5) - 1.0) < 1e-14
