"""Pins of the oracle's learned TV prox (network, head, loss gradient, Adam).

The network is 3x3 cross-correlation with zero padding, so every layer is a
sum over input channels of scipy.signal.correlate2d in 'same' mode; the head
reduces to a closed form when the network output is constant; the gradient is
checked against central finite differences of the oracle's own loss; Adam's
bias-corrected update has closed forms for the first step and for a constant
gradient.
"""
import numpy as np
import pytest
from scipy.signal import correlate2d

import oracle as O

CIN = [2, 32, 32, 32]
COUT = [32, 32, 32, 2]


def unpack(params):
    out, o = [], 0
    for ci, co in zip(CIN, COUT):
        w = params[o:o + 9 * ci * co].reshape(9, ci, co)
        o += 9 * ci * co
        b = params[o:o + co]
        o += co
        out.append((w, b))
    assert o == params.size
    return out


def he_params(rng, scale=1.0):
    parts = []
    for ci, co in zip(CIN, COUT):
        parts.append(rng.standard_normal(9 * ci * co) * scale * np.sqrt(2.0 / (9 * ci)))
        parts.append(rng.standard_normal(co) * 0.05)
    return np.concatenate(parts)


def scipy_forward(v, lam, params, nonneg):
    """The same network written with scipy's 2-D correlation per channel pair."""
    H, W = v.shape
    x = np.stack([v, np.full((H, W), lam)])
    layers = unpack(params)
    for l, (w, b) in enumerate(layers):
        ci, co = w.shape[1], w.shape[2]
        y = np.empty((co, H, W))
        for o in range(co):
            acc = np.full((H, W), b[o])
            for i in range(ci):
                k = w[:, i, o].reshape(3, 3)  # tap t = 3 * row + col, offsets -1..1
                acc = acc + correlate2d(x[i], k, mode="same", boundary="fill", fillvalue=0.0)
            y[o] = acc
        x = np.maximum(y, 0.0) if l < 3 else y
    qt = x
    z = v + O.div(O.proj_ball(qt, lam))
    if nonneg:
        z = np.maximum(z, 0.0)
    return qt, z


@pytest.mark.parametrize("shape,nonneg", [((7, 6), 0), ((5, 9), 1), ((1, 8), 0), ((6, 1), 1)])
def test_forward_matches_scipy_correlation(shape, nonneg):
    rng = np.random.default_rng(11 + shape[0])
    P = he_params(rng)
    v = rng.random((3,) + shape)
    lam = np.array([0.05, 0.2, 0.6])
    qt, z = O.cnn_forward(v, lam, P, nonneg)
    for b in range(3):
        qt_ref, z_ref = scipy_forward(v[b], lam[b], P, nonneg)
        np.testing.assert_allclose(qt[b], qt_ref, rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(z[b], z_ref, rtol=1e-12, atol=1e-12)


def test_head_closed_form_constant_dual():
    """All conv weights zero: qt is the last bias everywhere, q = P_lam(bias),
    and div of a constant field lives on the border rows and columns only."""
    H, W = 6, 7
    rng = np.random.default_rng(3)
    P = np.zeros(O.cnn_param_count())
    cy, cx = 0.3, -0.4          # |(cy, cx)| = 0.5
    P[-2:] = [cy, cx]
    v = rng.random((2, H, W))
    lam = np.array([1.0, 0.25])  # inside the ball, then scaled by 0.25 / 0.5
    qt, z = O.cnn_forward(v, lam, P)
    assert np.all(qt[:, 0] == cy) and np.all(qt[:, 1] == cx)
    for b, s in ((0, 1.0), (1, 0.5)):
        e = np.zeros((H, W))
        e[0, :] += s * cy
        e[H - 1, :] -= s * cy
        e[:, 0] += s * cx
        e[:, W - 1] -= s * cx
        np.testing.assert_allclose(z[b], v[b] + e, rtol=0, atol=1e-15)


def test_lambda_zero_returns_projected_input():
    rng = np.random.default_rng(5)
    P = he_params(rng)
    v = rng.standard_normal((2, 5, 5))
    _, z = O.cnn_forward(v, 0.0, P, nonneg=0)
    assert np.array_equal(z, v)
    _, z = O.cnn_forward(v, 0.0, P, nonneg=1)
    assert np.array_equal(z, np.maximum(v, 0.0))


def test_loss_is_half_mean_square():
    rng = np.random.default_rng(6)
    P = he_params(rng)
    v = rng.random((2, 6, 5))
    zt = rng.random((2, 6, 5))
    qtg = rng.standard_normal((2, 2, 6, 5)) * 0.1
    lam = np.array([0.1, 0.4])
    qt, z = O.cnn_forward(v, lam, P)
    loss, _ = O.cnn_loss_grad(v, lam, P, zt, want_grad=False)
    assert abs(loss - 0.5 * np.mean((z - zt) ** 2)) < 1e-15
    q = np.stack([O.proj_ball(qt[b], lam[b]) for b in range(2)])
    loss2, _ = O.cnn_loss_grad(v, lam, P, zt, want_grad=False, q_target=qtg, mu=0.7)
    ref = 0.5 * (np.sum((z - zt) ** 2) + 0.7 * np.sum((q - qtg) ** 2)) / z.size
    assert abs(loss2 - ref) < 1e-15


@pytest.mark.parametrize("nonneg,seed,mu", [(0, 21, 0.0), (1, 22, 0.0), (1, 23, 2.0)])
def test_gradient_central_differences(nonneg, seed, mu):
    rng = np.random.default_rng(seed)
    P = he_params(rng, scale=1.5)
    v = rng.random((2, 6, 5)) - 0.3 * nonneg
    lam = np.array([0.08, 0.3])
    zt = rng.random((2, 6, 5)) * 0.5
    qtg = rng.standard_normal((2, 2, 6, 5)) * 0.1 if mu else None
    loss, g = O.cnn_loss_grad(v, lam, P, zt, nonneg, q_target=qtg, mu=mu)
    # Loss ~ 0.1: the rounding error of a central difference is ~ 2e-17 / h,
    # the truncation error ~ h^2.  A random direction moves every
    # pre-activation, so its step stays small enough not to cross a ReLU or
    # projection kink; a single coordinate moves few of them.
    h_dir, h = 1e-6, 5e-5

    def L(p):
        return O.cnn_loss_grad(v, lam, p, zt, nonneg, want_grad=False, q_target=qtg, mu=mu)[0]

    # random directions: every parameter at once
    for _ in range(4):
        d = rng.standard_normal(P.size)
        fd = (L(P + h_dir * d) - L(P - h_dir * d)) / (2 * h_dir)
        an = g @ d
        assert abs(fd - an) <= 1e-7 * abs(an), (fd, an)
    # single coordinates in every layer, weights and biases
    offs = np.cumsum([0] + [9 * ci * co + co for ci, co in zip(CIN, COUT)])
    idx = []
    for l in range(4):
        idx += list(rng.integers(offs[l], offs[l + 1], 4))
        idx.append(offs[l + 1] - 1)  # last bias of the layer
    for i in idx:
        e = np.zeros(P.size)
        e[i] = 1.0
        fd = (L(P + h * e) - L(P - h * e)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(abs(g[i]), 1e-3 * np.abs(g).max()), (i, fd, g[i])


def test_adam_first_step_and_constant_gradient():
    rng = np.random.default_rng(9)
    n = 50
    g = rng.standard_normal(n)
    p0 = rng.standard_normal(n)
    p, m, v = p0.copy(), np.zeros(n), np.zeros(n)
    lr, eps = 1e-2, 1e-8
    for k in range(1, 6):
        O.adam_step(p, g, m, v, k, lr, eps=eps)
        # bias-corrected m and v equal g and g^2 at every step
        np.testing.assert_allclose(p, p0 - k * lr * g / (np.abs(g) + eps), rtol=0, atol=1e-13)
