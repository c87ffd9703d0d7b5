"""CPU FP64 oracle of the ProxSkip / PDHGSkip TV hot path (ctypes wrapper).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package.  It shares no code with the GPU
library (paper_2411_00688_amd) and neither imports the other.

Parity status of each function (what pins it lives in tests/test_oracle_*.py):
  grad, div, tv, proj_ball ........ pinned (adjoint identity, closed-form |D|^2,
                                     brute-force tiny cases, invariants)
  fgp, tv_gap ..................... pinned (taut string in 1-D, 2-pixel closed
                                     form, alpha = 0, constants, gap -> 0)
  blur apply / adjoint ............ pinned (numpy FFT circular convolution)
  joseph apply / adjoint .......... pinned (dense transpose, cardinal angles,
                                     disk chord lengths)
  proxskip / pdhgskip ............. pinned (p = 1 equals the separately written
                                     PGD / PDHG bitwise; fixed points; same
                                     minimiser as the reference solver)
  coin ............................ pinned (published SplitMix64 outputs of
                                     state 0, Bernoulli and run statistics)
  op_norm ......................... pinned (identity, blur = 1, SVD of small A)
  fista ........................... pinned (first call step equals one PGD
                                     step bitwise; momentum sequence against a
                                     separate t-recursion on A = I quadratics;
                                     converges to PGD's minimum)
  pdhgskip1 ....................... pinned (p = 1 equals the separately
                                     written PDHG bitwise; skipped iterations
                                     leave x bitwise; same minimum as PDHG)
  subset, subset_apply/adjoint .... pinned (uniform counts, pure function of
                                     (seed, stream, k); the rows of the full A)
  spdhgskip ....................... pinned (untouched subsets keep their rows
                                     bitwise; z = A^T y after a run; converges
                                     to the minimiser of PDHG / the explicit
                                     solver at several n and p)
  pdhg_explicit ................... pinned (agrees with PGD/PDHG minimisers and
                                     with the exact 1-D/2-pixel solutions)
  dual_rof_proxskip ............... pinned (p = 1 equals the separately written
                                     ProjGD bitwise; 2-pixel closed forms of
                                     Dual-ROF and Dual-Huber-ROF; the primal
                                     iterate reaches the TV prox, 1-D taut
                                     string; duality gap -> 0)
  tv_prox_skip .................... pinned (unconstrained: the separately
                                     written Dual-ROF ProxSkip bitwise, ProjGD
                                     at p_in = 1; 1-D taut string, clipped
                                     with u >= 0; constrained gap -> 0)
  proxskip_inner / pdhgskip_inner . pinned (one step on A = I is the TV prox;
                                     reference minimisers of denoising and CT;
                                     bitwise resume; inner coin stream)
  cnn_forward ..................... pinned (layers against scipy correlate2d,
                                     head closed form with zero weights)
  cnn_loss_grad ................... pinned (central finite differences)
  adam_step ....................... pinned (first step = -lr sign(g); constant-
                                     gradient closed form)
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
_lib = None

IDENTITY, BLUR, JOSEPH = 0, 1, 2


class OrcOp(C.Structure):
    _fields_ = [("kind", C.c_int), ("H", C.c_int), ("W", C.c_int),
                ("kernel", C.POINTER(C.c_double)), ("kh", C.c_int), ("kw", C.c_int),
                ("n_ang", C.c_int), ("angles", C.POINTER(C.c_double)),
                ("n_det", C.c_int), ("pixel", C.c_double), ("det_spacing", C.c_double)]


class OrcParams(C.Structure):
    _fields_ = [("alpha", C.c_double), ("step", C.c_double), ("dual_step", C.c_double),
                ("p", C.c_double), ("outer_iters", C.c_int64), ("inner_iters", C.c_int32),
                ("nonneg", C.c_int32), ("seed", C.c_uint64), ("stream_id", C.c_uint64),
                ("k0", C.c_int64)]


def lib():
    global _lib
    if _lib is None:
        path = os.path.join(_HERE, "liboracle.so")
        if not os.path.exists(path):
            _build.build()
        L = C.CDLL(path)
        dp = C.POINTER(C.c_double)
        L.orc_grad.argtypes = [C.c_int, C.c_int, dp, dp]
        L.orc_div.argtypes = [C.c_int, C.c_int, dp, dp]
        L.orc_tv.argtypes = [C.c_int, C.c_int, dp]
        L.orc_tv.restype = C.c_double
        L.orc_proj_ball.argtypes = [C.c_size_t, dp, C.c_double, dp]
        L.orc_fgp.argtypes = [C.c_int, C.c_int, dp, C.c_double, C.c_int, C.c_int, dp, dp]
        L.orc_tv_gap.argtypes = [C.c_int, C.c_int, dp, C.c_double, C.c_int, dp, dp]
        L.orc_tv_gap.restype = C.c_double
        L.orc_op_out_size.argtypes = [C.POINTER(OrcOp)]
        L.orc_op_out_size.restype = C.c_size_t
        L.orc_op_apply.argtypes = [C.POINTER(OrcOp), dp, dp]
        L.orc_op_adjoint.argtypes = [C.POINTER(OrcOp), dp, dp]
        L.orc_objective.argtypes = [C.POINTER(OrcOp), dp, dp, C.c_double]
        L.orc_objective.restype = C.c_double
        L.orc_splitmix64_mix.argtypes = [C.c_uint64]
        L.orc_splitmix64_mix.restype = C.c_uint64
        L.orc_coin.argtypes = [C.c_uint64, C.c_uint64, C.c_int64, C.c_double]
        L.orc_coin.restype = C.c_int
        u8p = C.POINTER(C.c_uint8)
        L.orc_proxskip.argtypes = [C.POINTER(OrcOp), dp, dp, dp, dp, C.POINTER(OrcParams), u8p, dp]
        L.orc_proxskip.restype = C.c_int64
        L.orc_pgd.argtypes = [C.POINTER(OrcOp), dp, dp, dp, C.POINTER(OrcParams), dp]
        L.orc_pdhgskip.argtypes = [C.POINTER(OrcOp), dp, dp, dp, dp, dp, C.POINTER(OrcParams), u8p, dp]
        L.orc_pdhgskip.restype = C.c_int64
        L.orc_pdhg.argtypes = [C.POINTER(OrcOp), dp, dp, dp, dp, C.POINTER(OrcParams), dp]
        L.orc_fista.argtypes = [C.POINTER(OrcOp), dp, dp, dp, C.POINTER(OrcParams), dp]
        L.orc_pdhgskip1.argtypes = [C.POINTER(OrcOp), dp, dp, dp, dp, C.POINTER(OrcParams), u8p, dp]
        L.orc_pdhgskip1.restype = C.c_int64
        L.orc_subset.argtypes = [C.c_uint64, C.c_uint64, C.c_int64, C.c_int]
        L.orc_subset.restype = C.c_int
        L.orc_subset_apply.argtypes = [C.POINTER(OrcOp), C.c_int, C.c_int, dp, dp]
        L.orc_subset_adjoint.argtypes = [C.POINTER(OrcOp), C.c_int, C.c_int, dp, dp]
        L.orc_spdhgskip.argtypes = [C.POINTER(OrcOp), dp, C.c_int, dp, dp, dp, dp,
                                    C.POINTER(OrcParams), u8p, C.POINTER(C.c_int32), dp]
        L.orc_spdhgskip.restype = C.c_int64
        L.orc_op_norm.argtypes = [C.POINTER(OrcOp), C.c_int, C.c_uint64]
        L.orc_op_norm.restype = C.c_double
        L.orc_pdhg_explicit.argtypes = [C.POINTER(OrcOp), dp, C.c_double, C.c_int, C.c_int64,
                                        dp, dp, dp, C.c_int64, dp]
        L.orc_dual_rof_proxskip.argtypes = [C.c_int, C.c_int, dp, C.c_double, C.c_double,
                                            C.c_double, C.c_double, C.c_int64, C.c_uint64,
                                            C.c_uint64, C.c_int64, dp, dp, u8p, dp, dp]
        L.orc_dual_rof_proxskip.restype = C.c_int64
        L.orc_dual_rof_projgd.argtypes = [C.c_int, C.c_int, dp, C.c_double, C.c_double,
                                          C.c_double, C.c_int64, dp]
        L.orc_tv_prox_skip.argtypes = [C.c_int, C.c_int, dp, C.c_double, C.c_int, C.c_int,
                                       C.c_double, C.c_uint64, C.c_uint64, C.c_int64, dp, dp, dp]
        L.orc_tv_prox_skip.restype = C.c_int64
        i64p = C.POINTER(C.c_int64)
        L.orc_proxskip_inner.argtypes = [C.POINTER(OrcOp), dp, dp, dp, dp, dp, C.c_double,
                                         C.POINTER(OrcParams), u8p, dp, i64p]
        L.orc_proxskip_inner.restype = C.c_int64
        L.orc_pdhgskip_inner.argtypes = [C.POINTER(OrcOp), dp, dp, dp, dp, dp, dp, C.c_double,
                                         C.POINTER(OrcParams), u8p, dp, i64p]
        L.orc_pdhgskip_inner.restype = C.c_int64
        L.orc_cnn_param_count.argtypes = []
        L.orc_cnn_param_count.restype = C.c_size_t
        L.orc_cnn_forward.argtypes = [C.c_int, C.c_int, C.c_int, dp, dp, C.c_int, dp, dp, dp]
        L.orc_cnn_loss_grad.argtypes = [C.c_int, C.c_int, C.c_int, dp, dp, C.c_int, dp, dp, dp,
                                        C.c_double, dp]
        L.orc_cnn_loss_grad.restype = C.c_double
        L.orc_adam_step.argtypes = [C.c_size_t, dp, dp, dp, dp, C.c_int64, C.c_double,
                                    C.c_double, C.c_double, C.c_double]
        _lib = L
    return _lib


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


# ---------------------------------------------------------------- operators
def grad(u):
    u = _f64(u)
    H, W = u.shape
    q = np.empty((2, H, W))
    lib().orc_grad(H, W, _p(u), _p(q))
    return q


def div(q):
    q = _f64(q)
    _, H, W = q.shape
    u = np.empty((H, W))
    lib().orc_div(H, W, _p(q), _p(u))
    return u


def tv(u):
    u = _f64(u)
    H, W = u.shape
    return lib().orc_tv(H, W, _p(u))


def proj_ball(w, lam):
    w = _f64(w)
    out = np.empty_like(w)
    n = w[0].size
    lib().orc_proj_ball(n, _p(w), float(lam), _p(out))
    return out


def fgp(v, lam, iters, nonneg=0, q=None):
    """TV prox by FGP.  Returns (z, q_new); q (if given) is not modified."""
    v = _f64(v)
    H, W = v.shape
    qq = np.zeros((2, H, W)) if q is None else _f64(q).copy()
    z = np.empty((H, W))
    lib().orc_fgp(H, W, _p(v), float(lam), int(iters), int(nonneg), _p(qq), _p(z))
    return z, qq


def tv_gap(v, lam, q, nonneg=0):
    """(gap, primal) of the TV prox at dual point q."""
    v = _f64(v)
    q = _f64(q)
    H, W = v.shape
    primal = C.c_double(0.0)
    g = lib().orc_tv_gap(H, W, _p(v), float(lam), int(nonneg), _p(q), C.byref(primal))
    return g, primal.value


class Op:
    """Holds an orc_op and the arrays it points to."""

    def __init__(self, kind, H, W, kernel=None, angles=None, n_det=0, pixel=1.0,
                 det_spacing=1.0):
        self.kind, self.H, self.W = kind, H, W
        self._kernel = None if kernel is None else _f64(kernel)
        self._angles = None if angles is None else _f64(angles)
        s = OrcOp()
        s.kind, s.H, s.W = kind, H, W
        if self._kernel is not None:
            s.kernel = _p(self._kernel)
            s.kh, s.kw = self._kernel.shape
        if self._angles is not None:
            s.angles = _p(self._angles)
            s.n_ang = len(self._angles)
        s.n_det = n_det
        s.pixel, s.det_spacing = pixel, det_spacing
        self.s = s
        self.out_shape = (len(self._angles), n_det) if kind == JOSEPH else (H, W)

    def apply(self, x):
        x = _f64(x)
        y = np.empty(self.out_shape)
        lib().orc_op_apply(C.byref(self.s), _p(x), _p(y))
        return y

    def adjoint(self, y):
        y = _f64(y)
        x = np.empty((self.H, self.W))
        lib().orc_op_adjoint(C.byref(self.s), _p(y), _p(x))
        return x

    def norm(self, iters=200, seed=1):
        return lib().orc_op_norm(C.byref(self.s), int(iters), int(seed))


def identity(H, W):
    return Op(IDENTITY, H, W)


def blur(H, W, kernel):
    return Op(BLUR, H, W, kernel=kernel)


def joseph(H, W, angles, n_det, pixel, det_spacing):
    return Op(JOSEPH, H, W, angles=angles, n_det=n_det, pixel=pixel, det_spacing=det_spacing)


def objective(A: Op, b, x, alpha):
    b = _f64(b)
    x = _f64(x)
    return lib().orc_objective(C.byref(A.s), _p(b), _p(x), float(alpha))


# ---------------------------------------------------------------- coin
def mix64(z: int) -> int:
    return lib().orc_splitmix64_mix(z & 0xFFFFFFFFFFFFFFFF)


def coin(seed, stream, k, p) -> int:
    return lib().orc_coin(int(seed), int(stream), int(k), float(p))


# ---------------------------------------------------------------- solvers
def _params(alpha, step, dual_step, p, outer, inner, nonneg, seed, stream, k0):
    P = OrcParams()
    P.alpha, P.step, P.dual_step, P.p = alpha, step, dual_step, p
    P.outer_iters, P.inner_iters, P.nonneg = outer, inner, nonneg
    P.seed, P.stream_id, P.k0 = seed, stream, k0
    return P


def _state(a, shape):
    return np.zeros(shape) if a is None else _f64(a).copy()


def proxskip(A: Op, b, alpha, step, p, outer, inner, nonneg=0, seed=0, stream=0,
             k0=0, x=None, h=None, q=None, want_obj=False):
    """Returns dict(x, h, q, theta, obj, nprox)."""
    b = _f64(b)
    H, W = A.H, A.W
    x, h, q = _state(x, (H, W)), _state(h, (H, W)), _state(q, (2, H, W))
    theta = np.zeros(outer, dtype=np.uint8)
    obj = np.zeros(outer) if want_obj else None
    P = _params(alpha, step, 0.0, p, outer, inner, nonneg, seed, stream, k0)
    n = lib().orc_proxskip(C.byref(A.s), _p(b), _p(x), _p(h), _p(q), C.byref(P),
                           theta.ctypes.data_as(C.POINTER(C.c_uint8)),
                           _p(obj) if want_obj else None)
    return dict(x=x, h=h, q=q, theta=theta, obj=obj, nprox=int(n))


def pgd(A: Op, b, alpha, step, outer, inner, nonneg=0, x=None, q=None, want_obj=False):
    b = _f64(b)
    H, W = A.H, A.W
    x, q = _state(x, (H, W)), _state(q, (2, H, W))
    obj = np.zeros(outer) if want_obj else None
    P = _params(alpha, step, 0.0, 1.0, outer, inner, nonneg, 0, 0, 0)
    lib().orc_pgd(C.byref(A.s), _p(b), _p(x), _p(q), C.byref(P), _p(obj) if want_obj else None)
    return dict(x=x, q=q, obj=obj)


def pdhgskip(A: Op, b, alpha, sigma, tau, p, outer, inner, nonneg=0, seed=0, stream=0,
             k0=0, x=None, h=None, y=None, q=None, want_obj=False):
    b = _f64(b)
    H, W = A.H, A.W
    x, h, q = _state(x, (H, W)), _state(h, (H, W)), _state(q, (2, H, W))
    y = _state(y, A.out_shape)
    theta = np.zeros(outer, dtype=np.uint8)
    obj = np.zeros(outer) if want_obj else None
    P = _params(alpha, sigma, tau, p, outer, inner, nonneg, seed, stream, k0)
    n = lib().orc_pdhgskip(C.byref(A.s), _p(b), _p(x), _p(h), _p(y), _p(q), C.byref(P),
                           theta.ctypes.data_as(C.POINTER(C.c_uint8)),
                           _p(obj) if want_obj else None)
    return dict(x=x, h=h, y=y, q=q, theta=theta, obj=obj, nprox=int(n))


def pdhg(A: Op, b, alpha, sigma, tau, outer, inner, nonneg=0, x=None, y=None, q=None,
         want_obj=False):
    b = _f64(b)
    H, W = A.H, A.W
    x, q = _state(x, (H, W)), _state(q, (2, H, W))
    y = _state(y, A.out_shape)
    obj = np.zeros(outer) if want_obj else None
    P = _params(alpha, sigma, tau, 1.0, outer, inner, nonneg, 0, 0, 0)
    lib().orc_pdhg(C.byref(A.s), _p(b), _p(x), _p(y), _p(q), C.byref(P),
                   _p(obj) if want_obj else None)
    return dict(x=x, y=y, q=q, obj=obj)


def fista(A: Op, b, alpha, step, outer, inner, nonneg=0, x=None, q=None, want_obj=False):
    """Alg. FISTA (Beck-Teboulle momentum) with the FGP prox; the momentum
    restarts at every call.  Returns dict(x, q, obj)."""
    b = _f64(b)
    x, q = _state(x, (A.H, A.W)), _state(q, (2, A.H, A.W))
    obj = np.zeros(outer) if want_obj else None
    P = _params(alpha, step, 0.0, 1.0, outer, inner, nonneg, 0, 0, 0)
    lib().orc_fista(C.byref(A.s), _p(b), _p(x), _p(q), C.byref(P), _p(obj) if want_obj else None)
    return dict(x=x, q=q, obj=obj)


def pdhgskip1(A: Op, b, alpha, sigma, tau, p, outer, inner, nonneg=0, seed=0, stream=0, k0=0,
              x=None, y=None, q=None, want_obj=False):
    """Alg. PDHGSkip-1 (omega + 1 = 1/p).  Returns dict(x, y, q, theta, obj, nprox)."""
    b = _f64(b)
    x, q = _state(x, (A.H, A.W)), _state(q, (2, A.H, A.W))
    y = _state(y, A.out_shape)
    theta = np.zeros(outer, dtype=np.uint8)
    obj = np.zeros(outer) if want_obj else None
    P = _params(alpha, sigma, tau, p, outer, inner, nonneg, seed, stream, k0)
    n = lib().orc_pdhgskip1(C.byref(A.s), _p(b), _p(x), _p(y), _p(q), C.byref(P),
                            theta.ctypes.data_as(C.POINTER(C.c_uint8)),
                            _p(obj) if want_obj else None)
    return dict(x=x, y=y, q=q, theta=theta, obj=obj, nprox=int(n))


def subset(seed, stream, k, n) -> int:
    """Angle subset drawn at outer iteration k (uniform on 0..n-1)."""
    return int(lib().orc_subset(seed & 0xFFFFFFFFFFFFFFFF, stream & 0xFFFFFFFFFFFFFFFF, int(k),
                                int(n)))


def subset_rows(n_ang, n, j):
    """Angle indices of subset j of n (the rows of A_j in order)."""
    return np.arange(j, n_ang, n)


def subset_apply(A: Op, n, j, x):
    x = _f64(x)
    yj = np.empty((len(subset_rows(A.out_shape[0], n, j)), A.out_shape[1]))
    lib().orc_subset_apply(C.byref(A.s), int(n), int(j), _p(x), _p(yj))
    return yj


def subset_adjoint(A: Op, n, j, yj):
    yj = _f64(yj)
    x = np.empty((A.H, A.W))
    lib().orc_subset_adjoint(C.byref(A.s), int(n), int(j), _p(yj), _p(x))
    return x


def spdhgskip(A: Op, b, n_sub, alpha, sigma, tau, p, outer, inner, nonneg=0, seed=0, stream=0,
              k0=0, x=None, h=None, y=None, q=None, want_obj=False):
    """SPDHG over angle subsets with the skipped prox.  Returns dict(x, h, y,
    q, theta, subset, obj, nprox)."""
    b = _f64(b)
    H, W = A.H, A.W
    x, h, q = _state(x, (H, W)), _state(h, (H, W)), _state(q, (2, H, W))
    y = _state(y, A.out_shape)
    theta = np.zeros(outer, dtype=np.uint8)
    sub = np.zeros(outer, dtype=np.int32)
    obj = np.zeros(outer) if want_obj else None
    P = _params(alpha, sigma, tau, p, outer, inner, nonneg, seed, stream, k0)
    n = lib().orc_spdhgskip(C.byref(A.s), _p(b), int(n_sub), _p(x), _p(h), _p(y), _p(q),
                            C.byref(P), theta.ctypes.data_as(C.POINTER(C.c_uint8)),
                            sub.ctypes.data_as(C.POINTER(C.c_int32)),
                            _p(obj) if want_obj else None)
    return dict(x=x, h=h, y=y, q=q, theta=theta, subset=sub, obj=obj, nprox=int(n))


def pdhg_explicit(A: Op, b, alpha, nonneg, iters, x=None, y1=None, y2=None, obj_every=0):
    b = _f64(b)
    H, W = A.H, A.W
    x = _state(x, (H, W))
    y1 = _state(y1, A.out_shape)
    y2 = _state(y2, (2, H, W))
    nrec = iters // obj_every if obj_every > 0 else 0
    obj = np.zeros(max(nrec, 1))
    lib().orc_pdhg_explicit(C.byref(A.s), _p(b), float(alpha), int(nonneg), int(iters),
                            _p(x), _p(y1), _p(y2), int(obj_every), _p(obj))
    return dict(x=x, y1=y1, y2=y2, obj=obj[:nrec])


# ---------------------------------------------------------------- light prox (Sec. 2)
def dual_rof_proxskip(b, alpha, eps, gamma, p, K, seed=0, stream=0, k0=0, q=None, h=None,
                      u_ref=None):
    """ProxSkip on Dual-ROF (eps = 0) / Dual-Huber-ROF.  Returns dict(q, h,
    u = b + div q, theta, nprox, err)."""
    b = _f64(b)
    H, W = b.shape
    q = _state(q, (2, H, W))
    h = _state(h, (2, H, W))
    theta = np.zeros(max(K, 1), dtype=np.uint8)
    err = np.zeros(max(K, 1)) if u_ref is not None else None
    ur = None if u_ref is None else _f64(u_ref)
    n = lib().orc_dual_rof_proxskip(H, W, _p(b), float(alpha), float(eps), float(gamma),
                                    float(p), int(K), int(seed), int(stream), int(k0), _p(q),
                                    _p(h), theta.ctypes.data_as(C.POINTER(C.c_uint8)),
                                    _p(ur) if ur is not None else None,
                                    _p(err) if err is not None else None)
    return dict(q=q, h=h, u=b + div(q), theta=theta[:K], nprox=int(n),
                err=None if err is None else err[:K])


def dual_rof_projgd(b, alpha, eps, gamma, K, q=None):
    b = _f64(b)
    H, W = b.shape
    q = _state(q, (2, H, W))
    lib().orc_dual_rof_projgd(H, W, _p(b), float(alpha), float(eps), float(gamma), int(K), _p(q))
    return dict(q=q, u=b + div(q))


# ---------------------------------------------------------------- inner-solver skip
INNER_STREAM = 1 << 62


def tv_prox_skip(v, lam, iters, p_in, nonneg=0, seed=0, stream=0, k0=0, q=None, h=None):
    """TV prox by ProxSkip on its dual (step 1/8).  Returns dict(z, q, h, nproj)."""
    v = _f64(v)
    H, W = v.shape
    q = _state(q, (2, H, W))
    h = _state(h, (2, H, W))
    z = np.zeros((H, W))
    n = lib().orc_tv_prox_skip(H, W, _p(v), float(lam), int(nonneg), int(iters), float(p_in),
                               int(seed), int(stream), int(k0), _p(q), _p(h), _p(z))
    return dict(z=z, q=q, h=h, nproj=int(n))


def proxskip_inner(A: Op, b, alpha, step, p, outer, inner, p_in, nonneg=0, seed=0, stream=0,
                   k0=0, x=None, h=None, q=None, h_in=None, want_obj=False):
    """ProxSkip with the TV prox by tv_prox_skip.  Returns dict(x, h, q, h_in, theta,
    obj, nprox, nproj)."""
    b = _f64(b)
    H, W = A.H, A.W
    x, h = _state(x, (H, W)), _state(h, (H, W))
    q, h_in = _state(q, (2, H, W)), _state(h_in, (2, H, W))
    theta = np.zeros(outer, dtype=np.uint8)
    obj = np.zeros(outer) if want_obj else None
    nproj = C.c_int64(0)
    P = _params(alpha, step, 0.0, p, outer, inner, nonneg, seed, stream, k0)
    n = lib().orc_proxskip_inner(C.byref(A.s), _p(b), _p(x), _p(h), _p(q), _p(h_in),
                                 float(p_in), C.byref(P),
                                 theta.ctypes.data_as(C.POINTER(C.c_uint8)),
                                 _p(obj) if want_obj else None, C.byref(nproj))
    return dict(x=x, h=h, q=q, h_in=h_in, theta=theta, obj=obj, nprox=int(n),
                nproj=int(nproj.value))


def pdhgskip_inner(A: Op, b, alpha, sigma, tau, p, outer, inner, p_in, nonneg=0, seed=0,
                   stream=0, k0=0, x=None, h=None, y=None, q=None, h_in=None, want_obj=False):
    """PDHGSkip-2 with the TV prox by tv_prox_skip.  Returns dict(x, h, y, q, h_in,
    theta, obj, nprox, nproj)."""
    b = _f64(b)
    H, W = A.H, A.W
    x, h = _state(x, (H, W)), _state(h, (H, W))
    q, h_in = _state(q, (2, H, W)), _state(h_in, (2, H, W))
    y = _state(y, A.out_shape)
    theta = np.zeros(outer, dtype=np.uint8)
    obj = np.zeros(outer) if want_obj else None
    nproj = C.c_int64(0)
    P = _params(alpha, sigma, tau, p, outer, inner, nonneg, seed, stream, k0)
    n = lib().orc_pdhgskip_inner(C.byref(A.s), _p(b), _p(x), _p(h), _p(y), _p(q), _p(h_in),
                                 float(p_in), C.byref(P),
                                 theta.ctypes.data_as(C.POINTER(C.c_uint8)),
                                 _p(obj) if want_obj else None, C.byref(nproj))
    return dict(x=x, h=h, y=y, q=q, h_in=h_in, theta=theta, obj=obj, nprox=int(n),
                nproj=int(nproj.value))


# ---------------------------------------------------------------- learned prox
def cnn_param_count() -> int:
    return int(lib().orc_cnn_param_count())


def _batch(v, lam):
    v = _f64(v)
    if v.ndim == 2:
        v = v[None]
    lam = _f64(np.broadcast_to(np.asarray(lam, dtype=np.float64), (v.shape[0],)))
    return v, lam


def cnn_forward(v, lam, params, nonneg=0):
    """v: [n][H][W] (or [H][W]), lam: scalar or [n].  Returns (qt [n][2][H][W], z [n][H][W])."""
    v, lam = _batch(v, lam)
    n, H, W = v.shape
    params = _f64(params)
    assert params.size == cnn_param_count()
    qt = np.empty((n, 2, H, W))
    z = np.empty((n, H, W))
    lib().orc_cnn_forward(n, H, W, _p(v), _p(lam), int(nonneg), _p(params), _p(qt), _p(z))
    return qt, z


def cnn_loss_grad(v, lam, params, z_target, nonneg=0, want_grad=True, q_target=None, mu=0.0):
    """Returns (loss, grad or None); the dual term needs q_target [n][2][H][W]."""
    v, lam = _batch(v, lam)
    n, H, W = v.shape
    params = _f64(params)
    zt = _f64(z_target).reshape(n, H, W)
    qt = None if q_target is None else _f64(q_target).reshape(n, 2, H, W)
    g = np.empty(params.size) if want_grad else None
    loss = lib().orc_cnn_loss_grad(n, H, W, _p(v), _p(lam), int(nonneg), _p(params), _p(zt),
                                   _p(qt) if qt is not None else None, float(mu),
                                   _p(g) if want_grad else None)
    return loss, g


def adam_step(params, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """In place on params, m, v (float64 arrays)."""
    for a in (params, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    g = _f64(grad)
    lib().orc_adam_step(params.size, _p(params), _p(g), _p(m), _p(v), int(step), float(lr),
                        float(beta1), float(beta2), float(eps))
