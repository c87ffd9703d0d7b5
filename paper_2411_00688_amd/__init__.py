"""ProxSkip / PDHGSkip-2 for TV-regularised imaging on MI355X (gfx950).

Thin Python binding of libtvskip.so: the functions below carry the C ABI's
names (include/tvskip.h) and only marshal arguments (torch device tensors to
raw device pointers, the current torch stream to a HIP stream).  Every step
of the method runs in the library's HIP kernels; there is no CPU fallback,
and the calls raise if the library has not been built.

Handles (contexts, operators) are plain integers (C pointers).
"""
from __future__ import annotations

import ctypes as C

from ._lib import (TVS_F32, TVS_F64, TVS_FLAG_GRAPH, TvsError, check, lib, tvs_batch_params,
                   tvs_dual_rof_params, tvs_params, tvs_report, tvs_slice, tvs_solve_ext,
                   tvs_state)

__all__ = [
    "TVS_F32", "TVS_F64", "TVS_FLAG_GRAPH", "TvsError",
    "tvs_ctx_create", "tvs_ctx_destroy", "tvs_ctx_set_stream", "tvs_sync", "tvs_last_error",
    "tvs_op_identity", "tvs_op_blur_periodic", "tvs_op_ct_joseph", "tvs_op_destroy",
    "tvs_op_out_size", "tvs_op_apply", "tvs_op_adjoint", "tvs_op_norm",
    "tvs_op_joseph_set_groups", "tvs_op_joseph_groups",
    "tvs_grad", "tvs_div", "tvs_tv_prox", "tvs_tv_prox_noalloc", "tvs_tv_gap", "tvs_objective",
    "tvs_coin",
    "tvs_proxskip", "tvs_pdhgskip", "tvs_proxskip_ex", "tvs_pdhgskip_ex",
    "tvs_spdhgskip", "tvs_subset", "tvs_fista", "tvs_pdhgskip1",
    "tvs_dual_rof_proxskip",
    "tvs_fgp_variant_count", "tvs_fgp_variant", "tvs_fgp_set_variant", "tvs_fgp_autotune",
    "tvs_proxskip_batched", "tvs_fgp_set_variant_batched", "tvs_fgp_autotune_batched",
    "tvs_fgp_query", "tvs_fgp_query_batched", "tvs_tune_clear", "tvs_tune_save", "tvs_tune_load",
    "tvs_cnn_create", "tvs_cnn_destroy", "tvs_cnn_param_count", "tvs_cnn_get_params",
    "tvs_cnn_set_params", "tvs_cnn_forward", "tvs_cnn_loss_grad", "tvs_cnn_adam_step",
    "tvs_cnn_train_step", "tvs_cnn_prox", "tvs_cnn_set_fast_forward", "tvs_cnn_save",
    "tvs_cnn_load",
]


def _dtype_code(t) -> int:
    import torch
    if t.dtype == torch.float32:
        return TVS_F32
    if t.dtype == torch.float64:
        return TVS_F64
    raise TypeError(f"tensor dtype must be float32 or float64, got {t.dtype}")


def _ptr(t, numel=None, dtype=None):
    """Device pointer of a contiguous CUDA/HIP tensor (checked)."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("tensors must live on the GPU (torch device 'cuda')")
    if not t.is_contiguous():
        raise ValueError("tensors must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"tensor has {t.numel()} elements, {numel} expected")
    if dtype is not None and _dtype_code(t) != dtype:
        raise TypeError("all tensors of one call must share a dtype")
    return C.c_void_p(t.data_ptr())


def _current_stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


# ---------------------------------------------------------------- context
def tvs_ctx_create(device: int = 0, stream=None) -> int:
    """Context on `device`, bound to `stream` (a torch.cuda.Stream, a raw
    hipStream_t int, or None for torch's current stream)."""
    if stream is None:
        s = _current_stream()
    elif isinstance(stream, int):
        s = C.c_void_p(stream)
    else:
        s = C.c_void_p(stream.cuda_stream)
    out = C.c_void_p()
    check(lib().tvs_ctx_create(int(device), s, C.byref(out)))
    return out.value


def tvs_ctx_destroy(ctx: int) -> None:
    lib().tvs_ctx_destroy(C.c_void_p(ctx))


def tvs_ctx_set_stream(ctx: int, stream=None) -> None:
    s = _current_stream() if stream is None else (
        C.c_void_p(stream) if isinstance(stream, int) else C.c_void_p(stream.cuda_stream))
    check(lib().tvs_ctx_set_stream(C.c_void_p(ctx), s))


def tvs_sync(ctx: int) -> None:
    check(lib().tvs_sync(C.c_void_p(ctx)))


def tvs_last_error() -> str:
    m = lib().tvs_last_error()
    return m.decode() if m else ""


# -------------------------------------------------------------- operators
def tvs_op_identity(ctx: int, H: int, W: int) -> int:
    out = C.c_void_p()
    check(lib().tvs_op_identity(C.c_void_p(ctx), int(H), int(W), C.byref(out)))
    return out.value


def tvs_op_blur_periodic(ctx: int, H: int, W: int, kernel) -> int:
    import numpy as np
    k = np.ascontiguousarray(kernel, dtype=np.float64)
    out = C.c_void_p()
    check(lib().tvs_op_blur_periodic(C.c_void_p(ctx), int(H), int(W),
                                     k.ctypes.data_as(C.POINTER(C.c_double)),
                                     int(k.shape[0]), int(k.shape[1]), C.byref(out)))
    return out.value


def tvs_op_ct_joseph(ctx: int, H: int, W: int, angles, n_det: int, pixel: float,
                     det_spacing: float) -> int:
    import numpy as np
    a = np.ascontiguousarray(angles, dtype=np.float64)
    out = C.c_void_p()
    check(lib().tvs_op_ct_joseph(C.c_void_p(ctx), int(H), int(W), int(a.size),
                                 a.ctypes.data_as(C.POINTER(C.c_double)), int(n_det),
                                 float(pixel), float(det_spacing), C.byref(out)))
    return out.value


def tvs_op_destroy(op: int) -> None:
    lib().tvs_op_destroy(C.c_void_p(op))


def tvs_op_out_size(op: int) -> int:
    return int(lib().tvs_op_out_size(C.c_void_p(op)))


def tvs_op_apply(op: int, x, y) -> None:
    d = _dtype_code(x)
    check(lib().tvs_op_apply(C.c_void_p(op), d, _ptr(x), _ptr(y, tvs_op_out_size(op), d)))


def tvs_op_adjoint(op: int, y, x) -> None:
    d = _dtype_code(y)
    check(lib().tvs_op_adjoint(C.c_void_p(op), d, _ptr(y, tvs_op_out_size(op)), _ptr(x, None, d)))


def tvs_op_joseph_set_groups(op: int, groups: int) -> None:
    check(lib().tvs_op_joseph_set_groups(C.c_void_p(op), int(groups)))


def tvs_op_joseph_groups(op: int) -> int:
    return int(lib().tvs_op_joseph_groups(C.c_void_p(op)))


def tvs_op_norm(op: int, iters: int = 200, seed: int = 1) -> float:
    out = C.c_double()
    check(lib().tvs_op_norm(C.c_void_p(op), int(iters), int(seed), C.byref(out)))
    return out.value


# ------------------------------------------------------ TV building blocks
def tvs_grad(ctx: int, u, q) -> None:
    H, W = u.shape
    d = _dtype_code(u)
    check(lib().tvs_grad(C.c_void_p(ctx), d, H, W, _ptr(u), _ptr(q, 2 * H * W, d)))


def tvs_div(ctx: int, q, u) -> None:
    H, W = u.shape
    d = _dtype_code(q)
    check(lib().tvs_div(C.c_void_p(ctx), d, H, W, _ptr(q, 2 * H * W), _ptr(u, H * W, d)))


def tvs_tv_prox(ctx: int, v, lam: float, inner_iters: int, nonneg: int, q, z,
                want_gap: bool = False):
    """FGP TV prox; q (2,H,W) is the warm dual in and the final dual out.
    Returns the relative duality gap if want_gap, else None."""
    H, W = v.shape
    d = _dtype_code(v)
    g = C.c_double()
    check(lib().tvs_tv_prox(C.c_void_p(ctx), d, H, W, _ptr(v), float(lam), int(inner_iters),
                            int(nonneg), _ptr(q, 2 * H * W, d), _ptr(z, H * W, d),
                            C.byref(g) if want_gap else None))
    return g.value if want_gap else None


def tvs_tv_prox_noalloc(ctx: int, v, lam: float, inner_iters: int, nonneg: int, q, z):
    """tvs_tv_prox on the library's static device array (allocates nothing;
    calls overlapping on one device race).  q is the warm dual in and the
    final dual out."""
    H, W = v.shape
    d = _dtype_code(v)
    check(lib().tvs_tv_prox_noalloc(C.c_void_p(ctx), d, H, W, _ptr(v), float(lam),
                                    int(inner_iters), int(nonneg), _ptr(q, 2 * H * W, d),
                                    _ptr(z, H * W, d)))


def tvs_tv_gap(ctx: int, v, lam: float, nonneg: int, q):
    H, W = v.shape
    d = _dtype_code(v)
    gap, primal = C.c_double(), C.c_double()
    check(lib().tvs_tv_gap(C.c_void_p(ctx), d, H, W, _ptr(v), float(lam), int(nonneg),
                           _ptr(q, 2 * H * W, d), C.byref(gap), C.byref(primal)))
    return gap.value, primal.value


def tvs_objective(op: int, b, x, alpha: float) -> float:
    d = _dtype_code(x)
    out = C.c_double()
    check(lib().tvs_objective(C.c_void_p(op), d, _ptr(b, tvs_op_out_size(op), d), _ptr(x),
                              float(alpha), C.byref(out)))
    return out.value


def tvs_coin(seed: int, stream_id: int, k: int, p: float) -> int:
    return int(lib().tvs_coin(int(seed), int(stream_id), int(k), float(p)))


def tvs_subset(seed: int, stream_id: int, k: int, n: int) -> int:
    return int(lib().tvs_subset(int(seed), int(stream_id), int(k), int(n)))


# ---------------------------------------------------------------- solvers
def _solve(fn, op, b, x, h, q, y, alpha, step, dual_step, p, outer_iters, inner_iters, nonneg,
           seed, stream_id, k0, graph, want_obj, want_theta, ext=None):
    import numpy as np
    d = _dtype_code(x)
    n = x.numel()
    st = tvs_state(_ptr(x), _ptr(h, n, d), _ptr(q, 2 * n, d),
                   _ptr(y, tvs_op_out_size(op), d) if y is not None else None)
    P = tvs_params(alpha=float(alpha), step=float(step), dual_step=float(dual_step), p=float(p),
                   outer_iters=int(outer_iters), inner_iters=int(inner_iters),
                   nonneg=int(nonneg), seed=int(seed), stream_id=int(stream_id), k0=int(k0),
                   flags=TVS_FLAG_GRAPH if graph else 0, reserved=0)
    rep = tvs_report()
    obj = np.zeros(max(int(outer_iters), 1)) if want_obj else None
    th = np.zeros(max(int(outer_iters), 1), dtype=np.uint8) if want_theta else None
    args = [C.c_void_p(op), d, _ptr(b, tvs_op_out_size(op), d), C.byref(st), C.byref(P)]
    if ext is not None:
        args.append(C.byref(ext))
    check(fn(*args, obj.ctypes.data_as(C.POINTER(C.c_double)) if want_obj else None,
             th.ctypes.data_as(C.POINTER(C.c_uint8)) if want_theta else None, C.byref(rep)))
    out = dict(n_prox=rep.n_prox, iters=rep.iters,
               obj=obj[:outer_iters] if want_obj else None,
               theta=th[:outer_iters] if want_theta else None)
    if ext is not None:
        out.update(n_fallback=ext.n_fallback, n_recorded=ext.n_recorded,
                   n_inner_proj=ext.n_inner_proj)
    return out


def _ext(cnn, gap_tol, v_record, inner_p=0.0, inner_h=None, x=None):
    e = tvs_solve_ext()
    e.cnn = C.c_void_p(cnn) if cnn else None
    e.gap_tol = float(gap_tol)
    if v_record is not None:
        e.v_record = _ptr(v_record)
        e.max_record = int(v_record.shape[0])
    e.inner_p = float(inner_p)
    if inner_h is not None:
        e.inner_h = _ptr(inner_h, 2 * x.numel(), _dtype_code(x))
    return e


def tvs_proxskip(op: int, b, x, h, q, alpha, step, p, outer_iters, inner_iters, nonneg=0,
                 seed=0, stream_id=0, k0=0, graph=False, want_obj=False, want_theta=False):
    """ProxSkip in place on (x, h, q).  Returns dict(n_prox, iters, obj, theta)."""
    return _solve(lib().tvs_proxskip, op, b, x, h, q, None, alpha, step, 0.0, p, outer_iters,
                  inner_iters, nonneg, seed, stream_id, k0, graph, want_obj, want_theta)


def tvs_pdhgskip(op: int, b, x, h, q, y, alpha, sigma, tau, p, outer_iters, inner_iters,
                 nonneg=0, seed=0, stream_id=0, k0=0, graph=False, want_obj=False,
                 want_theta=False):
    """PDHGSkip-2 in place on (x, h, q, y).  Returns dict(n_prox, iters, obj, theta)."""
    return _solve(lib().tvs_pdhgskip, op, b, x, h, q, y, alpha, sigma, tau, p, outer_iters,
                  inner_iters, nonneg, seed, stream_id, k0, graph, want_obj, want_theta)


def tvs_fista(op: int, b, x, q, alpha, step, outer_iters, inner_iters, nonneg=0, graph=False,
              want_obj=False):
    """FISTA with the FGP prox (momentum restarted per call), in place on
    (x, q).  Returns dict(n_prox, iters, obj)."""
    import numpy as np
    d = _dtype_code(x)
    n = x.numel()
    st = tvs_state(_ptr(x), None, _ptr(q, 2 * n, d), None)
    P = tvs_params(alpha=float(alpha), step=float(step), dual_step=0.0, p=1.0,
                   outer_iters=int(outer_iters), inner_iters=int(inner_iters),
                   nonneg=int(nonneg), seed=0, stream_id=0, k0=0,
                   flags=TVS_FLAG_GRAPH if graph else 0, reserved=0)
    rep = tvs_report()
    obj = np.zeros(max(int(outer_iters), 1)) if want_obj else None
    check(lib().tvs_fista(C.c_void_p(op), d, _ptr(b, tvs_op_out_size(op), d), C.byref(st),
                          C.byref(P), obj.ctypes.data_as(C.POINTER(C.c_double)) if want_obj else None,
                          C.byref(rep)))
    return dict(n_prox=rep.n_prox, iters=rep.iters, obj=obj[:outer_iters] if want_obj else None)


def tvs_pdhgskip1(op: int, b, x, q, y, alpha, sigma, tau, p, outer_iters, inner_iters, nonneg=0,
                  seed=0, stream_id=0, k0=0, graph=False, want_obj=False, want_theta=False):
    """PDHGSkip-1 (omega + 1 = 1/p) in place on (x, q, y).  Returns dict(n_prox,
    iters, obj, theta)."""
    import numpy as np
    d = _dtype_code(x)
    n = x.numel()
    st = tvs_state(_ptr(x), None, _ptr(q, 2 * n, d), _ptr(y, tvs_op_out_size(op), d))
    P = tvs_params(alpha=float(alpha), step=float(sigma), dual_step=float(tau), p=float(p),
                   outer_iters=int(outer_iters), inner_iters=int(inner_iters),
                   nonneg=int(nonneg), seed=int(seed), stream_id=int(stream_id), k0=int(k0),
                   flags=TVS_FLAG_GRAPH if graph else 0, reserved=0)
    rep = tvs_report()
    K = max(int(outer_iters), 1)
    obj = np.zeros(K) if want_obj else None
    th = np.zeros(K, dtype=np.uint8) if want_theta else None
    check(lib().tvs_pdhgskip1(C.c_void_p(op), d, _ptr(b, tvs_op_out_size(op), d), C.byref(st),
                              C.byref(P), obj.ctypes.data_as(C.POINTER(C.c_double)) if want_obj else None,
                              th.ctypes.data_as(C.POINTER(C.c_uint8)) if want_theta else None,
                              C.byref(rep)))
    return dict(n_prox=rep.n_prox, iters=rep.iters, obj=obj[:outer_iters] if want_obj else None,
                theta=th[:outer_iters] if want_theta else None)


def tvs_spdhgskip(op: int, b, x, h, q, y, n_subsets, alpha, sigma, tau, p, outer_iters,
                  inner_iters, nonneg=0, seed=0, stream_id=0, k0=0, graph=False, want_obj=False,
                  want_theta=False, want_subsets=False):
    """Stochastic angle subsets with the skipped prox, in place on (x, h, q,
    y).  Returns dict(n_prox, iters, obj, theta, subsets)."""
    import numpy as np
    d = _dtype_code(x)
    n = x.numel()
    st = tvs_state(_ptr(x), _ptr(h, n, d), _ptr(q, 2 * n, d), _ptr(y, tvs_op_out_size(op), d))
    P = tvs_params(alpha=float(alpha), step=float(sigma), dual_step=float(tau), p=float(p),
                   outer_iters=int(outer_iters), inner_iters=int(inner_iters),
                   nonneg=int(nonneg), seed=int(seed), stream_id=int(stream_id), k0=int(k0),
                   flags=TVS_FLAG_GRAPH if graph else 0, reserved=0)
    rep = tvs_report()
    K = max(int(outer_iters), 1)
    obj = np.zeros(K) if want_obj else None
    th = np.zeros(K, dtype=np.uint8) if want_theta else None
    sub = np.zeros(K, dtype=np.int32) if want_subsets else None
    check(lib().tvs_spdhgskip(C.c_void_p(op), d, _ptr(b, tvs_op_out_size(op), d), C.byref(st),
                              C.byref(P), int(n_subsets),
                              obj.ctypes.data_as(C.POINTER(C.c_double)) if want_obj else None,
                              th.ctypes.data_as(C.POINTER(C.c_uint8)) if want_theta else None,
                              sub.ctypes.data_as(C.POINTER(C.c_int32)) if want_subsets else None,
                              C.byref(rep)))
    return dict(n_prox=rep.n_prox, iters=rep.iters,
                obj=obj[:outer_iters] if want_obj else None,
                theta=th[:outer_iters] if want_theta else None,
                subsets=sub[:outer_iters] if want_subsets else None)


def tvs_proxskip_ex(op: int, b, x, h, q, alpha, step, p, outer_iters, inner_iters, nonneg=0,
                    seed=0, stream_id=0, k0=0, graph=False, want_obj=False, want_theta=False,
                    cnn=None, gap_tol=1e-3, v_record=None, inner_p=0.0, inner_h=None):
    """tvs_proxskip with the learned prox (cnn), the skipping inner solver
    (inner_p > 0 with its control variate inner_h, a (2, H, W) tensor kept
    across runs) and / or prox-input recording (v_record: (max_record, H, W)
    tensor).  Adds n_fallback, n_recorded, n_inner_proj."""
    return _solve(lib().tvs_proxskip_ex, op, b, x, h, q, None, alpha, step, 0.0, p, outer_iters,
                  inner_iters, nonneg, seed, stream_id, k0, graph, want_obj, want_theta,
                  ext=_ext(cnn, gap_tol, v_record, inner_p, inner_h, x))


def tvs_pdhgskip_ex(op: int, b, x, h, q, y, alpha, sigma, tau, p, outer_iters, inner_iters,
                    nonneg=0, seed=0, stream_id=0, k0=0, graph=False, want_obj=False,
                    want_theta=False, cnn=None, gap_tol=1e-3, v_record=None, inner_p=0.0,
                    inner_h=None):
    """tvs_pdhgskip with the same extensions as tvs_proxskip_ex."""
    return _solve(lib().tvs_pdhgskip_ex, op, b, x, h, q, y, alpha, sigma, tau, p, outer_iters,
                  inner_iters, nonneg, seed, stream_id, k0, graph, want_obj, want_theta,
                  ext=_ext(cnn, gap_tol, v_record, inner_p, inner_h, x))


# ------------------------------------------------------------- FGP tuning
def tvs_fgp_variant_count() -> int:
    return int(lib().tvs_fgp_variant_count())


def tvs_fgp_variant(index: int):
    tw, th, ts = C.c_int(), C.c_int(), C.c_int()
    check(lib().tvs_fgp_variant(int(index), C.byref(tw), C.byref(th), C.byref(ts)))
    return tw.value, th.value, ts.value


def tvs_fgp_set_variant(ctx: int, dtype: int, H: int, W: int, index: int) -> None:
    check(lib().tvs_fgp_set_variant(C.c_void_p(ctx), int(dtype), int(H), int(W), int(index)))


def tvs_fgp_autotune(ctx: int, dtype: int, H: int, W: int, inner_iters: int = 50, reps: int = 3):
    """Times every FGP tile variant; keeps the fastest for (H, W, dtype) in the
    context.  Returns (best_index, [ms per FGP iteration per variant])."""
    import numpy as np
    n = tvs_fgp_variant_count()
    ms = np.zeros(n)
    best = C.c_int()
    check(lib().tvs_fgp_autotune(C.c_void_p(ctx), int(dtype), int(H), int(W), int(inner_iters),
                                 int(reps), C.byref(best), ms.ctypes.data_as(C.POINTER(C.c_double))))
    return best.value, ms.tolist()


def tvs_fgp_query(ctx: int, dtype: int, H: int, W: int):
    """(variant index, measured ms per FGP iteration or -1) an H x W prox uses."""
    idx, ms = C.c_int(), C.c_double()
    check(lib().tvs_fgp_query(C.c_void_p(ctx), int(dtype), int(H), int(W), C.byref(idx),
                              C.byref(ms)))
    return idx.value, ms.value


def tvs_tune_clear(ctx: int) -> None:
    check(lib().tvs_tune_clear(C.c_void_p(ctx)))


def tvs_tune_save(ctx: int, path: str) -> None:
    check(lib().tvs_tune_save(C.c_void_p(ctx), str(path).encode()))


def tvs_tune_load(ctx: int, path: str) -> None:
    check(lib().tvs_tune_load(C.c_void_p(ctx), str(path).encode()))


# ------------------------------------------------------------ light prox (Sec. 2)
def tvs_dual_rof_proxskip(ctx: int, b, q, h, alpha, eps, step, p, outer_iters, seed=0,
                          stream_id=0, k0=0, graph=False, want_theta=False):
    """ProxSkip on Dual-ROF (eps = 0) / Dual-Huber-ROF in place on q, h
    ((2, H, W)).  Returns dict(n_prox, theta)."""
    import numpy as np
    H, W = b.shape
    d = _dtype_code(b)
    P = tvs_dual_rof_params(alpha=float(alpha), eps=float(eps), step=float(step), p=float(p),
                            outer_iters=int(outer_iters), seed=int(seed),
                            stream_id=int(stream_id), k0=int(k0),
                            flags=TVS_FLAG_GRAPH if graph else 0, reserved=0)
    th = np.zeros(max(int(outer_iters), 1), dtype=np.uint8) if want_theta else None
    n = C.c_int64()
    check(lib().tvs_dual_rof_proxskip(C.c_void_p(ctx), d, H, W, _ptr(b), _ptr(q, 2 * H * W, d),
                                      _ptr(h, 2 * H * W, d), C.byref(P),
                                      th.ctypes.data_as(C.POINTER(C.c_uint8)) if want_theta
                                      else None, C.byref(n)))
    return dict(n_prox=n.value, theta=th[:outer_iters] if want_theta else None)


# ------------------------------------------------------------ batched form
def _slice_array(slices):
    n = len(slices)
    arr = (tvs_slice * n)()
    for i, sl in enumerate(slices):
        arr[i] = tvs_slice(int(sl["H"]), int(sl["W"]), int(sl.get("offset", 0)),
                           float(sl["alpha"]), float(sl["p"]), int(sl.get("seed", 0)),
                           int(sl.get("stream_id", 0)))
    return arr
def tvs_proxskip_batched(ctx: int, slices, b_pool, x_pool, h_pool, q_pool, step, outer_iters,
                         inner_iters, nonneg=0, k0=0, graph=False, fgp_variant=-1):
    """Batched ProxSkip (A = I) in place on the pools.  `slices`: sequence of
    dicts with H, W, offset, alpha, p, seed, stream_id.  Returns the prox
    count per slice (numpy int64)."""
    import numpy as np
    n = len(slices)
    arr = (tvs_slice * n)()
    total = 0
    for i, sl in enumerate(slices):
        arr[i] = tvs_slice(int(sl["H"]), int(sl["W"]), int(sl["offset"]), float(sl["alpha"]),
                           float(sl["p"]), int(sl["seed"]), int(sl["stream_id"]))
        total = max(total, int(sl["offset"]) + int(sl["H"]) * int(sl["W"]))
    d = _dtype_code(x_pool)
    for t, need in ((b_pool, total), (x_pool, total), (h_pool, total), (q_pool, 2 * total)):
        if t.numel() < need:
            raise ValueError(f"pool has {t.numel()} elements, {need} needed")
        _ptr(t, None, d)
    P = tvs_batch_params(step=float(step), outer_iters=int(outer_iters),
                         inner_iters=int(inner_iters), nonneg=int(nonneg), k0=int(k0),
                         flags=TVS_FLAG_GRAPH if graph else 0, fgp_variant=int(fgp_variant))
    nprox = np.zeros(n, dtype=np.int64)
    check(lib().tvs_proxskip_batched(C.c_void_p(ctx), d, n, arr, _ptr(b_pool), _ptr(x_pool),
                                     _ptr(h_pool), _ptr(q_pool), C.byref(P),
                                     nprox.ctypes.data_as(C.POINTER(C.c_int64))))
    return nprox


def tvs_fgp_set_variant_batched(ctx: int, dtype: int, n_slices: int, index: int) -> None:
    check(lib().tvs_fgp_set_variant_batched(C.c_void_p(ctx), int(dtype), int(n_slices), int(index)))


def tvs_fgp_autotune_batched(ctx: int, dtype: int, slices, inner_iters: int = 50, reps: int = 2):
    """Times every FGP variant on the passes a run of these slices makes at
    its first 8 outer iterations (the slices whose coin is 1 there); keeps
    the fastest for len(slices) slices.  Returns (best_index, [ms per iter])."""
    import numpy as np
    ms = np.zeros(tvs_fgp_variant_count())
    best = C.c_int()
    check(lib().tvs_fgp_autotune_batched(C.c_void_p(ctx), int(dtype), len(slices),
                                         _slice_array(slices), int(inner_iters), int(reps),
                                         C.byref(best), ms.ctypes.data_as(C.POINTER(C.c_double))))
    return best.value, ms.tolist()


def tvs_fgp_query_batched(ctx: int, dtype: int, n_slices: int):
    idx, ms = C.c_int(), C.c_double()
    check(lib().tvs_fgp_query_batched(C.c_void_p(ctx), int(dtype), int(n_slices), C.byref(idx),
                                      C.byref(ms)))
    return idx.value, ms.value


# ---------------------------------------------------------------- learned prox
def _lam_array(lam, n):
    try:
        vals = [float(x) for x in lam]
    except TypeError:
        vals = [float(lam)] * n
    if len(vals) != n:
        raise ValueError(f"{len(vals)} lam values for a batch of {n}")
    return (C.c_double * n)(*vals)


def _batch_shape(v):
    if v.dim() == 2:
        return 1, v.shape[0], v.shape[1]
    if v.dim() == 3:
        return v.shape[0], v.shape[1], v.shape[2]
    raise ValueError("v must be (H, W) or (n, H, W)")


def _f32(t):
    import torch
    if t is not None and t.dtype != torch.float32:
        raise TypeError("the learned prox works on float32 tensors")
    return t


def tvs_cnn_param_count() -> int:
    return int(lib().tvs_cnn_param_count())


def tvs_cnn_create(ctx: int, seed: int = 0) -> int:
    out = C.c_void_p()
    check(lib().tvs_cnn_create(C.c_void_p(ctx), int(seed), C.byref(out)))
    return out.value


def tvs_cnn_destroy(cnn: int) -> None:
    lib().tvs_cnn_destroy(C.c_void_p(cnn))


def tvs_cnn_get_params(cnn: int):
    import numpy as np
    p = np.empty(tvs_cnn_param_count(), dtype=np.float32)
    check(lib().tvs_cnn_get_params(C.c_void_p(cnn), C.c_void_p(p.ctypes.data)))
    return p


def tvs_cnn_set_params(cnn: int, params) -> None:
    import numpy as np
    p = np.ascontiguousarray(params, dtype=np.float32)
    if p.size != tvs_cnn_param_count():
        raise ValueError(f"{p.size} parameters, {tvs_cnn_param_count()} expected")
    check(lib().tvs_cnn_set_params(C.c_void_p(cnn), C.c_void_p(p.ctypes.data)))


def tvs_cnn_forward(cnn: int, v, lam, nonneg: int = 0, qt=None, z=None) -> None:
    """v (n,H,W) or (H,W) float32; lam scalar or n values; fills qt (n,2,H,W)
    and/or z (same shape as v)."""
    n, H, W = _batch_shape(_f32(v))
    check(lib().tvs_cnn_forward(C.c_void_p(cnn), n, H, W, _ptr(v), _lam_array(lam, n),
                                int(nonneg), _ptr(_f32(qt), 2 * n * H * W),
                                _ptr(_f32(z), n * H * W)))


def tvs_cnn_loss_grad(cnn: int, v, lam, z_target, nonneg: int = 0, grad=None, q_target=None,
                      mu: float = 0.0) -> float:
    n, H, W = _batch_shape(_f32(v))
    loss = C.c_double()
    check(lib().tvs_cnn_loss_grad(C.c_void_p(cnn), n, H, W, _ptr(v), _lam_array(lam, n),
                                  int(nonneg), _ptr(_f32(z_target), n * H * W),
                                  _ptr(_f32(q_target), 2 * n * H * W), float(mu), C.byref(loss),
                                  _ptr(_f32(grad), tvs_cnn_param_count())))
    return loss.value


def tvs_cnn_adam_step(cnn: int, lr: float, grad=None) -> None:
    check(lib().tvs_cnn_adam_step(C.c_void_p(cnn), _ptr(_f32(grad), tvs_cnn_param_count()),
                                  float(lr)))


def tvs_cnn_train_step(cnn: int, v, lam, z_target, lr: float, nonneg: int = 0,
                       want_loss: bool = True, q_target=None, mu: float = 0.0):
    n, H, W = _batch_shape(_f32(v))
    loss = C.c_double()
    check(lib().tvs_cnn_train_step(C.c_void_p(cnn), n, H, W, _ptr(v), _lam_array(lam, n),
                                   int(nonneg), _ptr(_f32(z_target), n * H * W),
                                   _ptr(_f32(q_target), 2 * n * H * W), float(mu), float(lr),
                                   C.byref(loss) if want_loss else None))
    return loss.value if want_loss else None


def tvs_cnn_prox(cnn: int, v, lam: float, nonneg: int, gap_tol: float, fallback_iters: int,
                 q, z):
    """Gap-gated learned prox of one image.  Returns (fell_back, rel_gap)."""
    H, W = _f32(v).shape
    fb = C.c_int()
    rg = C.c_double()
    check(lib().tvs_cnn_prox(C.c_void_p(cnn), H, W, _ptr(v), float(lam), int(nonneg),
                             float(gap_tol), int(fallback_iters), _ptr(_f32(q), 2 * H * W),
                             _ptr(_f32(z), H * W), C.byref(fb), C.byref(rg)))
    return bool(fb.value), rg.value


def tvs_cnn_set_fast_forward(cnn: int, fast: bool) -> None:
    check(lib().tvs_cnn_set_fast_forward(C.c_void_p(cnn), int(bool(fast))))


def tvs_cnn_save(cnn: int, path: str) -> None:
    check(lib().tvs_cnn_save(C.c_void_p(cnn), str(path).encode()))


def tvs_cnn_load(cnn: int, path: str) -> None:
    check(lib().tvs_cnn_load(C.c_void_p(cnn), str(path).encode()))
