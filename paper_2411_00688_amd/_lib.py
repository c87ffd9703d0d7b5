"""ctypes declarations of libtvskip.so (the C ABI in include/tvskip.h).

Argument marshalling only: every computation happens in the HIP library.
Loading fails loudly if the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtvskip.so")

TVS_OK = 0
STATUS_NAMES = {0: "TVS_OK", 1: "TVS_ERR_INVALID_ARG", 2: "TVS_ERR_SHAPE", 3: "TVS_ERR_DEVICE",
                4: "TVS_ERR_OOM", 5: "TVS_ERR_NONFINITE", 6: "TVS_ERR_UNSUPPORTED"}
TVS_F32, TVS_F64 = 0, 1
TVS_FLAG_GRAPH = 1


class TvsError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class tvs_params(C.Structure):
    _fields_ = [("alpha", C.c_double), ("step", C.c_double), ("dual_step", C.c_double),
                ("p", C.c_double), ("outer_iters", C.c_int64), ("inner_iters", C.c_int32),
                ("nonneg", C.c_int32), ("seed", C.c_uint64), ("stream_id", C.c_uint64),
                ("k0", C.c_int64), ("flags", C.c_int32), ("reserved", C.c_int32)]


class tvs_state(C.Structure):
    _fields_ = [("x", C.c_void_p), ("h", C.c_void_p), ("q", C.c_void_p), ("y", C.c_void_p)]


class tvs_report(C.Structure):
    _fields_ = [("n_prox", C.c_int64), ("iters", C.c_int64)]


class tvs_slice(C.Structure):
    _fields_ = [("H", C.c_int32), ("W", C.c_int32), ("offset", C.c_int64), ("alpha", C.c_double),
                ("p", C.c_double), ("seed", C.c_uint64), ("stream_id", C.c_uint64)]


class tvs_dual_rof_params(C.Structure):
    _fields_ = [("alpha", C.c_double), ("eps", C.c_double), ("step", C.c_double),
                ("p", C.c_double), ("outer_iters", C.c_int64), ("seed", C.c_uint64),
                ("stream_id", C.c_uint64), ("k0", C.c_int64), ("flags", C.c_int32),
                ("reserved", C.c_int32)]


class tvs_solve_ext(C.Structure):
    _fields_ = [("cnn", C.c_void_p), ("gap_tol", C.c_double), ("v_record", C.c_void_p),
                ("max_record", C.c_int64), ("n_fallback", C.c_int64), ("n_recorded", C.c_int64),
                ("inner_p", C.c_double), ("inner_h", C.c_void_p), ("n_inner_proj", C.c_int64)]


class tvs_batch_params(C.Structure):
    _fields_ = [("step", C.c_double), ("outer_iters", C.c_int64), ("inner_iters", C.c_int32),
                ("nonneg", C.c_int32), ("k0", C.c_int64), ("flags", C.c_int32),
                ("fgp_variant", C.c_int32)]


_lib = None

vp = C.c_void_p
dp = C.POINTER(C.c_double)
ip = C.POINTER(C.c_int)

# name: (restype, argtypes)
PROTOTYPES = {
    "tvs_ctx_create": (C.c_int, [C.c_int, vp, C.POINTER(vp)]),
    "tvs_ctx_destroy": (None, [vp]),
    "tvs_ctx_set_stream": (C.c_int, [vp, vp]),
    "tvs_last_error": (C.c_char_p, []),
    "tvs_sync": (C.c_int, [vp]),
    "tvs_op_identity": (C.c_int, [vp, C.c_int, C.c_int, C.POINTER(vp)]),
    "tvs_op_blur_periodic": (C.c_int, [vp, C.c_int, C.c_int, dp, C.c_int, C.c_int, C.POINTER(vp)]),
    "tvs_op_ct_joseph": (C.c_int, [vp, C.c_int, C.c_int, C.c_int, dp, C.c_int, C.c_double,
                                   C.c_double, C.POINTER(vp)]),
    "tvs_op_destroy": (None, [vp]),
    "tvs_op_out_size": (C.c_size_t, [vp]),
    "tvs_op_joseph_set_groups": (C.c_int, [vp, C.c_int]),
    "tvs_op_joseph_groups": (C.c_int, [vp]),
    "tvs_op_apply": (C.c_int, [vp, C.c_int, vp, vp]),
    "tvs_op_adjoint": (C.c_int, [vp, C.c_int, vp, vp]),
    "tvs_op_norm": (C.c_int, [vp, C.c_int, C.c_uint64, dp]),
    "tvs_grad": (C.c_int, [vp, C.c_int, C.c_int, C.c_int, vp, vp]),
    "tvs_div": (C.c_int, [vp, C.c_int, C.c_int, C.c_int, vp, vp]),
    "tvs_tv_prox": (C.c_int, [vp, C.c_int, C.c_int, C.c_int, vp, C.c_double, C.c_int, C.c_int,
                              vp, vp, dp]),
    "tvs_tv_prox_noalloc": (C.c_int, [vp, C.c_int, C.c_int, C.c_int, vp, C.c_double, C.c_int,
                                      C.c_int, vp, vp]),
    "tvs_tv_gap": (C.c_int, [vp, C.c_int, C.c_int, C.c_int, vp, C.c_double, C.c_int, vp, dp, dp]),
    "tvs_objective": (C.c_int, [vp, C.c_int, vp, vp, C.c_double, dp]),
    "tvs_coin": (C.c_int, [C.c_uint64, C.c_uint64, C.c_int64, C.c_double]),
    "tvs_subset": (C.c_int, [C.c_uint64, C.c_uint64, C.c_int64, C.c_int]),
    "tvs_fista": (C.c_int, [vp, C.c_int, vp, C.POINTER(tvs_state), C.POINTER(tvs_params), dp,
                            C.POINTER(tvs_report)]),
    "tvs_pdhgskip1": (C.c_int, [vp, C.c_int, vp, C.POINTER(tvs_state), C.POINTER(tvs_params), dp,
                                C.POINTER(C.c_uint8), C.POINTER(tvs_report)]),
    "tvs_spdhgskip": (C.c_int, [vp, C.c_int, vp, C.POINTER(tvs_state), C.POINTER(tvs_params),
                                C.c_int, dp, C.POINTER(C.c_uint8), C.POINTER(C.c_int32),
                                C.POINTER(tvs_report)]),
    "tvs_proxskip": (C.c_int, [vp, C.c_int, vp, C.POINTER(tvs_state), C.POINTER(tvs_params), dp,
                               C.POINTER(C.c_uint8), C.POINTER(tvs_report)]),
    "tvs_pdhgskip": (C.c_int, [vp, C.c_int, vp, C.POINTER(tvs_state), C.POINTER(tvs_params), dp,
                               C.POINTER(C.c_uint8), C.POINTER(tvs_report)]),
    "tvs_proxskip_ex": (C.c_int, [vp, C.c_int, vp, C.POINTER(tvs_state), C.POINTER(tvs_params),
                                  C.POINTER(tvs_solve_ext), dp, C.POINTER(C.c_uint8),
                                  C.POINTER(tvs_report)]),
    "tvs_pdhgskip_ex": (C.c_int, [vp, C.c_int, vp, C.POINTER(tvs_state), C.POINTER(tvs_params),
                                  C.POINTER(tvs_solve_ext), dp, C.POINTER(C.c_uint8),
                                  C.POINTER(tvs_report)]),
    "tvs_dual_rof_proxskip": (C.c_int, [vp, C.c_int, C.c_int, C.c_int, vp, vp, vp,
                                        C.POINTER(tvs_dual_rof_params), C.POINTER(C.c_uint8),
                                        C.POINTER(C.c_int64)]),
    "tvs_fgp_variant_count": (C.c_int, []),
    "tvs_fgp_variant": (C.c_int, [C.c_int, ip, ip, ip]),
    "tvs_fgp_set_variant": (C.c_int, [vp, C.c_int, C.c_int, C.c_int, C.c_int]),
    "tvs_fgp_autotune": (C.c_int, [vp, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, ip, dp]),
    "tvs_proxskip_batched": (C.c_int, [vp, C.c_int, C.c_int, C.POINTER(tvs_slice), vp, vp, vp, vp,
                                       C.POINTER(tvs_batch_params), C.POINTER(C.c_int64)]),
    "tvs_fgp_set_variant_batched": (C.c_int, [vp, C.c_int, C.c_int, C.c_int]),
    "tvs_fgp_autotune_batched": (C.c_int, [vp, C.c_int, C.c_int, C.POINTER(tvs_slice), C.c_int,
                                           C.c_int, ip, dp]),
    "tvs_fgp_query": (C.c_int, [vp, C.c_int, C.c_int, C.c_int, ip, dp]),
    "tvs_fgp_query_batched": (C.c_int, [vp, C.c_int, C.c_int, ip, dp]),
    "tvs_tune_clear": (C.c_int, [vp]),
    "tvs_tune_save": (C.c_int, [vp, C.c_char_p]),
    "tvs_tune_load": (C.c_int, [vp, C.c_char_p]),
    "tvs_cnn_create": (C.c_int, [vp, C.c_uint64, C.POINTER(vp)]),
    "tvs_cnn_destroy": (None, [vp]),
    "tvs_cnn_param_count": (C.c_int64, []),
    "tvs_cnn_get_params": (C.c_int, [vp, vp]),
    "tvs_cnn_set_params": (C.c_int, [vp, vp]),
    "tvs_cnn_forward": (C.c_int, [vp, C.c_int, C.c_int, C.c_int, vp, dp, C.c_int, vp, vp]),
    "tvs_cnn_loss_grad": (C.c_int, [vp, C.c_int, C.c_int, C.c_int, vp, dp, C.c_int, vp, vp,
                                    C.c_double, dp, vp]),
    "tvs_cnn_adam_step": (C.c_int, [vp, vp, C.c_double]),
    "tvs_cnn_train_step": (C.c_int, [vp, C.c_int, C.c_int, C.c_int, vp, dp, C.c_int, vp, vp,
                                     C.c_double, C.c_double, dp]),
    "tvs_cnn_prox": (C.c_int, [vp, C.c_int, C.c_int, vp, C.c_double, C.c_int, C.c_double,
                               C.c_int, vp, vp, ip, dp]),
    "tvs_cnn_set_fast_forward": (C.c_int, [vp, C.c_int]),
    "tvs_cnn_save": (C.c_int, [vp, C.c_char_p]),
    "tvs_cnn_load": (C.c_int, [vp, C.c_char_p]),
}


def lib() -> C.CDLL:
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build it with `python -m paper_2411_00688_amd.build` "
                f"(hipcc, gfx950). There is no CPU fallback.")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in PROTOTYPES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(status: int) -> None:
    if status != TVS_OK:
        msg = lib().tvs_last_error()
        raise TvsError(status, msg.decode() if msg else "")
