"""ctypes binding of libmdemap.so (the C ABI declared in include/mdemap.h).

Argument marshalling only: torch tensors are used for device memory and streams,
every step of the computation runs in the library's HIP kernels.  If the shared
library is missing the import fails loudly; there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmdemap.so")

MD_OK = 0
STATUS_NAMES = {
    0: "MD_OK", -1: "MD_EINVAL", -2: "MD_ENOTPOW2", -3: "MD_ELABEL", -4: "MD_EDIM",
    -5: "MD_ENOMEM", -6: "MD_EHIP", -7: "MD_ENODEV", -8: "MD_EUNSUPPORTED", -9: "MD_ENONFINITE",
}
PREC = {"fp32": 0, "fp16": 1, "bf16": 2, "bf16_scores": 3}

# name -> (restype, argtypes)
_P = ctypes.c_void_p
_I = ctypes.c_int
_I64 = ctypes.c_int64
_U64 = ctypes.c_uint64
_D = ctypes.c_double
_F = ctypes.c_float
SIGNATURES = {
    "awgn_sample": (_I, [_P, _I, _I, _U64, _U64, _I64, _D, _P, _P, _P]),
    "llr_exact": (_I, [_P, _P, _I, _I, _P, _I64, _D, _I, _P, _P]),
    "llr_maxlog": (_I, [_P, _P, _I, _I, _P, _I64, _D, _P, _P]),
    "llr_exact_noalloc": (_I, [_P, _P, _I, _I, _P, _I64, _D, _I, _P, _P]),
    "gmi_reduce": (_I, [_P, _I64, _I, _P, _P, _P, _P, _P, _P]),
    "gmi_status": (_I, [_P, ctypes.POINTER(ctypes.c_int64)]),
    "llr_exact_gmi": (_I, [_P, _P, _I, _I, _P, _I64, _D, _I, _P, _P, _P, _P, _P]),
    "alloc_fault_inject": (_I, [_I]),
    "alloc_stats": (_I, [ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]),
    "ber_count": (_I, [_P, _I64, _I, _P, _P, _P, _P, _P]),
    "q_factor_db": (_I, [_P, _I64, _P, _P]),
    "llr_path_counts": (_I, [_P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]),
    "mlp_create": (_I, [_I, _I, _I, _U64, ctypes.POINTER(ctypes.c_void_p)]),
    "mlp_destroy": (_I, [_P]),
    "mlp_num_params": (_I64, [_P]),
    "mlp_info": (_I, [_P, _P, _P, _P, _P]),
    "mlp_get": (_I, [_P, _I, _P]),
    "mlp_set_scales": (_I, [_P, _F, _F]),
    "mlp_get_scales": (_I, [_P, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float)]),
    "mlp_set": (_I, [_P, _I, _P]),
    "mlp_grad": (_I, [_P, _P, _P, _I64, _P, _P]),
    "mlp_adam_step": (_I, [_P, _F, _P]),
    "mlp_train_step": (_I, [_P, _P, _P, _I64, _F, _P, _P]),
    "mlp_fit": (_I, [_P, _P, _P, _I64, _I64, _I64, _F, _F, _U64, _P, _P]),
    "llr_learned": (_I, [_P, _P, _I64, _P, _P]),
    "mlp_save": (_I, [_P, ctypes.c_char_p]),
    "mlp_load": (_I, [ctypes.c_char_p, ctypes.POINTER(ctypes.c_void_p)]),
    "sweep_plan_create": (_I, [_P, _I, _P, _I, _I, ctypes.POINTER(ctypes.c_void_p)]),
    "sweep_plan_info": (_I, [_P, _P, _P, _P, _P]),
    "sweep_plan_class": (_I, [_P, _I, _P, _P, _P, _P, _P]),
    "sweep_tuning_clear": (_I, []),
    "sweep_run": (_I, [_P, _P, _I, _P]),
    "sweep_run_stats": (_I, [_P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int), _P]),
    "sweep_plan_destroy": (_I, [_P]),
    "rx_create": (_I, [_P, _P, _I, _I, _D, _P, ctypes.POINTER(ctypes.c_void_p)]),
    "rx_run": (_I, [_P, _P, _P, _I64, _I64, _P, _P, _P, _P]),
    "rx_destroy": (_I, [_P]),
    "kernel_timing": (_I, [_I, _P]),
    "kernel_timing_read": (_I, [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64), _P]),
    "release_cache": (_I, []),
    "last_error": (ctypes.c_char_p, []),
    "ddlms_equalize": (_I, [_P, _I64, _I64, _P, _I, _P, _P, _D, _P, _P, _P, _P, _P]),
    "ddlms_equalize_chain": (_I, [_P, _I64, _I64, _P, _I, _D, _P, _P, _P, _P, _P]),
    "kk_frontend": (_I, [_P, _I64, _F, _D, _P, _P]),
    "ubench": (_I, [_I, _I64, _P, _P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double), _P]),
    "mdemap_version": (_I, []),
}


class SweepInstance(ctypes.Structure):
    """md_sweep_instance of mdemap.h."""
    _fields_ = [("d_X", ctypes.c_void_p), ("d_labels", ctypes.c_void_p), ("M", ctypes.c_int), ("D", ctypes.c_int),
                ("N", ctypes.c_int64), ("seed", ctypes.c_uint64)]


class RxConfig(ctypes.Structure):
    """md_rx_config of mdemap.h."""
    _fields_ = [("mode", ctypes.c_int), ("n_streams", ctypes.c_int), ("buf_symbols", ctypes.c_int64),
                ("bin_symbols", ctypes.c_int64), ("eq_instances", ctypes.c_int), ("eq_mu", ctypes.c_double),
                ("eq_h0", ctypes.c_double * 8), ("eq_g0", ctypes.c_double * 8)]


RX_MODE = {"hard": 0, "exact": 1}


class MdemapError(RuntimeError):
    def __init__(self, fn: str, status: int, msg: str):
        super().__init__(f"{fn}: {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2104_06311_amd.build` "
                              "(the HIP library is required; there is no CPU fallback)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(fn: str, status: int):
    if status != MD_OK:
        msg = lib().last_error().decode(errors="replace")
        raise MdemapError(fn, status, msg)
