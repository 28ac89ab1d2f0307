"""ctypes binding of ``libscd.so`` (the C ABI declared in include/scd.h).

Argument marshalling only: every numerical step runs in the library's HIP kernels. Importing this module
does not load the library; the first call does, and raises if the library has not been built.
"""
from __future__ import annotations

import ctypes
import os
import threading

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libscd.so")

SCD_OK = 0
SCD_ERR_NULL = -1
SCD_ERR_SIZE = -2
SCD_ERR_ALIAS = -3
SCD_ERR_NOMEM = -4
SCD_ERR_HIP = -5
SCD_ERR_MODEL = -6
SCD_ERR_UNSUPPORTED = -7
SCD_ERR_PTR = -8

PRECISIONS = {"fp32": 0, "split_bf16": 1, "split_fp16": 2, "bf16": 3, "fp16": 4}


class ScdError(RuntimeError):
    """A non-zero status from the C ABI; ``code`` is the SCD_ERR_* value."""

    def __init__(self, code: int, msg: str):
        super().__init__(f"SCD error {code}: {msg}")
        self.code = code


class ScdOpts(ctypes.Structure):
    _fields_ = [
        ("precision", ctypes.c_int),
        ("batch", ctypes.c_int),
        ("x_stride", ctypes.c_int64),
        ("out_stride", ctypes.c_int64),
        ("stream", ctypes.c_void_p),
        ("workspace", ctypes.c_void_p),
        ("workspace_bytes", ctypes.c_size_t),
    ]


class ScdSelector(ctypes.Structure):
    _fields_ = [
        ("Np", ctypes.c_int),
        ("params", ctypes.c_void_p),
        ("mu", ctypes.c_void_p),
        ("sigma", ctypes.c_void_p),
        ("theta", ctypes.c_float),
        ("conf_min", ctypes.c_float),
    ]


class ScdSscaItem(ctypes.Structure):
    _fields_ = [
        ("x", ctypes.c_void_p),
        ("N", ctypes.c_int64),
        ("Np", ctypes.c_int),
        ("win", ctypes.c_void_p),
        ("out", ctypes.c_void_p),
        ("selector", ctypes.POINTER(ScdSelector)),
        ("mask", ctypes.c_void_p),
    ]


_lock = threading.Lock()
_lib = None

_P = ctypes.c_void_p
_SIGS = {
    "scd_ssca": (ctypes.c_int, [_P, ctypes.c_int64, ctypes.c_int, _P, _P]),
    "scd_ssca_ex": (ctypes.c_int, [_P, ctypes.c_int64, ctypes.c_int, _P, _P, ctypes.POINTER(ScdOpts)]),
    "scd_ssca_block_ex": (ctypes.c_int, [_P, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, ctypes.c_int, _P, _P,
                                         ctypes.POINTER(ScdOpts)]),
    "scd_ssca_cross_ex": (ctypes.c_int, [_P, _P, ctypes.c_int64, ctypes.c_int, _P, ctypes.c_int, _P,
                                         ctypes.POINTER(ScdOpts)]),
    "scd_ssca_strips": (ctypes.c_int, [_P, ctypes.c_int64, ctypes.c_int, _P, _P, ctypes.c_int, _P,
                                       ctypes.POINTER(ScdOpts)]),
    "scd_ssca_stage1_ex": (ctypes.c_int, [_P, ctypes.c_int64, ctypes.c_int, _P, _P, ctypes.POINTER(ScdOpts)]),
    "scd_ssca_stage2_ex": (ctypes.c_int, [_P, ctypes.c_int64, ctypes.c_int, _P, ctypes.POINTER(ScdOpts)]),
    "scd_fam": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int, ctypes.c_int, _P, _P]),
    "scd_fam_ex": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int, ctypes.c_int, _P, _P, ctypes.POINTER(ScdOpts)]),
    "scd_fam_cross_ex": (ctypes.c_int, [_P, _P, ctypes.c_int, ctypes.c_int, ctypes.c_int, _P, ctypes.c_int, _P,
                                        ctypes.POINTER(ScdOpts)]),
    "scd_fam_power_ex": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int, ctypes.c_int, _P, _P,
                                        ctypes.POINTER(ScdOpts)]),
    "scd_ssca_workspace_size": (ctypes.c_int, [ctypes.c_int64, ctypes.c_int, ctypes.c_int,
                                               ctypes.POINTER(ctypes.c_size_t)]),
    "scd_fam_workspace_size": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                              ctypes.POINTER(ctypes.c_size_t)]),
    "scd_mlp_param_count": (ctypes.c_int, [ctypes.c_int]),
    "scd_features": (ctypes.c_int, [_P, ctypes.c_int64, ctypes.c_int, _P, _P, ctypes.POINTER(ScdOpts)]),
    "scd_strip_labels": (ctypes.c_int, [_P, ctypes.c_int64, ctypes.c_int, _P, _P, ctypes.POINTER(ScdOpts)]),
    "scd_standardize": (ctypes.c_int, [_P, _P, _P, _P, ctypes.c_int, ctypes.c_int, _P]),
    "scd_mlp_forward": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, _P, _P, _P, _P, _P, _P]),
    "scd_mlp_backward": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, _P, _P, _P, _P, _P, _P, _P, _P, _P]),
    "scd_adam_step": (ctypes.c_int, [ctypes.c_int, _P, _P, _P, _P, ctypes.c_int, ctypes.c_float, ctypes.c_float,
                                     ctypes.c_float, ctypes.c_float, _P]),
    "scd_select": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int, ctypes.c_float, _P, _P, _P]),
    "scd_ssca_learned": (ctypes.c_int, [_P, ctypes.c_int64, ctypes.c_int, _P, ctypes.POINTER(ScdSelector), _P, _P,
                                        ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ScdOpts)]),
    "scd_selector_run": (ctypes.c_int, [_P, ctypes.c_int64, ctypes.c_int, _P, ctypes.POINTER(ScdSelector), _P, _P, _P,
                                        _P, ctypes.POINTER(ScdOpts)]),
    "scd_ssca_batch": (ctypes.c_int, [ctypes.POINTER(ScdSscaItem), ctypes.c_int, ctypes.POINTER(ScdOpts)]),
    "scd_ssca_noalloc": (ctypes.c_int, [_P, ctypes.c_int64, ctypes.c_int, _P, _P, ctypes.POINTER(ScdOpts)]),
    "scd_ssca_noalloc_limit": (ctypes.c_size_t, []),
    "scd_receiver_create": (ctypes.c_int, [ctypes.c_int64, ctypes.c_int, _P, ctypes.c_int, ctypes.POINTER(_P),
                                           ctypes.c_int, _P, ctypes.POINTER(ctypes.c_void_p)]),
    "scd_receiver_push": (ctypes.c_int, [_P, _P, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int64)]),
    "scd_receiver_finish": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int64)]),
    "scd_receiver_wait_copy": (ctypes.c_int, [_P]),
    "scd_receiver_destroy": (ctypes.c_int, [_P]),
    "scd_model_create": (ctypes.c_int, [ctypes.c_int, _P, _P, _P, ctypes.c_float, ctypes.c_float,
                                        ctypes.POINTER(ctypes.c_void_p)]),
    "scd_model_destroy": (ctypes.c_int, [_P]),
    "scd_model_selector": (ctypes.c_int, [_P, ctypes.POINTER(ScdSelector)]),
    "scd_model_read": (ctypes.c_int, [_P, _P, _P, _P]),
    "scd_model_write": (ctypes.c_int, [ctypes.c_char_p, ctypes.c_int, _P, _P, _P, ctypes.c_float, ctypes.c_float]),
    "scd_model_save": (ctypes.c_int, [_P, ctypes.c_char_p]),
    "scd_model_load": (ctypes.c_int, [ctypes.c_char_p, ctypes.POINTER(ctypes.c_void_p)]),
    "scd_set_stream": (ctypes.c_int, [_P]),
    "scd_last_error": (ctypes.c_char_p, []),
    "scd_version": (ctypes.c_int, []),
    "scd_shutdown": (None, []),
}


def lib():
    """The loaded library (loaded once). Raises RuntimeError if it has not been built."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError(f"{LIB_PATH} is missing: build it first (python -c 'import __graft_entry__ as g; "
                                   "g.build()' or python paper_2506_18003_amd/build.py)")
            h = ctypes.CDLL(LIB_PATH)
            for name, (res, args) in _SIGS.items():
                fn = getattr(h, name, None)
                if fn is None:
                    continue
                fn.restype = res
                fn.argtypes = args
            _lib = h
        return _lib


def check(rc: int) -> None:
    if rc != SCD_OK:
        raise ScdError(rc, lib().scd_last_error().decode(errors="replace"))
