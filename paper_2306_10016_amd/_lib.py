"""Loader and ctypes signatures for libhdc.so (the C-ABI of include/hdc.h)."""
from __future__ import annotations

import ctypes
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhdc.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "hdc.h")

_I64 = ctypes.c_int64
_P = ctypes.c_void_p
_PP = ctypes.POINTER(ctypes.c_void_p)
_PI64 = ctypes.POINTER(ctypes.c_int64)
_ST = ctypes.c_int

_lib = None


class HdcError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"hdc status {status}: {msg}")
        self.status = status


class AxisDesc(ctypes.Structure):
    _fields_ = [("L", _I64), ("M", _I64), ("m", _I64), ("p", _I64), ("q", _I64), ("N", _I64), ("D", _I64),
                ("C", _I64), ("q_out", _I64), ("m1", _I64), ("m2", _I64), ("variant", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class Problem(ctypes.Structure):
    """hdc_problem (include/hdc_tune.h)."""
    _fields_ = [("ndim", ctypes.c_int32), ("L", _I64 * 3), ("M", _I64 * 3), ("dtype", ctypes.c_int),
                ("batch", _I64)]


class Params(ctypes.Structure):
    """hdc_params (include/hdc_tune.h): per-axis m, p, q, D, C and column tile."""
    _fields_ = [("m", _I64 * 3), ("p", _I64 * 3), ("q", _I64 * 3), ("D", _I64 * 3), ("C", _I64 * 3),
                ("tile", ctypes.c_int32 * 3)]


COST_FN = ctypes.CFUNCTYPE(ctypes.c_double, ctypes.POINTER(Problem), ctypes.POINTER(Params), ctypes.c_void_p)

SIGNATURES = {
    "hdc_derive": [_I64, _I64, _I64, _I64, _I64, _I64, _I64, ctypes.c_int, ctypes.POINTER(AxisDesc)],
    "hdc_plan": [_PP, _I64, _I64, _I64, _I64, _I64, _I64, _I64, ctypes.c_int],
    "hdc_plan_nd": [_PP, ctypes.c_int, _PI64, _PI64, _PI64, _PI64, _PI64, _PI64, ctypes.c_int],
    "hdc_plan_nd_check": [ctypes.c_int, _PI64, _PI64, _PI64, _PI64, _PI64, _PI64, ctypes.c_int,
                          ctypes.POINTER(AxisDesc)],
    "hdc_uneq_derive": [_I64, _I64, _I64, _I64, _I64, _I64, _I64, ctypes.c_int, ctypes.POINTER(AxisDesc),
                        ctypes.POINTER(AxisDesc), ctypes.POINTER(ctypes.c_int)],
    "hdc_plan_uneq": [_PP, _I64, _I64, _I64, _I64, _I64, _I64, _I64, ctypes.c_int],
    "hdc_forward_operand": [_P, ctypes.c_int, _P, _P, _I64, _P, _P],
    "hdc_uneq_nd_check": [ctypes.c_int, _PI64, _PI64, _PI64, _PI64, _PI64, _PI64, ctypes.c_int,
                          ctypes.POINTER(AxisDesc), ctypes.POINTER(AxisDesc), ctypes.POINTER(ctypes.c_int)],
    "hdc_plan_uneq_nd": [_PP, ctypes.c_int, _PI64, _PI64, _PI64, _PI64, _PI64, _PI64, ctypes.c_int],
    "hdc_plan_multi": [_PP, ctypes.c_int, _I64, _I64, _I64, _I64, _I64, _I64, _I64, ctypes.c_int],
    "hdc_convolve_multi": [_P, ctypes.POINTER(ctypes.c_void_p), _P, _P, _P],
    "hdc_plan_multi_nd": [_PP, ctypes.c_int, ctypes.c_int, _PI64, _PI64, _PI64, _PI64, ctypes.c_int],
    "hdc_plan_destroy": [_P],
    "hdc_plan_axis": [_P, ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(AxisDesc)],
    "hdc_workspace_size": [_P, ctypes.POINTER(ctypes.c_size_t)],
    "hdc_residue_buffer_size": [_P, ctypes.POINTER(ctypes.c_size_t)],
    "hdc_convolve": [_P, _P, _P, _P, _P, _P],
    "hdc_convolve_noalloc": [_P, _P, _P, _P, _P],
    "hdc_forward": [_P, _P, _P, _I64, _P, _P],
    "hdc_multiply": [_P, _P, _P, _I64, _P],
    "hdc_backward": [_P, _P, _P, _I64, _P, _P],
    "hdc_residues_natural": [_P, _P, _I64, _P, _P],
    "hdc_batch_plan": [_PP, _I64, _PI64, _PI64, _PI64, ctypes.c_int],
    "hdc_batch_workspace_size": [_P, ctypes.POINTER(ctypes.c_size_t)],
    "hdc_batch_default_m": [_I64, _PI64],
    "hdc_batch_convolve": [_P, _P, _P, _P, _P, _P],
    "hdc_batch_convolve_eager": [_P, _P, _P, _P, _P, _P],
    "hdc_batch_info": [_P, _PI64, _PI64, _PI64],
    "hdc_batch_destroy": [_P],
    "hdc_time_convolve": [_P, _P, _P, _P, _P, _P, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_float)],
    "hdc_convolve_profiled": [_P, _P, _P, _P, _P, _P, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                              ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_float),
                              ctypes.POINTER(ctypes.c_double)],
    "hdc_profile_begin": [_P],
    "hdc_profile_end": [ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int32),
                        ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_double)],
    "hdc_plan_params": [_PP, ctypes.POINTER(Problem), ctypes.POINTER(Params)],
    "hdc_params_check": [ctypes.POINTER(Problem), ctypes.POINTER(Params), ctypes.POINTER(Params)],
    "hdc_tune": [ctypes.POINTER(Problem), ctypes.c_int, ctypes.c_char_p, ctypes.POINTER(Params),
                 ctypes.POINTER(ctypes.c_double)],
    "hdc_tune_host": [ctypes.POINTER(Problem), ctypes.c_int, ctypes.c_char_p, ctypes.c_char_p, ctypes.c_char_p,
                      COST_FN, ctypes.c_void_p, ctypes.POINTER(Params), ctypes.POINTER(ctypes.c_double)],
    "hdc_build_id": [],
    "hdc_batch_db_choose": [_I64, _PI64, _PI64, ctypes.c_int, ctypes.c_char_p, ctypes.c_char_p, ctypes.c_char_p,
                            _PI64],
    "hdc_batch_db_record": [ctypes.c_char_p, _I64, ctypes.c_int, _I64, ctypes.c_double, ctypes.c_char_p,
                            ctypes.c_char_p],
    "hdc_batch_plan_db": [_PP, _I64, _PI64, _PI64, ctypes.c_int, ctypes.c_char_p],
    "hdc_predictor_load": [_PP, ctypes.c_char_p],
    "hdc_predict": [_P, ctypes.POINTER(Problem), ctypes.POINTER(Params), ctypes.POINTER(ctypes.c_float)],
    "hdc_predictor_destroy": [_P],
    "hdc_last_error": [],
    "hdc_version": [],
}


def lib():
    """The loaded libhdc.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"libhdc.so not found at {LIB_PATH}: build it with "
                              f"`python -m paper_2306_10016_amd.build` (there is no CPU fallback)")
        # PyTorch ships its own HIP runtime under the same soname as the system's
        # (libamdhip64.so.7); the first one loaded serves the whole process.  Loading
        # torch first keeps one runtime, torch's, for the library and for the
        # tensors it is handed; loaded first, the library would pull in the system
        # runtime and torch would then find no device.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        for name, args in SIGNATURES.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = ctypes.c_char_p if name in ("hdc_last_error", "hdc_version", "hdc_build_id") else _ST
        try:
            from . import mlp as _mlp
            _mlp.bind(L)
        except ImportError:
            pass
        _lib = L
    return _lib


def check(status: int):
    if status != 0:
        raise HdcError(status, lib().hdc_last_error().decode())


def header_symbols(path: str = HEADER):
    """Function names declared in a C header (used by the export test)."""
    src = open(path).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    src = re.sub(r"//[^\n]*", "", src)
    return sorted(set(re.findall(r"\b(hdc_[a-z0-9_]+)\s*\(", src)))
