"""ctypes binding of libipb.so (the C ABI in include/ipb.h): argument
marshalling only.  Every step of the completion runs in the HIP kernels; if
the library is not built, every call raises."""
from __future__ import annotations

import ctypes
import os
import re
from typing import List

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libipb.so")
HEADER = os.path.join(os.path.dirname(PKG), "include", "ipb.h")

IPB_OK = 0
IPB_ERR_INVALID_ARG = -1
IPB_ERR_UNSUPPORTED = -2
IPB_ERR_WORKSPACE = -3
IPB_ERR_HIP = -4
IPB_ERR_SCRATCH = -5


class CParams(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32),
        ("dilate_shape", ctypes.c_int32),
        ("dilate_size", ctypes.c_int32),
        ("close_size", ctypes.c_int32),
        ("fill_size", ctypes.c_int32),
        ("extrapolate", ctypes.c_int32),
        ("large_fill_size", ctypes.c_int32),
        ("median_size", ctypes.c_int32),
        ("gauss_size", ctypes.c_int32),
        ("gauss_sigma", ctypes.c_float),
        ("max_depth", ctypes.c_float),
        ("valid_thresh", ctypes.c_float),
        ("tile_local", ctypes.c_int32),
        ("tile_global", ctypes.c_int32),
        ("blur", ctypes.c_int32),
        ("bilateral_sigma_space", ctypes.c_float),
        ("bilateral_sigma_color", ctypes.c_float),
        ("extend_rows", ctypes.c_int32),
    ]


class CFrame(ctypes.Structure):
    _fields_ = [
        ("in_", ctypes.c_void_p),
        ("out", ctypes.c_void_p),
        ("H", ctypes.c_int32),
        ("W", ctypes.c_int32),
    ]


class IpbError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        msg = f"{what}: {status_string(status)} (status {status})"
        if status == IPB_ERR_HIP:
            msg += f", hipError {lib().ipb_last_hip_error()}"
        super().__init__(msg)


_lib = None

_P = ctypes.POINTER
_SIGS = {
    "ipb_params_default": (None, [_P(CParams)]),
    "ipb_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int, ctypes.c_int, _P(CParams)]),
    "ipb_complete": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, _P(CParams),
                                    ctypes.c_void_p, ctypes.c_void_p]),
    "ipb_complete_ws": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, _P(CParams),
                                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "ipb_complete_static": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, _P(CParams),
                                           ctypes.c_void_p, ctypes.c_void_p]),
    "ipb_complete_stage": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, _P(CParams),
                                          ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_size_t,
                                          ctypes.c_void_p]),
    "ipb_batch_workspace_bytes": (ctypes.c_size_t, [_P(CFrame), ctypes.c_int, _P(CParams)]),
    "ipb_complete_batch": (ctypes.c_int, [_P(CFrame), ctypes.c_int, _P(CParams), ctypes.c_void_p,
                                          ctypes.c_size_t, ctypes.c_void_p]),
    "ipb_batch_plan_bytes": (ctypes.c_size_t, [ctypes.c_int]),
    "ipb_batch_plan": (ctypes.c_int, [_P(CFrame), ctypes.c_int, _P(CParams), ctypes.c_void_p, ctypes.c_size_t,
                                      ctypes.c_void_p, ctypes.c_size_t]),
    "ipb_complete_planned": (ctypes.c_int, [ctypes.c_void_p, _P(CParams), ctypes.c_int, ctypes.c_int,
                                            ctypes.c_int, ctypes.c_int, ctypes.c_void_p]),
    "ipb_plan_totals": (ctypes.c_int, [ctypes.c_void_p, _P(ctypes.c_int), _P(ctypes.c_int), _P(ctypes.c_int),
                                       _P(ctypes.c_int)]),
    "ipb_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "ipb_last_hip_error": (ctypes.c_int, []),
    "ipb_stream_create": (ctypes.c_int, [_P(ctypes.c_void_p)]),
    "ipb_stream_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "ipb_tile_shape": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, _P(ctypes.c_int), _P(ctypes.c_int)]),
    "ipb_tile_count": (ctypes.c_int, [ctypes.c_int]),
}


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1802_00036_amd.build` "
                               "(there is no fallback implementation)")
        h = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(h, name)
            fn.restype = res
            fn.argtypes = args
        _lib = h
    return _lib


def header_functions() -> List[str]:
    """Names of the functions include/ipb.h declares."""
    with open(HEADER) as fh:
        text = fh.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ipb_[a-z_]+)\s*\(", text)))


def status_string(status: int) -> str:
    return lib().ipb_status_string(status).decode()


def check(status: int, what: str) -> None:
    if status != IPB_OK:
        raise IpbError(status, what)
