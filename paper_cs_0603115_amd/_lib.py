"""ctypes loader for ``libff.so`` (the C ABI declared in ``include/ff.h``).

The library is built in-tree by ``paper_cs_0603115_amd.build``.  There is no
fallback: if the library is missing or stale the import of this module fails
with an error that says how to build it.
"""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libff.so")

_P = ctypes.c_void_p          # device pointers and streams
_i64 = ctypes.c_int64
_i32 = ctypes.c_int32
_sz = ctypes.c_size_t
_st = ctypes.c_int32          # ff_status


class DotCfg(ctypes.Structure):
    """``ff_dot_cfg``: launch shape of the batched float-float dot."""
    _fields_ = [("block", ctypes.c_int32), ("chunk", ctypes.c_int32),
                ("grid", ctypes.c_int32), ("unroll", ctypes.c_int32)]

    def as_tuple(self):
        return (self.block, self.chunk, self.grid, self.unroll)


_EW = ([_P, _P, _P, _P, _P, _P, _i64, _P], _st)

# name -> (argtypes, restype); must list every function of include/ff.h.
SIGNATURES = {
    "ff_status_str": ([_st], ctypes.c_char_p),
    "ff_abi_version": ([], _i32),
    "ff_build_info": ([], ctypes.c_char_p),
    "ff_last_error": ([], ctypes.c_char_p),
    "ff_add": _EW,
    "ff_sub": _EW,
    "ff_mul": _EW,
    "ff_mul_dekker": _EW,
    "ff_div": _EW,
    "ff_add_accurate": _EW,
    "ff_sub_accurate": _EW,
    "ff_mul_accurate": _EW,
    "ff_div_accurate": _EW,
    "ff_copy": ([_P, _P, _i64, _P], _st),
    "ff_add12": ([_P, _P, _P, _P, _i64, _P], _st),
    "ff_mul12": ([_P, _P, _P, _P, _i64, _P], _st),
    "ff_mul12_dekker": ([_P, _P, _P, _P, _i64, _P], _st),
    "ff_f32_add": ([_P, _P, _P, _i64, _P], _st),
    "ff_f32_mul": ([_P, _P, _P, _i64, _P], _st),
    "ff_f32_mad": ([_P, _P, _P, _P, _i64, _P], _st),
    "ff_dot_batched_workspace_size": ([_i64, _i32, ctypes.POINTER(DotCfg)], _sz),
    "ff_dot_batched": ([_P, _P, _P, _i32, _i64, ctypes.POINTER(DotCfg), _P, _sz, _P, _P, _P],
                       _st),
    "ff_dot_ff_batched": ([_P, _P, _P, _P, _P, _i32, _i64, ctypes.POINTER(DotCfg), _P, _sz, _P,
                           _P, _P], _st),
    "ff_sum_batched": ([_P, _P, _i32, _i64, ctypes.POINTER(DotCfg), _P, _sz, _P, _P, _P], _st),
    "ff_sum_ff_batched": ([_P, _P, _P, _i32, _i64, ctypes.POINTER(DotCfg), _P, _sz, _P, _P, _P],
                          _st),
    "ff_dot2_batched": ([_P, _P, _P, _i32, _i64, ctypes.POINTER(DotCfg), _P, _sz, _P, _P, _P],
                        _st),
    "ff_sum2_batched": ([_P, _P, _i32, _i64, ctypes.POINTER(DotCfg), _P, _sz, _P, _P, _P], _st),
    "ff_dot_batched_noalloc": ([_P, _P, _P, _i32, _i64, ctypes.POINTER(DotCfg), _P, _P, _P], _st),
    "ff_dot_batched_autotune": ([_P, _P, _P, _i32, _i64, _P, _sz, _P, _P, _i32, _P,
                                 ctypes.POINTER(DotCfg), ctypes.POINTER(ctypes.c_float)], _st),
    "ff_matvec": ([_i64, _i64, _P, _P, _i64, _P, _P, _P, _P, _i32, _P], _st),
    "ff_matvec_backward_workspace_size": ([_i64, _i64, _i32], _sz),
    "ff_matvec_backward": ([_i64, _i64, _P, _P, _i64, _P, _P, _P, _P, _P, _P, _i64, _P, _P, _i32,
                            _P, _sz, _P], _st),
    "ff_dot_backward": ([_P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _i64, _P], _st),
    "ff_from_f64": ([_P, _P, _P, _i64, _P], _st),
    "ff_to_f64": ([_P, _P, _P, _i64, _P], _st),
    "ff_horner_f32": ([_P, _i32, _P, _P, _i64, _P], _st),
    "ff_horner_comp": ([_P, _i32, _P, _P, _i64, _P], _st),
    "ff_horner_ff": ([_P, _P, _i32, _P, _P, _P, _P, _i64, _P], _st),
    "ff_dot_batched_backward_workspace_size": ([_i64], _sz),
    "ff_dot_batched_backward": ([_P, _P, _P, _i32, _i64, _P, _P, _P, _P, _P, _P, _P, _P,
                                 _P, _sz, _P], _st),
    "ff_gemm_workspace_size": ([_i64, _i64, _i64, _i32], _sz),
    "ff_gemm": ([_i64, _i64, _i64, _P, _P, _i64, _P, _P, _i64, _P, _P, _i64, _i32, _P, _sz, _P],
                _st),
}

GEMM_FMA_LOOP = 0
GEMM_SLICED_BF16 = 1
GEMM_SLICED_I8 = 2

MATVEC_FAST = 0
MATVEC_PLAIN = 1

FF_OK = 0
STATUS_NAMES = {0: "FF_OK", 1: "FF_ERR_NULL", 2: "FF_ERR_SIZE", 3: "FF_ERR_ALIGN",
                4: "FF_ERR_WORKSPACE", 5: "FF_ERR_UNSUPPORTED", 6: "FF_ERR_HIP",
                7: "FF_ERR_ARG"}


class FFError(RuntimeError):
    """A libff entry point returned a status other than FF_OK."""

    def __init__(self, fn: str, status: int, detail: str = ""):
        self.status = status
        name = STATUS_NAMES.get(status, str(status))
        super().__init__(f"{fn} failed: {name}" + (f" ({detail})" if detail else ""))


def _load() -> ctypes.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"libff.so not found at {LIB_PATH}: build the HIP library first "
            "(python paper_cs_0603115_amd/build.py, or __graft_entry__.build())")
    handle = ctypes.CDLL(LIB_PATH)
    for name, (args, res) in SIGNATURES.items():
        fn = getattr(handle, name)
        fn.argtypes = args
        fn.restype = res
    if handle.ff_abi_version() != 1:
        raise ImportError("libff.so ABI version mismatch: rebuild the library")
    return handle


lib = _load()


def check(fn_name: str, status: int) -> None:
    """Raise FFError unless ``status`` is FF_OK."""
    if status != FF_OK:
        detail = lib.ff_last_error().decode() if status == 6 else ""
        raise FFError(fn_name, status, detail)
