"""ctypes declarations of the C ABI in include/qw.h (libqw.so, built in-tree)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libqw.so")

QW_OK, QW_EINVAL, QW_ENOMEM, QW_ECAPACITY, QW_EDEVICE, QW_ENOTSUP = 0, -1, -2, -3, -4, -5
QW_REQUIRE_SYMMETRIC = 0x1
QW_INIT_RAW = 0x1
QW_COUNT, QW_NORM, QW_J_MARGINAL, QW_PROJECT, QW_STATS = 1, 2, 3, 4, 5


QW_LANES_8, QW_LANES_16 = 1 << 16, 2 << 16
QW_XCD_ROWS = 1 << 18


def lanes_flag(lanes: int) -> int:
    """Load flags for the lanes that share a row of s >= 16 slots (0: the
    library's rule)."""
    return {0: 0, 8: QW_LANES_8, 16: QW_LANES_16}[int(lanes)]


def word_length(w: int) -> int:
    """Load flags for fixed-point data of word length w (QW_WORD_LENGTH)."""
    return (int(w) & 0x3F) << 8

# every symbol the header declares
SYMBOLS = [
    "qw_load_csc", "qw_load_csc_batched", "qw_ctx_info", "qw_ctx_ninst", "qw_state_init", "qw_step",
    "qw_step_adjoint", "qw_measure", "qw_export", "qw_export_complex", "qw_state_import", "qw_state_import_complex", "qw_sync", "qls_run",
    "qw_cks_coeffs", "qw_grad", "qw_state_free", "qw_ctx_free", "qw_last_error", "qw_set_launch",
    "qw_shutdown", "qw_load_csc_hermitian", "qw_kappa", "qw_grad_noalloc", "qw_grad_complex",
]

ALLOC_T = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_T = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class QwAllocator(ctypes.Structure):
    _fields_ = [("alloc", ALLOC_T), ("free", FREE_T), ("user", ctypes.c_void_p)]


class QwError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"qw error {code}: {msg}")
        self.code = code


_lib = None


def load() -> ctypes.CDLL:
    """Load libqw.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2303_06890_amd.build.build() "
                          "(the walk has no CPU fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    PP = ctypes.POINTER(ctypes.c_void_p)
    i32, i64, u32, dbl = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_double
    ip = ctypes.POINTER(ctypes.c_int32)
    lp = ctypes.POINTER(ctypes.c_int64)
    dp = ctypes.POINTER(ctypes.c_double)
    up = ctypes.POINTER(ctypes.c_uint64)
    ap = ctypes.POINTER(QwAllocator)
    c_int = ctypes.c_int
    sig = {
        "qw_load_csc": (c_int, [PP, i32, ip, ip, dp, i64, dbl, u32, ap, P]),
        "qw_load_csc_batched": (c_int, [PP, i32, ip, lp, lp, ip, ip, dp, dp, u32, ap, P]),
        "qw_load_csc_hermitian": (c_int, [PP, i32, ip, lp, lp, ip, ip, dp, dp, dp, u32, ap, P]),
        "qw_ctx_info": (c_int, [P, i32, ip, ip, ip, dp, dp]),
        "qw_kappa": (c_int, [P, i32, dp]),
        "qw_ctx_ninst": (i32, [P]),
        "qw_state_init": (c_int, [PP, P, dp, dp, u32, i64, P]),
        "qw_step": (c_int, [P, i32, P]),
        "qw_step_adjoint": (c_int, [P, i32, P]),
        "qw_measure": (c_int, [P, i32, P, i64, P]),
        "qw_export": (c_int, [P, up, dp, dp, i64, lp, P]),
        "qw_export_complex": (c_int, [P, up, dp, i64, lp, P]),
        "qw_state_import": (c_int, [P, up, dp, dp, i64, P]),
        "qw_state_import_complex": (c_int, [P, up, dp, i64, P]),
        "qw_sync": (c_int, [P, P]),
        "qls_run": (c_int, [P, dp, dbl, dbl, i32, dp, dp, dp, dp, lp, P]),
        "qw_cks_coeffs": (c_int, [i64, i32, dp]),
        "qw_grad": (c_int, [P, dp, i32, dp, dp, dp, dp, P]),
        "qw_grad_noalloc": (c_int, [P, dp, i32, dp, dp, dp, dp, P]),
        "qw_grad_complex": (c_int, [P, dp, i32, dp, dp, dp, dp, dp, P]),
        "qw_state_free": (None, [P]),
        "qw_ctx_free": (None, [P]),
        "qw_last_error": (ctypes.c_char_p, []),
        "qw_set_launch": (c_int, [P, i32, i32]),
        "qw_shutdown": (None, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def check(rc: int) -> None:
    if rc != QW_OK:
        raise QwError(rc, load().qw_last_error().decode())
