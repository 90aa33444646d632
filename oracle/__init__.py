"""Quantum-walk oracle: TEST INFRASTRUCTURE ONLY.

A ctypes wrapper around ``qw_oracle.cpp``, the plain single-threaded CPU model
of the register-level walk (ordered map from register tuple to complex double,
operators applied one register-level operation at a time, Alg. 5 / Alg. 6 of
arXiv:2303.06890).  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no
code with the GPU library ``paper_2303_06890_amd``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "qw_oracle.cpp")
_LIB = os.path.join(_HERE, "libqworacle.so")
TAU = 1e-13

_lib = None


def build() -> str:
    """Compile the oracle with g++ (always recompiles)."""
    cmd = ["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-o", _LIB + ".tmp", _SRC]
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def _load():
    """Load the oracle library; QW_ORACLE_LIB names another build of it (the
    tests' planted-mistake copies)."""
    global _lib
    if _lib is not None:
        return _lib
    path = os.environ.get("QW_ORACLE_LIB") or _LIB
    if path == _LIB and not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    i32, i64, u64, dbl = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int32)
    up = ctypes.POINTER(ctypes.c_uint64)
    u8p = ctypes.POINTER(ctypes.c_uint8)
    i64p = ctypes.POINTER(ctypes.c_int64)
    sig = {
        "orc_last_error": (ctypes.c_char_p, []),
        "orc_matrix_new": (P, [i32, ip, ip, dp, dp, i64, dbl]),
        "orc_matrix_free": (None, [P]),
        "orc_matrix_info": (None, [P, ip, ip, ip, dp]),
        "orc_matrix_ell": (None, [P, ip, dp, dp, u8p]),
        "orc_qbs": (u64, [ip, i32, u64]),
        "orc_state_new": (P, [P, dbl]),
        "orc_state_free": (None, [P]),
        "orc_state_clone": (P, [P]),
        "orc_set_b": (ctypes.c_int, [P, dp, dp, i32]),
        "orc_import": (ctypes.c_int, [P, up, dp, dp, i64]),
        "orc_apply_op": (ctypes.c_int, [P, i32]),
        "orc_apply_T": (ctypes.c_int, [P, i32]),
        "orc_step": (ctypes.c_int, [P, i32]),
        "orc_step_adjoint": (ctypes.c_int, [P, i32]),
        "orc_count": (i64, [P]),
        "orc_ambiguous": (i64, [P, i32]),
        "orc_pruned_mass": (dbl, [P]),
        "orc_max_size": (ctypes.c_int64, [P]),
        "orc_export": (ctypes.c_int, [P, up, dp, dp]),
        "orc_norm2": (dbl, [P]),
        "orc_j_marginal": (None, [P, dp]),
        "orc_project0": (ctypes.c_int, [P, dp, dp]),
        "orc_schedule": (None, [dbl, dbl, i64p, ip]),
        "orc_cks_coeffs": (None, [i64, i32, dp]),
        "orc_cheb_series": (ctypes.c_int, [P, dp, dp, i32, i32, dp, dp, dp]),
        "orc_matrix_set_word": (ctypes.c_int, [P, i32]),
        "orc_fx_sqrt": (u64, [u64, i32]),
        "orc_fx_arccos": (u64, [u64, i32]),
        "orc_fx_rotation": (None, [u64, i32, u64, u64, dp, dp, dp]),
        "orc_qls_walk": (ctypes.c_int, [P, dp, i32, i32, dp, dbl, dp, dp]),
        "orc_grad": (ctypes.c_int, [P, dp, dp, i32, i32, dp, dbl, dp, dp, dp, dp]),
        "orc_grad_complex": (ctypes.c_int, [P, dp, dp, i32, i32, dp, dbl, dp, dp, dp, dp, dp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _d(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _i(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _check(rc):
    if rc != 0:
        raise RuntimeError("oracle: " + _load().orc_last_error().decode())


def fx_sqrt(q: int, w: int) -> int:
    """The fixed-point square-root register for the word magnitude q."""
    return int(_load().orc_fx_sqrt(int(q), int(w)))


def fx_arccos(r: int, w: int) -> int:
    """The fixed-point angle register (units of (pi/2) / 2^w) for r / 2^w."""
    return int(_load().orc_fx_arccos(int(r), int(w)))


def fx_rotation(word: int, w: int, j: int, k: int):
    """(f, g) of the rotation for the sign-magnitude fixed-point QRAM word."""
    fr, fi, g = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    _load().orc_fx_rotation(int(word), int(w), int(j), int(k), ctypes.byref(fr), ctypes.byref(fi),
                            ctypes.byref(g))
    return complex(fr.value, fi.value), g.value


# operation codes for OracleState.apply_op
OP_H, OP_OA, OP_OS, OP_OSINV, OP_R, OP_RDAG, OP_P, OP_S = range(8)


class OracleMatrix:
    """Preprocessed matrix (rescale, pow2 s, zero fill, pow2 N).  word > 0:
    the scaled values are fixed-point numbers of that word length and the
    rotation is computed in fixed point."""

    def __init__(self, csc, scale: float = 0.0, word: int = 0):
        lib = _load()
        cp, cpp = _i(csc.colptr)
        ri, rip = _i(csc.rowidx)
        self.complex = np.iscomplexobj(csc.vals)
        va, vap = _d(np.real(csc.vals))
        vi, vip = _d(np.imag(csc.vals)) if self.complex else (None, None)
        self._h = lib.orc_matrix_new(csc.n, cpp, rip, vap, vip, csc.nnz, float(scale))
        if not self._h:
            raise ValueError("oracle: " + lib.orc_last_error().decode())
        N, s, nb = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        sc = ctypes.c_double()
        lib.orc_matrix_info(self._h, ctypes.byref(N), ctypes.byref(s), ctypes.byref(nb), ctypes.byref(sc))
        self.N, self.s, self.nbits, self.scale = N.value, s.value, nb.value, sc.value
        self.n = csc.n
        self.word = int(word)
        if self.word:
            _check(lib.orc_matrix_set_word(self._h, self.word))

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.orc_matrix_free(self._h)
            self._h = None

    def ell(self):
        """(col, value, stored-entry flag), each N x s; values are complex for
        a complex matrix."""
        col = np.zeros(self.N * self.s, np.int32)
        val = np.zeros(self.N * self.s, np.float64)
        vim = np.zeros(self.N * self.s, np.float64)
        real = np.zeros(self.N * self.s, np.uint8)
        _load().orc_matrix_ell(self._h, col.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                               val.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                               vim.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                               real.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)))
        v = val + 1j * vim if self.complex else val
        return col.reshape(self.N, self.s), v.reshape(self.N, self.s), real.reshape(self.N, self.s)

    # --- solver helpers
    def cheb_series(self, b, j0: int, coef):
        """sum_k a_k T_{2k+1}(A/s) b (complex for a complex matrix or b)."""
        b = np.asarray(b)
        br, brp = _d(np.real(b))
        bi, bip = _d(np.imag(b) if np.iscomplexobj(b) else np.zeros(b.shape[0]))
        coef, cp = _d(coef)
        yr, yi = np.zeros(self.N), np.zeros(self.N)
        _check(_load().orc_cheb_series(self._h, brp, bip, br.shape[0], int(j0), cp, _d(yr)[1], _d(yi)[1]))
        return yr + 1j * yi if (self.complex or np.iscomplexobj(b)) else yr

    def qls_walk(self, b, j0: int, coef, tau: float = TAU):
        b, bp = _d(b)
        coef, cp = _d(coef)
        yr, yi = np.zeros(self.N), np.zeros(self.N)
        _check(_load().orc_qls_walk(self._h, bp, b.shape[0], int(j0), cp, tau, _d(yr)[1], _d(yi)[1]))
        return yr + 1j * yi

    def grad(self, b, w, nsteps: int, tau: float = TAU):
        """Reverse mode with stored states: returns (loss, dv[N,s], db complex).
        For a complex matrix dv is complex: dL/dRe v + i dL/dIm v per slot."""
        b = np.asarray(b)
        br, brp = _d(b.real)
        bi, bip = _d(np.imag(b) if np.iscomplexobj(b) else np.zeros(b.shape[0]))
        w, wp = _d(w)
        dv = np.zeros(self.N * self.s)
        dbr, dbi = np.zeros(self.N), np.zeros(self.N)
        loss = ctypes.c_double()
        if self.complex:
            dvi = np.zeros(self.N * self.s)
            _check(_load().orc_grad_complex(self._h, brp, bip, br.shape[0], int(nsteps), wp, tau,
                                            _d(dv)[1], _d(dvi)[1], _d(dbr)[1], _d(dbi)[1], ctypes.byref(loss)))
            g = np.empty(self.N * self.s, np.complex128)
            g.real, g.imag = dv, dvi  # not dv + 1j * dvi: 1j * nan is nan + nan i
            return loss.value, g.reshape(self.N, self.s), dbr + 1j * dbi
        _check(_load().orc_grad(self._h, brp, bip, br.shape[0], int(nsteps), wp, tau,
                                _d(dv)[1], _d(dbr)[1], _d(dbi)[1], ctypes.byref(loss)))
        return loss.value, dv.reshape(self.N, self.s), dbr + 1j * dbi


class OracleState:
    def __init__(self, mat: OracleMatrix, tau: float = TAU, _h=None):
        self.mat = mat
        self._h = _h if _h is not None else _load().orc_state_new(mat._h, tau)

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.orc_state_free(self._h)
            self._h = None

    def clone(self):
        return OracleState(self.mat, _h=_load().orc_state_clone(self._h))

    def set_b(self, b):
        b = np.asarray(b)
        br, brp = _d(b.real)
        bi, bip = _d(np.imag(b) if np.iscomplexobj(b) else np.zeros(b.shape[0]))
        _check(_load().orc_set_b(self._h, brp, bip, br.shape[0]))
        return self

    def import_(self, keys, amps):
        keys = np.ascontiguousarray(keys, dtype=np.uint64)
        re, rp = _d(np.real(amps))
        im, ip = _d(np.imag(amps))
        _check(_load().orc_import(self._h, keys.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), rp, ip,
                                  keys.shape[0]))
        return self

    def apply_op(self, code: int):
        _check(_load().orc_apply_op(self._h, int(code)))
        return self

    def T(self):
        _check(_load().orc_apply_T(self._h, 0))
        return self

    def Tdag(self):
        _check(_load().orc_apply_T(self._h, 1))
        return self

    def step(self, n: int = 1):
        _check(_load().orc_step(self._h, int(n)))
        return self

    def step_adjoint(self, n: int = 1):
        _check(_load().orc_step_adjoint(self._h, int(n)))
        return self

    def count(self) -> int:
        return int(_load().orc_count(self._h))

    def ambiguous(self, total: bool = False) -> int:
        return int(_load().orc_ambiguous(self._h, 1 if total else 0))

    def max_size(self) -> int:
        """Largest branch count after any single register-level operation so
        far, inside walk steps included."""
        return int(_load().orc_max_size(self._h))

    def pruned_mass(self) -> float:
        return float(_load().orc_pruned_mass(self._h))

    def export(self):
        m = self.count()
        keys = np.zeros(m, np.uint64)
        re, im = np.zeros(m), np.zeros(m)
        _check(_load().orc_export(self._h, keys.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                  _d(re)[1], _d(im)[1]))
        return keys, re + 1j * im

    def norm2(self) -> float:
        return float(_load().orc_norm2(self._h))

    def j_marginal(self):
        p = np.zeros(self.mat.N)
        _load().orc_j_marginal(self._h, _d(p)[1])
        return p

    def project0(self):
        yr, yi = np.zeros(self.mat.N), np.zeros(self.mat.N)
        _check(_load().orc_project0(self._h, _d(yr)[1], _d(yi)[1]))
        return yr + 1j * yi


def qbs(row, target: int) -> int:
    row, rp = _i(row)
    return int(_load().orc_qbs(rp, row.shape[0], int(target)))


def schedule(kappa: float, eps: float = 1e-3):
    beta = ctypes.c_int64()
    j0 = ctypes.c_int32()
    _load().orc_schedule(float(kappa), float(eps), ctypes.byref(beta), ctypes.byref(j0))
    return int(beta.value), int(j0.value)


def cks_coeffs(beta: int, j0: int):
    out = np.zeros(j0 + 1)
    _load().orc_cks_coeffs(int(beta), int(j0), _d(out)[1])
    return out


def pack_key(nbits: int, jc, j, b1, kc, k, b2, inst=0):
    """Packed key layout [inst | j_c | j | b1 | k_c | k | b2] (high to low)."""
    n = nbits
    key = int(inst)
    for v, w in ((jc, n), (j, n), (b1, 1), (kc, n), (k, n), (b2, 1)):
        key = (key << w) | int(v)
    return key
