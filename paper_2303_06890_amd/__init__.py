"""MI355X quantum-walk library: Python binding of libqw.so.

The walk of arXiv:2303.06890 (W = S T~ P T~^dagger on the registers
j_c, j, b1, k_c, k, b2 of a sparse symmetric or complex Hermitian matrix
stored in QRAM) runs in
hand-written HIP kernels behind the C ABI of include/qw.h.  This module only
marshals arguments: torch provides device memory (through the allocator
hooks) and the current stream; every step of the walk runs in the library.
"""
from __future__ import annotations

import atexit
import ctypes
import weakref

import numpy as np
import torch  # noqa: F401  (imported before the atexit hook below is registered, so the hook runs first)

from . import _lib
from ._lib import QwError, check  # noqa: F401

__all__ = ["Walk", "State", "QwError", "WalkObservable", "cks_coeffs", "pack_key", "stream"]


# At interpreter exit, library objects still alive are freed and the kernels
# are released from the HIP runtime (qw_shutdown) by an atexit hook, while
# Python, torch and the runtime are intact; nothing of the library is left
# for the process's native teardown.
_live_states: "weakref.WeakSet" = weakref.WeakSet()
_live_walks: "weakref.WeakSet" = weakref.WeakSet()
_exiting = False


@atexit.register
def _release_all():
    global _exiting
    for st in list(_live_states):
        st.close()
    for w in list(_live_walks):
        w.close()
    if _lib._lib is not None:
        _lib._lib.qw_shutdown()
    _exiting = True


def _torch():
    import torch

    return torch


_streams = {}


def stream():
    """The torch stream every library call of this binding runs on (one per
    device, default priority).  Work on it is ordered; record timing events
    on it.  A non-null stream lets the library replay step loops from
    captured HIP graphs."""
    torch = _torch()
    dev = torch.cuda.current_device()
    if dev not in _streams:
        _streams[dev] = torch.cuda.Stream(device=dev)
    return _streams[dev]


def _stream():
    return ctypes.c_void_p(stream().cuda_stream)


class _TorchAllocator:
    """Device memory from torch's caching allocator."""

    def __init__(self, device):
        self.device = device
        self.live = {}
        self._a = _lib.ALLOC_T(self._alloc)
        self._f = _lib.FREE_T(self._free)
        self.struct = _lib.QwAllocator(self._a, self._f, None)

    def _alloc(self, nbytes, user):
        try:
            t = _torch().empty(int(nbytes), dtype=_torch().uint8, device=self.device)
        except Exception:  # out of memory: report NULL to the library
            return None
        p = t.data_ptr()
        self.live[p] = t
        return p

    def _free(self, p, user):
        self.live.pop(p, None)


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _lp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


def _up(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))


class Walk:
    """One or more sparse symmetric (or complex Hermitian) matrices
    preprocessed and resident on the GPU (a ``qw_ctx``).  ``mats``: a CSC
    object (attributes n, colptr, rowidx, vals) or a list of them (batched
    form); complex values select the Hermitian loader.  ``scale``: None
    (automatic 1/max(1, max|a|)), a float, or one float per matrix.
    ``word``: 0 for FP64 values, or the word length (1 ... 32) of fixed-point
    data, whose rotation is then computed in fixed point.  ``lanes``: 0 for
    the library's rule, or 8 / 16 lanes of a step-kernel wavefront per row of
    s >= 16 slots; ``xcd``: number the one-pass step and adjoint kernels' row blocks by XCD
    (QW_XCD_ROWS).  Both are tuning choices that leave results unchanged (see
    autotune)."""

    def __init__(self, mats, scale=None, symmetric: bool = True, torch_alloc: bool = True, word: int = 0,
                 lanes: int = 0, xcd: bool = False):
        lib = _lib.load()
        self.mats = list(mats) if isinstance(mats, (list, tuple)) else [mats]
        self.ninst = len(self.mats)
        self._alloc = _TorchAllocator(_torch().device("cuda", _torch().cuda.current_device())) if torch_alloc else None
        n = np.array([m.n for m in self.mats], np.int32)
        colptr = np.concatenate([np.asarray(m.colptr, np.int32) for m in self.mats])
        rowidx = np.concatenate([np.asarray(m.rowidx, np.int32) for m in self.mats])
        self.complex = any(np.iscomplexobj(m.vals) for m in self.mats)
        allv = np.concatenate([np.asarray(m.vals) for m in self.mats])
        vals = np.ascontiguousarray(np.real(allv), np.float64)
        vim = np.ascontiguousarray(np.imag(allv), np.float64) if self.complex else None
        coff = np.cumsum([0] + [m.n + 1 for m in self.mats[:-1]]).astype(np.int64)
        zoff = np.cumsum([0] + [len(m.rowidx) for m in self.mats[:-1]]).astype(np.int64)
        if scale is None:
            sc = None
        else:
            sc = np.broadcast_to(np.asarray(scale, np.float64), (self.ninst,)).copy()
        self._keep = (n, colptr, rowidx, vals, vim, coff, zoff, sc)
        h = ctypes.c_void_p()
        flags = (_lib.QW_REQUIRE_SYMMETRIC if symmetric else 0) | _lib.word_length(word) | _lib.lanes_flag(lanes)
        if xcd:
            flags |= _lib.QW_XCD_ROWS
        self.word = int(word)
        self.lanes = int(lanes)
        self.xcd = bool(xcd)
        self.load_args = dict(scale=scale, symmetric=symmetric, torch_alloc=torch_alloc, word=word)
        alloc = ctypes.byref(self._alloc.struct) if self._alloc else None
        scp = _dp(sc) if sc is not None else None
        if self.complex:
            check(lib.qw_load_csc_hermitian(ctypes.byref(h), self.ninst, _ip(n), _lp(coff), _lp(zoff), _ip(colptr),
                                            _ip(rowidx), _dp(vals), _dp(vim), scp, flags, alloc, _stream()))
        else:
            check(lib.qw_load_csc_batched(ctypes.byref(h), self.ninst, _ip(n), _lp(coff), _lp(zoff), _ip(colptr),
                                          _ip(rowidx), _dp(vals), scp, flags, alloc, _stream()))
        self._h = h
        _live_walks.add(self)
        self.info = []
        for i in range(self.ninst):
            N, s, nb = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
            scv = ctypes.c_double()
            check(lib.qw_ctx_info(h, i, ctypes.byref(N), ctypes.byref(s), ctypes.byref(nb), ctypes.byref(scv), None))
            self.info.append(dict(N=N.value, s=s.value, nbits=nb.value, scale=scv.value))
        self.nbits = self.info[0]["nbits"]
        self.N_total = sum(d["N"] for d in self.info)
        self.n_total = int(n.sum())
        self.nnz_total = int(vals.shape[0])

    def close(self):
        """Release this handle; states made from the walk stay valid (each
        holds its own reference to the library context)."""
        if getattr(self, "_h", None) and not _exiting:
            _lib.load().qw_ctx_free(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def state(self, b, raw: bool = False, capacity: int = 0) -> "State":
        """T~|b~> (or |b~> with raw=True); ``b``: sum n_i values, instance
        after instance (a list of per-instance vectors is concatenated)."""
        if isinstance(b, (list, tuple)):
            b = np.concatenate([np.asarray(x) for x in b])
        b = np.asarray(b)
        if b.shape[0] != self.n_total:
            raise ValueError(f"b has {b.shape[0]} entries, expected {self.n_total}")
        br = np.ascontiguousarray(b.real, dtype=np.float64)
        bi = np.ascontiguousarray(np.imag(b) if np.iscomplexobj(b) else np.zeros_like(br), dtype=np.float64)
        h = ctypes.c_void_p()
        check(_lib.load().qw_state_init(ctypes.byref(h), self._h, _dp(br), _dp(bi),
                                         _lib.QW_INIT_RAW if raw else 0, int(capacity), _stream()))
        return State(self, h)

    def kappa(self, inst: int = 0) -> float:
        """Condition number 1 / min |lambda(A/s)| of one instance (qw_kappa:
        computed by the library once, then kept)."""
        k = ctypes.c_double()
        check(_lib.load().qw_kappa(self._h, int(inst), ctypes.byref(k)))
        return k.value

    def kappa_known(self, inst: int = 0) -> float:
        """The condition number if the library has computed it, else NaN."""
        k = ctypes.c_double()
        check(_lib.load().qw_ctx_info(self._h, int(inst), None, None, None, None, ctypes.byref(k)))
        return k.value

    def qls(self, b, kappa: float | None = None, eps: float = 1e-3, j0: int | None = None):
        """Walk-based CKS solve on instance 0: returns (x, p_succ, walk_steps,
        y_norm) with x = y / |y| the post-selected, normalised solution and
        y_norm = |y| (y = y_norm * x is the unnormalised LCU output).
        kappa None: the library's own condition number."""
        b = np.ascontiguousarray(b, dtype=np.float64)
        n0 = self.mats[0].n
        xr, xi = np.zeros(n0), np.zeros(n0)
        p, yn = ctypes.c_double(), ctypes.c_double()
        steps = ctypes.c_int64()
        check(_lib.load().qls_run(self._h, _dp(b), 0.0 if kappa is None else float(kappa), float(eps),
                                  -1 if j0 is None else int(j0), _dp(xr), _dp(xi), ctypes.byref(yn),
                                  ctypes.byref(p), ctypes.byref(steps), _stream()))
        return xr + 1j * xi, p.value, steps.value, yn.value


class State:
    """A walk state on the GPU (a ``qw_state``)."""

    def __init__(self, walk: Walk, h):
        self.walk = walk
        self._h = h
        _live_states.add(self)

    def close(self):
        if getattr(self, "_h", None) and not _exiting:
            _lib.load().qw_state_free(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n: int = 1) -> "State":
        check(_lib.load().qw_step(self._h, int(n), _stream()))
        return self

    def step_adjoint(self, n: int = 1) -> "State":
        check(_lib.load().qw_step_adjoint(self._h, int(n), _stream()))
        return self

    def sync(self) -> "State":
        check(_lib.load().qw_sync(self._h, _stream()))
        return self

    def set_launch(self, wg_size: int = 0, grid: int = 0) -> "State":
        check(_lib.load().qw_set_launch(self._h, int(wg_size), int(grid)))
        return self

    def _measure(self, kind, out):
        check(_lib.load().qw_measure(self._h, kind, out.ctypes.data_as(ctypes.c_void_p), out.size, _stream()))
        return out

    def count(self) -> int:
        return int(self._measure(_lib.QW_COUNT, np.zeros(1, np.int64))[0])

    def norm2(self) -> float:
        return float(self._measure(_lib.QW_NORM, np.zeros(1))[0])

    def j_marginal(self) -> np.ndarray:
        return self._measure(_lib.QW_J_MARGINAL, np.zeros(self.walk.N_total))

    def project(self) -> np.ndarray:
        out = self._measure(_lib.QW_PROJECT, np.zeros(2 * self.walk.N_total))
        return out[0::2] + 1j * out[1::2]

    def stats(self) -> dict:
        o = self._measure(_lib.QW_STATS, np.zeros(8, np.int64))
        return dict(launches=int(o[0]), branches=int(o[1]), list_capacity=int(o[2]), list_count=int(o[3]),
                    total_written=int(o[4]), real_amplitudes=bool(o[5]), lanes_per_row_s16=int(o[6]),
                    xcd_rows=bool(o[7]))

    def export(self):
        """(keys uint64 sorted, amplitudes complex128).  The library copies
        keys and amplitudes into one pinned host buffer (torch's pinned
        allocator), which both returned arrays share."""
        m = self.count()
        buf = _torch().empty(max(1, 3 * m), dtype=_torch().float64, pin_memory=True).numpy()
        keys, amps = buf[:m].view(np.uint64), buf[m:3 * m]
        got = ctypes.c_int64()
        check(_lib.load().qw_export_complex(self._h, _up(keys), _dp(amps), m, ctypes.byref(got), _stream()))
        return keys[:got.value], amps.view(np.complex128)[:got.value]

    def import_(self, keys, amps) -> "State":
        keys = np.ascontiguousarray(keys, dtype=np.uint64)
        amps = np.ascontiguousarray(amps, dtype=np.complex128)
        if amps.shape != keys.shape:
            raise ValueError("one amplitude per key")
        check(_lib.load().qw_state_import_complex(self._h, _up(keys), _dp(amps.view(np.float64)), keys.shape[0],
                                                  _stream()))
        return self

    def grad(self, w, nsteps: int):
        """Reverse-mode gradient of sum_j w_j p_j after ``nsteps`` steps from
        T~|b~>: returns (loss, dvals in CSC order, db complex).  For complex
        Hermitian values dvals is complex, dL/dRe v + i dL/dIm v
        (qw_grad_complex); for real values it is real (qw_grad).  The library
        copies the results into pinned host buffers (torch's pinned
        allocator), which a real dvals then shares."""
        torch = _torch()
        w = np.ascontiguousarray(w, dtype=np.float64)
        if w.shape[0] != self.walk.n_total:
            raise ValueError("w must have one weight per column of every instance")
        nnz = self.walk.nnz_total
        dv = torch.empty((2 if self.walk.complex else 1) * nnz, dtype=torch.float64, pin_memory=True)
        dbb = torch.empty(2 * self.walk.n_total, dtype=torch.float64, pin_memory=True)
        dp = ctypes.POINTER(ctypes.c_double)
        loss = ctypes.c_double()
        ptr = lambda t, off=0: ctypes.cast(t.data_ptr() + 8 * off, dp)  # noqa: E731
        n = self.walk.n_total
        if self.walk.complex:
            check(_lib.load().qw_grad_complex(self._h, _dp(w), int(nsteps), ptr(dv), ptr(dv, nnz), ptr(dbb),
                                              ptr(dbb, n), ctypes.byref(loss), _stream()))
            g = dv.numpy()
            dvals = np.empty(nnz, np.complex128)
            dvals.real = g[:nnz]  # not re + 1j * im: 1j * nan is nan + nan i
            dvals.imag = g[nnz:]
        else:
            check(_lib.load().qw_grad(self._h, _dp(w), int(nsteps), ptr(dv), ptr(dbb), ptr(dbb, n),
                                      ctypes.byref(loss), _stream()))
            dvals = dv.numpy()
        db = dbb.numpy()
        dbc = np.empty(n, np.complex128)
        dbc.real = db[:n]
        dbc.imag = db[n:]
        return loss.value, dvals, dbc


def cks_coeffs(beta: int, j0: int) -> np.ndarray:
    out = np.zeros(j0 + 1)
    check(_lib.load().qw_cks_coeffs(int(beta), int(j0), _dp(out)))
    return out


def pack_key(nbits: int, jc, j, b1, kc, k, b2, inst=0) -> int:
    """Key layout [inst | j_c | j | b1 | k_c | k | b2] (high to low bits)."""
    key = int(inst)
    for v, wdt in ((jc, nbits), (j, nbits), (b1, 1), (kc, nbits), (k, nbits), (b2, 1)):
        key = (key << wdt) | int(v)
    return key


class _CscArrays:
    def __init__(self, n, colptr, rowidx, vals):
        self.n, self.colptr, self.rowidx, self.vals = n, colptr, rowidx, vals


def _make_walk_observable():
    torch = _torch()

    class WalkObservable(torch.autograd.Function):
        """p = j-register marginal of W^nsteps T~|b~> for the matrix with the
        given CSC pattern and (already scaled) values, real or complex
        Hermitian; differentiable in the values and in b (torch's convention
        for complex inputs: dL/dRe + i dL/dIm).  The backward pass is the
        library's reverse sweep (qw_grad, qw_grad_complex): earlier states
        are recomputed with W^dagger."""

        @staticmethod
        def forward(ctx, vals, b, pattern, nsteps):
            v = vals.detach().cpu().numpy()
            v = v.astype(np.complex128 if np.iscomplexobj(v) else np.float64)
            mat = _CscArrays(pattern.n, np.asarray(pattern.colptr, np.int32), np.asarray(pattern.rowidx, np.int32), v)
            walk = Walk(mat, scale=1.0, symmetric=False)  # entries are independent parameters
            st = walk.state(b.detach().cpu().numpy())
            st.step(int(nsteps))
            p = st.j_marginal()[: pattern.n]
            ctx.walk, ctx.st, ctx.nsteps = walk, st, int(nsteps)
            ctx.b_complex = b.is_complex()
            return torch.from_numpy(p.copy())

        @staticmethod
        def backward(ctx, grad_p):
            w = grad_p.detach().cpu().numpy().astype(np.float64)
            _, dv, db = ctx.st.grad(w, ctx.nsteps)
            ctx.st.close()
            gv = torch.from_numpy(dv)
            gb = torch.from_numpy(db) if ctx.b_complex else torch.from_numpy(db.real.copy())
            return gv, gb, None, None

    return WalkObservable


class _Lazy:
    _cls = None

    def __getattr__(self, name):
        if _Lazy._cls is None:
            _Lazy._cls = _make_walk_observable()
        return getattr(_Lazy._cls, name)


WalkObservable = _Lazy()
