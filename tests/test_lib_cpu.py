"""CPU-side checks of the HIP library: it loads, exports every symbol its
header declares, and rejects invalid matrices before touching the GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    text = open(os.path.join(ROOT, "include", "qw.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(q\w+)\s*\(", text)) - {"qw_allocator"})


@pytest.fixture(scope="module")
def lib():
    from paper_2303_06890_amd import _lib

    return _lib.load()


def test_header_symbols_exported(lib):
    from paper_2303_06890_amd import _lib

    names = _declared_symbols()
    assert len(names) >= 15
    assert sorted(names) == sorted(_lib.SYMBOLS)
    for name in names:
        assert hasattr(lib, name), name


def _load(lib, csc, scale=0.0, flags=1):
    from paper_2303_06890_amd import _lib

    h = ctypes.c_void_p()
    cp = np.ascontiguousarray(csc.colptr, np.int32)
    ri = np.ascontiguousarray(csc.rowidx, np.int32)
    va = np.ascontiguousarray(csc.vals, np.float64)
    rc = lib.qw_load_csc(ctypes.byref(h), csc.n, cp.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                         ri.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                         va.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), csc.nnz, scale, flags, None, None)
    return rc, lib.qw_last_error().decode()


def _mutate(csc, rowidx=None, vals=None):
    return W.Csc(csc.n, csc.colptr, csc.rowidx if rowidx is None else rowidx,
                 csc.vals if vals is None else vals)


def test_rejects_unsorted_rows(lib):
    csc = W.offset_matrix(16, 5, seed=1)
    r = csc.rowidx.copy()
    r[0], r[1] = r[1], r[0]
    rc, msg = _load(lib, _mutate(csc, rowidx=r))
    assert rc == -1 and "sorted" in msg


def test_rejects_duplicate_rows(lib):
    csc = W.offset_matrix(16, 5, seed=1)
    r = csc.rowidx.copy()
    r[1] = r[0]
    rc, msg = _load(lib, _mutate(csc, rowidx=r))
    assert rc == -1


def test_rejects_negative_diagonal(lib):
    a = np.diag([1.0, -0.5, 0.7, 0.2])
    rc, msg = _load(lib, W.from_dense(a))
    assert rc == -1 and "diagonal" in msg


def test_rejects_value_above_one_after_scale(lib):
    csc = W.tiny_tridiagonal()[0]
    rc, msg = _load(lib, csc, scale=1.0)
    assert rc == -1 and "|a| > 1" in msg


def test_rejects_asymmetric(lib):
    a = np.array([[0.5, 0.2, 0], [0.1, 0.5, 0], [0, 0, 0.5]])
    rc, msg = _load(lib, W.from_dense(a))
    assert rc == -1 and "symmetric" in msg


def test_rejects_rows_longer_than_64(lib):
    a = np.full((80, 80), 0.01)
    rc, msg = _load(lib, W.from_dense(a))
    assert rc == -5


def test_rejects_row_index_out_of_range(lib):
    csc = W.offset_matrix(16, 5, seed=2)
    r = csc.rowidx.copy()
    r[-1] = 99
    rc, msg = _load(lib, _mutate(csc, rowidx=r))
    assert rc == -1


def _load_hermitian(lib, csc, flags=1, with_im=True, scale=None):
    h = ctypes.c_void_p()
    n = np.array([csc.n], np.int32)
    cp = np.ascontiguousarray(csc.colptr, np.int32)
    ri = np.ascontiguousarray(csc.rowidx, np.int32)
    re_ = np.ascontiguousarray(np.real(csc.vals), np.float64)
    im_ = np.ascontiguousarray(np.imag(csc.vals), np.float64)
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int32)
    rc = lib.qw_load_csc_hermitian(ctypes.byref(h), 1, n.ctypes.data_as(ip), None, None, cp.ctypes.data_as(ip),
                                   ri.ctypes.data_as(ip), re_.ctypes.data_as(dp),
                                   im_.ctypes.data_as(dp) if with_im else None,
                                   ctypes.byref(ctypes.c_double(scale)) if scale else None, flags, None, None)
    return rc, lib.qw_last_error().decode()


def test_hermitian_loader_validation(lib):
    csc = W.hermitian_offset_matrix(16, 5, seed=3)
    # a mirrored pair that is equal instead of conjugate
    d = csc.dense()
    k = np.argwhere(np.abs(d.imag) > 0)[0]
    bad = d.copy()
    bad[k[1], k[0]] = d[k[0], k[1]]
    rc, msg = _load_hermitian(lib, W.from_dense(bad))
    assert rc == -1 and "Hermitian" in msg
    # an imaginary diagonal entry
    bad = d.copy()
    bad[2, 2] += 0.1j
    rc, msg = _load_hermitian(lib, W.from_dense(bad))
    assert rc == -1 and "diagonal" in msg
    # |a| > 1 measured as the modulus (each part alone is below 1)
    rc, msg = _load_hermitian(lib, W.from_dense(np.array([[0.5, 0.8 + 0.8j], [0.8 - 0.8j, 0.5]])), scale=1.0)
    assert rc == -1 and "|a| > 1" in msg
    rc, msg = _load_hermitian(lib, csc, with_im=False)
    assert rc == -1 and "vals_im" in msg


def test_rejects_keys_wider_than_64_bits(lib):
    """4 log2 N + 2 key bits (plus the instance bits of a batch) must fit 64:
    N = 65536 does not (66 bits); eight instances of N = 32768 do not either
    (3 + 62)."""
    from paper_2303_06890_amd import _lib

    big = W.Csc(65536, np.arange(65537, dtype=np.int32), np.arange(65536, dtype=np.int32), np.full(65536, 0.5))
    rc, msg = _load(lib, big)
    assert rc == -5 and "64 bits" in msg
    h = ctypes.c_void_p()
    n = np.full(8, 32768, np.int32)
    colptr = np.concatenate([np.arange(32769, dtype=np.int32)] * 8)
    rowidx = np.concatenate([np.arange(32768, dtype=np.int32)] * 8)
    vals = np.full(8 * 32768, 0.5)
    coff = (np.arange(8) * 32769).astype(np.int64)
    zoff = (np.arange(8) * 32768).astype(np.int64)
    ip, lp, dp = ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double)
    rc = lib.qw_load_csc_batched(ctypes.byref(h), 8, n.ctypes.data_as(ip), coff.ctypes.data_as(lp),
                                 zoff.ctypes.data_as(lp), colptr.ctypes.data_as(ip), rowidx.ctypes.data_as(ip),
                                 vals.ctypes.data_as(dp), None, 1, None, None)
    assert rc == -5 and "64 bits" in lib.qw_last_error().decode()


def test_fixed_point_load_validation(lib):
    """Fixed-point data (QW_WORD_LENGTH): values must be words of the given
    length, the length at most 32, the matrix real.  All checked on the host
    before any device work."""
    from paper_2303_06890_amd import _lib

    csc = W.fixed_point_band(16, 2, 6, seed=1)
    rc, msg = _load(lib, csc, flags=1 | _lib.word_length(5))   # needs 6 bits
    assert rc == -1 and "fixed-point" in msg
    rc, msg = _load(lib, W.tiny_tridiagonal()[0], flags=1 | _lib.word_length(16))
    assert rc == -1 and "fixed-point" in msg
    rc, msg = _load(lib, csc, flags=1 | _lib.word_length(33))
    assert rc == -1 and "word length" in msg
    rc, msg = _load_hermitian(lib, W.hermitian_offset_matrix(16, 4, seed=1), flags=1 | _lib.word_length(8))
    assert rc == -5 and "real" in msg


def test_cks_coeffs_host(lib):
    """The library's coefficients (Stirling + ratio recurrence) agree with an
    exact rational evaluation and with the binomial tail."""
    from fractions import Fraction
    from math import comb

    from scipy.stats import binom

    import paper_2303_06890_amd as Q

    for beta, j0 in ((1, 0), (7, 4), (63, 20), (64, 20), (200, 50)):
        got = Q.cks_coeffs(beta, j0)
        ref = [float(4 * (-1) ** j * Fraction(sum(comb(2 * beta, beta + i) for i in range(j + 1, beta + 1)),
                                               4 ** beta)) for j in range(j0 + 1)]
        assert np.allclose(got, ref, rtol=1e-13, atol=0)
    beta, j0 = 966624, 4620
    got = Q.cks_coeffs(beta, j0)
    ks = np.array([0, 3, 50, 700, 3000, 4620])
    assert np.allclose(got[ks], 4 * (-1.0) ** ks * binom.sf(beta + ks, 2 * beta, 0.5), rtol=1e-9)


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    """Without the built library the binding raises at load: the walk has no
    CPU fallback."""
    from paper_2303_06890_amd import _lib

    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "libqw.so"))
    with pytest.raises(ImportError, match="no CPU fallback"):
        _lib.load()


def test_failing_allocator_reports_enomem(lib):
    """A caller's allocator that returns NULL: qw_load_csc reports QW_ENOMEM
    (after validating the matrix on the host) and leaks nothing it could
    free; the call neither throws nor aborts."""
    from paper_2303_06890_amd import _lib

    calls = []

    def alloc(nbytes, user):
        calls.append(int(nbytes))
        return None

    def free(p, user):
        raise AssertionError("nothing was allocated, nothing may be freed")

    a = _lib.QwAllocator(_lib.ALLOC_T(alloc), _lib.FREE_T(free), None)
    csc = W.offset_matrix(64, 5, seed=1)
    h = ctypes.c_void_p()
    cp = np.ascontiguousarray(csc.colptr, np.int32)
    ri = np.ascontiguousarray(csc.rowidx, np.int32)
    va = np.ascontiguousarray(csc.vals, np.float64)
    rc = lib.qw_load_csc(ctypes.byref(h), csc.n, cp.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                         ri.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                         va.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), csc.nnz, 0.0, 1, ctypes.byref(a), None)
    assert rc == _lib.QW_ENOMEM, lib.qw_last_error().decode()
    assert "allocation failed" in lib.qw_last_error().decode()
    assert h.value is None and len(calls) >= 1


def test_solver_and_kappa_argument_checks(lib):
    """qls_run / qw_kappa reject bad arguments before touching a context."""
    from paper_2303_06890_amd import _lib

    k = ctypes.c_double()
    assert lib.qw_kappa(None, 0, ctypes.byref(k)) == _lib.QW_EINVAL
    b = np.ones(4)
    bp = b.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    assert lib.qls_run(None, bp, 10.0, 1e-3, -1, None, None, None, None, None, None) == _lib.QW_EINVAL
    assert lib.qw_ctx_info(None, 0, None, None, None, None, ctypes.byref(k)) == _lib.QW_EINVAL


def test_gradient_argument_checks(lib):
    """The three gradient entry points reject a missing state or weight
    vector before touching the device."""
    from paper_2303_06890_amd import _lib

    w = np.ones(4)
    out = np.zeros(8)
    dp = ctypes.POINTER(ctypes.c_double)
    wp, op = w.ctypes.data_as(dp), out.ctypes.data_as(dp)
    loss = ctypes.c_double()
    assert lib.qw_grad(None, wp, 1, op, op, op, ctypes.byref(loss), None) == _lib.QW_EINVAL
    assert lib.qw_grad_noalloc(None, wp, 1, op, op, op, ctypes.byref(loss), None) == _lib.QW_EINVAL
    assert lib.qw_grad_complex(None, wp, 1, op, op, op, op, ctypes.byref(loss), None) == _lib.QW_EINVAL
    assert b"missing" in lib.qw_last_error()
