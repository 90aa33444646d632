"""The library's condition number of A/s (host code, qw_kappa.cpp) against
numpy's dense eigenvalues, on the CPU: the source is compiled here with a
small C shim (the library itself needs a GPU to load a matrix)."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import workloads as W
from dense_sim import preprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2303_06890_amd", "csrc")

SHIM = r'''
#include "qw_kappa.h"
#include <cstring>
#include <string>
extern "C" int kappa_shim(int n, int s, int nbits, const int* col, const double* val, const double* vim,
                          int angles, double* lam, char* err, int errlen) {
  std::string e;
  int rc = qw::min_abs_eigenvalue(n, s, nbits, col, val, vim, angles != 0, lam, e);
  std::strncpy(err, e.c_str(), errlen - 1);
  err[errlen - 1] = 0;
  return rc;
}
'''


@pytest.fixture(scope="module")
def shim(tmp_path_factory):
    d = tmp_path_factory.mktemp("kappa")
    (d / "shim.cpp").write_text(SHIM)
    lib = d / "libkappa.so"
    subprocess.run(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-pthread", "-I", CSRC, "-o", str(lib),
                    str(d / "shim.cpp"), os.path.join(CSRC, "qw_kappa.cpp")], check=True)
    f = ctypes.CDLL(str(lib)).kappa_shim
    f.restype = ctypes.c_int
    return f


def _kappa(shim, csc, angles=None):
    """(rc, min |lambda| of A/s, message) through the shim, from the QRAM
    table built by the preprocessing rule (fillers = smallest absent rows)."""
    N, nbits, s, scale, col, val = preprocess(csc)
    col = np.ascontiguousarray(col, np.int32)
    re = np.ascontiguousarray(np.real(val) if angles is None else angles, np.float64)
    vim = None
    if np.iscomplexobj(val):
        vim = np.ascontiguousarray(np.imag(val).T, np.float64)  # by home: (l << nbits) + j
    lam = ctypes.c_double()
    err = ctypes.create_string_buffer(512)
    rc = shim(csc.n, s, nbits, col.ctypes.data_as(ctypes.c_void_p), re.ctypes.data_as(ctypes.c_void_p),
              vim.ctypes.data_as(ctypes.c_void_p) if vim is not None else None, 0 if angles is None else 1,
              ctypes.byref(lam), err, 512)
    return rc, lam.value, err.value.decode(), (N, s, scale)


def _numpy_min_abs(csc):
    N, nbits, s, scale, col, val = preprocess(csc)
    H = csc.dense() * scale / s
    return np.abs(np.linalg.eigvalsh(H)).min()


@pytest.mark.parametrize("case", ["laplacian32", "offset64_c5", "tridiag16", "band_n300"])
def test_dense_path_matches_eigvalsh(shim, case):
    csc = {"laplacian32": lambda: W.solver_problem()[0],
           "offset64_c5": lambda: W.offset_matrix(64, 5, seed=3),  # indefinite, fillers
           "tridiag16": lambda: W.tiny_tridiagonal()[0],
           "band_n300": lambda: W.band_matrix(300, 3, seed=2)}[case]()  # n not a power of two
    rc, lam, err, _ = _kappa(shim, csc)
    assert rc == 0, err
    assert lam == pytest.approx(_numpy_min_abs(csc), rel=1e-11)


def test_laplacian_schedule(shim):
    """The solver workload's kappa and the schedule it implies (9241 walk
    steps at eps = 1e-3, the value the classical closed form gives)."""
    rc, lam, err, _ = _kappa(shim, W.solver_problem()[0])
    assert rc == 0, err
    kappa = 1 / lam
    assert kappa == pytest.approx(277.7017914659025, rel=1e-12)
    beta = np.ceil(kappa ** 2 * np.log(kappa / 1e-3))
    j0 = int(np.ceil(np.sqrt(beta * np.log(4 * beta / 1e-3))))
    assert 2 * j0 + 1 == 9241


def test_complex_hermitian(shim):
    csc = W.hermitian_offset_matrix(32, 5, seed=4)
    rc, lam, err, _ = _kappa(shim, csc)
    assert rc == 0, err
    assert lam == pytest.approx(_numpy_min_abs(csc), rel=1e-11)


def test_fixed_point_angles_encode_cos_squared(shim):
    """Fixed-point data: the table holds each slot's rotation angle y (units
    of pi) and the walk encodes sign(y) sin^2(pi |y|)."""
    csc = W.offset_matrix(32, 5, seed=5)
    N, nbits, s, scale, col, val = preprocess(csc)
    rng = np.random.default_rng(1)
    # a symmetric table of angles: the value of (j, col) equals that of (col, j)
    y = np.zeros_like(val)
    for j in range(N):
        for l in range(s):
            c = col[j, l]
            if val[j, l] != 0 and c >= j:
                a = np.sign(val[j, l]) * rng.uniform(0.05, 0.45)
                y[j, l] = a
                y[c, list(col[c]).index(j)] = a
    rc, lam, err, _ = _kappa(shim, csc, angles=y)
    assert rc == 0, err
    A = np.zeros((N, N))
    for j in range(N):
        for l in range(s):
            if y[j, l] != 0:
                A[col[j, l], j] = np.sign(y[j, l]) * np.sin(np.pi * abs(y[j, l])) ** 2
    assert lam == pytest.approx(np.abs(np.linalg.eigvalsh(A / s)).min(), rel=1e-11)


def test_lanczos_path(shim):
    """n = 4096 > 2048: the Lanczos estimate (5-point Laplacian on 64 x 64 +
    0.1 I, a definite matrix, so the iteration runs on A/s itself)."""
    csc = W.laplacian_2d(64, 0.1)
    rc, lam, err, _ = _kappa(shim, csc)
    assert rc == 0, err
    # closed form of the Dirichlet Laplacian's smallest eigenvalue
    m = 64
    lam_a = 0.1 + 2 * 4 * np.sin(np.pi / (2 * (m + 1))) ** 2
    N, nbits, s, scale, col, val = preprocess(csc)
    assert lam == pytest.approx(lam_a * scale / s, rel=1e-7)


def test_rejects_unsymmetric_and_singular(shim):
    a = np.array([[1.0, 0.5, 0.0], [0.2, 1.0, 0.0], [0.0, 0.0, 1.0]])
    rc, _, err, _ = _kappa(shim, W.from_dense(a))
    assert rc == -5 and "symmetric" in err
    b = np.array([[1.0, 1.0], [1.0, 1.0]])
    rc, _, err, _ = _kappa(shim, W.from_dense(b))
    assert rc == -1 and "singular" in err


def test_dense_path_does_not_depend_on_the_thread_count(shim):
    """The dense reduction shares its rows among as many threads as the
    calling thread may run on, in fixed chunks summed in a fixed order: one
    CPU or all of them give the same bits."""
    csc = W.offset_matrix(512, 6, seed=9)  # 512 rows: the threaded reduction
    saved = os.sched_getaffinity(0)
    try:
        os.sched_setaffinity(0, {min(saved)})
        rc1, lam1, err1, _ = _kappa(shim, csc)
    finally:
        os.sched_setaffinity(0, saved)
    rc2, lam2, err2, _ = _kappa(shim, csc)
    assert rc1 == 0 and rc2 == 0, (err1, err2)
    assert lam1 == lam2
    assert lam1 == pytest.approx(_numpy_min_abs(csc), rel=1e-11)
