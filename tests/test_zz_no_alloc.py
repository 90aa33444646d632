"""qw_grad_noalloc (the gradient on the library's own device array, no
allocation) against qw_grad, through the C ABI: two calls in a row, the
second on a smaller matrix, each equal to qw_grad's output entry by entry to
the gradient tests' bar (1e-8 relative plus the rounding floor); then a
context too large for the array is rejected."""
import ctypes

import numpy as np
import pytest

import workloads as W
from tests.test_gpu_grad import _close, _floor_db, _floor_dv

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def Q():
    import torch

    assert torch.cuda.is_available()
    import paper_2303_06890_amd as Q

    return Q


def _call(Q, fn_name, st, w, nsteps, nnz, n):
    from paper_2303_06890_amd import _lib

    lib = _lib.load()
    dv, dbr, dbi = np.zeros(nnz), np.zeros(n), np.zeros(n)
    loss = ctypes.c_double()
    dp = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    rc = getattr(lib, fn_name)(st._h, dp(np.ascontiguousarray(w, np.float64)), int(nsteps), dp(dv), dp(dbr), dp(dbi),
                               ctypes.byref(loss), ctypes.c_void_p(Q.stream().cuda_stream))
    return rc, lib.qw_last_error().decode(), loss.value, dv, dbr + 1j * dbi


def _case(Q, n, c, seed, nsteps):
    a = W.offset_matrix(n, c, seed=seed)
    a = W.Csc(a.n, a.colptr, a.rowidx, a.vals / np.abs(a.vals).max())
    b = W.uniform_b(n)
    w = np.zeros(n)
    w[np.random.default_rng(seed).choice(n, size=n // 16, replace=False)] = 1.0
    walk = Q.Walk(a, scale=1.0)
    out = []
    for fn in ("qw_grad", "qw_grad_noalloc"):
        st = walk.state(b).step(nsteps)
        assert st.stats()["real_amplitudes"]
        rc, msg, loss, dv, db = _call(Q, fn, st, w, nsteps, a.nnz, n)
        assert rc == 0, (fn, msg)
        out.append((loss, dv, db))
        st.close()
    (l1, dv1, db1), (l2, dv2, db2) = out
    assert l2 == pytest.approx(l1, rel=1e-13)
    s = walk.info[0]["s"]
    _close(dv2, dv1, _floor_dv(a.vals, s, nsteps), where=f"dvals n={n}")
    _close(db2, db1, _floor_db(s, nsteps), where=f"db n={n}")
    return np.array_equal(np.nan_to_num(dv1, nan=7.0), np.nan_to_num(dv2, nan=7.0))


def test_noalloc_gradient_equals_qw_grad_twice(Q):
    # the first call fills the array for 16384 x 8; the second, smaller one
    # must not see its leftovers
    bitwise_big = _case(Q, 16384, 8, 41, 12)
    bitwise_small = _case(Q, 1024, 8, 42, 20)
    assert bitwise_big and bitwise_small  # the same kernels in the same order


def test_noalloc_rejects_what_it_cannot_hold(Q):
    # 2M slots (32768 columns x 64) need about 117 MB, more than the 32 MiB array
    n = 32768
    a = W.band_matrix(n, 31, seed=43)
    walk = Q.Walk(a)
    st = walk.state(W.uniform_b(n)).step(1)
    assert st.stats()["real_amplitudes"]
    rc, msg, *_ = _call(Q, "qw_grad_noalloc", st, np.ones(n), 1, a.nnz, n)
    assert rc == -1 and "bytes of the library's device array" in msg
    # and a state on the complex planes is turned away (complex b)
    small = W.offset_matrix(64, 6, seed=44)
    st2 = Q.Walk(small).state(W.gaussian_b(64, seed=45) * (1 + 0.5j)).step(3)
    rc, msg, *_ = _call(Q, "qw_grad_noalloc", st2, np.ones(64), 3, small.nnz, 64)
    assert rc == -5 and "one double per cell" in msg
