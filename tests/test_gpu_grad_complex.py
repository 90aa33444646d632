"""GPU reverse-mode gradient for complex Hermitian values (qw_grad_complex)
against the oracle's stored-state reverse mode, entry by entry, and against
central differences of the GPU's own forward walk; the autograd function with
complex values; the real and complex entry points refuse each other's
contexts."""
import ctypes

import numpy as np
import pytest

import workloads as W
from tests.test_gpu_grad import _close, _floor_db, _floor_dv, _scaled

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def Q():
    import torch

    assert torch.cuda.is_available()
    import paper_2303_06890_amd as Q

    return Q


def _oracle_csc_grad(oracle_mod, csc, b, w, nsteps):
    m = oracle_mod.OracleMatrix(csc, scale=1.0)
    loss, dv, db = m.grad(b, w, nsteps)
    col, _, _ = m.ell()
    g = np.zeros(csc.nnz, np.complex128)
    for c in range(csc.n):
        for p in range(csc.colptr[c], csc.colptr[c + 1]):
            g[p] = dv[c, int(np.nonzero(col[c] == csc.rowidx[p])[0][0])]
    return loss, g, db[:csc.n]


def _gpu(Q, csc, b, w, nsteps):
    walk = Q.Walk(csc, scale=1.0, symmetric=False)
    st = walk.state(b).step(nsteps)
    return st.grad(w, nsteps)


def _gpu_loss(Q, csc, b, w, nsteps):
    walk = Q.Walk(csc, scale=1.0, symmetric=False)
    st = walk.state(b).step(nsteps)
    return float(np.dot(st.j_marginal()[:csc.n], w))


def _check(csc, s, nsteps, g, o, gdb, odb, where):
    v = csc.vals
    cut = (v.imag == 0) & (v.real < 0)
    # where the oracle's derivative does not exist (the imaginary part on the
    # negative real axis, both parts at |v| = 1) the GPU's is not finite
    # either (the GPU also multiplies it by zero amplitudes, so it may be NaN
    # at a site the oracle never visits)
    assert not np.any(np.isfinite(g.real) & ~np.isfinite(o.real)), where
    assert not np.any(np.isfinite(g.imag) & ~np.isfinite(o.imag)), where
    assert np.all(np.isnan(g.imag[cut]))
    floor = _floor_dv(np.abs(v), s, nsteps)
    fr, wr, _ = _close(g.real, o.real, floor, where=where + " Re")
    fi, wi, _ = _close(g.imag, o.imag, floor, where=where + " Im")
    assert fr.sum() >= csc.nnz - 2 and fi.sum() >= csc.nnz - 2 - cut.sum()
    _close(gdb, odb, _floor_db(s, nsteps), where=where + " db")
    return max(wr, wi)


@pytest.mark.parametrize("n,c,seed,nsteps", [(16, 5, 101, 5), (64, 7, 102, 9), (64, 12, 103, 5), (256, 9, 104, 6)])
def test_complex_grad_matches_oracle(Q, oracle_mod, n, c, seed, nsteps):
    csc = _scaled(W.hermitian_offset_matrix(n, c, seed=seed))
    b = W.gaussian_b(n, seed=seed + 1) * np.exp(1j * np.linspace(0.0, 3.0, n))
    b = b / np.linalg.norm(b)
    w = np.zeros(n)
    w[np.random.default_rng(seed).choice(n, size=max(2, n // 4), replace=False)] = 1.0
    ol, og, odb = _oracle_csc_grad(oracle_mod, csc, b, w, nsteps)
    gl, gg, gdb = _gpu(Q, csc, b, w, nsteps)
    assert np.iscomplexobj(gg) and gg.shape == (csc.nnz,)
    assert gl == pytest.approx(ol, rel=1e-12)
    s = Q.Walk(csc, scale=1.0, symmetric=False).info[0]["s"]
    _check(csc, s, nsteps, gg, og, gdb, odb, f"n={n} c={c}")


def test_complex_grad_1024_vs_oracle_and_fd(Q, oracle_mod):
    """The complex counterpart of the adjoint workload: a complex Hermitian
    offset matrix n = 1024 with 8 entries per column, uniform b, 20 steps,
    loss over 32 seeded outcomes; every entry against the oracle, 8 entries
    in each direction against central differences (h = 1e-6)."""
    csc = _scaled(W.hermitian_offset_matrix(1024, 8, seed=4))
    b = W.uniform_b(1024)
    w = np.zeros(1024)
    w[np.random.default_rng(5).choice(1024, size=32, replace=False)] = 1.0
    nsteps = 20
    gl, gg, gdb = _gpu(Q, csc, b, w, nsteps)
    ol, og, odb = _oracle_csc_grad(oracle_mod, csc, b, w, nsteps)
    assert gl == pytest.approx(ol, rel=1e-12)
    worst = _check(csc, 8, nsteps, gg, og, gdb, odb, "n=1024")
    from tests import oracle_jobs

    oracle_jobs.record("grad_complex_1024", worst_ratio=worst,
                       max_abs_err_re=float(np.nanmax(np.abs(gg.real - og.real))),
                       max_abs_err_im=float(np.nanmax(np.abs(gg.imag - og.imag))))
    v = csc.vals
    rng = np.random.default_rng(6)
    inner = (np.abs(v) > 1e-4) & (np.abs(v) < 1 - 1e-4)
    h = 1e-6
    for d, pool in ((1.0, np.nonzero(inner)[0]), (1j, np.nonzero(inner & (v.imag != 0))[0])):
        for p in rng.choice(pool, size=8, replace=False):
            vp, vm = v.copy(), v.copy()
            vp[p] += h * d
            vm[p] -= h * d
            fd = (_gpu_loss(Q, W.Csc(csc.n, csc.colptr, csc.rowidx, vp), b, w, nsteps)
                  - _gpu_loss(Q, W.Csc(csc.n, csc.colptr, csc.rowidx, vm), b, w, nsteps)) / (2 * h)
            ref = gg[p].real if d == 1.0 else gg[p].imag
            assert abs(fd - ref) <= 1e-8 * abs(ref) + 1e-10, (p, d, fd, ref)


def test_walk_observable_complex_values(Q):
    import torch

    csc = _scaled(W.hermitian_offset_matrix(64, 6, seed=105))
    b = W.gaussian_b(64, seed=106) * (1 - 0.5j)
    w = np.random.default_rng(107).uniform(size=64)
    vals = torch.tensor(csc.vals, requires_grad=True)
    bt = torch.tensor(b, requires_grad=True)
    p = Q.WalkObservable.apply(vals, bt, csc, 7)
    loss = (p * torch.tensor(w)).sum()
    loss.backward()
    gl, gg, gdb = _gpu(Q, csc, b, w, 7)
    assert float(loss.detach()) == pytest.approx(gl, rel=1e-12)
    assert vals.grad.dtype == torch.complex128
    assert np.allclose(vals.grad.numpy(), gg, rtol=1e-12, atol=1e-14, equal_nan=True)
    assert np.allclose(bt.grad.numpy(), gdb, rtol=1e-12, atol=1e-14)


def test_entry_points_refuse_the_other_kind(Q):
    from paper_2303_06890_amd import _lib

    lib = _lib.load()
    dp = ctypes.POINTER(ctypes.c_double)
    out = np.zeros(4096)
    loss = ctypes.c_double()
    P = lambda a: a.ctypes.data_as(dp)  # noqa: E731
    real = _scaled(W.offset_matrix(64, 5, seed=108))
    cplx = _scaled(W.hermitian_offset_matrix(64, 5, seed=108))
    w = np.ones(64)
    for csc, fn in ((real, "qw_grad_complex"), (cplx, "qw_grad")):
        st = Q.Walk(csc, scale=1.0).state(W.uniform_b(64)).step(3)
        if fn == "qw_grad":
            rc = lib.qw_grad(st._h, P(w), 3, P(out), P(out), P(out), ctypes.byref(loss), None)
        else:
            rc = lib.qw_grad_complex(st._h, P(w), 3, P(out), P(out), P(out), P(out), ctypes.byref(loss), None)
        assert rc == -5, (fn, rc)  # QW_ENOTSUP
        assert b"takes" in lib.qw_last_error()
        st.close()


def test_complex_grad_batched_mixed_s(Q, oracle_mod):
    """Two complex Hermitian instances of different s in one context: each
    instance's part of the gradient equals the oracle's for that matrix alone."""
    mats = [_scaled(W.hermitian_offset_matrix(128, 6, seed=109)), _scaled(W.hermitian_offset_matrix(64, 11, seed=110))]
    bs = [W.uniform_b(128) * 1j, W.gaussian_b(64, seed=111) * (0.6 + 0.8j)]
    bs[1] = bs[1] / np.linalg.norm(bs[1])
    ws = [np.zeros(128), np.zeros(64)]
    ws[0][::5] = 1.0
    ws[1][1::3] = 1.0
    nsteps = 7
    walk = Q.Walk(mats, scale=1.0, symmetric=False)
    assert len({d["s"] for d in walk.info}) == 2
    st = walk.state(bs).step(nsteps)
    gl, gg, gdb = st.grad(np.concatenate(ws), nsteps)
    off, boff, total = 0, 0, 0.0
    for csc, b, w, d in zip(mats, bs, ws, walk.info):
        ol, og, odb = _oracle_csc_grad(oracle_mod, csc, b, w, nsteps)
        total += ol
        _check(csc, d["s"], nsteps, gg[off:off + csc.nnz], og, gdb[boff:boff + csc.n], odb, f"n={csc.n}")
        off += csc.nnz
        boff += csc.n
    assert gl == pytest.approx(total, rel=1e-12)
