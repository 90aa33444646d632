"""Pins of the oracle's reverse-mode gradient for complex Hermitian matrices
(no GPU).

The walk takes f = sqrt(A*_{jk}) of the value a + i b a QRAM row holds (the
principal root off the real axis, the +-i rule on the negative real axis;
Sec. IV) and g = sqrt(1 - |a + i b|).  The gradient of L = sum_j w_j p_j
comes out per stored entry as dL/da + i dL/db, each entry an independent
parameter.  It is pinned by central differences of the oracle's own forward
walk (a different computation: no stored states, no reverse pass) and by
torch autograd through the independent dense simulator."""
import numpy as np
import pytest

import workloads as W
from tests.dense_sim import torch_loss

H = 1e-6


def _case():
    csc = W.hermitian_offset_matrix(16, 5, seed=91)
    scale = 1.0 / np.abs(csc.vals).max()
    csc = W.Csc(csc.n, csc.colptr, csc.rowidx, csc.vals * scale)
    b = W.gaussian_b(16, seed=92) * np.exp(1j * np.linspace(0.0, 2.0, 16))
    w = np.zeros(16)
    w[[0, 3, 7, 12]] = 1.0
    w[5] = 0.5
    return csc, b, w


def _csc_slot(m, csc):
    col, _, _ = m.ell()
    out = np.zeros(csc.nnz, np.int64)
    for c in range(csc.n):
        for p in range(csc.colptr[c], csc.colptr[c + 1]):
            out[p] = c * m.s + int(np.nonzero(col[c] == csc.rowidx[p])[0][0])
    return out


def _loss(oracle_mod, csc, b, w, nsteps):
    m = oracle_mod.OracleMatrix(csc, scale=1.0)
    st = oracle_mod.OracleState(m, tau=0.0).set_b(b).T().step(nsteps)
    return float(np.dot(st.j_marginal(), w))


def _fd(oracle_mod, csc, b, w, nsteps, p, d):
    vp, vm = csc.vals.copy(), csc.vals.copy()
    vp[p] += H * d
    vm[p] -= H * d
    lp = _loss(oracle_mod, W.Csc(csc.n, csc.colptr, csc.rowidx, vp), b, w, nsteps)
    lm = _loss(oracle_mod, W.Csc(csc.n, csc.colptr, csc.rowidx, vm), b, w, nsteps)
    return (lp - lm) / (2 * H)


def test_case_covers_the_three_kinds_of_entry():
    csc, _, _ = _case()
    v = csc.vals
    assert np.any(v.imag != 0)  # off the axis
    assert np.any((v.imag == 0) & (v.real > 0))  # positive axis (the diagonal)
    assert np.any((v.imag == 0) & (v.real < 0))  # the cut: +-i rule


def test_complex_grad_vs_central_differences(oracle_mod):
    csc, b, w = _case()
    nsteps = 5
    m = oracle_mod.OracleMatrix(csc, scale=1.0)
    loss, dv, db = m.grad(b, w, nsteps, tau=0.0)
    assert np.iscomplexobj(dv)
    assert loss == pytest.approx(_loss(oracle_mod, csc, b, w, nsteps), abs=1e-15)
    g = dv.reshape(-1)[_csc_slot(m, csc)]
    v = csc.vals
    mod = np.abs(v)
    inner = (mod > 1e-4) & (mod < 1 - 1e-4)
    rng = np.random.default_rng(93)
    off = np.nonzero(inner & (v.imag != 0))[0]
    pos = np.nonzero(inner & (v.imag == 0) & (v.real > 0))[0]
    neg = np.nonzero(inner & (v.imag == 0) & (v.real < 0))[0]
    picks = list(rng.choice(off, 8, replace=False)) + list(rng.choice(pos, 3, replace=False)) \
        + list(rng.choice(neg, 3, replace=False))
    for p in picks:
        fd = _fd(oracle_mod, csc, b, w, nsteps, p, 1.0)
        assert abs(fd - g[p].real) <= 1e-8 * abs(g[p].real) + 1e-10, ("re", p)
        if p in neg:
            # on the cut the +-i rule is one side of the principal root's
            # jump: no derivative in the imaginary direction
            assert np.isnan(g[p].imag), p
            continue
        fd = _fd(oracle_mod, csc, b, w, nsteps, p, 1j)
        assert abs(fd - g[p].imag) <= 1e-8 * abs(g[p].imag) + 1e-10, ("im", p)
    for j in (1, 6, 14):
        for d in (1.0, 1j):
            bp, bm = b.copy(), b.copy()
            bp[j] += H * d
            bm[j] -= H * d
            fd = (_loss(oracle_mod, csc, bp, w, nsteps) - _loss(oracle_mod, csc, bm, w, nsteps)) / (2 * H)
            ref = db[j].real if d == 1.0 else db[j].imag
            assert abs(fd - ref) <= 1e-8 * abs(ref) + 1e-10


def test_complex_grad_vs_torch_autograd_on_dense(oracle_mod):
    csc, b, w = _case()
    nsteps = 4
    m = oracle_mod.OracleMatrix(csc, scale=1.0)
    loss, dv, db = m.grad(b, w, nsteps, tau=0.0)
    tl, tv, tb = torch_loss(csc, csc.vals, b, w, nsteps)
    tl.backward()
    assert loss == pytest.approx(float(tl.detach()), abs=1e-14)
    g = dv.reshape(-1)[_csc_slot(m, csc)]
    ref = tv.grad.numpy()  # torch's convention for a real loss: dL/dRe + i dL/dIm
    v = csc.vals
    edge = np.abs(v) == 1.0  # g = sqrt(1 - |v|) has no derivative at |v| = 1 (the entry the scale sets)
    assert 1 <= edge.sum() <= 2
    cut = (v.imag == 0) & (v.real < 0)
    assert np.all(np.isnan(g.imag[cut])) and np.all(np.isfinite(g.real[~edge]))
    ok = ~cut & ~edge
    assert np.all(np.isfinite(g.imag[ok]))
    assert np.allclose(g.real[~edge], ref.real[~edge], rtol=1e-9, atol=1e-12)
    assert np.allclose(g.imag[ok], ref.imag[ok], rtol=1e-9, atol=1e-12)
    assert np.allclose(db[:16], tb.grad.numpy(), rtol=1e-9, atol=1e-12)


def test_real_part_equals_the_real_gradient_on_a_real_matrix(oracle_mod):
    # a real symmetric matrix loaded with zero imaginary parts: dL/da is the
    # real gradient; dL/db exists for positive entries only
    csc = W.offset_matrix(16, 5, seed=81)
    scale = 1.0 / np.abs(csc.vals).max()
    real = W.Csc(csc.n, csc.colptr, csc.rowidx, csc.vals * scale)
    as_complex = W.Csc(csc.n, csc.colptr, csc.rowidx, (csc.vals * scale).astype(np.complex128))
    b = W.gaussian_b(16, seed=82)
    w = np.zeros(16)
    w[[1, 4, 9, 13]] = 1.0
    mr = oracle_mod.OracleMatrix(real, scale=1.0)
    mc = oracle_mod.OracleMatrix(as_complex, scale=1.0)
    if not mc.complex:
        pytest.skip("the oracle loads a zero imaginary part as a real matrix")
    lr, dvr, dbr = mr.grad(b, w, 4, tau=0.0)
    lc, dvc, dbc = mc.grad(b, w, 4, tau=0.0)
    assert lc == lr
    fin = np.isfinite(dvr)
    assert np.array_equal(dvc.real[fin], dvr[fin])
    assert np.array_equal(dbc, dbr)
