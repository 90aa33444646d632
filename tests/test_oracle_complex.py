"""Pins of the oracle for complex Hermitian matrices (no GPU).

With a complex value the QRAM row j holds A*_{jk} of a Hermitian A and the
rotation takes f = sqrt(A*_{jk}) (the principal root, Sec. IV; the footnote's
+-i rule stays on the negative real axis).  Each pin fixes the walk without
comparing the oracle with itself: an independent dense state-vector
simulation, the block encoding, the Chebyshev closed form and the eigenphase
relation of the walk (Sec. IV, CKS paragraph), unitarity, and the classical
series and the walk-based solver against each other and against LU."""
import numpy as np
import pytest

import workloads as W
from tests.dense_sim import DenseWalk, preprocess


def _dense(st, shape):
    keys, amps = st.export()
    out = np.zeros(int(np.prod(shape)), complex)
    out[keys.astype(np.int64)] = amps
    return out


def _scaled_dense(csc):
    N, nbits, s, scale, col, val = preprocess(csc)
    A = np.zeros((N, N), complex)
    A[:csc.n, :csc.n] = csc.dense() * scale
    return A, s


def test_generator_is_hermitian_with_negative_real_entries():
    a = W.hermitian_offset_matrix(32, 6, seed=1).dense()
    assert np.array_equal(a, a.conj().T)
    off = a[~np.eye(32, dtype=bool)]
    assert np.any((off.imag == 0) & (off.real < 0)) and np.any(off.imag != 0)


@pytest.mark.parametrize("n,c,seed,prep", [(16, 5, 3, True), (8, 4, 4, False), (16, 4, 5, True)])
def test_complex_matches_dense_simulator(oracle_mod, n, c, seed, prep):
    csc = W.hermitian_offset_matrix(n, c, seed=seed)
    b = W.gaussian_b(n, seed=seed + 1) * np.exp(0.3j * np.arange(n))
    dw = DenseWalk(csc)
    m = oracle_mod.OracleMatrix(csc)
    assert (m.N, m.s) == (dw.N, dw.s)
    psi = dw.basis_b(b)
    st = oracle_mod.OracleState(m, tau=0.0).set_b(b)
    if prep:
        psi = dw.T(psi)
        st.T()
    for t in range(10):
        psi = dw.W(psi)
        st.step(1)
        o = _dense(st, dw.shape)
        assert np.abs(o - psi).max() < 1e-14, t
        assert np.all(np.abs(psi[o == 0]) < 1e-15)


def test_complex_block_encoding(oracle_mod):
    """<k~| T~^dagger S T~ |j~> = A_kj / s for a complex Hermitian A."""
    csc = W.hermitian_offset_matrix(16, 5, seed=6)
    A, s = _scaled_dense(csc)
    m = oracle_mod.OracleMatrix(csc)
    got = np.zeros((16, 16), complex)
    for j in range(16):
        st = oracle_mod.OracleState(m, tau=0.0).set_b(W.basis_b(16, j)).T()
        st.apply_op(oracle_mod.OP_S)
        got[:, j] = st.project0()
    assert np.abs(got - A / s).max() < 1e-15
    assert np.abs(A.imag).max() > 0.1


@pytest.mark.parametrize("n,c,seed", [(16, 5, 7), (64, 7, 8), (32, 4, 9)])
def test_complex_chebyshev_identity(oracle_mod, n, c, seed):
    """Pi_0 T~^dagger W^n T~ |b~> = T_n(A/s) b (three-term recurrence on the
    dense matrix)."""
    csc = W.hermitian_offset_matrix(n, c, seed=seed)
    A, s = _scaled_dense(csc)
    H = A / s
    b = W.gaussian_b(n, seed=seed) * np.exp(0.7j * np.arange(n))
    ref = [b.astype(complex), H @ b]
    for _ in range(2, 17):
        ref.append(2 * H @ ref[-1] - ref[-2])
    m = oracle_mod.OracleMatrix(csc)
    st = oracle_mod.OracleState(m, tau=0.0).set_b(b).T()
    assert np.abs(st.project0() - ref[0]).max() < 1e-15
    for k in range(1, 17):
        st.step(1)
        assert np.abs(st.project0() - ref[k]).max() < 2e-15, k


def test_complex_eigenphase_relation(oracle_mod):
    csc = W.hermitian_offset_matrix(16, 4, seed=10)
    A, s = _scaled_dense(csc)
    lam, vec = np.linalg.eigh(A / s)
    m = oracle_mod.OracleMatrix(csc)
    size = 1 << (4 * m.nbits + 2)
    for idx in (0, 9, 15):
        st0 = oracle_mod.OracleState(m, tau=0.0).set_b(vec[:, idx]).T()
        st1 = st0.clone().step(1)
        st2 = st1.clone().step(1)
        d = []
        for st in (st0, st1, st2):
            v = np.zeros(size, complex)
            k, a = st.export()
            v[k.astype(np.int64)] = a
            d.append(v)
        assert np.abs(d[2] - (2 * lam[idx] * d[1] - d[0])).max() < 1e-14


def test_complex_unitarity_and_roundtrip(oracle_mod):
    csc = W.hermitian_offset_matrix(64, 6, seed=11)
    b = W.gaussian_b(64, seed=12) * (1 - 0.5j)
    b = b / np.linalg.norm(b)
    m = oracle_mod.OracleMatrix(csc)
    st = oracle_mod.OracleState(m).set_b(b).T()
    k0, a0 = st.export()
    for _ in range(20):
        st.step(1)
        assert abs(st.norm2() - 1.0) < 1e-14
    st.step_adjoint(20)
    k1, a1 = st.export()
    assert np.array_equal(k0, k1)
    assert np.abs(a0 - a1).max() < 1e-14


def test_complex_series_and_walk_solver(oracle_mod):
    """The oracle's classical series equals the dense recurrence, the
    walk-based solver equals the series, and with enough terms the series
    approaches A^-1 b (shifted so that A/s is well conditioned)."""
    csc = W.hermitian_offset_matrix(32, 5, seed=13)
    A, s = _scaled_dense(csc)
    H = A / s
    lam = np.linalg.eigvalsh(H)
    kappa = 1.0 / np.abs(lam).min()
    b = W.gaussian_b(32, seed=14)
    beta, j0 = oracle_mod.schedule(kappa, 1e-3)
    coef = oracle_mod.cks_coeffs(beta, j0)
    m = oracle_mod.OracleMatrix(csc)
    y = m.cheb_series(b, j0, coef)
    t = [b.astype(complex), H @ b]
    ref = coef[0] * t[1]
    for k in range(1, j0 + 1):
        for _ in range(2):
            t = [t[1], 2 * H @ t[1] - t[0]]
        ref = ref + coef[k] * t[1]
    assert np.abs(y - ref).max() < 1e-10 * np.abs(ref).max()
    yw = m.qls_walk(b, j0, coef)
    assert np.abs(yw - y).max() < 1e-10 * np.abs(y).max()
    x = np.linalg.solve(H, b)
    fid = abs(np.vdot(x / np.linalg.norm(x), y / np.linalg.norm(y))) ** 2
    assert fid > 1 - 1e-4
