"""Pins of the oracle for fixed-point matrix data (no GPU).

The paper's matrix elements are fixed-point numbers of a given word length
(Sec. V.B), and the conditional rotation of T~ is computed from the QRAM word
with a fixed-point square root, a fixed-point arccos and a rotation by a
fixed-point angle (appendix table of basic operations).  The reading taken
here: the square-root register holds sqrt(q / 2^w) truncated to w fraction
bits, the angle register the arccos of that in units of (pi/2) / 2^w rounded
to the nearest integer, and the rotation is by that angle.

Each pin fixes a part without comparing the oracle with itself: the integer
square root by its bracket, the angle register by its distance to the exact
arccos and by exact special values, the rotation by unitarity, monotonicity,
the sign rule and the error bound of the approximation; the walk by an
independent dense state-vector simulation, the block encoding (within the
fixed-point error bound of A), the Chebyshev structure of the walk,
unitarity and the limit of long words."""
import math

import numpy as np
import pytest

import workloads as W
from tests.dense_sim import DenseWalk

SIGN = 1 << 63


def _bound(w):
    """|cos^2(theta_q) - a| <= (2 + pi/4) 2^-w: the truncated root gives
    |r^2 - a| <= 2 * 2^-w, the rounded angle |d cos^2| <= (1/2) |d theta|
    <= (pi/4) 2^-w."""
    return (2.0 + math.pi / 4.0) * 2.0 ** -w


@pytest.mark.parametrize("w", [1, 2, 7, 12])
def test_square_root_register_is_truncated_root(oracle_mod, w):
    for q in range(1 << w):
        r = oracle_mod.fx_sqrt(q, w)
        assert r * r <= (q << w) < (r + 1) * (r + 1), (q, r)


def test_square_root_register_wide_words(oracle_mod):
    rng = np.random.default_rng(0)
    w = 32
    for q in [0, 1, 2, (1 << w) - 1, (1 << w) - 2, 1 << (w - 2)] + [int(x) for x in rng.integers(1, 1 << w, 200)]:
        r = oracle_mod.fx_sqrt(q, w)
        assert r * r <= (q << w) < (r + 1) * (r + 1), (q, r)
    assert oracle_mod.fx_sqrt(1 << (w - 2), w) == 1 << (w - 1)  # sqrt(1/4) = 1/2 exactly


@pytest.mark.parametrize("w", [3, 8, 12])
def test_angle_register_is_nearest(oracle_mod, w):
    unit = (math.pi / 2) / (1 << w)
    for r in range(1 << w):
        t = oracle_mod.fx_arccos(r, w)
        assert 0 <= t <= (1 << w)
        assert abs(t * unit - math.acos(r / (1 << w))) <= 0.5 * unit * (1 + 1e-12), (r, t)
    assert oracle_mod.fx_arccos(0, w) == 1 << w              # arccos 0 = pi/2
    assert oracle_mod.fx_arccos(1 << (w - 1), w) == round((1 << (w + 1)) / 3)  # arccos 1/2 = pi/3


@pytest.mark.parametrize("w", [4, 8, 10])
def test_rotation_unitary_monotone_and_bounded(oracle_mod, w):
    prev = -1.0
    for q in range(1 << w):
        f, g = oracle_mod.fx_rotation(q, w, 0, 1)
        a = q / (1 << w)
        assert f.imag == 0.0 and f.real >= 0.0 and g >= 0.0
        assert abs(f.real ** 2 + g * g - 1.0) < 5e-16
        assert abs(f.real ** 2 - a) <= _bound(w), (q, f)
        assert f.real >= prev  # cos of a non-increasing angle
        prev = f.real


def test_rotation_special_values(oracle_mod):
    for w in (1, 8, 16, 32):
        assert oracle_mod.fx_rotation(0, w, 3, 5) == (0j, 1.0)          # filler: f = 0, g = 1
        assert oracle_mod.fx_rotation(SIGN, w, 3, 5) == (0j, 1.0)
    # a = 1/4: r = 1/2 exactly, theta within half a unit of pi/3
    for w in (8, 16, 32):
        f, g = oracle_mod.fx_rotation(1 << (w - 2), w, 0, 0)
        dtheta = 0.5 * (math.pi / 2) / (1 << w)
        assert abs(f.real - 0.5) <= math.sin(math.pi / 3) * dtheta * (1 + 1e-9)
        assert abs(g - math.sqrt(0.75)) <= 0.5 * dtheta * (1 + 1e-9)


def test_rotation_sign_rule(oracle_mod):
    for w in (6, 16):
        for q in (1, 5, (1 << w) - 1):
            fp, gp = oracle_mod.fx_rotation(q, w, 2, 4)
            lo, glo = oracle_mod.fx_rotation(SIGN | q, w, 2, 4)   # row <= column: +i
            hi, ghi = oracle_mod.fx_rotation(SIGN | q, w, 4, 2)   # row > column: -i
            eq, geq = oracle_mod.fx_rotation(SIGN | q, w, 3, 3)
            assert lo == 1j * fp and hi == -1j * fp and eq == 1j * fp
            assert gp == glo == ghi == geq


def test_long_words_approach_the_exact_rotation(oracle_mod):
    rng = np.random.default_rng(1)
    w = 32
    for q in rng.integers(1, 1 << w, 100):
        a = int(q) / 2.0 ** w
        f, g = oracle_mod.fx_rotation(int(q), w, 0, 1)
        assert abs(f.real - math.sqrt(a)) < 3e-5 and abs(g - math.sqrt(1 - a)) < 3e-5
        assert abs(f.real ** 2 - a) <= _bound(w)


def test_word_validation(oracle_mod):
    csc = W.fixed_point_band(16, 2, 6, seed=1)
    oracle_mod.OracleMatrix(csc, word=6)
    oracle_mod.OracleMatrix(csc, word=9)        # q / 2^6 is also a 9-bit word
    with pytest.raises(RuntimeError, match="fixed-point"):
        oracle_mod.OracleMatrix(csc, word=5)    # needs 6 bits
    with pytest.raises(RuntimeError, match="word length"):
        oracle_mod.OracleMatrix(csc, word=33)
    with pytest.raises(RuntimeError, match="fixed-point"):
        oracle_mod.OracleMatrix(W.tridiagonal(16, seed=1), word=16)
    with pytest.raises(RuntimeError, match="real"):
        oracle_mod.OracleMatrix(W.hermitian_offset_matrix(16, 4, seed=1), word=8)


def _dense(st, shape):
    keys, amps = st.export()
    out = np.zeros(int(np.prod(shape)), complex)
    out[keys.astype(np.int64)] = amps
    return out


@pytest.mark.parametrize("n,bw,w,neg,prep", [(8, 1, 6, 0.0, True), (16, 2, 8, 0.5, True),
                                             (16, 1, 10, 0.5, False), (8, 2, 3, 0.3, True)])
def test_fixed_point_walk_matches_dense_simulator(oracle_mod, n, bw, w, neg, prep):
    csc = W.fixed_point_band(n, bw, w, seed=n + w, negative=neg)
    b = W.gaussian_b(n, seed=w)
    dw = DenseWalk(csc, word=w)
    m = oracle_mod.OracleMatrix(csc, word=w)
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


def _block(oracle_mod, m, n):
    """<k~| T~^dagger S T~ |j~> for every j, k."""
    got = np.zeros((n, n), complex)
    for j in range(n):
        st = oracle_mod.OracleState(m, tau=0.0).set_b(W.basis_b(n, j)).T()
        st.apply_op(oracle_mod.OP_S)
        got[:, j] = st.project0()[:n]
    return got


@pytest.mark.parametrize("w,neg", [(4, 0.0), (8, 0.5), (12, 0.5)])
def test_fixed_point_block_encoding_within_bound(oracle_mod, w, neg):
    """The walk block-encodes a symmetric A' with |A' - A| <= (2 + pi/4) 2^-w
    entrywise and the sparsity pattern of A."""
    n = 16
    csc = W.fixed_point_band(n, 2, w, seed=w, negative=neg)
    A = csc.dense()
    m = oracle_mod.OracleMatrix(csc, word=w)
    Ap = _block(oracle_mod, m, n) * m.s
    assert np.abs(Ap.imag).max() < 1e-15
    assert np.abs(Ap - Ap.T).max() < 1e-15
    assert np.array_equal(Ap.real != 0, A != 0)
    err = np.abs(Ap.real - A).max()
    assert 0 < err <= _bound(w)
    assert np.array_equal(np.sign(Ap.real), np.sign(A))


@pytest.mark.parametrize("w", [5, 8])
def test_fixed_point_chebyshev_structure(oracle_mod, w):
    """Pi_0 T~^dagger W^n T~ = T_n(H) with H = Pi_0 T~^dagger W T~ read off the
    walk itself (its block encoding), for n up to 16."""
    n = 16
    csc = W.fixed_point_band(n, 3, w, seed=20 + w, negative=0.4)
    m = oracle_mod.OracleMatrix(csc, word=w)
    H = np.zeros((n, n), complex)
    for j in range(n):
        H[:, j] = oracle_mod.OracleState(m, tau=0.0).set_b(W.basis_b(n, j)).T().step(1).project0()[:n]
    b = W.gaussian_b(n, seed=w)
    ref = [b.astype(complex), H @ b]
    for _ in range(2, 17):
        ref.append(2 * H @ ref[-1] - ref[-2])
    st = oracle_mod.OracleState(m, tau=0.0).set_b(b).T()
    for k in range(1, 17):
        st.step(1)
        assert np.abs(st.project0()[:n] - ref[k]).max() < 4e-15, k
    assert np.abs(H - H.conj().T).max() < 1e-15


def test_fixed_point_unitarity_and_roundtrip(oracle_mod):
    csc = W.fixed_point_band(64, 3, 8, seed=5, negative=0.3)
    b = W.gaussian_b(64, seed=6)
    m = oracle_mod.OracleMatrix(csc, word=8)
    st = oracle_mod.OracleState(m).set_b(b).T()
    k0, a0 = st.export()
    for _ in range(20):
        st.step(1)
        assert abs(st.norm2() - 1.0) < 1e-14
    st.step_adjoint(20)
    k1, a1 = st.export()
    assert np.array_equal(k0, k1)
    assert np.abs(a0 - a1).max() < 1e-14


def test_long_words_approach_the_real_valued_walk(oracle_mod):
    """With 32-bit words the fixed-point walk stays within the accumulated
    approximation error of the walk on the same values taken as FP64."""
    csc = W.fixed_point_band(32, 3, 32, seed=7, negative=0.3)
    b = W.gaussian_b(32, seed=8)
    fx = oracle_mod.OracleState(oracle_mod.OracleMatrix(csc, word=32), tau=0.0).set_b(b).T()
    fl = oracle_mod.OracleState(oracle_mod.OracleMatrix(csc), tau=0.0).set_b(b).T()
    for _ in range(10):
        fx.step(1)
        fl.step(1)
    size = 1 << (4 * 5 + 2)
    d = np.abs(_dense(fx, (size,)) - _dense(fl, (size,))).max()
    assert 0 < d < 1e-6


def test_classical_series_refuses_fixed_point_data(oracle_mod):
    csc = W.fixed_point_band(16, 1, 8, seed=1)
    m = oracle_mod.OracleMatrix(csc, word=8)
    with pytest.raises(RuntimeError, match="fixed-point"):
        m.cheb_series(W.uniform_b(16), 2, np.ones(3))
