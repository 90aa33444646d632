"""Pins of the CPU oracle against what the paper and mathematics fix.

Every test here runs on the CPU.  None compares the oracle with itself: the
references are brute force, the dense state-vector simulator (an independent
formulation), closed forms (Chebyshev polynomials, eigenphases, the block
encoding A/s), unitarity, and the paper's worked examples.
"""

import numpy as np
import pytest

import workloads as W
from tests.conftest import load_golden
from tests.dense_sim import DenseWalk, preprocess


# ---------------------------------------------------------------- QBS, O_s'

def _definition_position(row, target):
    """Definition of QBS: the index of target in the sorted list, else 0."""
    for i, v in enumerate(row):
        if v == target:
            return i
    return 0


@pytest.mark.parametrize("s", list(range(1, 17)) + [31, 32, 33, 63, 64])
def test_qbs_brute_force(oracle_mod, s):
    rng = np.random.default_rng(100 + s)
    for _ in range(5):
        row = np.sort(rng.choice(4 * s + 8, size=s, replace=False))
        for target in range(-1, 4 * s + 10):
            assert oracle_mod.qbs(row, target if target >= 0 else 2**40) == \
                _definition_position(row, target if target >= 0 else 2**40)


def test_qbs_worked_example(oracle_mod):
    # row with nonzero columns {2, 5, 8, 10}, s = 4 (Sec. III.B, Fig. 3)
    row = [2, 5, 8, 10]
    assert oracle_mod.qbs(row, 5) == 1
    assert oracle_mod.qbs(row, 10) == 3
    assert oracle_mod.qbs(row, 3) == 0
    assert oracle_mod.qbs(row, 2) == 0


def _matrix_with_row(oracle_mod, row_cols, N=16):
    """Symmetric 0/1 pattern whose row 0 is exactly row_cols (s = len)."""
    a = np.zeros((N, N))
    for c in row_cols:
        a[0, c] = a[c, 0] = 0.5
    for j in range(1, N):
        a[j, j] = 0.5
    return W.from_dense(a)


def test_os_inverse_worked_example(oracle_mod):
    # O_s'^dagger on k = 0, k_c = 0 in a row {2, 5, 8, 10}: QBS misses, the
    # QRAM read at slot 0 gives column 2, so (l, z) = (0, 2)  (the appendix's
    # worked example; tests/golden/os_inverse_worked_example.json)
    g = load_golden("os_inverse_worked_example.json")
    csc = _matrix_with_row(oracle_mod, g["row"])
    m = oracle_mod.OracleMatrix(csc)
    col, _, _ = m.ell()
    assert list(col[0]) == g["row"]
    st = oracle_mod.OracleState(m, tau=0.0)
    key = oracle_mod.pack_key(m.nbits, 0, 0, 0, g["input"]["k_c"], g["input"]["k"], 0)
    st.import_(np.array([key], np.uint64), np.array([1.0 + 0j]))
    st.apply_op(oracle_mod.OP_OSINV)
    keys, _ = st.export()
    # k_c holds z, k holds l
    assert int(keys[0]) == oracle_mod.pack_key(m.nbits, 0, 0, 0, g["output"]["k_c"], g["output"]["k"], 0)
    # a valid input: k = 8 is slot 2 of row 0 -> (l, z) = (2, 0), the plain O_s
    st.import_(np.array([oracle_mod.pack_key(m.nbits, 0, 0, 0, 0, 8, 0)], np.uint64), np.array([1.0 + 0j]))
    st.apply_op(oracle_mod.OP_OSINV)
    keys, _ = st.export()
    assert int(keys[0]) == oracle_mod.pack_key(m.nbits, 0, 0, 0, 0, 2, 0)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_os_bijection_roundtrip(oracle_mod, seed):
    csc = W.offset_matrix(32, 5, seed=seed)
    m = oracle_mod.OracleMatrix(csc)
    N, s = m.N, m.s
    keys = np.array([oracle_mod.pack_key(m.nbits, 0, j, 0, z, l, 0)
                     for j in range(N) for l in range(s) for z in range(N)], np.uint64)
    amps = np.arange(1, keys.size + 1) * (1.0 + 0.5j)
    st = oracle_mod.OracleState(m, tau=0.0).import_(keys, amps)
    st.apply_op(oracle_mod.OP_OS)
    fk, fa = st.export()
    assert fk.size == keys.size  # injective on (l < s, z < N)
    kc = (fk.astype(np.int64) >> (m.nbits + 1)) & (N - 1)
    assert kc.max() < s  # image lands in k_c < s
    st.apply_op(oracle_mod.OP_OSINV)
    bk, ba = st.export()
    order = np.argsort(keys)
    assert np.array_equal(bk, keys[order]) and np.array_equal(ba, amps[order])
    # z = 0, l < s reproduces the plain sparsity oracle |j,l> -> |j,k_{j,l}>, k_c = 0
    col, _, _ = m.ell()
    j, l = 3, 1
    st.import_(np.array([oracle_mod.pack_key(m.nbits, 0, j, 0, 0, l, 0)], np.uint64), np.array([1.0 + 0j]))
    st.apply_op(oracle_mod.OP_OS)
    k1, _ = st.export()
    assert int(k1[0]) == oracle_mod.pack_key(m.nbits, 0, j, 0, 0, int(col[j, l]), 0)


# ---------------------------------------------------------------- preprocessing

def test_padding_rule(oracle_mod):
    csc = W.offset_matrix(16, 5, seed=3)  # 5 per column -> s = 8, 3 filler slots
    m = oracle_mod.OracleMatrix(csc)
    col, val, real = m.ell()
    assert m.s == 8 and m.N == 16
    dense = csc.dense() * m.scale
    for j in range(16):
        rows = set(csc.rowidx[csc.colptr[j]:csc.colptr[j + 1]])
        missing = [r for r in range(16) if r not in rows][:3]
        assert sorted(rows | set(missing)) == list(col[j])
        for l in range(8):
            if col[j, l] in rows:
                assert real[j, l] == 1 and val[j, l] == dense[col[j, l], j]
            else:
                assert real[j, l] == 0 and val[j, l] == 0.0
    assert np.abs(val).max() == pytest.approx(1.0)


def test_scale_and_pow2_n(oracle_mod):
    csc = W.offset_matrix(12, 3, seed=1)
    m = oracle_mod.OracleMatrix(csc)
    assert m.N == 16 and m.s == 4
    assert m.scale == pytest.approx(1.0 / np.abs(csc.vals).max())
    col, val, real = m.ell()
    assert np.all(val[12:] == 0) and np.all(real[12:] == 0)
    assert list(col[13]) == [0, 1, 2, 3]


# ---------------------------------------------------------------- dense simulator

def _oracle_dense(oracle_mod, st, shape):
    keys, amps = st.export()
    out = np.zeros(int(np.prod(shape)), complex)
    out[keys.astype(np.int64)] = amps
    return out


@pytest.mark.parametrize("case", ["tridiag16", "offset16_c5", "offset8_c4_raw"])
def test_oracle_matches_dense_simulator(oracle_mod, case):
    if case == "tridiag16":
        csc, b = W.tiny_tridiagonal()
        prep = True
    elif case == "offset16_c5":
        csc = W.offset_matrix(16, 5, seed=7)
        b = W.gaussian_b(16, seed=8)
        prep = True
    else:
        csc = W.offset_matrix(8, 4, seed=9)
        b = W.gaussian_b(8, seed=10)
        prep = False
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
        o = _oracle_dense(oracle_mod, st, dw.shape)
        assert np.abs(o - psi).max() < 1e-14, (case, t)
        # every branch the dense vector holds above rounding level is in the oracle
        assert np.all(np.abs(psi[o == 0]) < 1e-15)


def test_dense_wdag_and_tdag(oracle_mod):
    csc = W.offset_matrix(16, 5, seed=11)
    b = W.gaussian_b(16, seed=12)
    dw = DenseWalk(csc)
    m = oracle_mod.OracleMatrix(csc)
    st = oracle_mod.OracleState(m, tau=0.0).set_b(b).T().step(4)
    psi = _oracle_dense(oracle_mod, st, dw.shape)
    st.step_adjoint(1)
    ref = dw.T(dw.P(dw.Tdag(dw.S(psi))))  # W^dagger = T~ P T~^dagger S, S applied first
    assert np.abs(_oracle_dense(oracle_mod, st, dw.shape) - ref).max() < 1e-14


# ---------------------------------------------------------------- closed forms

def _cheb_reference(csc, b, nmax):
    N, nbits, s, scale, col, val = preprocess(csc)
    A = np.zeros((N, N))
    A[:csc.n, :csc.n] = csc.dense() * scale
    H = A / s
    bb = np.zeros(N)
    bb[:len(b)] = b
    out = [bb.copy(), H @ bb]
    for _ in range(2, nmax + 1):
        out.append(2 * H @ out[-1] - out[-2])
    return out


@pytest.mark.parametrize("case", ["tridiag16", "offset64_c5", "offset64_c8", "offset32_c3"])
def test_chebyshev_identity(oracle_mod, case):
    """T~^dagger W^n T~ on the |j~> block equals T_n(A/s) (Sec. IV, CKS paragraph)."""
    if case == "tridiag16":
        csc, b = W.tiny_tridiagonal()
    elif case == "offset64_c5":
        csc, b = W.offset_matrix(64, 5, seed=21), W.gaussian_b(64, seed=22)
    elif case == "offset64_c8":
        csc, b = W.offset_matrix(64, 8, seed=23), W.uniform_b(64)
    else:
        csc, b = W.offset_matrix(32, 3, seed=24), W.basis_b(32, 5)
    ref = _cheb_reference(csc, b, 16)
    m = oracle_mod.OracleMatrix(csc)
    st = oracle_mod.OracleState(m, tau=0.0).set_b(b).T()
    y0 = st.project0()
    assert np.abs(y0 - ref[0]).max() < 1e-15
    for n in range(1, 17):
        st.step(1)
        assert np.abs(st.project0() - ref[n]).max() < 2e-15, n


def test_block_encoding(oracle_mod):
    """<k~| T~^dagger S T~ |j~> = A_kj / s, negative off-diagonals included."""
    csc = W.offset_matrix(16, 5, seed=31)
    N, nbits, s, scale, col, val = preprocess(csc)
    A = csc.dense() * scale
    m = oracle_mod.OracleMatrix(csc)
    got = np.zeros((16, 16), complex)
    for j in range(16):
        st = oracle_mod.OracleState(m, tau=0.0).set_b(W.basis_b(16, j)).T()
        st.apply_op(oracle_mod.OP_S)
        got[:, j] = st.project0()
    assert np.abs(got - A / s).max() < 1e-15
    assert np.any(A < 0)


def test_eigenphase_relation(oracle_mod):
    """W^2 T~|lam> = 2 lam W T~|lam> - T~|lam> for eigenpairs of A/s, i.e. the
    walk rotates span{T~|lam>, S T~|lam>} by e^{+-i arccos lam}."""
    csc = W.offset_matrix(16, 4, seed=41)
    N, nbits, s, scale, col, val = preprocess(csc)
    H = csc.dense() * scale / s
    lam, vec = np.linalg.eigh(H)
    m = oracle_mod.OracleMatrix(csc)
    for idx in (0, 7, 15):
        st0 = oracle_mod.OracleState(m, tau=0.0).set_b(vec[:, idx]).T()
        st1 = st0.clone().step(1)
        st2 = st1.clone().step(1)
        size = 1 << (4 * m.nbits + 2)
        d0 = np.zeros(size, complex)
        d1 = np.zeros(size, complex)
        d2 = np.zeros(size, complex)
        for st, d in ((st0, d0), (st1, d1), (st2, d2)):
            k, a = st.export()
            d[k.astype(np.int64)] = a
        assert np.abs(d2 - (2 * lam[idx] * d1 - d0)).max() < 1e-14


# ---------------------------------------------------------------- unitarity, sizes

def test_unitarity_and_roundtrip(oracle_mod):
    csc = W.offset_matrix(64, 6, seed=51)
    b = W.gaussian_b(64, seed=52)
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


def test_branch_count_invariant(oracle_mod):
    """From T~|b~> the state stays within 4 N s branches; with an unpadded
    symmetric pattern the steady count is 3 N s - (number of |a| = 1 entries) - 1."""
    csc = W.offset_matrix(256, 8, seed=61)
    m = oracle_mod.OracleMatrix(csc)
    st = oracle_mod.OracleState(m).set_b(W.uniform_b(256)).T()
    Ns = m.N * m.s
    assert st.count() == 2 * Ns - 1  # one slot has |a| = 1 exactly, so g = 0
    for _ in range(8):
        st.step(1)
        assert st.count() <= 4 * Ns
    assert st.count() == 3 * Ns - 2


def test_raw_single_column_start_is_degenerate(oracle_mod):
    csc = W.offset_matrix(64, 8, seed=71)
    m = oracle_mod.OracleMatrix(csc)
    st = oracle_mod.OracleState(m).set_b(W.basis_b(64, 3))
    for _ in range(5):
        st.step(1)
        assert st.count() == 1
