"""GPU parity of the walk-based linear solver (qls_run) against the oracle."""
import numpy as np
import pytest

import workloads as W
from tests.dense_sim import preprocess

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def Q():
    import torch

    assert torch.cuda.is_available()
    import paper_2303_06890_amd as Q

    return Q


def _kappa(csc):
    N, nbits, s, scale, col, val = preprocess(csc)
    H = csc.dense() * scale / s
    return 1.0 / np.abs(np.linalg.eigvalsh(H)).min(), H


def test_qls_tiny_matches_oracle_walk_and_series(Q, oracle_mod):
    """kappa from the library (qw_kappa inside qls_run), checked against
    numpy's eigenvalues; the post-selected x and |y| against the oracle."""
    csc, _ = W.tiny_tridiagonal()
    b = W.gaussian_b(16, seed=3)
    kappa, H = _kappa(csc)
    beta, j0 = oracle_mod.schedule(kappa, 1e-2)
    coef = oracle_mod.cks_coeffs(beta, j0)
    m = oracle_mod.OracleMatrix(csc)
    y_series = m.cheb_series(b, j0, coef)
    y_walk = m.qls_walk(b, j0, coef)
    walk = Q.Walk(csc)
    assert np.isnan(walk.kappa_known())
    x, p_succ, steps, yn = walk.qls(b, eps=1e-2)
    assert walk.kappa_known() == pytest.approx(kappa, rel=1e-11)
    assert steps == 2 * j0 + 1
    assert np.linalg.norm(x) == pytest.approx(1.0, abs=1e-14)
    y = yn * x
    scale = np.abs(y_series).max()
    assert np.abs(y - y_walk).max() < 1e-12 * scale
    assert np.abs(y - y_series).max() < 1e-11 * scale
    assert p_succ == pytest.approx(np.dot(y_series, y_series) / np.abs(coef).sum() ** 2, rel=1e-9)


def test_qls_laplacian_32x32(Q, oracle_mod):
    """5-point Laplacian on 32x32 + 0.1 I, kappa from its closed-form spectrum,
    eps = 1e-3: 9241 walk steps; output equal to the oracle's truncated series,
    and its fidelity against the LU solution."""
    csc, b = W.solver_problem()
    lam = (0.1 + 4 - 4 * np.cos(np.pi / 33)) / 4.1 / 8
    kappa = 1.0 / lam
    k2, H = _kappa(csc)
    assert kappa == pytest.approx(k2, rel=1e-10)
    beta, j0 = oracle_mod.schedule(kappa, 1e-3)
    assert 2 * j0 + 1 == 9241
    coef = oracle_mod.cks_coeffs(beta, j0)
    y_ref = oracle_mod.OracleMatrix(csc).cheb_series(b, j0, coef)
    walk = Q.Walk(csc)
    assert walk.kappa(0) == pytest.approx(kappa, rel=1e-11)  # the library's own, then kept
    x, p_succ, steps, yn = walk.qls(b, eps=1e-3)
    assert steps == 9241
    y = yn * x
    assert np.abs(y.imag).max() < 1e-10
    assert np.abs(y - y_ref).max() <= 1e-10 * np.abs(y_ref).max()
    x = np.linalg.solve(H, b)
    fid = abs(np.vdot(x, y)) ** 2 / (np.vdot(x, x).real * np.vdot(y, y).real)
    assert fid > 1 - 1e-9
    assert 1e-4 < p_succ < 1e-3


@pytest.mark.parametrize("mixed", [False, True])
def test_qls_on_the_complex_planes(Q, oracle_mod, mixed):
    """A real matrix whose negative value has a positive partner keeps the
    complex planes (the f and g kernels' fused projection, one s and mixed
    s): equal to the oracle's walk-based solve, through a 64-step graph."""
    a = np.diag(np.full(64, 0.5))
    for j in range(63):
        a[j + 1, j] = a[j, j + 1] = 0.2
    a[7, 8] = -0.2  # its mirror a[8, 7] stays positive
    csc = W.from_dense(a)
    b = W.gaussian_b(64, seed=47)
    kappa, j0 = 30.0, 40
    om = oracle_mod.OracleMatrix(csc)
    beta, _ = oracle_mod.schedule(kappa, 1e-3)
    y_ref = om.qls_walk(b, j0, oracle_mod.cks_coeffs(beta, j0))
    mats = [csc, W.offset_matrix(64, 11, seed=48)] if mixed else [csc]
    walk = Q.Walk(mats, symmetric=False)
    st = walk.state([b] + [W.uniform_b(64)] * (len(mats) - 1) if mixed else b)
    assert not st.stats()["real_amplitudes"]
    x, _, steps, yn = walk.qls(b, kappa=kappa, eps=1e-3, j0=j0)
    assert steps == 2 * j0 + 1
    y = yn * x
    assert np.abs(y - y_ref).max() <= 1e-12 * np.abs(y_ref).max()
