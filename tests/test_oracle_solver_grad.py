"""Pins of the oracle's linear-solver and reverse-mode gradient parts."""
from fractions import Fraction
from math import comb

import numpy as np
import pytest

import workloads as W
from tests.conftest import load_golden
from tests.dense_sim import preprocess, torch_loss


# ---------------------------------------------------------------- coefficients

def _exact_coeffs(beta, j0):
    tot = Fraction(0)
    den = 4 ** beta
    out = []
    for j in range(j0 + 1):
        tail = sum(comb(2 * beta, beta + i) for i in range(j + 1, beta + 1))
        out.append(float(4 * (-1) ** j * Fraction(tail, den)))
    return np.array(out)


@pytest.mark.parametrize("beta,j0", [(1, 0), (5, 3), (40, 20), (300, 60)])
def test_cks_coeffs_exact(oracle_mod, beta, j0):
    got = oracle_mod.cks_coeffs(beta, j0)
    ref = _exact_coeffs(beta, j0)
    assert np.allclose(got, ref, rtol=1e-13, atol=1e-300)


def test_cks_coeffs_large_beta_vs_binomial_tail(oracle_mod):
    from scipy.stats import binom

    beta, j0 = 966624, 4620
    got = oracle_mod.cks_coeffs(beta, j0)
    ks = np.array([0, 1, 10, 100, 1000, 2000, 4000, 4620])
    ref = 4 * (-1.0) ** ks * binom.sf(beta + ks, 2 * beta, 0.5)
    assert np.allclose(got[ks], ref, rtol=1e-9)


def test_f_of_x_identity(oracle_mod):
    """sum_j a_j T_{2j+1}(x) reproduces f(x) = (1 - (1-x^2)^b)/x (Eq. fx) when
    the series is not truncated (j0 = b - 1)."""
    beta = 12
    a = oracle_mod.cks_coeffs(beta, beta - 1)
    for x in (0.05, 0.3, 0.7, 0.99, -0.4):
        th = np.arccos(x)
        series = sum(a[j] * np.cos((2 * j + 1) * th) for j in range(beta))
        assert series == pytest.approx((1 - (1 - x * x) ** beta) / x, rel=1e-12)


# ---------------------------------------------------------------- schedule

def test_schedule_laplacian(oracle_mod):
    # 5-point Laplacian 32x32 + 0.1 I, scaled by 1/4.1, s = 8: smallest
    # eigenvalue in closed form
    lam = (0.1 + 4 - 4 * np.cos(np.pi / 33)) / 4.1 / 8
    beta, j0 = oracle_mod.schedule(1 / lam, 1e-3)
    assert j0 == 4620 and 2 * j0 + 1 == 9241
    assert beta == int(np.ceil((1 / lam) ** 2 * np.log(1 / lam / 1e-3)))


_SETTINGS = load_golden("experimental_settings.json")


@pytest.mark.parametrize("kappa_printed,j0_printed",
                         [(r["kappa"], r["j0"]) for r in _SETTINGS["rows"] if r["j0"] is not None])
def test_schedule_reproduces_table1(oracle_mod, kappa_printed, j0_printed):
    """The table of experimental settings prints kappa to two significant
    digits; some kappa in [printed, printed + one unit of the second digit)
    gives the printed j0 with natural logarithms and eps = 1e-3
    (tests/golden/experimental_settings.json)."""
    unit = 10 ** (np.floor(np.log10(kappa_printed)) - 1)
    lo, hi = kappa_printed, kappa_printed + unit
    assert oracle_mod.schedule(lo, 1e-3)[1] <= j0_printed <= oracle_mod.schedule(hi, 1e-3)[1]
    # bisection for the exact kappa
    for _ in range(80):
        mid = 0.5 * (lo + hi)
        if oracle_mod.schedule(mid, 1e-3)[1] < j0_printed:
            lo = mid
        else:
            hi = mid
    assert oracle_mod.schedule(hi, 1e-3)[1] == j0_printed


def test_walk_steps_of_matrix_c():
    """The text gives 212245 = 2 j0 + 1 walk steps for the 1024 matrix."""
    c = next(r for r in _SETTINGS["rows"] if r["name"] == "C")
    assert _SETTINGS["walk_steps_C"] == 2 * c["j0"] + 1


@pytest.mark.parametrize("row", _SETTINGS["rows"], ids=lambda r: r["name"])
def test_workload_shapes_match_the_table(oracle_mod, row):
    """The band workloads of the five experiments have the table's row size,
    sparsity (footnote b: s = 2^ceil(log2(2 * bandwidth + 1))) and word
    length."""
    csc, _ = W.table1_band(row["name"])
    m = oracle_mod.OracleMatrix(csc)
    assert (csc.n, m.N, m.s) == (row["row_size"], row["row_size"], row["s"])
    r, c = np.nonzero(csc.dense())
    bw = int(np.abs(r - c).max())
    assert 2 ** int(np.ceil(np.log2(2 * bw + 1))) == row["s"]
    assert W.TABLE1_WORD[row["name"]] == row["word_length"]
    assert W.TABLE1_PAPER_SECONDS_PER_STEP[row["name"]] == pytest.approx(row["seconds_per_step"])


# ---------------------------------------------------------------- series and walk solver

def test_classical_series_vs_lu(oracle_mod):
    csc, b = W.solver_problem()
    m = oracle_mod.OracleMatrix(csc)
    N, nbits, s, scale, col, val = preprocess(csc)
    H = csc.dense() * scale / s
    lam = np.abs(np.linalg.eigvalsh(H)).min()
    beta, j0 = oracle_mod.schedule(1 / lam, 1e-3)
    coef = oracle_mod.cks_coeffs(beta, j0)
    y = m.cheb_series(b, j0, coef)
    x = np.linalg.solve(H, b)
    fid = abs(np.dot(x, y)) ** 2 / (np.dot(x, x) * np.dot(y, y))
    assert fid > 1 - 1e-9
    assert np.linalg.norm(y - x) / np.linalg.norm(x) < 2e-3
    p_succ = np.dot(y, y) / np.abs(coef).sum() ** 2
    assert 1e-4 < p_succ < 1e-3


def test_walk_solver_equals_series(oracle_mod):
    csc, _ = W.tiny_tridiagonal()
    b = W.gaussian_b(16, seed=3)
    m = oracle_mod.OracleMatrix(csc)
    N, nbits, s, scale, col, val = preprocess(csc)
    H = csc.dense() * scale / s
    lam = np.abs(np.linalg.eigvalsh(H)).min()
    beta, j0 = oracle_mod.schedule(1 / lam, 1e-2)
    assert j0 < 1000
    coef = oracle_mod.cks_coeffs(beta, j0)
    y_series = m.cheb_series(b, j0, coef)
    y_walk = m.qls_walk(b, j0, coef, tau=0.0)
    assert np.abs(y_walk - y_series).max() < 1e-12
    assert np.abs(y_walk.imag).max() < 1e-14


# ---------------------------------------------------------------- gradient

def _grad_case():
    csc = W.offset_matrix(16, 5, seed=81)
    scale = 1.0 / np.abs(csc.vals).max()
    csc = W.Csc(csc.n, csc.colptr, csc.rowidx, csc.vals * scale)
    b = W.gaussian_b(16, seed=82)
    w = np.zeros(16)
    w[[1, 4, 9, 13]] = 1.0
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


def test_grad_vs_central_differences(oracle_mod):
    csc, b, w = _grad_case()
    nsteps = 5
    m = oracle_mod.OracleMatrix(csc, scale=1.0)
    loss, dv, db = m.grad(b, w, nsteps, tau=0.0)
    assert loss == pytest.approx(_loss(oracle_mod, csc, b, w, nsteps), abs=1e-15)
    slot = _csc_slot(m, csc)
    g = dv.reshape(-1)[slot]
    rng = np.random.default_rng(83)
    ok = np.nonzero((np.abs(csc.vals) > 1e-4) & (np.abs(csc.vals) < 1 - 1e-4))[0]
    h = 1e-6
    for p in rng.choice(ok, size=12, replace=False):
        vp = csc.vals.copy()
        vm = csc.vals.copy()
        vp[p] += h
        vm[p] -= h
        fd = (_loss(oracle_mod, W.Csc(csc.n, csc.colptr, csc.rowidx, vp), b, w, nsteps)
              - _loss(oracle_mod, W.Csc(csc.n, csc.colptr, csc.rowidx, vm), b, w, nsteps)) / (2 * h)
        assert abs(fd - g[p]) <= 1e-8 * abs(g[p]) + 1e-10, p
    for j in (0, 5, 11):
        for d in (1.0, 1j):
            bp = b.astype(complex).copy()
            bm = b.astype(complex).copy()
            bp[j] += h * d
            bm[j] -= h * d
            fd = (_loss(oracle_mod, csc, bp, w, nsteps) - _loss(oracle_mod, csc, bm, w, nsteps)) / (2 * h)
            ref = db[j].real if d == 1.0 else db[j].imag
            assert abs(fd - ref) <= 1e-8 * abs(ref) + 1e-10


def test_grad_vs_torch_autograd_on_dense(oracle_mod):
    csc, b, w = _grad_case()
    nsteps = 4
    m = oracle_mod.OracleMatrix(csc, scale=1.0)
    loss, dv, db = m.grad(b, w, nsteps, tau=0.0)
    tl, tv, tb = torch_loss(csc, csc.vals, b, w, nsteps)
    tl.backward()
    assert loss == pytest.approx(float(tl.detach()), abs=1e-14)
    g = dv.reshape(-1)[_csc_slot(m, csc)]
    ref = tv.grad.numpy()
    fin = np.isfinite(ref) & np.isfinite(g)
    assert fin.sum() >= csc.nnz - 2
    assert np.allclose(g[fin], ref[fin], rtol=1e-9, atol=1e-12)
    # torch's complex gradient convention: dL/dRe + i dL/dIm
    assert np.allclose(db[:16], tb.grad.numpy(), rtol=1e-9, atol=1e-12)
