"""Fixed-point matrix data on the GPU (values are words of a given word
length; the rotation is computed with a fixed-point square root, arccos and
angle): the walk, W^dagger, measurements, the batched form and the solver
against the oracle, at the shapes and word lengths of the paper's table of
experimental settings."""
import numpy as np
import pytest

import workloads as W
from tests.parity import compare_states

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def Q():
    import torch

    assert torch.cuda.is_available()
    import paper_2303_06890_amd as Q

    return Q


def _pair(Q, oracle_mod, csc, b, word, raw=False):
    walk = Q.Walk(csc, word=word)
    st = walk.state(b, raw=raw)
    om = oracle_mod.OracleMatrix(csc, word=word)
    ost = oracle_mod.OracleState(om).set_b(b)
    if not raw:
        ost.T()
    assert (walk.info[0]["N"], walk.info[0]["s"]) == (om.N, om.s)
    return walk, st, ost


def _check(st, ost, where):
    gk, ga = st.export()
    ok, oa = ost.export()
    assert ost.ambiguous() == 0
    compare_states(gk, ga, ok, oa, where=where)


@pytest.mark.parametrize("name,steps", [("A", 100), ("B", 30), ("C", 3)])
def test_table1_shapes_fixed_point(Q, oracle_mod, name, steps):
    """The paper's shapes A-C with their word length (8 bits)."""
    csc, b, word = W.table1_fixed_point_band(name)
    walk, st, ost = _pair(Q, oracle_mod, csc, b, word)
    _check(st, ost, f"{name} init")
    done = 0
    for t in sorted({1, 2, steps // 2, steps}):
        st.step(t - done)
        ost.step(t - done)
        done = t
        _check(st, ost, f"{name} step {t}")


@pytest.mark.parametrize("n,bw,word,neg,seed,steps", [(64, 2, 4, 0.5, 1, 100), (200, 5, 16, 0.5, 2, 100),
                                                      (96, 1, 32, 0.3, 3, 100), (80, 20, 12, 0.2, 4, 40),
                                                      (48, 9, 1, 0.0, 5, 100)])
def test_fixed_point_walk(Q, oracle_mod, n, bw, word, neg, seed, steps):
    """Word lengths 1 ... 32, negative entries (the +-i rule), s from 4 to 64,
    ragged dimensions."""
    csc = W.fixed_point_band(n, bw, word, seed=seed, negative=neg)
    walk, st, ost = _pair(Q, oracle_mod, csc, W.gaussian_b(n, seed=seed), word)
    done = 0
    for t in (1, 10, steps):
        st.step(t - done)
        ost.step(t - done)
        done = t
        _check(st, ost, f"n={n} bw={bw} w={word} step {t}")


@pytest.mark.parametrize("shape", [(128, 4), (64, 1), (256, 0)])
def test_fixed_point_launch_shapes(Q, oracle_mod, shape):
    """Grids too small for one pass (the grid-stride kernels) and the default
    grid (one pass) give the oracle's state."""
    csc = W.fixed_point_band(300, 6, 16, seed=9, negative=0.3)
    walk, st, ost = _pair(Q, oracle_mod, csc, W.gaussian_b(300, seed=9), 16)
    st.set_launch(*shape)
    st.step(30)
    ost.step(30)
    _check(st, ost, f"shape {shape} step 30")


def test_fixed_point_raw_start_adjoint_and_measurements(Q, oracle_mod):
    csc = W.fixed_point_band(128, 4, 10, seed=6, negative=0.4)
    b = W.gaussian_b(128, seed=7)
    walk, st, ost = _pair(Q, oracle_mod, csc, b, 10, raw=True)
    st.step(12)
    ost.step(12)
    _check(st, ost, "raw step 12")
    st.step_adjoint(5)
    ost.step_adjoint(5)
    _check(st, ost, "W^dagger 5")
    walk, st, ost = _pair(Q, oracle_mod, csc, b, 10)
    st.step(9)
    ost.step(9)
    assert abs(st.norm2() - 1.0) < 1e-13
    assert np.abs(st.j_marginal() - ost.j_marginal()).max() < 1e-14
    assert np.abs(st.project() - ost.project0()).max() < 1e-14


def test_fixed_point_batched_vs_oracle(Q, oracle_mod):
    """Instances of different shapes with one word length in one context."""
    word = 8
    mats = [W.fixed_point_band(64, 3, word, seed=11), W.fixed_point_band(100, 7, word, seed=12, negative=0.5),
            W.fixed_point_band(32, 1, word, seed=13)]
    bs = [W.gaussian_b(m.n, seed=20 + i) for i, m in enumerate(mats)]
    walk = Q.Walk(mats, word=word)
    st = walk.state(bs).step(15)
    keys, amps = st.export()
    from tests.test_gpu_batched import _slice, unpack

    F = unpack(keys, walk.nbits)
    for i, (a, b) in enumerate(zip(mats, bs)):
        om = oracle_mod.OracleMatrix(a, word=word)
        ok, oa = oracle_mod.OracleState(om).set_b(b).T().step(15).export()
        gk, ga = _slice(F, amps, i, om.nbits)
        compare_states(gk, ga, ok, oa, where=f"fixed-point instance {i}")


def test_fixed_point_solver(Q, oracle_mod):
    """Walk-based CKS solve on fixed-point data (the solve inverts the matrix
    the fixed-point rotation encodes): equal to the oracle's walk-based
    solve."""
    csc, b, word = W.table1_fixed_point_band("A")
    om = oracle_mod.OracleMatrix(csc, word=word)
    kappa, j0 = 30.0, 40
    beta, _ = oracle_mod.schedule(kappa, 1e-3)
    coef = oracle_mod.cks_coeffs(beta, j0)
    y_ref = om.qls_walk(b, j0, coef)
    x, p_succ, steps, yn = Q.Walk(csc, word=word).qls(b, kappa=kappa, eps=1e-3, j0=j0)
    assert steps == 2 * j0 + 1
    y = yn * x
    assert np.abs(y - y_ref).max() <= 1e-10 * np.abs(y_ref).max()


def test_fixed_point_gradient_not_provided(Q):
    from paper_2303_06890_amd import QwError

    csc = W.fixed_point_band(32, 2, 8, seed=51)
    st = Q.Walk(csc, word=8).state(W.uniform_b(32)).step(3)
    with pytest.raises(QwError, match="fixed-point"):
        st.grad(np.ones(32), 3)


def test_long_words_approach_fp64_values(Q):
    """32-bit words on the GPU stay close to the walk on the same values as
    FP64 numbers (the approximation error of the fixed-point rotation)."""
    csc = W.fixed_point_band(512, 3, 32, seed=71)
    b = W.uniform_b(512)
    k1, a1 = Q.Walk(csc, word=32).state(b).step(10).export()
    k2, a2 = Q.Walk(csc).state(b).step(10).export()
    d1 = dict(zip(k1.tolist(), a1.tolist()))
    d2 = dict(zip(k2.tolist(), a2.tolist()))
    big = {k for k, v in d2.items() if abs(v) > 1e-6}
    assert big <= set(d1)
    assert max(abs(d1.get(k, 0) - d2.get(k, 0)) for k in set(d1) | set(d2)) < 1e-6
