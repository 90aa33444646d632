"""One double per cell on the GPU: for a real matrix whose negative values
pair up (a symmetric one) and a real b, every amplitude of the walk from
T~|b~> is real, except those of the R0 cells of slots of negative value,
which are imaginary; the walk steps then run on 8-byte planes (the
qwk_step_r / qwk_step_t kernels; qwk_step_rg / qwk_step_tg for instances of
mixed s).  Uses that change the state otherwise (W^dagger, other launch
shapes) move it back to the complex planes; measurements and the export read
a copy there.  Parity with the oracle across those switches, graph
replays, the branch count, negative values and fixed-point data."""
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


def _pair(Q, oracle_mod, csc, b, word=0):
    walk = Q.Walk(csc, word=word)
    st = walk.state(b)
    ost = oracle_mod.OracleState(oracle_mod.OracleMatrix(csc, word=word)).set_b(b).T()
    return walk, st, ost


def _check(st, ost, where):
    gk, ga = st.export()
    ok, oa = ost.export()
    assert ost.ambiguous() == 0
    assert np.all((ga.real == 0.0) | (ga.imag == 0.0))  # one double per cell
    compare_states(gk, ga, ok, oa, where=where)


@pytest.mark.parametrize("case", ["A", "B", "band300", "offsets", "offsets_s16"])
def test_real_amplitudes_match_the_oracle(Q, oracle_mod, case):
    if case == "band300":
        csc, b = W.band_matrix(300, 5, seed=31), W.gaussian_b(300, seed=32)  # s = 16, ragged n
    elif case == "offsets":  # negative values: imaginary R0 cells
        csc, b = W.offset_matrix(1024, 8, seed=4), W.gaussian_b(1024, seed=5)
    elif case == "offsets_s16":
        csc, b = W.offset_matrix(200, 11, seed=6), W.gaussian_b(200, seed=7)
    else:
        csc, b = W.table1_band(case)
    walk, st, ost = _pair(Q, oracle_mod, csc, b)
    assert st.stats()["real_amplitudes"]
    done = 0
    for t in (1, 2, 19, 40):  # single launches and graph replays
        st.step(t - done)
        ost.step(t - done)
        done = t
        _check(st, ost, f"{case} step {t}")


@pytest.mark.parametrize("kind", ["offsets", "fixed_point"])
def test_mixed_s_batch_on_real_planes(Q, oracle_mod, kind):
    """Instances of s = 4, 8 and 16 in one context (the one-pass kernels of
    mixed s on one double per cell): negative values, fillers of value 0
    where the column count is not a power of two (skipped in place), a ragged
    dimension; each instance against its own oracle walk."""
    from tests.test_gpu_batched import _slice, unpack

    word = 0
    if kind == "offsets":
        mats = [W.offset_matrix(64, 3, seed=81), W.offset_matrix(128, 6, seed=82),
                W.offset_matrix(256, 11, seed=83), W.band_matrix(300, 2, seed=84)]
    else:
        word = 12
        mats = [W.fixed_point_band(64, 1, word, seed=85, negative=0.5),
                W.fixed_point_band(200, 3, word, seed=86, negative=0.3),
                W.fixed_point_band(128, 6, word, seed=87, negative=0.5)]
    bs = [W.gaussian_b(m.n, seed=90 + i) for i, m in enumerate(mats)]
    walk = Q.Walk(mats, word=word)
    assert len({d["s"] for d in walk.info}) == 3
    st = walk.state(bs)
    assert st.stats()["real_amplitudes"]
    osts = [oracle_mod.OracleState(oracle_mod.OracleMatrix(m, word=word)).set_b(b).T() for m, b in zip(mats, bs)]
    done = 0
    for t in (1, 2, 19, 40):  # single launches and graph replays
        st.step(t - done)
        keys, amps = st.export()
        assert np.all((amps.real == 0.0) | (amps.imag == 0.0))  # one double per cell
        F = unpack(keys, walk.nbits)
        for i, ost in enumerate(osts):
            ost.step(t - done)
            ok, oa = ost.export()
            gk, ga = _slice(F, amps, i, ost.mat.nbits)
            compare_states(gk, ga, ok, oa, where=f"{kind} instance {i} step {t}")
        done = t


@pytest.mark.parametrize("word", [0, 10])
def test_solver_projection_on_real_planes(Q, oracle_mod, word):
    """The solver's fused projection on one double per cell, in a context of
    instances of mixed s (the solve works on instance 0): equal to the
    oracle's walk-based solve of instance 0."""
    if word:
        a = W.fixed_point_band(128, 3, word, seed=95, negative=0.4)
        other = W.fixed_point_band(64, 6, word, seed=96)
    else:
        a, other = W.offset_matrix(128, 6, seed=95), W.offset_matrix(64, 11, seed=96)
    b = W.gaussian_b(128, seed=97)
    kappa, j0 = 40.0, 150  # 301 launches: one, a 256-step graph replay, 44 more
    om = oracle_mod.OracleMatrix(a, word=word)
    beta, _ = oracle_mod.schedule(kappa, 1e-3)
    y_ref = om.qls_walk(b, j0, oracle_mod.cks_coeffs(beta, j0))
    for mats in ([a], [a, other]):
        walk = Q.Walk(mats, word=word)
        x, p_succ, steps, yn = walk.qls(b, kappa=kappa, eps=1e-3, j0=j0)
        assert steps == 2 * j0 + 1
        y = yn * x
        assert np.abs(y - y_ref).max() <= 1e-12 * np.abs(y_ref).max(), len(mats)


def test_switches_between_the_representations(Q, oracle_mod):
    csc, b = W.band_matrix(300, 5, seed=33), W.gaussian_b(300, seed=34)
    walk, st, ost = _pair(Q, oracle_mod, csc, b)
    st.step(20)
    ost.step(20)
    assert np.abs(st.j_marginal() - ost.j_marginal()).max() < 1e-14
    st.set_launch(64, 1)  # too few workgroups for one pass: the complex grid-stride kernel
    st.step(5)
    ost.step(5)
    st.set_launch(64, 64)  # one pass again: real planes
    st.step(18)
    ost.step(18)
    assert np.abs(st.project() - ost.project0()).max() < 1e-14
    st.step_adjoint(7)  # the swap passes run on the complex planes
    ost.step_adjoint(7)
    st.step(3)
    ost.step(3)
    _check(st, ost, "after the switches")
    assert st.stats()["real_amplitudes"]


def test_measurements_leave_the_state_on_the_real_planes(Q):
    """A measurement reads a copy of the real planes and leaves the state on
    them: graph-replayed calls with measurements in between, a swap pass (on
    the complex planes) right after a measurement, then more steps; the state
    equals, bit for bit, one that was never measured."""
    csc, b = W.offset_matrix(512, 6, seed=36), W.uniform_b(512)
    walk = Q.Walk(csc)
    a, g = walk.state(b), walk.state(b)
    for n in (40, 1, 300, 33):
        a.step(n)
        a.count()
        a.j_marginal()
        assert a.stats()["real_amplitudes"]
        a.project()
        g.step(n)
    a.step_adjoint(5)
    g.step_adjoint(5)
    a.count()
    a.step(50)
    g.step(50)
    k1, a1 = a.export()
    k2, a2 = g.export()
    assert np.array_equal(k1, k2) and np.array_equal(a1, a2)
    # the marginal is summed with atomics: equal up to the order of the sum
    assert np.allclose(a.j_marginal(), g.j_marginal(), rtol=1e-13, atol=0)


def test_branch_count_on_real_planes(Q):
    csc, b = W.band_matrix(256, 3, seed=35), W.uniform_b(256)
    walk = Q.Walk(csc)
    a = walk.state(b)
    t0, counts = a.stats()["total_written"], []
    for _ in range(20):
        a.step(1)
        counts.append(a.count())
    assert a.stats()["total_written"] - t0 == sum(counts)
    g = walk.state(b)
    g0 = g.stats()["total_written"]
    g.step(20)
    assert g.stats()["total_written"] - g0 == sum(counts)
    k1, a1 = a.export()
    k2, a2 = g.export()
    assert np.array_equal(k1, k2) and np.array_equal(a1, a2)


@pytest.mark.parametrize("neg", [0.0, 0.4])
def test_fixed_point_real_amplitudes(Q, oracle_mod, neg):
    csc = W.fixed_point_band(400, 6, 16, seed=36, negative=neg)
    walk, st, ost = _pair(Q, oracle_mod, csc, W.gaussian_b(400, seed=37), word=16)
    assert st.stats()["real_amplitudes"]
    st.step(30)
    ost.step(30)
    _check(st, ost, f"fixed point, negative fraction {neg}, step 30")


def test_when_cells_are_not_real(Q, oracle_mod):
    """A negative value whose partner is positive (an unsymmetric pattern), or
    a complex b, keeps the complex planes."""
    a = np.diag(np.full(64, 0.5))
    for j in range(63):
        a[j + 1, j] = a[j, j + 1] = 0.2
    a[7, 8] = -0.2  # its mirror a[8, 7] stays positive
    st = Q.Walk(W.from_dense(a), symmetric=False).state(W.uniform_b(64))
    assert not st.stats()["real_amplitudes"]
    csc = W.band_matrix(128, 3, seed=38)
    b = W.gaussian_b(128, seed=39) * np.exp(0.3j * np.arange(128))
    walk, st, ost = _pair(Q, oracle_mod, csc, b)
    assert not st.stats()["real_amplitudes"]
    st.step(20)
    ost.step(20)
    gk, ga = st.export()
    ok, oa = ost.export()
    compare_states(gk, ga, ok, oa, where="complex b")
