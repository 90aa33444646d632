"""Real amplitudes on the GPU: with no negative and no complex matrix value
and a real b, every amplitude of the walk from T~|b~> is real and the walk
steps run on 8-byte planes (the qwk_step_r / qwk_step_t kernels).  Every
other use of the state (measurements, export, W^dagger, other launch shapes)
moves it back to the complex planes.  Parity with the oracle across those
switches, graph replays, the branch count and fixed-point data."""
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
    assert np.all(ga.imag == 0.0)
    compare_states(gk, ga, ok, oa, where=where)


@pytest.mark.parametrize("case", ["A", "B", "band300"])
def test_real_amplitudes_match_the_oracle(Q, oracle_mod, case):
    if case == "band300":
        csc, b = W.band_matrix(300, 5, seed=31), W.gaussian_b(300, seed=32)  # s = 16, ragged n
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


def test_fixed_point_real_amplitudes(Q, oracle_mod):
    csc = W.fixed_point_band(400, 6, 16, seed=36)  # nonnegative words
    walk, st, ost = _pair(Q, oracle_mod, csc, W.gaussian_b(400, seed=37), word=16)
    assert st.stats()["real_amplitudes"]
    st.step(30)
    ost.step(30)
    _check(st, ost, "fixed point, step 30")


def test_when_amplitudes_are_not_real(Q, oracle_mod):
    """A negative entry, or a complex b, keeps the complex planes."""
    csc = W.band_matrix(128, 3, seed=38)
    d = csc.dense()
    d[5, 6] = d[6, 5] = -0.25
    neg = W.from_dense(d)
    st = Q.Walk(neg).state(W.uniform_b(128))
    assert not st.stats()["real_amplitudes"]
    b = W.gaussian_b(128, seed=39) * np.exp(0.3j * np.arange(128))
    walk, st, ost = _pair(Q, oracle_mod, csc, b)
    assert not st.stats()["real_amplitudes"]
    st.step(20)
    ost.step(20)
    gk, ga = st.export()
    ok, oa = ost.export()
    compare_states(gk, ga, ok, oa, where="complex b")
