"""Long runs through the captured step graphs, against the oracle: 256-step
replays and graphs of exactly the remaining count, with the single launches
around them, the one launch that moves a state onto the parity its long
graph was captured at, each representation (one double per cell, complex
planes, a grid-stride launch shape), the bound on the graphs a state keeps,
and the solver's 64-step graph with its coefficient window."""
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


@pytest.mark.parametrize("kind", ["real", "complex", "grid_stride"])
def test_long_runs_match_the_oracle(Q, oracle_mod, kind):
    if kind == "complex":
        csc = W.hermitian_offset_matrix(64, 4, seed=41)
        b = W.gaussian_b(64, seed=42) * np.exp(0.2j * np.arange(64))
    else:
        csc, b = W.offset_matrix(64, 4, seed=43), W.gaussian_b(64, seed=44)
    st = Q.Walk(csc).state(b)
    if kind == "grid_stride":
        st.set_launch(64, 1)
    ost = oracle_mod.OracleState(oracle_mod.OracleMatrix(csc)).set_b(b).T()
    assert st.stats()["real_amplitudes"] == (kind != "complex")
    total = 0
    # 600 from the T~ start: one launch, two 256-step replays, one 87-step
    # graph; 300 from the other parity: one launch to reach the long graph's
    # parity, then a replay and a 43-step graph; then counts around the graph
    # lengths and the single-launch limit (odd ones leave the other parity)
    for n in (600, 300, 17, 256, 513, 16, 2, 1, 257, 33, 290):
        st.step(n)
        ost.step(n)
        total += n
        gk, ga = st.export()
        ok, oa = ost.export()
        compare_states(gk, ga, ok, oa, where=f"{kind}, {total} steps")
        assert st.stats()["launches"] == total


def test_solver_graph_window(Q, oracle_mod):
    """A solve of 2 j0 + 1 = 801 launches: one launch, three 256-step
    replays with the window node ahead of each, 32 launches; equal to the
    oracle's walk-based solve."""
    csc, b = W.offset_matrix(64, 4, seed=45), W.gaussian_b(64, seed=46)
    kappa, j0 = 60.0, 400
    om = oracle_mod.OracleMatrix(csc)
    beta, _ = oracle_mod.schedule(kappa, 1e-3)
    y_ref = om.qls_walk(b, j0, oracle_mod.cks_coeffs(beta, j0))
    x, _, steps, yn = Q.Walk(csc).qls(b, kappa=kappa, eps=1e-3, j0=j0)
    assert steps == 801
    y = yn * x
    assert np.abs(y - y_ref).max() <= 1e-12 * np.abs(y_ref).max()


def test_many_step_counts_keep_a_bounded_graph_cache(Q, oracle_mod):
    """Twenty distinct step counts above the single-launch limit, odd and
    even, on one state (more graphs than the state keeps, so the oldest are
    released between calls), then repeats of earlier counts (captured again
    where released) and short calls: equal to the oracle throughout."""
    csc, b = W.offset_matrix(128, 6, seed=61), W.gaussian_b(128, seed=62)
    st = Q.Walk(csc).state(b)
    ost = oracle_mod.OracleState(oracle_mod.OracleMatrix(csc)).set_b(b).T()
    total = 0
    # calls of more than 32 steps replay a graph of exactly their count
    counts = list(range(34, 74, 2)) + [33, 35, 37, 39, 41] + [34, 36, 72, 33, 33, 70, 5, 1]
    for i, n in enumerate(counts):
        st.step(n)
        ost.step(n)
        total += n
        if i % 5 == 4 or i == len(counts) - 1:
            gk, ga = st.export()
            ok, oa = ost.export()
            compare_states(gk, ga, ok, oa, where=f"after {total} steps (count {n})")
    assert st.stats()["launches"] == total


def test_launch_shape_change_behind_a_running_replay(Q):
    """qw_set_launch discards the graphs while a replay may still run: it
    waits for the device first.  A shape change right behind an enqueued
    600-step call (no synchronisation), then more steps, equals the same
    walk run straight through, bit for bit."""
    csc, b = W.offset_matrix(2048, 8, seed=71), W.uniform_b(2048)
    walk = Q.Walk(csc)
    a, g = walk.state(b), walk.state(b)
    a.set_launch(128, 0).step(600)
    a.set_launch(256, 0)  # the one-pass kernels: the same arithmetic in another launch shape
    a.step(300)
    g.step(900)
    k1, a1 = a.export()
    k2, a2 = g.export()
    assert np.array_equal(k1, k2) and np.array_equal(a1, a2)

