"""Sixteen lanes per row: a context that would have at most 1024 step-kernel
wavefronts with eight lanes per row gives its instances with s >= 16 sixteen
(two, four slots per lane for s = 32, 64).  Parity with the oracle for every
kernel family that then runs with that mapping: one double per cell (FP64
and fixed-point words), the complex planes (a complex b), complex Hermitian
values, a grid-stride launch shape and W^dagger."""
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


def _run(Q, oracle_mod, csc, b, word=0, shape=None, steps=(1, 2, 17, 40), adjoint=0):
    walk = Q.Walk(csc, word=word)
    assert walk.info[0]["s"] >= 16
    st = walk.state(b)
    assert st.stats()["lanes_per_row_s16"] == 16
    if shape:
        st.set_launch(*shape)
    ost = oracle_mod.OracleState(oracle_mod.OracleMatrix(csc, word=word)).set_b(b).T()
    done = 0
    for t in steps:
        st.step(t - done)
        ost.step(t - done)
        done = t
        gk, ga = st.export()
        ok, oa = ost.export()
        assert ost.ambiguous() == 0
        compare_states(gk, ga, ok, oa, where=f"s={walk.info[0]['s']} step {t}")
    if adjoint:
        st.step_adjoint(adjoint)
        ost.step_adjoint(adjoint)
        gk, ga = st.export()
        ok, oa = ost.export()
        compare_states(gk, ga, ok, oa, where=f"s={walk.info[0]['s']} W^dagger {adjoint}")
    return st


@pytest.mark.parametrize("c", [11, 21, 40])
def test_real_planes(Q, oracle_mod, c):
    csc, b = W.offset_matrix(64, c, seed=100 + c), W.gaussian_b(64, seed=200 + c)
    st = _run(Q, oracle_mod, csc, b, adjoint=5)
    assert st.stats()["real_amplitudes"]


@pytest.mark.parametrize("c", [11, 21, 40])
def test_complex_b(Q, oracle_mod, c):
    csc = W.offset_matrix(64, c, seed=110 + c)
    b = W.gaussian_b(64, seed=210 + c) * np.exp(0.3j * np.arange(64))
    _run(Q, oracle_mod, csc, b)


@pytest.mark.parametrize("c", [11, 21, 40])
def test_hermitian(Q, oracle_mod, c):
    csc = W.hermitian_offset_matrix(64, c, seed=120 + c)
    b = W.gaussian_b(64, seed=220 + c)
    _run(Q, oracle_mod, csc, b)


@pytest.mark.parametrize("bw", [5, 12, 25])
def test_fixed_point_words(Q, oracle_mod, bw):
    csc = W.fixed_point_band(96, bw, 12, seed=130 + bw, negative=0.4)
    _run(Q, oracle_mod, csc, W.gaussian_b(96, seed=230 + bw), word=12)


@pytest.mark.parametrize("c", [11, 40])
def test_grid_stride_shape(Q, oracle_mod, c):
    csc, b = W.offset_matrix(64, c, seed=140 + c), W.gaussian_b(64, seed=240 + c)
    _run(Q, oracle_mod, csc, b, shape=(64, 1))


def test_large_contexts_keep_eight_lanes(Q):
    """Shape E (16384 rows, s = 64: 2048 wavefronts with eight lanes) and a
    batch of 256 instances keep eight lanes per row; shape D (8192 rows,
    s = 32: 1024 wavefronts) takes sixteen."""
    assert Q.Walk(W.table1_band("E")[0]).state(W.uniform_b(16384)).stats()["lanes_per_row_s16"] == 8
    assert Q.Walk(W.table1_band("D")[0]).state(W.uniform_b(8192)).stats()["lanes_per_row_s16"] == 16
    inst = W.batched_instances(count=256)
    st = Q.Walk([a for a, _ in inst]).state([b for _, b in inst])
    assert st.stats()["lanes_per_row_s16"] == 8


@pytest.mark.parametrize("lanes", [8, 16])
@pytest.mark.parametrize("shape", ["C", "E"])
def test_lanes_flag_forces_the_mapping(Q, oracle_mod, lanes, shape):
    """QW_LANES_8 / QW_LANES_16 replace the library's rule: the paper's shape
    C (s = 32, which the rule gives 16 lanes) and E (s = 64, which it gives
    8), each with both mappings, equal the oracle."""
    csc, b = W.table1_band(shape)
    if shape == "E":  # a smaller band of the same s keeps the oracle quick
        csc, b = W.band_matrix(512, 31, seed=7), W.uniform_b(512)
    walk = Q.Walk(csc, lanes=lanes)
    st = walk.state(b)
    assert st.stats()["lanes_per_row_s16"] == lanes
    ost = oracle_mod.OracleState(oracle_mod.OracleMatrix(csc)).set_b(b).T()
    st.step(9)
    ost.step(9)
    gk, ga = st.export()
    ok, oa = ost.export()
    compare_states(gk, ga, ok, oa, where=f"shape {shape}, {lanes} lanes per row")


def test_tune_walk_chooses_a_tile_and_logs_it(Q, oracle_mod):
    """The autotuner loads the four tiles of an s = 32 matrix (8 or 16 lanes
    per row, with and without the XCD numbering of row blocks), times them,
    and returns a walk that equals the oracle."""
    from paper_2303_06890_amd import autotune

    csc, b = W.band_matrix(256, 15, seed=8), W.uniform_b(256)
    walk, shape, log = autotune.tune_walk(csc, b)
    tiles = sorted((c["lanes_per_row"][0], c["xcd_rows"]) for c in log["tile_choices"])
    assert tiles == [(8, False), (8, True), (16, False), (16, True)]
    assert log["chosen_lanes_per_row"] in ([8], [16]) and len(log["launch_candidates"]) >= 4
    assert walk.xcd == log["chosen_xcd_rows"]
    st = walk.state(b)
    autotune.apply(st, shape)
    st.step(40)
    ok, oa = oracle_mod.OracleState(oracle_mod.OracleMatrix(csc)).set_b(b).T().step(40).export()
    gk, ga = st.export()
    compare_states(gk, ga, ok, oa, where="tuned walk")


_XCD_CASES = {
    "G1024x8": lambda: (W.offset_matrix(1024, 8, seed=41), W.gaussian_b(1024, seed=42), 0, 0),
    "band_s32_16lanes": lambda: (W.band_matrix(2048, 15, seed=43), W.uniform_b(2048), 16, 0),
    "band_s64_8lanes": lambda: (W.band_matrix(1024, 31, seed=44), W.gaussian_b(1024, seed=45), 8, 0),
    "fixed_point_w16": lambda: (W.fixed_point_band(1024, 15, 16, seed=46), W.uniform_b(1024), 16, 16),
    "batch_mixed_s": lambda: ([a for a, _ in W.batched_instances(count=24, seed=47)],
                              [b for _, b in W.batched_instances(count=24, seed=47)], 0, 0),
}


@pytest.mark.parametrize("case", list(_XCD_CASES))
def test_xcd_rows_change_nothing(Q, case):
    """QW_XCD_ROWS renumbers the row blocks of the one-pass step and adjoint
    kernels by XCD.  Only which workgroup runs which rows changes, so the
    states, branch counts and gradients equal those of the plain numbering bit
    for bit.  Grids are multiples of 8, where the numbering applies."""
    from paper_2303_06890_amd import autotune

    mats, b, lanes, word = _XCD_CASES[case]()
    out = []
    for xcd in (False, True):
        walk = Q.Walk(mats, lanes=lanes, word=word, xcd=xcd)
        shape = (64, -(-autotune._waves(walk) // 8) * 8)  # one pass; blocks past the rows return at once
        st = walk.state(b)
        st.set_launch(*shape)
        assert st.stats()["xcd_rows"] == xcd
        st.step(3).step(37)  # single launches, then a graph
        k, a = st.export()
        adj = st.step_adjoint(5).export()
        res = [k, a, adj[0], adj[1], st.stats()["total_written"]]
        if word == 0:
            g = walk.state(b)
            g.set_launch(*shape)
            w = np.random.default_rng(48).random(walk.n_total)
            loss, dv, db = g.step(12).grad(w, 12)
            res += [loss, dv.copy(), db.copy()]
        out.append(res)
        walk.close()
    for x, y in zip(out[0], out[1]):
        np.testing.assert_array_equal(x, y, err_msg=case)


def test_xcd_rows_change_nothing_in_the_solver(Q):
    """The solver's steps run the _acc forms, which have XCD-numbered
    versions too: the same solve with and without the numbering gives the same
    bits (x, success probability, walk steps, |y|)."""
    A, b = W.solver_problem(32)  # 1024 rows, s = 8: 128 wavefronts, 32 or more workgroups (a multiple of 8)
    plain = Q.Walk(A).qls(b, eps=1e-2)
    xcd = Q.Walk(A, xcd=True).qls(b, eps=1e-2)
    np.testing.assert_array_equal(plain[0], xcd[0])
    assert plain[1:] == xcd[1:]


_SPLIT_CASES = {}


def _split_case(oracle_mod, word):
    """The band of half-width 31 at n = 1024 (s = 64) and the oracle's states
    after 3 and 40 steps, computed once per word length."""
    if word not in _SPLIT_CASES:
        n = 1024
        csc = W.band_matrix(n, 31, seed=61) if word == 0 else W.fixed_point_band(n, 31, word, seed=61)
        b = W.gaussian_b(n, seed=62)
        b = b / np.linalg.norm(b)
        ost = oracle_mod.OracleState(oracle_mod.OracleMatrix(csc, word=word)).set_b(b).T()
        snaps = {}
        done = 0
        for t in (3, 40):
            ost.step(t - done)
            done = t
            snaps[t] = ost.export()
            assert ost.ambiguous() == 0
        _SPLIT_CASES[word] = (csc, b, snaps)
    return _SPLIT_CASES[word]


@pytest.mark.parametrize("lanes", [8, 16])
@pytest.mark.parametrize("word", [0, 32])
def test_split_rows_for_s64(Q, oracle_mod, word, lanes):
    """s = 64: in workgroups of a multiple of K wavefronts the real step
    kernels split each row's 64 slots over K wavefronts (K = 2 with eight
    lanes per row, 4 with sixteen; their row sums joined through LDS); in
    other workgroups a wavefront keeps whole rows.  Both against the oracle
    (single launches, then graphs), FP64 values and 32-bit fixed-point words;
    the split form with and without the XCD numbering of row blocks bit for
    bit; the solver's fused projection through the split _acc forms."""
    n = 1024
    csc, b, snaps = _split_case(oracle_mod, word)
    waves = n // 8 if lanes == 8 else n // 4
    results = {}
    for shape, xcd in (((256, waves // 4), False), ((128, waves // 2), False), ((64, waves), False),
                       ((256, waves // 4), True)):
        walk = Q.Walk(csc, word=word, lanes=lanes, xcd=xcd)
        assert walk.info[0]["s"] == 64
        st = walk.state(b)
        st.set_launch(*shape)
        assert st.stats()["real_amplitudes"]
        done = 0
        for t in (3, 40):
            st.step(t - done)  # 3 single launches, then a graph of 37
            done = t
            gk, ga = st.export()
            ok, oa = snaps[t]
            compare_states(gk, ga, ok, oa, where=f"word={word} shape={shape} xcd={xcd} step {t}")
        results[(shape, xcd)] = st.export()
        walk.close()
    split, split_x = results[((256, waves // 4), False)], results[((256, waves // 4), True)]
    np.testing.assert_array_equal(split[0], split_x[0])
    np.testing.assert_array_equal(split[1], split_x[1])
    if lanes == 8:  # the pair's two wavefronts in workgroups of 2 or 4: the same arithmetic
        other = results[((128, waves // 2), False)]
        np.testing.assert_array_equal(split[0], other[0])
        np.testing.assert_array_equal(split[1], other[1])
    if word == 0 and lanes == 8:
        # a well-conditioned band (kappa of A/s about 330: some 9400 walk steps)
        A = W.from_dense(W.band_matrix(256, 31, seed=63).dense() + 40.0 * np.eye(256))
        walk = Q.Walk(A)
        assert walk.info[0]["s"] == 64
        x0 = walk.qls(W.uniform_b(256), eps=1e-2)
        y = np.linalg.solve(A.dense(), W.uniform_b(256))
        fid = abs(np.vdot(y / np.linalg.norm(y), x0[0])) ** 2
        assert fid > 1 - 1e-3, fid
