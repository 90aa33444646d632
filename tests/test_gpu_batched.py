"""Batched walks: many matrices of uneven size and sparsity advance in one
launch per step; each instance's slice must equal its plain run."""
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


def unpack(keys, n):
    """Register fields [inst, j_c, j, b1, k_c, k, b2] of packed keys (M x 7)."""
    k = np.asarray(keys, np.uint64).copy()
    m = np.uint64((1 << n) - 1)
    one, nn = np.uint64(1), np.uint64(n)
    b2 = k & one
    k >>= one
    kk = k & m
    k >>= nn
    kc = k & m
    k >>= nn
    b1 = k & one
    k >>= one
    j = k & m
    k >>= nn
    jc = k & m
    k >>= nn
    return np.stack([k, jc, j, b1, kc, kk, b2], axis=1)


def repack(F, n):
    """Keys of fields [j_c, j, b1, k_c, k, b2] with register width n."""
    F = np.asarray(F, np.uint64)
    key = F[:, 0].copy()
    for col, w in ((1, n), (2, 1), (3, n), (4, n), (5, 1)):
        key = (key << np.uint64(w)) | F[:, col]
    return key


def _slice(F, amps, i, n):
    sel = F[:, 0] == np.uint64(i)
    k = repack(F[sel, 1:], n)
    a = amps[sel]
    order = np.argsort(k)
    return k[order], a[order]


def _plain(Q, csc, b, nsteps):
    """The same walk alone.  The batch and the single walk may run different
    kernels (one double per cell or complex planes, other lane shapes), so
    amplitudes agree to rounding, keys exactly."""
    walk = Q.Walk(csc)
    keys, amps = walk.state(b).step(nsteps).export()
    return walk.nbits, keys, amps


def test_batched_equals_plain_runs(Q):
    inst = W.batched_instances(count=24, seed=7, emin=4, emax=9)
    mats = [a for a, _ in inst]
    bs = [b for _, b in inst]
    walk = Q.Walk(mats)
    assert len({d["s"] for d in walk.info}) > 1 and len({d["N"] for d in walk.info}) > 1
    st = walk.state(bs).step(30)
    keys, amps = st.export()
    F = unpack(keys, walk.nbits)
    for i, (a, b) in enumerate(inst):
        n, rk, ra = _plain(Q, a, b, 30)
        gk, ga = _slice(F, amps, i, n)
        assert np.array_equal(gk, rk), i
        assert np.abs(ga - ra).max() < 1e-13, i


def test_batched_vs_oracle(Q, oracle_mod):
    inst = W.batched_instances(count=6, seed=8, emin=4, emax=8)
    walk = Q.Walk([a for a, _ in inst])
    st = walk.state([b for _, b in inst]).step(20)
    keys, amps = st.export()
    F = unpack(keys, walk.nbits)
    for i, (a, b) in enumerate(inst):
        om = oracle_mod.OracleMatrix(a)
        ok, oa = oracle_mod.OracleState(om).set_b(b).T().step(20).export()
        gk, ga = _slice(F, amps, i, om.nbits)
        compare_states(gk, ga, ok, oa, where=f"instance {i}")


@pytest.mark.parametrize("kind", ["small_s", "wide_s"])
def test_batched_mixed_row_lengths(Q, oracle_mod, kind):
    """Instances whose s differ (1 ... 8 with instances smaller than a
    wavefront's rows, or 4 ... 64): the step kernel reads each wavefront's
    lane mapping from its instance; every slice must match the oracle."""
    diag = W.from_dense(np.diag(np.linspace(0.2, 0.8, 12)))           # s = 1
    pair = W.from_dense(np.array([[0.3, 0.5], [0.5, 0.6]]))           # s = 2
    if kind == "small_s":
        mats = [diag, W.offset_matrix(40, 3, seed=51), pair, W.offset_matrix(100, 7, seed=52)]
    else:  # every instance has a full wavefront of rows: the one-pass kernel
        mats = [W.offset_matrix(64, 33, seed=53), W.offset_matrix(24, 3, seed=54),
                W.offset_matrix(128, 20, seed=55), W.offset_matrix(96, 12, seed=56)]
    bs = [W.gaussian_b(m.n, seed=60 + i) for i, m in enumerate(mats)]
    walk = Q.Walk(mats)
    st = walk.state(bs).step(15)
    keys, amps = st.export()
    F = unpack(keys, walk.nbits)
    for i, (a, b) in enumerate(zip(mats, bs)):
        om = oracle_mod.OracleMatrix(a)
        ok, oa = oracle_mod.OracleState(om).set_b(b).T().step(15).export()
        gk, ga = _slice(F, amps, i, om.nbits)
        compare_states(gk, ga, ok, oa, where=f"{kind} instance {i}")


def test_batched_workload_256_sampled_vs_oracle(Q, oracle_mod):
    """The 256-instance workload after 50 graph-replayed steps: sampled
    instances (the two with the fewest slots and those at the first quartile
    and the median of the slot count, which the oracle finishes in seconds)
    match the oracle."""
    inst = W.batched_instances()
    walk = Q.Walk([a for a, _ in inst])
    st = walk.state([b for _, b in inst]).step(50)
    keys, amps = st.export()
    F = unpack(keys, walk.nbits)
    sizes = [d["N"] * d["s"] for d in walk.info]
    order = sorted(range(len(inst)), key=lambda k: sizes[k])
    for i in order[:2] + [order[len(order) // 4], order[len(order) // 2]]:
        a, b = inst[i]
        om = oracle_mod.OracleMatrix(a)
        ok, oa = oracle_mod.OracleState(om).set_b(b).T().step(50).export()
        gk, ga = _slice(F, amps, i, om.nbits)
        compare_states(gk, ga, ok, oa, where=f"instance {i}")


def test_batched_workload_256(Q):
    """The 256-instance workload (n in 64..4096, 4..16 entries per column,
    single-column starts, 50 graph-replayed steps): every instance keeps unit
    norm and sampled instances equal their plain runs."""
    inst = W.batched_instances()
    walk = Q.Walk([a for a, _ in inst])
    st = walk.state([b for _, b in inst]).step(50)
    p = st.j_marginal()
    off = np.cumsum([0] + [d["N"] for d in walk.info])
    norms = np.array([p[off[i]:off[i + 1]].sum() for i in range(len(inst))])
    assert np.abs(norms - 1.0).max() < 1e-12
    keys, amps = st.export()
    F = unpack(keys, walk.nbits)
    for i in (0, 17, 101, 255):
        a, b = inst[i]
        n, rk, ra = _plain(Q, a, b, 50)
        gk, ga = _slice(F, amps, i, n)
        assert np.array_equal(gk, rk), i
        assert np.abs(ga - ra).max() < 1e-13, i
