"""GPU reverse-mode gradient (qw_grad: reverse sweep with W^dagger
recomputation) against the oracle's stored-state reverse mode and central
finite differences."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def Q():
    import torch

    assert torch.cuda.is_available()
    import paper_2303_06890_amd as Q

    return Q


def _scaled(csc):
    sc = 1.0 / np.abs(csc.vals).max()
    return W.Csc(csc.n, csc.colptr, csc.rowidx, csc.vals * sc)


def _oracle_csc_grad(oracle_mod, csc, b, w, nsteps):
    m = oracle_mod.OracleMatrix(csc, scale=1.0)
    loss, dv, db = m.grad(b, w, nsteps)
    col, _, _ = m.ell()
    g = np.zeros(csc.nnz)
    for c in range(csc.n):
        for p in range(csc.colptr[c], csc.colptr[c + 1]):
            g[p] = dv[c, int(np.nonzero(col[c] == csc.rowidx[p])[0][0])]
    return loss, g, db[:csc.n]


def _gpu_grad(Q, csc, b, w, nsteps):
    walk = Q.Walk(csc, scale=1.0, symmetric=False)
    st = walk.state(b).step(nsteps)
    return st.grad(w, nsteps)


def _gpu_loss(Q, csc, b, w, nsteps):
    # every stored entry is an independent parameter: a perturbed entry breaks symmetry
    walk = Q.Walk(csc, scale=1.0, symmetric=False)
    st = walk.state(b).step(nsteps)
    return float(np.dot(st.j_marginal()[:csc.n], w))


EPS = np.finfo(np.float64).eps / 2  # unit roundoff


def _floor_dv(vals, s, nsteps):
    """Rounding bound of a gradient entry w.r.t. a value a.  The entry sums
    nsteps + 1 terms (one per rotation site); each is a product of the
    adjoint and forward group amplitudes (norms <= 1 for w in [0, 1] and a
    unit b) with the derivative factor D = |df/da| + |dg/da| =
    1 / (2 sqrt|a|) + 1 / (2 sqrt(1 - |a|)); after t steps an amplitude
    carries at most t (2 s) u of rounding (a step sums the 2 s amplitudes of a
    group, u the unit roundoff).  Summed over the sites, for the two
    computations compared:  floor = 2 * 2 s u * nsteps (nsteps + 1) * D.
    Entries that are not differentiable (a = 0, |a| = 1) come out infinite."""
    a = np.abs(np.asarray(vals))
    with np.errstate(divide="ignore"):
        D = 0.5 / np.sqrt(a) + 0.5 / np.sqrt(1.0 - a)
    return 2 * 2 * s * EPS * nsteps * (nsteps + 1) * D


def _floor_db(s, nsteps):
    """Rounding bound of dL/db_j = 2 <psi~_j|lambda_0>: lambda_0 is w psi_n
    (psi_n with at most nsteps (2 s) u of rounding) carried back nsteps
    steps, another nsteps (2 s) u; the projection adds one sum of 2 s terms.
    For the two computations compared:  floor = 2 * 2 * 2 s u * (2 nsteps + 1)."""
    return 2 * 2 * 2 * s * EPS * (2 * nsteps + 1)


def _close(g, o, floor, rel=1e-8, where=""):
    """Entry by entry: |g - o| <= rel |o| + floor (finite entries)."""
    floor = np.broadcast_to(floor, np.shape(o))
    fin = np.isfinite(g) & np.isfinite(o)
    bad = np.abs(g[fin] - o[fin]) > rel * np.abs(o[fin]) + floor[fin]
    assert not bad.any(), (where, int(bad.sum()), float(np.abs(g[fin] - o[fin]).max()))
    ratio = np.abs(g[fin] - o[fin]) / (rel * np.abs(o[fin]) + floor[fin])
    return fin, float(ratio.max()), int(np.count_nonzero(floor[fin] > rel * np.abs(o[fin])))


@pytest.mark.parametrize("real_b", [False, True])
@pytest.mark.parametrize("n,c,seed,nsteps", [(16, 5, 81, 5), (64, 7, 82, 9), (64, 12, 83, 5), (64, 20, 84, 4)])
def test_grad_matches_oracle_small(Q, oracle_mod, n, c, seed, nsteps, real_b):
    """A complex b keeps the reverse sweep on the complex planes; a real b
    runs it on one double per cell (s = 8 and 16 lanes per row for s = 16
    and 32 at these sizes)."""
    csc = _scaled(W.offset_matrix(n, c, seed=seed))
    b = W.gaussian_b(n, seed=seed + 1) * (1 if real_b else (1 + 0.3j))
    b = b / np.linalg.norm(b)
    w = np.zeros(n)
    w[np.random.default_rng(seed).choice(n, size=max(2, n // 4), replace=False)] = 1.0
    ol, og, odb = _oracle_csc_grad(oracle_mod, csc, b, w, nsteps)
    gl, gg, gdb = _gpu_grad(Q, csc, b, w, nsteps)
    assert gl == pytest.approx(ol, rel=1e-12)
    s = Q.Walk(csc, scale=1.0, symmetric=False).info[0]["s"]
    fin, _, _ = _close(gg, og, _floor_dv(csc.vals, s, nsteps), where="dvals")
    assert fin.sum() >= csc.nnz - 2  # |a| = 1 entries are not differentiable
    _close(gdb, odb, _floor_db(s, nsteps), where="db")


def test_grad_1024_vs_oracle_and_fd(Q, oracle_mod):
    """G(1024, 8), uniform b, 20 steps, loss = total probability of 32 seeded
    column outcomes: gradient over all 8192 values against the oracle's
    reverse mode, and 16 entries against central differences (h = 1e-6)."""
    a, b, w = W.adjoint_problem()
    csc = _scaled(a)
    nsteps = 20
    gl, gg, gdb = _gpu_grad(Q, csc, b, w, nsteps)
    ol, og, odb = _oracle_csc_grad(oracle_mod, csc, b, w, nsteps)
    assert gl == pytest.approx(ol, rel=1e-12)
    assert gl == pytest.approx(_gpu_loss(Q, csc, b, w, nsteps), rel=1e-13)
    _, worst, by_floor = _close(gg, og, _floor_dv(csc.vals, 8, nsteps), where="dvals")
    _, worst_b, _ = _close(gdb, odb, _floor_db(8, nsteps), where="db")
    from tests import oracle_jobs

    oracle_jobs.record("grad_1024", worst_ratio=worst, entries_decided_by_floor=by_floor, worst_ratio_db=worst_b,
                       max_abs_err=float(np.nanmax(np.abs(gg - og))), max_abs_grad=float(np.nanmax(np.abs(og))))
    h = 1e-6
    for p in W.fd_sample(csc.vals):
        vp, vm = csc.vals.copy(), csc.vals.copy()
        vp[p] += h
        vm[p] -= h
        fd = (_gpu_loss(Q, W.Csc(csc.n, csc.colptr, csc.rowidx, vp), b, w, nsteps)
              - _gpu_loss(Q, W.Csc(csc.n, csc.colptr, csc.rowidx, vm), b, w, nsteps)) / (2 * h)
        assert abs(fd - gg[p]) <= 1e-8 * abs(gg[p]) + 1e-10, (p, fd, gg[p])


def test_walk_observable_autograd(Q):
    import torch

    csc = _scaled(W.offset_matrix(64, 6, seed=91))
    b = W.gaussian_b(64, seed=92)
    w = np.random.default_rng(93).uniform(size=64)
    vals = torch.tensor(csc.vals, requires_grad=True)
    bt = torch.tensor(b, requires_grad=True)
    p = Q.WalkObservable.apply(vals, bt, csc, 7)
    loss = (p * torch.tensor(w)).sum()
    loss.backward()
    gl, gg, gdb = _gpu_grad(Q, csc, b, w, 7)
    assert float(loss.detach()) == pytest.approx(gl, rel=1e-12)
    assert np.allclose(vals.grad.numpy(), gg, rtol=1e-12, atol=1e-14, equal_nan=True)
    assert np.allclose(bt.grad.numpy(), gdb.real, rtol=1e-12, atol=1e-14)


def test_grad_batched_mixed_s_on_real_planes(Q, oracle_mod):
    """Two instances of different s in one context with real b: the reverse
    sweep runs the mixed-s kernel on one double per cell; each instance's
    gradient equals the oracle's for that matrix alone."""
    mats = [_scaled(W.offset_matrix(128, 6, seed=85)), _scaled(W.offset_matrix(64, 11, seed=86))]
    bs = [W.uniform_b(128), W.gaussian_b(64, seed=87)]
    bs[1] = bs[1] / np.linalg.norm(bs[1])
    ws = [np.zeros(128), np.zeros(64)]
    ws[0][::5] = 1.0
    ws[1][1::3] = 1.0
    nsteps = 7
    walk = Q.Walk(mats, scale=1.0, symmetric=False)
    assert len({d["s"] for d in walk.info}) == 2
    st = walk.state(bs).step(nsteps)
    assert st.stats()["real_amplitudes"]
    gl, gg, gdb = st.grad(np.concatenate(ws), nsteps)
    off, boff, total = 0, 0, 0.0
    for csc, b, w, d in zip(mats, bs, ws, walk.info):
        ol, og, odb = _oracle_csc_grad(oracle_mod, csc, b, w, nsteps)
        total += ol
        _close(gg[off:off + csc.nnz], og, _floor_dv(csc.vals, d["s"], nsteps), where=f"dvals n={csc.n}")
        _close(gdb[boff:boff + csc.n], odb, _floor_db(d["s"], nsteps), where=f"db n={csc.n}")
        off += csc.nnz
        boff += csc.n
    assert gl == pytest.approx(total, rel=1e-12)


@pytest.mark.parametrize("lanes", [8, 16])
def test_grad_s64_rows_split(Q, oracle_mod, lanes):
    """s = 64 (a band of half-width 31 on 64 rows, real b): in 256-thread
    workgroups the one-pass adjoint kernels split each row over two (eight
    lanes per row) or four (sixteen) wavefronts, joining both group sums
    through LDS; the gradient entry by entry against the oracle's reverse
    mode, and against the whole-row form of 64-thread workgroups up to
    rounding.  (The oracle's stored-state reverse mode grows steeply with the
    steps at s = 64: 0.5 s for 4 steps here, about 2 minutes for 4 steps on
    128 rows.)"""
    n, nsteps = 64, 4
    csc = _scaled(W.band_matrix(n, 31, seed=87))
    b = W.gaussian_b(n, seed=88)
    b = b / np.linalg.norm(b)
    w = np.zeros(n)
    w[np.random.default_rng(89).choice(n, size=n // 4, replace=False)] = 1.0
    ol, og, odb = _oracle_csc_grad(oracle_mod, csc, b, w, nsteps)
    out = {}
    for wg in (256, 64):
        walk = Q.Walk(csc, scale=1.0, symmetric=False, lanes=lanes)
        assert walk.info[0]["s"] == 64
        waves = n * lanes // 64
        st = walk.state(b)
        st.set_launch(wg, waves // (wg // 64))
        st.step(nsteps)
        assert st.stats()["real_amplitudes"]
        gl, gg, gdb = st.grad(w, nsteps)
        assert gl == pytest.approx(ol, rel=1e-12)
        fin, _, _ = _close(gg, og, _floor_dv(csc.vals, 64, nsteps), where=f"dvals lanes={lanes} wg={wg}")
        assert fin.sum() >= csc.nnz - 2
        _close(gdb, odb, _floor_db(64, nsteps), where=f"db lanes={lanes} wg={wg}")
        out[wg] = (gg, gdb)
        walk.close()
    fin = np.isfinite(out[256][0]) & np.isfinite(out[64][0])
    assert np.allclose(out[256][0][fin], out[64][0][fin], rtol=1e-12, atol=1e-15)
