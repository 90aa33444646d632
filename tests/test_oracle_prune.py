"""Pins of the oracle's zero-clearing rule (Sec. V.A: the interference
operation ends by removing zero branches).

The reading taken (pruning threshold tau = 1e-13): a branch is removed when
|Re| <= tau and |Im| <= tau, and only at the boundary of a whole W, W^dagger
or T~; inside a step only exact zeros go.  The reference here is the dense
state-vector simulator (tests/dense_sim.py), which never prunes: the test
applies the rule itself, once per boundary, to the dense vector and compares
the surviving key set, the pruned probability and the count of amplitudes
within 1e-15 of tau with what the oracle reports.

Each wrong reading of the rule fails one of these tests (checked by
tests/test_oracle_prune_mutants.py, which rebuilds the oracle with each):
  * removal by modulus (|amp| <= tau): the branch (0.9, 0.9) tau;
  * removal when either part is small ("or"): the branch (0, -1.1) tau;
  * removal after every operation instead of at the boundary: a branch of
    1.5 tau that the Hadamard fan-out of T~^dagger splits below tau and T~
    recombines, and the raw tridiagonal start, whose wavefront carries
    amplitudes near 1e-13.
"""
import numpy as np
import pytest

import workloads as W
from dense_sim import DenseWalk

TAU = 1e-13
MARGIN = 1e-15


def _key(nbits, jc, j, b1, kc, k, b2):
    key = 0
    for v, w in ((jc, nbits), (j, nbits), (b1, 1), (kc, nbits), (k, nbits), (b2, 1)):
        key = (key << w) | int(v)
    return key


def _boundary_rule(psi):
    """The reading applied to a dense vector: (kept vector, pruned mass,
    number of amplitudes within MARGIN of TAU)."""
    mx = np.maximum(np.abs(psi.real), np.abs(psi.imag))
    drop = mx <= TAU
    mass = float(np.sum(np.abs(psi[drop]) ** 2))
    amb = int(np.count_nonzero(np.abs(mx - TAU) <= MARGIN))
    out = psi.copy()
    out[drop] = 0.0
    return out, mass, amb


def _dense_of(st, size):
    keys, amps = st.export()
    psi = np.zeros(size, complex)
    psi[keys.astype(np.int64)] = amps
    return psi


def _assert_same(st, ref, where):
    keys, amps = st.export()
    want = np.nonzero(ref)[0].astype(np.uint64)
    assert np.array_equal(keys, want), (
        f"{where}: {np.setdiff1d(want, keys).size} kept branches missing, "
        f"{np.setdiff1d(keys, want).size} extra")
    assert np.abs(amps - ref[keys.astype(np.int64)]).max() <= 1e-14 * max(1.0, np.abs(ref).max())


# Hand-placed branches around tau.  Branches with b1 = 1 lie outside the span
# of the T~|j~> (b1 = 0 there), so W maps them to -S(key): the amplitude
# comes out negated at the swapped key, and its position relative to tau is
# set by the input alone.  b2 = 1 keeps the images (b1 = b2 = 1) apart from
# every key a group member can reach.
PLACED = {
    "kept_real": 1.2e-13,
    "both_parts_below": 0.9e-13 + 0.9e-13j,  # |amp| = 1.27e-13 > tau, yet removed
    "imag_only": -1.1e-13j,                  # Re = 0 <= tau, yet kept
    "tau_plus_2e-15": TAU + 2e-15,
    "tau_minus_2e-15": TAU - 2e-15,
    "margin_above": TAU + 0.5e-15,           # kept, and counted as ambiguous
    "margin_below": -(TAU - 0.4e-15) * 1j,   # removed, and counted as ambiguous
    "split_mid_step": 1.5e-13,               # below tau after the fan-out of T~^dagger
}


def _placed_state(nbits):
    keys, amps, names = [], [], []
    for i, (name, a) in enumerate(PLACED.items()):
        j, k = (3 * i + 1) % 16, (5 * i + 2) % 16
        keys.append(_key(nbits, 0, j, 1, 0, k, 1))
        amps.append(a)
        names.append(name)
    # two group members of ordinary size, so that the step also reflects,
    # fans out and leaves rounding residues that the boundary must remove
    keys += [_key(nbits, 0, 2, 0, 0, 0, 0), _key(nbits, 0, 5, 0, 0, 0, 1)]
    amps += [0.6, -0.3 + 0.2j]
    return np.array(keys, np.uint64), np.array(amps, complex), names


def _member_keys(m, nbits, j):
    col, _, _ = m.ell()
    return [_key(nbits, 0, j, 0, 0, int(c), b2) for c in col[j] for b2 in (0, 1)]


def test_one_step_survivors_mass_and_margin(oracle_mod):
    """One W on hand-placed branches: survivors, pruned mass and margin count
    equal the rule applied to the unpruned dense step."""
    csc = W.offset_matrix(16, 5, seed=7)  # s = 8: fillers, negative entries
    m = oracle_mod.OracleMatrix(csc)
    dw = DenseWalk(csc)
    keys, amps, names = _placed_state(m.nbits)
    # the group members must be real members (their columns are in the row)
    keys[-2] = _member_keys(m, m.nbits, 2)[0]
    keys[-1] = _member_keys(m, m.nbits, 5)[3]
    psi = np.zeros(dw.size, complex)
    psi[keys.astype(np.int64)] = amps
    out = dw.W(psi)
    ref, mass, amb = _boundary_rule(out)
    st = oracle_mod.OracleState(m).import_(keys, amps).step(1)
    _assert_same(st, ref, "W")
    # the placed branches land where the rule says, with the outcome intended
    for name, k0, a in zip(names, keys, amps):
        img = int(dw.s_perm[int(k0)])
        assert abs(out[img] + a) <= 1e-28, name  # -S(key), amplitude negated
    kept = {n: bool(ref[int(dw.s_perm[int(k)])] != 0) for n, k in zip(names, keys)}
    assert kept == {"kept_real": True, "both_parts_below": False, "imag_only": True, "tau_plus_2e-15": True,
                    "tau_minus_2e-15": False, "margin_above": True, "margin_below": False,
                    "split_mid_step": True}
    assert amb >= 2
    assert st.ambiguous() == amb
    assert st.pruned_mass() == pytest.approx(mass, rel=1e-9, abs=1e-30)  # rounding residues: < 1e-15 each


def test_split_branch_falls_below_tau_inside_the_step(oracle_mod):
    """The 1.5 tau branch really is below tau after T~^dagger's fan-out: a
    rule applied there would lose it (it survives the step above)."""
    csc = W.offset_matrix(16, 5, seed=7)
    m = oracle_mod.OracleMatrix(csc)
    dw = DenseWalk(csc)
    keys, amps, names = _placed_state(m.nbits)
    i = names.index("split_mid_step")
    psi = np.zeros(dw.size, complex)
    psi[int(keys[i])] = amps[i]
    mid = dw.Tdag(psi)
    assert np.count_nonzero(np.abs(mid) > 1e-20) >= 8
    assert np.maximum(np.abs(mid.real), np.abs(mid.imag)).max() < TAU
    assert abs(dw.W(psi)[int(dw.s_perm[int(keys[i])])] + amps[i]) < 1e-28


def test_prepare_survivors_mass_and_margin(oracle_mod):
    """T~ on a raw |b~> whose entries put its outputs b_j f / sqrt(s) and
    b_j g / sqrt(s) around tau, with complex b_j so that both the modulus and
    the separate parts decide differently."""
    csc = W.offset_matrix(16, 5, seed=7)
    m = oracle_mod.OracleMatrix(csc)
    dw = DenseWalk(csc)
    rng = np.random.default_rng(21)
    mag = TAU * np.sqrt(m.s) * rng.uniform(0.9, 2.5, 16)
    b = mag * np.exp(1j * rng.choice([0.0, np.pi / 4, np.pi / 2, 3 * np.pi / 4], 16))
    out = dw.T(dw.basis_b(b))
    ref, mass, amb = _boundary_rule(out)
    mx = np.maximum(np.abs(out.real), np.abs(out.imag))
    nz = np.abs(out) > 1e-20
    # the input exercises every side of the rule
    assert np.any(nz & (np.abs(out) > TAU) & (mx <= TAU))  # modulus above, both parts below
    assert np.any((mx > TAU) & (np.minimum(np.abs(out.real), np.abs(out.imag)) <= TAU))
    assert np.any(nz & (mx <= TAU)) and np.any(mx > TAU)
    st = oracle_mod.OracleState(m).set_b(b).T()
    _assert_same(st, ref, "T~")
    assert st.ambiguous() == amb
    assert st.pruned_mass() == pytest.approx(mass, rel=1e-9, abs=1e-30)  # rounding residues: < 1e-15 each


def _walk_against_dense(oracle_mod, csc, b, prepare, steps, jc_dim=None):
    m = oracle_mod.OracleMatrix(csc)
    dw = DenseWalk(csc, jc_dim=jc_dim)
    psi = dw.basis_b(b)
    st = oracle_mod.OracleState(m).set_b(b)
    if prepare:
        psi, _, _ = _boundary_rule(dw.T(psi))
        st.T()
    pruned_steps = 0
    for t in range(steps):
        psi, mass, _ = _boundary_rule(dw.W(psi))
        st.step(1)
        pruned_steps += mass > 0
        keys, amps = st.export()
        mx = np.maximum(np.abs(psi.real), np.abs(psi.imag))
        band = np.abs(mx - TAU) <= MARGIN
        # keys outside the margin band: equal sets
        got = keys[~band[keys.astype(np.int64)]]
        want = np.nonzero((psi != 0) & ~band)[0].astype(np.uint64)
        assert np.array_equal(got, want), (t, np.setdiff1d(want, got).size, np.setdiff1d(got, want).size)
        ref = psi[keys.astype(np.int64)]
        assert np.abs(amps - ref).max() < 1e-14, t
    return pruned_steps


def test_raw_tridiagonal_start_100_steps(oracle_mod):
    """The raw single-column start of the tridiagonal 16 x 16 matrix: its
    wavefront carries genuine amplitudes near 1e-13, which the rule removes
    step after step."""
    csc, b = W.tiny_tridiagonal()
    pruned = _walk_against_dense(oracle_mod, csc, b, prepare=False, steps=100)
    assert pruned >= 10  # the rule acts on many boundaries


@pytest.mark.slow
def test_cyclic32_prepared_start_100_steps(oracle_mod):
    """T~|b~> on a cyclic-offset 32 x 32 matrix (5 entries per column, s = 8,
    fillers, negative entries), 100 steps; the dense vector (2^20 amplitudes)
    holds j_c < s only, which the walk never leaves.  At 64 x 64 the same
    dense walk costs about 3 s per step, too slow for this suite."""
    csc = W.offset_matrix(32, 5, seed=31)
    b = W.gaussian_b(32, seed=32)
    _walk_against_dense(oracle_mod, csc, b, prepare=True, steps=100, jc_dim=8)
