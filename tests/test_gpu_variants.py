"""Every one-pass step kernel family of one s against the oracle, element by
element after 12 steps: s = 1 ... 64; eight or sixteen lanes per row for
s >= 16 (so one, two, four or eight slots per lane: the kernels that read
the rotation table and those that take the square roots, the row sums that
cross rows with the permlane swaps and with lane shuffles); matrices whose
slots all have a partner and band matrices with unpartnered fillers (the two
forms of the Q0 load); a real b (one double per cell) and a complex b (the
complex planes)."""
import numpy as np
import pytest

import workloads as W
from tests.parity import compare_states

pytestmark = pytest.mark.gpu

STEPS = 12


def _matrix(s, kind):
    """(csc, rows): G(N, s) has exactly s entries in every column, so no
    fillers and every slot paired; the band of half-width (s - 1) // 2 has
    fillers at its edges, slots without a partner."""
    n = 64 if s == 64 else (128 if s == 32 else 256)
    if s == 1:  # a positive diagonal (a negative one is not encodable)
        return W.band_matrix(n, 0, seed=11)
    if kind == "paired":
        return W.offset_matrix(n, s, seed=10 + s)
    return W.band_matrix(n, (s - 1) // 2, seed=20 + s)


CASES = []
for s in (1, 2, 4, 8, 16, 32, 64):
    for lanes in ((8, 16) if s >= 16 else (0,)):
        for kind in (("paired", "band") if s >= 4 else ("paired",)):
            CASES.append((s, lanes, kind))


@pytest.fixture(scope="module")
def Q():
    import torch

    assert torch.cuda.is_available()
    import paper_2303_06890_amd as Q

    return Q


@pytest.mark.parametrize("b_kind", ["real", "complex"])
@pytest.mark.parametrize("s,lanes,kind", CASES)
def test_kernel_family_matches_the_oracle(Q, oracle_mod, s, lanes, kind, b_kind):
    csc = _matrix(s, kind)
    b = W.gaussian_b(csc.n, seed=s + lanes)
    if b_kind == "complex":
        b = b * (1 + 0.5j)
    b = b / np.linalg.norm(b)
    walk = Q.Walk(csc, lanes=lanes)
    assert walk.info[0]["s"] == s
    st = walk.state(b).step(STEPS)
    stats = st.stats()
    assert stats["real_amplitudes"] == (b_kind == "real")
    if s >= 16:
        assert stats["lanes_per_row_s16"] == lanes
    ost = oracle_mod.OracleState(oracle_mod.OracleMatrix(csc)).set_b(b).T().step(STEPS)
    gk, ga = st.export()
    ok, oa = ost.export()
    compare_states(gk, ga, ok, oa, where=f"s={s} lanes={lanes} {kind} {b_kind} b")
