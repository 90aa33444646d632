"""The context's buffer pool: a state made from buffers a freed state left
behind (its planes, 8-byte planes, counters, list) starts exactly as a state
from fresh buffers does; the gradient's pooled arrays likewise."""
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


@pytest.mark.parametrize("complex_b", [False, True])
def test_reused_buffers_start_clean(Q, complex_b):
    csc = W.offset_matrix(256, 8, seed=301)
    b = W.gaussian_b(256, seed=302) * (np.exp(0.2j * np.arange(256)) if complex_b else 1.0)
    walk = Q.Walk(csc)
    ref = walk.state(b).step(20)
    rk, ra = ref.export()
    rt = ref.stats()["total_written"]
    ref.close()
    for seed in (303, 304, 305):
        dirty = walk.state(W.gaussian_b(256, seed=seed)).step(37)  # other contents in the buffers
        dirty.close()
        raw = walk.state(W.gaussian_b(256, seed=seed), raw=True).step(5)  # a filled branch list
        raw.close()
        st = walk.state(b).step(20)
        k, a = st.export()
        assert np.array_equal(k, rk) and np.array_equal(a, ra), seed
        assert st.stats()["total_written"] == rt, seed
        st.close()


def test_gradient_twice(Q):
    a, b, w = W.adjoint_problem(n=256, c=8)
    sc = 1.0 / np.abs(a.vals).max()
    a = W.Csc(a.n, a.colptr, a.rowidx, a.vals * sc)
    walk = Q.Walk(a, scale=1.0, symmetric=False)
    first = walk.state(b).step(12).grad(w, 12)
    for _ in range(2):
        again = walk.state(b).step(12).grad(w, 12)
        assert again[0] == first[0]
        assert np.array_equal(again[1], first[1]) and np.array_equal(again[2], first[2])
