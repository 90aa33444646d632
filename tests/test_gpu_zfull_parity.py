"""Full-size parity against the oracle, key by key and amplitude by
amplitude, at sizes where the oracle takes minutes (its runs start in the
background when collection ends, tests/oracle_jobs.py):
  * the benchmark's workload G(16384, 8) after 100 walk steps, in the launch
    shape the benchmark tunes and times;
  * the paper's shape C (1024 columns, s = 32) with FP64 values, 24 steps;
  * the two largest instances (4096 columns, s = 16) of the 256-instance
    batch after 50 steps of the batched launch.
The file is collected after the other GPU test files, so the oracle runs
overlap them."""
import numpy as np
import pytest

import workloads as W
from tests import oracle_jobs
from tests.parity import compare_states
from tests.test_gpu_batched import _slice, unpack

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def Q():
    import torch

    assert torch.cuda.is_available()
    import paper_2303_06890_amd as Q

    return Q


@pytest.mark.oracle_job("g16384_100")
@pytest.mark.timeout(1500)
def test_g16384_100_steps_elementwise(Q):
    from paper_2303_06890_amd import autotune

    csc, b = W.paper_scale()
    walk, shape, _ = autotune.tune_walk(csc, b)  # the configuration the benchmark times
    st = walk.state(b)
    autotune.apply(st, shape)
    st.step(100)
    assert st.stats()["real_amplitudes"]
    gk, ga = st.export()
    ok, oa, amb = oracle_jobs.result("g16384_100")[100]
    assert gk.size == ok.size == 3 * 16384 * 8 - 2
    err = compare_states(gk, ga, ok, oa, atol=1e-12, where="G(16384, 8) after 100 steps")
    oracle_jobs.record("g16384_100", max_abs_err=err, branches=gk.size, oracle_ambiguous_total=amb,
                       launch_shape=list(shape))


@pytest.mark.oracle_job("shapeC_24")
@pytest.mark.timeout(900)
def test_shape_c_fp64_24_steps(Q):
    csc, b = W.table1_band("C")
    walk = Q.Walk(csc)
    assert (walk.info[0]["N"], walk.info[0]["s"]) == (1024, 32)
    st = walk.state(b)
    snaps = oracle_jobs.result("shapeC_24")
    done, errs = 0, []
    for t in sorted(snaps):
        st.step(t - done)
        done = t
        ok, oa, _ = snaps[t]
        gk, ga = st.export()
        errs.append(compare_states(gk, ga, ok, oa, atol=1e-12, where=f"shape C after {t} steps"))
    oracle_jobs.record("shapeC_24", max_abs_err=max(errs), branches=int(gk.size))


@pytest.mark.oracle_job("batch_largest_0", "batch_largest_1")
@pytest.mark.timeout(900)
def test_batched_largest_instances_vs_oracle(Q):
    from paper_2303_06890_amd import autotune

    inst = W.batched_instances()
    bs = [b for _, b in inst]
    walk, shape, _ = autotune.tune_walk([a for a, _ in inst], bs)  # the batched leg's configuration
    st = walk.state(bs)
    autotune.apply(st, shape)
    st.step(50)
    keys, amps = st.export()
    F = unpack(keys, walk.nbits)
    for j, i in enumerate(oracle_jobs.largest_batch_instances()):
        assert walk.info[i]["N"] == 4096
        ok, oa, _ = oracle_jobs.result(f"batch_largest_{j}")[50]
        nbits = int(np.log2(walk.info[i]["N"]))
        gk, ga = _slice(F, amps, i, nbits)
        err = compare_states(gk, ga, ok, oa, atol=1e-12, where=f"batch instance {i} after 50 steps")
        oracle_jobs.record(f"batch_largest_{j}", instance=i, max_abs_err=err, branches=int(gk.size),
                           s=walk.info[i]["s"])
