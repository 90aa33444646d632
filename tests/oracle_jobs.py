"""Oracle runs of the full-size parity cases, started in background threads
as soon as pytest has collected a test that needs one (tests/conftest.py),
so that they overlap the GPU tests collected ahead of it.  The oracle's C
calls release the interpreter lock.  Each job logs one line per walk step to
oracle_jobs.log in the directory named by QW_TEST_LOG_DIR (else the system's
temporary directory), so that a long run shows progress."""
import os
import tempfile
import threading
import time

import numpy as np

import workloads as W

_jobs = {}
_lock = threading.Lock()


def _log_path():
    d = os.environ.get("QW_TEST_LOG_DIR") or tempfile.gettempdir()
    os.makedirs(d, exist_ok=True)
    return os.path.join(d, "oracle_jobs.log")


def _log(msg):
    with _lock, open(_log_path(), "a") as f:
        f.write(f"{time.strftime('%H:%M:%S')} {msg}\n")


def largest_batch_instances(count=2):
    """Indices of the `count` instances of the 256-instance workload with the
    most slots (N s), largest last."""
    inst = W.batched_instances()

    def slots(i):
        a = inst[i][0]
        n = 1 << max(1, int(np.ceil(np.log2(a.n))))
        s = 1 << int(np.ceil(np.log2(max(1, np.diff(a.colptr).max()))))
        return (n * s, i)

    return sorted(range(len(inst)), key=slots)[-count:]


def _walk(name, csc, b, snapshots):
    """T~|b~> then walk steps; exports at the given step counts."""
    import oracle

    st = oracle.OracleState(oracle.OracleMatrix(csc)).set_b(b).T()
    out = {}
    t0 = time.time()
    for t in range(1, max(snapshots) + 1):
        st.step(1)
        _log(f"{name}: step {t}/{max(snapshots)}, {st.count()} branches, {time.time() - t0:.0f} s")
        if t in snapshots:
            k, a = st.export()
            out[t] = (k, a, st.ambiguous(total=True))
    return out


def _spec(name):
    if name == "g16384_100":
        csc, b = W.paper_scale()
        return csc, b, (100,)
    if name == "shapeC_24":
        csc, b = W.table1_band("C")
        return csc, b, (1, 12, 24)
    if name.startswith("batch_largest_"):
        i = largest_batch_instances()[int(name.rsplit("_", 1)[1])]
        a, b = W.batched_instances()[i]
        return a, b, (50,)
    raise KeyError(name)


class _Job:
    def __init__(self, name):
        self.name = name
        self.result = None
        self.error = None
        self.done = threading.Event()
        self.thread = threading.Thread(target=self._run, name=f"oracle-{name}", daemon=True)

    def _run(self):
        try:
            csc, b, snaps = _spec(self.name)
            self.result = _walk(self.name, csc, b, snaps)
        except BaseException as e:  # reported to the test that waits
            self.error = e
        finally:
            self.done.set()


def start(names):
    """Start the named jobs (once each)."""
    for name in sorted(names):
        if name not in _jobs:
            _spec(name)  # unknown names fail here, at collection
            _jobs[name] = _Job(name)
            _log(f"{name}: started")
            _jobs[name].thread.start()


def result(name, timeout=1200.0):
    """{step: (keys, amps, ambiguous count so far)} of a job, waiting for it."""
    start([name])
    job = _jobs[name]
    if not job.done.wait(timeout):
        raise TimeoutError(f"oracle job {name} did not finish in {timeout} s")
    if job.error is not None:
        raise job.error
    return job.result


def record(name, **stats):
    """Append a line of measured statistics (errors, counts) of a GPU test to
    test_stats.jsonl beside the job log."""
    import json

    with _lock, open(os.path.join(os.path.dirname(_log_path()), "test_stats.jsonl"), "a") as f:
        f.write(json.dumps({"test": name, **{k: float(v) if np.isscalar(v) else v for k, v in stats.items()}}) + "\n")
