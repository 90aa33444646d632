#!/usr/bin/env python3
"""Walk-step throughput on one MI355X.

Workload: the 16384-dimensional real symmetric matrix with 8 stored entries
per column (diagonal + 3 mirrored seeded random cyclic offsets + offset N/2,
values U[-1,1], diagonal shifted by +7, seed 2), rescaled by its largest
entry; start T~|b~> with b the uniform superposition over all 16384 columns;
FP64 amplitudes (one double per cell: the matrix is real symmetric and b
real).  One benchmark step is one walk step W (one launch of the fused step
kernel) on that state; the state reaches its steady size of 3Ns - 2 = 393214
branches after the second step, so warm-up steps put the timed region in the
steady state.  After the warm-up steps one more untimed call of the timed
step count captures the step graphs that the timed call replays.

Output: one JSON line on stdout with the metric (amplitude updates/s = sum
over timed steps of the branches each step writes, divided by the time of the
step loop), the roofline of the step kernel (algorithmic bytes per launch =
24 B x (branches in + branches out) + 12 B x ELL slots, divided by the
average launch time measured with HIP events on the kernels' stream, against
8 TB/s), and the oracle's rate on the host CPU for a bounded sample.
"""
import argparse
import hashlib
import json
import os
import re
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
VERBOSE = False  # --verbose: the autotuner prints every candidate it times (progress of long runs)
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "step_kernel_G16384x8_traffic.md")
BATCHED_TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "batched_256_instances_traffic.md")
E_TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "step_kernel_E_traffic.md")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2303_06890_amd", "csrc", f) for f in ("qw_kernels.hip", "qw_internal.h")]


def measured_traffic(path: str = TRAFFIC_PROFILE, xcd: bool = False, lanes16: bool = False):
    """HBM bytes per step launch from a committed counter summary (calibrated
    FETCH_SIZE + WRITE_SIZE) for one tile: the library's lane mapping or
    sixteen lanes per row (lanes16), row blocks in the plain numbering or by
    XCD (xcd, QW_XCD_ROWS).  None when the summary is missing, lacks that
    tile's figure or was taken on other kernel sources than the ones in this
    tree."""
    try:
        with open(path) as f:
            text = f.read()
        digest = hashlib.sha256(b"".join(open(p, "rb").read() for p in KERNEL_SOURCES)).hexdigest()
    except OSError:
        return None
    key = "traffic_bytes_per_launch" + ("_lanes16" if lanes16 else "") + ("_xcd" if xcd else "")
    m = re.search(key + r": (\d+)", text)
    h = re.search(r"sha256 ([0-9a-f]{64})", text)
    if not m or not h or h.group(1) != digest:
        return None
    return float(m.group(1))


def xcd_active(walk, shape) -> bool:
    """Whether the step kernels of `walk` at launch `shape` number their row
    blocks by XCD: the walk was loaded with the numbering and the grid is a
    multiple of 8 (other grids run the plain numbering)."""
    return bool(walk.xcd and shape and int(shape[1]) % 8 == 0)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def cpu_baseline(csc, b, steps: int):
    """The oracle (single-threaded std::map model) on the same workload:
    T~|b~> then `steps` walk steps; rate = branches written / time of the
    step loop."""
    import oracle

    om = oracle.OracleMatrix(csc)
    ost = oracle.OracleState(om).set_b(b).T()
    # The oracle runs on the calling thread: pin it to one core while timed.
    saved = os.sched_getaffinity(0)
    core = min(saved)
    os.sched_setaffinity(0, {core})
    try:
        written = 0
        t0 = time.perf_counter()
        for _ in range(steps):
            ost.step(1)
            written += ost.count()
        dt = time.perf_counter() - t0
    finally:
        os.sched_setaffinity(0, saved)
    return {
        "value": written / dt,
        "unit": "amplitude updates/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"T~|b~> then {steps} walk steps of the same 16384-dim workload "
                  f"({written} branch updates in {dt:.1f} s), one thread pinned to core {core} of {cpu_model()} "
                  f"(nproc={os.cpu_count()})",
    }


def batched_cpu_baseline(inst, steps: int = 10, count: int = 64):
    """The oracle over independent instances on the host's cores (a thread
    pool; the oracle's C calls release the interpreter lock): T~|b~> then
    `steps` walk steps of the first `count` instances of the batched
    workload."""
    from concurrent.futures import ThreadPoolExecutor

    import oracle

    threads = max(1, min(16, os.cpu_count() or 1))
    sample = inst[:count]
    mats = [oracle.OracleMatrix(a) for a, _ in sample]

    def run(i):
        ost = oracle.OracleState(mats[i]).set_b(sample[i][1]).T()
        written = 0
        for _ in range(steps):
            ost.step(1)
            written += ost.count()
        return written

    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as pool:
        written = sum(pool.map(run, range(len(sample))))
    dt = time.perf_counter() - t0
    return {
        "value": written / dt,
        "unit": "amplitude updates/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"first {len(sample)} of the 256 instances, T~|b~> then {steps} walk steps each "
                  f"({written} branch updates in {dt:.1f} s), {threads} threads on {cpu_model()}",
    }


def launch_floors(torch, launches: int = 256):
    """Per-launch time of an empty kernel and of one coalesced kernel moving
    about the step's bytes (4.5 MB read, 2.25 MB written; the counters
    measure 4.25 and 2.25 MB for one step on one double per cell), each back
    to back in a graph of `launches` launches: the floors of the step kernel
    at 16384 x 8."""
    out = {}
    tiny = torch.zeros(1, device="cuda")
    n = 2_250_000 // 8
    src = torch.ones(2 * n, dtype=torch.float64, device="cuda")
    dst = torch.zeros(n, dtype=torch.float64, device="cuda")
    s = torch.cuda.Stream()
    for name, op in (("empty_kernel_us", lambda: tiny.zero_()),
                     ("copy_floor_us", lambda: torch.add(src[:n], src[n:], out=dst))):
        g = torch.cuda.CUDAGraph()
        with torch.cuda.stream(s):  # capture and replay on s, where the events are recorded
            op()
            torch.cuda.synchronize()
            with torch.cuda.graph(g, stream=s):
                for _ in range(launches):
                    op()
            g.replay()
            torch.cuda.synchronize()
            best = None
            for _ in range(3):
                t = _timed_on(torch, s, g.replay) * 1e3 / launches
                best = t if best is None else min(best, t)
        out[name] = best
    return out


SPACER_CYCLES = 250_000  # about 0.1 ms of GPU clock


def _timed_on(torch, stream, fn):
    """GPU time (ms) of the work fn() enqueues on `stream`, by HIP events on
    that stream.  The device is synchronised first; then torch's
    clock-counting wait kernel (a fixed number of GPU cycles, about 0.1 ms;
    it touches no memory, so the caches keep the state) is enqueued ahead of
    the start event, so that the host has queued fn()'s work before the GPU
    reaches the start event: the interval between the events holds that work
    alone, run back to back, and not the host's time to submit it."""
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        torch.cuda._sleep(SPACER_CYCLES)
    e0.record(stream)
    t0 = time.perf_counter()
    fn()
    HOST_MS.append((time.perf_counter() - t0) * 1e3)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1)


HOST_MS = []  # host time of each timed call (ms), to compare with the spacer


def spacer_ms(torch, stream):
    """GPU time of the spacer alone (ms)."""
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    with torch.cuda.stream(stream):
        torch.cuda._sleep(SPACER_CYCLES)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1)


def _timed(Q, fn):
    """GPU time (ms) of fn() on the library's stream (see _timed_on)."""
    import torch

    return _timed_on(torch, Q.stream(), fn)


def host_inclusive_leg(Q, csc, b, lanes: int, shape, steps: int, updates_per_step: float, reps: int = 5):
    """The same walk from host memory to host memory: the matrix loaded from
    host CSC arrays (preprocessing and tables included), then, per job, the
    state made from the host vector b, `steps` walk steps and the export of
    every branch (packed keys and complex amplitudes) into host arrays.  Host
    wall clock, median of `reps` jobs; a second pass with a synchronisation
    after each part gives the split."""
    import numpy as np
    import torch

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    walk = Q.Walk(csc, lanes=lanes)
    torch.cuda.synchronize()
    load_ms = (time.perf_counter() - t0) * 1e3

    def job(split):
        t = [time.perf_counter()]
        st = walk.state(b)
        if shape:
            st.set_launch(*shape)
        if split:
            torch.cuda.synchronize()
            t.append(time.perf_counter())
        st.step(steps)
        if split:
            torch.cuda.synchronize()
            t.append(time.perf_counter())
        keys, amps = st.export()
        t.append(time.perf_counter())
        st.close()
        return [1e3 * (y - x) for x, y in zip(t, t[1:])], keys.nbytes + amps.nbytes

    job(False)  # captures the graph of this step count
    jobs = sorted(job(False)[0][0] for _ in range(reps))
    split, export_bytes = job(True)
    ms = jobs[reps // 2]
    # The way back: the exported branches imported into a fresh state.
    st = walk.state(b)
    keys, amps = st.step(steps).export()
    st.close()
    imp = walk.state(np.zeros(len(b)))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    imp.import_(keys, amps)
    torch.cuda.synchronize()
    import_ms = (time.perf_counter() - t0) * 1e3
    imp.close()
    walk.close()
    return {
        "what": "host b in, walk steps, every branch exported to host (keys + amplitudes); host wall clock",
        "steps": steps,
        "ms_per_job": ms,
        "updates_per_s": updates_per_step * steps / (ms / 1e3),
        "split_ms": {"state_from_host_b": split[0], "steps": split[1], "export_to_host": split[2]},
        "export_bytes": export_bytes,
        "import_of_export_ms": import_ms,
        "matrix_load_ms": load_ms,
    }


def batched_leg(Q, W, autotune, tune: bool, steps: int = 50, cpu: bool = True):
    """256 instances (n = 2^U{6..12}, 4..16 entries per column, single-column
    starts) in one launch per step, against the same instances advanced one
    walk at a time on the same GPU."""
    inst = W.batched_instances()
    mats, bs = [a for a, _ in inst], [b for _, b in inst]
    walk, shape, tune_log = autotune.tune_walk(mats, bs, verbose=VERBOSE) if tune else (Q.Walk(mats), None, None)
    st = walk.state(bs)
    if shape:
        autotune.apply(st, shape)
    st.step(steps)  # the same call untimed: captures the step graphs outside the timed region
    s0 = st.stats()
    ms = _timed(Q, lambda: st.step(steps))
    s1 = st.stats()
    upd = s1["total_written"] - s0["total_written"]
    upd_in = upd - s1["branches"] + s0["branches"]
    slots = int(sum(d["N"] * d["s"] for d in walk.info))
    traffic = measured_traffic(BATCHED_TRAFFIC_PROFILE, xcd=xcd_active(walk, shape), lanes16=walk.lanes == 16)
    step_s = ms / 1e3 / steps
    singles = []
    for a, b in inst:
        w1 = Q.Walk(a)
        singles.append((w1, w1.state(b).step(steps)))
    t0 = [x[1].stats()["total_written"] for x in singles]
    ms_plain = _timed(Q, lambda: [x[1].step(steps) for x in singles])
    upd_plain = sum(x[1].stats()["total_written"] - t for x, t in zip(singles, t0))
    assert upd_plain == upd, (upd_plain, upd)
    return {
        "workload": "256 instances, n = 2^U{6..12}, 4..16 entries/column, single-column T~ starts, 50 steps",
        "slots": slots,
        "steps": steps,
        "ms": ms,
        "value": upd / (ms / 1e3),
        "plain_ms": ms_plain,
        "plain_value": upd_plain / (ms_plain / 1e3),
        "speedup_vs_plain": ms_plain / ms,
        # against HBM: the counters' bytes per launch (the state, ~150 MB in
        # doubles, does not fit the caches); the algorithmic bytes (24 B per
        # branch in and out + 12 B per slot) count keys and complex values
        # this layout does not move, so they exceed what the kernel reads
        "roofline": {
            "bound": "hbm",
            "kernel": "batched step kernel",
            "traffic": traffic,
            "achieved": traffic / step_s / 1e9 if traffic else None,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": traffic / step_s / 1e9 / HBM_PEAK_GBS if traffic else None,
            "alg_bytes_per_launch": (24.0 * (upd + upd_in) + 12.0 * slots * steps) / steps,
        },
        "launch_shape": list(shape) if shape else "default",
        "autotune": tune_log,
        "cpu_baseline": batched_cpu_baseline(inst) if cpu else None,
    }


def table1_leg(Q, W, autotune, tune: bool):
    """Walk steps on band matrices of the shapes of the paper's five
    experiments (n = 16 ... 16384, s = 8 ... 64), uniform b, T~ start; the
    paper's single-core time per step is quoted as context only (another
    machine, another code)."""
    def run(csc, b, word):
        walk, shape, tune_log = autotune.tune_walk(csc, b, word=word, verbose=VERBOSE) if tune else (Q.Walk(csc, word=word), None, None)
        st = walk.state(b)
        if shape:
            autotune.apply(st, shape)
        steps = 2000 if csc.n <= 1024 else 400
        st.step(steps)  # the same call untimed (graph capture)
        s0 = st.stats()
        ms = _timed(Q, lambda: st.step(steps))
        upd = st.stats()["total_written"] - s0["total_written"]
        res = {
            "s": walk.info[0]["s"],
            "branches": st.count(),
            "us_per_step": 1e3 * ms / steps,
            "value": upd / (ms / 1e3),
            "launch_shape": list(shape) if shape else "default",
            "lanes_per_row": tune_log["chosen_lanes_per_row"] if tune_log else "default",
            "xcd_rows": tune_log["chosen_xcd_rows"] if tune_log else False,
            "xcd_rows_active": xcd_active(walk, shape),
            "autotune_tiles": tune_log["tile_choices"] if tune_log else None,
        }
        st.close()
        return res

    out = {}
    for name in ("A", "B", "C", "D", "E"):
        csc, b = W.table1_band(name)
        res = run(csc, b, 0)
        paper = W.TABLE1_PAPER_SECONDS_PER_STEP[name]
        res.update(n=csc.n, paper_single_core_s_per_step=paper,
                   time_ratio_vs_paper=paper / (res["us_per_step"] * 1e-6))
        # the same shape with the table's fixed-point entries and word length
        fcsc, fb, word = W.table1_fixed_point_band(name)
        fx = run(fcsc, fb, word)
        res["fixed_point"] = {"word_length": word, "us_per_step": fx["us_per_step"], "value": fx["value"],
                              "branches": fx["branches"], "launch_shape": fx["launch_shape"]}
        if name == "E" and res["lanes_per_row"] in ([8], [16]):
            # counters of each tile the tuner can choose for this shape
            traffic = measured_traffic(E_TRAFFIC_PROFILE, xcd=res["xcd_rows_active"], lanes16=res["lanes_per_row"] == [16])
            res["traffic"] = traffic
            res["counter_gbs"] = traffic / (res["us_per_step"] * 1e-6) / 1e9 if traffic else None
        out[name] = res
    return out


def complex_leg(Q, W, autotune, tune: bool, steps: int = 2000):
    """The main workload's shape with complex Hermitian values: 16384 columns,
    8 entries per column (the off-diagonal pairs v, conj(v)), uniform b."""
    csc = W.hermitian_offset_matrix(16384, 8, seed=2)
    b = W.uniform_b(16384)
    walk, shape, _ = autotune.tune_walk(csc, b, verbose=VERBOSE) if tune else (Q.Walk(csc), None, None)
    st = walk.state(b)
    if shape:
        autotune.apply(st, shape)
    st.step(steps)  # the same call untimed (graph capture)
    s0 = st.stats()
    ms = _timed(Q, lambda: st.step(steps))
    upd = st.stats()["total_written"] - s0["total_written"]
    return {
        "workload": "complex Hermitian offset matrix n = 16384, 8 entries/column, seed 2, uniform b, T~ start",
        "branches": st.count(),
        "us_per_step": 1e3 * ms / steps,
        "value": upd / (ms / 1e3),
        "launch_shape": list(shape) if shape else "default",
    }


def max_size_leg(Q, W, steps: int = 50, oracle_steps: int = 10):
    """Branch count of the walk versus N and s on band matrices (uniform b,
    T~ start): the largest count at step boundaries over `steps` steps on the
    GPU, and for n <= 256 also the oracle's largest count after any single
    register-level operation (inside a step, as an op-by-op simulator holds
    the state), over `oracle_steps` steps."""
    import numpy as np

    import oracle

    cases = [(n, 1) for n in (64, 256, 1024, 4096, 16384)] + [(n, 3) for n in (64, 256, 1024, 4096, 16384)]
    cases += [(4096, w) for w in (7, 15, 31)]
    rows = []
    for n, w in cases:
        csc = W.band_matrix(n, w, seed=5)
        b = W.uniform_b(n)
        walk = Q.Walk(csc)
        st = walk.state(b)
        mmax = st.count()
        for _ in range(steps):
            st.step(1)
            mmax = max(mmax, st.count())
        N, s = walk.info[0]["N"], walk.info[0]["s"]
        row = {"n": n, "s": s, "m_max_boundary": mmax, "per_Ns": mmax / (N * s)}
        if n <= 256:
            ost = oracle.OracleState(oracle.OracleMatrix(csc)).set_b(b).T().step(oracle_steps)
            row["m_max_inside_step_oracle"] = ost.max_size()
        rows.append(row)
        st.close()
        walk.close()

    def slope(xs, ys):
        return float(np.polyfit(np.log(xs), np.log(ys), 1)[0])

    by_s = [r for r in rows if r["n"] == 4096]
    out = {"rows": rows,
           "loglog_slope_vs_s_at_n4096": slope([r["s"] for r in by_s], [r["m_max_boundary"] for r in by_s])}
    for s_ in (4, 8):
        by_n = [r for r in rows if r["s"] == s_]
        out[f"loglog_slope_vs_n_at_s{s_}"] = slope([r["n"] for r in by_n], [r["m_max_boundary"] for r in by_n])
    return out


def solver_leg(Q, W):
    """The walk-based CKS solve of the 32 x 32 five-point Laplacian + 0.1 I
    (kappa of A/s computed by the library, eps = 1e-3): walk steps, wall time
    of the whole solve on the library's stream, fidelity of the post-selected
    x against LU.  The library's kappa is timed on its own (host work, once
    per matrix)."""
    import numpy as np

    csc, b = W.solver_problem()
    walk = Q.Walk(csc)
    t0 = time.perf_counter()
    kappa = walk.kappa(0)
    t_kappa = time.perf_counter() - t0
    walk.qls(b, eps=1e-3)  # warm: kernels loaded, allocator primed
    t0 = time.perf_counter()
    x, p_succ, steps, _ = walk.qls(b, eps=1e-3)
    dt = time.perf_counter() - t0
    info = walk.info[0]
    H = csc.dense() * info["scale"] / info["s"]
    ref = np.linalg.solve(H, b)  # the fidelity's reference only
    fid = abs(np.vdot(ref, x)) ** 2 / (np.vdot(ref, ref).real * np.vdot(x, x).real)
    return {
        "workload": "5-point Laplacian 32x32 + 0.1 I, b = normalised Gaussian (seed 0), eps = 1e-3",
        "kappa": kappa,
        "kappa_ms": t_kappa * 1e3,
        "walk_steps": steps,
        "solve_ms": dt * 1e3,
        "us_per_walk_step": dt * 1e6 / steps,
        "fidelity_vs_lu": float(fid),
        "p_succ": p_succ,
    }


def adjoint_leg(Q, W, steps: int = 20, reps: int = 5):
    """Gradient of the total probability of 32 column outcomes after 20 steps
    w.r.t. all stored values and b (forward walk + reverse sweep with
    recomputation), against the forward walk alone: on G(1024, 8) (8192
    values) and on the benchmark's G(16384, 8) (131072 values), on the
    complex Hermitian offset matrices of the same sizes (the real and the
    imaginary part of every value), and on the band of the paper's shape E
    (s = 64)."""
    import numpy as np

    out = {}
    cases = []
    for n in (1024, 16384):
        a, b, w = W.adjoint_problem(n)
        cases.append((f"G({n}, 8)", f"G({n}, 8)", a, b, w))
    for n in (1024, 16384):
        _, b, w = W.adjoint_problem(n)
        cases.append((f"complex Hermitian {n}x8", f"complex Hermitian offset matrix n = {n}, 8 entries/column, seed 4",
                      W.hermitian_offset_matrix(n, 8, seed=4), b, w))
    e_csc, e_b = W.table1_band("E")
    _, _, e_w = W.adjoint_problem(e_csc.n)
    cases.append(("band E", "band matrix of the paper's shape E (16384 rows, bandwidth 31, s = 64)", e_csc, e_b, e_w))
    for label, what, a, b, w in cases:
        sc = 1.0 / np.abs(a.vals).max()
        a = W.Csc(a.n, a.colptr, a.rowidx, a.vals * sc)
        walk = Q.Walk(a, scale=1.0)

        def forward():
            st = walk.state(b).step(steps)
            st.sync()
            return st

        def gradient():
            st = walk.state(b).step(steps)
            st.grad(w, steps)

        forward(), gradient()
        t_fwd = sorted(_timed(Q, forward) for _ in range(reps))[reps // 2]
        t_grad = sorted(_timed(Q, gradient) for _ in range(reps))[reps // 2]
        st = walk.state(b)
        s0 = st.stats()
        st.step(steps)
        s1 = st.stats()
        upd = s1["total_written"] - s0["total_written"]
        out[label] = {
            "workload": f"{what}, uniform b, {steps} steps, loss over 32 outcomes, {a.nnz} values",
            "forward_ms": t_fwd,
            "forward_plus_gradient_ms": t_grad,
            "gradient_over_forward": t_grad / t_fwd,
            "forward_updates_per_s": upd / (t_fwd / 1e3),
            "forward_us_per_walk_step": 1e3 * t_fwd / steps,
            "reverse_us_per_walk_step": 1e3 * (t_grad - t_fwd) / steps,
            "reverse_over_forward_per_step": (t_grad - t_fwd) / t_fwd,
            "real_planes": bool(s1["real_amplitudes"]),
        }
    out["note"] = ("API calls end to end (state allocation, T~, copies and synchronisation included; "
                   "median of 5); reverse = (forward + gradient) - forward")
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=64)
    ap.add_argument("--cpu-steps", type=int, default=8, help="walk steps of the oracle sample (about 15 s)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the batched, adjoint, solver, complex, paper-shape and branch-count legs")
    ap.add_argument("--no-tune", action="store_true", help="keep the default launch shape")
    ap.add_argument("--launch", default=None, metavar="WG,GRID",
                    help="fixed launch shape of the main leg (workgroup size, workgroups)")
    ap.add_argument("--only", choices=["batched", "adjoint", "table1", "complex", "max_size", "solver"], default=None,
                    help="run one extra leg alone (for profiling) and print its JSON")
    ap.add_argument("--verbose", action="store_true", help="print every autotuner candidate as it is timed")
    ap.add_argument("--xcd", action="store_true",
                    help="--pmc-run: load with the XCD numbering of row blocks (QW_XCD_ROWS)")
    ap.add_argument("--lanes", default="0", choices=["0", "8", "16"],
                    help="lanes per row of s >= 16 slots for the counter run of --only table1 (0: the library's rule)")
    ap.add_argument("--pmc-run", action="store_true",
                    help="counter run: a torch copy of 64 MiB (byte calibration), then 64 walk steps of "
                         "the main workload (default launch shape unless --launch), of the batched leg "
                         "with --only batched, or of the paper's shape E with --only table1; prints "
                         "nothing else")
    args = ap.parse_args()
    global VERBOSE
    VERBOSE = args.verbose
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path "
              "(a single walk instance would shard by row owner with one all-to-all per step)",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2303_06890_amd as Q
    import workloads as W

    from paper_2303_06890_amd import autotune

    torch.cuda.set_device(0)
    if args.pmc_run:
        src = torch.ones(8 << 20, dtype=torch.float64, device="cuda")  # 64 MiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        if args.only == "batched":  # counters of the batched step kernel instead
            inst = W.batched_instances()
            st = Q.Walk([a for a, _ in inst], lanes=int(args.lanes), xcd=args.xcd).state([b for _, b in inst])
            if args.launch:
                st.set_launch(*(int(v) for v in args.launch.split(",")))
            st.step(64)
            st.sync()
            print(json.dumps({"pmc_run": True, "copy_bytes": 8 << 23, "batched_steps": 64, "xcd": args.xcd}),
                  flush=True)
            return
        if args.only == "table1":  # counters of the paper's shape E (16384 rows, s = 64)
            csc, b = W.table1_band("E")
            st = Q.Walk(csc, lanes=int(args.lanes), xcd=args.xcd).state(b)
            if args.launch:
                st.set_launch(*(int(v) for v in args.launch.split(",")))
            st.step(64)
            st.sync()
            print(json.dumps({"pmc_run": True, "copy_bytes": 8 << 23, "shape": "E", "steps": 64, "xcd": args.xcd}),
                  flush=True)
            return
        csc, b = W.paper_scale()
        st = Q.Walk(csc, xcd=args.xcd).state(b)
        if args.launch:
            st.set_launch(*(int(v) for v in args.launch.split(",")))
        st.step(64)
        st.sync()
        print(json.dumps({"pmc_run": True, "copy_bytes": 8 << 23, "steps": 64, "xcd": args.xcd}), flush=True)
        return
    if args.only == "batched":
        print(json.dumps(batched_leg(Q, W, autotune, not args.no_tune, cpu=not args.no_cpu_baseline)), flush=True)
        return
    if args.only == "adjoint":
        print(json.dumps(adjoint_leg(Q, W)), flush=True)
        return
    if args.only == "solver":
        print(json.dumps(solver_leg(Q, W)), flush=True)
        return
    if args.only == "max_size":
        print(json.dumps(max_size_leg(Q, W)), flush=True)
        return
    if args.only == "complex":
        print(json.dumps(complex_leg(Q, W, autotune, not args.no_tune)), flush=True)
        return
    if args.only == "table1":
        print(json.dumps(table1_leg(Q, W, autotune, not args.no_tune)), flush=True)
        return
    csc, b = W.paper_scale()
    tune_log = None
    if args.launch:
        walk, shape = Q.Walk(csc), tuple(int(v) for v in args.launch.split(","))
    elif args.no_tune:
        walk, shape = Q.Walk(csc), None
    else:
        walk, shape, tune_log = autotune.tune_walk(csc, b, verbose=VERBOSE)
    N, s = walk.info[0]["N"], walk.info[0]["s"]
    st = walk.state(b)
    if shape:
        autotune.apply(st, shape)
    st.step(args.warmup)
    # One more untimed call of exactly the timed count: it captures the step
    # graph that the timed calls replay (the library keeps a graph of exactly
    # the remainder of a call after its 256-step replays).
    st.step(args.steps)
    torch.cuda.synchronize()
    # Five timed loops of exactly K steps, each bracketed by synchronisation;
    # the value is their median.
    loops = []
    del HOST_MS[:]
    for _ in range(5):
        m_in0 = st.count()
        s0 = st.stats()
        ms = _timed(Q, lambda: st.step(args.steps))
        s1 = st.stats()
        out_total = s1["total_written"] - s0["total_written"]
        loops.append((ms, out_total, out_total - s1["branches"] + m_in0))
    ms, out_total, in_total = sorted(loops)[2]
    repeats = [1e3 * x[0] / args.steps for x in loops]
    alg_bytes = 24.0 * (in_total + out_total) + 12.0 * N * s * args.steps
    launch_s = ms / 1e3 / args.steps
    achieved = alg_bytes / args.steps / launch_s / 1e9
    traffic = measured_traffic(xcd=xcd_active(walk, shape))
    floors = launch_floors(torch)
    if args.steps != 256:
        # The same floors in graphs of the timed call's length: a short graph
        # costs more per launch, and the timed call is one such graph.
        floors.update({f"{k[:-3]}_{args.steps}_launch_graph_us": v
                       for k, v in launch_floors(torch, args.steps).items()})
    value = out_total / (ms / 1e3)
    line = {
        "metric": "walk-step amplitude updates/s (16384-dim, 8 nnz/col)",
        "value": value,
        "unit": "amplitude updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "graph_capture_steps": args.steps,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "walk steps on G(16384, 8): symmetric, 8 entries/column, seed 2, uniform b, T~ start",
            "N": N,
            "nnz_per_col": 8,
            "s": s,
            "branches": st.count(),
            "graph_steps_per_replay": "256, then one graph of the remaining count",
            "launch_shape": list(shape) if shape else "default",
            "autotune": tune_log,
            "timing": "median of 5 loops of exactly `steps` steps, HIP events on the kernels' stream",
            "host_ms_per_call": HOST_MS[:5],
            "spacer_gpu_ms": spacer_ms(torch, Q.stream()),
        },
        # The step kernel at this size is bound by latency, not by bandwidth:
        # the whole state sits in the 256 MB Infinity Cache and one launch
        # costs the launch floor plus the longest chain of dependent loads,
        # row sum and stores (`floors`: an empty kernel and a copy of the
        # step's bytes, each back to back in a 256-launch graph).  `frac` is
        # the algorithmic bytes of the 24 B/branch model over 8 TB/s;
        # `counter_frac` is the bytes the counters measure over 8 TB/s.
        "roofline": {
            "bound": "latency",
            "kernel": "step_kernel",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "counter_frac": traffic / launch_s / 1e9 / HBM_PEAK_GBS if traffic else None,
            "alg_bytes_per_launch": alg_bytes / args.steps,
            "avg_launch_us": launch_s * 1e6,
            "floors": floors,
            "note": ("frac prices every branch read and written at 24 bytes (key and complex amplitude); "
                     "this layout keeps one 8-byte double per branch with an implicit key, so frac can pass 1. "
                     "counter_frac uses the bytes the counters measure; the step is bound by latency "
                     "(floors: an empty kernel and a step-sized copy per launch in 256-launch graphs, "
                     "and in graphs of the timed step count)"),
        },
        "us_per_step_repeats": repeats,
    }
    print(f"[bench] {args.steps} steps in {ms:.3f} ms (median of 5; {launch_s * 1e6:.2f} us/step), "
          f"{value:.3e} updates/s, {achieved:.0f} GB/s algorithmic", file=sys.stderr, flush=True)
    line["host_inclusive"] = host_inclusive_leg(Q, csc, b, walk.lanes, shape, args.steps, out_total / args.steps)
    print(f"[bench] host inclusive: {line['host_inclusive']}", file=sys.stderr, flush=True)
    if not args.no_extras:
        line["batched"] = batched_leg(Q, W, autotune, not args.no_tune, cpu=not args.no_cpu_baseline)
        print(f"[bench] batched: {line['batched']}", file=sys.stderr, flush=True)
        line["adjoint"] = adjoint_leg(Q, W)
        print(f"[bench] adjoint: {line['adjoint']}", file=sys.stderr, flush=True)
        line["solver"] = solver_leg(Q, W)
        print(f"[bench] solver: {line['solver']}", file=sys.stderr, flush=True)
        line["complex"] = complex_leg(Q, W, autotune, not args.no_tune)
        print(f"[bench] complex: {line['complex']}", file=sys.stderr, flush=True)
        line["table1_shapes"] = table1_leg(Q, W, autotune, not args.no_tune)
        print(f"[bench] table1 shapes: {line['table1_shapes']}", file=sys.stderr, flush=True)
        line["max_size"] = max_size_leg(Q, W)
        print(f"[bench] max size: {line['max_size']}", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(csc, b, args.cpu_steps)
        print(f"[bench] oracle: {line['cpu_baseline']['value']:.3e} updates/s", file=sys.stderr, flush=True)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
