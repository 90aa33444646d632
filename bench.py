#!/usr/bin/env python3
"""Walk-step throughput on one MI355X.

Workload: the 16384-dimensional real symmetric matrix with 8 stored entries
per column (diagonal + 3 mirrored seeded random cyclic offsets + offset N/2,
values U[-1,1], diagonal shifted by +7, seed 2), rescaled by its largest
entry; start T~|b~> with b the uniform superposition over all 16384 columns;
FP64 complex amplitudes.  One benchmark step is one walk step W (one launch of
the fused step kernel) on that state; the state reaches its steady size of
3Ns - 2 = 393214 branches after the second step, so warm-up steps put the
timed region in the steady state.

Output: one JSON line on stdout with the metric (amplitude updates/s = sum
over timed steps of the branches each step writes, divided by the time of the
step loop), the roofline of the step kernel (algorithmic bytes per launch =
24 B x (branches in + branches out) + 12 B x ELL slots, divided by the
average launch time measured with HIP events on the kernels' stream, against
8 TB/s), and the oracle's rate on the host CPU for a bounded sample.
"""
import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


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
    written = 0
    t0 = time.perf_counter()
    for _ in range(steps):
        ost.step(1)
        written += ost.count()
    dt = time.perf_counter() - t0
    return {
        "value": written / dt,
        "unit": "amplitude updates/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"T~|b~> then {steps} walk steps of the same 16384-dim workload "
                  f"({written} branch updates in {dt:.1f} s), one thread on {cpu_model()} "
                  f"(nproc={os.cpu_count()})",
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=64)
    ap.add_argument("--cpu-steps", type=int, default=5, help="walk steps of the oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path "
              "(a single walk instance would shard by row owner with one all-to-all per step)",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2303_06890_amd as Q
    import workloads as W

    torch.cuda.set_device(0)
    csc, b = W.paper_scale()
    walk = Q.Walk(csc)
    N, s = walk.info[0]["N"], walk.info[0]["s"]
    st = walk.state(b)
    st.step(args.warmup)
    torch.cuda.synchronize()
    m_in0 = st.count()
    s0 = st.stats()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(Q.stream())  # the stream the step kernels are launched on
    st.step(args.steps)
    ev1.record(Q.stream())
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    s1 = st.stats()
    out_total = s1["total_written"] - s0["total_written"]
    in_total = out_total - s1["branches"] + m_in0
    alg_bytes = 24.0 * (in_total + out_total) + 12.0 * N * s * args.steps
    launch_s = ms / 1e3 / args.steps
    achieved = alg_bytes / args.steps / launch_s / 1e9
    value = out_total / (ms / 1e3)
    line = {
        "metric": "walk-step amplitude updates/s (16384-dim, 8 nnz/col)",
        "value": value,
        "unit": "amplitude updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
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
            "branches": s1["branches"],
            "graph_steps_per_replay": 16,
        },
        "roofline": {
            "bound": "hbm",
            "kernel": "step_kernel",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": None,
            "alg_bytes_per_launch": alg_bytes / args.steps,
            "avg_launch_us": launch_s * 1e6,
        },
    }
    print(f"[bench] {args.steps} steps in {ms:.2f} ms ({launch_s * 1e6:.2f} us/step), "
          f"{value:.3e} updates/s, {achieved:.0f} GB/s algorithmic", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(csc, b, args.cpu_steps)
        print(f"[bench] oracle: {line['cpu_baseline']['value']:.3e} updates/s", file=sys.stderr, flush=True)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
