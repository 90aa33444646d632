"""Autotuner of the step kernel's tile and launch shape.

Two choices change how fast a walk step runs and never what it computes:

* the tile: how many lanes of a wavefront share a row of the QRAM table
  (8, or 16 for rows of s >= 16 slots: the QW_LANES_8 / QW_LANES_16 load
  flags), which fixes the slots each lane holds (s / lanes) and the
  wavefronts of a pass.  It is a property of the loaded matrix, so each
  choice is a separate load.  (Four lanes per row, two to sixteen slots per
  lane, measured slower than eight for every workload here: G(16384, 8),
  the 256-instance batch and the paper's band shapes.)  The tile also says
  whether the one-pass kernels number their row blocks by XCD (QW_XCD_ROWS:
  neighbouring rows, which share cache lines, then run on one XCD's L2);
  which is faster depends on the matrix.
* the launch shape: workgroup size and number of workgroups.

`tune_walk` loads the matrices once per tile choice that applies, times the
launch-shape candidates of each on a scratch state (HIP events on the
library's stream, graph-replayed steps), re-times the best shape of each tile
(median of three loops) to choose between tiles, and returns the fastest
walk, its launch shape and the log of every candidate.  `tune` tunes the launch shape
of a walk already loaded.  Results are remembered under (device, padded
dimensions, largest s, instance count, branch-count bucket, value kind,
tile), in memory and optionally in a JSON file.
"""
from __future__ import annotations

import json
import math
import os
import sys

_cache: dict = {}

TIMED_STEPS = 64  # more than a call replays as single launches: the graph path


def _key(walk, branches: int) -> str:
    import torch

    name = torch.cuda.get_device_name()
    smax = max(d["s"] for d in walk.info)
    bucket = int(math.log2(max(1, branches)))
    # the value kind selects the kernel family
    kind = "complex" if walk.complex else (f"word{walk.word}" if walk.word else "real")
    return (f"{name}|N={walk.N_total}|s={smax}|inst={walk.ninst}|m2^{bucket}|{kind}|lanes={walk.lanes}"
            f"|xcd={int(walk.xcd)}")


def lanes_per_row(walk, s: int) -> int:
    """The lanes that share a row of s slots in the library's lane mapping:
    min(s, 8), or 16 for s >= 16 when the walk was loaded with lanes=16, or
    by the library's rule (lanes=0: 16 when the context has at most 1024
    wavefronts with 8)."""
    if s < 16:
        return min(s, 8)
    if walk.lanes:
        return walk.lanes
    waves8 = sum(-(-d["N"] // (64 // min(d["s"], 8))) for d in walk.info)
    return 16 if 2 * waves8 <= 2048 else 8


def _waves(walk) -> int:
    """Wavefronts of one step-kernel pass under the walk's lane mapping."""
    return sum(-(-d["N"] // (64 // lanes_per_row(walk, d["s"]))) for d in walk.info)


def candidates(walk):
    """(workgroup size, workgroups) to time: the one-pass grid and a few
    grid-stride ones.  A walk loaded with the XCD numbering of row blocks also
    gets the one-pass grid rounded up to a multiple of 8 (the numbering needs
    one; the workgroups past the rows return at once)."""
    waves = _waves(walk)
    lanes = 64 * waves
    out = []
    for wg in (64, 128, 256):
        one_pass = max(1, -(-lanes // wg))
        grids = {min(one_pass, 65536), 1024, 2048, 4096, 8192}
        if walk.xcd and -(-one_pass // 8) * 8 <= 65536:
            grids.add(-(-one_pass // 8) * 8)
        for grid in sorted(grids):
            if grid <= one_pass or grid == -(-one_pass // 8) * 8:
                out.append((wg, grid))
    return out


def _time_shapes(walk, b, warm: int = 16, steps: int = TIMED_STEPS, verbose: bool = False):
    """[(us per step, (wg, grid))] for every candidate launch shape, and the
    branch count of the scratch state."""
    import torch

    from . import stream

    st = walk.state(b).step(warm)
    branches = st.count()
    out = []
    for wg, grid in candidates(walk):
        st.set_launch(wg, grid)
        st.step(steps)  # captures the graph for this shape
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream())
        st.step(steps)
        e1.record(stream())
        e1.synchronize()
        t = e0.elapsed_time(e1) * 1e3 / steps
        if verbose:
            print(f"[autotune] lanes={walk.lanes} xcd={int(walk.xcd)} wg={wg:4d} grid={grid:5d}: {t:8.3f} us/step",
                  file=sys.stderr, flush=True)
        out.append((t, (wg, grid)))
    st.close()
    return out, branches


def _load_cache(cache_path):
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as f:
            _cache.update(json.load(f))


def _save_cache(cache_path):
    if cache_path:
        with open(cache_path, "w") as f:
            json.dump(_cache, f, indent=1)


def tune(walk, b, cache_path: str | None = None, verbose: bool = False):
    """Return the fastest (wg_size, grid) for stepping `walk` from T~|b~>."""
    _load_cache(cache_path)
    st = walk.state(b).step(16)
    key = _key(walk, st.count())
    st.close()
    if key not in _cache:
        times, _ = _time_shapes(walk, b, verbose=verbose)
        _cache[key] = [list(min(times)[1]), min(times)[0]]
        _save_cache(cache_path)
    return tuple(_cache[key][0])


def _smax(mats) -> int:
    """Largest QRAM row length s over the matrices (the power of two at or
    above the largest column count)."""
    import numpy as np

    mats = list(mats) if isinstance(mats, (list, tuple)) else [mats]
    return max(1 << int(math.ceil(math.log2(max(1, int(np.diff(np.asarray(m.colptr)).max()))))) for m in mats)


def _retime(walk, b, shape, reps: int = 3, warm: int = 16, steps: int = TIMED_STEPS) -> float:
    """Median over `reps` graph-replayed loops of the time per step at one
    launch shape (us)."""
    import torch

    from . import stream

    st = walk.state(b).step(warm)
    st.set_launch(*shape)
    st.step(steps)
    ts = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream())
        st.step(steps)
        e1.record(stream())
        e1.synchronize()
        ts.append(e0.elapsed_time(e1) * 1e3 / steps)
    st.close()
    return sorted(ts)[reps // 2]


def tune_walk(mats, b, verbose: bool = False, **walk_kwargs):
    """Load `mats` with each tile choice that applies (8 and 16 lanes per row
    when some row has s >= 16 slots, else the one mapping there is; for real
    values each with and without the XCD numbering of row blocks), tune the
    launch shape of each, and return (walk, (wg, grid), log): the fastest
    walk (the others are released), its launch shape, and a log of every
    candidate timed, for the record of the run."""
    import numpy as np

    from . import Walk

    lanes_choices = [8, 16] if _smax(mats) >= 16 else [0]
    # the numbering by XCD exists for the one-double-per-cell kernels (real
    # values); complex values would time the same kernels twice
    mlist = list(mats) if isinstance(mats, (list, tuple)) else [mats]
    xcd_choices = (False,) if any(np.iscomplexobj(m.vals) for m in mlist) else (False, True)
    log = {"tile_choices": [], "launch_candidates": []}
    best = None
    for lanes in lanes_choices:
        for xcd in xcd_choices:
            walk = Walk(mats, lanes=lanes, xcd=xcd, **walk_kwargs)
            times, _ = _time_shapes(walk, b, verbose=verbose)
            shape = min(times)[1]
            t = _retime(walk, b, shape)
            lpr = sorted({lanes_per_row(walk, d["s"]) for d in walk.info})
            log["tile_choices"].append({"lanes_per_row": lpr, "xcd_rows": xcd, "wavefronts": _waves(walk),
                                        "best_us_per_step": t, "best_launch": list(shape)})
            log["launch_candidates"] += [{"lanes_per_row": lpr, "xcd_rows": xcd, "wg": s[0], "grid": s[1],
                                          "us_per_step": u} for u, s in times]
            if best is None or t < best[0]:
                if best is not None:
                    best[1].close()
                best = (t, walk, shape, lpr, xcd)
            else:
                walk.close()
    t, walk, shape, lpr, xcd = best
    log.update(chosen_lanes_per_row=lpr, chosen_xcd_rows=xcd, chosen_launch=list(shape), chosen_us_per_step=t)
    return walk, shape, log


def apply(state, shape) -> None:
    state.set_launch(int(shape[0]), int(shape[1]))


__all__ = ["tune", "tune_walk", "apply", "candidates", "lanes_per_row"]
