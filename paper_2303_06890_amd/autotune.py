"""Launch-shape autotuner of the step kernel.

The step kernel strides over wavefronts (each covers 64 / min(s, 8) rows,
min(s, 8) lanes per row; 16 lanes for s >= 16 in small contexts), so its
launch shape is free: workgroup size and number of workgroups.  `tune` times candidate shapes on a scratch state
of the given workload (HIP events on the library's stream), keeps the fastest,
and remembers it under (device name, padded dimensions, largest s, instance
count, branch-count bucket), in memory and optionally in a JSON file.
"""
from __future__ import annotations

import json
import math
import os

_cache: dict = {}


def _key(walk, branches: int) -> str:
    import torch

    name = torch.cuda.get_device_name()
    smax = max(d["s"] for d in walk.info)
    bucket = int(math.log2(max(1, branches)))
    # the value kind selects the kernel family
    kind = "complex" if walk.complex else (f"word{walk.word}" if walk.word else "real")
    return f"{name}|N={walk.N_total}|s={smax}|inst={walk.ninst}|m2^{bucket}|{kind}"


def _waves(walk) -> int:
    """Wavefronts of one step-kernel pass, by the library's lane mapping:
    min(s, 8) lanes per row, or 16 for s >= 16 when that keeps the context
    at 2048 wavefronts or fewer."""
    def count(lanes_of):
        return sum(-(-d["N"] // (64 // lanes_of(d["s"]))) for d in walk.info)

    waves8 = count(lambda s: min(s, 8))
    if 2 * waves8 <= 2048:
        return count(lambda s: 16 if s >= 16 else min(s, 8))
    return waves8


def candidates(walk):
    waves = _waves(walk)
    lanes = 64 * waves
    out = []
    for wg in (64, 128, 256):
        one_pass = max(1, -(-lanes // wg))
        for grid in sorted({min(one_pass, 65536), 1024, 2048, 4096, 8192}):
            if grid <= one_pass:
                out.append((wg, grid))
    return out


def tune(walk, b, steps: int = 32, warm: int = 16, cache_path: str | None = None, verbose: bool = False):
    """Return the fastest (wg_size, grid) for stepping `walk` from T~|b~>."""
    import torch

    from . import stream

    st = walk.state(b).step(warm)
    key = _key(walk, st.count())
    if key not in _cache and cache_path and os.path.exists(cache_path):
        with open(cache_path) as f:
            _cache.update(json.load(f))
    if key in _cache:
        st.close()
        return tuple(_cache[key])
    best, best_t = None, math.inf
    for wg, grid in candidates(walk):
        st.set_launch(wg, grid)
        st.step(steps)  # warm the captured graph for this shape
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream())
        st.step(steps)
        e1.record(stream())
        e1.synchronize()
        t = e0.elapsed_time(e1) / steps
        if verbose:
            print(f"[autotune] wg={wg:4d} grid={grid:5d}: {t * 1e3:8.2f} us/step")
        if t < best_t:
            best, best_t = (wg, grid), t
    st.close()
    _cache[key] = list(best)
    if cache_path:
        with open(cache_path, "w") as f:
            json.dump(_cache, f, indent=1)
    return best


def apply(state, shape) -> None:
    state.set_launch(int(shape[0]), int(shape[1]))


__all__ = ["tune", "apply", "candidates"]
