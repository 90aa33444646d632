"""The autotuner's host logic on the CPU: lane mapping, wavefront counts and
launch-shape candidates (no GPU: a stand-in for the loaded walk)."""
from types import SimpleNamespace

from paper_2303_06890_amd import autotune


def _walk(rows, lanes=0, xcd=False):
    return SimpleNamespace(info=[{"N": n, "s": s} for n, s in rows], lanes=lanes, xcd=xcd)


def test_lanes_per_row_rule():
    w = _walk([(16384, 8)])
    assert autotune.lanes_per_row(w, 8) == 8 and autotune.lanes_per_row(w, 4) == 4
    assert autotune.lanes_per_row(_walk([(16384, 64)], lanes=16), 64) == 16
    assert autotune.lanes_per_row(_walk([(16384, 64)]), 64) == 8  # 2048 wavefronts with eight: stays eight
    assert autotune.lanes_per_row(_walk([(1024, 32)]), 32) == 16  # small contexts take sixteen


def test_wavefronts_of_a_pass():
    assert autotune._waves(_walk([(16384, 8)])) == 2048  # eight rows per wavefront
    assert autotune._waves(_walk([(8192, 32)], lanes=16)) == 2048  # four rows per wavefront
    assert autotune._waves(_walk([(64, 4), (128, 8)])) == 4 + 16  # sixteen rows of s = 4, eight of s = 8


def test_candidates_cover_one_pass_and_round_up_for_the_xcd_numbering():
    plain = autotune.candidates(_walk([(1000, 8)]))
    xcd = autotune.candidates(_walk([(1000, 8)], xcd=True))
    # 125 wavefronts: one-pass grids 125, 63, 32 workgroups at 64, 128, 256 threads
    assert (64, 125) in plain and (128, 63) in plain and (256, 32) in plain
    assert all(g <= -(-125 // (wg // 64)) for wg, g in plain)
    # the XCD-numbered walk also gets those grids rounded up to a multiple of 8
    assert (64, 128) in xcd and (128, 64) in xcd and (256, 32) in xcd
    assert set(plain) <= set(xcd)
    assert not [c for c in plain if c not in xcd]
