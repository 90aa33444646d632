"""Comparison of a GPU state with the oracle's: key sets equal (subject to the
oracle's margin list of amplitudes within 1e-15 of the pruning threshold) and
amplitudes within an absolute tolerance."""
import numpy as np

TAU = 1e-13
MARGIN = 1e-15


def compare_states(gk, ga, ok, oa, atol=1e-12, where=""):
    gk = np.asarray(gk, np.uint64)
    ok = np.asarray(ok, np.uint64)
    assert np.all(np.diff(gk.astype(np.float64)) >= 0) or np.all(gk[1:] > gk[:-1]), "GPU export not sorted"
    only_g = np.setdiff1d(gk, ok)
    only_o = np.setdiff1d(ok, gk)
    if only_g.size or only_o.size:
        # a mismatch is allowed only for keys whose amplitude sits within the
        # margin of the threshold on the side that has them
        amb_o = np.abs(np.maximum(np.abs(oa.real), np.abs(oa.imag)) - TAU) <= MARGIN
        amb_g = np.abs(np.maximum(np.abs(ga.real), np.abs(ga.imag)) - TAU) <= MARGIN
        bad_o = np.setdiff1d(only_o, ok[amb_o])
        bad_g = np.setdiff1d(only_g, gk[amb_g])
        assert bad_o.size == 0 and bad_g.size == 0, (
            f"{where}: key sets differ: {only_o.size} only in oracle, {only_g.size} only on GPU")
    common, gi, oi = np.intersect1d(gk, ok, return_indices=True)
    err = np.abs(ga[gi] - oa[oi]).max() if common.size else 0.0
    assert err <= atol, f"{where}: max amplitude error {err:.3e} > {atol:.1e}"
    return err
