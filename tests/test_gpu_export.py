"""The export's key order (the GPU radix sort behind qw_export).

The walk tests compare exported states with the oracle key for key; these
cases aim at the sort itself: branches of the general list imported in a
shuffled order, states of zero and one branch, and a full-size state whose
58-bit keys take several digit passes, checked against a measurement that
does not go through the export.
"""
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


def test_shuffled_list_branches_come_out_sorted(Q):
    """Branches outside the static homes (j_c != 0) sit in the list in the
    order they were imported; the export returns every branch in key order
    with its own amplitude."""
    csc = W.offset_matrix(64, 6, seed=31)
    walk = Q.Walk(csc)
    st = walk.state(W.gaussian_b(64, seed=32)).step(3)
    keys, amps = st.export()
    assert np.all(np.diff(keys.astype(np.uint64)) > 0)
    nb, s = walk.nbits, walk.info[0]["s"]
    rng = np.random.default_rng(41)
    extra = np.unique(np.array([Q.pack_key(nb, int(rng.integers(1, s)), int(rng.integers(64)), int(rng.integers(2)),
                                           int(rng.integers(s)), int(rng.integers(64)), int(rng.integers(2)))
                                for _ in range(3000)], np.uint64))
    ea = rng.normal(size=extra.size) + 1j * rng.normal(size=extra.size)
    allk = np.concatenate([keys, extra])
    alla = np.concatenate([amps, ea])
    perm = rng.permutation(allk.size)
    imp = walk.state(np.zeros(64), capacity=2 * extra.size).import_(allk[perm], alla[perm])
    assert imp.stats()["list_count"] == extra.size
    gk, ga = imp.export()
    order = np.argsort(allk)
    np.testing.assert_array_equal(gk, allk[order])
    np.testing.assert_allclose(ga, alla[order], rtol=1e-15, atol=0)


def test_zero_and_one_branch(Q):
    csc = W.offset_matrix(64, 6, seed=31)
    walk = Q.Walk(csc)
    empty = walk.state(np.zeros(64))
    k, a = empty.export()
    assert k.size == 0 and a.size == 0
    key = np.array([Q.pack_key(walk.nbits, 1, 5, 0, 2, 7, 1)], np.uint64)
    one = walk.state(np.zeros(64), capacity=4).import_(key, np.array([0.25 - 0.5j]))
    k, a = one.export()
    np.testing.assert_array_equal(k, key)
    assert a[0] == 0.25 - 0.5j


def test_full_size_export_pairs_keys_and_amplitudes(Q):
    """G(16384, 8) after 3 steps (393 214 branches, keys of 58 bits): keys
    strictly increasing, and the j-register marginal rebuilt from the
    exported (key, amplitude) pairs equals the one the measurement kernel
    computes from the planes."""
    csc, b = W.paper_scale()
    walk = Q.Walk(csc)
    st = walk.state(b).step(3)
    keys, amps = st.export()
    assert keys.size == st.count() == 393214
    assert np.all(np.diff(keys) > 0)
    n = walk.nbits
    j = ((keys >> np.uint64(2 * n + 2)) & np.uint64((1 << n) - 1)).astype(np.int64)
    rebuilt = np.bincount(j, weights=np.abs(amps) ** 2, minlength=walk.N_total)
    np.testing.assert_allclose(rebuilt, st.j_marginal(), rtol=1e-12, atol=1e-18)


def test_split_and_interleaved_exports_agree(Q):
    """qw_export (re and im arrays) and qw_export_complex (interleaved) return
    the same keys and the same amplitudes, bit for bit."""
    import ctypes

    from paper_2303_06890_amd import _lib

    csc = W.offset_matrix(1024, 8, seed=5)
    st = Q.Walk(csc).state(W.gaussian_b(1024, seed=6)).step(7)
    m = st.count()
    lib = _lib.load()
    dp = ctypes.POINTER(ctypes.c_double)
    up = ctypes.POINTER(ctypes.c_uint64)
    k1, re, im = np.zeros(m, np.uint64), np.zeros(m), np.zeros(m)
    k2, amps = np.zeros(m, np.uint64), np.zeros(m, np.complex128)
    got1, got2 = ctypes.c_int64(), ctypes.c_int64()
    _lib.check(lib.qw_export(st._h, k1.ctypes.data_as(up), re.ctypes.data_as(dp), im.ctypes.data_as(dp), m,
                             ctypes.byref(got1), Q._stream()))
    _lib.check(lib.qw_export_complex(st._h, k2.ctypes.data_as(up), amps.ctypes.data_as(dp), m, ctypes.byref(got2),
                                     Q._stream()))
    assert got1.value == got2.value == m
    np.testing.assert_array_equal(k1, k2)
    np.testing.assert_array_equal(re, amps.real)
    np.testing.assert_array_equal(im, amps.imag)
    k3, a3 = st.export()
    np.testing.assert_array_equal(k3, k1)
    np.testing.assert_array_equal(a3, amps)


def test_split_and_interleaved_imports_agree(Q):
    """qw_state_import (re and im arrays) and qw_state_import_complex
    (interleaved) build the same state: equal keys summed, branches at or
    below 1e-13 in both parts dropped, the rest placed by key."""
    import ctypes

    from paper_2303_06890_amd import _lib

    csc = W.offset_matrix(64, 6, seed=31)
    walk = Q.Walk(csc)
    keys, amps = walk.state(W.gaussian_b(64, seed=32)).step(4).export()
    rng = np.random.default_rng(7)
    dup = rng.choice(keys.size, 50, replace=False)
    tiny = rng.choice(keys.size, 20, replace=False)
    k = np.concatenate([keys, keys[dup], keys[tiny]])
    a = np.concatenate([amps, 0.5 * amps[dup], -amps[tiny] + 1e-14])  # the tiny ones cancel to 1e-14
    perm = rng.permutation(k.size)
    k, a = np.ascontiguousarray(k[perm]), np.ascontiguousarray(a[perm])
    lib = _lib.load()
    dp = ctypes.POINTER(ctypes.c_double)
    up = ctypes.POINTER(ctypes.c_uint64)
    s1 = walk.state(np.zeros(64))
    re, im = np.ascontiguousarray(a.real), np.ascontiguousarray(a.imag)
    _lib.check(lib.qw_state_import(s1._h, k.ctypes.data_as(up), re.ctypes.data_as(dp), im.ctypes.data_as(dp), k.size,
                                   Q._stream()))
    s2 = walk.state(np.zeros(64))
    _lib.check(lib.qw_state_import_complex(s2._h, k.ctypes.data_as(up), a.view(np.float64).ctypes.data_as(dp), k.size,
                                           Q._stream()))
    k1, a1 = s1.export()
    k2, a2 = s2.export()
    np.testing.assert_array_equal(k1, k2)
    np.testing.assert_array_equal(a1, a2)
    # what the import should hold: sums per key, then the pruning rule
    expect = {}
    for kk, aa in zip(k, a):
        expect[int(kk)] = expect.get(int(kk), 0) + aa
    kept = sorted(kk for kk, aa in expect.items() if abs(aa.real) > 1e-13 or abs(aa.imag) > 1e-13)
    np.testing.assert_array_equal(k1, np.array(kept, np.uint64))
    np.testing.assert_allclose(a1, np.array([expect[kk] for kk in kept]), rtol=1e-15, atol=1e-17)
