"""The C ABI on its own: one matrix through qw_load_csc (library allocation,
the null stream, no Python classes), stepped, measured and exported, against
the oracle; then fixed-point data through QW_WORD_LENGTH the same way."""
import ctypes

import numpy as np
import pytest

import workloads as W
from tests.parity import compare_states

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch

    assert torch.cuda.is_available()
    from paper_2303_06890_amd import _lib

    return _lib.load()


def _run(lib, csc, b, nsteps, flags):
    ip, dp = ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double)
    cp = np.ascontiguousarray(csc.colptr, np.int32)
    ri = np.ascontiguousarray(csc.rowidx, np.int32)
    va = np.ascontiguousarray(csc.vals, np.float64)
    br = np.ascontiguousarray(b, np.float64)
    ctx, st = ctypes.c_void_p(), ctypes.c_void_p()
    rc = lib.qw_load_csc(ctypes.byref(ctx), csc.n, cp.ctypes.data_as(ip), ri.ctypes.data_as(ip),
                         va.ctypes.data_as(dp), csc.nnz, 0.0, flags, None, None)
    assert rc == 0, lib.qw_last_error().decode()
    try:
        rc = lib.qw_state_init(ctypes.byref(st), ctx, br.ctypes.data_as(dp), None, 0, 0, None)
        assert rc == 0, lib.qw_last_error().decode()
        assert lib.qw_step(st, nsteps, None) == 0, lib.qw_last_error().decode()
        count = np.zeros(1, np.int64)
        assert lib.qw_measure(st, 1, count.ctypes.data_as(ctypes.c_void_p), 1, None) == 0
        cap = int(count[0])
        keys = np.zeros(cap, np.uint64)
        re, im = np.zeros(cap), np.zeros(cap)
        m = ctypes.c_int64()
        rc = lib.qw_export(st, keys.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), re.ctypes.data_as(dp),
                           im.ctypes.data_as(dp), cap, ctypes.byref(m), None)
        assert rc == 0 and m.value == cap, lib.qw_last_error().decode()
        return keys, re + 1j * im
    finally:
        lib.qw_state_free(st)
        lib.qw_ctx_free(ctx)


def test_c_abi_end_to_end(lib, oracle_mod):
    csc = W.offset_matrix(300, 6, seed=61)
    b = W.gaussian_b(300, seed=62)
    gk, ga = _run(lib, csc, b, 40, 1)
    ok, oa = oracle_mod.OracleState(oracle_mod.OracleMatrix(csc)).set_b(b).T().step(40).export()
    compare_states(gk, ga, ok, oa, where="C ABI, 40 steps")


def test_c_abi_fixed_point(lib, oracle_mod):
    from paper_2303_06890_amd import _lib

    csc = W.fixed_point_band(200, 4, 12, seed=63, negative=0.3)
    b = W.gaussian_b(200, seed=64)
    gk, ga = _run(lib, csc, b, 30, 1 | _lib.word_length(12))
    ok, oa = oracle_mod.OracleState(oracle_mod.OracleMatrix(csc, word=12)).set_b(b).T().step(30).export()
    compare_states(gk, ga, ok, oa, where="C ABI, fixed point, 30 steps")
