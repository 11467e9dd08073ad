"""Batched ABI on the host: workspace sizes and validation without a GPU."""

import ctypes as C

import numpy as np

from paper_1110_5450_amd import _lib as L


def _batch(n_u, n_v, n=3, p=3, q=3):
    arr = lambda v: np.ascontiguousarray(np.array(v, np.int32))
    keep = dict(pn=arr([10] * n), pd=arr([p] * n), qn=arr([8] * n), qd=arr([q] * n), nu=arr(n_u), nv=arr(n_v))
    ip = lambda a: a.ctypes.data_as(C.POINTER(C.c_int32))
    b = L.SweepBatch(n, 0, ip(keep["pn"]), ip(keep["pd"]), ip(keep["qn"]), ip(keep["qd"]), None,
                     ip(keep["nu"]), ip(keep["nv"]), None, None, 0x100000, 0x100000)
    return b, keep


def test_batched_workspace_size():
    b, keep = _batch([100, 200, 300], [10, 20, 30])
    o = L.default_options()
    s = L.sweep_batched_workspace_size(b, o)
    b2, keep2 = _batch([100, 200, 3000], [10, 20, 30])
    assert 0 < s < L.sweep_batched_workspace_size(b2, o)


def test_batched_validation():
    b, keep = _batch([100, 1, 300], [10, 20, 30])
    st = L.sweep_eval_batched(b, L.default_options(), 0x100000, 0, 0x100000, 1 << 40, 0)
    assert L.STATUS[st] == "SWEEP_ERR_BAD_GRID" and "sweep 1" in L.last_error()
    b, keep = _batch([100, 10, 300], [10, 20, 30], p=9)
    st = L.sweep_eval_batched(b, L.default_options(), 0x100000, 0, 0x100000, 1 << 40, 0)
    assert L.STATUS[st] == "SWEEP_ERR_BAD_DEGREE" and "sweep 0 path" in L.last_error()
    b, keep = _batch([100, 10, 300], [10, 20, 30])
    need = L.sweep_batched_workspace_size(b, L.default_options())
    st = L.sweep_eval_batched(b, L.default_options(), 0x100000, 0, 0x100000, need - 1, 0)
    assert L.STATUS[st] == "SWEEP_ERR_WORKSPACE"
    b.n_sweeps = 0
    st = L.sweep_eval_batched(b, L.default_options(), 0x100000, 0, 0x100000, 1 << 40, 0)
    assert L.STATUS[st] == "SWEEP_ERR_BAD_COUNT"
