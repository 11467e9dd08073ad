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
    b, keep = _batch([100, 10, 300], [10, 20, 30])
    for bad in (-1, 5):
        o = L.default_options()
        o.batch_stages = bad
        st = L.sweep_eval_batched(b, o, 0x100000, 0, 0x100000, 1 << 40, 0)
        assert L.STATUS[st] == "SWEEP_ERR_BAD_OPTION" and "batch_stages" in L.last_error()
        assert L.sweep_batched_workspace_size(b, o) == 0


def test_batched_validation_names_the_sweep_and_curve():
    # the message carries the failing sweep's index and which curve failed,
    # also for a sweep after valid ones, and the details of the curve check
    b, keep = _batch([100, 10, 300], [10, 20, 30])
    keep["qd"][2] = 0
    st = L.sweep_eval_batched(b, L.default_options(), 0x100000, 0, 0x100000, 1 << 40, 0)
    msg = L.last_error()
    assert L.STATUS[st] == "SWEEP_ERR_BAD_DEGREE" and msg.startswith("sweep 2 profile") and "degree 0" in msg
    keep["qd"][2] = 3
    keep["pn"][1] = 2
    st = L.sweep_eval_batched(b, L.default_options(), 0x100000, 0, 0x100000, 1 << 40, 0)
    msg = L.last_error()
    assert L.STATUS[st] == "SWEEP_ERR_BAD_COUNT" and msg.startswith("sweep 1 path") and "2 control points" in msg


def test_batched_output_elems_padded_layout():
    # plane stride = n_u*n_v rounded up to 64 elements
    b, keep = _batch([100, 7, 64], [10, 9, 3])
    assert L.sweep_batched_output_elems(b) == 3 * (1024 + 64 + 192)
    b, keep = _batch([64, 64], [64, 1], n=2)
    assert L.sweep_batched_output_elems(b) == 3 * (4096 + 64)
    b.n_sweeps = 0
    assert L.sweep_batched_output_elems(b) == 0


def test_python_batch_layout_matches_abi():
    import torch
    import synth
    from paper_1110_5450_amd import api
    specs = synth.c4(n_sweeps=40, seed=3)
    b = api.Batch.from_specs(specs, device="cpu")
    assert b.out_elems == L.sweep_batched_output_elems(b.c_struct())
    assert np.all(b.plane % 64 == 0) and np.all(b.plane - b.n_u * b.n_v < 64)
    assert np.all(np.diff(b.offsets) == 3 * b.plane[:-1])
    flat = torch.arange(b.out_elems, dtype=torch.float64)
    for k in (0, 17, 39):
        v = b.view(flat, k)
        assert v.shape == (3, specs[k].n_u, specs[k].n_v)
        assert float(v[1, 0, 0]) == b.offsets[k] + b.plane[k]
        assert float(v[2, -1, -1]) == b.offsets[k] + 2 * b.plane[k] + specs[k].n_u * specs[k].n_v - 1
    blocks = [np.full((3, s.n_u, s.n_v), k + 1.0) for k, s in enumerate(specs)]
    packed = b.pack(blocks, torch.float64)
    assert float(packed.sum()) == sum((k + 1.0) * 3 * s.n_u * s.n_v for k, s in enumerate(specs))
