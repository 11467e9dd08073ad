"""The C ABI without a GPU: the library loads, exports every entry point the
header declares, reports defaults and workspace sizes, and rejects invalid
metadata with the documented status before anything is launched."""

import ctypes as C
import math
import os
import re

import numpy as np
import pytest

from paper_1110_5450_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FAKE = 0x100000  # never dereferenced: every call below fails validation first


def _header_functions():
    text = open(os.path.join(ROOT, "include", "sweep.h")).read()
    return sorted(set(re.findall(r"^[A-Za-z_][\w\s\*]*?\b(sweep_\w+)\s*\(", text, flags=re.M)))


def test_exports_every_declared_symbol():
    names = _header_functions()
    assert len(names) >= 11
    lib = L.lib()
    for n in names:
        assert hasattr(lib, n), n


def test_version_and_defaults():
    assert L.sweep_version() == 105
    o = L.default_options()
    assert (o.out_precision, o.frame_precision, o.reorthonormalize, o.has_initial_normal, o.tile_config) == (0, 1, 1, 0, -1)
    assert L.sweep_tile_config_count() >= 8


def _curves(n=16, p=3, m=8, q=3, closed=1, pk=None, qk=None):
    pkp = None if pk is None else pk.ctypes.data_as(C.POINTER(C.c_double))
    qkp = None if qk is None else qk.ctypes.data_as(C.POINTER(C.c_double))
    return L.SweepCurve(n, p, 0, 0, FAKE, pkp), L.SweepCurve(m, q, closed, 0, FAKE, qkp)


def test_workspace_size_valid_and_monotone():
    o = L.default_options()
    a, b = _curves()
    s1 = L.sweep_eval_workspace_size(a, b, 256, 64, o)
    s2 = L.sweep_eval_workspace_size(a, b, 4096, 64, o)
    s3 = L.sweep_eval_workspace_size(a, b, 4096, 1024, o)
    assert 0 < s1 < s2 < s3 and s1 % 256 == 0
    o.out_precision = 1
    assert L.sweep_eval_workspace_size(a, b, 4096, 1024, o) > s3
    assert L.sweep_eval_workspace_size(a, b, 1, 64, o) == 0


def _call(path, prof, n_u=256, n_v=64, opt=None, pos=FAKE, ws=FAKE, ws_bytes=1 << 40):
    opt = opt or L.default_options()
    return L.sweep_eval(path, prof, n_u, n_v, opt, pos, FAKE, ws, ws_bytes, 0)


def _expect(status, name, fragment=None):
    assert L.STATUS[status] == name, (L.STATUS.get(status), L.last_error())
    if fragment:
        assert fragment in L.last_error()


def test_null_arguments():
    a, b = _curves()
    o = L.default_options()
    _expect(L.lib().sweep_eval(None, C.byref(b), 256, 64, C.byref(o), FAKE, FAKE, FAKE, 1 << 40, None),
            "SWEEP_ERR_NULL_ARG", "path")
    a.ctrl = None
    _expect(_call(a, b), "SWEEP_ERR_NULL_ARG", "ctrl")
    a, b = _curves()
    _expect(_call(a, b, pos=0), "SWEEP_ERR_NULL_ARG", "pos")


@pytest.mark.parametrize("p", [0, 8, -1])
def test_bad_degree(p):
    a, b = _curves(p=p)
    _expect(_call(a, b), "SWEEP_ERR_BAD_DEGREE")


def test_bad_counts():
    a, b = _curves(n=3, p=3)
    _expect(_call(a, b), "SWEEP_ERR_BAD_COUNT")
    a, b = _curves(m=3, q=3)
    _expect(_call(a, b), "SWEEP_ERR_BAD_COUNT")


def test_bad_knots():
    n, p = 8, 3
    good = np.array([0, 0, 0, 0, .2, .4, .6, .8, 1, 1, 1, 1], float)
    a, b = _curves(n=n, p=p, pk=good.copy())
    assert L.sweep_eval_workspace_size(a, b, 256, 64, L.default_options()) > 0
    for bad, frag in [(np.array([0, 0, 0, 0, .4, .2, .6, .8, 1, 1, 1, 1.]), "decrease"),
                      (np.array([0, 0, 0, 0, .2, np.nan, .6, .8, 1, 1, 1, 1.]), "finite"),
                      (np.array([0, 0, 0, 0, .5, .5, .5, .5, 1, 1, 1, 1.]), "multiplicity"),
                      (np.array([0, 0, 0, 0, 0, .4, .6, .8, 1, 1, 1, 1.]), "multiplicity")]:
        a, b = _curves(n=n, p=p, pk=bad)
        _expect(_call(a, b), "SWEEP_ERR_BAD_KNOTS", frag)


def test_unsupported_forms():
    a, b = _curves()
    a.closed = 1
    _expect(_call(a, b), "SWEEP_ERR_UNSUPPORTED", "closed paths")
    k = np.arange(15, dtype=float)
    a, b = _curves(qk=k)
    _expect(_call(a, b), "SWEEP_ERR_UNSUPPORTED", "knots must be NULL")


@pytest.mark.parametrize("n_u,n_v", [(1, 64), (256, 2), (0, 0), (65536, 32768)])
def test_bad_grid(n_u, n_v):
    a, b = _curves()
    _expect(_call(a, b, n_u=n_u, n_v=n_v), "SWEEP_ERR_BAD_GRID")


def test_bad_options():
    a, b = _curves()
    for field, val, name in [("out_precision", 7, "SWEEP_ERR_BAD_PRECISION"),
                             ("frame_precision", -2, "SWEEP_ERR_BAD_PRECISION"),
                             ("reorthonormalize", 2, "SWEEP_ERR_BAD_OPTION"),
                             ("tile_config", 999, "SWEEP_ERR_BAD_OPTION"),
                             ("tile_config", -2, "SWEEP_ERR_BAD_OPTION")]:
        o = L.default_options()
        setattr(o, field, val)
        _expect(_call(a, b, opt=o), name)
    o = L.default_options()
    o.has_initial_normal = 1
    o.initial_normal[1] = math.inf
    _expect(_call(a, b, opt=o), "SWEEP_ERR_BAD_OPTION")


def test_workspace_checks():
    a, b = _curves()
    need = L.sweep_eval_workspace_size(a, b, 256, 64, L.default_options())
    _expect(_call(a, b, ws_bytes=need - 1), "SWEEP_ERR_WORKSPACE", str(need))
    _expect(_call(a, b, ws=0), "SWEEP_ERR_WORKSPACE")
    _expect(_call(a, b, ws=FAKE + 8), "SWEEP_ERR_WORKSPACE", "aligned")


def test_frame_mode_and_law_options():
    a, b = _curves()
    o = L.default_options()
    assert o.frame_mode == 0 and not o.law
    o.frame_mode = 2
    _expect(_call(a, b, opt=o), "SWEEP_ERR_BAD_OPTION")
    # a law is validated like an open curve
    law = L.SweepCurve(3, 5, 0, 0, FAKE, None)
    o = L.default_options()
    o.law = C.cast(C.pointer(law), C.c_void_p)
    _expect(_call(a, b, opt=o), "SWEEP_ERR_BAD_COUNT")
    law = L.SweepCurve(4, 1, 1, 0, FAKE, None)
    o.law = C.cast(C.pointer(law), C.c_void_p)
    _expect(_call(a, b, opt=o), "SWEEP_ERR_UNSUPPORTED")
    # extended rows need a larger workspace
    law = L.SweepCurve(4, 1, 0, 0, FAKE, None)
    o.law = C.cast(C.pointer(law), C.c_void_p)
    base = L.sweep_eval_workspace_size(a, b, 256, 64, L.default_options())
    assert L.sweep_eval_workspace_size(a, b, 256, 64, o) > base
    o2 = L.default_options()
    o2.frame_mode = 1
    assert L.sweep_eval_workspace_size(a, b, 256, 64, o2) > base
    # frames-only entry point and batches do not take frame modes or laws
    st = L.sweep_frames(a, 256, o2, FAKE, FAKE, 1 << 40, 0)
    assert L.STATUS[st] == "SWEEP_ERR_UNSUPPORTED"


def test_u_sampling_options():
    a, b = _curves()
    o = L.default_options()
    assert o.u_sampling == 0
    o.u_sampling = 3
    _expect(_call(a, b, opt=o), "SWEEP_ERR_BAD_OPTION", "u_sampling")
    # adaptive sampling: a finite weight >= 0
    for lam in (-1.0, math.inf, math.nan):
        o = L.default_options()
        o.u_sampling = 2
        o.u_lambda = lam
        _expect(_call(a, b, opt=o), "SWEEP_ERR_BAD_OPTION", "u_lambda")
    o = L.default_options()
    o.u_sampling = 2
    o.u_lambda = 0.5
    assert L.sweep_eval_workspace_size(a, b, 256, 64, o) > L.sweep_eval_workspace_size(a, b, 256, 64,
                                                                                       L.default_options())
    # arc-length sampling needs room for the length table and sample parameters
    o = L.default_options()
    o.u_sampling = 1
    base = L.sweep_eval_workspace_size(a, b, 256, 64, L.default_options())
    arc = L.sweep_eval_workspace_size(a, b, 256, 64, o)
    assert arc >= base + 8 * (16 - 3) * 32 + 8 * 256
    assert L.sweep_frames_workspace_size(a, 256, o) > L.sweep_frames_workspace_size(a, 256, L.default_options())
    # not together with a law
    law = L.SweepCurve(4, 1, 0, 0, FAKE, None)
    o.law = C.cast(C.pointer(law), C.c_void_p)
    _expect(_call(a, b, opt=o), "SWEEP_ERR_UNSUPPORTED", "arc-length or adaptive")


def test_triangles_validation():
    n = C.c_int64(-1)
    lib = L.lib()
    # the count is reported before the buffer is looked at
    st = lib.sweep_triangles(5, 7, 1, None, 0, C.byref(n), None)
    assert L.STATUS[st] == "SWEEP_ERR_NULL_ARG" and n.value == 2 * 4 * 7
    st = lib.sweep_triangles(5, 7, 0, FAKE, 2 * 4 * 6 - 1, C.byref(n), None)
    assert L.STATUS[st] == "SWEEP_ERR_WORKSPACE" and n.value == 2 * 4 * 6
    assert L.STATUS[lib.sweep_triangles(5, 7, 2, FAKE, 1 << 40, None, None)] == "SWEEP_ERR_BAD_OPTION"
    assert L.STATUS[lib.sweep_triangles(1, 7, 1, FAKE, 1 << 40, None, None)] == "SWEEP_ERR_BAD_GRID"


def test_backward_ex_requires_a_gradient():
    import synth
    from paper_1110_5450_amd import api
    # host tensors stand in for device buffers: nothing below is dereferenced
    spec = synth.single(3, 8, 6, 32, 16)
    b = api.Batch.from_specs([spec], device="cpu")
    o = L.default_options()
    st = L.sweep_backward_ex(b.c_struct(), o, 0, 0, FAKE, FAKE, None, FAKE, 1 << 40, 0)
    assert L.STATUS[st] == "SWEEP_ERR_NULL_ARG" and "both NULL" in L.last_error()
    # knot and weight gradients need the matching batch fields
    for name in ("path_knots", "prof_knots", "path_weights", "prof_weights"):
        pg = L.SweepParamGrads()
        setattr(pg, name, FAKE)
        st = L.sweep_backward_ex(b.c_struct(), o, FAKE, 0, FAKE, FAKE, pg, FAKE, 1 << 40, 0)
        assert L.STATUS[st] == "SWEEP_ERR_BAD_OPTION", name
    st = L.sweep_backward(b.c_struct(), o, 0, FAKE, FAKE, FAKE, 1 << 40, 0)
    assert L.STATUS[st] == "SWEEP_ERR_NULL_ARG" and "grad_pos" in L.last_error()
    assert L.sweep_backward_workspace_size(b.c_struct(), o) > 0
