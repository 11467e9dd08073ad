"""ctypes binding of libsweep.so (argument marshalling only).

Every entry point of ``include/sweep.h`` is exposed with the same name.  The
library must be built (``python -m paper_1110_5450_amd.build``); loading
raises if it is not -- there is no fallback implementation.
"""

from __future__ import annotations

import ctypes as C
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libsweep.so")

SWEEP_OK = 0
STATUS = {
    0: "SWEEP_OK", -1: "SWEEP_ERR_NULL_ARG", -2: "SWEEP_ERR_BAD_COUNT", -3: "SWEEP_ERR_BAD_DEGREE",
    -4: "SWEEP_ERR_BAD_KNOTS", -5: "SWEEP_ERR_BAD_GRID", -6: "SWEEP_ERR_BAD_PRECISION",
    -7: "SWEEP_ERR_WORKSPACE", -8: "SWEEP_ERR_UNSUPPORTED", -9: "SWEEP_ERR_HIP", -10: "SWEEP_ERR_BAD_OPTION",
}
SWEEP_F32, SWEEP_F64 = 0, 1
SWEEP_FRAME_RMF, SWEEP_FRAME_FRENET = 0, 1
SWEEP_U_PARAMETER, SWEEP_U_ARCLENGTH, SWEEP_U_ADAPTIVE = 0, 1, 2

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)


class SweepCurve(C.Structure):
    _fields_ = [("n_ctrl", C.c_int32), ("degree", C.c_int32), ("closed", C.c_int32), ("reserved", C.c_int32),
                ("ctrl", C.c_void_p), ("knots", _dp), ("weights", C.c_void_p)]


class SweepOptions(C.Structure):
    _fields_ = [("out_precision", C.c_int32), ("frame_precision", C.c_int32),
                ("reorthonormalize", C.c_int32), ("has_initial_normal", C.c_int32),
                ("initial_normal", C.c_double * 3), ("tile_config", C.c_int32), ("frame_mode", C.c_int32),
                ("law", C.c_void_p), ("u_sampling", C.c_int32), ("batch_stages", C.c_int32),
                ("u_lambda", C.c_double)]


class SweepParamGrads(C.Structure):
    _fields_ = [("path_knots", C.c_void_p), ("prof_knots", C.c_void_p), ("path_weights", C.c_void_p),
                ("prof_weights", C.c_void_p)]


class SweepBatch(C.Structure):
    _fields_ = [("n_sweeps", C.c_int32), ("reserved", C.c_int32),
                ("path_n", _ip), ("path_degree", _ip), ("prof_n", _ip), ("prof_degree", _ip),
                ("prof_closed", _ip), ("n_u", _ip), ("n_v", _ip),
                ("path_knots", _dp), ("prof_knots", _dp),
                ("path_ctrl", C.c_void_p), ("prof_ctrl", C.c_void_p),
                ("path_weights", C.c_void_p), ("prof_weights", C.c_void_p)]


class SweepError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


_lib = None


def lib():
    """Load libsweep.so.  Raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_1110_5450_amd.build`")
        L = C.CDLL(LIB_PATH)
        vp, sz = C.c_void_p, C.c_size_t
        L.sweep_default_options.argtypes = [C.POINTER(SweepOptions)]
        L.sweep_default_options.restype = None
        L.sweep_eval.argtypes = [C.POINTER(SweepCurve), C.POINTER(SweepCurve), C.c_int32, C.c_int32,
                                 C.POINTER(SweepOptions), vp, vp, vp, sz, vp]
        L.sweep_eval.restype = C.c_int32
        L.sweep_eval_noalloc.argtypes = [C.POINTER(SweepCurve), C.POINTER(SweepCurve), C.c_int32, C.c_int32,
                                         C.POINTER(SweepOptions), vp, vp, vp]
        L.sweep_eval_noalloc.restype = C.c_int32
        L.sweep_eval_workspace_size.argtypes = [C.POINTER(SweepCurve), C.POINTER(SweepCurve), C.c_int32,
                                                C.c_int32, C.POINTER(SweepOptions)]
        L.sweep_eval_workspace_size.restype = sz
        L.sweep_frames.argtypes = [C.POINTER(SweepCurve), C.c_int32, C.POINTER(SweepOptions), vp, vp, sz, vp]
        L.sweep_frames.restype = C.c_int32
        L.sweep_frames_workspace_size.argtypes = [C.POINTER(SweepCurve), C.c_int32, C.POINTER(SweepOptions)]
        L.sweep_frames_workspace_size.restype = sz
        L.sweep_eval_batched.argtypes = [C.POINTER(SweepBatch), C.POINTER(SweepOptions), vp, vp, vp, sz, vp]
        L.sweep_eval_batched.restype = C.c_int32
        L.sweep_batched_workspace_size.argtypes = [C.POINTER(SweepBatch), C.POINTER(SweepOptions)]
        L.sweep_batched_workspace_size.restype = sz
        L.sweep_batched_output_elems.argtypes = [C.POINTER(SweepBatch)]
        L.sweep_batched_output_elems.restype = C.c_int64
        L.sweep_backward.argtypes = [C.POINTER(SweepBatch), C.POINTER(SweepOptions), vp, vp, vp, vp, sz, vp]
        L.sweep_backward.restype = C.c_int32
        L.sweep_backward_ex.argtypes = [C.POINTER(SweepBatch), C.POINTER(SweepOptions), vp, vp, vp, vp,
                                        C.POINTER(SweepParamGrads), vp, sz, vp]
        L.sweep_backward_ex.restype = C.c_int32
        L.sweep_backward_workspace_size.argtypes = [C.POINTER(SweepBatch), C.POINTER(SweepOptions)]
        L.sweep_backward_workspace_size.restype = sz
        L.sweep_trace_enable.argtypes = [C.c_int32]
        L.sweep_trace_enable.restype = C.c_int32
        L.sweep_trace_read.argtypes = [_ip, C.POINTER(C.c_float), C.c_int32]
        L.sweep_trace_read.restype = C.c_int32
        L.sweep_autotune.argtypes = [C.POINTER(SweepCurve), C.POINTER(SweepCurve), C.c_int32, C.c_int32,
                                     C.POINTER(SweepOptions), vp, vp, vp, sz, vp, _ip, C.POINTER(C.c_float)]
        L.sweep_autotune.restype = C.c_int32
        L.sweep_autotune_batched.argtypes = [C.POINTER(SweepBatch), C.POINTER(SweepOptions), vp, vp, vp, sz, vp, _ip,
                                             C.POINTER(C.c_float)]
        L.sweep_autotune_batched.restype = C.c_int32
        L.sweep_batched_config_for.argtypes = [C.POINTER(SweepBatch), C.POINTER(SweepOptions), C.c_int32]
        L.sweep_batched_config_for.restype = C.c_int32
        L.sweep_surface_config_for.argtypes = [C.c_int32, C.c_int32, C.c_int32]
        L.sweep_surface_config_for.restype = C.c_int32
        L.sweep_triangles.argtypes = [C.c_int32, C.c_int32, C.c_int32, vp, C.c_int64, C.POINTER(C.c_int64), vp]
        L.sweep_triangles.restype = C.c_int32
        L.sweep_tile_config_count.argtypes = []
        L.sweep_tile_config_count.restype = C.c_int32
        L.sweep_tile_config_info.argtypes = [C.c_int32, _ip]
        L.sweep_tile_config_info.restype = C.c_int32
        L.sweep_last_error.argtypes = []
        L.sweep_last_error.restype = C.c_char_p
        L.sweep_version.argtypes = []
        L.sweep_version.restype = C.c_int32
        L.sweep_release_caches.argtypes = []
        L.sweep_release_caches.restype = None
        _lib = L
    return _lib


def last_error() -> str:
    return lib().sweep_last_error().decode()


def check(status: int) -> None:
    if status != SWEEP_OK:
        raise SweepError(status, last_error())


def default_options() -> SweepOptions:
    o = SweepOptions()
    lib().sweep_default_options(C.byref(o))
    return o


# Same-named thin wrappers over the C entry points.

def sweep_default_options(opt: SweepOptions) -> None:
    lib().sweep_default_options(C.byref(opt))


def sweep_eval(path: SweepCurve, profile: SweepCurve, n_u: int, n_v: int, opt: SweepOptions,
               pos: int, nrm: int, workspace: int, ws_bytes: int, stream: int) -> int:
    return lib().sweep_eval(C.byref(path), C.byref(profile), n_u, n_v, C.byref(opt), pos, nrm, workspace,
                            ws_bytes, stream)


def sweep_eval_noalloc(path: SweepCurve, profile: SweepCurve, n_u: int, n_v: int, opt: SweepOptions,
                       pos: int, nrm: int, stream: int) -> int:
    return lib().sweep_eval_noalloc(C.byref(path), C.byref(profile), n_u, n_v, C.byref(opt), pos, nrm, stream)


def sweep_eval_workspace_size(path: SweepCurve, profile: SweepCurve, n_u: int, n_v: int, opt: SweepOptions) -> int:
    return lib().sweep_eval_workspace_size(C.byref(path), C.byref(profile), n_u, n_v, C.byref(opt))


def sweep_frames(path: SweepCurve, n_u: int, opt: SweepOptions, frames: int, workspace: int, ws_bytes: int,
                 stream: int) -> int:
    return lib().sweep_frames(C.byref(path), n_u, C.byref(opt), frames, workspace, ws_bytes, stream)


def sweep_frames_workspace_size(path: SweepCurve, n_u: int, opt: SweepOptions) -> int:
    return lib().sweep_frames_workspace_size(C.byref(path), n_u, C.byref(opt))


def sweep_eval_batched(batch: SweepBatch, opt: SweepOptions, pos: int, nrm: int, workspace: int,
                       ws_bytes: int, stream: int) -> int:
    return lib().sweep_eval_batched(C.byref(batch), C.byref(opt), pos, nrm, workspace, ws_bytes, stream)


def sweep_batched_workspace_size(batch: SweepBatch, opt: SweepOptions) -> int:
    return lib().sweep_batched_workspace_size(C.byref(batch), C.byref(opt))


def sweep_backward(batch: SweepBatch, opt: SweepOptions, grad_pos: int, grad_path_ctrl: int,
                   grad_prof_ctrl: int, workspace: int, ws_bytes: int, stream: int) -> int:
    return lib().sweep_backward(C.byref(batch), C.byref(opt), grad_pos, grad_path_ctrl, grad_prof_ctrl,
                                workspace, ws_bytes, stream)


def sweep_backward_ex(batch: SweepBatch, opt: SweepOptions, grad_pos: int, grad_nrm: int, grad_path_ctrl: int,
                      grad_prof_ctrl: int, params, workspace: int, ws_bytes: int, stream: int) -> int:
    """params: a SweepParamGrads or None."""
    return lib().sweep_backward_ex(C.byref(batch), C.byref(opt), grad_pos, grad_nrm, grad_path_ctrl,
                                   grad_prof_ctrl, C.byref(params) if params is not None else None, workspace,
                                   ws_bytes, stream)


def sweep_batched_output_elems(batch: SweepBatch) -> int:
    return lib().sweep_batched_output_elems(C.byref(batch))


def sweep_backward_workspace_size(batch: SweepBatch, opt: SweepOptions) -> int:
    return lib().sweep_backward_workspace_size(C.byref(batch), C.byref(opt))


def sweep_triangles(n_u: int, n_v: int, closed_v: int, tri: int, max_tri: int, stream: int):
    """(status, n_tri)."""
    n = C.c_int64(0)
    st = lib().sweep_triangles(n_u, n_v, closed_v, tri, max_tri, C.byref(n), stream)
    return st, n.value


def sweep_trace_enable(max_calls: int) -> int:
    return lib().sweep_trace_enable(max_calls)


def sweep_trace_read(max_records: int = 8192):
    """[(stage, ms), ...] of the recorded calls (stage 0 frame, 1 surface)."""
    st = (C.c_int32 * max_records)()
    ms = (C.c_float * max_records)()
    n = lib().sweep_trace_read(st, ms, max_records)
    if n < 0:
        raise SweepError(n, last_error())
    return [(int(st[k]), float(ms[k])) for k in range(n)]


def sweep_autotune(path: SweepCurve, profile: SweepCurve, n_u: int, n_v: int, opt: SweepOptions,
                   pos: int, nrm: int, workspace: int, ws_bytes: int, stream: int):
    """Returns (status, best_config, best_ms)."""
    best = C.c_int32(-1)
    ms = C.c_float(0.0)
    st = lib().sweep_autotune(C.byref(path), C.byref(profile), n_u, n_v, C.byref(opt), pos, nrm, workspace,
                              ws_bytes, stream, C.byref(best), C.byref(ms))
    return st, best.value, ms.value


def sweep_surface_config_for(n_u: int, n_v: int, out_precision: int) -> int:
    return lib().sweep_surface_config_for(n_u, n_v, out_precision)


def sweep_tile_config_count() -> int:
    return lib().sweep_tile_config_count()


def sweep_tile_config_info(k: int):
    """(status, (kind, rows_per_block, tile_vertices, nontemporal))."""
    a = (C.c_int32 * 4)()
    st = lib().sweep_tile_config_info(k, a)
    return st, tuple(a)


def sweep_last_error() -> str:
    return last_error()


def sweep_version() -> int:
    return lib().sweep_version()


def sweep_release_caches() -> None:
    lib().sweep_release_caches()


def sweep_autotune_batched(batch: SweepBatch, opt: SweepOptions, pos: int, nrm: int, workspace: int, ws_bytes: int,
                           stream: int):
    """(status, best_config, best_ms)."""
    c = C.c_int32(-1)
    t = C.c_float(0.0)
    st = lib().sweep_autotune_batched(C.byref(batch), C.byref(opt), pos, nrm, workspace, ws_bytes, stream,
                                      C.byref(c), C.byref(t))
    return st, c.value, t.value


def sweep_batched_config_for(batch: SweepBatch, opt: SweepOptions, with_normals: int) -> int:
    return lib().sweep_batched_config_for(C.byref(batch), C.byref(opt), with_normals)
