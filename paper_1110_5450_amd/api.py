"""PyTorch-facing wrappers of the C ABI.

torch supplies device memory (outputs and workspace) and the current HIP
stream; every step of the computation runs in libsweep's HIP kernels.
Control points must be CUDA (HIP) float64 tensors of shape (n, 3).
"""

from __future__ import annotations

import ctypes as C
from typing import Optional, Sequence, Tuple

import numpy as np
import torch

from . import _lib as L

_DT = {torch.float32: L.SWEEP_F32, torch.float64: L.SWEEP_F64}


def _check_ctrl(t: torch.Tensor, what: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{what} must be a device tensor")
    if t.dtype != torch.float64:
        raise TypeError(f"{what} must be float64")
    if t.dim() != 2 or t.shape[1] != 3:
        raise ValueError(f"{what} must have shape (n, 3)")
    return t.contiguous()


def _weights(w, n: int, what: str) -> Optional[torch.Tensor]:
    """Device float64 weights (n,) or None; positivity is the caller's
    responsibility (device data is not inspected)."""
    if w is None:
        return None
    if not isinstance(w, torch.Tensor) or not w.is_cuda:
        raise TypeError(f"{what} must be a device tensor")
    if w.dtype != torch.float64:
        raise TypeError(f"{what} must be float64")
    w = w.contiguous().reshape(-1)
    if w.shape[0] != n:
        raise ValueError(f"{what} needs {n} values, got {w.shape[0]}")
    return w


def _wptr(w: Optional[torch.Tensor]) -> Optional[int]:
    return None if w is None else w.data_ptr()


def _knots_ptr(knots) -> Tuple[Optional[np.ndarray], Optional[C.POINTER(C.c_double)]]:
    if knots is None:
        return None, None
    a = np.ascontiguousarray(np.asarray(knots, dtype=np.float64))
    return a, a.ctypes.data_as(C.POINTER(C.c_double))


_FRAME_MODES = {"rmf": L.SWEEP_FRAME_RMF, "frenet": L.SWEEP_FRAME_FRENET}


class Law:
    """A sweep law: an open B-spline whose control points (device float64,
    (n, 3)) hold (scale, twist angle in radians, unused) along the path;
    degree, optional knot vector (host) and weights."""

    def __init__(self, ctrl: torch.Tensor, degree: int, knots=None, weights=None):
        self.ctrl = _check_ctrl(ctrl, "law ctrl")
        self.degree = int(degree)
        self._knots, kp = _knots_ptr(knots)
        self.weights = _weights(weights, self.ctrl.shape[0], "law weights")
        self.c = L.SweepCurve(self.ctrl.shape[0], self.degree, 0, 0, self.ctrl.data_ptr(), kp, _wptr(self.weights))


_U_SAMPLING = {"parameter": L.SWEEP_U_PARAMETER, "arclength": L.SWEEP_U_ARCLENGTH,
               "adaptive": L.SWEEP_U_ADAPTIVE}


def make_options(out_dtype=torch.float32, frame_dtype=torch.float64, reorthonormalize: bool = True,
                 initial_normal=None, tile_config: int = -1, frame_mode: str = "rmf",
                 law: Optional[Law] = None, u_sampling: str = "parameter", u_lambda: float = 0.0) -> L.SweepOptions:
    o = L.default_options()
    o.out_precision = _DT[out_dtype]
    o.frame_precision = _DT[frame_dtype]
    o.reorthonormalize = int(bool(reorthonormalize))
    if initial_normal is not None:
        o.has_initial_normal = 1
        for k in range(3):
            o.initial_normal[k] = float(initial_normal[k])
    o.tile_config = int(tile_config)
    if frame_mode not in _FRAME_MODES:
        raise ValueError(f"frame_mode must be one of {sorted(_FRAME_MODES)}")
    o.frame_mode = _FRAME_MODES[frame_mode]
    if u_sampling not in _U_SAMPLING:
        raise ValueError(f"u_sampling must be one of {sorted(_U_SAMPLING)}")
    o.u_sampling = _U_SAMPLING[u_sampling]
    o.u_lambda = float(u_lambda)
    if law is not None:
        o.law = C.cast(C.pointer(law.c), C.c_void_p)
        o._law_ref = law          # keeps the curve struct and its buffers alive
    return o


def _nbytes(t: torch.Tensor) -> int:
    return t.numel() * t.element_size()


def _check_out(t: torch.Tensor, numel: int, dtype, what: str) -> None:
    """An output buffer must hold at least `numel` contiguous elements of
    `dtype` on a GPU: the kernels write through its raw pointer."""
    if not isinstance(t, torch.Tensor) or t.dtype != dtype or not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{what} must be a contiguous {dtype} CUDA tensor")
    if t.numel() < numel:
        raise ValueError(f"{what} holds {t.numel()} elements, {numel} are written")


def _stream_handle(stream) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def sweep_eval(path_ctrl: torch.Tensor, path_degree: int, prof_ctrl: torch.Tensor, prof_degree: int,
               n_u: int, n_v: int, *, prof_closed: bool = True, path_knots=None, prof_knots=None,
               out_dtype=torch.float32, frame_dtype=torch.float64, reorthonormalize: bool = True,
               initial_normal=None, tile_config: int = -1, normals: bool = True,
               path_weights=None, prof_weights=None, frame_mode: str = "rmf", law: Optional[Law] = None,
               u_sampling: str = "parameter", u_lambda: float = 0.0,
               out: Optional[Tuple[torch.Tensor, Optional[torch.Tensor]]] = None,
               workspace: Optional[torch.Tensor] = None, stream=None):
    """Positions (3, n_u, n_v) and normals (or None) of one sweep; with
    weights (device float64, one per control point) a curve is rational;
    u_sampling="arclength" places the path samples at equal arc length,
    "adaptive" at equal steps of arc length + u_lambda x turning angle."""
    pc = _check_ctrl(path_ctrl, "path_ctrl")
    qc = _check_ctrl(prof_ctrl, "prof_ctrl")
    pw = _weights(path_weights, pc.shape[0], "path_weights")
    qw = _weights(prof_weights, qc.shape[0], "prof_weights")
    pk, pkp = _knots_ptr(path_knots)
    qk, qkp = _knots_ptr(prof_knots)
    path = L.SweepCurve(pc.shape[0], int(path_degree), 0, 0, pc.data_ptr(), pkp, _wptr(pw))
    prof = L.SweepCurve(qc.shape[0], int(prof_degree), int(bool(prof_closed)), 0, qc.data_ptr(), qkp, _wptr(qw))
    opt = make_options(out_dtype, frame_dtype, reorthonormalize, initial_normal, tile_config, frame_mode, law,
                       u_sampling, u_lambda)
    ws_bytes = L.sweep_eval_workspace_size(path, prof, int(n_u), int(n_v), opt)
    if ws_bytes == 0:
        # invalid metadata: let the call report the reason
        L.check(L.sweep_eval(path, prof, int(n_u), int(n_v), opt, 0, 0, 0, 0, 0))
    dev = pc.device
    if out is None:
        pos = torch.empty((3, n_u, n_v), dtype=out_dtype, device=dev)
        nrm = torch.empty((3, n_u, n_v), dtype=out_dtype, device=dev) if normals else None
    else:
        pos, nrm = out
        _check_out(pos, 3 * n_u * n_v, out_dtype, "out[0]")
        if nrm is not None:
            _check_out(nrm, 3 * n_u * n_v, out_dtype, "out[1]")
    if workspace is None or _nbytes(workspace) < ws_bytes:
        workspace = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    st = L.sweep_eval(path, prof, int(n_u), int(n_v), opt, pos.data_ptr(),
                      nrm.data_ptr() if nrm is not None else 0, workspace.data_ptr(), _nbytes(workspace),
                      _stream_handle(stream))
    L.check(st)
    return pos, nrm


def sweep_autotune(path_ctrl: torch.Tensor, path_degree: int, prof_ctrl: torch.Tensor, prof_degree: int,
                   n_u: int, n_v: int, *, prof_closed: bool = True, path_knots=None, prof_knots=None,
                   out_dtype=torch.float32, frame_dtype=torch.float64, reorthonormalize: bool = True,
                   initial_normal=None, normals: bool = True, path_weights=None, prof_weights=None,
                   frame_mode: str = "rmf", law: Optional[Law] = None, u_sampling: str = "parameter",
                   u_lambda: float = 0.0, stream=None):
    """Times every surface configuration on this sweep and records the
    fastest for its shape class; returns (best_config, best_ms, pos, nrm)."""
    pc = _check_ctrl(path_ctrl, "path_ctrl")
    qc = _check_ctrl(prof_ctrl, "prof_ctrl")
    pw = _weights(path_weights, pc.shape[0], "path_weights")
    qw = _weights(prof_weights, qc.shape[0], "prof_weights")
    pk, pkp = _knots_ptr(path_knots)
    qk, qkp = _knots_ptr(prof_knots)
    path = L.SweepCurve(pc.shape[0], int(path_degree), 0, 0, pc.data_ptr(), pkp, _wptr(pw))
    prof = L.SweepCurve(qc.shape[0], int(prof_degree), int(bool(prof_closed)), 0, qc.data_ptr(), qkp, _wptr(qw))
    opt = make_options(out_dtype, frame_dtype, reorthonormalize, initial_normal, frame_mode=frame_mode, law=law,
                       u_sampling=u_sampling, u_lambda=u_lambda)
    ws_bytes = L.sweep_eval_workspace_size(path, prof, int(n_u), int(n_v), opt)
    if ws_bytes == 0:
        L.check(L.sweep_eval(path, prof, int(n_u), int(n_v), opt, 0, 0, 0, 0, 0))
    dev = pc.device
    pos = torch.empty((3, n_u, n_v), dtype=out_dtype, device=dev)
    nrm = torch.empty((3, n_u, n_v), dtype=out_dtype, device=dev) if normals else None
    workspace = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    st, best, ms = L.sweep_autotune(path, prof, int(n_u), int(n_v), opt, pos.data_ptr(),
                                    nrm.data_ptr() if nrm is not None else 0, workspace.data_ptr(),
                                    _nbytes(workspace), _stream_handle(stream))
    L.check(st)
    return best, ms, pos, nrm


def surface_config_for(n_u: int, n_v: int, out_dtype=torch.float32) -> int:
    """Configuration index that tile_config=-1 selects for this shape."""
    return L.sweep_surface_config_for(int(n_u), int(n_v),
                                      L.SWEEP_F64 if out_dtype == torch.float64 else L.SWEEP_F32)


def sweep_frames(path_ctrl: torch.Tensor, path_degree: int, n_u: int, *, path_knots=None,
                 out_dtype=torch.float64, frame_dtype=torch.float64, reorthonormalize: bool = True,
                 initial_normal=None, path_weights=None, frame_mode: str = "rmf",
                 u_sampling: str = "parameter", u_lambda: float = 0.0,
                 workspace: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """Row records (n_u, 16): x, r, s, t, |C'|, a, b, 0 of the moving frame
    (rotation-minimizing; other frame modes are sweep_eval only)."""
    pc = _check_ctrl(path_ctrl, "path_ctrl")
    pw = _weights(path_weights, pc.shape[0], "path_weights")
    pk, pkp = _knots_ptr(path_knots)
    path = L.SweepCurve(pc.shape[0], int(path_degree), 0, 0, pc.data_ptr(), pkp, _wptr(pw))
    opt = make_options(out_dtype, frame_dtype, reorthonormalize, initial_normal, frame_mode=frame_mode,
                       u_sampling=u_sampling, u_lambda=u_lambda)
    ws_bytes = L.sweep_frames_workspace_size(path, int(n_u), opt)
    if ws_bytes == 0:
        L.check(L.sweep_frames(path, int(n_u), opt, 0, 0, 0, 0))
    out = torch.empty((n_u, 16), dtype=out_dtype, device=pc.device)
    if workspace is None or _nbytes(workspace) < ws_bytes:
        workspace = torch.empty(ws_bytes, dtype=torch.uint8, device=pc.device)
    L.check(L.sweep_frames(path, int(n_u), opt, out.data_ptr(), workspace.data_ptr(), _nbytes(workspace),
                           _stream_handle(stream)))
    return out


def eval_workspace_size(n_path: int, path_degree: int, n_prof: int, prof_degree: int, n_u: int, n_v: int, *,
                        prof_closed: bool = True, out_dtype=torch.float32, frame_dtype=torch.float64,
                        frame_mode: str = "rmf", law: Optional[Law] = None, u_sampling: str = "parameter",
                        u_lambda: float = 0.0) -> int:
    path = L.SweepCurve(n_path, path_degree, 0, 0, 1, None, None)
    prof = L.SweepCurve(n_prof, prof_degree, int(prof_closed), 0, 1, None, None)
    return L.sweep_eval_workspace_size(path, prof, n_u, n_v,
                                       make_options(out_dtype, frame_dtype, frame_mode=frame_mode, law=law,
                                                    u_sampling=u_sampling, u_lambda=u_lambda))


def triangle_count(n_u: int, n_v: int, closed_v: bool = True) -> int:
    return 2 * (int(n_u) - 1) * (int(n_v) if closed_v else int(n_v) - 1)


def triangles(n_u: int, n_v: int, closed_v: bool = True, *, out: Optional[torch.Tensor] = None,
              device="cuda", stream=None) -> torch.Tensor:
    """Triangle list (n_tri, 3) int32 of the n_u x n_v grid of a sweep
    (vertex (i, j) = i*n_v + j), counter-clockwise about X_v x X_u."""
    nt = triangle_count(n_u, n_v, closed_v)
    if out is None:
        out = torch.empty((max(nt, 0), 3), dtype=torch.int32, device=device)
    else:
        _check_out(out, 3 * nt, torch.int32, "out")
    st, n = L.sweep_triangles(int(n_u), int(n_v), int(bool(closed_v)), out.data_ptr() if out.numel() else 0,
                              out.numel() // 3, _stream_handle(stream))
    L.check(st)
    assert n == nt
    return out


class Batch:
    """A batch of independent sweeps packed for sweep_eval_batched /
    sweep_backward.  Control points are packed into one device float64 buffer
    per curve kind; per-sweep counts, degrees, grid sizes and knot vectors
    stay in host memory.  Flat outputs use the padded batched layout: sweep
    k's planes have stride plane[k] (n_u*n_v rounded up to a multiple of
    PLANE_ALIGN elements) and its block starts at element offsets[k]; a flat
    buffer holds out_elems elements (view() gives a sweep's block)."""

    PLANE_ALIGN = 64

    def __init__(self, path_ctrl: Sequence, path_degree: Sequence[int], prof_ctrl: Sequence,
                 prof_degree: Sequence[int], n_u: Sequence[int], n_v: Sequence[int], *, prof_closed=None,
                 path_knots=None, prof_knots=None, path_weights=None, prof_weights=None, device="cuda"):
        n = len(path_ctrl)
        self.n_sweeps = n
        as_np = lambda a: np.ascontiguousarray(a.detach().cpu().numpy() if isinstance(a, torch.Tensor) else a,
                                               dtype=np.float64).reshape(-1, 3)
        P = [as_np(a) for a in path_ctrl]
        Q = [as_np(a) for a in prof_ctrl]
        self.path_n = np.array([a.shape[0] for a in P], np.int32)
        self.prof_n = np.array([a.shape[0] for a in Q], np.int32)
        self.path_degree = np.array(path_degree, np.int32)
        self.prof_degree = np.array(prof_degree, np.int32)
        self.n_u = np.array(n_u, np.int32)
        self.n_v = np.array(n_v, np.int32)
        self.prof_closed = None if prof_closed is None else np.array(prof_closed, np.int32)
        # Knot vectors: all paths or none; all open profiles or none.
        if path_knots is not None and any(k is None for k in path_knots):
            raise ValueError("path_knots must give a vector for every path (or be None)")
        self.path_knots = None if path_knots is None else np.ascontiguousarray(np.concatenate(
            [np.asarray(k, np.float64) for k in path_knots]))
        self.prof_knots = None
        if prof_knots is not None:
            closed = self.prof_closed if self.prof_closed is not None else np.ones(n, np.int32)
            if any((k is None) != bool(c) for k, c in zip(prof_knots, closed)):
                raise ValueError("prof_knots must give a vector for every open profile and None for closed ones")
            ks = [np.asarray(k, np.float64) for k in prof_knots if k is not None]
            self.prof_knots = np.ascontiguousarray(np.concatenate(ks)) if ks else None
        self.path_ctrl = torch.as_tensor(np.concatenate(P)).to(device)
        self.prof_ctrl = torch.as_tensor(np.concatenate(Q)).to(device)
        # Weights: for every path (profile) or for none; packed like the control points.
        self.path_weights = self._pack_weights(path_weights, P, "path_weights", device)
        self.prof_weights = self._pack_weights(prof_weights, Q, "prof_weights", device)
        sizes = self.n_u.astype(np.int64) * self.n_v.astype(np.int64)
        a = self.PLANE_ALIGN
        self.plane = (sizes + a - 1) // a * a
        self.offsets = np.concatenate([[0], np.cumsum(3 * self.plane)[:-1]]).astype(np.int64)
        self.out_elems = int(3 * self.plane.sum())
        self.n_vertices = int(sizes.sum())
        self.path_offsets = np.concatenate([[0], np.cumsum(self.path_n)[:-1]]).astype(np.int64)
        self.prof_offsets = np.concatenate([[0], np.cumsum(self.prof_n)[:-1]]).astype(np.int64)
        # offsets of each sweep's knots in the packed knot arrays (-1: none)
        closed = self.prof_closed if self.prof_closed is not None else np.ones(n, np.int32)
        pk_len = (self.path_n + self.path_degree + 1).astype(np.int64)
        qk_len = np.where(closed == 0, self.prof_n + self.prof_degree + 1, 0).astype(np.int64)
        self.path_knot_offsets = (np.concatenate([[0], np.cumsum(pk_len)[:-1]]) if self.path_knots is not None
                                  else np.full(n, -1)).astype(np.int64)
        self.prof_knot_offsets = (np.where(closed == 0, np.concatenate([[0], np.cumsum(qk_len)[:-1]]), -1)
                                  if self.prof_knots is not None else np.full(n, -1)).astype(np.int64)

    @staticmethod
    def _pack_weights(ws, ctrl, what, device):
        if ws is None:
            return None
        if any(w is None for w in ws):
            raise ValueError(f"{what} must give weights for every curve (or be None)")
        flat = []
        for w, c in zip(ws, ctrl):
            w = np.asarray(w.detach().cpu().numpy() if isinstance(w, torch.Tensor) else w, np.float64).reshape(-1)
            if w.shape[0] != c.shape[0]:
                raise ValueError(f"{what}: one weight per control point")
            flat.append(w)
        return torch.as_tensor(np.concatenate(flat)).to(device)

    @classmethod
    def from_specs(cls, specs, device="cuda") -> "Batch":
        """From objects with path/profile (ctrl, degree, closed, knots,
        weights), n_u, n_v."""
        pk = [s.path.knots for s in specs]
        qk = [s.profile.knots for s in specs]
        pw = [getattr(s.path, "weights", None) for s in specs]
        qw = [getattr(s.profile, "weights", None) for s in specs]
        return cls([s.path.ctrl for s in specs], [s.path.degree for s in specs],
                   [s.profile.ctrl for s in specs], [s.profile.degree for s in specs],
                   [s.n_u for s in specs], [s.n_v for s in specs],
                   prof_closed=[int(s.profile.closed) for s in specs],
                   path_knots=None if all(k is None for k in pk) else pk,
                   prof_knots=None if all(k is None for k in qk) else qk,
                   path_weights=None if all(w is None for w in pw) else pw,
                   prof_weights=None if all(w is None for w in qw) else qw, device=device)

    def c_struct(self) -> L.SweepBatch:
        ip = lambda a: None if a is None else a.ctypes.data_as(C.POINTER(C.c_int32))
        dp = lambda a: None if a is None else a.ctypes.data_as(C.POINTER(C.c_double))
        return L.SweepBatch(self.n_sweeps, 0, ip(self.path_n), ip(self.path_degree), ip(self.prof_n),
                            ip(self.prof_degree), ip(self.prof_closed), ip(self.n_u), ip(self.n_v),
                            dp(self.path_knots), dp(self.prof_knots),
                            self.path_ctrl.data_ptr(), self.prof_ctrl.data_ptr(),
                            _wptr(self.path_weights), _wptr(self.prof_weights))

    def view(self, flat: torch.Tensor, k: int) -> torch.Tensor:
        """Sweep k's (3, n_u, n_v) block of a flat batched output (a view with
        plane stride plane[k])."""
        o, nu, nv, P = int(self.offsets[k]), int(self.n_u[k]), int(self.n_v[k]), int(self.plane[k])
        return flat[o: o + 3 * P].view(3, P)[:, :nu * nv].view(3, nu, nv)

    def pack(self, blocks, dtype=torch.float32) -> torch.Tensor:
        """A flat buffer in the batched layout from per-sweep (3, n_u, n_v)
        blocks (padding 0)."""
        flat = torch.zeros(self.out_elems, dtype=dtype, device=self.path_ctrl.device)
        for k, blk in enumerate(blocks):
            self.view(flat, k).copy_(torch.as_tensor(blk))
        return flat

    def path_knot_slice(self, k: int) -> slice:
        o = int(self.path_knot_offsets[k])
        return slice(o, o + int(self.path_n[k] + self.path_degree[k] + 1))

    def prof_knot_slice(self, k: int) -> slice:
        o = int(self.prof_knot_offsets[k])
        return slice(o, o + int(self.prof_n[k] + self.prof_degree[k] + 1))

    def path_slice(self, k: int) -> slice:
        return slice(int(self.path_offsets[k]), int(self.path_offsets[k] + self.path_n[k]))

    def prof_slice(self, k: int) -> slice:
        return slice(int(self.prof_offsets[k]), int(self.prof_offsets[k] + self.prof_n[k]))


def sweep_eval_batched(batch: Batch, *, out_dtype=torch.float32, frame_dtype=torch.float64,
                       reorthonormalize: bool = True, initial_normal=None, tile_config: int = -1,
                       normals: bool = True, frame_mode: str = "rmf", out=None,
                       workspace: Optional[torch.Tensor] = None, stream=None, stages: int = 0,
                       law: Optional[Law] = None, u_sampling: str = "parameter", u_lambda: float = 0.0):
    """Flat positions and normals (or None) of a batch in the padded batched
    layout.  frame_mode, law and u_sampling apply to every sweep of the
    batch (one law for all; they need the FP64 frame; arc-length sampling
    without a frame mode or law).  stages: pipeline stages of the
    frame/surface schedule (0: automatic)."""
    b = batch.c_struct()
    opt = make_options(out_dtype, frame_dtype, reorthonormalize, initial_normal, tile_config, frame_mode, law,
                       u_sampling, u_lambda)
    opt.batch_stages = int(stages)
    ws_bytes = L.sweep_batched_workspace_size(b, opt)
    if ws_bytes == 0:
        L.check(L.sweep_eval_batched(b, opt, 0, 0, 0, 0, 0))
    dev = batch.path_ctrl.device
    if out is None:
        pos = torch.empty(batch.out_elems, dtype=out_dtype, device=dev)
        nrm = torch.empty(batch.out_elems, dtype=out_dtype, device=dev) if normals else None
    else:
        pos, nrm = out
        _check_out(pos, batch.out_elems, out_dtype, "out[0]")
        if nrm is not None:
            _check_out(nrm, batch.out_elems, out_dtype, "out[1]")
    if workspace is None or _nbytes(workspace) < ws_bytes:
        workspace = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    L.check(L.sweep_eval_batched(b, opt, pos.data_ptr(), nrm.data_ptr() if nrm is not None else 0,
                                 workspace.data_ptr(), _nbytes(workspace), _stream_handle(stream)))
    return pos, nrm


def autotune_batched(batch: Batch, *, out_dtype=torch.float32, frame_dtype=torch.float64,
                     reorthonormalize: bool = True, initial_normal=None, normals: bool = True, out=None,
                     workspace: Optional[torch.Tensor] = None, stream=None):
    """Time every batched surface tile configuration on this batch (into
    `out` or fresh buffers) and record the fastest for its shape class;
    returns (best_config, best_ms)."""
    b = batch.c_struct()
    opt = make_options(out_dtype, frame_dtype, reorthonormalize, initial_normal, -1)
    ws_bytes = L.sweep_batched_workspace_size(b, opt)
    if ws_bytes == 0:
        L.check(L.sweep_eval_batched(b, opt, 0, 0, 0, 0, 0))
    dev = batch.path_ctrl.device
    if out is None:
        pos = torch.empty(batch.out_elems, dtype=out_dtype, device=dev)
        nrm = torch.empty(batch.out_elems, dtype=out_dtype, device=dev) if normals else None
    else:
        pos, nrm = out
        _check_out(pos, batch.out_elems, out_dtype, "out[0]")
        if nrm is not None:
            _check_out(nrm, batch.out_elems, out_dtype, "out[1]")
    if workspace is None or _nbytes(workspace) < ws_bytes:
        workspace = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    st, cfg, ms = L.sweep_autotune_batched(b, opt, pos.data_ptr(), nrm.data_ptr() if nrm is not None else 0,
                                           workspace.data_ptr(), _nbytes(workspace), _stream_handle(stream))
    L.check(st)
    return cfg, ms


def batched_config_for(batch: Batch, *, out_dtype=torch.float32, frame_dtype=torch.float64,
                       tile_config: int = -1, normals: bool = True) -> int:
    """The tile_config index sweep_eval_batched uses for this batch."""
    return L.sweep_batched_config_for(batch.c_struct(),
                                      make_options(out_dtype, frame_dtype, tile_config=tile_config), int(normals))


def tile_config_name(k: int) -> str:
    """Human-readable description of surface configuration k."""
    st, (kind, rows, tv, nt) = L.sweep_tile_config_info(int(k))
    L.check(st)
    store = "nontemporal" if nt else "plain"
    if kind == 0:
        return f"config {k}: column tiles, 256 columns x {rows} row(s) per block, {store} stores"
    return f"config {k}: linear tiles of {tv} vertices per block, {store} stores"


def batched_workspace_size(batch: Batch, out_dtype=torch.float32, frame_dtype=torch.float64,
                           frame_mode: str = "rmf", law: Optional[Law] = None, u_sampling: str = "parameter",
                           u_lambda: float = 0.0) -> int:
    """Workspace bytes of sweep_eval_batched (a frame mode or law: longer row
    records; arc-length or adaptive sampling: the length tables)."""
    return L.sweep_batched_workspace_size(batch.c_struct(),
                                          make_options(out_dtype, frame_dtype, frame_mode=frame_mode, law=law,
                                                       u_sampling=u_sampling, u_lambda=u_lambda))


_PARAM_GRADS = ("path_knots", "prof_knots", "path_weights", "prof_weights")


def sweep_backward(batch: Batch, grad_pos: Optional[torch.Tensor], *, grad_nrm: Optional[torch.Tensor] = None,
                   params: Sequence[str] = (), initial_normal=None, workspace=None, stream=None):
    """Gradients of L with dL/dpos = grad_pos and dL/dnrm = grad_nrm (flat,
    like the batched outputs; their dtype is the output precision; either may
    be None, not both) with respect to the packed path and profile control
    points: (g_path (sum path_n, 3), g_prof (sum prof_n, 3)), float64.  With
    params (names among path_knots, prof_knots, path_weights, prof_weights)
    a third item maps each name to its float64 gradient, packed like the
    batch's knot or weight array."""
    b = batch.c_struct()
    given = [t for t in (grad_pos, grad_nrm) if t is not None]
    if not given:
        raise ValueError("grad_pos and grad_nrm are both None")
    dt = given[0].dtype
    if dt not in _DT or any(t.dtype != dt for t in given):
        raise TypeError("grad_pos / grad_nrm must both be float32 or both float64")
    g = grad_pos.contiguous() if grad_pos is not None else None
    gn = grad_nrm.contiguous() if grad_nrm is not None else None
    for t, what in ((g, "grad_pos"), (gn, "grad_nrm")):
        if t is not None and t.numel() != batch.out_elems:
            raise ValueError(f"{what} has the wrong size")
    opt = make_options(dt, torch.float64, True, initial_normal)
    ws_bytes = L.sweep_backward_workspace_size(b, opt)
    if ws_bytes == 0:
        L.check(L.sweep_backward_ex(b, opt, 0, 0, 0, 0, None, 0, 0, 0))
    dev = batch.path_ctrl.device
    gP = torch.empty((int(batch.path_n.sum()), 3), dtype=torch.float64, device=dev)
    gQ = torch.empty((int(batch.prof_n.sum()), 3), dtype=torch.float64, device=dev)
    if workspace is None or _nbytes(workspace) < ws_bytes:
        workspace = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    extra, pg = {}, None
    if params:
        pg = L.SweepParamGrads()
        sizes = {"path_knots": None if batch.path_knots is None else batch.path_knots.shape[0],
                 "prof_knots": None if batch.prof_knots is None else batch.prof_knots.shape[0],
                 "path_weights": None if batch.path_weights is None else batch.path_weights.numel(),
                 "prof_weights": None if batch.prof_weights is None else batch.prof_weights.numel()}
        for name in params:
            if name not in _PARAM_GRADS:
                raise ValueError(f"unknown parameter gradient {name!r}")
            if not sizes[name]:
                raise ValueError(f"{name} gradients need the batch's {name}")
            extra[name] = torch.zeros(sizes[name], dtype=torch.float64, device=dev)
            setattr(pg, name, extra[name].data_ptr())
    L.check(L.sweep_backward_ex(b, opt, g.data_ptr() if g is not None else 0, gn.data_ptr() if gn is not None else 0,
                                gP.data_ptr(), gQ.data_ptr(), pg, workspace.data_ptr(), _nbytes(workspace),
                                _stream_handle(stream)))
    return (gP, gQ, extra) if params else (gP, gQ)


def backward_workspace_size(batch: Batch, out_dtype=torch.float32) -> int:
    return L.sweep_backward_workspace_size(batch.c_struct(), make_options(out_dtype, torch.float64))
