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


def _knots_ptr(knots) -> Tuple[Optional[np.ndarray], Optional[C.POINTER(C.c_double)]]:
    if knots is None:
        return None, None
    a = np.ascontiguousarray(np.asarray(knots, dtype=np.float64))
    return a, a.ctypes.data_as(C.POINTER(C.c_double))


def make_options(out_dtype=torch.float32, frame_dtype=torch.float64, reorthonormalize: bool = True,
                 initial_normal=None, tile_config: int = -1) -> L.SweepOptions:
    o = L.default_options()
    o.out_precision = _DT[out_dtype]
    o.frame_precision = _DT[frame_dtype]
    o.reorthonormalize = int(bool(reorthonormalize))
    if initial_normal is not None:
        o.has_initial_normal = 1
        for k in range(3):
            o.initial_normal[k] = float(initial_normal[k])
    o.tile_config = int(tile_config)
    return o


def _stream_handle(stream) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def sweep_eval(path_ctrl: torch.Tensor, path_degree: int, prof_ctrl: torch.Tensor, prof_degree: int,
               n_u: int, n_v: int, *, prof_closed: bool = True, path_knots=None, prof_knots=None,
               out_dtype=torch.float32, frame_dtype=torch.float64, reorthonormalize: bool = True,
               initial_normal=None, tile_config: int = -1, normals: bool = True,
               out: Optional[Tuple[torch.Tensor, Optional[torch.Tensor]]] = None,
               workspace: Optional[torch.Tensor] = None, stream=None):
    """Positions (3, n_u, n_v) and normals (or None) of one sweep."""
    pc = _check_ctrl(path_ctrl, "path_ctrl")
    qc = _check_ctrl(prof_ctrl, "prof_ctrl")
    pk, pkp = _knots_ptr(path_knots)
    qk, qkp = _knots_ptr(prof_knots)
    path = L.SweepCurve(pc.shape[0], int(path_degree), 0, 0, pc.data_ptr(), pkp)
    prof = L.SweepCurve(qc.shape[0], int(prof_degree), int(bool(prof_closed)), 0, qc.data_ptr(), qkp)
    opt = make_options(out_dtype, frame_dtype, reorthonormalize, initial_normal, tile_config)
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
    if workspace is None or workspace.numel() < ws_bytes:
        workspace = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    st = L.sweep_eval(path, prof, int(n_u), int(n_v), opt, pos.data_ptr(),
                      nrm.data_ptr() if nrm is not None else 0, workspace.data_ptr(), workspace.numel(),
                      _stream_handle(stream))
    L.check(st)
    return pos, nrm


def eval_workspace_size(n_path: int, path_degree: int, n_prof: int, prof_degree: int, n_u: int, n_v: int, *,
                        prof_closed: bool = True, out_dtype=torch.float32, frame_dtype=torch.float64) -> int:
    path = L.SweepCurve(n_path, path_degree, 0, 0, 1, None)
    prof = L.SweepCurve(n_prof, prof_degree, int(prof_closed), 0, 1, None)
    return L.sweep_eval_workspace_size(path, prof, n_u, n_v, make_options(out_dtype, frame_dtype))
