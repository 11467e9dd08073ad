"""Helpers for the GPU tests: run the HIP path through the C ABI on seeded
inputs and measure it against the oracle with the parity rule:

* positions: max |dX| / (bounding-box diagonal of the oracle's X)
  <= 1e-12 (FP64 output) or 1e-5 (FP32 output);
* normals: |dN| <= tau * max(1, kappa) with the same tau, on vertices whose
  condition number kappa (the oracle's) is at most 1e6; the rest are masked
  and counted.
"""

from __future__ import annotations

import sys

import numpy as np
import torch

import oracle
from paper_1110_5450_amd import api

TOL = {torch.float64: 1e-12, torch.float32: 1e-5}
KAPPA_MAX = 1e6


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev_ctrl(a) -> torch.Tensor:
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _dev_w(w):
    return None if w is None else dev_ctrl(w)


def gpu_sweep(spec, out_dtype=torch.float32, frame_dtype=torch.float64, **kw):
    p, q = spec.path, spec.profile
    return api.sweep_eval(dev_ctrl(p.ctrl), p.degree, dev_ctrl(q.ctrl), q.degree, spec.n_u, spec.n_v,
                          prof_closed=q.closed, path_knots=p.knots, prof_knots=q.knots,
                          path_weights=_dev_w(getattr(p, "weights", None)),
                          prof_weights=_dev_w(getattr(q, "weights", None)),
                          out_dtype=out_dtype, frame_dtype=frame_dtype, **kw)


def parity(pos_ref, nrm_ref, kap_ref, pos, nrm, tol, diag=None):
    diag = oracle.bbox_diag(pos_ref) if diag is None else diag
    r = oracle.compare(pos_ref, nrm_ref, kap_ref, pos, nrm, diag, KAPPA_MAX)
    r["diag"] = diag
    ok = r["pos_rel"] <= tol and (nrm is None or r["nrm_scaled"] <= tol)
    return ok, r


def check_full(spec, out_dtype=torch.float32, frame_dtype=torch.float64, tol=None, n0=None, reorth=True, **kw):
    """Whole-grid parity of one sweep; returns the figures."""
    say(f"[case] n_u={spec.n_u} n_v={spec.n_v} p={spec.path.degree} q={spec.profile.degree} "
        f"out={out_dtype} frame={frame_dtype} kw={kw}")
    ref = oracle.sweep(spec.path, spec.profile, spec.n_u, spec.n_v, n0=n0)
    pos, nrm = gpu_sweep(spec, out_dtype, frame_dtype, initial_normal=n0, reorthonormalize=reorth, **kw)
    torch.cuda.synchronize()
    tol = TOL[out_dtype] if tol is None else tol
    ok, r = parity(ref.pos, ref.nrm, ref.kappa, pos.cpu().numpy(), nrm.cpu().numpy(), tol)
    say("   ", r)
    assert ok, r
    return r
