"""sweep_eval_noalloc (workspace in the library's static device array)
against sweep_eval (caller workspace) through the C ABI: two calls in a row
on the same GPU, the second with a smaller sweep, each compared with
sweep_eval's output on the same input (same kernels and arithmetic, so the
outputs agree bitwise), and with the oracle under the FP32 / FP64 parity
rule.  Also: a sweep too large for the static array is rejected before
anything is enqueued."""

from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
import synth
from paper_1110_5450_amd import _lib as L
from paper_1110_5450_amd import api
from tests.gpu_util import TOL, parity, say

pytestmark = pytest.mark.gpu


def _curves(spec):
    p, q = spec.path, spec.profile
    pc = torch.as_tensor(np.ascontiguousarray(p.ctrl, dtype=np.float64)).cuda()
    qc = torch.as_tensor(np.ascontiguousarray(q.ctrl, dtype=np.float64)).cuda()
    path = L.SweepCurve(pc.shape[0], p.degree, 0, 0, pc.data_ptr(), None, None)
    prof = L.SweepCurve(qc.shape[0], q.degree, int(q.closed), 0, qc.data_ptr(), None, None)
    return pc, qc, path, prof


def _run_both(spec, out_dtype):
    pc, qc, path, prof = _curves(spec)
    opt = api.make_options(out_dtype)
    n = 3 * spec.n_u * spec.n_v
    need = L.sweep_eval_workspace_size(path, prof, spec.n_u, spec.n_v, opt)
    assert 0 < need <= 64 << 20
    say(f"[case] noalloc n_u={spec.n_u} n_v={spec.n_v} out={out_dtype} workspace={need} B")
    # static-array call first, into buffers filled with NaN
    pos_s = torch.full((n,), float("nan"), dtype=out_dtype, device="cuda")
    nrm_s = torch.full((n,), float("nan"), dtype=out_dtype, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    L.check(L.sweep_eval_noalloc(path, prof, spec.n_u, spec.n_v, opt, pos_s.data_ptr(), nrm_s.data_ptr(), stream))
    # the caller-workspace call
    pos_w = torch.full((n,), float("nan"), dtype=out_dtype, device="cuda")
    nrm_w = torch.full((n,), float("nan"), dtype=out_dtype, device="cuda")
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    L.check(L.sweep_eval(path, prof, spec.n_u, spec.n_v, opt, pos_w.data_ptr(), nrm_w.data_ptr(), ws.data_ptr(),
                         need, stream))
    torch.cuda.synchronize()
    shape = (3, spec.n_u, spec.n_v)
    return pos_s.view(shape), nrm_s.view(shape), pos_w.view(shape), nrm_w.view(shape)


def test_noalloc_matches_sweep_eval_two_calls_second_smaller():
    big = synth.c2(n_u=4096, n_v=1024)      # 4.2 M vertices, FP32
    small = synth.c1()                      # 256 x 64, FP64 out
    for spec, dt in ((big, torch.float32), (small, torch.float64)):
        ps, ns, pw, nw = _run_both(spec, dt)
        assert torch.isfinite(ps).all() and torch.isfinite(ns).all()
        assert torch.equal(ps, pw) and torch.equal(ns, nw), "noalloc output differs from sweep_eval's"
        ref = oracle.sweep(spec.path, spec.profile, spec.n_u, spec.n_v)
        ok, r = parity(ref.pos, ref.nrm, ref.kappa, ps.double().cpu().numpy(), ns.double().cpu().numpy(), TOL[dt])
        say("   ", r)
        assert ok, r


def test_noalloc_rejects_a_sweep_beyond_the_static_array():
    spec = synth.c3()
    pc, qc, path, prof = _curves(spec)
    opt = api.make_options(torch.float32)
    need = L.sweep_eval_workspace_size(path, prof, spec.n_u, spec.n_v, opt)
    assert need > 64 << 20
    say(f"[case] noalloc rejects n_u={spec.n_u}: workspace {need} B")
    st = L.sweep_eval_noalloc(path, prof, spec.n_u, spec.n_v, opt, 0, 0, 0)
    assert L.STATUS[st] == "SWEEP_ERR_WORKSPACE", (st, L.last_error())
    assert "static array" in L.last_error()
