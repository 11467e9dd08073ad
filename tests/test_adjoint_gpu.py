"""The adjoint kernels against the oracle's FP64 central finite differences
(h = 1e-6) of L = sum w . X, and torch.autograd.gradcheck on a tiny FP64
sweep."""

import numpy as np
import pytest
import torch

import oracle
import synth
from paper_1110_5450_amd import api
from paper_1110_5450_amd.autograd import sweep as dsweep
from tests.gpu_util import say

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _check(specs, out_dtype, tol, seed=55):
    b = api.Batch.from_specs(specs)
    ws = synth.loss_weights(specs, seed)
    g = b.pack(ws, out_dtype)
    gP, gQ = api.sweep_backward(b, g)
    torch.cuda.synchronize()
    gP, gQ = gP.cpu().numpy(), gQ.cpu().numpy()
    worst = 0.0
    for k, s in enumerate(specs):
        fP, fQ = oracle.fd_grad(s.path, s.profile, s.n_u, s.n_v, ws[k])
        eP, eQ = _rel(gP[b.path_slice(k)], fP), _rel(gQ[b.prof_slice(k)], fQ)
        say(f"   sweep {k} ({s.n_u}x{s.n_v} p={s.path.degree} q={s.profile.degree}): path rel {eP:.2e} prof rel {eQ:.2e}")
        worst = max(worst, eP, eQ)
    assert worst <= tol, worst
    return worst


def test_adjoint_fp64_against_fd():
    rng = np.random.default_rng(12)
    specs = []
    for k, (p, q, n_u, n_v) in enumerate([(3, 3, 300, 40), (2, 3, 257, 13), (3, 2, 64, 64), (5, 4, 700, 70),
                                          (1, 3, 90, 20), (7, 1, 120, 9)]):
        P = synth.random_walk(rng, max(p + 1, 14))
        Q = synth.perturbed_circle(rng, max(q + 1, 9))
        if k == 3:
            Q[:, 2] = 0.1 * rng.standard_normal(Q.shape[0])
        specs.append(synth.SweepSpec(synth.CurveSpec(P, p), synth.CurveSpec(Q, q, True), n_u, n_v))
    say("[case] adjoint FP64 vs FD")
    _check(specs, torch.float64, 1e-7)


def test_adjoint_fp32_differentiation_workload_sampled():
    specs = synth.c5()
    say(f"[case] adjoint FP32, {len(specs)} sweeps 1024x64 (FD on 3 sweeps)")
    b = api.Batch.from_specs(specs)
    ws = synth.loss_weights(specs, 55)
    g = b.pack(ws, torch.float32)
    gP, gQ = api.sweep_backward(b, g)
    torch.cuda.synchronize()
    gP, gQ = gP.cpu().numpy(), gQ.cpu().numpy()
    for k in (0, 131, 255):
        s = specs[k]
        # the GPU read w rounded to FP32; give the oracle the same weights
        w32 = ws[k].astype(np.float32).astype(np.float64)
        fP, fQ = oracle.fd_grad(s.path, s.profile, s.n_u, s.n_v, w32)
        eP, eQ = _rel(gP[b.path_slice(k)], fP), _rel(gQ[b.prof_slice(k)], fQ)
        say(f"   sweep {k}: path rel {eP:.2e} prof rel {eQ:.2e}")
        assert eP <= 1e-4 and eQ <= 1e-4


def test_autograd_function_and_gradcheck():
    rng = np.random.default_rng(3)
    P = synth.random_walk(rng, 7)
    Q = synth.perturbed_circle(rng, 6)
    spec = synth.SweepSpec(synth.CurveSpec(P, 3), synth.CurveSpec(Q, 3, True), 24, 8)
    b = api.Batch.from_specs([spec])
    Pt = torch.as_tensor(P).cuda().requires_grad_(True)
    Qt = torch.as_tensor(Q).cuda().requires_grad_(True)
    w = torch.randn(b.out_elems, dtype=torch.float64, device="cuda")
    pos, nrm = dsweep(Pt, Qt, b, out_dtype=torch.float64)
    (pos * w).sum().backward()
    assert Pt.grad is not None and Qt.grad is not None
    f = lambda a, c: dsweep(a, c, b, out_dtype=torch.float64)[0]
    assert torch.autograd.gradcheck(f, (Pt.detach().requires_grad_(True), Qt.detach().requires_grad_(True)),
                                    eps=1e-6, atol=1e-6, rtol=1e-5, nondet_tol=0.0)
    # normals are differentiable too (their gradients: test_adjoint_normals_gpu)
    pos, nrm = dsweep(Pt, Qt, b, out_dtype=torch.float64)
    assert nrm.requires_grad


def test_two_forwards_on_one_batch_keep_their_own_control_points():
    """One Batch, two differentiable calls with different control points and
    one summed loss: each call's gradient is its own (against the oracle's
    finite differences), the Batch itself is left unchanged, and an in-place
    change of a control-point tensor before backward raises."""
    rng = np.random.default_rng(31)
    P1, P2 = synth.random_walk(rng, 8), synth.random_walk(rng, 8)
    Q1, Q2 = synth.perturbed_circle(rng, 6), synth.perturbed_circle(rng, 6)
    spec = synth.SweepSpec(synth.CurveSpec(P1, 3), synth.CurveSpec(Q1, 3, True), 40, 12)
    b = api.Batch.from_specs([spec])
    own_P, own_Q = b.path_ctrl.clone(), b.prof_ctrl.clone()
    t = [torch.as_tensor(a).cuda().requires_grad_(True) for a in (P1, Q1, P2, Q2)]
    w1, w2 = (rng.standard_normal((3, 40, 12)) for _ in range(2))
    pos1, _ = dsweep(t[0], t[1], b, out_dtype=torch.float64)
    pos2, _ = dsweep(t[2], t[3], b, out_dtype=torch.float64)
    loss = (pos1 * b.pack([w1], torch.float64)).sum() + (pos2 * b.pack([w2], torch.float64)).sum()
    loss.backward()
    assert torch.equal(b.path_ctrl, own_P) and torch.equal(b.prof_ctrl, own_Q)
    for (P, Q, w), gp, gq in (((P1, Q1, w1), t[0].grad, t[1].grad), ((P2, Q2, w2), t[2].grad, t[3].grad)):
        s = synth.SweepSpec(synth.CurveSpec(P, 3), synth.CurveSpec(Q, 3, True), 40, 12)
        fP, fQ = oracle.fd_grad(s.path, s.profile, 40, 12, w)
        eP, eQ = _rel(gp.cpu().numpy(), fP), _rel(gq.cpu().numpy(), fQ)
        say(f"    own gradient: path rel {eP:.2e} prof rel {eQ:.2e}")
        assert eP <= 1e-7 and eQ <= 1e-7
    Pt = torch.as_tensor(P1).cuda().requires_grad_(True)
    leaf = Pt * 1.0
    pos, _ = dsweep(leaf, t[1].detach(), b, out_dtype=torch.float64)
    with torch.no_grad():
        leaf.add_(1.0)
    with pytest.raises(RuntimeError, match="modified by an inplace operation"):
        pos.sum().backward()
