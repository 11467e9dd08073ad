"""Gradients through the normals (next-row f3): sweep_backward_ex with
g = dL/dN against the oracle's FP64 finite differences of
L = sum w . X + sum g . N, on sweeps of path degrees 1-7, profiles off their
plane (S_z != 0, so that the frame's rate of turn enters X_u), rational path
and profile, FP64 and FP32 gradients; the translation and joint-scaling
invariants of the normal term on the full 256-sweep differentiation
workload; and torch.autograd.gradcheck through the normals output.

The reference gradient is Richardson-extrapolated central differences,
(4 D(h/2) - D(h)) / 3 with h = 2e-6: the normal term has large third
derivatives where a profile bends sharply, and plain central differences at
h = 1e-6 were off by up to 4e-6 (relative) there, shrinking as h^2."""

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


def _fd(s, w, g, h=2e-6):
    a = oracle.fd_grad(s.path, s.profile, s.n_u, s.n_v, w, g=g, h=h)
    b = oracle.fd_grad(s.path, s.profile, s.n_u, s.n_v, w, g=g, h=h / 2)
    return tuple((4 * y - x) / 3 for x, y in zip(a, b))


def _specs(seed=21, rational=False):
    rng = np.random.default_rng(seed)
    specs = []
    for k, (p, q, n_u, n_v) in enumerate([(3, 3, 300, 40), (2, 3, 257, 13), (3, 2, 64, 64), (5, 4, 200, 70),
                                          (1, 3, 90, 20), (7, 1, 120, 9)]):
        P = synth.random_walk(rng, max(p + 1, 14))
        Q = synth.perturbed_circle(rng, max(q + 1, 9))
        Q[:, 2] = 0.1 * rng.standard_normal(Q.shape[0])
        path, prof = synth.CurveSpec(P, p), synth.CurveSpec(Q, q, True)
        if rational:
            path.weights = rng.uniform(0.5, 2.0, P.shape[0])
            prof.weights = rng.uniform(0.5, 2.0, Q.shape[0])
        specs.append(synth.SweepSpec(path, prof, n_u, n_v))
    return specs


def _check(specs, out_dtype, tol, with_pos, seed=56):
    b = api.Batch.from_specs(specs)
    rng = np.random.default_rng(seed)
    gs = [rng.standard_normal((3, s.n_u, s.n_v)) for s in specs]
    ws = synth.loss_weights(specs, seed + 1) if with_pos else None
    if out_dtype == torch.float32:
        # the GPU reads the weights rounded to FP32; give the oracle the same
        gs = [x.astype(np.float32).astype(np.float64) for x in gs]
        if ws is not None:
            ws = [x.astype(np.float32).astype(np.float64) for x in ws]
    gP, gQ = api.sweep_backward(b, b.pack(ws, out_dtype) if with_pos else None, grad_nrm=b.pack(gs, out_dtype))
    torch.cuda.synchronize()
    gP, gQ = gP.cpu().numpy(), gQ.cpu().numpy()
    worst = 0.0
    for k, s in enumerate(specs):
        fP, fQ = _fd(s, ws[k] if with_pos else None, gs[k])
        eP, eQ = _rel(gP[b.path_slice(k)], fP), _rel(gQ[b.prof_slice(k)], fQ)
        say(f"   sweep {k} ({s.n_u}x{s.n_v} p={s.path.degree} q={s.profile.degree}): path rel {eP:.2e} prof rel {eQ:.2e}")
        worst = max(worst, eP, eQ)
    assert worst <= tol, worst
    return worst


@pytest.mark.parametrize("with_pos", [False, True])
def test_normal_adjoint_fp64_against_fd(with_pos):
    say(f"[case] normal adjoint FP64 vs FD, positions too: {with_pos}")
    _check(_specs(), torch.float64, 1e-6, with_pos)


def test_normal_adjoint_rational_against_fd():
    say("[case] normal adjoint, rational path and profile, FP64 vs FD")
    _check(_specs(22, rational=True), torch.float64, 1e-6, True)


def test_normal_adjoint_fp32_against_fd():
    say("[case] normal adjoint FP32 vs FD")
    _check(_specs(23), torch.float32, 1e-5, True)


def test_normal_adjoint_invariants_on_the_differentiation_workload():
    # Translating a sweep (its path control points) or scaling path and
    # profile together about the origin leaves every normal unchanged, so the
    # normal term's gradient satisfies sum_k dL/dP_k = 0 and
    # sum_k P_k . dL/dP_k + sum_l Q_l . dL/dQ_l = 0 for every sweep.
    specs = synth.c5()
    rng = np.random.default_rng(57)
    for s in specs[::16]:
        s.profile.ctrl[:, 2] = 0.05 * rng.standard_normal(s.profile.ctrl.shape[0])
    b = api.Batch.from_specs(specs)
    say(f"[case] normal-term invariants, {len(specs)} sweeps 1024x64")
    gs = [rng.standard_normal((3, s.n_u, s.n_v)) for s in specs]
    gP, gQ = api.sweep_backward(b, None, grad_nrm=b.pack(gs, torch.float32))
    torch.cuda.synchronize()
    gP, gQ = gP.cpu().numpy(), gQ.cpu().numpy()
    worst_t = worst_s = 0.0
    for k, s in enumerate(specs):
        p, q = gP[b.path_slice(k)], gQ[b.prof_slice(k)]
        scale = max(np.abs(p).max(), np.abs(q).max())
        assert scale > 0
        worst_t = max(worst_t, np.abs(p.sum(axis=0)).max() / (scale * p.shape[0]))
        mix = np.sum(s.path.ctrl * p) + np.sum(s.profile.ctrl * q)
        worst_s = max(worst_s, abs(mix) / (scale * (np.abs(s.path.ctrl).sum() + np.abs(s.profile.ctrl).sum())))
    say(f"   translation {worst_t:.2e}, scaling {worst_s:.2e}")
    assert worst_t <= 1e-10 and worst_s <= 1e-10


def test_autograd_through_normals_and_gradcheck():
    rng = np.random.default_rng(4)
    P = synth.random_walk(rng, 7)
    Q = synth.perturbed_circle(rng, 6)
    Q[:, 2] = 0.1 * rng.standard_normal(6)
    spec = synth.SweepSpec(synth.CurveSpec(P, 3), synth.CurveSpec(Q, 3, True), 24, 8)
    b = api.Batch.from_specs([spec])
    Pt = torch.as_tensor(P).cuda().requires_grad_(True)
    Qt = torch.as_tensor(Q).cuda().requires_grad_(True)
    gn = torch.randn(b.out_elems, dtype=torch.float64, device="cuda")
    pos, nrm = dsweep(Pt, Qt, b, out_dtype=torch.float64)
    assert nrm.requires_grad
    (nrm * gn).sum().backward()
    assert Pt.grad is not None and Qt.grad is not None
    f = lambda a, c: dsweep(a, c, b, out_dtype=torch.float64)[1]
    assert torch.autograd.gradcheck(f, (Pt.detach().requires_grad_(True), Qt.detach().requires_grad_(True)),
                                    eps=1e-6, atol=1e-5, rtol=1e-4, nondet_tol=0.0)
    both = lambda a, c: sum(t.sum() for t in dsweep(a, c, b, out_dtype=torch.float64))
    assert torch.autograd.gradcheck(both, (Pt.detach().requires_grad_(True), Qt.detach().requires_grad_(True)),
                                    eps=1e-6, atol=1e-5, rtol=1e-4, nondet_tol=0.0)
