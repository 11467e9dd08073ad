"""Rational (NURBS) path and profile curves on the GPU: parity with the
oracle for random weights (single sweep, batch, frames, adjoint), and the
closed forms that rational curves make exact end-to-end on the device --
a cylinder and a torus built from 9-point NURBS circles."""

from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
import synth
from paper_1110_5450_amd import api
from tests.gpu_util import TOL, check_full, dev_ctrl, gpu_sweep, parity, say
from tests.test_oracle_rational import nurbs_circle

pytestmark = pytest.mark.gpu


def _rational_spec(seed, n_path=12, n_prof=9, p=3, q=3, n_u=700, n_v=100, closed=True):
    rng = np.random.default_rng(seed)
    P = synth.random_walk(rng, n_path)
    Q = synth.perturbed_circle(rng, n_prof)
    wp = rng.uniform(0.4, 2.5, n_path)
    wq = rng.uniform(0.4, 2.5, n_prof)
    return synth.SweepSpec(synth.CurveSpec(P, p, weights=wp), synth.CurveSpec(Q, q, closed, weights=wq), n_u, n_v)


@pytest.mark.parametrize("out_dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("p,q", [(3, 3), (2, 2), (5, 1)])
def test_rational_sweep_matches_oracle(out_dtype, p, q):
    spec = _rational_spec(10 + p, p=p, q=q, n_path=max(p + 1, 12))
    check_full(spec, out_dtype)


def test_rational_open_profile_with_knots_and_initial_normal():
    rng = np.random.default_rng(77)
    spec = _rational_spec(21, closed=False)
    spec.profile.knots = np.concatenate([np.zeros(4), np.sort(rng.uniform(0, 1, 5)), np.ones(4)])
    check_full(spec, torch.float64, n0=np.array([0.2, -1.0, 0.3]))


def test_exact_torus_on_the_gpu():
    R, rho = 2.0, 0.5
    pc, pw, pU = nurbs_circle(R)
    qc, qw, qU = nurbs_circle(rho)
    spec = synth.SweepSpec(synth.CurveSpec(pc, 2, False, pU, pw), synth.CurveSpec(qc, 2, False, qU, qw), 513, 257)
    say("[case] exact torus, 513 x 257, FP64")
    pos, nrm = gpu_sweep(spec, torch.float64, initial_normal=np.array([0.0, 0.0, 1.0]))
    torch.cuda.synchronize()
    X, N = pos.cpu().numpy(), nrm.cpu().numpy()
    dxy = np.hypot(X[0], X[1])
    dist = np.hypot(dxy - R, X[2])
    say("   max |dist - rho| =", np.abs(dist - rho).max())
    assert np.abs(dist - rho).max() <= 1e-14 * R
    cp = np.stack([R * X[0] / dxy, R * X[1] / dxy, np.zeros_like(dxy)])
    dots = (N * (X - cp) / rho).sum(0)
    assert np.abs(np.abs(dots) - 1).max() <= 1e-12
    assert np.all(np.sign(dots) == np.sign(dots.flat[0]))


def test_exact_cylinder_on_the_gpu_fp32():
    rho = 0.4
    qc, qw, qU = nurbs_circle(rho)
    path = synth.CurveSpec(np.array([[0, 0, -1.0], [0, 0, 0.0], [0, 0, 1.5], [0, 0, 3.0]]), 3)
    spec = synth.SweepSpec(path, synth.CurveSpec(qc, 2, False, qU, qw), 1000, 1024)
    say("[case] exact cylinder, 1000 x 1024, FP32 out")
    pos, nrm = gpu_sweep(spec, torch.float32)
    torch.cuda.synchronize()
    X = pos.double().cpu().numpy()
    d = np.hypot(X[0], X[1])
    # FP32 output: the radius to a few ulps of the coordinates
    assert np.abs(d - rho).max() <= 4 * np.finfo(np.float32).eps * 3.0


def test_rational_frames_match_oracle():
    spec = _rational_spec(31, n_u=5000)
    p = spec.path
    say("[case] rational frames n_u=5000")
    rows = api.sweep_frames(dev_ctrl(p.ctrl), p.degree, spec.n_u, path_weights=dev_ctrl(p.weights)).cpu().numpy()
    x, d1, d2, ft = oracle.path_samples(p, spec.n_u)
    R, _ = oracle.frame(x, d1, ft)
    eps = np.finfo(float).eps
    dx = np.abs(rows[:, 0:3] - x).max() / max(1.0, np.abs(x).max())
    dR = max(np.abs(rows[:, 3 + 3 * c: 6 + 3 * c] - R[:, :, c]).max() for c in range(3))
    say(f"    x {dx:.2e}  frame {dR:.2e}")
    assert dx <= 1e-14 and dR <= 8 * spec.n_u * eps


def test_rational_batch_matches_oracle_and_single():
    specs = [_rational_spec(40 + k, n_u=int(n_u), n_v=int(n_v), p=int(p))
             for k, (n_u, n_v, p) in enumerate([(200, 40, 3), (999, 17, 2), (64, 256, 3), (1500, 9, 4)])]
    b = api.Batch.from_specs(specs)
    assert b.path_weights is not None and b.prof_weights is not None
    pos, nrm = api.sweep_eval_batched(b, out_dtype=torch.float64)
    torch.cuda.synchronize()
    for k, s in enumerate(specs):
        ref = oracle.sweep(s.path, s.profile, s.n_u, s.n_v)
        ok, r = parity(ref.pos, ref.nrm, ref.kappa, b.view(pos, k).cpu().numpy(), b.view(nrm, k).cpu().numpy(),
                       TOL[torch.float64])
        say(f"   sweep {k}: {r}")
        assert ok, (k, r)
        # the single-sweep evaluation agrees to rounding (the batched frame
        # kernels group the samples into runs differently)
        p1, n1 = gpu_sweep(s, torch.float64, tile_config=13)
        torch.cuda.synchronize()
        ok, r = parity(p1.cpu().numpy(), n1.cpu().numpy(), ref.kappa, b.view(pos, k).cpu().numpy(),
                       b.view(nrm, k).cpu().numpy(), 1e-13)
        assert ok, (k, r)


def test_rational_adjoint_against_fd():
    specs = [_rational_spec(60, n_u=300, n_v=30), _rational_spec(61, p=2, q=2, n_u=257, n_v=13, closed=False)]
    b = api.Batch.from_specs(specs)
    ws = synth.loss_weights(specs, 66)
    gP, gQ = api.sweep_backward(b, b.pack(ws, torch.float64))
    torch.cuda.synchronize()
    gP, gQ = gP.cpu().numpy(), gQ.cpu().numpy()
    for k, s in enumerate(specs):
        fP, fQ = oracle.fd_grad(s.path, s.profile, s.n_u, s.n_v, ws[k])
        eP = np.linalg.norm(gP[b.path_slice(k)] - fP) / np.linalg.norm(fP)
        eQ = np.linalg.norm(gQ[b.prof_slice(k)] - fQ) / np.linalg.norm(fQ)
        say(f"   sweep {k}: path rel {eP:.2e} prof rel {eQ:.2e}")
        assert eP <= 1e-7 and eQ <= 1e-7
