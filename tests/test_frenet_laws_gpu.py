"""Frame modes and sweep laws on the GPU (next-row f2): parity with the
oracle's Frenet frame and scale/twist laws, single sweeps and batches, and
the closed forms they produce (a cone, a twisted offset tube, an elliptic
torus), computed on the device end to end."""

from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
import synth
from paper_1110_5450_amd import _lib, api
from tests.gpu_util import TOL, dev_ctrl, gpu_sweep, parity, say
from tests.test_oracle_rational import nurbs_circle

pytestmark = pytest.mark.gpu


def _law(seed, n=6, p=3):
    rng = np.random.default_rng(seed)
    ctrl = np.zeros((n, 3))
    ctrl[:, 0] = rng.uniform(0.6, 1.6, n)           # scale
    ctrl[:, 1] = np.cumsum(rng.uniform(-1.0, 1.0, n))  # twist angle
    return synth.CurveSpec(ctrl, p)


def _check(spec, out_dtype, mode="rmf", law=None, tol=None, n0=None):
    say(f"[case] {mode} law={law is not None} n_u={spec.n_u} n_v={spec.n_v} p={spec.path.degree} out={out_dtype}")
    ref, _ = oracle.sweep_ex(spec.path, spec.profile, spec.n_u, spec.n_v, n0=n0, mode=mode, law=law)
    glaw = None if law is None else api.Law(dev_ctrl(law.ctrl), law.degree, law.knots)
    pos, nrm = gpu_sweep(spec, out_dtype, frame_mode=mode, law=glaw, initial_normal=n0)
    torch.cuda.synchronize()
    ok, r = parity(ref.pos, ref.nrm, ref.kappa, pos.cpu().numpy(), nrm.cpu().numpy(),
                   TOL[out_dtype] if tol is None else tol)
    say("   ", r)
    assert ok, r
    return r


@pytest.mark.parametrize("out_dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("p", [3, 2, 5])
def test_frenet_mode_matches_oracle(out_dtype, p):
    spec = synth.single(90 + p, 14, 9, 1500, 96, p_path=p)
    _check(spec, out_dtype, mode="frenet")


@pytest.mark.parametrize("mode", ["rmf", "frenet"])
@pytest.mark.parametrize("out_dtype", [torch.float64, torch.float32])
def test_laws_match_oracle(mode, out_dtype):
    spec = synth.single(95, 12, 9, 700, 128)
    _check(spec, out_dtype, mode=mode, law=_law(7))


def test_law_with_knots_and_rational_path():
    spec = synth.single(96, 10, 8, 513, 64)
    rng = np.random.default_rng(3)
    spec.path.weights = rng.uniform(0.5, 2.0, spec.path.n)
    law = _law(8, n=7, p=2)
    law.knots = np.concatenate([np.zeros(3), np.sort(rng.uniform(0, 1, 4)), np.ones(3)]) * 2.0 + 0.5
    _check(spec, torch.float64, mode="frenet", law=law, n0=np.array([0.0, 1.0, 0.0]))


def _straight_path(H=2.0):
    return synth.CurveSpec(np.array([[0.0, 0.0, 0.0], [0.0, 0.0, H]]), 1)


def test_cone_from_a_scale_law_on_the_gpu():
    rho, H = 0.4, 2.0
    qc, qw, qU = nurbs_circle(rho)
    spec = synth.SweepSpec(_straight_path(H), synth.CurveSpec(qc, 2, False, qU, qw), 257, 129)
    law = api.Law(dev_ctrl([[1.0, 0.0, 0.0], [2.0, 0.0, 0.0]]), 1)
    pos, nrm = gpu_sweep(spec, torch.float64, law=law)
    torch.cuda.synchronize()
    X, N = pos.cpu().numpy(), nrm.cpu().numpy()
    u = np.linspace(0, 1, spec.n_u)
    assert np.abs(np.hypot(X[0], X[1]) - rho * (1 + u)[:, None]).max() <= 1e-15
    phi = np.arctan2(X[1], X[0])
    nr = np.stack([H * np.cos(phi), H * np.sin(phi), -rho * np.ones_like(phi)])
    nr /= np.linalg.norm(nr, axis=0)
    dots = (N * nr).sum(0)
    assert np.abs(np.abs(dots) - 1).max() <= 1e-13
    assert np.all(np.sign(dots) == np.sign(dots.flat[0]))


def test_twisted_offset_tube_on_the_gpu():
    rho, d, H, Th = 0.2, 0.6, 2.0, 3.0
    qc, qw, qU = nurbs_circle(rho)
    spec = synth.SweepSpec(_straight_path(H), synth.CurveSpec(qc + [d, 0, 0], 2, False, qU, qw), 129, 65)
    law = api.Law(dev_ctrl([[1.0, 0.0, 0.0], [1.0, Th, 0.0]]), 1)
    pos, nrm = gpu_sweep(spec, torch.float64, law=law)
    torch.cuda.synchronize()
    X = pos.cpu().numpy()
    u = np.linspace(0, 1, spec.n_u)[:, None]
    # each row is the offset circle turned by Th u: its centre is at
    # distance d from the axis at angle Th u
    cx, cy = d * np.cos(Th * u), d * np.sin(Th * u)
    assert np.abs(np.hypot(X[0] - cx, X[1] - cy) - rho).max() <= 1e-15
    assert np.abs(X[2] - H * u).max() <= 1e-15


def test_elliptic_torus_frenet_on_the_gpu_fp32():
    R, a, b = 2.0, 0.5, 0.2
    pc, pw, pU = nurbs_circle(R)
    ang = np.linspace(0, 2 * np.pi, 48, endpoint=False)
    prof = synth.CurveSpec(np.stack([a * np.cos(ang), b * np.sin(ang), np.zeros(48)], 1), 3, True)
    spec = synth.SweepSpec(synth.CurveSpec(pc, 2, False, pU, pw), prof, 1025, 256)
    pos, nrm = gpu_sweep(spec, torch.float32, frame_mode="frenet")
    torch.cuda.synchronize()
    X, N = pos.double().cpu().numpy(), nrm.double().cpu().numpy()
    S, _ = oracle.profile_samples(prof, spec.n_v)
    e32 = np.finfo(np.float32).eps
    assert np.abs(np.hypot(X[0], X[1]) - (R - S[None, :, 0])).max() <= 8 * e32 * R
    assert np.abs(X[2] - S[None, :, 1]).max() <= 8 * e32 * R
    radial = np.stack([X[0], X[1]]) / np.hypot(X[0], X[1])
    assert np.abs(N[0] * (-radial[1]) + N[1] * radial[0]).max() <= 1e-5


@pytest.mark.parametrize("mode,with_law", [("frenet", False), ("rmf", True), ("frenet", True)])
@pytest.mark.parametrize("out_dtype", [torch.float64, torch.float32])
def test_batched_frame_modes_and_laws_match_oracle(mode, with_law, out_dtype):
    """A batch with the Frenet frame and/or one sweep law for every sweep:
    sweeps framed by one wave (<= 256 u-samples), by one block (path in LDS)
    and by the chunk-walking kernel (> 4096), path degrees 1-5, one rational
    path; each against the oracle's sweep with the same mode and law (the
    law's knots given).  The scan bound 8 n eps applies to the long
    rotation-minimizing sweeps."""
    rng = np.random.default_rng(31)
    specs = []
    for k, (p, n_u, n_v) in enumerate([(3, 200, 40), (2, 1500, 17), (5, 900, 33), (1, 120, 9), (3, 5000, 8),
                                       (4, 3000, 12)]):
        P = synth.random_walk(rng, int(rng.integers(p + 3, 30)))
        Q = synth.perturbed_circle(rng, int(rng.integers(5, 12)))
        specs.append(synth.SweepSpec(synth.CurveSpec(P, p), synth.CurveSpec(Q, 3, True), n_u, n_v))
    law = _law(12, n=6, p=2)
    law.knots = np.array([0, 0, 0, 0.2, 0.5, 0.7, 1, 1, 1], dtype=float)
    glaw = api.Law(dev_ctrl(law.ctrl), law.degree, law.knots) if with_law else None
    b = api.Batch.from_specs(specs)
    say(f"[case] batch {mode} law={with_law} out={out_dtype}: {len(specs)} sweeps")
    pos, nrm = api.sweep_eval_batched(b, out_dtype=out_dtype, frame_mode=mode, law=glaw)
    again = api.sweep_eval_batched(b, out_dtype=out_dtype, frame_mode=mode, law=glaw)
    torch.cuda.synchronize()
    assert torch.equal(pos, again[0]) and torch.equal(nrm, again[1])
    for k, s in enumerate(specs):
        ref, _ = oracle.sweep_ex(s.path, s.profile, s.n_u, s.n_v, mode=mode, law=law if with_law else None)
        tol = TOL[out_dtype]
        if out_dtype == torch.float64 and mode == "rmf":
            tol = max(tol, 8 * s.n_u * np.finfo(float).eps)
        ok, r = parity(ref.pos, ref.nrm, ref.kappa, b.view(pos, k).cpu().numpy(), b.view(nrm, k).cpu().numpy(), tol)
        say(f"   sweep {k} ({s.n_u}x{s.n_v}, p={s.path.degree}): {r}")
        assert ok, (k, r)


def test_frame_modes_and_laws_rejected_where_unsupported():
    spec = synth.c1()
    b = api.Batch.from_specs([spec])
    with pytest.raises(_lib.SweepError, match="UNSUPPORTED"):
        api.sweep_eval_batched(b, frame_mode="frenet", frame_dtype=torch.float32)
    g = torch.zeros(b.out_elems, dtype=torch.float32, device="cuda")
    opt = api.make_options(frame_mode="frenet")
    gP = torch.empty(3 * spec.path.n, dtype=torch.float64, device="cuda")
    gQ = torch.empty(3 * spec.profile.n, dtype=torch.float64, device="cuda")
    ws = torch.empty(1 << 24, dtype=torch.uint8, device="cuda")
    st = _lib.sweep_backward(b.c_struct(), opt, g.data_ptr(), gP.data_ptr(), gQ.data_ptr(), ws.data_ptr(),
                             ws.numel(), 0)
    assert _lib.STATUS[st] == "SWEEP_ERR_UNSUPPORTED"
    with pytest.raises(_lib.SweepError, match="UNSUPPORTED"):
        api.sweep_frames(dev_ctrl(spec.path.ctrl), spec.path.degree, spec.n_u, frame_mode="frenet")
