"""Pins of the oracle's normal condition number kappa (step O8).

kappa is the number that the normal parity rule scales its tolerance by and
masks on, so a wrong kappa would loosen every normal check.  It is defined
as a first-order bound on how much a relative perturbation of the terms of
X_u and X_v moves the unit normal:

    kappa = |X_v| (|C'| + |S_x a| + |S_y b| + |S_z| (|a| + |b|)) / |X_v x X_u|

(and the analogue with the frame derivatives and the law terms for frame
modes and sweep laws).  The pins below fix it without retyping it:

  * exact cylinder (straight path): X_u = |C'| t is perpendicular to X_v, so
    kappa = 1 at every vertex;
  * exact torus section (exact circle samples, one frame vector on the
    circle's axis): kappa = (R + |d|) / |R + d| with d the vertex's distance
    from the torus axis minus R, read off the output positions;
  * cone of revolution (straight path, linear scale law, exact NURBS circle):
    X_u is perpendicular to X_v, so kappa = (H + rho |cos a| + rho |sin a|) /
    sqrt(H^2 + rho^2) with a the vertex's angle in the frame;
  * as a sensitivity bound: random relative perturbations of size delta of
    every input of the surface step move each normal by at most a small
    multiple of kappa * delta, and by a sizeable fraction of it somewhere.
"""

from __future__ import annotations

import numpy as np

import oracle
import synth
from tests.test_oracle_frame import _tilted_circle
from tests.test_oracle_frenet_laws import _straight_path
from tests.test_oracle_rational import nurbs_circle

rng = np.random.default_rng(2024)


def _circle_profile(rho, nv, z=0.0, c=(0.0, 0.0)):
    phi = 2 * np.pi * np.arange(nv) / nv
    S = np.stack([c[0] + rho * np.cos(phi), c[1] + rho * np.sin(phi), np.full(nv, z)], 1)
    dS = np.stack([-rho * np.sin(phi), rho * np.cos(phi), np.zeros(nv)], 1)
    return S, dS


def test_kappa_is_one_on_the_exact_cylinder():
    n, p, L = 12, 3, 5.0
    e = np.array([0.3, -1.0, 0.6]); e /= np.linalg.norm(e)
    U = oracle.Curve(np.zeros((n, 3)), p).knot_vector()
    xi = np.array([U[k + 1:k + p + 1].sum() / p for k in range(n)])
    P = np.array([1.0, 2.0, -0.5]) + L * xi[:, None] * e
    prof = synth.perturbed_circle(rng, 11)
    r = oracle.sweep(synth.CurveSpec(P, p), synth.CurveSpec(prof, 3, True), 97, 29)
    assert np.abs(r.kappa - 1.0).max() < 1e-13, np.abs(r.kappa - 1.0).max()


def _torus_kappa_case(start_normal: str):
    Rad, rho = 2.0, 0.45
    th, c0, nh, x, d1, d2 = _tilted_circle(Rad, np.array([0.4, -0.3, 0.85]), 150, 1.6 * np.pi)
    n0 = nh if start_normal == "axis" else (x[0] - c0) / Rad
    S, dS = _circle_profile(rho, 48)
    pos, nrm, kap, R = oracle.sweep_from_samples(x, d1, d2, S, dS, n0=n0)
    Y = pos - c0[:, None, None]
    h = np.einsum("a,aij->ij", nh, Y)
    rad = np.sqrt(np.maximum(np.einsum("aij,aij->ij", Y, Y) - h * h, 0))
    d = rad - Rad
    ref = (Rad + np.abs(d)) / np.abs(Rad + d)
    return kap, ref


def test_kappa_closed_form_on_the_exact_torus_frame_vector_on_the_axis():
    kap, ref = _torus_kappa_case("axis")
    assert np.abs(kap - ref).max() < 1e-12, np.abs(kap - ref).max()
    assert ref.max() > 1.5          # the inner side of the tube is ill-conditioned, the outer is not
    assert np.abs(ref.min() - 1.0) < 1e-12


def test_kappa_closed_form_on_the_exact_torus_frame_vector_radial():
    kap, ref = _torus_kappa_case("radial")
    assert np.abs(kap - ref).max() < 1e-12, np.abs(kap - ref).max()


def test_kappa_closed_form_on_a_cone_from_a_scale_law():
    rho, H = 0.4, 2.0
    qc, qw, qU = nurbs_circle(rho)
    prof = synth.CurveSpec(qc, 2, False, qU, qw)
    law = synth.CurveSpec(np.array([[1.0, 0.0, 0.0], [2.0, 0.0, 0.0]]), 1)
    n_u = 25
    res, _ = oracle.sweep_ex(_straight_path(H), prof, n_u, 37, law=law)
    u = np.linspace(0.0, 1.0, n_u)
    off = res.pos.copy()
    off[2] -= H * u[:, None]                       # minus the path point (0, 0, H u): the offset in the frame plane
    pr = np.einsum("ia,aij->ij", res.frame[:, :, 0], off)
    ps = np.einsum("ia,aij->ij", res.frame[:, :, 1], off)
    a = np.arctan2(ps, pr)
    ref = (H + rho * (np.abs(np.cos(a)) + np.abs(np.sin(a)))) / np.hypot(H, rho)
    assert np.abs(res.kappa - ref).max() < 1e-12, np.abs(res.kappa - ref).max()


def _perturbed(a, delta):
    return a * (1.0 + delta * rng.uniform(-1.0, 1.0, np.shape(a)))


def _sensitivity_ratios(surface, inputs, kap, nrm, delta=1e-7, trials=6):
    """max over trials of |N(perturbed inputs) - N| / (kappa delta), per vertex."""
    worst = np.zeros_like(kap)
    for _ in range(trials):
        _, n2, _ = surface(*[None if v is None else _perturbed(v, delta) for v in inputs])
        dn = np.linalg.norm(n2 - nrm, axis=0)
        worst = np.maximum(worst, dn / (kap * delta))
    return worst


def test_kappa_bounds_the_normal_sensitivity_with_an_offset_profile():
    # exact circle path (constant speed) and a profile lifted along t by S_z =
    # 12, so that the S_z t' term dominates X_u on part of the surface
    Rad = 1.0
    th, c0, nh, x, d1, d2 = _tilted_circle(Rad, np.array([0.1, 0.2, 0.95]), 60, 1.2 * np.pi)
    S, dS = _circle_profile(0.3, 36, z=12.0, c=(0.1, -0.05))
    R, _ = oracle.frame(x, d1)
    pos, nrm, kap = oracle.surface_from_samples(x, d1, d2, R, S, dS)
    ok = np.isfinite(kap) & (kap < 1e5)
    assert ok.mean() > 0.95

    def surface(x_, d1_, d2_, R_, S_, dS_):
        return oracle.surface_from_samples(x_, d1_, d2_, R_, S_, dS_)

    worst = _sensitivity_ratios(surface, [x, d1, d2, R, S, dS], kap, nrm)[ok]
    assert worst.max() <= 4.0, worst.max()
    assert worst.max() >= 0.1, worst.max()


def test_kappa_bounds_the_normal_sensitivity_with_frame_rate_and_law():
    # helix samples with the Frenet rotation rate and a scale/twist law with a
    # fast twist of an off-centre profile (the law-derivative terms dominate)
    u = np.linspace(0.0, 2.0, 50)
    Rh, w, hh = 1.0, 1.3, 0.5
    c, s = np.cos(w * u), np.sin(w * u)
    x = np.stack([Rh * c, Rh * s, hh * u], 1)
    d1 = np.stack([-Rh * w * s, Rh * w * c, np.full_like(u, hh)], 1)
    d2 = np.stack([-Rh * w * w * c, -Rh * w * w * s, np.zeros_like(u)], 1)
    R, _ = oracle.frame(x, d1)
    omega = np.full(50, 0.37)
    law = np.stack([1.0 + 0.3 * u, 0.5 * u * u, np.full_like(u, 0.3), 9.0 * u], 1)
    S, dS = _circle_profile(0.25, 30, z=0.4, c=(0.6, 0.2))
    pos, nrm, kap = oracle.surface_ex_from_samples(x, d1, d2, R, omega, law, S, dS)
    ok = np.isfinite(kap) & (kap < 1e5)
    assert ok.mean() > 0.95

    def surface(x_, d1_, d2_, R_, om_, lw_, S_, dS_):
        return oracle.surface_ex_from_samples(x_, d1_, d2_, R_, om_, lw_, S_, dS_)

    worst = _sensitivity_ratios(surface, [x, d1, d2, R, omega, law, S, dS], kap, nrm)[ok]
    assert worst.max() <= 4.0, worst.max()
    assert worst.max() >= 0.1, worst.max()
