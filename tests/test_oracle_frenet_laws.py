"""Pins of the oracle's frame modes and sweep laws (next-row f2):

* Frenet frame and torsion rate on an analytic helix (closed forms of T, N,
  B, curvature and torsion);
* rotation-minimizing mode without laws equals the plain sweep;
* surfaces whose closed form is known, compared position by position and
  with normals from central differences of the closed form:
  - an elliptic tube around an analytic helix with the Frenet frame (the
    torsion term of the frame derivative matters: the profile is not round);
  - a cone from a linear scale law on a straight path;
  - a twisted offset tube from a linear twist law;
  - an elliptic torus from a NURBS-circle path with the Frenet frame.
"""

from __future__ import annotations

import numpy as np
import pytest

import oracle
import synth
from tests.test_oracle_rational import nurbs_circle

EPS = np.finfo(float).eps


def _helix(R, w, h, u):
    c, s = np.cos(w * u), np.sin(w * u)
    x = np.stack([R * c, R * s, h * u], 1)
    d1 = np.stack([-R * w * s, R * w * c, np.full_like(u, h)], 1)
    d2 = np.stack([-R * w * w * c, -R * w * w * s, np.zeros_like(u)], 1)
    d3 = np.stack([R * w ** 3 * s, -R * w ** 3 * c, np.zeros_like(u)], 1)
    return x, d1, d2, d3


def _helix_frenet(R, w, h, u):
    c, s = np.cos(w * u), np.sin(w * u)
    L = np.sqrt(R * R * w * w + h * h)
    T = np.stack([-R * w * s, R * w * c, np.full_like(u, h)], 1) / L
    N = np.stack([-c, -s, np.zeros_like(u)], 1)
    B = np.cross(T, N)
    return T, N, B, L


def test_frenet_frame_and_torsion_rate_on_a_helix():
    R, w, h = 1.5, 2.0, 0.7
    u = np.linspace(0.0, 3.0, 301)
    x, d1, d2, d3 = _helix(R, w, h, u)
    t = d1 / np.linalg.norm(d1, axis=1, keepdims=True)
    F, om = oracle.frenet(t, d1, d2, d3)
    T, N, B, L = _helix_frenet(R, w, h, u)
    assert np.abs(F[:, :, 0] - N).max() <= 16 * EPS
    assert np.abs(F[:, :, 1] - B).max() <= 16 * EPS
    tau = h * w / (R * R * w * w + h * h)
    assert np.abs(om - L * tau).max() <= 64 * EPS * L * tau


def test_frenet_straight_piece_falls_back_to_the_axis_rule():
    u = np.linspace(0, 1, 5)
    d1 = np.tile([0.0, 0.0, 2.0], (5, 1))
    d2 = np.tile([0.0, 0.0, 0.5], (5, 1))       # parallel to C': no normal direction
    d3 = np.zeros((5, 3))
    F, om = oracle.frenet(d1 / 2.0, d1, d2, d3)
    assert np.all(F[:, :, 0] == [1.0, 0.0, 0.0]) and np.all(om == 0.0)


def test_rmf_mode_without_law_equals_the_plain_sweep():
    s = synth.c1()
    a = oracle.sweep(s.path, s.profile, s.n_u, s.n_v)
    b, om = oracle.sweep_ex(s.path, s.profile, s.n_u, s.n_v, mode="rmf")
    assert np.array_equal(a.pos, b.pos) and np.all(om == 0)
    assert np.abs(a.nrm - b.nrm).max() <= 1e-12


def _fd_normals(Xf, u, v, h=1e-6):
    """Normals (3, nu, nv) of the closed-form surface Xf(u, v) -> (3, ...) by
    central differences, oriented as X_v x X_u."""
    U, V = np.meshgrid(u, v, indexing="ij")
    Xu = (Xf(U + h, V) - Xf(U - h, V)) / (2 * h)
    Xv = (Xf(U, V + h) - Xf(U, V - h)) / (2 * h)
    n = np.cross(Xv, Xu, axis=0)
    return n / np.linalg.norm(n, axis=0)


def test_elliptic_tube_around_a_helix_with_the_frenet_frame():
    R, w, h, a, b = 1.5, 2.0, 0.7, 0.3, 0.12
    u = np.linspace(0.0, 3.0, 97)
    v = np.linspace(0.0, 2 * np.pi, 41, endpoint=False)
    x, d1, d2, d3 = _helix(R, w, h, u)
    t = d1 / np.linalg.norm(d1, axis=1, keepdims=True)
    F, om = oracle.frenet(t, d1, d2, d3)
    S = np.stack([a * np.cos(v), b * np.sin(v), np.zeros_like(v)], 1)
    dS = np.stack([-a * np.sin(v), b * np.cos(v), np.zeros_like(v)], 1)
    pos, nrm, _ = oracle.surface_ex_from_samples(x, d1, d2, F, om, None, S, dS)

    def Xf(U, V):
        c, s = np.cos(w * U), np.sin(w * U)
        L = np.sqrt(R * R * w * w + h * h)
        T = np.stack([-R * w * s, R * w * c, np.full_like(U, h)]) / L
        N = np.stack([-c, -s, np.zeros_like(U)])
        B = np.cross(T, N, axis=0)
        C = np.stack([R * c, R * s, h * U])
        return C + a * np.cos(V) * N + b * np.sin(V) * B

    assert np.abs(pos - Xf(*np.meshgrid(u, v, indexing="ij"))).max() <= 1e-14
    assert np.abs(nrm - _fd_normals(Xf, u, v)).max() <= 1e-7


def _straight_path(H=2.0):
    return synth.CurveSpec(np.array([[0.0, 0.0, 0.0], [0.0, 0.0, H]]), 1)


def test_scale_law_makes_a_cone():
    rho, H = 0.4, 2.0
    qc, qw, qU = nurbs_circle(rho)
    prof = synth.CurveSpec(qc, 2, False, qU, qw)
    law = synth.CurveSpec(np.array([[1.0, 0.0, 0.0], [2.0, 0.0, 0.0]]), 1)
    n_u, n_v = 33, 41
    res, _ = oracle.sweep_ex(_straight_path(H), prof, n_u, n_v, law=law)
    u = np.linspace(0, 1, n_u)
    ang = 2 * np.pi * np.linspace(0, 1, n_v)      # the NURBS circle is not arc-length parametrised
    X = res.pos
    assert np.abs(np.hypot(X[0], X[1]) - rho * (1 + u)[:, None]).max() <= 16 * EPS
    assert np.abs(X[2] - H * u[:, None]).max() <= 4 * EPS
    # normals: the cone (rho(1+u) cos a, rho(1+u) sin a, H u), oriented like X_v x X_u
    phi = np.arctan2(X[1], X[0])
    nr = np.stack([H * np.cos(phi), H * np.sin(phi), -rho * np.ones_like(phi)])
    nr /= np.linalg.norm(nr, axis=0)
    dots = (res.nrm * nr).sum(0)
    assert np.abs(np.abs(dots) - 1).max() <= 1e-13
    assert np.all(np.sign(dots) == np.sign(dots.flat[0]))


def test_twist_law_makes_a_twisted_offset_tube():
    rho, d, H, Th = 0.2, 0.6, 2.0, 3.0
    qc, qw, qU = nurbs_circle(rho)
    qc = qc + np.array([d, 0.0, 0.0])
    prof = synth.CurveSpec(qc, 2, False, qU, qw)
    law = synth.CurveSpec(np.array([[1.0, 0.0, 0.0], [1.0, Th, 0.0]]), 1)
    n_u, n_v = 65, 33
    res, _ = oracle.sweep_ex(_straight_path(H), prof, n_u, n_v, law=law)
    u = np.linspace(0, 1, n_u)
    S, dS = oracle.profile_samples(prof, n_v)
    c, s = np.cos(Th * u)[:, None], np.sin(Th * u)[:, None]
    Xx = c * S[None, :, 0] - s * S[None, :, 1]
    Xy = s * S[None, :, 0] + c * S[None, :, 1]
    assert np.abs(res.pos[0] - Xx).max() <= 16 * EPS and np.abs(res.pos[1] - Xy).max() <= 16 * EPS
    # closed form: X(u, a) = (Rot(Th u)(d + rho cos a, rho sin a), H u)

    def Xf(U, A):
        px, py = d + rho * np.cos(A), rho * np.sin(A)
        cu, su = np.cos(Th * U), np.sin(Th * U)
        return np.stack([cu * px - su * py, su * px + cu * py, H * U])

    # the profile's own parameter is not the angle: compare with the
    # closed-form normal at the angle of each profile sample
    A = np.arctan2(S[:, 1], S[:, 0] - d)
    U, AA = np.meshgrid(u, A, indexing="ij")
    hh = 1e-6
    Xu = (Xf(U + hh, AA) - Xf(U - hh, AA)) / (2 * hh)
    Xa = (Xf(U, AA + hh) - Xf(U, AA - hh)) / (2 * hh)
    n = np.cross(Xa, Xu, axis=0)
    n /= np.linalg.norm(n, axis=0)
    assert np.abs(res.nrm - n).max() <= 1e-7


def test_elliptic_torus_from_a_nurbs_circle_with_the_frenet_frame():
    R, a, b = 2.0, 0.5, 0.2
    pc, pw, pU = nurbs_circle(R)
    path = synth.CurveSpec(pc, 2, False, pU, pw)
    ang = np.linspace(0, 2 * np.pi, 48, endpoint=False)
    prof = synth.CurveSpec(np.stack([a * np.cos(ang), b * np.sin(ang), np.zeros(48)], 1), 3, True)
    n_u, n_v = 65, 40
    res, om = oracle.sweep_ex(path, prof, n_u, n_v, mode="frenet")
    assert np.abs(om).max() <= 1e-12           # planar path: no torsion
    F = res.frame
    x, _, _, _ = oracle.path_samples(path, n_u)
    inward = -x / np.linalg.norm(x, axis=1, keepdims=True)
    assert np.abs(F[:, :, 0] - inward).max() <= 1e-14
    assert np.abs(F[:, :, 1] - [0, 0, 1]).max() <= 1e-14
    S, _ = oracle.profile_samples(prof, n_v)
    # X = C + S_x n + S_y e_z: a surface of revolution about z; its points
    # lie at radius R - S_x and height S_y
    X = res.pos
    assert np.abs(np.hypot(X[0], X[1]) - (R - S[None, :, 0])).max() <= 1e-14
    assert np.abs(X[2] - S[None, :, 1]).max() <= 1e-15
    # normals of a surface of revolution lie in the meridian plane
    radial = np.stack([X[0], X[1]]) / np.hypot(X[0], X[1])
    perp = res.nrm[0] * (-radial[1]) + res.nrm[1] * radial[0]
    assert np.abs(perp).max() <= 1e-13
