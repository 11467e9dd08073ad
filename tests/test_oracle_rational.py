"""Pins of the oracle's rational (NURBS) curves (The NURBS Book ch. 4):

* exact homogeneous evaluation: C, C', C'' of random rational curves (clamped,
  given-knot and periodic; degrees 1-4) against exact ``Fraction`` de Boor on
  the homogeneous control net and the expanded quotient rule;
* equal weights give the polynomial curve;
* the quadratic 9-point NURBS circle is a circle: |C| = r, C . C' = 0 and
  curvature 1/r at every sample (a wrong term in the derivative recursion
  breaks the curvature);
* sweeps with rational curves reproduce closed forms: an exact cylinder and
  an exact torus (distance to the axis / centre circle and radial normals).
"""

from __future__ import annotations

from fractions import Fraction as F

import numpy as np
import pytest

import oracle
import synth
from tests import exact_bspline as ex

rng = np.random.default_rng(4321)
EPS = np.finfo(float).eps


def nurbs_circle(r: float, z: float = 0.0):
    """The 9-point quadratic NURBS circle of radius r in the plane z, centre
    on the z axis, starting at (r, 0, z), counter-clockwise."""
    s = np.sqrt(0.5)
    P = np.array([[r, 0], [r, r], [0, r], [-r, r], [-r, 0], [-r, -r], [0, -r], [r, -r], [r, 0]], float)
    ctrl = np.column_stack([P, np.full(9, z)])
    w = np.array([1, s, 1, s, 1, s, 1, s, 1], float)
    U = np.array([0, 0, 0, .25, .25, .5, .5, .75, .75, 1, 1, 1], float)
    return ctrl, w, U


def _cases():
    out = []
    for p in (1, 2, 3, 4):
        out.append(("clamped", p + 4, p))
    out += [("user", 8, 2), ("user", 7, 3), ("closed", 7, 3), ("closed", 5, 2), ("closed", 6, 1)]
    return out


@pytest.mark.parametrize("kind,n,p", _cases())
def test_rational_matches_exact_homogeneous_evaluation(kind, n, p):
    ctrl = np.round(rng.standard_normal((n, 3)) * 64) / 64
    w = np.round(rng.uniform(0.4, 2.5, n) * 64) / 64          # dyadic weights: exact products
    if kind == "closed":
        c = oracle.Curve(ctrl, p, closed=True, weights=w)
        Uf = ex.periodic_knots(n, p)
        Pf = ex.wrap(ex.to_frac(ctrl), p)
        wf = [F(float(w[k % n])) for k in range(n + p)]
    else:
        knots = None
        if kind == "user":
            inner = np.sort(rng.uniform(0, 1, n - p - 1))
            knots = np.concatenate([np.zeros(p + 1), inner, np.ones(p + 1)])
        c = oracle.Curve(ctrl, p, knots=knots, weights=w)
        Uf = [F(float(x)) for x in c.knot_vector()]
        Pf = ex.to_frac(ctrl)
        wf = [F(float(x)) for x in w]
    for u in list(c.params(19)) + [float(x) for x in c.knot_vector()[p:len(Pf) + 1]]:
        got = c.eval(u, nd=2)
        ref = np.array([[float(v) for v in row] for row in ex.rational_derivatives(Uf, Pf, wf, p, F(u))])
        for d in range(3):
            scale = np.abs(ref[: d + 1]).max()
            assert np.abs(got[d] - ref[d]).max() <= 2048 * EPS * max(scale, 1.0), (kind, n, p, u, d, got[d], ref[d])


@pytest.mark.parametrize("closed", [False, True])
def test_equal_weights_give_the_polynomial_curve(closed):
    ctrl = rng.standard_normal((9, 3))
    a = oracle.Curve(ctrl, 3, closed=closed)
    b = oracle.Curve(ctrl, 3, closed=closed, weights=np.full(9, 2.75))
    for u in a.params(31):
        ea, eb = a.eval(u), b.eval(u)
        assert np.abs(ea - eb).max() <= 64 * EPS * (np.abs(ea).max() + 1)


@pytest.mark.parametrize("r", [1.0, 0.3, 7.5])
def test_nurbs_circle_is_exact(r):
    ctrl, w, U = nurbs_circle(r)
    c = oracle.Curve(ctrl, 2, knots=U, weights=w)
    us = list(c.params(101)) + [0.125, 0.3, 0.61, 0.999]
    for u in us:
        C0, C1, C2 = c.eval(u)
        assert abs(np.linalg.norm(C0[:2]) - r) <= 8 * EPS * r
        assert abs(C0 @ C1) <= 64 * EPS * r * np.linalg.norm(C1)
        kappa = (C1[0] * C2[1] - C1[1] * C2[0]) / np.linalg.norm(C1) ** 3
        assert abs(kappa * r - 1.0) <= 1e-13, (u, kappa * r)
        assert C0[2] == 0.0 and C1[2] == 0.0 and C2[2] == 0.0


def test_rational_derivatives_match_finite_differences():
    ctrl = rng.standard_normal((8, 3))
    w = rng.uniform(0.3, 3.0, 8)
    c = oracle.Curve(ctrl, 3, weights=w)
    h = 1e-5
    # off the knots k/5, where the third derivative jumps and the central
    # difference of C' is only first order
    for u in 0.05 + 0.9 * (np.arange(13) + 0.37) / 13:
        C0, C1, C2 = c.eval(u)
        Cp, Cm = c.eval(u + h), c.eval(u - h)
        assert np.abs((Cp[0] - Cm[0]) / (2 * h) - C1).max() <= 1e-7 * (1 + np.abs(C1).max())
        assert np.abs((Cp[1] - Cm[1]) / (2 * h) - C2).max() <= 1e-6 * (1 + np.abs(C2).max())


def test_exact_cylinder_with_nurbs_profile():
    rho = 0.4
    ctrl, w, U = nurbs_circle(rho)
    path = synth.CurveSpec(np.array([[0, 0, -1.0], [0, 0, 0.0], [0, 0, 1.5], [0, 0, 3.0]]), 3)
    prof = synth.CurveSpec(ctrl, 2, False, U, w)
    res = oracle.sweep(path, prof, 17, 41)
    X, N = res.pos, res.nrm
    d = np.hypot(X[0], X[1])
    assert np.abs(d - rho).max() <= 16 * EPS
    radial = np.stack([X[0] / d, X[1] / d, np.zeros_like(d)])
    dots = (N * radial).sum(0)
    assert np.abs(np.abs(dots) - 1).max() <= 1e-13
    assert np.all(np.sign(dots) == np.sign(dots.flat[0]))


def test_exact_torus_from_two_nurbs_circles():
    R, rho = 2.0, 0.5
    pc, pw, pU = nurbs_circle(R)
    qc, qw, qU = nurbs_circle(rho)
    path = synth.CurveSpec(pc, 2, False, pU, pw)
    prof = synth.CurveSpec(qc, 2, False, qU, qw)
    res = oracle.sweep(path, prof, 65, 33, n0=np.array([0.0, 0.0, 1.0]))
    X, N = res.pos, res.nrm
    dxy = np.hypot(X[0], X[1])
    dist = np.hypot(dxy - R, X[2])
    assert np.abs(dist - rho).max() <= 1e-14 * R
    cp = np.stack([R * X[0] / dxy, R * X[1] / dxy, np.zeros_like(dxy)])
    radial = (X - cp) / rho
    dots = (N * radial).sum(0)
    assert np.abs(np.abs(dots) - 1).max() <= 1e-12
    assert np.all(np.sign(dots) == np.sign(dots.flat[0]))
