"""Pins of the oracle's arc-length sampling and triangle list (next-row f4):

* a straight path with uneven control points: samples equally spaced along
  the line and the total length equal to the end-point distance;
* the 9-point NURBS circle (not arc-length parametrised): samples at equal
  angles and total length 2 pi r;
* end points, monotonicity, given-knot domains;
* a sweep sampled by arc length equals the plain evaluation at those
  parameters;
* the triangle list: counts, closed-profile wrap, and every triangle wound
  counter-clockwise about the oracle's vertex normal.
"""

from __future__ import annotations

import numpy as np
import pytest

import oracle
import synth
from tests.test_oracle_rational import nurbs_circle

EPS = np.finfo(float).eps


def test_arclength_on_an_unevenly_parametrised_line():
    P = np.array([[0, 0, 0], [0.1, 0.2, 0.3], [0.15, 0.3, 0.45], [1, 2, 3], [2, 4, 6.0]])
    spec = synth.CurveSpec(P, 3)
    u, total = oracle.arclength_params(spec, 101)
    assert abs(total - np.linalg.norm(P[-1] - P[0])) <= 8 * EPS * total
    x, = oracle.curve_at(spec, u, nd=0)
    d = np.linalg.norm(np.diff(x, axis=0), axis=1)
    assert np.abs(d - total / 100).max() <= 64 * EPS * total
    # the uniform-parameter samples are far from equally spaced
    xu, = oracle.curve_at(spec, np.linspace(0, 1, 101), nd=0)
    assert np.ptp(np.linalg.norm(np.diff(xu, axis=0), axis=1)) > 0.01


@pytest.mark.parametrize("r", [1.0, 0.3])
def test_arclength_on_a_nurbs_circle(r):
    ctrl, w, U = nurbs_circle(r)
    spec = synth.CurveSpec(ctrl, 2, False, U, w)
    u, total = oracle.arclength_params(spec, 97)
    assert abs(total - 2 * np.pi * r) <= 16 * EPS * r
    x, = oracle.curve_at(spec, u, nd=0)
    ang = np.unwrap(np.arctan2(x[:, 1], x[:, 0]))
    assert np.abs(ang - 2 * np.pi * np.arange(97) / 96).max() <= 64 * EPS


def test_arclength_endpoints_monotone_and_given_domain():
    rng = np.random.default_rng(5)
    P = synth.random_walk(rng, 9)
    U = np.concatenate([np.full(4, 0.5), np.sort(rng.uniform(0.5, 2.5, 5)), np.full(4, 2.5)])
    u, total = oracle.arclength_params(synth.CurveSpec(P, 3, knots=U), 200)
    assert u[0] == 0.5 and u[-1] == 2.5 and np.all(np.diff(u) > 0)
    # the arc length from the start to each sample is proportional to its
    # index: an independent integration (64-point Gauss-Legendre on 4 pieces
    # between consecutive samples, split at the knots)
    gx, gw = np.polynomial.legendre.leggauss(64)
    c = oracle.Curve(P, 3, knots=U)

    def length(a, b):
        cuts = [a] + [k for k in U if a < k < b] + [b]
        acc = 0.0
        for lo, hi in zip(cuts[:-1], cuts[1:]):
            for m in range(4):
                l2, h2 = lo + (hi - lo) * m / 4, lo + (hi - lo) * (m + 1) / 4
                t = 0.5 * (l2 + h2) + 0.5 * (h2 - l2) * gx
                acc += 0.5 * (h2 - l2) * sum(wi * np.linalg.norm(c.eval(ti, nd=1)[1]) for ti, wi in zip(t, gw))
        return acc

    s = np.cumsum([0.0] + [length(a, b) for a, b in zip(u[:-1], u[1:])])
    assert abs(s[-1] - total) <= 1e-13 * total
    assert np.abs(s - total * np.arange(200) / 199).max() <= 1e-13 * total


def test_arclength_sweep_is_the_sweep_at_those_parameters():
    s = synth.c1()
    a, _ = oracle.sweep_ex(s.path, s.profile, s.n_u, s.n_v, arclength=True)
    u, _ = oracle.arclength_params(s.path, s.n_u)
    x, d1, d2 = oracle.curve_at(s.path, u, nd=2)
    S, dS = oracle.profile_samples(s.profile, s.n_v)
    _, ft = None, oracle.path_samples(s.path, s.n_u)[3]
    pos, nrm, _, _ = oracle.sweep_from_samples(x, d1, d2, S, dS, fallback_t=ft)
    assert np.abs(a.pos - pos).max() <= 1e-13 and np.abs(a.nrm - nrm).max() <= 1e-12


@pytest.mark.parametrize("closed", [True, False])
def test_triangles_count_wrap_and_orientation(closed):
    s = synth.c1()
    n_u, n_v = 17, 12
    if not closed:
        rng = np.random.default_rng(8)
        Q = np.stack([np.linspace(-0.4, 0.4, 7), 0.2 * np.sin(np.arange(7)), np.zeros(7)], 1)
        prof = synth.CurveSpec(Q, 3, False)
    else:
        prof = s.profile
    tri = oracle.triangles(n_u, n_v, closed)
    nq = n_v if closed else n_v - 1
    assert tri.shape == (2 * (n_u - 1) * nq, 3) and tri.min() == 0 and tri.max() == n_u * n_v - 1
    if closed:
        assert tri[2 * (nq - 1), 1] == 0       # the last quad of row 0 wraps to column 0
    # a smooth, well-resolved surface: a path of gentle curvature
    path = synth.CurveSpec(np.array([[0, 0, 0], [1, 0.2, 0], [2, 0, 0.3], [3, -0.3, 0.5], [4, 0, 0.4]]), 3)
    res = oracle.sweep(path, prof, n_u, n_v)
    X = res.pos.reshape(3, -1).T
    N = res.nrm.reshape(3, -1).T
    a, b, c = X[tri[:, 0]], X[tri[:, 1]], X[tri[:, 2]]
    fn = np.cross(b - a, c - a)
    vn = N[tri[:, 0]] + N[tri[:, 1]] + N[tri[:, 2]]
    assert np.all((fn * vn).sum(1) > 0)


# ------------------------------------------ curvature-adaptive sampling
# density |C'| (1 + lam kappa): equal steps of arc length + lam x turning angle

def test_adaptive_with_lam_zero_is_arc_length():
    spec = synth.c1().path
    a, ta = oracle.arclength_params(spec, 300)
    b, tb = oracle.arclength_params(spec, 300, lam=0.0)
    assert np.array_equal(a, b) and ta == tb


@pytest.mark.parametrize("r,lam", [(1.0, 0.7), (0.3, 2.0)])
def test_adaptive_on_a_circle_is_arc_length(r, lam):
    # constant curvature: the density is a constant multiple of |C'|
    ctrl, w, U = nurbs_circle(r)
    spec = synth.CurveSpec(ctrl, 2, False, U, w)
    ua, _ = oracle.arclength_params(spec, 97)
    ub, total = oracle.arclength_params(spec, 97, lam=lam)
    assert abs(total - 2 * np.pi * (r + lam)) <= 64 * EPS * (r + lam)
    assert np.abs(ua - ub).max() <= 1e-13


@pytest.mark.parametrize("lam", [0.25, 1.5])
def test_adaptive_on_a_parabola(lam):
    # y = x^2 on [0, 1] as a quadratic Bezier curve with x(u) = u: arc length
    # s(x) = x sqrt(1 + 4x^2)/2 + asinh(2x)/4, turning angle atan(2x)
    P = np.array([[0, 0, 0], [0.5, 0, 0], [1, 1, 0.0]])
    spec = synth.CurveSpec(P, 2)
    ns = 65
    u, total = oracle.arclength_params(spec, ns, lam=lam)
    m = lambda x: x * np.sqrt(1 + 4 * x * x) / 2 + np.arcsinh(2 * x) / 4 + lam * np.arctan(2 * x)
    assert abs(total - m(1.0)) <= 1e-13 * m(1.0)
    x, = oracle.curve_at(spec, u, nd=0)
    assert np.abs(x[:, 0] - u).max() <= 4 * EPS
    assert np.abs(m(x[:, 0]) - total * np.arange(ns) / (ns - 1)).max() <= 1e-13 * total
    # denser where the curve turns (near x = 0, where kappa = 2)
    a, _ = oracle.arclength_params(spec, ns)
    assert u[1] < a[1]
