"""Pins of the oracle's knots, spans, basis functions and curve evaluation
(steps O1-O4) against mathematics that does not go through the oracle's code:
exact-rational de Boor evaluation, Bernstein polynomials, the uniform cubic
blending polynomials, partition of unity, linear precision at the Greville
abscissae and the values of periodic uniform B-splines at knots."""

from fractions import Fraction as F
from math import comb

import numpy as np
import pytest

import oracle
from tests import exact_bspline as ex

rng = np.random.default_rng(1234)


def _ulp_close(a, b, scale, k=64):
    return np.abs(np.asarray(a) - np.asarray(b)).max() <= k * np.finfo(float).eps * max(scale, 1.0)


# ------------------------------------------------------------------- knots

@pytest.mark.parametrize("n,p", [(4, 3), (5, 3), (16, 3), (1024, 3), (7, 2), (9, 1), (12, 5)])
def test_clamped_uniform_knots_are_exact_rationals(n, p):
    U = oracle.Curve(np.zeros((n, 3)), p).knot_vector()
    ref = ex.clamped_uniform_knots(n, p)
    assert len(U) == n + p + 1
    # each stored knot is the correctly rounded value of k/(n-p)
    assert all(U[k] == float(ref[k]) for k in range(len(U)))


def test_periodic_knots():
    U = oracle.Curve(np.zeros((8, 3)), 3, closed=True).knot_vector()
    assert list(U) == list(range(8 + 2 * 3 + 1))


def test_sample_params_open_and_closed():
    c = oracle.Curve(np.zeros((16, 3)), 3)
    u = c.params(256)
    assert u[0] == 0.0 and u[-1] == 1.0
    assert all(u[i] == i / 255 for i in range(256))
    q = oracle.Curve(np.zeros((8, 3)), 3, closed=True)
    t = q.params(64)
    assert t[0] == 3.0 and t[-1] < 3.0 + 8
    assert all(t[j] == 3 + (8 * j) / 64 for j in range(64))


def test_span_rule_at_knots_and_end():
    n, p = 10, 3
    c = oracle.Curve(np.zeros((n, 3)), p)
    U = c.knot_vector()
    # at each interior knot the span starts there; the right end maps to n-1
    for k in range(p + 1, n):
        assert c.span(U[k]) == k
        assert c.span(np.nextafter(U[k], -1.0)) == k - 1
    assert c.span(1.0) == n - 1
    assert c.span(0.0) == p
    # user knots with an interior knot of multiplicity p
    Uu = np.array([0, 0, 0, 0, .5, .5, .5, 1, 1, 1, 1], float)
    cu = oracle.Curve(np.zeros((7, 3)), 3, knots=Uu)
    assert cu.span(0.5) == 6 and cu.span(0.4999) == 3 and cu.span(1.0) == 6


def test_sample_on_knot_has_exact_span():
    # u_i = i/(n_u-1) hits knot k/(n-p) exactly when the rationals agree
    n, p, nu = 13, 3, 31          # n-p = 10, n_u-1 = 30: i = 3k lands on knot k
    c = oracle.Curve(np.zeros((n, 3)), p)
    for i in range(nu):
        u = c.param(i, nu)
        fr = F(i, nu - 1)
        k = min(p + int(fr * (n - p)), n - 1)
        assert c.span(u) == k


# ------------------------------------------------------------------- basis

def _random_knots(n, p, mult=False):
    inner = np.sort(rng.uniform(0.0, 1.0, n - p - 1))
    if mult and len(inner) >= 3:
        inner[1] = inner[2] = inner[0]   # an interior knot of multiplicity 3
    return np.concatenate([np.zeros(p + 1), inner, np.ones(p + 1)])


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 7])
@pytest.mark.parametrize("mult", [False, True])
def test_partition_of_unity_and_derivative_sums(p, mult):
    n = p + 6
    U = _random_knots(n, p, mult)
    for u in np.concatenate([rng.uniform(0, 1, 40), U[p:n + 1]]):
        span = oracle.lib().or_span(oracle._ptr(U), n, p, float(u))
        B = oracle.basis(U, p, span, u, nd=2)
        assert abs(B[0].sum() - 1.0) < 1e-14
        assert (B[0] >= -1e-15).all()
        scale = np.abs(B[1]).max() + np.abs(B[2]).max()
        assert abs(B[1].sum()) <= 1e-12 * max(1, scale)
        assert abs(B[2].sum()) <= 1e-11 * max(1, scale)


@pytest.mark.parametrize("p", [1, 2, 3, 4, 6])
def test_bezier_knots_give_bernstein(p):
    U = np.array([0.0] * (p + 1) + [1.0] * (p + 1))
    for u in np.linspace(0, 1, 33):
        B = oracle.basis(U, p, p, u, nd=2)
        for k in range(p + 1):
            b0 = comb(p, k) * u ** k * (1 - u) ** (p - k)
            # d/du of u^k (1-u)^(p-k) and its second derivative
            def term(e_u, e_v, c):
                return c * (u ** e_u if e_u >= 0 else 0.0) * ((1 - u) ** e_v if e_v >= 0 else 0.0)
            b1 = comb(p, k) * (term(k - 1, p - k, k) - term(k, p - k - 1, p - k))
            b2 = comb(p, k) * (term(k - 2, p - k, k * (k - 1)) - 2 * term(k - 1, p - k - 1, k * (p - k))
                               + term(k, p - k - 2, (p - k) * (p - k - 1)))
            assert abs(B[0, k] - b0) < 1e-14
            assert abs(B[1, k] - b1) < 1e-12 * p * p
            assert abs(B[2, k] - b2) < 1e-11 * p ** 4


def test_uniform_cubic_blending_polynomials():
    # periodic uniform cubic on span k, local parameter s in [0,1):
    # (1-s)^3/6, (3s^3-6s^2+4)/6, (-3s^3+3s^2+3s+1)/6, s^3/6
    U = np.arange(20, dtype=float)
    for s in np.linspace(0, 1, 17, endpoint=False):
        u = 8.0 + s
        B = oracle.basis(U, 3, 8, u, nd=2)
        ref = [(1 - s) ** 3 / 6, (3 * s ** 3 - 6 * s ** 2 + 4) / 6, (-3 * s ** 3 + 3 * s ** 2 + 3 * s + 1) / 6, s ** 3 / 6]
        d1 = [-(1 - s) ** 2 / 2, (9 * s ** 2 - 12 * s) / 6, (-9 * s ** 2 + 6 * s + 3) / 6, s ** 2 / 2]
        d2 = [(1 - s), (18 * s - 12) / 6, (-18 * s + 6) / 6, s]
        assert np.allclose(B[0], ref, atol=1e-15, rtol=0)
        assert np.allclose(B[1], d1, atol=1e-14, rtol=0)
        assert np.allclose(B[2], d2, atol=1e-13, rtol=0)


# ------------------------------------------------------------------ curves

def _cases():
    out = []
    for p in (1, 2, 3, 4):
        for n in (p + 1, p + 3, 8):
            out.append(("clamped", n, p))
    out += [("user", 7, 3), ("user", 8, 2), ("closed", 8, 3), ("closed", 5, 2), ("closed", 4, 3), ("closed", 6, 1)]
    return out


@pytest.mark.parametrize("kind,n,p", _cases())
def test_curve_matches_exact_de_boor(kind, n, p):
    ctrl = np.round(rng.standard_normal((n, 3)) * 64) / 64  # dyadic: exact in binary
    if kind == "closed":
        c = oracle.Curve(ctrl, p, closed=True)
        Uf = ex.periodic_knots(n, p)
        Pf = ex.wrap(ex.to_frac(ctrl), p)
    elif kind == "user":
        U = _random_knots(n, p, mult=True)
        c = oracle.Curve(ctrl, p, knots=U)
        Uf = [F(float(x)) for x in U]
        Pf = ex.to_frac(ctrl)
    else:
        c = oracle.Curve(ctrl, p)
        # the stored (rounded) knots define the spline; their rounding is
        # pinned by test_clamped_uniform_knots_are_exact_rationals
        Uf = [F(float(x)) for x in c.knot_vector()]
        assert Uf == [F(float(x)) for x in ex.clamped_uniform_knots(n, p)]
        Pf = ex.to_frac(ctrl)
    ns = 23
    us = c.params(ns)
    extra = [float(x) for x in c.knot_vector()[p:len(Pf) + 1]]
    for u in list(us) + extra:
        got = c.eval(u, nd=2)
        ref = np.array([[float(v) for v in row] for row in ex.derivatives(Uf, Pf, p, F(u), 2)])
        for d in range(3):
            scale = np.abs(ref[d]).max() + np.abs(ref[0]).max()
            assert _ulp_close(got[d], ref[d], scale, k=256), (kind, n, p, u, d, got[d], ref[d])


def test_greville_linear_precision():
    for p, n in [(2, 7), (3, 16), (3, 1024), (5, 11)]:
        U = oracle.Curve(np.zeros((n, 3)), p).knot_vector()
        xi = np.array([U[k + 1:k + p + 1].sum() / p for k in range(n)])
        ctrl = np.stack([xi, np.zeros(n), np.zeros(n)], 1)
        c = oracle.Curve(ctrl, p)
        x, d1, d2 = c.samples(97)
        u = c.params(97)
        assert np.abs(x[:, 0] - u).max() < 1e-14
        assert np.abs(x[:, 1:]).max() == 0.0
        assert np.abs(d1[:, 0] - 1).max() < 1e-11
        assert np.abs(d2[:, 0]).max() < 1e-8 * n * n


@pytest.mark.parametrize("m", [4, 5, 8, 13, 64])
def test_periodic_cubic_at_knots(m):
    Q = rng.standard_normal((m, 3))
    c = oracle.Curve(Q, 3, closed=True)
    for k in range(m):
        # knot u = p + k starts span p+k, whose blending weights at s = 0 are
        # (1/6, 4/6, 1/6, 0) on Q_k, Q_{k+1}, Q_{k+2}, Q_{k+3}
        C = c.eval(3.0 + k, nd=1)
        ref = (Q[k % m] + 4 * Q[(k + 1) % m] + Q[(k + 2) % m]) / 6
        dref = (Q[(k + 2) % m] - Q[k % m]) / 2
        assert np.abs(C[0] - ref).max() < 1e-14
        assert np.abs(C[1] - dref).max() < 1e-13


def test_periodic_quadratic_at_knots():
    m = 7
    Q = rng.standard_normal((m, 3))
    c = oracle.Curve(Q, 2, closed=True)
    for k in range(m):
        C = c.eval(2.0 + k, nd=1)
        assert np.abs(C[0] - (Q[k % m] + Q[(k + 1) % m]) / 2).max() < 1e-15
        assert np.abs(C[1] - (Q[(k + 1) % m] - Q[k % m])).max() < 1e-14


def test_regular_polygon_radius_at_knots():
    m, r = 8, 0.3
    ang = 2 * np.pi * np.arange(m) / m
    Q = np.stack([r * np.cos(ang), r * np.sin(ang), np.zeros(m)], 1)
    c = oracle.Curve(Q, 3, closed=True)
    S, dS = c.samples(64, nd=1)
    at_knots = S[::8]
    radius = np.linalg.norm(at_knots, axis=1)
    assert np.abs(radius - r * (4 + 2 * np.cos(2 * np.pi / m)) / 6).max() < 1e-15
    assert abs((4 + 2 * np.cos(2 * np.pi / 8)) / 6 - 0.90237) < 1e-5
    # counter-clockwise: S x S' has positive z everywhere
    assert (np.cross(S, dS)[:, 2] > 0).all()
