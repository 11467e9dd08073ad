"""Exact rational B-spline evaluation by de Boor's algorithm (test pin).

An implementation independent of the oracle's basis-function route: points
come from de Boor's corner-cutting triangle (de Boor 1972), derivatives from
the derivative control net
    Q_k = p (P_{k+1} - P_k) / (U_{k+p+1} - U_{k+1})      (0/0 := 0),
a degree p-1 B-spline on the knot vector with its first and last knot removed
(Piegl & Tiller, The NURBS Book, sec. 3.3).  All arithmetic is in
``fractions.Fraction``, so the only rounding in a comparison is the oracle's.

The span rule (largest k in [p, nb-1] with U_k <= u, and nb-1 for u >= U_nb)
and the knot vectors (clamped uniform with interior knots k/(n-p); periodic
uniform U_k = k over the wrapped polygon) restate the definitions the oracle
implements.
"""

from __future__ import annotations

from fractions import Fraction as F
from typing import List, Sequence


def clamped_uniform_knots(n: int, p: int) -> List[F]:
    return [F(0)] * (p + 1) + [F(k, n - p) for k in range(1, n - p)] + [F(1)] * (p + 1)


def periodic_knots(m: int, p: int) -> List[F]:
    return [F(k) for k in range(m + 2 * p + 1)]


def wrap(ctrl: Sequence[Sequence[F]], p: int) -> List[List[F]]:
    m = len(ctrl)
    return [list(ctrl[k % m]) for k in range(m + p)]


def span(U: Sequence[F], nb: int, p: int, u: F) -> int:
    if u >= U[nb]:
        return nb - 1
    k = p
    while k + 1 < nb and U[k + 1] <= u:
        k += 1
    return k


def de_boor(U: Sequence[F], P: Sequence[Sequence[F]], p: int, u: F) -> List[F]:
    """Point of the degree-p B-spline with knots U and control points P."""
    nb = len(P)
    if p == 0:
        return list(P[span(U, nb, 0, u)])
    k = span(U, nb, p, u)
    d = [list(P[j + k - p]) for j in range(p + 1)]
    for r in range(1, p + 1):
        for j in range(p, r - 1, -1):
            lo = U[j + k - p]
            hi = U[j + 1 + k - r]
            a = (u - lo) / (hi - lo) if hi != lo else F(0)
            d[j] = [(1 - a) * d[j - 1][c] + a * d[j][c] for c in range(len(d[j]))]
    return d[p]


def derivative_net(U: Sequence[F], P: Sequence[Sequence[F]], p: int):
    """Control points and knots of C' (degree p-1)."""
    Q = []
    dim = len(P[0])
    for k in range(len(P) - 1):
        den = U[k + p + 1] - U[k + 1]
        if den == 0:
            Q.append([F(0)] * dim)
        else:
            Q.append([p * (P[k + 1][c] - P[k][c]) / den for c in range(dim)])
    return list(U[1:-1]), Q


def derivatives(U: Sequence[F], P: Sequence[Sequence[F]], p: int, u: F, nd: int) -> List[List[F]]:
    """[C(u), C'(u), ..., C^(nd)(u)]; derivatives above the degree are 0."""
    out = []
    Uc, Pc, pc = list(U), [list(x) for x in P], p
    dim = len(P[0])
    for d in range(nd + 1):
        if pc < 0:
            out.append([F(0)] * dim)
            continue
        out.append(de_boor(Uc, Pc, pc, u))
        if pc == 0:
            pc = -1
            continue
        Uc, Pc = derivative_net(Uc, Pc, pc)
        pc -= 1
    return out


def rational_derivatives(U: Sequence[F], P: Sequence[Sequence[F]], w: Sequence[F], p: int, u: F) -> List[List[F]]:
    """[C, C', C''] of the rational curve with weights w: the homogeneous
    curve (w P, w) is evaluated exactly (points and derivative nets above),
    C = A / W, and the derivatives of the quotient are taken in expanded form
        C'  = (A' W - A W') / W^2,
        C'' = (A'' W^2 - A W'' W - 2 A' W' W + 2 A W'^2) / W^3."""
    Pw = [[w[k] * P[k][c] for c in range(3)] + [w[k]] for k in range(len(P))]
    H = derivatives(U, Pw, p, u, 2)
    A = [H[d][:3] for d in range(3)]
    W = [H[d][3] for d in range(3)]
    C0 = [A[0][c] / W[0] for c in range(3)]
    C1 = [(A[1][c] * W[0] - A[0][c] * W[1]) / (W[0] ** 2) for c in range(3)]
    C2 = [(A[2][c] * W[0] ** 2 - A[0][c] * W[2] * W[0] - 2 * A[1][c] * W[1] * W[0] + 2 * A[0][c] * W[1] ** 2)
          / (W[0] ** 3) for c in range(3)]
    return [C0, C1, C2]


def to_frac(a) -> List[List[F]]:
    return [[F(float(v)) for v in row] for row in a]
