"""Pins of the oracle's finite-difference gradient (O10) of L = sum w . X:
the profile gradient against its closed form (X is linear in the profile
control points, with exact-rational basis values), and two invariants of the
path gradient: translating every path control point translates X
(sum_k dL/dP_k = sum w), and scaling the path about the origin scales C and
leaves the frame unchanged (sum_k P_k . dL/dP_k = sum_ij w_ij . x_i)."""

from fractions import Fraction as F

import numpy as np

import oracle
import synth
from tests import exact_bspline as ex


def _small(seed=3, n_path=8, m=6, nu=64, nv=16):
    rng = np.random.default_rng(seed)
    P = synth.random_walk(rng, n_path)
    Q = synth.perturbed_circle(rng, m)
    w = rng.standard_normal((3, nu, nv))
    return synth.CurveSpec(P, 3), synth.CurveSpec(Q, 3, True), nu, nv, w


def _exact_profile_basis(m, p, nv):
    """B[l, j] = sum_{k = l mod m} N_{k,p}(t_j), exact rationals, at the
    closed-curve sample parameters t_j = p + m j / n_v."""
    U = ex.periodic_knots(m, p)
    B = np.zeros((m, nv))
    for l in range(m):
        ctrl = [[F(1) if (k % m) == l else F(0), F(0), F(0)] for k in range(m + p)]
        for j in range(nv):
            t = F(p) + F(m * j, nv)
            B[l, j] = float(ex.de_boor(U, ctrl, p, t)[0])
    return B


def test_profile_gradient_closed_form():
    path, prof, nu, nv, w = _small()
    gP, gQ = oracle.fd_grad(path, prof, nu, nv, w, want_path=False)
    r = oracle.sweep(path, prof, nu, nv, want_nrm=False, want_kappa=False)
    R = r.frame                                          # (nu, 3, 3), columns r s t
    B = _exact_profile_basis(prof.ctrl.shape[0], 3, nv)  # (m, nv)
    RtW = np.einsum("iab,aij->ijb", R, w)                 # R_i^T w_ij
    ref = np.einsum("lj,ijb->lb", B, RtW)
    assert np.abs(gQ - ref).max() <= 1e-7 * np.abs(ref).max()


def test_path_gradient_translation_and_scaling_invariants():
    path, prof, nu, nv, w = _small(seed=9)
    gP, _ = oracle.fd_grad(path, prof, nu, nv, w, want_profile=False)
    scale = np.abs(gP).max()
    assert np.abs(gP.sum(axis=0) - w.sum(axis=(1, 2))).max() <= 1e-7 * scale
    x, _, _, _ = oracle.path_samples(path, nu)
    lhs = np.sum(path.ctrl * gP)
    rhs = np.einsum("aij,ia->", w, x)
    assert abs(lhs - rhs) <= 1e-7 * scale * np.abs(path.ctrl).max() * path.ctrl.shape[0]


def test_loss_is_weighted_sum_of_positions():
    path, prof, nu, nv, w = _small(seed=4)
    r = oracle.sweep(path, prof, nu, nv, want_nrm=False, want_kappa=False)
    assert abs(oracle.loss(path, prof, nu, nv, w) - float(np.sum(w * r.pos))) < 1e-10
