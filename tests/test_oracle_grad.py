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


# ------------------------------------------------ the normal term of the loss
# L_N = sum g . N (N the unit normal).  Normals are unchanged when the whole
# sweep is translated or scaled about the origin (the frame depends on
# directions only), which fixes two combinations of the gradient; on an exact
# cylinder the normals are the radial directions whatever the radius.

def test_normal_loss_is_weighted_sum_of_normals():
    path, prof, nu, nv, _ = _small(seed=5)
    g = np.random.default_rng(50).standard_normal((3, nu, nv))
    r = oracle.sweep(path, prof, nu, nv, want_kappa=False)
    assert abs(oracle.loss(path, prof, nu, nv, None, g=g) - float(np.sum(g * r.nrm))) < 1e-10
    w = np.random.default_rng(51).standard_normal((3, nu, nv))
    both = oracle.loss(path, prof, nu, nv, w, g=g)
    assert abs(both - float(np.sum(w * r.pos) + np.sum(g * r.nrm))) < 1e-10


def test_normal_loss_on_an_exact_cylinder():
    from tests.test_oracle_rational import nurbs_circle
    rho, nu, nv = 0.4, 17, 40
    ctrl, wts, U = nurbs_circle(rho)
    path = synth.CurveSpec(np.array([[0, 0, -1.0], [0, 0, 0.0], [0, 0, 1.5], [0, 0, 3.0]]), 3)
    prof = synth.CurveSpec(ctrl, 2, False, U, wts)
    r = oracle.sweep(path, prof, nu, nv, want_kappa=False)
    d = np.hypot(r.pos[0], r.pos[1])
    radial = np.stack([r.pos[0] / d, r.pos[1] / d, np.zeros_like(d)])
    sign = np.sign(np.sum(radial[:, 0, 0] * r.nrm[:, 0, 0]))
    # g = the radial direction: every vertex contributes +-1
    assert abs(oracle.loss(path, prof, nu, nv, None, g=radial) - sign * nu * nv) <= 1e-11 * nu * nv
    # the normals do not depend on the radius: scaling the profile control
    # points leaves L_N unchanged
    g = np.random.default_rng(52).standard_normal((3, nu, nv))
    _, gQ = oracle.fd_grad(path, prof, nu, nv, None, g=g, want_path=False)
    assert abs(np.sum(prof.ctrl * gQ)) <= 1e-7 * np.abs(gQ).max() * ctrl.shape[0]
    assert np.abs(gQ).max() > 1e-3


def test_normal_gradient_translation_and_scaling_invariants():
    path, prof, nu, nv, _ = _small(seed=11)
    # a profile off its plane (S_z != 0): with S_z = 0 the normal is the
    # direction of (R S') x t and each curve's scaling alone leaves it as is
    prof.ctrl[:, 2] = 0.15 * np.random.default_rng(54).standard_normal(prof.ctrl.shape[0])
    g = np.random.default_rng(53).standard_normal((3, nu, nv))
    gP, gQ = oracle.fd_grad(path, prof, nu, nv, None, g=g)
    scale = max(np.abs(gP).max(), np.abs(gQ).max())
    assert scale > 1e-2
    # translating the path translates the surface
    assert np.abs(gP.sum(axis=0)).max() <= 1e-7 * scale * path.ctrl.shape[0]
    # scaling path and profile together scales the surface
    total = np.sum(path.ctrl * gP) + np.sum(prof.ctrl * gQ)
    assert abs(total) <= 1e-7 * scale * (np.abs(path.ctrl).sum() + np.abs(prof.ctrl).sum())
    # neither holds for one curve alone
    assert abs(np.sum(path.ctrl * gP)) > 1e-3 * scale
    assert abs(np.sum(prof.ctrl * gQ)) > 1e-3 * scale


# ------------------------------------- knot and weight gradients (FD helper)
# The curve is unchanged when every knot is shifted or scaled together (the
# samples follow the domain) or when every weight is scaled: the gradient of
# any loss satisfies sum_m dL/dU_m = 0, sum_m U_m dL/dU_m = 0 and
# sum_k w_k dL/dw_k = 0.  The first and last knots of a clamped vector do not
# enter the curve at all.

def _knotted(seed, rational=False, nu=48, nv=12):
    rng = np.random.default_rng(seed)
    n, p = 9, 3
    P = synth.random_walk(rng, n)
    inner = np.sort(rng.uniform(0.1, 0.9, n - p - 1))
    U = np.concatenate([np.full(p + 1, 0.2), 0.2 + 1.3 * inner, np.full(p + 1, 1.5)])
    Q = synth.perturbed_circle(rng, 7)
    Q[:, 2] = 0.1 * rng.standard_normal(7)
    path = synth.CurveSpec(P, p, knots=U)
    prof = synth.CurveSpec(Q, 3, True)
    if rational:
        path.weights = rng.uniform(0.5, 2.0, n)
        prof.weights = rng.uniform(0.5, 2.0, 7)
    w = rng.standard_normal((3, nu, nv))
    g = rng.standard_normal((3, nu, nv))
    return path, prof, nu, nv, w, g


def test_knot_gradient_invariants():
    path, prof, nu, nv, w, g = _knotted(31)
    U = path.knots
    p = path.degree
    # interior knots one by one; the clamped end runs moved as a whole
    start, end = list(range(0, p + 1)), list(range(len(U) - p - 1, len(U)))
    groups = [start] + [[k] for k in range(p + 1, len(U) - p - 1)] + [end]
    d = oracle.fd_param_grad(path, prof, nu, nv, w, "path_knots", g=g, groups=groups)
    scale = np.abs(d).max()
    assert scale > 1e-2
    assert abs(d.sum()) <= 1e-6 * scale * len(d)
    vals = np.array([U[grp[0]] for grp in groups])
    assert abs(np.sum(vals * d)) <= 1e-6 * scale * np.abs(vals).sum()
    # the outermost knots do not enter
    ends = oracle.fd_param_grad(path, prof, nu, nv, w, "path_knots", g=g, entries=[0, len(U) - 1])
    assert np.all(ends == 0.0)


def test_weight_gradient_invariant():
    path, prof, nu, nv, w, g = _knotted(32, rational=True)
    for which, c in (("path_weights", path), ("prof_weights", prof)):
        d = oracle.fd_param_grad(path, prof, nu, nv, w, which, g=g)
        scale = np.abs(d).max()
        assert scale > 1e-2
        assert abs(np.sum(c.weights * d)) <= 1e-6 * scale * np.abs(c.weights).sum()


def test_profile_weight_gradient_closed_form():
    # positions only: X is linear in the profile point S, and a rational
    # point moves with its weight as dS/dw_k = N_k (Q_k - S) / W
    # (W = sum_l w_l N_l), so dL/dw_k = sum_j h_j . N_k(v_j) (Q_k - S_j) / W_j
    # with h_j = sum_i R_i^T w_ij.
    path, prof, nu, nv, w, _ = _knotted(33, rational=True)
    d = oracle.fd_param_grad(path, prof, nu, nv, w, "prof_weights")
    r = oracle.sweep(path, prof, nu, nv, want_nrm=False, want_kappa=False)
    h = np.einsum("iab,aij->jb", r.frame, w)
    c = oracle.Curve.of(prof)
    U, q, m = c.knot_vector(), c.degree, c.n
    S, _ = oracle.profile_samples(prof, nv)
    ref = np.zeros(m)
    for j in range(nv):
        v = c.param(j, nv)
        sp = c.span(v)
        N = oracle.basis(U, q, sp, v, nd=0)[0]
        ks = [(sp - q + l) % m for l in range(q + 1)]
        W = sum(prof.weights[k] * N[l] for l, k in enumerate(ks))
        for l, k in enumerate(ks):
            ref[k] += N[l] * (h[j] @ (prof.ctrl[k] - S[j])) / W
    assert np.abs(d - ref).max() <= 1e-7 * np.abs(ref).max()
