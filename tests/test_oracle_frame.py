"""Pins of the oracle's frame and surface (steps O5-O8) against closed forms
and invariants: orthonormality, planar paths (bitwise), straight paths
(exact cylinder), exact circle samples (rotation about the circle's axis by
the arc angle, exact torus), the helix's analytic rotation-minimizing frame
(fourth-order convergence of the double reflection), rigid-motion
equivariance, linearity in the profile, the tangent-reversal and
stationary-point rules, and the normal against finite differences of X."""

import numpy as np
import pytest

import oracle
import synth

rng = np.random.default_rng(77)
EPS = np.finfo(float).eps


def _rot(axis, ang):
    axis = np.asarray(axis, float) / np.linalg.norm(axis)
    K = np.array([[0, -axis[2], axis[1]], [axis[2], 0, -axis[0]], [-axis[1], axis[0], 0]])
    return np.eye(3) + np.sin(ang) * K + (1 - np.cos(ang)) * K @ K


def _frame_of(spec, n_u, n0=None):
    x, d1, d2, ft = oracle.path_samples(spec.path, n_u)
    R, nf = oracle.frame(x, d1, ft, n0)
    return x, d1, d2, R, nf


# ----------------------------------------------------------- invariants

def test_frame_orthonormal_right_handed_tangent_column():
    s = synth.c1()
    x, d1, d2, R, nf = _frame_of(s, 4096)
    assert nf == 0
    G = np.einsum("nji,njk->nik", R, R)
    assert np.abs(G - np.eye(3)).max() < 8 * EPS
    assert np.abs(np.linalg.det(R) - 1).max() < 8 * EPS
    t = d1 / np.linalg.norm(d1, axis=1, keepdims=True)
    assert np.abs(R[:, :, 2] - t).max() == 0.0
    # consecutive frames differ by a rotation taking t_i to t_{i+1}: M_i = R_{i+1} R_i^T
    M = np.einsum("nij,nkj->nik", R[1:], R[:-1])
    assert np.abs(np.einsum("nij,nj->ni", M, t[:-1]) - t[1:]).max() < 16 * EPS


def test_initial_frame_axis_rule_and_user_normal():
    s = synth.c1()
    x, d1, d2, R, _ = _frame_of(s, 64)
    t0 = R[0, :, 2]
    a = int(np.argmin(np.abs(t0)))
    e = np.zeros(3); e[a] = 1
    r0 = e - (e @ t0) * t0
    assert np.abs(R[0, :, 0] - r0 / np.linalg.norm(r0)).max() < 4 * EPS
    n0 = np.array([0.3, -1.0, 2.0])
    _, _, _, R2, _ = _frame_of(s, 64, n0=n0)
    q = n0 - (n0 @ t0) * t0
    assert np.abs(R2[0, :, 0] - q / np.linalg.norm(q)).max() < 4 * EPS
    # a user normal parallel to t0 falls back to the axis rule
    _, _, _, R3, _ = _frame_of(s, 64, n0=5 * t0)
    assert np.abs(R3[0] - R[0]).max() < 4 * EPS


def test_planar_path_keeps_e_z_bitwise():
    n = 40
    P = np.zeros((n, 3))
    P[1:, :2] = np.cumsum(rng.standard_normal((n - 1, 2)), axis=0)
    spec = synth.SweepSpec(synth.CurveSpec(P, 3), synth.CurveSpec(np.zeros((4, 3)), 3, True), 2000, 8)
    x, d1, d2, R, _ = _frame_of(spec, 2000)
    assert (R[:, :, 0] == np.array([0.0, 0.0, 1.0])).all()
    assert (R[:, 2, 1] == 0.0).all() and (R[:, 2, 2] == 0.0).all()


def test_straight_axis_line_constant_frame_bitwise():
    n = 12
    P = np.zeros((n, 3)); P[:, 1] = np.cumsum(rng.uniform(0.1, 1.0, n))
    spec = synth.SweepSpec(synth.CurveSpec(P, 3), synth.CurveSpec(np.zeros((4, 3)), 3, True), 500, 8)
    x, d1, d2, R, _ = _frame_of(spec, 500)
    assert (R == R[0]).all()


def test_cylinder_closed_form():
    # Greville-placed control points on a line: C(u) = p0 + L u e exactly,
    # so X_ij = p0 + L u_i e + R_0 S_j and N_ij = R_0 (S'_y, -S'_x, 0)/|S'|.
    n, p, L = 20, 3, 7.5
    e = np.array([1.0, 2.0, -0.5]); e /= np.linalg.norm(e)
    p0 = np.array([0.25, -1.0, 3.0])
    U = oracle.Curve(np.zeros((n, 3)), p).knot_vector()
    xi = np.array([U[k + 1:k + p + 1].sum() / p for k in range(n)])
    P = p0 + L * xi[:, None] * e
    prof = synth.perturbed_circle(rng, 9)
    nu, nv = 300, 48
    r = oracle.sweep(synth.CurveSpec(P, p), synth.CurveSpec(prof, 3, True), nu, nv)
    u = oracle.Curve(P, p).params(nu)
    S, dS = oracle.profile_samples(synth.CurveSpec(prof, 3, True), nv)
    R0 = r.frame[0]
    assert np.abs(r.frame - R0).max() < 64 * EPS
    X = p0[:, None, None] + L * u[None, :, None] * e[:, None, None] + np.einsum("ab,jb->aj", R0, S)[:, None, :]
    assert np.abs(r.pos - X).max() < 1e-13 * L
    n2 = np.stack([dS[:, 1], -dS[:, 0], np.zeros(nv)], 1)
    n2 /= np.linalg.norm(n2, axis=1, keepdims=True)
    Nref = np.einsum("ab,jb->aj", R0, n2)
    assert np.abs(r.nrm - Nref[:, None, :]).max() < 1e-14
    # outward: away from the axis line
    radial = r.pos - (p0[:, None, None] + L * u[None, :, None] * e[:, None, None])
    assert (np.einsum("aij,aij->ij", radial, r.nrm) > 0).all()


def _tilted_circle(Rad, n_hat, nsamp, th_end):
    n_hat = n_hat / np.linalg.norm(n_hat)
    a = np.cross(n_hat, [1.0, 0.0, 0.0]); a /= np.linalg.norm(a)
    b = np.cross(n_hat, a)
    th = np.linspace(0.0, th_end, nsamp)
    c0 = np.array([0.5, -0.2, 1.0])
    x = c0 + Rad * (np.cos(th)[:, None] * a + np.sin(th)[:, None] * b)
    d1 = Rad * (-np.sin(th)[:, None] * a + np.cos(th)[:, None] * b)
    d2 = -Rad * (np.cos(th)[:, None] * a + np.sin(th)[:, None] * b)
    return th, c0, n_hat, x, d1, d2


def test_exact_circle_frame_rotates_by_arc_angle():
    th, c0, nh, x, d1, d2 = _tilted_circle(2.0, np.array([0.3, 0.4, 0.85]), 257, 1.7 * np.pi)
    R, nf = oracle.frame(x, d1)
    assert nf == 0
    for i in range(0, len(th), 16):
        ref = _rot(nh, th[i] - th[0]) @ R[0]
        assert np.abs(R[i] - ref).max() < 2e-13


def test_exact_torus_section():
    Rad, rho = 2.0, 0.3
    th, c0, nh, x, d1, d2 = _tilted_circle(Rad, np.array([-0.2, 0.9, 0.1]), 180, 1.5 * np.pi)
    phi = 2 * np.pi * np.arange(40) / 40
    S = np.stack([rho * np.cos(phi), rho * np.sin(phi), np.zeros_like(phi)], 1)
    dS = np.stack([-rho * np.sin(phi), rho * np.cos(phi), np.zeros_like(phi)], 1)
    pos, nrm, kap, R = oracle.sweep_from_samples(x, d1, d2, S, dS)
    Y = pos - c0[:, None, None]
    h = np.einsum("a,aij->ij", nh, Y)
    rad = np.sqrt(np.maximum(np.einsum("aij,aij->ij", Y, Y) - h * h, 0))
    assert np.abs((rad - Rad) ** 2 + h ** 2 - rho ** 2).max() < 1e-13
    # normal = (X - nearest point of the centre circle)/rho, pointing outward
    inplane = Y - h[None] * nh[:, None, None]
    centre = Rad * inplane / np.linalg.norm(inplane, axis=0, keepdims=True)
    Nref = (Y - centre) / rho
    assert np.abs(nrm - Nref).max() < 1e-12


def _helix_rmf_error(nsamp, a=1.0, b=0.4, th_end=3.0):
    c = np.hypot(a, b)
    th = np.linspace(0.0, th_end, nsamp)
    x = np.stack([a * np.cos(th), a * np.sin(th), b * th], 1)
    d1 = np.stack([-a * np.sin(th), a * np.cos(th), np.full_like(th, b)], 1)
    R, _ = oracle.frame(x, d1)
    T = d1 / c
    Nf = np.stack([-np.cos(th), -np.sin(th), np.zeros_like(th)], 1)
    Bf = np.cross(T, Nf)
    phi0 = np.arctan2(R[0, :, 0] @ Bf[0], R[0, :, 0] @ Nf[0])
    phi = phi0 - (b / c) * th            # RMF: phi' = -torsion * ds/dtheta
    r = np.cos(phi)[:, None] * Nf + np.sin(phi)[:, None] * Bf
    return np.abs(R[:, :, 0] - r).max()


def test_helix_double_reflection_is_fourth_order():
    e1 = _helix_rmf_error(33)
    e2 = _helix_rmf_error(65)
    e3 = _helix_rmf_error(129)
    assert e1 < 1e-4
    assert 12 < e1 / e2 < 20 and 12 < e2 / e3 < 20, (e1, e2, e3)


def test_rigid_motion_equivariance_and_translation():
    s = synth.c1()
    n0 = np.array([0.2, 0.7, -0.4])
    base = oracle.sweep(s.path, s.profile, 128, 32, n0=n0)
    Qr = _rot([0.3, -0.5, 0.8], 1.1)
    shift = np.array([3.0, -2.0, 0.5])
    moved = oracle.sweep(synth.CurveSpec(s.path.ctrl @ Qr.T + shift, 3), s.profile, 128, 32, n0=Qr @ n0)
    assert np.abs(moved.pos - (np.einsum("ab,bij->aij", Qr, base.pos) + shift[:, None, None])).max() < 1e-12
    assert np.abs(moved.nrm - np.einsum("ab,bij->aij", Qr, base.nrm)).max() < 1e-12


def test_linearity_in_profile():
    s = synth.c1()
    Qa = s.profile.ctrl
    Qb = rng.standard_normal(Qa.shape) * 0.2
    def off(Q):
        r = oracle.sweep(s.path, synth.CurveSpec(Q, 3, True), 96, 24, want_nrm=False, want_kappa=False)
        x, _, _, _ = oracle.path_samples(s.path, 96)
        return r.pos - x.T[:, :, None]
    assert np.abs(off(Qa + Qb) - (off(Qa) + off(Qb))).max() < 1e-14


def test_tangent_reversal_uses_pi_rotation():
    # degree-1 path out along +x and back: at the turn H1 maps t_i onto
    # t_{i+1} = -t_i, so the second reflection is undefined and the step is a
    # rotation by pi about the axis-rule direction of t_i (e_y here)
    P = np.array([[0.0, 0, 0], [1.0, 0, 0], [0.0, 0, 0]])
    x, d1, d2, R, nf = _frame_of(synth.SweepSpec(synth.CurveSpec(P, 1), None, 0, 0), 11)
    assert nf == 1
    first = R[:5]
    assert (first[:, :, 0] == [0, 1, 0]).all() and (first[:, :, 1] == [0, 0, 1]).all()
    last = R[6:]
    assert np.abs(last[:, :, 0] - [0, 1, 0]).max() < 4 * EPS
    assert np.abs(last[:, :, 1] - [0, 0, -1]).max() < 4 * EPS
    assert (last[:, :, 2] == [-1, 0, 0]).all()


def test_stationary_segment_carries_tangent_and_frame():
    P = np.array([[0.0, 0, 0], [1.0, 0.5, 0], [1.0, 0.5, 0], [2.0, 2.0, 1.0]])
    spec = synth.SweepSpec(synth.CurveSpec(P, 1), synth.CurveSpec(synth.perturbed_circle(rng, 6), 2, True), 31, 12)
    x, d1, d2, R, nf = _frame_of(spec, 31)
    zero = np.linalg.norm(d1, axis=1) == 0
    assert zero.any()
    idx = np.where(zero)[0]
    # every stationary sample keeps the frame of the sample before it
    for i in idx:
        assert np.abs(R[i] - R[i - 1]).max() < 4 * EPS
    r = oracle.sweep(spec.path, spec.profile, 31, 12)
    assert (r.nrm[:, idx, :] == 0).all() and np.isinf(r.kappa[idx]).all()


def test_zero_start_tangent_uses_first_leg():
    P = np.array([[1.0, 1.0, 1.0], [1.0, 1.0, 1.0], [2.0, 3.0, 1.0], [4.0, 3.0, 0.0]])
    x, d1, d2, ft = oracle.path_samples(synth.CurveSpec(P, 1), 13)
    assert np.linalg.norm(d1[0]) == 0
    ref = np.array([1.0, 2.0, 0.0]) / np.sqrt(5)
    assert np.abs(ft - ref).max() < 4 * EPS
    R, _ = oracle.frame(x, d1, ft)
    assert np.abs(R[0, :, 2] - ref).max() < 4 * EPS


def test_normal_against_finite_differences_with_focal_region():
    # a tight helix swept by a large, non-planar profile: alpha = |C'| - S.(a,b)
    # changes sign on part of the surface, and S_z != 0 exercises t'
    th = np.linspace(0, 2 * np.pi, 14)
    P = np.stack([0.6 * np.cos(th), 0.6 * np.sin(th), 0.3 * th], 1)
    m = 11
    ang = 2 * np.pi * np.arange(m) / m
    Q = np.stack([0.8 * np.cos(ang), 0.8 * np.sin(ang), 0.25 * np.sin(2 * ang)], 1)
    nu, nv = 6001, 401
    r = oracle.sweep(synth.CurveSpec(P, 3), synth.CurveSpec(Q, 3, True), nu, nv)
    X, N, K = r.pos, r.nrm, r.kappa
    i = np.arange(1, nu - 1, 37)
    j = np.arange(0, nv, 5)
    Xu = (X[:, i + 1][:, :, j] - X[:, i - 1][:, :, j])
    Xv = (X[:, i][:, :, (j + 1) % nv] - X[:, i][:, :, (j - 1) % nv])
    n_ = N[:, i][:, :, j]
    k_ = K[i][:, j]
    good = k_ < 50
    assert good.sum() > 0.8 * good.size
    cu = np.abs(np.einsum("aij,aij->ij", n_, Xu)) / np.linalg.norm(Xu, axis=0)
    cv = np.abs(np.einsum("aij,aij->ij", n_, Xv)) / np.linalg.norm(Xv, axis=0)
    assert cu[good].max() < 1e-3 and cv[good].max() < 1e-3
    orient = np.einsum("aij,aij->ij", n_, np.cross(Xv, Xu, axis=0))
    assert (orient[good] > 0).all()
    # the focal region is really there: some unmasked normals point inward
    x, d1, d2, _ = oracle.path_samples(synth.CurveSpec(P, 3), nu)
    inward = np.einsum("aij,aij->ij", n_, X[:, i][:, :, j] - x[i].T[:, :, None]) < 0
    assert (inward & good).any()
