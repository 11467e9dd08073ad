"""FP64 CPU oracle for dense swept-surface evaluation -- TEST INFRASTRUCTURE.

Only ``tests/``, the smoke check and the bench's CPU-baseline leg may import
this package.  The product library never does, and this package imports
nothing from the product (it shares no code with the HIP path).

NumPy front end over ``sweep_oracle.c`` (built with gcc by ``oracle.build``).
Every array is float64; positions and normals come back as (3, n_u, n_v).

Methods followed (the framing paper defines none; see ``sweep_oracle.c``):
Cox-de Boor B-spline basis and derivatives; clamped uniform and periodic
uniform knots; double-reflection rotation-minimizing frame (Wang, Juettler,
Zheng & Liu 2008); surface X = C + [r s t] S with normal X_v x X_u; central
finite-difference gradient of L = sum w . X.
"""

from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence, Tuple

import numpy as np

from . import build as _build

_lib = None

_dp = C.POINTER(C.c_double)


class _Curve(C.Structure):
    _fields_ = [("n", C.c_int), ("p", C.c_int), ("closed", C.c_int),
                ("ctrl", _dp), ("knots", _dp), ("weights", _dp)]


def lib():
    """Load the oracle library, compiling it first if it is not built."""
    global _lib
    if _lib is None:
        # ORACLE_LIB names another build of sweep_oracle.c (the planted-mistake
        # builds of the pin tests); by default the library next to this file
        path = os.environ.get("ORACLE_LIB") or _build.LIB
        if path == _build.LIB and not os.path.exists(path):
            _build.build()
        L = C.CDLL(path)
        L.or_nbasis.restype = C.c_int
        L.or_nknots.restype = C.c_int
        L.or_knots.restype = None
        L.or_param.restype = C.c_double
        L.or_param.argtypes = [C.c_int, C.c_int, C.c_int, _dp, C.c_int, C.c_int]
        L.or_span.restype = C.c_int
        L.or_span.argtypes = [_dp, C.c_int, C.c_int, C.c_double]
        L.or_basis.restype = None
        L.or_basis.argtypes = [_dp, C.c_int, C.c_int, C.c_double, C.c_int, _dp]
        L.or_curve_eval.restype = None
        L.or_curve_eval.argtypes = [C.POINTER(_Curve), _dp, C.c_double, C.c_int, _dp]
        L.or_curve_samples.restype = None
        L.or_frame.restype = C.c_int
        L.or_surface_rows.restype = None
        L.or_sweep.restype = C.c_int
        L.or_loss.restype = C.c_double
        L.or_fd_grad.restype = None
        L.or_fd_grad.argtypes = [C.POINTER(_Curve), C.POINTER(_Curve), C.c_int, C.c_int,
                                 _dp, _dp, _dp, C.c_double, _dp, _dp]
        L.or_loss.argtypes = [C.POINTER(_Curve), C.POINTER(_Curve), C.c_int, C.c_int, _dp, _dp, _dp]
        L.or_max_threads.restype = C.c_int
        L.or_sweep_ex.restype = C.c_int
        L.or_sweep_ex.argtypes = [C.POINTER(_Curve), C.POINTER(_Curve), C.c_int, C.c_int, _dp, C.c_int, C.c_int,
                                  C.c_void_p, C.c_int, C.c_double, C.c_int, C.c_int, _dp, _dp, _dp, _dp, _dp]
        L.or_arclength_params.restype = C.c_double
        L.or_arclength_params.argtypes = [C.POINTER(_Curve), C.c_int, _dp]
        L.or_monitor_params.restype = C.c_double
        L.or_monitor_params.argtypes = [C.POINTER(_Curve), C.c_int, C.c_double, _dp]
        L.or_curve_samples_at.restype = None
        L.or_triangles.restype = C.c_longlong
        L.or_triangles.argtypes = [C.c_int, C.c_int, C.c_int, C.c_void_p]
        L.or_curve_samples3.restype = None
        L.or_frenet.restype = None
        L.or_surface_rows_ex.restype = None
        _lib = L
    return _lib


def _ptr(a: Optional[np.ndarray]):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_dp)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


class Curve:
    """A B-spline curve: ctrl (n, 3), degree p, closed (periodic uniform) or
    open with clamped uniform knots (knots=None) or the given knot vector;
    with weights (n positive values) a rational (NURBS) curve."""

    def __init__(self, ctrl, degree: int, closed: bool = False, knots=None, weights=None):
        self.ctrl = _f64(ctrl).reshape(-1, 3)
        self.degree = int(degree)
        self.closed = bool(closed)
        self.knots = None if knots is None else _f64(knots)
        self.weights = None if weights is None else _f64(weights).reshape(-1)
        if self.weights is not None and self.weights.shape[0] != self.ctrl.shape[0]:
            raise ValueError("one weight per control point")
        self._c = _Curve(self.ctrl.shape[0], self.degree, int(self.closed),
                         _ptr(self.ctrl), _ptr(self.knots), _ptr(self.weights))

    @classmethod
    def of(cls, spec) -> "Curve":
        """From any object with ctrl/degree/closed/knots(/weights) attributes."""
        if isinstance(spec, Curve):
            return spec
        return cls(spec.ctrl, spec.degree, spec.closed, getattr(spec, "knots", None),
                   getattr(spec, "weights", None))

    @property
    def n(self) -> int:
        return self.ctrl.shape[0]

    @property
    def ref(self):
        return C.byref(self._c)

    def knot_vector(self) -> np.ndarray:
        L = lib()
        nk = L.or_nknots(self.n, self.degree, int(self.closed))
        U = np.empty(nk)
        L.or_knots(self.n, self.degree, int(self.closed), _ptr(self.knots), _ptr(U))
        return U

    def n_basis(self) -> int:
        return lib().or_nbasis(self.n, self.degree, int(self.closed))

    def param(self, i: int, ns: int) -> float:
        U = self.knot_vector()
        return lib().or_param(self.n, self.degree, int(self.closed), _ptr(U), int(i), int(ns))

    def params(self, ns: int) -> np.ndarray:
        U = self.knot_vector()
        L = lib()
        return np.array([L.or_param(self.n, self.degree, int(self.closed), _ptr(U), i, ns)
                         for i in range(ns)])

    def span(self, u: float) -> int:
        U = self.knot_vector()
        return lib().or_span(_ptr(U), self.n_basis(), self.degree, float(u))

    def eval(self, u: float, nd: int = 2) -> np.ndarray:
        """(nd+1, 3): C, C', C'' at parameter u."""
        U = self.knot_vector()
        out = np.empty(9)
        lib().or_curve_eval(self.ref, _ptr(U), float(u), int(nd), _ptr(out))
        return out[: 3 * (nd + 1)].reshape(nd + 1, 3)

    def samples(self, ns: int, nd: int = 2) -> Tuple[np.ndarray, ...]:
        """Sampled points and derivatives at the ns sample parameters."""
        pts = np.empty((ns, 3))
        d1 = np.empty((ns, 3)) if nd >= 1 else None
        d2 = np.empty((ns, 3)) if nd >= 2 else None
        lib().or_curve_samples(self.ref, C.c_int(ns), _ptr(pts), _ptr(d1), _ptr(d2))
        return tuple(a for a in (pts, d1, d2) if a is not None)


def basis(U, p: int, span: int, u: float, nd: int = 2) -> np.ndarray:
    """(nd+1, p+1): D^d N_{span-p+j, p}(u)."""
    U = _f64(U)
    out = np.empty(3 * (p + 1))
    lib().or_basis(_ptr(U), int(p), int(span), float(u), int(nd), _ptr(out))
    return out[: (nd + 1) * (p + 1)].reshape(nd + 1, p + 1)


def frame(x, d1, fallback_t=None, n0=None, reorth: bool = True):
    """Sample-level frame: returns (R (n_u, 3, 3) with columns r, s, t,
    number of tangent-reversal fallbacks)."""
    x, d1 = _f64(x), _f64(d1)
    nu = x.shape[0]
    R = np.empty((nu, 9))
    ft = None if fallback_t is None else _f64(fallback_t)
    n0a = None if n0 is None else _f64(n0)
    nf = lib().or_frame(C.c_int(nu), _ptr(x), _ptr(d1), _ptr(ft), _ptr(n0a), C.c_int(int(reorth)), _ptr(R))
    return R.reshape(nu, 3, 3).transpose(0, 2, 1).copy(), nf


def surface_from_samples(x, d1, d2, R, S, dS, want_kappa: bool = True):
    """Sample-level surface: R (n_u, 3, 3) columns r, s, t.  Returns
    (pos (3,nu,nv), nrm (3,nu,nv), kappa (nu,nv))."""
    x, d1, d2 = _f64(x), _f64(d1), _f64(d2)
    S, dS = _f64(S), _f64(dS)
    nu, nv = x.shape[0], S.shape[0]
    Rr = _f64(np.asarray(R).transpose(0, 2, 1).reshape(nu, 9))
    pos = np.empty((3, nu, nv))
    nrm = np.empty((3, nu, nv))
    kap = np.empty((nu, nv)) if want_kappa else None
    lib().or_surface_rows(C.c_int(nu), C.c_int(nv), C.c_int(0), C.c_int(nu), _ptr(x), _ptr(d1), _ptr(d2),
                          _ptr(Rr), _ptr(S), _ptr(dS), _ptr(pos), _ptr(nrm), _ptr(kap), None, None, None)
    return pos, nrm, kap


def sweep_from_samples(x, d1, d2, S, dS, n0=None, fallback_t=None, reorth: bool = True):
    """Frame + surface from analytic samples (used for closed-form pins)."""
    R, nf = frame(x, d1, fallback_t, n0, reorth)
    pos, nrm, kap = surface_from_samples(x, d1, d2, R, S, dS)
    return pos, nrm, kap, R


class SweepResult:
    def __init__(self, pos, nrm, kappa, frame, n_fallback, rows):
        self.pos, self.nrm, self.kappa, self.frame = pos, nrm, kappa, frame
        self.n_fallback, self.rows = n_fallback, rows


def sweep(path, profile, n_u: int, n_v: int, n0=None, reorth: bool = True,
          rows: Optional[Tuple[int, int]] = None, want_pos=True, want_nrm=True,
          want_kappa=True) -> SweepResult:
    """Whole sweep O1-O8.  pos/nrm are (3, n_u, n_v) over the full grid but
    only rows [rows[0], rows[1]) are filled when ``rows`` is given (the rest
    is left uninitialised).  frame is (n_u, 3, 3) with columns r, s, t."""
    P, Q = Curve.of(path), Curve.of(profile)
    r0, r1 = (0, n_u) if rows is None else rows
    pos = np.empty((3, n_u, n_v)) if want_pos else None
    nrm = np.empty((3, n_u, n_v)) if want_nrm else None
    kap = np.empty((n_u, n_v)) if want_kappa else None
    R = np.empty((n_u, 9))
    n0a = None if n0 is None else _f64(n0)
    nf = lib().or_sweep(P.ref, Q.ref, C.c_int(n_u), C.c_int(n_v), _ptr(n0a), C.c_int(int(reorth)),
                        C.c_int(r0), C.c_int(r1), _ptr(pos), _ptr(nrm), _ptr(kap), _ptr(R))
    if nf < 0:
        raise ValueError("oracle: bad sweep input")
    return SweepResult(pos, nrm, kap, R.reshape(n_u, 3, 3).transpose(0, 2, 1).copy(), nf, (r0, r1))


FRAME_MODES = {"rmf": 0, "frenet": 1}

def frenet(t, d1, d2, d3):
    """Sample-level Frenet frame from tangents t and the first, second and
    third derivatives (each (n, 3)): (R (n, 3, 3) with columns r = n, s = b,
    t; omega (n,))."""
    t, d1, d2, d3 = (_f64(a).reshape(-1, 3) for a in (t, d1, d2, d3))
    n = t.shape[0]
    R = np.zeros((n, 9))
    R[:, 6:9] = t
    om = np.empty(n)
    lib().or_frenet(C.c_int(n), _ptr(d1), _ptr(d2), _ptr(d3), _ptr(R), _ptr(om))
    return R.reshape(n, 3, 3).transpose(0, 2, 1).copy(), om


def surface_ex_from_samples(x, d1, d2, R, omega, law, S, dS):
    """Sample-level surface with a general frame: R (n_u, 3, 3) columns
    r, s, t; omega (n_u,) or None; law (n_u, 4) = (sigma, theta, dsigma/du,
    dtheta/du) or None.  Returns (pos, nrm, kappa)."""
    x, d1, d2, S, dS = (_f64(a) for a in (x, d1, d2, S, dS))
    nu, nv = x.shape[0], S.shape[0]
    Rr = _f64(np.asarray(R).transpose(0, 2, 1).reshape(nu, 9))
    om = None if omega is None else _f64(omega)
    lw = None if law is None else _f64(law)
    pos = np.empty((3, nu, nv))
    nrm = np.empty((3, nu, nv))
    kap = np.empty((nu, nv))
    lib().or_surface_rows_ex(C.c_int(nu), C.c_int(nv), C.c_int(0), C.c_int(nu), _ptr(x), _ptr(d1), _ptr(d2),
                             _ptr(Rr), _ptr(om), _ptr(lw), _ptr(S), _ptr(dS), _ptr(pos), _ptr(nrm), _ptr(kap))
    return pos, nrm, kap



def sweep_ex(path, profile, n_u: int, n_v: int, n0=None, reorth: bool = True, mode: str = "rmf", law=None,
             rows: Optional[Tuple[int, int]] = None, want_kappa=True, arclength: bool = False, lam: float = 0.0):
    """Whole sweep with a frame mode ("rmf" or "frenet") and an optional law
    curve (open curve whose control points hold (scale, twist angle, -)).
    Returns (SweepResult, omega (n_u,))."""
    P, Q = Curve.of(path), Curve.of(profile)
    Lw = None if law is None else Curve.of(law)
    r0, r1 = (0, n_u) if rows is None else rows
    pos = np.empty((3, n_u, n_v))
    nrm = np.empty((3, n_u, n_v))
    kap = np.empty((n_u, n_v)) if want_kappa else None
    R = np.empty((n_u, 9))
    om = np.empty(n_u)
    n0a = None if n0 is None else _f64(n0)
    nf = lib().or_sweep_ex(P.ref, Q.ref, n_u, n_v, _ptr(n0a), int(reorth), FRAME_MODES[mode],
                           None if Lw is None else C.cast(Lw.ref, C.c_void_p), int(bool(arclength)), float(lam), r0, r1,
                           _ptr(pos), _ptr(nrm), _ptr(kap), _ptr(R), _ptr(om))
    if nf < 0:
        raise ValueError("oracle: bad sweep input")
    return SweepResult(pos, nrm, kap, R.reshape(n_u, 3, 3).transpose(0, 2, 1).copy(), nf, (r0, r1)), om


def sweep_rows_ex(path, profile, n_u: int, n_v: int, rows, n0=None, mode: str = "rmf", law=None,
                  arclength: bool = False, lam: float = 0.0):
    """sweep_ex on the listed rows only: (pos (3, len(rows), n_v), nrm,
    kappa (len(rows), n_v))."""
    rows = np.asarray(rows, dtype=np.int64)
    P, Q = Curve.of(path), Curve.of(profile)
    Lw = None if law is None else Curve.of(law)
    pos = np.empty((3, n_u, n_v))
    nrm = np.empty((3, n_u, n_v))
    kap = np.empty((n_u, n_v))
    n0a = None if n0 is None else _f64(n0)
    for i in rows:
        nf = lib().or_sweep_ex(P.ref, Q.ref, n_u, n_v, _ptr(n0a), 1, FRAME_MODES[mode],
                               None if Lw is None else C.cast(Lw.ref, C.c_void_p), int(bool(arclength)), float(lam),
                               int(i),
                               int(i) + 1, _ptr(pos), _ptr(nrm), _ptr(kap), None, None)
        if nf < 0:
            raise ValueError("oracle: bad sweep input")
    return pos[:, rows], nrm[:, rows], kap[rows]


def arclength_params(curve, ns: int, lam: float = 0.0):
    """(u (ns,), total) of the arc-length samples of an open curve, or with
    lam > 0 of the curvature-adaptive samples (total = arc length + lam x
    turning angle)."""
    c = Curve.of(curve)
    u = np.empty(ns)
    total = (lib().or_arclength_params(c.ref, int(ns), _ptr(u)) if lam == 0.0
             else lib().or_monitor_params(c.ref, int(ns), float(lam), _ptr(u)))
    if total < 0:
        raise ValueError("arc-length sampling needs an open curve")
    return u, total


def curve_at(curve, u, nd: int = 2):
    """Points and derivatives (nd+1 arrays (n, 3)) at the given parameters."""
    c = Curve.of(curve)
    u = _f64(u)
    n = u.shape[0]
    outs = [np.empty((n, 3)) for _ in range(4)]
    ptrs = [_ptr(outs[0])] + [_ptr(outs[d]) if d <= nd else None for d in (1, 2, 3)]
    lib().or_curve_samples_at(c.ref, C.c_int(n), _ptr(u), *ptrs)
    return outs[: nd + 1]


def triangles(n_u: int, n_v: int, closed_v: bool) -> np.ndarray:
    """(T, 3) int32 triangle list of the grid (see or_triangles)."""
    t = lib().or_triangles(int(n_u), int(n_v), int(bool(closed_v)), None)
    tri = np.empty((t, 3), np.int32)
    lib().or_triangles(int(n_u), int(n_v), int(bool(closed_v)), tri.ctypes.data_as(C.c_void_p))
    return tri


def sweep_rows(path, profile, n_u: int, n_v: int, rows, n0=None, reorth: bool = True):
    """Frame over all n_u samples, surface only on the listed rows.
    Returns (pos (3, len(rows), n_v), nrm, kappa (len(rows), n_v), frame
    (n_u, 3, 3))."""
    rows = np.asarray(rows, dtype=np.int64)
    x, d1, d2, ft = path_samples(path, n_u)
    S, dS = profile_samples(profile, n_v)
    R, _ = frame(x, d1, ft, n0, reorth)
    pos, nrm, kap = surface_from_samples(x[rows], d1[rows], d2[rows], R[rows], S, dS)
    return pos, nrm, kap, R


def path_samples(path, n_u: int):
    """(x, C', C'', fallback tangent) of the path at the n_u u-samples."""
    P = Curve.of(path)
    x, d1, d2 = (np.empty((n_u, 3)) for _ in range(3))
    ft = np.empty(3)
    lib().or_path_samples(P.ref, C.c_int(n_u), _ptr(x), _ptr(d1), _ptr(d2), _ptr(ft))
    return x, d1, d2, ft


def profile_samples(profile, n_v: int):
    """(S, S') of the profile at the n_v v-samples."""
    return Curve.of(profile).samples(n_v, nd=1)


def _grid_weights(a, n_u: int, n_v: int):
    if a is None:
        return None
    a = _f64(a)
    assert a.shape == (3, n_u, n_v)
    return a


def loss(path, profile, n_u: int, n_v: int, w, n0=None, g=None) -> float:
    """L = sum w . X + sum g . N, w and g shaped (3, n_u, n_v) (either may
    be None: that term is left out)."""
    P, Q = Curve.of(path), Curve.of(profile)
    w, g = _grid_weights(w, n_u, n_v), _grid_weights(g, n_u, n_v)
    n0a = None if n0 is None else _f64(n0)
    return lib().or_loss(P.ref, Q.ref, n_u, n_v, _ptr(n0a), _ptr(w), _ptr(g))


def fd_grad(path, profile, n_u: int, n_v: int, w, h: float = 1e-6, n0=None,
            want_path=True, want_profile=True, g=None):
    """Central-difference gradient of L = sum w . X + sum g . N with respect
    to the path and profile control points: (gP (n_path, 3), gQ (n_prof, 3))."""
    P, Q = Curve.of(path), Curve.of(profile)
    w, g = _grid_weights(w, n_u, n_v), _grid_weights(g, n_u, n_v)
    gP = np.zeros((P.n, 3)) if want_path else None
    gQ = np.zeros((Q.n, 3)) if want_profile else None
    n0a = None if n0 is None else _f64(n0)
    lib().or_fd_grad(P.ref, Q.ref, n_u, n_v, _ptr(n0a), _ptr(w), _ptr(g), float(h), _ptr(gP), _ptr(gQ))
    return gP, gQ


def fd_param_grad(path, profile, n_u: int, n_v: int, w, which: str, g=None, h: float = 1e-6, n0=None,
                  entries=None, groups=None):
    """Central-difference gradient of L = sum w . X + sum g . N with respect to
    the knot vector or the weights of one curve: which is "path_knots",
    "prof_knots" (open curves with given knots), "path_weights" or
    "prof_weights" (rational curves).  entries: the indices to perturb
    (default all); groups: lists of indices moved together by the same h
    (the result has one value per group).  Returns a float64 array."""
    curve_name, part = which.split("_")
    base = path if curve_name == "path" else profile
    vec = _f64(base.knots if part == "knots" else base.weights).copy()
    if groups is None:
        idx = range(vec.shape[0]) if entries is None else entries
        groups = [[k] for k in idx]

    def L_at(v):
        c = Curve(base.ctrl, base.degree, base.closed, v if part == "knots" else base.knots,
                  v if part == "weights" else getattr(base, "weights", None))
        return loss(c if curve_name == "path" else path, c if curve_name == "prof" else profile, n_u, n_v, w,
                    n0=n0, g=g)

    out = np.empty(len(groups))
    for q, grp in enumerate(groups):
        vp, vm = vec.copy(), vec.copy()
        vp[list(grp)] += h
        vm[list(grp)] -= h
        out[q] = (L_at(vp) - L_at(vm)) / (2.0 * h)
    return out


def max_threads() -> int:
    return lib().or_max_threads()


# ------------------------------------------------------------ parity metrics

def bbox_diag(pos: np.ndarray) -> float:
    """Diagonal of the axis-aligned bounding box of positions (3, ...)."""
    p = pos.reshape(3, -1)
    return float(np.linalg.norm(p.max(axis=1) - p.min(axis=1)))


def compare(pos_ref, nrm_ref, kappa_ref, pos, nrm, diag: float, kappa_max: float, kappa_wc: float = 10.0):
    """Parity figures of a result against the oracle on the same vertices:
    position error relative to the bounding-box diagonal (all vertices);
    normal error scaled by max(1, kappa) on vertices with kappa <= kappa_max
    (nrm_scaled); the plain normal error on the same vertices (nrm_abs) and
    on the well-conditioned ones, kappa <= kappa_wc (nrm_abs_wc, with their
    fraction wc_frac); and the count of masked vertices (kappa > kappa_max)."""
    dpos = np.abs(np.asarray(pos, np.float64) - pos_ref).max() / diag
    out = {"pos_rel": float(dpos)}
    if nrm is not None:
        mask = np.isfinite(kappa_ref) & (kappa_ref <= kappa_max)
        wc = mask & (kappa_ref <= kappa_wc)
        dn = np.linalg.norm(np.asarray(nrm, np.float64) - nrm_ref, axis=0)
        scaled = dn / np.maximum(1.0, np.where(mask, kappa_ref, 1.0))
        out["nrm_scaled"] = float(scaled[mask].max()) if mask.any() else 0.0
        out["nrm_abs"] = float(dn[mask].max()) if mask.any() else 0.0
        out["nrm_abs_wc"] = float(dn[wc].max()) if wc.any() else 0.0
        out["wc_frac"] = float(wc.mean())
        out["masked"] = int((~mask).sum())
    return out
