"""Seeded synthetic sweep inputs shared by the tests, the bench and the oracle.

This module only draws inputs (control points, grid sizes, loss weights) with
NumPy's PCG64 generator; it contains none of the sweep arithmetic (no knots,
no basis functions, no frames).  The same function with the same seed always
returns the same arrays.

Workloads (sizes and distributions of the five configurations the library is
measured on):

* ``c1`` plain single sweep: cubic clamped path with 16 control points drawn
  as a 3-D random walk with N(0, I) steps starting at the origin; closed cubic
  periodic profile with 8 control points on a circle of radius 0.3 whose radii
  are perturbed uniformly by +-10 %; grid 256 x 64; FP64 output.
* ``c2`` large single sweep: 1024 path / 64 profile control points, grid
  65536 x 1024 (67,108,864 vertices); FP32 output with FP64 frame scan.
* ``c2_rational`` the same curves with weights U(0.5, 2) (NURBS).
* ``c3`` precision study: the ``c1`` path and profile at 1,048,576 x 32.
* ``c4`` batched: 4096 sweeps; path counts uniform in [8, 512], profile counts
  uniform in [4, 64], path and profile degree each uniform in {2, 3}, n_u
  log-uniform in [16, 4096], n_v log-uniform in [8, 256]; FP32 output.
* ``c5`` differentiation: 256 sweeps, 64 path / 16 profile control points,
  grid 1024 x 64, FP32; loss weights w ~ N(0, 1) with the shape of the
  position output.

Draw order for one sweep: path steps, then profile radii.  For a batch: all
per-sweep scalars first (path count, profile count, path degree, profile
degree, n_u, n_v for every sweep), then the geometry of sweep 0, 1, ...
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

__all__ = [
    "CurveSpec", "SweepSpec", "random_walk", "perturbed_circle", "single",
    "config", "c1", "c2", "c2_rational", "sweep_law", "c3", "c4", "c5", "loss_weights",
]


@dataclass
class CurveSpec:
    """A B-spline curve as the boundary takes it: control points (n x 3,
    float64, row-major), degree, closed flag (periodic uniform), optional
    user knot vector (open curves only) and optional weights (n positive
    values: a rational curve)."""

    ctrl: np.ndarray
    degree: int
    closed: bool = False
    knots: Optional[np.ndarray] = None
    weights: Optional[np.ndarray] = None

    @property
    def n(self) -> int:
        return int(self.ctrl.shape[0])


@dataclass
class SweepSpec:
    path: CurveSpec
    profile: CurveSpec
    n_u: int
    n_v: int

    @property
    def n_vertices(self) -> int:
        return self.n_u * self.n_v


def random_walk(rng: np.random.Generator, n: int) -> np.ndarray:
    """P_0 = 0, P_{k+1} = P_k + xi_k with xi_k ~ N(0, I_3)."""
    steps = rng.standard_normal((n - 1, 3))
    pts = np.zeros((n, 3), dtype=np.float64)
    pts[1:] = np.cumsum(steps, axis=0)
    return pts


def perturbed_circle(rng: np.random.Generator, m: int, radius: float = 0.3,
                     jitter: float = 0.1) -> np.ndarray:
    """m points at equal angles 2*pi*l/m (counter-clockwise, z = 0) with radii
    radius * (1 + U(-jitter, jitter)); no angular jitter."""
    radii = radius * (1.0 + rng.uniform(-jitter, jitter, size=m))
    ang = 2.0 * np.pi * np.arange(m) / m
    return np.stack([radii * np.cos(ang), radii * np.sin(ang), np.zeros(m)], axis=1)


def single(seed: int, n_path: int, n_prof: int, n_u: int, n_v: int,
           p_path: int = 3, p_prof: int = 3) -> SweepSpec:
    """One open path (random walk) and one closed profile (perturbed circle)
    drawn from the seed."""
    rng = np.random.default_rng(seed)
    path = random_walk(rng, n_path)
    prof = perturbed_circle(rng, n_prof)
    return SweepSpec(CurveSpec(path, p_path, False), CurveSpec(prof, p_prof, True), n_u, n_v)


def c1() -> SweepSpec:
    return single(1, 16, 8, 256, 64)


def c2(n_u: int = 65536, n_v: int = 1024) -> SweepSpec:
    return single(2, 1024, 64, n_u, n_v)


def c2_rational(n_u: int = 65536, n_v: int = 1024, seed: int = 22) -> SweepSpec:
    """The large sweep's curves made rational: weights U(0.5, 2) per control
    point (path first, then profile)."""
    s = c2(n_u, n_v)
    rng = np.random.default_rng(seed)
    s.path.weights = rng.uniform(0.5, 2.0, s.path.n)
    s.profile.weights = rng.uniform(0.5, 2.0, s.profile.n)
    return s


def sweep_law(n: int = 16, degree: int = 3, seed: int = 23) -> CurveSpec:
    """A sweep law along the path: control points (sigma, theta, 0) with
    scale sigma ~ U(0.8, 1.2) and twist angle theta a random walk with
    U(-0.5, 0.5) radian steps."""
    rng = np.random.default_rng(seed)
    ctrl = np.zeros((n, 3))
    ctrl[:, 0] = rng.uniform(0.8, 1.2, n)
    ctrl[:, 1] = np.cumsum(rng.uniform(-0.5, 0.5, n))
    return CurveSpec(ctrl, degree)


def c3(n_u: int = 1048576, n_v: int = 32) -> SweepSpec:
    s = c1()
    return SweepSpec(s.path, s.profile, n_u, n_v)


def _log_uniform_int(rng, lo, hi, size):
    x = np.exp(rng.uniform(np.log(lo), np.log(hi), size=size))
    return np.clip(np.rint(x), lo, hi).astype(np.int64)


def c4(n_sweeps: int = 4096, seed: int = 4, u_range=(16, 4096), v_range=(8, 256),
       path_range=(8, 512), prof_range=(4, 64)) -> List[SweepSpec]:
    rng = np.random.default_rng(seed)
    n_path = rng.integers(path_range[0], path_range[1] + 1, size=n_sweeps)
    n_prof = rng.integers(prof_range[0], prof_range[1] + 1, size=n_sweeps)
    p_path = rng.integers(2, 4, size=n_sweeps)
    p_prof = rng.integers(2, 4, size=n_sweeps)
    n_u = _log_uniform_int(rng, u_range[0], u_range[1], n_sweeps)
    n_v = _log_uniform_int(rng, v_range[0], v_range[1], n_sweeps)
    out = []
    for k in range(n_sweeps):
        path = random_walk(rng, int(n_path[k]))
        prof = perturbed_circle(rng, int(n_prof[k]))
        out.append(SweepSpec(CurveSpec(path, int(p_path[k]), False),
                             CurveSpec(prof, int(p_prof[k]), True),
                             int(n_u[k]), int(n_v[k])))
    return out


def c5(n_sweeps: int = 256, seed: int = 5, n_u: int = 1024, n_v: int = 64) -> List[SweepSpec]:
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n_sweeps):
        path = random_walk(rng, 64)
        prof = perturbed_circle(rng, 16)
        out.append(SweepSpec(CurveSpec(path, 3, False), CurveSpec(prof, 3, True), n_u, n_v))
    return out


def loss_weights(sweeps: List[SweepSpec], seed: int = 55) -> List[np.ndarray]:
    """One N(0,1) weight per vertex and component, shaped like the position
    output of each sweep: (3, n_u, n_v)."""
    rng = np.random.default_rng(seed)
    return [rng.standard_normal((3, s.n_u, s.n_v)) for s in sweeps]


def config(name: str):
    return {"c1": c1, "c2": c2, "c3": c3, "c4": c4, "c5": c5}[name]()
