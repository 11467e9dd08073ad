"""Dense swept-surface evaluation on AMD Instinct MI355X (gfx950).

A B-spline profile S is swept along a B-spline path C with the
rotation-minimizing frame of the double-reflection method (Wang, Juettler,
Zheng & Liu, ACM TOG 2008); vertex positions and normals are written on a
(u, v) grid by hand-written HIP kernels behind the C ABI of
``include/sweep.h`` (``libsweep.so``).  This package is the thin Python
binding: ``_lib`` mirrors the C entry points, ``api`` wraps them for torch
tensors, ``autograd`` provides the differentiable form.
"""

from ._lib import SweepError, lib  # noqa: F401
from .api import sweep_eval, make_options, eval_workspace_size  # noqa: F401

__all__ = ["SweepError", "lib", "sweep_eval", "make_options", "eval_workspace_size"]
