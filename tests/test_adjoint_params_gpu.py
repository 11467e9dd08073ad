"""Knot and weight gradients (next-row f3): sweep_backward_ex with
sweep_param_grads against the oracle's FP64 central differences
(Richardson-extrapolated, h = 2e-6 and 1e-6) of L = sum w . X + sum g . N
with respect to every interior knot, the clamped end runs moved as a whole,
and every weight of rational paths and profiles (closed profiles wrap their
weights); the knot shift/scale and weight scale invariants on every sweep;
the outermost knots get exactly 0."""

import numpy as np
import pytest
import torch

import oracle
import synth
from paper_1110_5450_amd import api
from tests.gpu_util import say

pytestmark = pytest.mark.gpu


def _fd(s, w, g, which, **kw):
    a = oracle.fd_param_grad(s.path, s.profile, s.n_u, s.n_v, w, which, g=g, h=2e-6, **kw)
    b = oracle.fd_param_grad(s.path, s.profile, s.n_u, s.n_v, w, which, g=g, h=1e-6, **kw)
    return (4 * b - a) / 3


def _knots(rng, n, p, a=0.0, b=1.0):
    inner = np.sort(rng.uniform(0.05, 0.95, n - p - 1))
    return np.concatenate([np.full(p + 1, a), a + (b - a) * inner, np.full(p + 1, b)])


def _specs(seed, open_profiles=False, rational=False):
    rng = np.random.default_rng(seed)
    specs = []
    for k, (p, q, n_u, n_v) in enumerate([(3, 3, 200, 24), (2, 2, 130, 17), (5, 3, 90, 31), (1, 2, 70, 12)]):
        n = max(p + 1, 11)
        P = synth.random_walk(rng, n)
        path = synth.CurveSpec(P, p, knots=_knots(rng, n, p, -0.3 * k, 1.0 + 0.5 * k))
        m = max(q + 1, 8)
        if open_profiles:
            Q = np.stack([np.linspace(-0.4, 0.4, m), 0.2 * np.sin(np.arange(m)), 0.1 * np.cos(np.arange(m))], 1)
            prof = synth.CurveSpec(Q, q, False, _knots(rng, m, q, 0.1, 2.0))
        else:
            Q = synth.perturbed_circle(rng, m)
            Q[:, 2] = 0.1 * rng.standard_normal(m)
            prof = synth.CurveSpec(Q, q, True)
        if rational:
            path.weights = rng.uniform(0.5, 2.0, n)
            prof.weights = rng.uniform(0.5, 2.0, m)
        specs.append(synth.SweepSpec(path, prof, n_u, n_v))
    return specs


def _run(specs, names, seed=71):
    b = api.Batch.from_specs(specs)
    rng = np.random.default_rng(seed)
    ws = [rng.standard_normal((3, s.n_u, s.n_v)) for s in specs]
    gs = [rng.standard_normal((3, s.n_u, s.n_v)) for s in specs]
    gP, gQ, ex = api.sweep_backward(b, b.pack(ws, torch.float64), grad_nrm=b.pack(gs, torch.float64),
                                    params=names)
    torch.cuda.synchronize()
    return b, ws, gs, {k: v.cpu().numpy() for k, v in ex.items()}


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _knot_check(b, s, k, kg, w, g, which, tol):
    U = (s.path if which == "path_knots" else s.profile).knots
    p = (s.path if which == "path_knots" else s.profile).degree
    start, end = list(range(p + 1)), list(range(len(U) - p - 1, len(U)))
    groups = [start] + [[m] for m in range(p + 1, len(U) - p - 1)] + [end]
    ref = _fd(s, w, g, which, groups=groups)
    got = np.array([kg[grp].sum() for grp in groups])
    e = _rel(got, ref)
    say(f"   sweep {k} {which}: rel {e:.2e} (|grad| {np.abs(ref).max():.3g})")
    assert e <= tol, (k, which, e, got, ref)
    assert kg[0] == 0.0 and kg[-1] == 0.0
    # the curve is unchanged when every knot is shifted or scaled together
    scale = np.abs(kg).max()
    assert abs(kg.sum()) <= 1e-10 * scale * len(kg)
    assert abs(np.sum(U * kg)) <= 1e-10 * scale * np.abs(U).sum()
    return e


def test_path_knot_gradients_against_fd():
    specs = _specs(81)
    say(f"[case] path knot gradients, {len(specs)} sweeps")
    b, ws, gs, ex = _run(specs, ["path_knots"])
    for k, s in enumerate(specs):
        _knot_check(b, s, k, ex["path_knots"][b.path_knot_slice(k)], ws[k], gs[k], "path_knots", 1e-6)


def test_profile_knot_gradients_against_fd():
    specs = _specs(82, open_profiles=True)
    say(f"[case] path and open-profile knot gradients, {len(specs)} sweeps")
    b, ws, gs, ex = _run(specs, ["path_knots", "prof_knots"])
    for k, s in enumerate(specs):
        _knot_check(b, s, k, ex["prof_knots"][b.prof_knot_slice(k)], ws[k], gs[k], "prof_knots", 1e-6)
        _knot_check(b, s, k, ex["path_knots"][b.path_knot_slice(k)], ws[k], gs[k], "path_knots", 1e-6)


@pytest.mark.parametrize("open_profiles", [False, True])
def test_weight_gradients_against_fd(open_profiles):
    specs = _specs(83 + open_profiles, open_profiles=open_profiles, rational=True)
    say(f"[case] weight gradients (rational), open profiles {open_profiles}")
    names = ["path_weights", "prof_weights", "path_knots"] + (["prof_knots"] if open_profiles else [])
    b, ws, gs, ex = _run(specs, names)
    for k, s in enumerate(specs):
        for which, sl, c in (("path_weights", b.path_slice(k), s.path), ("prof_weights", b.prof_slice(k), s.profile)):
            got = ex[which][sl]
            ref = _fd(s, ws[k], gs[k], which)
            e = _rel(got, ref)
            say(f"   sweep {k} {which}: rel {e:.2e}")
            assert e <= 1e-6, (k, which, e)
            # scaling every weight leaves the curve unchanged
            assert abs(np.sum(c.weights * got)) <= 1e-10 * np.abs(got).max() * np.abs(c.weights).sum()
        _knot_check(b, s, k, ex["path_knots"][b.path_knot_slice(k)], ws[k], gs[k], "path_knots", 1e-6)


def test_parameter_gradients_leave_control_point_gradients_unchanged():
    specs = _specs(85, rational=True)
    b = api.Batch.from_specs(specs)
    rng = np.random.default_rng(72)
    g = b.pack([rng.standard_normal((3, s.n_u, s.n_v)) for s in specs], torch.float64)
    a = api.sweep_backward(b, g, grad_nrm=g)
    c = api.sweep_backward(b, g, grad_nrm=g, params=["path_knots", "path_weights", "prof_weights"])
    torch.cuda.synchronize()
    assert torch.equal(a[0], c[0]) and torch.equal(a[1], c[1])


def test_parameter_gradients_need_the_batch_fields():
    specs = _specs(86)
    for s in specs:
        s.path.knots = None
    b = api.Batch.from_specs(specs)
    g = torch.zeros(b.out_elems, dtype=torch.float64, device="cuda")
    for name in ("path_knots", "prof_knots", "path_weights", "prof_weights"):
        with pytest.raises(ValueError, match="need"):
            api.sweep_backward(b, g, params=[name])
