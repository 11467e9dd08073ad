"""Batched evaluation (profile, per-degree frame and surface launches,
replayed from a HIP graph): every sweep's block agrees with evaluating that
sweep alone (to rounding), matches the oracle, survives
repeated replays with pointer changes, and every sweep of the full
4096-sweep batch matches the oracle."""

import numpy as np
import pytest
import torch

import oracle
import synth
from paper_1110_5450_amd import _lib, api
from tests.gpu_util import TOL, check_full, dev_ctrl, gpu_sweep, parity, say

pytestmark = pytest.mark.gpu


def _mixed(seed=0, n=24):
    rng = np.random.default_rng(seed)
    specs = []
    for k in range(n):
        p = int(rng.integers(1, 8))
        q = int(rng.integers(1, 5))
        n_path = int(rng.integers(p + 1, 60))
        m = int(rng.integers(q + 1, 20))
        P = synth.random_walk(rng, n_path)
        closed = k % 5 != 3
        if closed:
            Q = synth.perturbed_circle(rng, m)
        else:
            Q = np.stack([np.linspace(-0.4, 0.4, m), 0.2 * np.sin(np.arange(m)), 0.05 * np.cos(np.arange(m))], 1)
        n_u = int(rng.choice([2, 3, 17, 255, 256, 257, 700, 1500]))
        n_v = int(rng.choice([3, 8, 31, 64, 100, 257]))
        specs.append(synth.SweepSpec(synth.CurveSpec(P, p), synth.CurveSpec(Q, q, closed), n_u, n_v))
    return specs


# Batched vs single: the batched frame kernels split a sweep's samples into
# runs differently (one wave per sweep up to 256 u-samples with runs of up to
# 4 per lane, one block with runs of 2 to 16 above that) from the
# single-sweep kernels (runs of 1 per thread below 131,072 samples), so the
# rotation products are associated differently and the two agree to
# rounding.
_CLOSE = {torch.float64: 1e-13, torch.float32: 1e-6}


@pytest.mark.parametrize("out_dtype", [torch.float32, torch.float64])
def test_batched_equals_single(out_dtype):
    specs = _mixed(1)
    say(f"[case] mixed batch of {len(specs)} out={out_dtype}")
    b = api.Batch.from_specs(specs)
    pos, nrm = api.sweep_eval_batched(b, out_dtype=out_dtype)
    torch.cuda.synchronize()
    for k, s in enumerate(specs):
        p1, n1 = gpu_sweep(s, out_dtype, tile_config=13)
        torch.cuda.synchronize()
        pb, nb = b.view(pos, k), b.view(nrm, k)
        ref = oracle.sweep(s.path, s.profile, s.n_u, s.n_v)
        ok, r = parity(p1.cpu().numpy(), n1.cpu().numpy(), ref.kappa, pb.cpu().numpy(), nb.cpu().numpy(),
                       _CLOSE[out_dtype])
        assert ok, (k, r)


def test_batched_padded_layout_zeroes_padding():
    specs = _mixed(4, n=12)
    b = api.Batch.from_specs(specs)
    say(f"[case] padded layout, {len(specs)} sweeps, {b.out_elems} elements")
    assert b.out_elems == _lib.sweep_batched_output_elems(b.c_struct())
    pos = torch.full((b.out_elems,), float("nan"), device="cuda")
    nrm = torch.full((b.out_elems,), float("nan"), device="cuda")
    api.sweep_eval_batched(b, out=(pos, nrm))
    torch.cuda.synchronize()
    mask = torch.ones(b.out_elems, dtype=torch.bool)
    for k, s in enumerate(specs):
        o, P, N = int(b.offsets[k]), int(b.plane[k]), s.n_u * s.n_v
        for c in range(3):
            mask[o + c * P: o + c * P + N] = False
    mask = mask.cuda()
    assert int(mask.sum()) == b.out_elems - 3 * b.n_vertices
    assert torch.all(pos[mask] == 0) and torch.all(nrm[mask] == 0)
    assert not torch.isnan(pos).any()


def test_batched_matches_oracle_and_replays():
    specs = _mixed(2, n=10)
    b = api.Batch.from_specs(specs)
    ws = torch.empty(api.batched_workspace_size(b, torch.float64), dtype=torch.uint8, device="cuda")
    outs = []
    for rep in range(3):
        # a new output buffer each replay: the graph's pointer arguments are updated
        pos, nrm = api.sweep_eval_batched(b, out_dtype=torch.float64, workspace=ws)
        torch.cuda.synchronize()
        outs.append((pos.clone(), nrm.clone()))
        del pos, nrm
    for rep in range(1, 3):
        assert torch.equal(outs[rep][0], outs[0][0]) and torch.equal(outs[rep][1], outs[0][1])
    pos, nrm = outs[0]
    for k, s in enumerate(specs):
        ref = oracle.sweep(s.path, s.profile, s.n_u, s.n_v)
        ok, r = parity(ref.pos, ref.nrm, ref.kappa, b.view(pos, k).cpu().numpy(), b.view(nrm, k).cpu().numpy(),
                       TOL[torch.float64])
        say(f"   sweep {k}: {r}")
        assert ok, (k, r)


def test_batched_user_knots_and_precision_variants():
    rng = np.random.default_rng(9)
    specs = []
    for k in range(6):
        P = synth.random_walk(rng, 9)
        U = np.array([0, 0, 0, 0, .1, .1, .45, .7, .7, 1, 1, 1, 1], float) * (1 + k)
        Q = synth.perturbed_circle(rng, 8)
        specs.append(synth.SweepSpec(synth.CurveSpec(P, 3, knots=U), synth.CurveSpec(Q, 3, True), 300 + 7 * k, 20 + k))
    b = api.Batch.from_specs(specs)
    for frame_dtype, reorth, tol in [(torch.float64, True, 1e-12), (torch.float32, True, 1e-4), (torch.float64, False, 1e-11)]:
        pos, nrm = api.sweep_eval_batched(b, out_dtype=torch.float64, frame_dtype=frame_dtype, reorthonormalize=reorth)
        torch.cuda.synchronize()
        for k, s in enumerate(specs):
            ref = oracle.sweep(s.path, s.profile, s.n_u, s.n_v)
            ok, r = parity(ref.pos, ref.nrm, ref.kappa, b.view(pos, k).cpu().numpy(), b.view(nrm, k).cpu().numpy(), tol)
            assert ok, (frame_dtype, reorth, k, r)


def test_batched_chunk_counts_and_every_degree():
    # Every path degree at every length: sweeps of one chunk of runs (up to
    # 4096 u-samples: 200, 1000, 2700) and of two and three chunks (4097,
    # 9000: the chunk-walking frame kernel), interleaved, and four with
    # stationary stretches; two replays agree
    # bitwise.  The oracle multiplies the step rotations in sequence, the GPU
    # in runs and a block scan: FP64 agreement to 8 n eps for long sweeps.
    rng = np.random.default_rng(12)
    specs = []
    for k in range(35):
        p, n_u = 1 + k % 7, [200, 1000, 2700, 4097, 9000][k % 5]
        P = synth.random_walk(rng, int(rng.integers(p + 1, 40)))
        Q = synth.perturbed_circle(rng, int(rng.integers(4, 12)))
        specs.append(synth.SweepSpec(synth.CurveSpec(P, p), synth.CurveSpec(Q, 3, True), n_u, 7 + k % 5))
    # stationary stretches (repeated control points of a degree-1 path): runs
    # whose first sample has C' = 0 take the carried tangent, in the
    # one-wave, one-block and chunk-walking kernels
    for n_u in (300, 1000, 3000, 5000):
        P = synth.random_walk(rng, 12)
        P[4] = P[3]
        P[11] = P[10]
        Q = synth.perturbed_circle(rng, 7)
        specs.append(synth.SweepSpec(synth.CurveSpec(P, 1), synth.CurveSpec(Q, 3, True), n_u, 8))
    b = api.Batch.from_specs(specs)
    say(f"[case] every length and degree: {len(specs)} sweeps")
    pos, nrm = api.sweep_eval_batched(b, out_dtype=torch.float64)
    again = api.sweep_eval_batched(b, out_dtype=torch.float64)
    torch.cuda.synchronize()
    assert torch.equal(pos, again[0]) and torch.equal(nrm, again[1])
    for k, s in enumerate(specs):
        ref = oracle.sweep(s.path, s.profile, s.n_u, s.n_v)
        tol = max(TOL[torch.float64], 8 * s.n_u * np.finfo(float).eps)
        ok, r = parity(ref.pos, ref.nrm, ref.kappa, b.view(pos, k).cpu().numpy(), b.view(nrm, k).cpu().numpy(), tol)
        say(f"   sweep {k} ({s.n_u}x{s.n_v}, p={s.path.degree}): {r}")
        assert ok, (k, r)


def _host_view(b, flat, k):
    o, nu, nv, P = int(b.offsets[k]), int(b.n_u[k]), int(b.n_v[k]), int(b.plane[k])
    return flat[o: o + 3 * P].reshape(3, P)[:, :nu * nv].reshape(3, nu, nv)


def test_full_batch_every_sweep():
    """All 4,096 sweeps of the batch workload (FP32) against the oracle, each
    with its own bounding-box diagonal; the plane padding is zero."""
    specs = synth.c4()
    b = api.Batch.from_specs(specs)
    say(f"[case] full batch: {len(specs)} sweeps, {b.n_vertices} vertices")
    pos, nrm = api.sweep_eval_batched(b)
    torch.cuda.synchronize()
    hp, hn = pos.cpu().numpy(), nrm.cpu().numpy()
    del pos, nrm
    torch.cuda.empty_cache()
    worst = {"pos_rel": 0.0, "nrm_scaled": 0.0, "nrm_abs_wc": 0.0, "masked": 0}
    for k, s in enumerate(specs):
        ref = oracle.sweep(s.path, s.profile, s.n_u, s.n_v)
        ok, r = parity(ref.pos, ref.nrm, ref.kappa, _host_view(b, hp, k), _host_view(b, hn, k), TOL[torch.float32])
        assert ok, (k, s.n_u, s.n_v, s.path.degree, s.profile.degree, r)
        for key in ("pos_rel", "nrm_scaled", "nrm_abs_wc"):
            worst[key] = max(worst[key], r[key])
        worst["masked"] += r["masked"]
        o, N, P = int(b.offsets[k]), int(b.n_u[k] * b.n_v[k]), int(b.plane[k])
        for c in range(3):
            assert not hp[o + c * P + N: o + (c + 1) * P].any() and not hn[o + c * P + N: o + (c + 1) * P].any(), k
    say(f"    every sweep: {worst}")


def test_batched_validation_errors():
    specs = _mixed(3, n=3)
    b = api.Batch.from_specs(specs)
    b.n_v[1] = 2
    with pytest.raises(_lib.SweepError, match="BAD_GRID"):
        api.sweep_eval_batched(b)


def test_batched_rejects_short_output_buffers():
    # the padded layout needs out_elems (> 3 * n_vertices) elements; a buffer
    # sized for the unpadded vertex count is refused before any launch
    specs = _mixed(3, n=3)
    b = api.Batch.from_specs(specs)
    assert b.out_elems > 3 * b.n_vertices
    short = torch.empty(3 * b.n_vertices, device="cuda")
    full = torch.empty(b.out_elems, device="cuda")
    with pytest.raises(ValueError, match="elements"):
        api.sweep_eval_batched(b, out=(short, full))
    with pytest.raises(ValueError, match="elements"):
        api.sweep_eval_batched(b, out=(full, short))
    with pytest.raises(ValueError, match="float32"):
        api.sweep_eval_batched(b, out=(full.double(), None))
