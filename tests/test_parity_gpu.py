"""Parity of the HIP path (through the C ABI) with the FP64 oracle on seeded
inputs: the plain FP64 sweep, FP32 output, every degree, user knots, open and
non-planar profiles, ragged grids spanning several frame chunks, every fixed
surface configuration, degenerate tangents, the full-size large sweep and
precision-study grids (every vertex, streamed in row chunks), and the largest
accepted grid on sampled rows."""

import numpy as np
import pytest
import torch

import oracle
import synth
from tests.gpu_util import TOL, check_full, dev_ctrl, gpu_sweep, parity, say, stream_parity

pytestmark = pytest.mark.gpu

rng = np.random.default_rng(2024)


def _spec(n_path, p, m, q, n_u, n_v, closed=True, seed=0, planar=True):
    r = np.random.default_rng(seed)
    P = synth.random_walk(r, n_path)
    Q = synth.perturbed_circle(r, m)
    if not planar:
        Q[:, 2] = 0.1 * r.standard_normal(m)
    return synth.SweepSpec(synth.CurveSpec(P, p), synth.CurveSpec(Q, q, closed), n_u, n_v)


def test_plain_fp64_sweep():
    r = check_full(synth.c1(), out_dtype=torch.float64)
    assert r["masked"] < 0.01 * 256 * 64


def test_plain_sweep_fp32_output():
    check_full(synth.c1(), out_dtype=torch.float32)


@pytest.mark.parametrize("p,q", [(1, 1), (2, 2), (3, 3), (4, 2), (5, 3), (6, 4), (7, 7), (2, 5)])
def test_degrees(p, q):
    check_full(_spec(max(p + 1, 12), p, max(q + 1, 9), q, 301, 37, seed=p * 10 + q), out_dtype=torch.float64)


@pytest.mark.parametrize("n_u,n_v", [(2, 3), (3, 4), (1023, 8), (1024, 8), (1025, 12), (3000, 37), (4100, 64)])
def test_ragged_grids_across_chunks(n_u, n_v):
    check_full(_spec(40, 3, 8, 3, n_u, n_v, seed=n_u), out_dtype=torch.float64)


def test_user_knots_and_open_profile():
    P = synth.random_walk(rng, 9)
    U = np.array([0, 0, 0, 0, .1, .1, .45, .7, .7, 1, 1, 1, 1], float)
    Q = np.stack([np.linspace(-0.5, 0.5, 7), 0.2 * np.sin(np.arange(7)), np.zeros(7)], 1)
    V = np.array([0, 0, 0, .3, .3, .6, .8, 1, 1, 1], float) * 2.0 - 1.0
    spec = synth.SweepSpec(synth.CurveSpec(P, 3, knots=U), synth.CurveSpec(Q, 2, False, knots=V), 777, 29)
    check_full(spec, out_dtype=torch.float64)
    check_full(spec, out_dtype=torch.float32)


def test_non_planar_profile_and_initial_normal():
    spec = _spec(20, 3, 10, 3, 513, 40, seed=5, planar=False)
    check_full(spec, out_dtype=torch.float64)
    check_full(spec, out_dtype=torch.float64, n0=np.array([0.3, -0.2, 0.9]))


def test_fp32_frame_and_raw_frame_variants():
    spec = _spec(16, 3, 8, 3, 2048, 32, seed=7)
    # FP32 step matrices and scan: error budget of single precision
    check_full(spec, out_dtype=torch.float32, frame_dtype=torch.float32, tol=1e-4)
    # no re-orthonormalisation in FP64: the defining values are unchanged
    check_full(spec, out_dtype=torch.float64, reorth=False, tol=1e-11)


@pytest.mark.parametrize("cfg", list(range(16)))
def test_every_fixed_surface_config(cfg):
    check_full(_spec(30, 3, 12, 3, 150, 1024, seed=11), out_dtype=torch.float32, tile_config=cfg)
    check_full(_spec(30, 3, 12, 3, 97, 516, seed=12), out_dtype=torch.float64, tile_config=cfg)


def test_tangent_reversal():
    P = np.array([[0.0, 0, 0], [1.0, 0, 0], [0.0, 0, 0]])
    Q = synth.perturbed_circle(rng, 6)
    spec = synth.SweepSpec(synth.CurveSpec(P, 1), synth.CurveSpec(Q, 3, True), 11, 16)
    check_full(spec, out_dtype=torch.float64)


def test_stationary_run_across_chunks_and_zero_start():
    # a stationary segment of ~1700 samples spanning chunk boundaries
    P = np.array([[0.0, 0, 0], [1.0, 0.5, 0], [1.0, 0.5, 0], [2.0, 2.0, 1.0]])
    Q = synth.perturbed_circle(rng, 7)
    spec = synth.SweepSpec(synth.CurveSpec(P, 1), synth.CurveSpec(Q, 2, True), 5000, 9)
    check_full(spec, out_dtype=torch.float64)
    P2 = np.array([[1.0, 1, 1], [1.0, 1, 1], [2.0, 3.0, 1.0], [4.0, 3.0, 0.0], [5, 5, 5]])
    spec2 = synth.SweepSpec(synth.CurveSpec(P2, 1), synth.CurveSpec(Q, 2, True), 3001, 9)
    check_full(spec2, out_dtype=torch.float64)


def test_deterministic_and_stream():
    spec = _spec(50, 3, 16, 3, 2000, 100, seed=3)
    a, na = gpu_sweep(spec)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        b, nb = gpu_sweep(spec, stream=s)
    s.synchronize()
    torch.cuda.synchronize()
    assert torch.equal(a, b) and torch.equal(na, nb)


def test_large_sweep_full_grid():
    """Every vertex of the 65,536 x 1,024 sweep (FP32 output, FP64 frame)
    against the oracle, streamed in row chunks."""
    spec = synth.c2()
    say(f"[case] full grid n_u={spec.n_u} n_v={spec.n_v} out=float32")
    pos, nrm = gpu_sweep(spec, torch.float32)
    torch.cuda.synchronize()
    ok, r = stream_parity(spec, pos, nrm, TOL[torch.float32])
    say("   ", r)
    assert ok, r


@pytest.mark.parametrize("frame_dtype,tol", [(torch.float64, 1e-5), (torch.float32, 1e-3)])
def test_precision_study_full_grid(frame_dtype, tol):
    """Every vertex of the 1,048,576 x 32 grid, FP64 and FP32 frame scans."""
    spec = synth.c3()
    say(f"[case] full grid n_u={spec.n_u} n_v={spec.n_v} frame={frame_dtype}")
    pos, nrm = gpu_sweep(spec, torch.float32, frame_dtype)
    torch.cuda.synchronize()
    ok, r = stream_parity(spec, pos, nrm, tol, chunk_rows=65536)
    say("   ", r)
    assert ok, r


@pytest.mark.parametrize("tile_config", [-1, 14])
def test_maximum_grid_sampled_rows(tile_config):
    """The largest grid the boundary accepts: n_u * n_v just under 2^31
    (1,048,575 x 2048 = 2,147,481,600 vertices, 51.5 GB of FP32 output), so
    every vertex index is near the top of the 32-bit range; the default
    column-tile kernel and the linear kernel (64-bit-multiply division by
    n_v) are both checked on sampled rows, including the last one."""
    spec = synth.c2(n_u=1048575, n_v=2048)
    assert spec.n_u * spec.n_v < 2 ** 31 and spec.n_u * (spec.n_v + 1) >= 2 ** 31
    rows = np.unique(np.concatenate([[0, 255, 256, 524288, spec.n_u - 2, spec.n_u - 1],
                                     rng.integers(0, spec.n_u, 6)]))
    say(f"[case] maximum grid tile_config={tile_config}")
    pos, nrm = gpu_sweep(spec, torch.float32, tile_config=tile_config)
    torch.cuda.synchronize()
    idx = torch.as_tensor(rows, device=pos.device)
    gp = pos.index_select(1, idx).cpu().numpy()
    gn = nrm.index_select(1, idx).cpu().numpy()
    del pos, nrm
    torch.cuda.empty_cache()
    x, _, _, _ = oracle.path_samples(spec.path, spec.n_u)
    rp, rn, rk, _ = oracle.sweep_rows(spec.path, spec.profile, spec.n_u, spec.n_v, rows)
    ok, r = parity(rp, rn, rk, gp, gn, TOL[torch.float32], diag=float(np.linalg.norm(x.max(0) - x.min(0))))
    say("   ", r)
    assert ok, r


def test_grid_limit_is_rejected():
    spec = synth.c2(n_u=1048576, n_v=2048)      # exactly 2^31 vertices
    with pytest.raises(Exception, match="BAD_GRID"):
        gpu_sweep(spec, torch.float32)


@pytest.mark.parametrize("name,n_u", [("c1", 256), ("c1", 5000), ("c3", 1048576), ("c2", 65536)])
def test_frames_match_oracle(name, n_u):
    """The whole frame (every u-sample) against the oracle's sequential FP64
    recurrence.  A product of n rotations carries O(n eps) rounding in either
    evaluation order, so the bound is 8 n eps (worst case); the measured
    difference is printed."""
    from paper_1110_5450_amd import api
    spec = synth.config(name)
    say(f"[case] frames {name} n_u={n_u}")
    rows = api.sweep_frames(torch.as_tensor(spec.path.ctrl).cuda(), spec.path.degree, n_u).cpu().numpy()
    x, d1, d2, ft = oracle.path_samples(spec.path, n_u)
    R, _ = oracle.frame(x, d1, ft)
    eps = np.finfo(float).eps
    dx = np.abs(rows[:, 0:3] - x).max() / max(1.0, np.abs(x).max())
    dR = max(np.abs(rows[:, 3 + 3 * c: 6 + 3 * c] - R[:, :, c]).max() for c in range(3))
    L = np.linalg.norm(d1, axis=1)
    a = np.einsum("ia,ia->i", R[:, :, 0], d2) / L
    b = np.einsum("ia,ia->i", R[:, :, 1], d2) / L
    dab = max(np.abs(rows[:, 13] - a).max(), np.abs(rows[:, 14] - b).max()) / max(1.0, np.abs(d2).max() / L.min())
    G = np.einsum("nki,nkj->nij", rows[:, 3:12].reshape(-1, 3, 3).transpose(0, 2, 1), rows[:, 3:12].reshape(-1, 3, 3).transpose(0, 2, 1))
    drift = np.abs(G - np.eye(3)).max()
    say(f"    x {dx:.2e}  frame {dR:.2e} (bound {8 * n_u * eps:.1e})  a,b {dab:.2e}  orthonormality {drift:.2e}")
    assert dx <= 1e-14 and dR <= 8 * n_u * eps and dab <= 1e-10 and drift <= 1e-14


def _stationary_path():
    # degree 1 through 12 points, segments 3 and 10 of zero length: with
    # 70,000 u-samples (274 frame chunks of 256) the stationary samples
    # cover chunks 75-99 and 249-273, so chunks whose first sample has
    # C' = 0 lie below and above chunk 256; the path ends stationary
    rng = np.random.default_rng(9)
    P = synth.random_walk(rng, 12)
    P[4] = P[3]
    P[11] = P[10]
    return P


def test_stationary_runs_beyond_256_chunks():
    """274 frame chunks: the fused frame kernel's carry takes two chunk
    products per thread, and the degenerate-start chunks (on both sides of
    chunk 256) are formed inside it.  The oracle multiplies the 70,000 step
    rotations in sequence, the GPU in a tree, so the frames differ by
    rounding that grows with the scan length: the FP64 bound is 8 n eps
    (about 1.2e-10 here) rather than 1e-12."""
    Q = synth.perturbed_circle(rng, 7)
    spec = synth.SweepSpec(synth.CurveSpec(_stationary_path(), 1), synth.CurveSpec(Q, 3, True), 70000, 8)
    check_full(spec, out_dtype=torch.float64, tol=8 * spec.n_u * np.finfo(float).eps)


def test_stationary_runs_chunk_carry_route():
    """More than 512 frame chunks (2,200,000 u-samples in runs of 16: 538
    chunks) take the one-block chunk carry and the separate row kernel;
    degenerate-start chunks are formed in the carry.  Bound 8 n eps as
    above."""
    Q = synth.perturbed_circle(rng, 7)
    spec = synth.SweepSpec(synth.CurveSpec(_stationary_path(), 1), synth.CurveSpec(Q, 3, True), 2200000, 4)
    check_full(spec, out_dtype=torch.float64, tol=8 * spec.n_u * np.finfo(float).eps)


def test_law_sweep_with_zero_speed_chunk_starts():
    """A sweep law takes the chunk-carry route at any length; stationary
    chunk starts below 256 chunks."""
    from paper_1110_5450_amd import api
    Q = synth.perturbed_circle(rng, 7)
    spec = synth.SweepSpec(synth.CurveSpec(_stationary_path(), 1), synth.CurveSpec(Q, 3, True), 30000, 8)
    law = synth.CurveSpec(np.array([[1.0, 0.0, 0.0], [1.3, 0.8, 0.0], [0.9, -0.4, 0.0], [1.1, 1.0, 0.0]]), 2)
    say(f"[case] law + stationary chunk starts n_u={spec.n_u}")
    ref, _ = oracle.sweep_ex(spec.path, spec.profile, spec.n_u, spec.n_v, law=law)
    pos, nrm = gpu_sweep(spec, torch.float64, law=api.Law(dev_ctrl(law.ctrl), law.degree, None))
    torch.cuda.synchronize()
    # sequential (oracle) against tree-ordered (GPU) rotation products:
    # rounding bound 8 n eps, as in test_stationary_runs_beyond_256_chunks
    tol = max(TOL[torch.float64], 8 * spec.n_u * np.finfo(float).eps)
    ok, r = parity(ref.pos, ref.nrm, ref.kappa, pos.cpu().numpy(), nrm.cpu().numpy(), tol)
    say("   ", r)
    assert ok, r


@pytest.mark.parametrize("n_u", [5000, 60000, 70000])
def test_fused_and_carry_frame_routes_agree(n_u):
    """Up to 512 chunks the plain sweep forms its frame in one launch (each
    block forms its entry normal from the chunk products below it, two per
    thread above 256 chunks: 70,000 samples); with a
    sweep law the same frame goes through the chunk-carry kernel.  An
    identity law (scale 1, twist 0) leaves the positions unchanged, so the
    two routes agree to rounding on the same input."""
    from paper_1110_5450_amd import api
    Q = synth.perturbed_circle(rng, 9)
    P = _stationary_path()
    spec = synth.SweepSpec(synth.CurveSpec(P, 1), synth.CurveSpec(Q, 3, True), n_u, 16)
    ident = api.Law(dev_ctrl(np.array([[1.0, 0.0, 0.0], [1.0, 0.0, 0.0]])), 1, None)
    say(f"[case] fused vs carry route n_u={n_u}")
    a, _ = gpu_sweep(spec, torch.float64)
    b, _ = gpu_sweep(spec, torch.float64, law=ident)
    torch.cuda.synchronize()
    diag = oracle.bbox_diag(a.cpu().numpy())
    d = (a - b).abs().max().item() / diag
    say(f"    max |dX| / diag = {d:.2e}")
    assert d <= 1e-13
