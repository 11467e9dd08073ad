#!/usr/bin/env python3
"""Throughput of dense swept-surface evaluation on one MI355X.

One step = one sweep_eval call over the large single sweep (path: cubic,
1024 control points, 3-D random walk; profile: closed cubic, 64 control
points, radius 0.3 +-10 %; grid 65536 x 1024 = 67,108,864 vertices; FP32
positions and normals, FP64 frame scan): curve samples, profile table, frame
scan, row table and surface write, all in libsweep's HIP kernels.  Inputs
(control points) are resident in device memory before timing.

Prints one JSON line: vertices/s over the timed steps, the surface kernel's
roofline figures (HIP events around every surface launch in the timed
region, on the launch stream), the error against the FP64 oracle on sampled
rows, the variants named by the metric (plain FP64 output; the 4096-sweep
batch in one graph launch versus the same sweeps as FP64 single calls; the
adjoint), and the FP64 CPU oracle timed on the same workload.

`--precision-study` instead prints the precision-study report (FP32 / FP64
frame scan, with and without re-orthonormalisation, on the 1,048,576 x 32
grid): time, frame error and orthonormality drift against the oracle, and
surface error on sampled rows.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "swept-surface vertices/s (pos+normal) and % HBM peak; batched/FP32 vs plain FP64"
HBM_PEAK_GBS = 8000.0
COPY_CAL_BYTES = 512 << 20
# Untimed calls before timing a batched entry point.  The first call of a
# plan builds it (descriptors, graph, the adjoint's unit and chunk lists):
# 6 ms for the 4096-sweep batch, 13 ms for the first backward call; the
# second call is within 0.3 ms of steady state and the later ones are
# steady (each warm-up call is timed and reported with the result).
GRAPH_WARMUP = 3
COUNTERS = os.path.join(ROOT, "profiles", "surface_c2_counters.json")
SURFACE_SRC = os.path.join(ROOT, "paper_1110_5450_amd", "csrc", "surface_kernels.hip")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def surface_source_hash() -> str:
    with open(SURFACE_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def stored_traffic():
    """HBM bytes per launch of the surface kernel from the committed rocprofv3
    counter summary, if it was taken on the current surface kernel source."""
    try:
        with open(COUNTERS) as f:
            c = json.load(f)
    except (OSError, ValueError):
        return None
    if c.get("surface_source_sha256_16") != surface_source_hash():
        return None
    return c.get("hbm_bytes_per_launch")


def _dev_spec(spec, dev):
    import torch
    return torch.as_tensor(spec.path.ctrl).to(dev), torch.as_tensor(spec.profile.ctrl).to(dev)


def _dev_weights(curve, dev):
    import torch
    w = getattr(curve, "weights", None)
    return None if w is None else torch.as_tensor(w).to(dev)


def time_single(spec, steps, warmup, out_dtype, frame_dtype=None, keep=False, frame_mode="rmf", law=None,
                u_sampling="parameter", u_lambda=0.0):
    """Wall time of `steps` sweep_eval calls, the per-call (frame, surface)
    stage times from the library's HIP events, and optionally the outputs."""
    import torch
    from paper_1110_5450_amd import _lib, api

    frame_dtype = frame_dtype or torch.float64
    dev = torch.device("cuda:0")
    P, Q = _dev_spec(spec, dev)
    pos = torch.empty((3, spec.n_u, spec.n_v), dtype=out_dtype, device=dev)
    nrm = torch.empty_like(pos)
    glaw = None if law is None else api.Law(torch.as_tensor(law.ctrl).to(dev), law.degree, law.knots)
    ws = torch.empty(api.eval_workspace_size(P.shape[0], spec.path.degree, Q.shape[0], spec.profile.degree,
                                             spec.n_u, spec.n_v, out_dtype=out_dtype, frame_dtype=frame_dtype,
                                             frame_mode=frame_mode, law=glaw, u_sampling=u_sampling,
                                             u_lambda=u_lambda),
                     dtype=torch.uint8, device=dev)

    Pw, Qw = _dev_weights(spec.path, dev), _dev_weights(spec.profile, dev)

    def step():
        api.sweep_eval(P, spec.path.degree, Q, spec.profile.degree, spec.n_u, spec.n_v, out_dtype=out_dtype,
                       frame_dtype=frame_dtype, path_weights=Pw, prof_weights=Qw, frame_mode=frame_mode, law=glaw,
                       u_sampling=u_sampling, u_lambda=u_lambda, out=(pos, nrm), workspace=ws)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    _lib.check(_lib.sweep_trace_enable(steps))
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    rec = _lib.sweep_trace_read()
    surf = [ms for st, ms in rec if st == 1]
    frame = [ms for st, ms in rec if st == 0]
    out = (pos, nrm) if keep else None
    if not keep:
        del pos, nrm
    del ws
    torch.cuda.empty_cache()
    return t1 - t0, surf, frame, out


def sampled_error(spec, pos, nrm, rows, tol, frame_mode="rmf", law=None, arclength=False, lam=0.0):
    """Parity figures of a GPU result on sampled rows against the oracle."""
    import numpy as np
    import torch
    import oracle

    idx = torch.as_tensor(rows, device=pos.device)
    gp = pos.index_select(1, idx).double().cpu().numpy()
    gn = nrm.index_select(1, idx).double().cpu().numpy()
    x, _, _, _ = oracle.path_samples(spec.path, spec.n_u)
    if frame_mode == "rmf" and law is None and not arclength:
        rp, rn, rk, _ = oracle.sweep_rows(spec.path, spec.profile, spec.n_u, spec.n_v, rows)
    else:
        rp, rn, rk = oracle.sweep_rows_ex(spec.path, spec.profile, spec.n_u, spec.n_v, rows, mode=frame_mode,
                                          law=law, arclength=arclength, lam=lam)
    diag = float(np.linalg.norm(x.max(0) - x.min(0)))
    r = oracle.compare(rp, rn, rk, gp, gn, diag, 1e6)
    r["rows"] = len(rows)
    r["tolerance"] = tol
    return r


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_rate(n_u: int, n_v: int, target_s: float, max_reps: int):
    """vertices/s of the oracle on the large sweep at n_u x n_v, repeated for
    about target_s seconds; (rate, reps, seconds, threads)."""
    import oracle
    import synth

    spec = synth.c2(n_u=n_u, n_v=n_v)
    reps, total = 0, 0.0
    while reps < max_reps and (total < target_s or reps < 2):
        t0 = time.perf_counter()
        r = oracle.sweep(spec.path, spec.profile, spec.n_u, spec.n_v, want_kappa=False)
        total += time.perf_counter() - t0
        reps += 1
        del r
    return spec.n_u * spec.n_v * reps / total, reps, total, oracle.max_threads()


def cpu_baseline(spec, target_s: float = 10.0, max_reps: int = 1000):
    """The oracle as it stands on the same workload: the whole grid (frame
    scan, positions and normals in FP64), repeated until about target_s of
    work has run, with all host threads; then one host thread in a child
    process (OMP_NUM_THREADS=1) on the first 4096 rows of the same sweep."""
    import subprocess

    rate, reps, total, threads = _oracle_rate(spec.n_u, spec.n_v, target_s, max_reps)
    out = {
        "value": rate, "unit": "vertices/s", "cores": threads, "kind": "oracle",
        "sample": (f"the full {spec.n_u}x{spec.n_v} grid (frame scan, FP64 positions and normals) "
                   f"run {reps} times, {total:.1f} s in all"),
        "nproc": os.cpu_count(), "cpu_model": _cpu_model(),
    }
    code = ("import json, sys; sys.path.insert(0, %r); import bench; "
            "r = bench._oracle_rate(4096, %d, %f, 1000); print(json.dumps(r))" % (ROOT, spec.n_v, target_s / 2))
    env = dict(os.environ, OMP_NUM_THREADS="1")
    try:
        res = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, timeout=120)
        r1, reps1, total1, th1 = json.loads(res.stdout.strip().splitlines()[-1])
        out["single_thread"] = {"value": r1, "unit": "vertices/s", "cores": th1,
                                "sample": f"the first 4096 rows ({4096}x{spec.n_v}) run {reps1} times, "
                                          f"{total1:.1f} s in all"}
    except Exception as e:  # the all-thread figure stands on its own
        out["single_thread"] = {"error": str(e)[:200]}
    return out


def rational_variant(steps: int):
    """The large sweep with rational (NURBS) path and profile: throughput,
    stage times and sampled parity against the oracle."""
    import numpy as np
    import torch
    import synth

    spec = synth.c2_rational()
    N = spec.n_u * spec.n_v
    el, surf, frame, res = time_single(spec, steps, 1, torch.float32, keep=True)
    rng = np.random.default_rng(8)
    rows = np.unique(np.concatenate([[0, spec.n_u - 1], rng.integers(0, spec.n_u, 6)]))
    err = sampled_error(spec, res[0], res[1], rows, 1e-5)
    del res
    torch.cuda.empty_cache()
    return {"workload": "the large sweep with weights U(0.5, 2) on path and profile control points",
            "vertices_per_s": N * steps / el, "ms_per_step": 1e3 * el / steps,
            "frame_ms": sum(frame) / len(frame), "surface_ms": sum(surf) / len(surf), "error_vs_oracle": err}


def frenet_law_variant(steps: int):
    """The large sweep with the Frenet frame and a scale/twist law (extended
    row records): throughput, stage times and sampled parity."""
    import numpy as np
    import torch
    import synth

    spec = synth.c2()
    law = synth.sweep_law()
    N = spec.n_u * spec.n_v
    el, surf, frame, res = time_single(spec, steps, 1, torch.float32, keep=True, frame_mode="frenet", law=law)
    rng = np.random.default_rng(9)
    rows = np.unique(np.concatenate([[0, spec.n_u - 1], rng.integers(0, spec.n_u, 6)]))
    err = sampled_error(spec, res[0], res[1], rows, 1e-5, frame_mode="frenet", law=law)
    del res
    torch.cuda.empty_cache()
    s_ms = sum(surf) / len(surf)
    return {"workload": "the large sweep, Frenet frame, scale/twist law (16 control points, cubic)",
            "vertices_per_s": N * steps / el, "ms_per_step": 1e3 * el / steps,
            "frame_ms": sum(frame) / len(frame), "surface_ms": s_ms,
            "surface_GBps": 24.0 * N / (s_ms * 1e-3) / 1e9, "error_vs_oracle": err}


def arclength_variant(steps: int):
    """The large sweep with its path sampled at equal arc length (length
    table, Newton inversion, then the same frame and surface): throughput,
    stage times and sampled parity."""
    import numpy as np
    import torch
    import synth

    spec = synth.c2()
    N = spec.n_u * spec.n_v
    el, surf, frame, res = time_single(spec, steps, 1, torch.float32, keep=True, u_sampling="arclength")
    rng = np.random.default_rng(10)
    rows = np.unique(np.concatenate([[0, spec.n_u - 1], rng.integers(0, spec.n_u, 6)]))
    err = sampled_error(spec, res[0], res[1], rows, 1e-5, arclength=True)
    del res
    torch.cuda.empty_cache()
    # curvature-adaptive: equal steps of arc length + 0.5 x turning angle
    ela, surfa, framea, resa = time_single(spec, steps, 1, torch.float32, keep=True, u_sampling="adaptive",
                                           u_lambda=0.5)
    erra = sampled_error(spec, resa[0], resa[1], rows, 1e-5, arclength=True, lam=0.5)
    del resa
    torch.cuda.empty_cache()
    return {"workload": "the large sweep, path samples at equal arc length",
            "vertices_per_s": N * steps / el, "ms_per_step": 1e3 * el / steps,
            "frame_ms": sum(frame) / len(frame), "surface_ms": sum(surf) / len(surf), "error_vs_oracle": err,
            "adaptive_lambda_0.5": {"vertices_per_s": N * steps / ela, "ms_per_step": 1e3 * ela / steps,
                                    "frame_ms": sum(framea) / len(framea), "error_vs_oracle": erra}}


def triangles_variant(steps: int):
    """The triangle list of the large sweep's grid (closed profile):
    2 (n_u-1) n_v triangles of 3 int32, write-only."""
    import torch
    import synth
    from paper_1110_5450_amd import api

    spec = synth.c2()
    nt = api.triangle_count(spec.n_u, spec.n_v, True)
    tri = torch.empty((nt, 3), dtype=torch.int32, device="cuda")
    api.triangles(spec.n_u, spec.n_v, True, out=tri)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        api.triangles(spec.n_u, spec.n_v, True, out=tri)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    del tri
    torch.cuda.empty_cache()
    return {"workload": f"triangle list of the {spec.n_u}x{spec.n_v} grid, closed profile", "triangles": nt,
            "ms": ms, "GBps": 12.0 * nt / (ms * 1e-3) / 1e9}


def batched_mode(b, specs, steps, pos, nrm, picked, frame_mode="rmf", law=None, u_sampling="parameter",
                 u_lambda=0.0):
    """The batch in another mode (arc-length or adaptive path samples, or the
    Frenet frame with one law for every sweep), FP32 output into the same
    buffers: graph time per call and whole-sweep parity on a few sweeps."""
    import torch
    import oracle
    from paper_1110_5450_amd import api

    glaw = None if law is None else api.Law(torch.as_tensor(law.ctrl).cuda(), law.degree, law.knots)
    kw = dict(frame_mode=frame_mode, law=glaw, u_sampling=u_sampling, u_lambda=u_lambda)
    ws = torch.empty(api.batched_workspace_size(b, **kw), dtype=torch.uint8, device="cuda")
    t1 = time.perf_counter()
    api.sweep_eval_batched(b, out=(pos, nrm), workspace=ws, **kw)
    torch.cuda.synchronize()
    first_ms = 1e3 * (time.perf_counter() - t1)
    for _ in range(GRAPH_WARMUP - 1):
        api.sweep_eval_batched(b, out=(pos, nrm), workspace=ws, **kw)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    for _ in range(steps):
        api.sweep_eval_batched(b, out=(pos, nrm), workspace=ws, **kw)
    ev[1].record()
    torch.cuda.synchronize()
    gpu_ms = ev[0].elapsed_time(ev[1]) / steps
    err = {"pos_rel": 0.0, "nrm_scaled": 0.0, "nrm_abs_wc": 0.0, "masked": 0}
    arc = u_sampling != "parameter"
    for k in picked:
        s = specs[k]
        ref, _ = oracle.sweep_ex(s.path, s.profile, s.n_u, s.n_v, mode=frame_mode, law=law, arclength=arc,
                                 lam=u_lambda if u_sampling == "adaptive" else 0.0)
        r = oracle.compare(ref.pos, ref.nrm, ref.kappa, b.view(pos, k).double().cpu().numpy(),
                           b.view(nrm, k).double().cpu().numpy(), oracle.bbox_diag(ref.pos), 1e6)
        for key in ("pos_rel", "nrm_scaled", "nrm_abs_wc"):
            err[key] = max(err[key], r[key])
        err["masked"] += r["masked"]
    err.update({"sweeps": list(picked), "tolerance": 1e-5})
    del ws
    return {"vertices_per_s": b.n_vertices / (gpu_ms * 1e-3), "gpu_ms_per_step": gpu_ms,
            "first_call_ms": round(first_ms, 3), "error_vs_oracle": err}


def batched_variants(steps: int):
    """The 4096-sweep batch: one graph launch (FP32) versus the same sweeps as
    single FP64 calls."""
    import torch
    import synth
    from paper_1110_5450_amd import api

    import numpy as np
    import oracle

    specs = synth.c4()
    b = api.Batch.from_specs(specs)
    N = b.n_vertices
    ws = torch.empty(api.batched_workspace_size(b), dtype=torch.uint8, device="cuda")
    pos = torch.empty(b.out_elems, dtype=torch.float32, device="cuda")
    nrm = torch.empty_like(pos)
    # the surface tile is chosen by the batched autotuner (untimed set-up);
    # tile_config = -1 then uses its choice
    t_tune = time.perf_counter()
    tuned, tuned_ms = api.autotune_batched(b, out=(pos, nrm), workspace=ws)
    t_tune = time.perf_counter() - t_tune
    assert api.batched_config_for(b) == tuned
    warm_ms = []
    for _ in range(GRAPH_WARMUP):
        t1 = time.perf_counter()
        api.sweep_eval_batched(b, out=(pos, nrm), workspace=ws)
        torch.cuda.synchronize()
        warm_ms.append(round(1e3 * (time.perf_counter() - t1), 3))
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    t0 = time.perf_counter()
    ev[0].record()
    for _ in range(steps):
        api.sweep_eval_batched(b, out=(pos, nrm), workspace=ws)
    ev[1].record()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    gpu_ms = ev[0].elapsed_time(ev[1]) / steps
    # error against the oracle on 16 sampled sweeps (whole sweeps)
    rng = np.random.default_rng(44)
    err = {"pos_rel": 0.0, "nrm_scaled": 0.0, "nrm_abs_wc": 0.0, "masked": 0}
    picked = sorted(int(k) for k in rng.choice(len(specs), 16, replace=False))
    for k in picked:
        s = specs[k]
        ref = oracle.sweep(s.path, s.profile, s.n_u, s.n_v)
        r = oracle.compare(ref.pos, ref.nrm, ref.kappa, b.view(pos, k).double().cpu().numpy(),
                           b.view(nrm, k).double().cpu().numpy(), oracle.bbox_diag(ref.pos), 1e6)
        for key in ("pos_rel", "nrm_scaled", "nrm_abs_wc"):
            err[key] = max(err[key], r[key])
        err["masked"] += r["masked"]
    err.update({"sweeps": picked, "tolerance": 1e-5})
    modes = {"arclength_graph": batched_mode(b, specs, steps, pos, nrm, picked[:4], u_sampling="arclength"),
             "adaptive_lambda_0.5_graph": batched_mode(b, specs, steps, pos, nrm, picked[:4],
                                                       u_sampling="adaptive", u_lambda=0.5),
             "frenet_law_graph": batched_mode(b, specs, steps, pos, nrm, picked[:4], frame_mode="frenet",
                                              law=synth.sweep_law())}
    del pos, nrm, ws
    torch.cuda.empty_cache()
    # the same sweeps, one FP64 sweep_eval call each
    Ps = [torch.as_tensor(s.path.ctrl).cuda() for s in specs]
    Qs = [torch.as_tensor(s.profile.ctrl).cuda() for s in specs]
    maxN = max(s.n_u * s.n_v for s in specs)
    buf = torch.empty(2 * 3 * maxN, dtype=torch.float64, device="cuda")
    wsz = max(api.eval_workspace_size(s.path.n, s.path.degree, s.profile.n, s.profile.degree, s.n_u, s.n_v,
                                      out_dtype=torch.float64) for s in specs)
    ws = torch.empty(wsz, dtype=torch.uint8, device="cuda")

    def singles():
        for k, s in enumerate(specs):
            n3 = 3 * s.n_u * s.n_v
            p = buf[:n3].view(3, s.n_u, s.n_v)
            q = buf[n3:2 * n3].view(3, s.n_u, s.n_v)
            api.sweep_eval(Ps[k], s.path.degree, Qs[k], s.profile.degree, s.n_u, s.n_v,
                           out_dtype=torch.float64, out=(p, q), workspace=ws)

    singles()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    singles()
    torch.cuda.synchronize()
    el64 = time.perf_counter() - t0
    del buf, ws
    torch.cuda.empty_cache()
    return {
        "workload": "4096 sweeps: path cps U{8..512}, profile cps U{4..64}, degrees U{2,3}, "
                    "n_u log-U[16,4096], n_v log-U[8,256]",
        "vertices": N,
        "batched_fp32_graph": {"vertices_per_s": N * steps / el, "ms_per_step": 1e3 * el / steps,
                               "gpu_ms_per_step": gpu_ms, "output_GBps": 24.0 * N / (gpu_ms * 1e-3) / 1e9,
                               "frac_of_hbm_peak": 24.0 * N / (gpu_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                               "tile_config": tuned, "tile": api.tile_config_name(tuned),
                               "autotune": {"best_ms": tuned_ms, "seconds": t_tune},
                               "warmup_call_ms": warm_ms,
                               "error_vs_oracle": err},
        **modes,
        "single_calls_fp64": {"vertices_per_s": N / el64, "ms_per_pass": 1e3 * el64, "calls": len(specs)},
    }


def c1_variant(calls: int = 200):
    """The plain single sweep (cubic path of 16 control points, closed cubic
    profile of 8, 256 x 64, FP64 positions and normals): `calls` sweep_eval
    calls after a warm-up, with the error against the oracle."""
    import torch
    import oracle
    import synth

    spec = synth.c1()
    el, surf, frame, (pos, nrm) = time_single(spec, calls, 10, torch.float64, torch.float64, keep=True)
    ref = oracle.sweep(spec.path, spec.profile, spec.n_u, spec.n_v)
    err = oracle.compare(ref.pos, ref.nrm, ref.kappa, pos.cpu().numpy(), nrm.cpu().numpy(),
                         oracle.bbox_diag(ref.pos), 1e6)
    err["tolerance"] = 1e-12
    N = spec.n_u * spec.n_v
    return {"workload": "plain single sweep: cubic path 16 cps, closed cubic profile 8 cps, 256x64, FP64 out",
            "calls": calls, "vertices_per_s": N * calls / el, "ms_per_call": 1e3 * el / calls,
            "gpu_frame_ms": sum(frame) / len(frame), "gpu_surface_ms": sum(surf) / len(surf),
            "error_vs_oracle": err}


def write_probe(nbytes: int = 4 << 30, reps: int = 5) -> dict:
    """Store ceiling of this GPU: a plain coalesced fill (torch's fill kernel,
    16-byte stores) of a 4 GiB buffer, mean of `reps` launches timed with
    events, after one untimed launch.  A reference for the surface kernel's
    rate, not part of the hot path."""
    import torch

    buf = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    buf.fill_(1.0)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    torch.cuda.synchronize()
    ev[0].record()
    for _ in range(reps):
        buf.fill_(0.0)
    ev[1].record()
    torch.cuda.synchronize()
    ms = ev[0].elapsed_time(ev[1]) / reps
    del buf
    torch.cuda.empty_cache()
    return {"GBps": nbytes / (ms * 1e-3) / 1e9, "bytes": nbytes, "ms": ms, "kernel": "torch fill_ (float32)"}


def adjoint_variant(steps: int):
    """The differentiation workload: 256 sweeps of 1024 x 64, FP32, backward."""
    import numpy as np
    import torch
    import synth
    from paper_1110_5450_amd import api

    import oracle

    specs = synth.c5()
    b = api.Batch.from_specs(specs)
    N = b.n_vertices
    # loss weights w ~ N(0, 1) per vertex and component (the configuration's)
    wl = synth.loss_weights(specs, 55)
    g = b.pack(wl, torch.float32)
    ws = torch.empty(api.backward_workspace_size(b), dtype=torch.uint8, device="cuda")
    warm_ms = []
    for _ in range(GRAPH_WARMUP):
        t1 = time.perf_counter()
        api.sweep_backward(b, g, workspace=ws)
        torch.cuda.synchronize()
        warm_ms.append(round(1e3 * (time.perf_counter() - t1), 3))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        api.sweep_backward(b, g, workspace=ws)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    # relative gradient error against the oracle's FP64 central differences
    # (h = 1e-6) on two sampled sweeps, with the FP32-rounded weights
    gP, gQ = api.sweep_backward(b, g, workspace=ws)
    gP, gQ = gP.cpu().numpy(), gQ.cpu().numpy()
    adj_err = {"path_rel": 0.0, "prof_rel": 0.0, "sweeps": [0, 201], "tolerance": 1e-4}
    for k in adj_err["sweeps"]:
        s = specs[k]
        fP, fQ = oracle.fd_grad(s.path, s.profile, s.n_u, s.n_v, wl[k].astype(np.float32).astype(np.float64))
        adj_err["path_rel"] = max(adj_err["path_rel"],
                                  float(np.linalg.norm(gP[b.path_slice(k)] - fP) / np.linalg.norm(fP)))
        adj_err["prof_rel"] = max(adj_err["prof_rel"],
                                  float(np.linalg.norm(gQ[b.prof_slice(k)] - fQ) / np.linalg.norm(fQ)))
    # positions and normals: the reduction reads both gradients
    gn = torch.randn(b.out_elems, dtype=torch.float32, device="cuda", generator=torch.Generator("cuda").manual_seed(6))
    for _ in range(GRAPH_WARMUP):
        api.sweep_backward(b, g, grad_nrm=gn, workspace=ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        api.sweep_backward(b, g, grad_nrm=gn, workspace=ws)
    torch.cuda.synchronize()
    el_n = time.perf_counter() - t0
    # knot and weight gradients as well: the same sweeps with their clamped
    # uniform knot vectors given explicitly and unit weights (rational form)
    import numpy as np
    for s in specs:
        n, p = s.path.n, s.path.degree
        s.path.knots = np.concatenate([np.zeros(p), np.arange(n - p + 1) / (n - p), np.ones(p)])
        s.path.weights = np.ones(n)
        s.profile.weights = np.ones(s.profile.n)
    bp = api.Batch.from_specs(specs)
    names = ["path_knots", "path_weights", "prof_weights"]
    wsp = torch.empty(api.backward_workspace_size(bp), dtype=torch.uint8, device="cuda")
    for _ in range(GRAPH_WARMUP):
        api.sweep_backward(bp, g, grad_nrm=gn, params=names, workspace=wsp)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        api.sweep_backward(bp, g, grad_nrm=gn, params=names, workspace=wsp)
    torch.cuda.synchronize()
    el_p = time.perf_counter() - t0
    del wsp
    fw = torch.empty(b.out_elems, dtype=torch.float32, device="cuda")
    fn = torch.empty_like(fw)
    wsf = torch.empty(api.batched_workspace_size(b), dtype=torch.uint8, device="cuda")
    for _ in range(GRAPH_WARMUP):
        api.sweep_eval_batched(b, out=(fw, fn), workspace=wsf)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        api.sweep_eval_batched(b, out=(fw, fn), workspace=wsf)
    torch.cuda.synchronize()
    elf = time.perf_counter() - t0
    return {"workload": "256 sweeps, 64/16 cps, 1024x64, FP32", "vertices": N,
            "forward_ms": 1e3 * elf / steps, "backward_ms": 1e3 * el / steps,
            "backward_warmup_call_ms": warm_ms,
            "backward_grad_read_GBps": 12.0 * N / (el / steps) / 1e9,
            "backward_with_normals_ms": 1e3 * el_n / steps,
            "backward_with_normals_grad_read_GBps": 24.0 * N / (el_n / steps) / 1e9,
            "backward_with_normals_knots_weights_ms": 1e3 * el_p / steps,
            "error_vs_oracle": adj_err}


def batch_graph_only(steps: int, **mode):
    """The 4096-sweep batch's graph replays alone (for counter and trace
    runs), in the plain mode or the given sampling mode."""
    import torch
    import synth
    from paper_1110_5450_amd import api

    b = api.Batch.from_specs(synth.c4())
    ws = torch.empty(api.batched_workspace_size(b, **mode), dtype=torch.uint8, device="cuda")
    pos = torch.empty(b.out_elems, dtype=torch.float32, device="cuda")
    nrm = torch.empty_like(pos)
    for _ in range(steps):
        api.sweep_eval_batched(b, out=(pos, nrm), workspace=ws, **mode)
    torch.cuda.synchronize()
    return {"vertices": b.n_vertices, "replays": steps, "tile_config": api.batched_config_for(b), **mode}


def adjoint_backward_only(steps: int):
    """The differentiation workload's positions-only backward calls alone (for counter runs)."""
    import torch
    import synth
    from paper_1110_5450_amd import api

    specs = synth.c5()
    b = api.Batch.from_specs(specs)
    g = b.pack(synth.loss_weights(specs, 55), torch.float32)
    ws = torch.empty(api.backward_workspace_size(b), dtype=torch.uint8, device="cuda")
    for _ in range(steps):
        api.sweep_backward(b, g, workspace=ws)
    torch.cuda.synchronize()
    return {"vertices": b.n_vertices, "calls": steps}


def precision_study(steps: int = 5):
    import numpy as np
    import torch
    import oracle
    import synth
    from paper_1110_5450_amd import api

    spec = synth.c3()
    n_u, n_v = spec.n_u, spec.n_v
    P = torch.as_tensor(spec.path.ctrl).cuda()
    x, d1, d2, ft = oracle.path_samples(spec.path, n_u)
    R, _ = oracle.frame(x, d1, ft)
    rng = np.random.default_rng(3)
    rows = np.unique(np.concatenate([[0, 1, n_u // 2, n_u - 1], rng.integers(0, n_u, 28)]))
    rp, rn, rk, _ = oracle.sweep_rows(spec.path, spec.profile, n_u, n_v, rows)
    diag = float(np.linalg.norm(x.max(0) - x.min(0)))
    out = {"workload": f"precision study: plain-sweep curves at {n_u}x{n_v}, FP32 output", "variants": []}
    for fd in (torch.float64, torch.float32):
        for reorth in (True, False):
            fr = api.sweep_frames(P, 3, n_u, out_dtype=torch.float64, frame_dtype=fd,
                                  reorthonormalize=reorth).cpu().numpy()
            Rg = fr[:, 3:12].reshape(-1, 3, 3).transpose(0, 2, 1)
            G = np.einsum("nki,nkj->nij", Rg, Rg)
            drift = float(np.abs(G - np.eye(3)).max())
            ferr = float(np.abs(Rg - R).max())
            # the rotation about t accumulated by the scan, against the oracle's
            ang = np.arctan2(np.einsum("na,na->n", Rg[:, :, 0], R[:, :, 1]),
                             np.einsum("na,na->n", Rg[:, :, 0], R[:, :, 0]))
            el, surf, frame, (pos, nrm) = time_single(spec, steps, 1, torch.float32, fd, keep=True) if reorth else \
                (None, None, None, (None, None))
            rec = {"frame_dtype": str(fd).replace("torch.", ""), "reorthonormalize": reorth,
                   "frame_max_abs_err": ferr, "twist_angle_max_err_rad": float(np.abs(ang).max()),
                   "orthonormality_drift": drift}
            if reorth:
                idx = torch.as_tensor(rows, device=pos.device)
                r = oracle.compare(rp, rn, rk, pos.index_select(1, idx).double().cpu().numpy(),
                                   nrm.index_select(1, idx).double().cpu().numpy(), diag, 1e6)
                rec.update({"surface_pos_rel_err": r["pos_rel"], "surface_nrm_scaled_err": r["nrm_scaled"],
                            "masked": r["masked"], "frame_ms": sum(frame) / len(frame),
                            "surface_ms": sum(surf) / len(surf),
                            "vertices_per_s": n_u * n_v * steps / el})
                del pos, nrm
                torch.cuda.empty_cache()
            out["variants"].append(rec)
            log(rec)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--precision-study", action="store_true")
    ap.add_argument("--variants-only", action="store_true",
                    help="run only the batched (4096 sweeps) and adjoint (256 sweeps) variants and print them")
    ap.add_argument("--variant", choices=["rational", "frenet_law", "arclength", "triangles", "batched", "adjoint",
                                          "c1", "batch-graph", "batch-graph-arclength", "adjoint-backward"],
                    help="run only this variant and print it")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a plain 512 MiB device copy (3 launches) whose counter readings scale "
                         "the surface kernel's HBM traffic counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the sweep shards "
              f"across GPUs only by design, see the design notes)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import synth

    if args.precision_study:
        print(json.dumps(precision_study()), flush=True)
        return
    if args.variants_only:
        log("[bench] batched ...")
        v = {"batched": batched_variants(args.steps)}
        log("[bench] adjoint ...")
        v["adjoint"] = adjoint_variant(args.steps)
        print(json.dumps(v), flush=True)
        return

    if args.copy_calibration:
        src = torch.ones(COPY_CAL_BYTES // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] copy calibration: 3 x {COPY_CAL_BYTES} bytes read and written")
        del src, dst
        torch.cuda.empty_cache()

    if args.variant:
        fn = {"rational": rational_variant, "frenet_law": frenet_law_variant, "arclength": arclength_variant,
              "triangles": triangles_variant, "batched": batched_variants, "adjoint": adjoint_variant,
              "c1": lambda steps: c1_variant(), "batch-graph": batch_graph_only,
              "batch-graph-arclength": lambda steps: batch_graph_only(steps, u_sampling="arclength"),
              "adjoint-backward": adjoint_backward_only}[args.variant]
        log(f"[bench] {args.variant} ...")
        print(json.dumps({args.variant: fn(args.steps)}), flush=True)
        return

    from paper_1110_5450_amd import _lib, api

    spec = synth.c2()
    N = spec.n_u * spec.n_v
    log(f"[bench] large sweep {spec.n_u}x{spec.n_v} FP32 out / FP64 frame, warmup {args.warmup}, steps {args.steps}")
    el, surf, frame, res = time_single(spec, args.steps, args.warmup, torch.float32, keep=True)
    ms_step = 1e3 * el / args.steps
    value = N * args.steps / el
    bytes_alg = 24.0 * N  # 6 FP32 planes, write-only
    surf_ms = sum(surf) / len(surf)
    achieved = bytes_alg / (surf_ms * 1e-3) / 1e9
    log(f"[bench] {ms_step:.3f} ms/step, surface {surf_ms:.3f} ms, frame {sum(frame) / len(frame):.3f} ms")
    rng = np.random.default_rng(7)
    rows = np.unique(np.concatenate([[0, spec.n_u - 1], rng.integers(0, spec.n_u, 14)]))
    err = sampled_error(spec, res[0], res[1], rows, 1e-5)
    del res
    torch.cuda.empty_cache()
    probe = write_probe()
    log(f"[bench] write probe {probe['GBps']:.0f} GB/s")
    out = {
        "metric": METRIC, "value": value, "unit": "vertices/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "large single sweep: cubic path 1024 cps (random walk), closed cubic profile "
                               "64 cps (r=0.3 +-10%), grid 65536x1024, FP32 positions+normals, FP64 frame scan",
                   "n_u": spec.n_u, "n_v": spec.n_v, "vertices": N, "frame_dtype": "f64",
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": stored_traffic(),
                     "kernel": "surface write, " + api.tile_config_name(
                         _lib.sweep_surface_config_for(spec.n_u, spec.n_v, _lib.SWEEP_F32)),
                     "alg_bytes_per_launch": bytes_alg,
                     "avg_launch_ms": surf_ms,
                     # the same rate against the measured store ceiling
                     "write_probe": probe, "frac_of_write_probe": achieved / probe["GBps"]},
        "stages_ms": {"frame": sum(frame) / len(frame), "surface": surf_ms},
        "error_vs_oracle": err,
    }
    if not args.no_variants:
        # every variant step takes well under a millisecond: timed over the
        # full step count, as when run alone (--variant)
        steps64 = args.steps
        el64, surf64, frame64, _ = time_single(spec, steps64, 1, torch.float64)
        s64 = sum(surf64) / len(surf64)
        out["variants"] = {
            "plain_fp64_out": {"vertices_per_s": N * steps64 / el64, "ms_per_step": 1e3 * el64 / steps64,
                               "surface_ms": s64, "surface_GBps": 48.0 * N / (s64 * 1e-3) / 1e9},
        }
        log("[bench] plain FP64 256x64 ...")
        out["variants"]["plain_fp64_256x64"] = c1_variant()
        log("[bench] rational ...")
        out["variants"]["rational_fp32_out"] = rational_variant(steps64)
        log("[bench] frenet + law ...")
        out["variants"]["frenet_law_fp32_out"] = frenet_law_variant(steps64)
        log("[bench] arc length ...")
        out["variants"]["arclength_fp32_out"] = arclength_variant(steps64)
        log("[bench] triangles ...")
        out["variants"]["triangles"] = triangles_variant(steps64)
        log("[bench] batched ...")
        out["variants"]["batched"] = batched_variants(args.steps)
        log("[bench] adjoint ...")
        out["variants"]["adjoint"] = adjoint_variant(args.steps)
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(spec)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
