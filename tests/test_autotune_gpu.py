"""Surface autotuners (single sweep and batch): each times its candidate
surface configurations, the output still meets the parity rule against the
oracle, the choice is recorded for the shape class (tile_config = -1 then
selects it, bitwise the same as asking for it by index), and the table is
written to the cache file."""

from __future__ import annotations

import os

import numpy as np
import pytest
import torch

import oracle
import synth
from paper_1110_5450_amd import api
from tests.gpu_util import TOL, dev_ctrl, gpu_sweep, parity, say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("out_dtype", [torch.float32, torch.float64])
def test_autotune_records_and_selects(tmp_path, out_dtype):
    cache = tmp_path / "tune.txt"
    os.environ["SWEEP_TUNE_CACHE"] = str(cache)
    try:
        # a shape class no other test uses: n_v = 384 (not a multiple of 256)
        spec = synth.single(71, 12, 9, 300, 384)
        p, q = spec.path, spec.profile
        say(f"[case] autotune n_u={spec.n_u} n_v={spec.n_v} out={out_dtype}")
        best, ms, pos, nrm = api.sweep_autotune(dev_ctrl(p.ctrl), p.degree, dev_ctrl(q.ctrl), q.degree,
                                                spec.n_u, spec.n_v, out_dtype=out_dtype)
        torch.cuda.synchronize()
        say("   best", best, ms)
        assert 0 <= best < api.L.sweep_tile_config_count()
        assert ms > 0.0
        ref = oracle.sweep(p, q, spec.n_u, spec.n_v)
        ok, r = parity(ref.pos, ref.nrm, ref.kappa, pos.cpu().numpy(), nrm.cpu().numpy(), TOL[out_dtype])
        assert ok, r
        assert api.surface_config_for(spec.n_u, spec.n_v, out_dtype) == best
        pa, na = gpu_sweep(spec, out_dtype)                      # tile_config = -1
        pb, nb = gpu_sweep(spec, out_dtype, tile_config=best)
        torch.cuda.synchronize()
        assert torch.equal(pa, pb) and torch.equal(na, nb)
        lines = [ln.split() for ln in cache.read_text().splitlines() if not ln.startswith("#")]
        t64 = 1 if out_dtype == torch.float64 else 0
        # kind arch cus t64 nv256 log2_nv log2_vertices 0 config ms
        mine = [ln for ln in lines
                if ln[0] == "single" and ln[3] == str(t64) and ln[4] == "0" and ln[5] == str(int(np.log2(384)))]
        assert mine and int(mine[-1][8]) == best
    finally:
        os.environ.pop("SWEEP_TUNE_CACHE", None)


def test_batched_autotune_records_and_selects(tmp_path):
    cache = tmp_path / "tune.txt"
    os.environ["SWEEP_TUNE_CACHE"] = str(cache)
    try:
        specs = synth.c4(n_sweeps=96, seed=41)
        b = api.Batch.from_specs(specs)
        say(f"[case] batched autotune: {len(specs)} sweeps")
        best, ms = api.autotune_batched(b)
        torch.cuda.synchronize()
        say("   best", best, ms)
        assert 0 <= best < api.L.sweep_tile_config_count() and ms > 0.0
        assert api.batched_config_for(b) == best
        pa, na = api.sweep_eval_batched(b)                       # tile_config = -1: the tuned one
        pb, nb = api.sweep_eval_batched(b, tile_config=best)
        torch.cuda.synchronize()
        assert torch.equal(pa, pb) and torch.equal(na, nb)
        for k, s in enumerate(specs):
            ref = oracle.sweep(s.path, s.profile, s.n_u, s.n_v)
            ok, r = parity(ref.pos, ref.nrm, ref.kappa, b.view(pa, k).double().cpu().numpy(),
                           b.view(na, k).double().cpu().numpy(), TOL[torch.float32])
            assert ok, (k, r)
        lines = [ln.split() for ln in cache.read_text().splitlines() if not ln.startswith("#")]
        mine = [ln for ln in lines if ln[0] == "batch"]
        assert mine and int(mine[-1][8]) == best
    finally:
        os.environ.pop("SWEEP_TUNE_CACHE", None)
