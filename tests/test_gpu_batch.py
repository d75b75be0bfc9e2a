"""Batched runs (many independent single-particle exit runs stepped by one set of
launches, optionally replayed as a HIP graph) against the same runs stepped alone and
against the FP64 oracle."""
import json
import os

import numpy as np
import pytest

import oracle
from gpu_helpers import compare_fields, compare_particles, say
from paper_2201_09084_amd import binding as B
from paper_2201_09084_amd import workloads as W

pytestmark = pytest.mark.gpu


def _small_runs(n, precision, seed=7):
    runs = W.batch_runs(n, seed=seed, steps_to_cross=25, nmin=24, nmax=72)
    out = []
    for r in runs:
        cfg = r.cfg.replace(precision=precision, pml=((min(r.cfg.pml[0][0], 12),) * 2,
                                                      (min(r.cfg.pml[1][0], 12),) * 2, (0, 0)))
        out.append((cfg, r.particles))
    return out


def _batch(runs, use_graph):
    b = B.PmlPicBatch([c for c, _ in runs], particles_per_run=1, use_graph=use_graph)
    for k, (_, p) in enumerate(runs):
        b.runs[k].add_particles(p.x, p.u, p.w)
    return b


@pytest.mark.parametrize("precision", [32, 64])
@pytest.mark.parametrize("use_graph", [False, True])
def test_batch_equals_runs_stepped_alone(precision, use_graph):
    runs = _small_runs(6, precision)
    b = _batch(runs, use_graph)
    b.step(25)
    b.step(15)
    b.synchronize()
    tol = 1e-6 if precision == 32 else 1e-13
    for k, (cfg, p) in enumerate(runs):
        alone = B.PmlPic(cfg, max_particles=1, flags=B.FLAG_NO_SORT)
        alone.add_particles(p.x, p.u, p.w)
        alone.step(40)
        fb, fa = b.runs[k].fields(), alone.fields()
        scale = max(np.max(np.abs(fa)), 1e-30)
        err = np.max(np.abs(fb - fa)) / scale
        say("run", k, "grid", cfg.n[:2], "pml", cfg.pml[0][0], "max rel diff", err,
            "bitwise" if np.array_equal(fb, fa) else "")
        assert err <= tol, (k, err)
        assert b.runs[k].diagnose()["n_pushes"] == alone.diagnose()["n_pushes"]


@pytest.mark.parametrize("mode", [W.ALPHA_DAMPED, W.ALPHA_WEIGHT])
def test_batch_matches_oracle_fp64(mode):
    runs = [(c.replace(alpha_mode=mode), p) for c, p in _small_runs(3, 64, seed=11)]
    b = _batch(runs, True)
    b.step(30)
    b.synchronize()
    for k, (cfg, p) in enumerate(runs):
        o = oracle.OracleSim(cfg)
        o.add_particles(p.x, p.u, p.w)
        o.step(30)
        compare_fields(b.runs[k], o, cfg, 1e-10, "batch run %d" % k)
        compare_particles(b.runs[k], o, 1e-10, 1e-10, "batch run %d" % k)


def test_graph_replays_match_eager_launches():
    """Several replays of the captured step with eager work (diagnostics, host copies)
    between them; every replay must equal the eager batch."""
    runs = _small_runs(4, 32, seed=13)
    bg = _batch(runs, True)
    be = _batch(runs, False)
    for rep in range(4):
        bg.step(7)
        be.step(7)
        for k in range(len(runs)):
            dg = bg.runs[k].diagnose()
            de = be.runs[k].diagnose()
            assert dg["n_pushes"] == de["n_pushes"]
            assert np.array_equal(bg.runs[k].fields(), be.runs[k].fields()), (rep, k)


def test_launch_shapes_give_identical_results():
    runs = _small_runs(4, 32, seed=17)
    ref = _batch(runs, False)
    ref.step(12)
    for bx in (32, 128, 256):
        b = _batch(runs, True)
        b.set_launch(bx, 300)
        b.step(12)
        for k in range(len(runs)):
            assert np.array_equal(b.runs[k].fields(), ref.runs[k].fields()), (bx, k)


def test_autotuner_picks_a_candidate_and_caches(tmp_path):
    from paper_2201_09084_amd import autotune
    cfgs = [c for c, _ in _small_runs(4, 32, seed=19)]
    path = str(tmp_path / "tune.json")
    bx, grid = autotune.tune_batch(cfgs, cache_path=path, steps=2, reps=1)
    assert bx in autotune.BLOCK_X and grid > 0
    data = json.load(open(path))
    assert len(data) == 1
    entry = list(data.values())[0]
    assert len(entry["candidates"]) == len(autotune.BLOCK_X) * len(autotune.BLOCKS_PER_CU)
    assert tuple(autotune.tune_batch(cfgs, cache_path=path)) == (bx, grid)


def test_batch_rejects_mixed_shapes():
    runs = _small_runs(2, 32)
    cfgs = [runs[0][0], runs[1][0].replace(shape_order=2)]
    with pytest.raises(B.PmlPicError):
        B.PmlPicBatch(cfgs)


@pytest.mark.parametrize("precision", [64, 32])
def test_batch_large_runs_thick_layers_against_oracle(precision):
    """Workload 3's own sizes: runs of 256-512 cells with layers of 8-32 cells (the draw of the
    benchmark's batch), each particle crossing the +x interface after 40 steps, stepped 70
    steps (30 of them with the particle in the layer or gone through the wall) in one batch
    replayed as a graph, against the FP64 oracle: FP64 1e-10, FP32 relative L2 1e-5 per
    component."""
    runs = W.batch_runs(5, seed=21, steps_to_cross=40, nmin=256, nmax=512)
    cfgs = [r.cfg.replace(precision=precision) for r in runs]
    say("runs", [(c.n[0], c.pml[0][0]) for c in cfgs])
    assert max(c.pml[0][0] for c in cfgs) >= 20
    b = B.PmlPicBatch(cfgs, particles_per_run=1, use_graph=True)
    for k, r in enumerate(runs):
        b.runs[k].add_particles(r.particles.x, r.particles.u, r.particles.w)
    b.step(70)
    b.synchronize()
    for k, r in enumerate(runs):
        cfg64 = cfgs[k].replace(precision=64)
        o = oracle.OracleSim(cfg64, parallel=True)
        o.add_particles(r.particles.x, r.particles.u, r.particles.w)
        o.step(70)
        if precision == 64:
            compare_fields(b.runs[k], o, cfg64, 1e-10, "batch run %d" % k)
            compare_particles(b.runs[k], o, 1e-10, 1e-10, "batch run %d" % k)
        else:
            worst = compare_fields(b.runs[k], o, cfg64, 1e-5, "batch fp32 run %d" % k, l2=True)
            say("run", k, "fp32 worst rel L2 %.3e" % worst)
