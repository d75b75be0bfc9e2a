"""Parity at the benchmark's full sizes, in the launch configuration bench.py times, with
particles inside the PML (the step the paper defines, Sec. II.A: particles enter the layer and
deposit alpha-damped current there).

* The 2D beam centred on the +x interface (1024^2 + 16-cell PML, 1,048,576 particles, a third of
  them in the layer at step 0, the fastest leaving through the outer wall within the window):
  FP64 and FP32 against the FP64 oracle (all-cores build) over 8 steps, every sample and
  particle, and over the 128-step window, every sample every 32 steps.
* The 3D beam whose head fills the +z layer (the benchmark's input): the oracle needs about a
  minute per step at 256^3 + 12 with 16.8M particles, so the parity case is the same workload
  on the largest sub-box it steps in seconds, 128^3 + 12 (2,129,920 particles, the same
  densities and the same beam cylinder ending in the +z layer), FP64 and FP32 against the
  oracle over 2 steps; at the full size, properties that hold at any size (FP32 against FP64
  on the GPU over 16 steps, the FP64 Gauss residual, the particle count).  The sub-box again at
  two particles per cell plus a dense cluster (over 2^22 particles, so that the dense tiles'
  push runs on the second stream as in the benchmark), against the oracle over 2 steps.

Also the beams at their original place (the box centre, hundreds of cells from the layers):
* 2D: FP64 and FP32 against the oracle over 4 steps, then FP32 against the oracle-checked FP64
  GPU path over 128 steps (relative L2 per field component 1e-5, the stated FP32 bound);
* 3D: FP32 against FP64 on the GPU over 10 steps, the FP64 Gauss residual, the particle count.
"""
import numpy as np
import pytest

from gpu_helpers import both, compare_fields, compare_particles, rel_l2, say
from paper_2201_09084_amd import binding as B
from paper_2201_09084_amd import workloads as W

pytestmark = pytest.mark.gpu

FP32_TOL = 1e-5


def _gpu(cfg, parts):
    g = B.PmlPic(cfg, max_particles=len(parts))
    g.add_particles(parts.x, parts.u, parts.w)
    return g


def _field_l2(a, b):
    Fa, Fb = a.fields(), b.fields()
    return [rel_l2(Fa[c], Fb[c]) if np.max(np.abs(Fb[c])) > 0 else float(np.max(np.abs(Fa[c])))
            for c in range(6)]


def test_beam2d_full_size_against_oracle():
    cfg = W.beam2d_config(precision=64)
    parts = W.beam2d_particles(cfg)
    say("beam2d full size, oracle 4 steps")
    g, o = both(cfg, parts)
    g32 = _gpu(cfg.replace(precision=32), parts)
    for s in (g, o, g32):
        s.step(4)
    compare_fields(g, o, cfg, 1e-10, "fp64 full size")
    compare_particles(g, o, 1e-10, 1e-10, "fp64 full size")
    worst = compare_fields(g32, o, cfg, FP32_TOL, "fp32 full size", l2=True)
    say("fp32 vs oracle, worst rel L2", worst)
    compare_particles(g32, o, 1e-4, 1e-4, "fp32 full size")


def test_beam2d_fp32_against_fp64_128_steps():
    cfg = W.beam2d_config(precision=64)
    parts = W.beam2d_particles(cfg)
    g64 = _gpu(cfg, parts)
    g32 = _gpu(cfg.replace(precision=32), parts)
    for k in range(4):
        g64.step(32)
        g32.step(32)
        errs = _field_l2(g32, g64)
        say("step", 32 * (k + 1), ["%.2e" % e for e in errs])
        assert max(errs) <= FP32_TOL, errs
    i64, X64, u64, _ = g64.particles()
    i32, X32, u32, _ = g32.particles()
    assert np.array_equal(i64, i32)
    assert np.max(np.abs(X64 - X32)) < 1e-3
    d64, d32 = g64.diagnose(), g32.diagnose()
    assert d64["n_pushes"] == d32["n_pushes"]
    assert d64["gauss_max"] <= 1e-9 * d64["rho_max"]


def test_beam3d_full_size_properties():
    cfg = W.beam3d_config(precision=64)
    parts = W.beam3d_particles(cfg)
    say("beam3d full size", len(parts))
    g64 = _gpu(cfg, parts)
    g32 = _gpu(cfg.replace(precision=32), parts)
    g64.step(10)
    g32.step(10)
    errs = _field_l2(g32, g64)
    say("beam3d fp32 vs fp64 rel L2", ["%.2e" % e for e in errs])
    assert max(errs) <= FP32_TOL, errs
    d64, d32 = g64.diagnose(), g32.diagnose()
    say("gauss", d64["gauss_max"], d32["gauss_max"], "rho_max", d64["rho_max"])
    assert d64["gauss_max"] <= 1e-9 * d64["rho_max"]
    assert d32["gauss_max"] <= 1e-4 * d32["rho_max"]
    assert d64["n_particles"] == d32["n_particles"] > 0.99 * len(parts)


def test_beam2d_straddling_pml_full_size_against_oracle():
    cfg = W.beam2d_config(precision=64)
    parts = W.beam2d_particles(cfg, straddle=True)
    in_pml = int(np.sum(parts.x[:, 0] > cfg.n[0]))
    say("beam2d straddling +x, %d of %d particles in the layer at step 0" % (in_pml, len(parts)))
    assert in_pml > 0.3 * len(parts)
    g, o = both(cfg, parts, parallel=True)
    g32 = _gpu(cfg.replace(precision=32), parts)
    for k in range(2):
        for s in (g, o, g32):
            s.step(4)
        compare_fields(g, o, cfg, 1e-10, "fp64 straddle @%d" % (4 * k + 4))
        compare_particles(g, o, 1e-10, 1e-10, "fp64 straddle")
        worst = compare_fields(g32, o, cfg, FP32_TOL, "fp32 straddle @%d" % (4 * k + 4), l2=True)
        say("step", 4 * k + 4, "fp32 vs oracle worst rel L2 %.3e" % worst)
        compare_particles(g32, o, 1e-4, 1e-4, "fp32 straddle")
    n_left = o.num_particles
    say("particles left", n_left)
    assert n_left < len(parts)                  # some went through the outer wall
    assert g.num_particles == n_left == g32.num_particles


def test_beam2d_straddling_pml_128_step_window_against_oracle():
    """The 128-step parity window with the beam in the +x layer from its first step: FP64
    and FP32 against the FP64 oracle (all-cores build) every 32 steps, fields and the live
    particles at the end (the fast head leaves through the outer wall meanwhile)."""
    cfg = W.beam2d_config(precision=64)
    parts = W.beam2d_particles(cfg, straddle=True)
    g, o = both(cfg, parts, parallel=True)
    g32 = _gpu(cfg.replace(precision=32), parts)
    for k in range(4):
        for s in (g, o, g32):
            s.step(32)
        compare_fields(g, o, cfg, 1e-10, "fp64 window @%d" % (32 * k + 32))
        worst = compare_fields(g32, o, cfg, FP32_TOL, "fp32 window @%d" % (32 * k + 32), l2=True)
        say("step", 32 * k + 32, "fp32 vs oracle worst rel L2 %.3e" % worst, "particles", o.num_particles)
    # positions (grid units, up to ~1056 cells) to the same relative 1e-10 as the fields: the
    # per-step roundings of two summation orders grow along 128 steps of self-consistent orbits
    compare_particles(g, o, 1e-10 * (cfg.n[0] + 2 * cfg.pml[0][1]), 1e-10, "fp64 window")
    assert g.num_particles == o.num_particles < len(parts)


def test_beam3d_straddling_pml_subbox_against_oracle():
    cfg = W.beam3d_config(precision=64, n=128)
    parts = W.beam3d_particles(cfg, n_beam=32768, straddle=True)
    in_pml = int(np.sum(parts.x[:, 2] > cfg.n[2]))
    say("beam3d 128^3 + 12 straddling +z: %d particles, %d in the layer" % (len(parts), in_pml))
    assert in_pml > 2000
    g, o = both(cfg, parts, parallel=True)
    g32 = _gpu(cfg.replace(precision=32), parts)
    for s in (g, o, g32):
        s.step(2)
    compare_fields(g, o, cfg, 1e-10, "fp64 3d straddle")
    compare_particles(g, o, 1e-10, 1e-10, "fp64 3d straddle")
    worst = compare_fields(g32, o, cfg, FP32_TOL, "fp32 3d straddle", l2=True)
    say("fp32 vs oracle worst rel L2 %.3e" % worst)
    compare_particles(g32, o, 1e-4, 1e-4, "fp32 3d straddle")


def test_beam3d_straddling_pml_subbox_side_stream_against_oracle():
    """The same sub-box at two background particles per cell plus a dense cluster (hundreds
    per cell): with 2^22 particle slots or more the dense tiles' push runs on the handle's
    second stream beside the tile-box push, as in the benchmark; FP64 and FP32 against the
    oracle over 2 steps."""
    cfg = W.beam3d_config(precision=64, n=128)
    parts = W.beam3d_particles(cfg, background_ppc=2.0, n_beam=32768, straddle=True)
    rng = np.random.default_rng(1017)
    n_dense = 4096
    centre = np.array([cfg.n[d] * 0.5 * cfg.dx[d] for d in range(3)])
    xd = centre + rng.normal(0.0, 0.7, (n_dense, 3)) * np.array(cfg.dx[:3])
    parts = W.Particles(x=np.concatenate([parts.x, xd]),
                        u=np.concatenate([parts.u, rng.normal(0.0, 0.03, (n_dense, 3))]),
                        w=np.concatenate([parts.w, np.full(n_dense, 0.01)]))
    say("beam3d 128^3 + 12, 2 per cell + dense cluster: %d particles" % len(parts))
    assert len(parts) >= 2 ** 22
    g, o = both(cfg, parts, parallel=True)
    g32 = _gpu(cfg.replace(precision=32), parts)
    for s in (g, o, g32):
        s.step(2)
    compare_fields(g, o, cfg, 1e-10, "fp64 3d side stream")
    compare_particles(g, o, 1e-10, 1e-10, "fp64 3d side stream")
    worst = compare_fields(g32, o, cfg, FP32_TOL, "fp32 3d side stream", l2=True)
    say("fp32 vs oracle worst rel L2 %.3e" % worst)
    compare_particles(g32, o, 1e-4, 1e-4, "fp32 3d side stream")


def test_beam3d_straddling_pml_full_size_properties():
    cfg = W.beam3d_config(precision=64)
    parts = W.beam3d_particles(cfg, straddle=True)
    say("beam3d full size straddling +z", len(parts))
    g64 = _gpu(cfg, parts)
    g32 = _gpu(cfg.replace(precision=32), parts)
    for k in range(2):
        g64.step(8)
        g32.step(8)
        errs = _field_l2(g32, g64)
        say("step", 8 * k + 8, "beam3d straddle fp32 vs fp64 rel L2", ["%.2e" % e for e in errs])
        assert max(errs) <= FP32_TOL, errs
    d64, d32 = g64.diagnose(), g32.diagnose()
    say("gauss", d64["gauss_max"], d32["gauss_max"], "rho_max", d64["rho_max"], "pml energy", d64["u_pml"])
    assert d64["gauss_max"] <= 1e-9 * d64["rho_max"]
    assert d32["gauss_max"] <= 1e-4 * d32["rho_max"]
    assert d64["n_particles"] == d32["n_particles"] > 0.99 * len(parts)
    assert d64["n_particles"] < len(parts)      # beam particles left through the +z wall
