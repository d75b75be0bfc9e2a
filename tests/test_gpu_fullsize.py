"""Parity at the benchmark's full sizes, in the launch configuration bench.py times.

* The 2D beam (1024^2 + 16-cell PML, 1,048,576 particles, quadratic shape): the FP64 and FP32
  GPU paths against the FP64 oracle over 4 steps (about 10 s of oracle time), every field
  sample and every particle; then FP32 against the oracle-checked FP64 GPU path over the
  128-step window (relative L2 per field component 1e-5, the stated FP32 bound).
* The 3D beam (256^3 + 12-cell PML, 16,842,752 particles): too large for the oracle, so
  properties that hold at any size: FP32 against FP64 on the GPU over 10 steps (relative L2
  per field component), the FP64 Gauss residual of the FP64 run at round-off relative to the
  charge density, and the particle count.
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
