"""Benchmark of the damped-current PML PIC step on one MI355X.

Default workload (the headline configuration): 3D 256^3 cells + 12-cell PML on every face
(cubic profile), linear shape, c dt = 0.5, FP32 fields and particles; 16,777,216 thermal
background electrons (1 per physical cell, T = 1e-3 m c^2) plus a gamma = 5 beam of 65,536
electrons in a radius-8 cylinder moving along +z, whose head fills the +z PML from step 0, so
every timed step deposits alpha-damped current in that layer (Sec. II.A).  Every step runs
sort_particles (every 8 steps), gather_push + deposit_current, the alpha damping and
update_yee_pml.  Inputs are seeded synthetic data, resident in HBM before timing.

Prints one JSON line: particle-pushes/s over the timed steps (whole job), the cell update
rate, the roofline of the dominant kernel (algorithmic bytes / its average duration from HIP
events on the library's stream) and of the whole step, the same steps on the plain FP64 GPU
path, and the FP64 CPU oracle timed on a bounded sample on the host (all cores, and one
thread).
"""
import argparse
import hashlib
import json
import os
import sys
import tempfile
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# the HIP kernels behind a timed phase (phase, dim, shape order), for the roofline record
PHASE_KERNELS = {
    ("gather_push", 3, 1): "k_push3d_tiles (tiles that are not dense) + k_push_deposit_tiles (dense tiles)",
    ("gather_push", 2, 2): "k_push_deposit_tiles",
    ("update_yee_pml", 3, 1): "k_fused_3d",
    ("update_yee_pml", 2, 2): "k_fused_2d",
}


def kernel_source_hash():
    """Hash of the kernel and launcher sources (the host control in api.hip launches them but
    does not change what one launch moves)."""
    h = hashlib.sha256()
    for f in ("particles.hip", "push3d.hip", "fields.hip", "fused3d.hip", "batch.hip", "beam.hip", "common.h",
              "field_core.h", "fused2d.h", "particle_core.h"):
        with open(os.path.join(ROOT, "paper_2201_09084_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_bytes(workload, phase, precision):
    """HBM bytes per launch from the committed PMC summary, if the kernel sources are
    the ones it was measured on (else None)."""
    tf = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(tf):
        return None
    with open(tf) as fh:
        t = json.load(fh)
    key = "%s/%s/fp%d" % (workload, phase, precision)
    if t.get("source_hash") != kernel_source_hash():
        return None
    return t.get("bytes_per_launch", {}).get(key)


def algorithmic_bytes(cfg, phase, pushes_per_launch, esz, occupied=0):
    """Algorithmic HBM bytes of one launch of a phase (each array read/written once).  The
    push launch also deposits: beside its particles it reads the six field components and
    writes the three current components once per occupied cell."""
    dim = cfg.dim
    cells = cfg.total_cells()
    pml = cfg.pml_cells()
    nsplit_e = 1 if dim == 2 else 3
    if phase == "gather_push":
        per = (4 + dim * esz + 3 * esz + esz) + (4 + dim * esz + 3 * esz)   # read + write
        return per * pushes_per_launch + occupied * (6 + 3) * esz
    if phase == "update_yee_pml_E":
        return cells * (3 + 3 + 3 + 3) * esz + pml * 2 * nsplit_e * esz     # E r+w, B r, J r
    if phase == "update_yee_pml_B":
        return cells * (3 + 3 + 3) * esz + pml * 2 * nsplit_e * esz         # B r+w, E r
    if phase == "update_yee_pml":   # one pass: E, B r+w, J r; split parts of E and B r+w
        return cells * (6 + 6 + 3) * esz + pml * 4 * nsplit_e * esz
    if phase == "clear_current":
        return cells * 3 * esz
    if phase == "filter_current":   # J r+w
        return cells * 6 * esz
    return None


def step_bytes(cfg, pushes_per_step, occupied_cells, esz):
    """Algorithmic HBM bytes of one whole step (FP32 per-unit figures scaled by esz/4):
    72 B per interior cell-update, 144 B (3D) / 112 B (2D) per PML cell-update, +24 B per
    cell holding particles (the gather's field read), 52 B (2D) / 60 B (3D) per push."""
    k = esz / 4.0
    cells, pml = cfg.total_cells(), cfg.pml_cells()
    per_pml = 144 if cfg.dim == 3 else 112
    per_push = 60 if cfg.dim == 3 else 52
    return k * ((cells - pml) * 72 + pml * per_pml + occupied_cells * 24 + pushes_per_step * per_push)


def occupied_cells(cfg, parts):
    """Cells holding at least one particle at the start (host count)."""
    import numpy as np
    M = [cfg.n[d] + cfg.pml[d][0] + cfg.pml[d][1] for d in range(cfg.dim)]
    idx = np.zeros(len(parts), dtype=np.int64)
    for d in reversed(range(cfg.dim)):
        c = np.floor(parts.x[:, d] / cfg.dx[d]).astype(np.int64) + cfg.pml[d][0]
        idx = idx * M[d] + c
    return int(np.unique(idx).size)


def run_gpu(args, cfg, parts, setup=None):
    """Timed region: args.steps plain steps between two synchronisations.  The per-kernel
    durations come from a second run of the same inputs through the same warm-up and
    timed steps, stepped with HIP events around every kernel phase on the library's
    stream: the launches timed are those of the timed steps, without the event markers
    slowing the timed run itself (they add idle time and about 3 us to each bracketed
    launch)."""
    import torch
    from paper_2201_09084_amd import binding as B

    def start():
        sim = B.PmlPic(cfg, max_particles=max(len(parts), int(cfg.max_particles)))
        if setup is not None:
            setup(sim)
        else:
            sim.add_particles(parts.x, parts.u, parts.w)
        torch.cuda.synchronize()
        if args.warmup:
            sim.step(args.warmup)
        return sim

    sim = start()
    d0 = sim.diagnose()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    d1 = sim.diagnose(allow_nonfinite=True)
    elapsed = t1 - t0
    pushes = d1["n_pushes"] - d0["n_pushes"]
    sim.close()
    twin = start()
    e0 = twin.diagnose()
    phases = twin.step_profiled(args.steps)
    prof_pushes = twin.diagnose(allow_nonfinite=True)["n_pushes"] - e0["n_pushes"]
    twin.close()
    return elapsed, pushes, phases, d0, d1, args.steps, prof_pushes


def run_batch(args):
    """Workload 3: 256 independent 2D single-particle exit runs (N ~ U{64..512}, PML ~
    U{8..32}, angle ~ U[0, 60] deg, ln gamma ~ U[ln 1.1, ln 20]), FP32, stepped as one
    batch whose step is a replayed HIP graph, launch shape from the autotuner."""
    import torch
    from paper_2201_09084_amd import autotune
    from paper_2201_09084_amd import binding as B
    from paper_2201_09084_amd import workloads as W
    runs = W.batch_runs(256)
    cfgs = [r.cfg for r in runs]
    cells = sum(c.total_cells() for c in cfgs)
    print("bench: batch of %d runs, %d cells in total, fp32; warmup %d, timed %d"
          % (len(runs), cells, args.warmup, args.steps), file=sys.stderr, flush=True)
    bx, grid = autotune.tune_batch(cfgs, cache_path=args.tune_cache)
    b = B.PmlPicBatch(cfgs, particles_per_run=1, use_graph=True)
    b.set_launch(bx, grid)
    for k, r in enumerate(runs):
        b.runs[k].add_particles(r.particles.x, r.particles.u, r.particles.w)
    if args.warmup:
        b.step(args.warmup)
    b.synchronize()
    p0 = sum(r.diagnose()["n_pushes"] for r in b.runs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(args.steps)
    b.synchronize()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    pushes = sum(r.diagnose()["n_pushes"] for r in b.runs) - p0
    n_prof = max(10, min(50, args.steps // 10))
    phases = b.step_profiled(n_prof)
    dom = max(phases.items(), key=lambda kv: kv[1][0])
    name, (ms_total, launches) = dom
    avg_s = ms_total / 1e3 / launches
    per = {k: sum(algorithmic_bytes(c, k, 0, 4) for c in cfgs)
           for k in ("update_yee_pml_B", "update_yee_pml_E", "update_yee_pml", "clear_current")}
    roof = None
    if name in per:
        ach = per[name] / avg_s / 1e9
        roof = {"kernel": name, "bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": traffic_bytes("batch", name, 32),
                "avg_launch_us": round(avg_s * 1e6, 2), "algorithmic_bytes_per_launch": int(per[name]),
                "timing": "HIP events around each kernel in %d eager steps after the timed graph replays" % n_prof}
    out = {
        "metric": "PIC particle-pushes/s & Yee+PML cell-updates/s; FP32 vs FP64 at stated err",
        "value": cells * args.steps / elapsed, "unit": "cell-updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * elapsed / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "batch", "runs": len(runs), "cells": cells, "launch": [bx, grid],
                   "graph": True},
        "particle_pushes_per_s": pushes / elapsed,
        "phases_ms_per_launch": {k: round(v[0] / v[1], 4) for k, v in phases.items()},
        "roofline": roof, "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def cpu_baseline(cfg, parts, n_steps, cells=None, parallel=False):
    import oracle
    oracle.build_library(force=False)
    o = oracle.OracleSim(cfg.replace(precision=64), parallel=parallel)
    if cells is not None:
        o.set_conductor(cells)
    o.add_particles(parts.x, parts.u, parts.w)
    t0 = time.perf_counter()
    o.step(n_steps)
    t1 = time.perf_counter()
    return len(parts) * n_steps / (t1 - t0), t1 - t0


def cavity_sample(cfg, parts, steps):
    """The source particles that have crossed the entry wall after `steps` steps, at their
    ballistic positions (a sample of the cavity workload for the CPU baseline)."""
    import numpy as np
    gam = np.sqrt(1.0 + np.sum(parts.u ** 2, axis=1))
    x = parts.x + steps * cfg.dt * parts.u / gam[:, None]
    lo = -cfg.pml[2][0] * cfg.dx[2]
    hi = (cfg.n[2] + cfg.pml[2][1]) * cfg.dx[2]
    keep = (x[:, 2] >= lo + 1.0) & (x[:, 2] < hi - 1.0)
    from paper_2201_09084_amd import workloads as W
    return W.Particles(x=x[keep], u=parts.u[keep], w=parts.w[keep])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default: 2000 beam2d, 100 beam3d, 600 batch, 300 sp3d, 200 cavity)")
    ap.add_argument("--warmup", type=int, default=None,
                    help="untimed steps first (default 10; cavity: 150, so that the beam fills the box)")
    ap.add_argument("--workload", choices=["beam2d", "beam3d", "batch", "sp3d", "cavity"], default="beam3d")
    ap.add_argument("--input", choices=["straddle", "centre"], default="straddle",
                    help="beams: straddling the PML face they move toward from step 0 (default), or at the box centre")
    ap.add_argument("--no-fp64", action="store_true", help="skip the plain FP64 GPU comparison run")
    ap.add_argument("--tune-cache", default=os.path.join(tempfile.gettempdir(), "pmlpic_autotune.json"),
                    help="where the batch autotuner keeps the launch shape it picked")
    ap.add_argument("--precision", type=int, choices=[32, 64], default=32)
    ap.add_argument("--cpu-steps", type=int, default=8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only copy a MIB-sized device buffer 10 times (calibrates the HBM byte counters)")
    ap.add_argument("--atomic-rates", action="store_true",
                    help="only measure the LDS and global float atomic add rates (pml_pic_atomic_rates)")
    args = ap.parse_args()
    if args.atomic_rates:
        import torch
        from paper_2201_09084_amd import binding as B
        torch.cuda.set_device(0)
        r = B.atomic_rates()
        cus = torch.cuda.get_device_properties(0).multi_processor_count
        clock_hz = 2.4e9
        print(json.dumps({"atomic_rates_lane_adds_per_s": r, "compute_units": cus,
                          "per_cu_per_clock_at_2.4GHz": {k: v / (cus * clock_hz) for k, v in r.items()}}),
              flush=True)
        return
    if args.copy_calibration:
        import torch
        n = args.copy_calibration * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(10):
            b.copy_(a)
        torch.cuda.synchronize()
        print("copied %d MiB x 10" % args.copy_calibration, flush=True)
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2201_09084_amd import workloads as W

    torch.cuda.set_device(0)
    if args.steps is None:
        args.steps = {"beam2d": 2000, "beam3d": 100, "batch": 600, "sp3d": 300, "cavity": 200}[args.workload]
    if args.warmup is None:
        args.warmup = 150 if args.workload == "cavity" else 10
    if args.workload == "batch":
        return run_batch(args)
    straddle = args.input == "straddle"
    if args.workload == "beam2d":
        cfg = W.beam2d_config(precision=args.precision)
        parts = W.beam2d_particles(cfg, straddle=straddle)
        wl = {"workload": "beam2d", "grid": "1024x1024+16pml", "particles": len(parts),
              "shape_order": 2, "steps_total": args.warmup + args.steps,
              "input": "Gaussian beam centred on the +x PML interface" if straddle else "beam at the box centre"}
    elif args.workload == "beam3d":
        cfg = W.beam3d_config(precision=args.precision)
        parts = W.beam3d_particles(cfg, straddle=straddle)
        wl = {"workload": "beam3d", "grid": "256^3+12pml", "particles": len(parts),
              "shape_order": 1, "steps_total": args.warmup + args.steps,
              "input": ("thermal background 1/cell + gamma-5 beam whose head fills the +z PML"
                        if straddle else "thermal background 1/cell + gamma-5 beam at the box centre")}
    elif args.workload == "cavity":   # the beam through the cavity of Sec. IV.A / App. A.2
        cfg = W.cavity_config(precision=args.precision)
        parts = W.cavity_beam(cfg)
        cond_cells = W.cavity_conductor(cfg)
        wl = {"workload": "cavity", "grid": "64x64x108+10pml(z)", "source_particles": len(parts),
              "shape_order": 1, "filter_passes": 1, "alpha_faces": "z: undamped entry, Eq. alpha exit",
              "steps_total": args.warmup + args.steps}

        def setup(sim, cells=cond_cells, parts=parts):
            sim.set_conductor(cells)
            sim.set_source(parts.x, parts.u, parts.w, axis=2)
    else:   # the 3D single-particle numerics of App. A: CK at c dt = dx, cubic shape, filter
        cfg = W.single_particle_3d_config(precision=args.precision)
        parts = W.single_particle(cfg, beta=0.9)
        wl = {"workload": "sp3d", "grid": "128^3+8pml", "particles": 1, "shape_order": 3,
              "solver": "CK", "filter_passes": 1, "steps_total": args.warmup + args.steps}
    print("bench: %s, %d particles, %d cells, fp%d; warmup %d, timed %d" %
          (args.workload, len(parts), cfg.total_cells(), args.precision, args.warmup, args.steps),
          file=sys.stderr, flush=True)

    elapsed, pushes, phases, d0, d1, n_prof, prof_pushes = run_gpu(
        args, cfg, parts, setup if args.workload == "cavity" else None)
    esz = 4 if args.precision == 32 else 8
    cells = cfg.total_cells()
    ms_per_step = 1e3 * elapsed / args.steps
    per_cell = args.workload == "sp3d"   # one particle: the field update is the work
    value = cells * args.steps / elapsed if per_cell else pushes / elapsed
    print("bench: %.3f ms/step, %.3e %s, phases %s" % (ms_per_step, value, "cell-updates/s" if per_cell else "pushes/s", phases),
          file=sys.stderr, flush=True)

    # dominant kernel: the phase with the largest total time
    dom = max(phases.items(), key=lambda kv: kv[1][0])
    name, (ms_total, launches) = dom
    avg_s = ms_total / 1e3 / launches
    roof = None
    occ = occupied_cells(cfg, parts) if not per_cell and args.workload in ("beam2d", "beam3d") else 0
    per_launch = algorithmic_bytes(cfg, name, prof_pushes / max(1, phases.get("gather_push", (0, 1))[1]), esz, occ)
    if per_launch is not None:
        ach = per_launch / avg_s / 1e9
        roof = {"kernel": name, "bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None,
                "avg_launch_us": round(avg_s * 1e6, 2), "algorithmic_bytes_per_launch": int(per_launch),
                "timing": "HIP events around each kernel phase on the library stream, in a second run "
                          "of the same inputs through the same warm-up and %d timed steps" % n_prof}
        if name == "gather_push":
            roof["model"] = "%d B/push" % ((60 if cfg.dim == 3 else 52) * esz // 4) + (
                " + %d B/occupied cell (fields read, current written), %d occupied cells" % (9 * esz, occ)
                if occ else "")
        kern = PHASE_KERNELS.get((name, cfg.dim, cfg.shape_order))
        if kern:
            roof["kernels"] = kern
        roof["traffic"] = traffic_bytes(args.workload, name, args.precision)

    srf = None
    if not per_cell and args.workload in ("beam2d", "beam3d"):
        sb = step_bytes(cfg, pushes / args.steps, occ, esz)
        ach = sb / (ms_per_step * 1e-3) / 1e9
        srf = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
               "frac": round(ach / HBM_PEAK_GBS, 4), "algorithmic_bytes_per_step": int(sb),
               "occupied_cells": occ,
               "model": "72 B/interior cell, %d B/PML cell, 24 B/occupied cell, %d B/push (x%d for FP64)"
                        % (144 if cfg.dim == 3 else 112, 60 if cfg.dim == 3 else 52, esz // 4)}

    fp64 = None
    if not args.no_fp64 and args.precision == 32 and args.workload in ("beam2d", "beam3d"):
        import torch
        from paper_2201_09084_amd import binding as B
        cfg64 = cfg.replace(precision=64)
        sim = B.PmlPic(cfg64, max_particles=len(parts))
        sim.add_particles(parts.x, parts.u, parts.w)
        if args.warmup:
            sim.step(args.warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(args.steps)
        torch.cuda.synchronize()
        e64 = time.perf_counter() - t0
        sim.close()
        del sim
        torch.cuda.empty_cache()
        fp64 = {"ms_per_step": 1e3 * e64 / args.steps, "speedup_fp32_over_fp64": e64 / elapsed,
                "accuracy": "FP32 within relative L2 1e-5 per field component of the FP64 oracle on this "
                            "workload's parity cases (tests/test_gpu_fullsize.py); FP64 within 1e-10"}
        print("bench: plain FP64 GPU path %.3f ms/step" % fp64["ms_per_step"], file=sys.stderr, flush=True)

    cpu = None
    if not args.no_cpu_baseline and args.workload == "beam3d":
        import oracle
        # bounded sample: the same workload on the 128^3 + 12 sub-box (same densities, the
        # beam's head in the +z layer), one step with all cores; one thread on 64^3 + 12
        sub = W.beam3d_config(precision=64, n=128)
        sp = W.beam3d_particles(sub, n_beam=32768, straddle=straddle)
        v, secs = cpu_baseline(sub, sp, 1, parallel=True)
        sub1 = W.beam3d_config(precision=64, n=64)
        sp1 = W.beam3d_particles(sub1, n_beam=8192, straddle=straddle)
        v1, secs1 = cpu_baseline(sub1, sp1, 1, parallel=False)
        cpu = {"value": v, "unit": "particle-pushes/s", "cores": oracle.num_threads(), "kind": "oracle",
               "sample": ("1 step of the same workload on the 128^3 + 12-cell sub-box (same densities: "
                          "%d particles, beam head in the +z PML), FP64 C oracle built with OpenMP over "
                          "cell loops and particles (per-thread current buffers), %d threads, %.1f s"
                          % (len(sp), oracle.num_threads(), secs)),
               "single_thread": {"value": v1, "cores": 1,
                                 "sample": "1 step on the 64^3 + 12-cell sub-box (%d particles), plain "
                                           "single-threaded oracle, %.1f s" % (len(sp1), secs1)}}
    elif not args.no_cpu_baseline:
        n_cpu = 2 if per_cell else args.cpu_steps
        sample_parts = parts
        if args.workload == "cavity":
            n_cpu = 1
            sample_parts = cavity_sample(cfg, parts, args.warmup)
        v, secs = cpu_baseline(cfg, sample_parts, n_cpu, cond_cells if args.workload == "cavity" else None)
        if per_cell:
            v = v / len(parts) * cells
        cpu = {"value": v, "unit": "cell-updates/s" if per_cell else "particle-pushes/s", "cores": 1,
               "kind": "oracle",
               "sample": ("%d steps of the same workload from its initial state (%d particles), "
                          "FP64 single-threaded C oracle, %.1f s" % (n_cpu, len(sample_parts), secs))
               if args.workload != "cavity" else
               ("%d oracle steps (FP64, single-threaded C) of the cavity with the %d beam particles that "
                "have entered after the warm-up, placed on their ballistic paths, with the conductor, %.1f s" % (n_cpu, len(sample_parts), secs))}

    out = {
        "metric": "PIC particle-pushes/s & Yee+PML cell-updates/s; FP32 vs FP64 at stated err",
        "value": value,
        "unit": "cell-updates/s" if per_cell else "particle-pushes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == 32 else "f64",
        "data": "synthetic",
        "config": wl,
        "cell_updates_per_s": cells * args.steps / elapsed,
        "phases_ms_per_step": {k: round(v[0] / n_prof, 4) for k, v in phases.items()},
        "gauss_residual_fp64": d1["gauss_max"],
        "particles_left": d1["n_particles"],
        "roofline": roof,
        "step_roofline": srf,
        "fp64_gpu": fp64,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
