"""Parity cases run against the bounds-checked library (PMLPIC_LIB=libpmlpic_check.so): every
kernel form of the step (2D and 3D tiled push, the 3D one-launch tile push, unfused and
unsorted forms, the deterministic mode, weight damping) and the pushed adjoint, each compared
with the FP64 oracle; any failed bounds check raises from the library call.  Started by
tests/test_gpu_checked_build.py in a process of its own."""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)
sys.path.insert(0, os.path.dirname(HERE))

from gpu_helpers import both, compare_fields, compare_particles  # noqa: E402
from paper_2201_09084_amd import adjoint as A  # noqa: E402
from paper_2201_09084_amd import binding as B  # noqa: E402
from paper_2201_09084_amd import workloads as W  # noqa: E402


def case(dim, order, seed, alpha_mode=W.ALPHA_DAMPED):
    if dim == 2:
        cfg = W.SimConfig(dim=2, n=(37, 29, 1), pml=((6, 9), (7, 5), (0, 0)), dx=(1.0, 0.9, 1.0), dt=0.6,
                          shape_order=order, alpha_mode=alpha_mode, damping_scale=1.3,
                          sigma_coef=((0.0, 0.5, 0.0, 2.5), (0.2, 0.0, 3.0), (0.0,)), push=1, precision=64,
                          tile=(8, 8, 1), sort_interval=3)
    else:
        cfg = W.SimConfig(dim=3, n=(21, 19, 17), pml=((4, 5), (3, 4), (5, 3)), dx=(1.0, 0.9, 1.1), dt=0.45,
                          shape_order=order, alpha_mode=alpha_mode, damping_scale=1.1,
                          sigma_coef=((0.0, 0.0, 0.0, 3.0), (0.1, 0.0, 2.0), (0.0, 1.0, 1.0)), push=1,
                          precision=64, tile=(4, 4, 4), sort_interval=2)
    parts = W.random_particles(cfg, 600, seed=seed, margin=1.5, umax=2.5)
    fields = W.random_split_fields(cfg, seed=seed + 1, amp=0.3)
    return cfg, parts, fields


def main():
    assert B.LIB_PATH.endswith("libpmlpic_check.so"), B.LIB_PATH
    runs = [(2, 2, 0, W.ALPHA_DAMPED), (2, 3, 0, W.ALPHA_WEIGHT), (3, 1, 0, W.ALPHA_DAMPED),
            (3, 2, 0, W.ALPHA_DAMPED), (2, 2, B.FLAG_UNFUSED | B.FLAG_NO_SORT, W.ALPHA_DAMPED),
            (3, 1, B.FLAG_DETERMINISTIC, W.ALPHA_DAMPED), (3, 1, B.FLAG_SEPARATE_FIELDS, W.ALPHA_ONE)]
    for k, (dim, order, flags, amode) in enumerate(runs):
        cfg, parts, fields = case(dim, order, 500 + k, amode)
        g, o = both(cfg, parts, fields, flags=flags)
        g.step(7)
        o.step(7)
        compare_fields(g, o, cfg, 1e-10, "checked %s" % (runs[k],))
        compare_particles(g, o, 1e-10, 1e-10, "checked %s" % (runs[k],))
        d = g.diagnose()
        print("checked case", runs[k], "particles", d["n_particles"], flush=True)
    cfg = W.adjoint_small_config().replace(push=1)
    p = W.adjoint_small_particles(cfg, 8)
    sim = A.make_sim(cfg, A.theta_of(cfg), p, 40, 9)
    sim.forward_ckpt(40)
    sim.backward()
    sim.particle_adjoint(len(p.w))
    print("checked runs ok", flush=True)


if __name__ == "__main__":
    main()
