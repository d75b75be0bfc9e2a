"""The all-cores build of the oracle (liboracle_omp.so: the same source with -fopenmp,
per-thread current buffers summed in thread order) computes the same step as the plain
single-threaded build: fields, current and particles agree to round-off (only the order
of the current sums differs), in 2D and 3D, with the push, removal at the walls and the
binomial filter."""
import numpy as np
import pytest

import oracle
from paper_2201_09084_amd import workloads as W


@pytest.mark.parametrize("dim,order,filt", [(2, 2, 0), (3, 1, 0), (3, 3, 1)])
def test_parallel_build_matches_serial(dim, order, filt):
    if dim == 2:
        cfg = W.SimConfig(dim=2, n=(37, 29, 1), pml=((6, 9), (7, 5), (0, 0)), dx=(1.0, 0.9, 1.0), dt=0.6,
                          shape_order=order, damping_scale=1.3, push=1)
    else:
        cfg = W.SimConfig(dim=3, n=(13, 11, 9), pml=((4, 5), (3, 4), (5, 3)), dx=(1.0, 0.9, 1.1), dt=0.45,
                          shape_order=order, push=1, filter_passes=filt)
    p = W.random_particles(cfg, 2000, seed=1, margin=0.2, umax=2.5)
    F = W.random_split_fields(cfg, seed=2, amp=0.3)
    a, b = oracle.OracleSim(cfg), oracle.OracleSim(cfg, parallel=True)
    for o in (a, b):
        o.set_split_fields(F)
        o.add_particles(p.x, p.u, p.w)
        o.step(5)
    fa, fb = a.split_fields(), b.split_fields()
    assert np.max(np.abs(fa - fb)) <= 1e-13 * np.max(np.abs(fa))
    ja, jb = a.current(), b.current()
    assert np.max(np.abs(ja - jb)) <= 1e-13 * np.max(np.abs(ja))
    ia, Xa, ua, wa = a.particles()
    ib, Xb, ub, wb = b.particles()
    assert len(ia) < len(p.w)                  # some left through the walls
    assert np.array_equal(ia, ib)
    assert np.max(np.abs(Xa - Xb)) <= 1e-12 and np.max(np.abs(ua - ub)) <= 1e-12
    assert np.array_equal(wa, wb)
