"""GPU parity of the beam-transport pieces of the cavity run (Sec. IV.A, App. A.2) against
the FP64 oracle on the same seeded inputs: per-face alpha modes, conductor cells, the beam
source injected through the entry PML, and the slab moments of the <u_x> diagnostic.

Tolerances are those of the other parity tests: FP64 agrees to round-off (1e-10 relative
max error over a few steps), FP32 to 1e-5 relative L2 per field component.
"""
import numpy as np
import pytest

from gpu_helpers import both, compare_current, compare_fields, compare_particles, say
from paper_2201_09084_amd import binding as B
from paper_2201_09084_amd import workloads as W

pytestmark = pytest.mark.gpu

ONE, ZERO, DAMPED = 2, 1, 3     # per-face entries: 1 + mode


def _faces_case(dim, seed, n_particles=300, precision=64):
    if dim == 2:
        cfg = W.SimConfig(dim=2, n=(37, 29, 1), pml=((6, 9), (7, 5), (0, 0)), dx=(1.0, 0.9, 1.0), dt=0.6,
                          shape_order=2, alpha_mode=W.ALPHA_DAMPED, damping_scale=1.3,
                          sigma_coef=((0.0, 0.5, 0.0, 2.5), (0.2, 0.0, 3.0), (0.0,)), push=1,
                          precision=precision, tile=(8, 8, 1), sort_interval=3,
                          alpha_face=((ONE, 0), (ZERO, DAMPED), (0, 0)))
    else:
        cfg = W.SimConfig(dim=3, n=(13, 11, 9), pml=((4, 5), (3, 4), (5, 3)), dx=(1.0, 0.9, 1.1), dt=0.45,
                          shape_order=1, alpha_mode=W.ALPHA_DAMPED, damping_scale=1.1,
                          sigma_coef=((0.0, 0.0, 0.0, 3.0), (0.1, 0.0, 2.0), (0.0, 1.0, 1.0)), push=1,
                          precision=precision, tile=(4, 4, 4), sort_interval=2,
                          alpha_face=((0, ZERO), (ONE, 0), (ONE, DAMPED)))
    parts = W.random_particles(cfg, n_particles, seed=seed, margin=1.5, umax=2.5)
    fields = W.random_split_fields(cfg, seed=seed + 1, amp=0.3)
    return cfg, parts, fields


@pytest.mark.parametrize("flags", [B.FLAG_KEEP_CURRENT, B.FLAG_SEPARATE_DAMP | B.FLAG_KEEP_CURRENT])
@pytest.mark.parametrize("dim", [2, 3])
def test_per_face_alpha_matches_oracle(dim, flags):
    cfg, parts, fields = _faces_case(dim, seed=500 + dim)
    say("faces", dim, flags)
    g, o = both(cfg, parts, fields, flags=flags)
    for k in range(3):
        g.step(1)
        o.step(1)
        compare_fields(g, o, cfg, 1e-10, "step %d" % (k + 1))
        compare_current(g, o, 1e-10, "J")
        compare_particles(g, o, 1e-10, 1e-10, "step %d" % (k + 1))


def _conductor_cells(o):
    M = o.M
    cells = np.zeros((M[2], M[1], M[0]), np.uint8)
    cells[: M[2] // 2, M[1] // 2:, : M[0] // 3] = 1        # a block reaching into three PMLs
    cells[M[2] - 4:, :, M[0] - 5:] = 1                     # and one in a corner
    return cells


@pytest.mark.parametrize("filter_passes", [0, 1])
@pytest.mark.parametrize("flags", [0, B.FLAG_UNFUSED | B.FLAG_NO_SORT])
def test_conductor_matches_oracle(flags, filter_passes):
    cfg, parts, fields = _faces_case(3, seed=610 + filter_passes)
    cfg = cfg.replace(conductor=1, alpha_face=((0, 0), (0, 0), (0, 0)), filter_passes=filter_passes)
    say("conductor", flags, filter_passes)
    g, o = both(cfg, parts, fields, flags=flags)
    cells = _conductor_cells(o)
    o.set_conductor(cells)
    g.set_conductor(cells)
    compare_fields(g, o, cfg, 1e-15, "after set_conductor")
    for k in range(3):
        g.step(2)
        o.step(2)
        compare_fields(g, o, cfg, 1e-10, "step %d" % (2 * k + 2))
        compare_particles(g, o, 1e-10, 1e-10, "step %d" % (2 * k + 2))
    F = g.split_fields()
    for c in range(6):       # both parts of every flagged sample are exactly zero
        nz = np.argwhere(F[2 * c] != 0.0)
        for (k3, j3, i3) in nz[:: max(1, len(nz) // 400)]:
            assert not o.sample_in_conductor(c, i3, j3, k3)


def test_conductor_removed_and_fp32():
    cfg64, parts, fields = _faces_case(3, seed=640)
    cfg64 = cfg64.replace(conductor=1)
    cfg32 = cfg64.replace(precision=32)
    g, _ = both(cfg32, parts, fields)
    _, o = both(cfg64, parts, fields)
    cells = _conductor_cells(o)
    g.set_conductor(cells)
    o.set_conductor(cells)
    g.step(5)
    o.step(5)
    compare_fields(g, o, cfg64, 1e-5, "fp32 conductor", l2=True)
    g.set_conductor(None)
    o.set_conductor(None)
    g.step(2)
    o.step(2)
    compare_fields(g, o, cfg64, 1e-5, "fp32 after removal", l2=True)


def _source_case(push, seed, ns=400, precision=64, sort_interval=0):
    cfg = W.SimConfig(dim=3, n=(12, 10, 16), pml=((0, 0), (0, 0), (5, 6)), dt=0.5, shape_order=1,
                      alpha_mode=W.ALPHA_DAMPED, sigma_coef=W.paper_conductivity_profile(5), push=push,
                      charge=1.0, mass=3.0, precision=precision, sort_interval=sort_interval,
                      max_source=ns, alpha_face=((0, 0), (0, 0), (ONE, DAMPED)))
    rng = np.random.default_rng(seed)
    x = np.stack([rng.uniform(2.0, 10.0, ns), rng.uniform(2.0, 8.0, ns), rng.uniform(-25.0, -5.2, ns)], axis=1)
    x[:20, 2] = rng.uniform(-4.5, 10.0, 20)          # some already inside at the start
    u = np.stack([rng.normal(0.0, 0.05, ns), rng.normal(0.0, 0.05, ns), rng.uniform(1.0, 6.0, ns)], axis=1)
    w = rng.uniform(0.5, 1.5, ns) * 0.05
    return cfg, (x, u, w)


@pytest.mark.parametrize("push,sort_interval", [(0, 0), (1, 0), (1, 3)])
def test_source_injection_matches_oracle(push, sort_interval):
    cfg, (x, u, w) = _source_case(push, seed=700 + push + sort_interval, sort_interval=sort_interval)
    say("source", push, sort_interval)
    g, o = both(cfg, max_particles=len(w) + 10, flags=B.FLAG_KEEP_CURRENT)
    g.set_source(x, u, w, axis=2)
    o.set_source(x, u, w, axis=2)
    for N in (1, 4, 10, 25, 45):
        g.step(N - o.step_count)
        o.step(N - o.step_count)
        compare_particles(g, o, 1e-10, 1e-10, "step %d" % N)
        compare_fields(g, o, cfg, 1e-10, "step %d" % N)
        compare_current(g, o, 1e-10, "J step %d" % N)
    assert g.num_particles > 0


@pytest.mark.parametrize("sort_interval", [0, 5])
def test_source_injection_2d_one_pass(sort_interval):
    """2D (one-pass field update, current boxes): a source entering through the low x PML;
    between sorts the injected particles are an unsorted tail pushed on their own."""
    ns = 300
    cfg = W.SimConfig(dim=2, n=(40, 24, 1), pml=((7, 8), (0, 0), (0, 0)), dt=0.6, shape_order=2,
                      alpha_mode=W.ALPHA_DAMPED, sigma_coef=W.cubic_profile(3.0), push=1, charge=1.0,
                      mass=2.0, precision=64, sort_interval=sort_interval, max_source=ns,
                      alpha_face=((ONE, DAMPED), (0, 0), (0, 0)))
    rng = np.random.default_rng(750 + sort_interval)
    x = np.stack([rng.uniform(-30.0, -7.2, ns), rng.uniform(3.0, 21.0, ns)], axis=1)
    u = np.stack([rng.uniform(1.0, 5.0, ns), rng.normal(0.0, 0.1, ns), rng.normal(0.0, 0.1, ns)], axis=1)
    w = rng.uniform(0.5, 1.5, ns) * 0.05
    g, o = both(cfg, max_particles=ns, flags=B.FLAG_KEEP_CURRENT)
    g.set_source(x, u, w, axis=0)
    o.set_source(x, u, w, axis=0)
    for N in (2, 7, 16, 33, 60):
        g.step(N - o.step_count)
        o.step(N - o.step_count)
        compare_particles(g, o, 1e-10, 1e-10, "step %d" % N)
        compare_fields(g, o, cfg, 1e-10, "step %d" % N)
        compare_current(g, o, 1e-10, "J step %d" % N)
    assert g.num_particles > 50


def test_source_rejected_and_replaced():
    cfg, (x, u, w) = _source_case(0, seed=731, ns=50)
    g, o = both(cfg, max_particles=60)
    with pytest.raises(B.PmlPicError):
        g.set_source(x, -u, w, axis=2)                     # moving away from the box
    with pytest.raises(B.PmlPicError):
        g.set_source(np.concatenate([x, x]), np.concatenate([u, u]), np.concatenate([w, w]), axis=2)   # > capacity
    g.set_source(x[:10], u[:10], w[:10], axis=2)
    g.set_source(x, u, w, axis=2)                          # replaces the first one
    o.set_source(x[:10], u[:10], w[:10], axis=2)           # ids as in the GPU run
    o.set_source(x, u, w, axis=2)
    g.step(30)
    o.step(30)
    compare_particles(g, o, 1e-10, 1e-10, "replaced source")


@pytest.mark.parametrize("dim", [2, 3])
def test_slab_moments_match_oracle(dim):
    cfg, parts, fields = _faces_case(dim, seed=800 + dim, n_particles=2000)
    g, o = both(cfg, parts, fields)
    g.step(3)
    o.step(3)
    ax = dim - 1
    lo, hi = -cfg.pml[ax][0] * cfg.dx[ax], (cfg.n[ax] + cfg.pml[ax][1]) * cfg.dx[ax]
    edges = np.linspace(lo + 0.3, hi - 0.7, 11)
    mg = g.slab_moments(ax, edges)
    mo = o.slab_moments(ax, edges)
    assert np.array_equal(mg[:, 0], mo[:, 0])
    assert np.allclose(mg[:, 1:], mo[:, 1:], rtol=1e-10, atol=1e-10 * np.max(np.abs(mo[:, 1:])))
    assert mg[:, 0].sum() > 100


def test_mini_cavity_all_pieces():
    """A reduced cavity run: pipe and cavity conductors, a proton-like source entering
    through the undamped low z PML and leaving through the damped high one, Yee at the CFL
    limit, one filter pass, the slab moments; FP64 against the oracle."""
    cfg = W.cavity_config(precision=64, n=(16, 16, 28), pml=6, max_source=600)
    cfg = cfg.replace(mass=20.0)                          # lighter, so the fields deflect it visibly
    beam = W.cavity_beam(cfg, n_macro=600, seed=77, sigma_z=4.0, sigma_r=0.6, x_offset=1.5, gamma=3.0)
    beam.w[:] *= 200.0
    cells = W.cavity_conductor(cfg, pipe_half=4.0, cavity=(9.0, 19.0))
    g, o = both(cfg, max_particles=cfg.max_source)
    g.set_conductor(cells)
    o.set_conductor(cells)
    g.set_source(beam.x, beam.u, beam.w, axis=2)
    o.set_source(beam.x, beam.u, beam.w, axis=2)
    edges = np.array([-6.0, 0.0, 9.0, 19.0, 28.0, 34.0])
    for N in (15, 30, 45):
        g.step(N - o.step_count)
        o.step(N - o.step_count)
        say("mini cavity step", N, g.num_particles)
        compare_fields(g, o, cfg, 1e-9, "step %d" % N)
        compare_particles(g, o, 1e-9, 1e-9, "step %d" % N)
        mg, mo = g.slab_moments(2, edges), o.slab_moments(2, edges)
        assert np.array_equal(mg[:, 0], mo[:, 0])
        assert np.allclose(mg[:, 1:], mo[:, 1:], rtol=1e-9, atol=1e-12)
    assert g.num_particles > 100


def test_all_pieces_with_ck_and_filter_fp64():
    """Cole-Karkkainen at c dt = dx, two filter passes, a conductor block, per-face damping
    and a source entering through the low z PML, together with random fields and particles:
    FP64 against the oracle."""
    ns = 200
    cfg = W.SimConfig(dim=3, n=(12, 10, 14), pml=((3, 4), (4, 3), (5, 5)), dx=(1.0, 1.0, 1.0), dt=1.0,
                      shape_order=2, alpha_mode=W.ALPHA_DAMPED, sigma_coef=W.paper_conductivity_profile(5),
                      push=1, charge=1.0, mass=4.0, precision=64, solver=1, filter_passes=2, conductor=1,
                      max_source=ns, alpha_face=((0, ZERO), (0, 0), (ONE, DAMPED)), sort_interval=3)
    parts = W.random_particles(cfg, 150, seed=901, margin=2.0, umax=1.5)
    fields = W.random_split_fields(cfg, seed=902, amp=0.2)
    rng = np.random.default_rng(903)
    x = np.stack([rng.uniform(2.0, 10.0, ns), rng.uniform(2.0, 8.0, ns), rng.uniform(-20.0, -5.2, ns)], axis=1)
    u = np.stack([rng.normal(0.0, 0.1, ns), rng.normal(0.0, 0.1, ns), rng.uniform(1.0, 4.0, ns)], axis=1)
    w = rng.uniform(0.5, 1.5, ns) * 0.05
    g, o = both(cfg, parts, fields, max_particles=len(parts) + ns, flags=B.FLAG_KEEP_CURRENT)
    cells = np.zeros((o.M[2], o.M[1], o.M[0]), np.uint8)
    cells[8:13, :, 10:] = 1
    for s in (g, o):
        s.set_conductor(cells)
        s.set_source(x, u, w, axis=2)
    for N in (2, 6, 15, 30):
        g.step(N - o.step_count)
        o.step(N - o.step_count)
        compare_fields(g, o, cfg, 1e-9, "step %d" % N)
        compare_current(g, o, 1e-9, "J step %d" % N)
        compare_particles(g, o, 1e-9, 1e-9, "step %d" % N)


def test_source_injection_fp32():
    """FP32 against the FP64 oracle with a source: relative L2 error 1e-5 per field
    component, measured against the norm of the largest component (B_z, driven by the
    small transverse currents of a beam moving along z, has a norm far below that of E,
    and rounding errors of the large components reach it in absolute terms)."""
    cfg64, (x, u, w) = _source_case(1, seed=960)
    cfg64 = cfg64.replace(dt=float(np.float32(0.5)))
    cfg32 = cfg64.replace(precision=32)
    g, _ = both(cfg32, max_particles=len(w))
    _, o = both(cfg64, max_particles=len(w))
    g.set_source(x, u, w, axis=2)
    o.set_source(x, u, w, axis=2)
    g.step(30)
    o.step(30)
    Fg, Fo = g.fields(), o.fields()
    big = max(np.linalg.norm(Fo[c]) for c in range(6))
    for c in range(6):
        e = np.linalg.norm(Fg[c] - Fo[c]) / big
        say("fp32 source component", c, e, np.linalg.norm(Fo[c]) / big)
        assert e <= 1e-5, (c, e)
    compare_particles(g, o, 1e-4, 1e-4, "fp32 source")


def test_source_capacity_is_checked_before_injecting():
    """Room for the source is checked when it is set; particles added afterwards can take that
    room, and the step that would inject past max_particles fails with E_CAPACITY instead of
    writing beyond the particle buffers."""
    cfg, (x, u, w) = _source_case(0, seed=980, ns=100)
    g, _ = both(cfg, max_particles=100)
    g.set_source(x, u, w, axis=2)
    extra = W.random_particles(cfg, 30, seed=981, margin=2.0, umax=0.1)
    g.add_particles(extra.x, extra.u, extra.w)
    with pytest.raises(B.PmlPicError) as e:
        g.step(60)
    assert e.value.code == -6
    with pytest.raises(B.PmlPicError):
        g.set_source(x, u, w, axis=2)          # 30 + 100 > 100
