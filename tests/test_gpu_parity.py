"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the same
seeded inputs, element by element.

Tolerances: FP64 runs agree to round-off (relative max error 1e-10 after many steps;
the only differences are summation order of the atomics and of the split parts).
FP32 runs are held to the relative L2 error 1e-5 per field component stated for the
FP32 production path (on workload 1 the larger of that and a multiple of the problem's own
one-ulp sensitivity, see ENVELOPE_K); components that vanish in the oracle must stay below
1e-12.
"""
import numpy as np
import pytest

import oracle

from gpu_helpers import both, compare_current, compare_fields, compare_particles, rel_err, rel_l2, say
from paper_2201_09084_amd import binding as B
from paper_2201_09084_amd import workloads as W

pytestmark = pytest.mark.gpu

# FP32 on workload 1 (one electron, q/m = -1, 400 steps) against the FP64 oracle.  The
# problem itself is ill-conditioned: a one-ulp (FP32) change of the initial momentum moves
# the FP64 oracle's fields by up to 1e-4 (relative L2) by step 200 when the particle is
# pushed (it is decelerated and turned back by its partner's field), and by 7e-6 in the
# decayed B_z of the ballistic run at step 400.  The FP32 run integrates velocities u/gamma
# that carry a few FP32 roundings (square root, division, products: within ~2 ulp) in every
# step, so its error is held to the larger of the stated 1e-5 and ENVELOPE_K times that
# one-ulp envelope, computed here from the oracle itself (u_x +- 1 ulp).  ENVELOPE_K = 4:
# the per-step roundings are of either sign and add up like a random walk over the steps
# during which the sensitivity grows (about 3.7 times one perturbation for the pushed run).
ENVELOPE_K = 4.0
FP32_TOL = 1e-5
CHECKPOINTS = (100, 200, 300, 400)


def _fields_at(cfg, p, u, steps):
    o = oracle.OracleSim(cfg)
    o.add_particles(p.x, u, p.w)
    out, done = {}, 0
    for s in steps:
        o.step(s - done)
        done = s
        out[s] = o.fields()
    return out


def _one_ulp_envelope(cfg64, p, base):
    """Per checkpoint and component, the largest relative L2 change of the oracle's fields when
    u_x of the initial momentum moves by one FP32 ulp either way."""
    ulp = 2.0 ** (np.floor(np.log2(abs(p.u[0, 0]))) - 23)
    env = {s: np.zeros(6) for s in CHECKPOINTS}
    for sign in (1.0, -1.0):
        u = p.u.copy()
        u[0, 0] += sign * ulp
        pert = _fields_at(cfg64, p, u, CHECKPOINTS)
        for s in CHECKPOINTS:
            for c in range(6):
                nb = np.linalg.norm(base[s][c])
                if nb > 0:
                    env[s][c] = max(env[s][c], np.linalg.norm(pert[s][c] - base[s][c]) / nb)
    return env


def _fp32_within_envelope(push):
    dt = float(np.float32(0.7))
    cfg64 = W.single_particle_config(precision=64, push=push).replace(dt=dt)
    cfg32 = cfg64.replace(precision=32)
    p = W.single_particle(cfg64)
    p = W.Particles(x=p.x, u=p.u.astype(np.float32).astype(np.float64), w=p.w)   # FP32-exact inputs
    g, _ = both(cfg32, p)
    base = _fields_at(cfg64, p, p.u, CHECKPOINTS)
    env = _one_ulp_envelope(cfg64, p, base)
    worst_ratio = 0.0
    done = 0
    for s in CHECKPOINTS:
        g.step(s - done)
        done = s
        Fg = g.fields()
        for c in range(6):
            nb = np.linalg.norm(base[s][c])
            if nb == 0.0:
                assert np.max(np.abs(Fg[c])) <= 1e-12, (s, c)
                continue
            err = np.linalg.norm(Fg[c] - base[s][c]) / nb
            bound = max(FP32_TOL, ENVELOPE_K * env[s][c])
            say("push %d step %d comp %d: fp32 rel L2 %.3e, one-ulp envelope %.3e, ratio %.2f"
                % (push, s, c, err, env[s][c], err / env[s][c] if env[s][c] > 0 else 0.0))
            worst_ratio = max(worst_ratio, err / bound)
            assert err <= bound, (push, s, c, err, env[s][c])
    return g, worst_ratio


def test_single_particle_fp64_400_steps():
    """Workload 1: 2D 128^2 + 10-cell cubic PML, one electron at 0.9c, FP64, 400 steps."""
    cfg = W.single_particle_config(precision=64, push=1)
    p = W.single_particle(cfg)
    g, o = both(cfg, p)
    for k in range(4):
        g.step(100)
        o.step(100)
        say("step", (k + 1) * 100)
        compare_fields(g, o, cfg, 1e-10, "fields @%d" % ((k + 1) * 100))
        compare_particles(g, o, 1e-10, 1e-10, "particles")
    d = g.diagnose()
    do = o.diagnose()
    assert d["gauss_max"] < 1e-12
    assert abs(d["u_interior"] - do["u_interior"]) <= 1e-10 * do["u_interior"]
    assert abs(d["u_pml"] - do["u_pml"]) <= 1e-9 * max(do["u_pml"], 1e-30) + 1e-20
    assert d["n_pushes"] == 400


@pytest.mark.parametrize("mode", [W.ALPHA_ZERO, W.ALPHA_ONE, W.ALPHA_DAMPED, W.ALPHA_WEIGHT])
def test_single_particle_exit_all_modes_fp64(mode):
    """The particle leaves through the +x PEC (ballistic): removal and all four
    damping schemes (three alpha schemes and the per-particle weight damping)."""
    cfg = W.single_particle_config(precision=64, push=0, alpha_mode=mode)
    p = W.single_particle(cfg)
    g, o = both(cfg, p)
    g.step(200)
    o.step(200)
    compare_fields(g, o, cfg, 1e-10, "mode %d" % mode)
    assert g.num_particles == 0 and o.num_particles == 0


def test_single_particle_fp32_ballistic_400_steps():
    """Workload 1 in FP32 against the FP64 oracle, ballistic particle, all 400 steps: relative
    L2 per field component within 1e-5, or within ENVELOPE_K times the oracle's own one-ulp
    envelope where the problem's conditioning exceeds that (the decayed B_z once the particle
    has left).  c dt and u are FP32 values in both runs, so the difference is FP32 arithmetic."""
    g, worst = _fp32_within_envelope(push=0)
    say("fp32 ballistic: worst error / bound %.3f" % worst)
    assert g.diagnose()["gauss_max"] < 1e-5


def test_single_particle_fp32_pushed_400_steps():
    """The same with the self-consistent push over all 400 steps: the electron is stopped and
    turned back by its partner's field, and FP32 rounding shifts the turning point within the
    envelope that a one-ulp change of the initial momentum produces in the FP64 oracle."""
    g, worst = _fp32_within_envelope(push=1)
    say("fp32 pushed: worst error / bound %.3f" % worst)


CASES = [(dim, order) for dim in (2, 3) for order in (1, 2, 3)]


def _random_case(dim, order, seed, n_particles, alpha_mode=W.ALPHA_DAMPED, push=1, precision=64):
    if dim == 2:
        cfg = W.SimConfig(dim=2, n=(37, 29, 1), pml=((6, 9), (7, 5), (0, 0)), dx=(1.0, 0.9, 1.0), dt=0.6,
                          shape_order=order, alpha_mode=alpha_mode, damping_scale=1.3,
                          sigma_coef=((0.0, 0.5, 0.0, 2.5), (0.2, 0.0, 3.0), (0.0,)), push=push,
                          precision=precision, tile=(8, 8, 1), sort_interval=3)
    else:
        cfg = W.SimConfig(dim=3, n=(13, 11, 9), pml=((4, 5), (3, 4), (5, 3)), dx=(1.0, 0.9, 1.1), dt=0.45,
                          shape_order=order, alpha_mode=alpha_mode, damping_scale=1.1,
                          sigma_coef=((0.0, 0.0, 0.0, 3.0), (0.1, 0.0, 2.0), (0.0, 1.0, 1.0)), push=push,
                          precision=precision, tile=(4, 4, 4), sort_interval=2)
    parts = W.random_particles(cfg, n_particles, seed=seed, margin=1.5, umax=2.5)
    fields = W.random_split_fields(cfg, seed=seed + 1, amp=0.3)
    return cfg, parts, fields


@pytest.mark.parametrize("dim,order", CASES)
def test_random_state_steps_fp64(dim, order):
    """Random fields in every split part (PML faces, edges, corners) and random
    particles over box and PML; several steps, fields, current and particles."""
    cfg, parts, fields = _random_case(dim, order, seed=100 + 10 * dim + order, n_particles=300)
    say("case", dim, order)
    g, o = both(cfg, parts, fields, flags=B.FLAG_KEEP_CURRENT)
    for k in range(3):
        g.step(1)
        o.step(1)
        compare_fields(g, o, cfg, 1e-10, "step %d" % (k + 1))
        compare_current(g, o, 1e-10, "J")
        compare_particles(g, o, 1e-10, 1e-10, "step %d" % (k + 1))
    g.step(4)
    o.step(4)
    compare_fields(g, o, cfg, 1e-9, "after 7 steps")
    compare_particles(g, o, 1e-9, 1e-9, "after 7 steps")


@pytest.mark.parametrize("flags", [B.FLAG_UNFUSED, B.FLAG_NO_SORT, B.FLAG_SEPARATE_DAMP, B.FLAG_KEEP_CURRENT,
                                   B.FLAG_UNFUSED | B.FLAG_SEPARATE_DAMP | B.FLAG_NO_SORT | B.FLAG_KEEP_CURRENT])
@pytest.mark.parametrize("dim", [2, 3])
def test_kernel_variants_match_oracle(flags, dim):
    """Unfused gather_push + deposit_current, no sorting, separate damp pass."""
    cfg, parts, fields = _random_case(dim, 2, seed=7 + dim, n_particles=200)
    g, o = both(cfg, parts, fields, flags=flags)
    g.step(3)
    o.step(3)
    compare_fields(g, o, cfg, 1e-10, "flags %d" % flags)
    compare_particles(g, o, 1e-10, 1e-10, "flags %d" % flags)


@pytest.mark.parametrize("mode", [W.ALPHA_ZERO, W.ALPHA_ONE, W.ALPHA_WEIGHT])
@pytest.mark.parametrize("dim", [2, 3])
def test_alpha_modes_random_state(mode, dim):
    cfg, parts, fields = _random_case(dim, 1, seed=30 + mode, n_particles=150, alpha_mode=mode)
    for flags in (0, B.FLAG_SEPARATE_DAMP):
        g, o = both(cfg, parts, fields, flags=flags)
        g.step(2)
        o.step(2)
        compare_fields(g, o, cfg, 1e-10, "mode %d flags %d" % (mode, flags))


@pytest.mark.parametrize("dim,order", [(2, 2), (3, 1)])
def test_random_state_fp32(dim, order):
    cfg64, parts, fields = _random_case(dim, order, seed=55 + dim, n_particles=300)
    cfg32 = cfg64.replace(precision=32)
    g, _ = both(cfg32, parts, fields)
    _, o = both(cfg64, parts, fields)
    g.step(5)
    o.step(5)
    compare_fields(g, o, cfg64, 1e-5, "fp32", l2=True)
    compare_particles(g, o, 1e-4, 1e-4, "fp32")


def test_ballistic_and_no_particles():
    cfg, parts, fields = _random_case(2, 3, seed=3, n_particles=100, push=0)
    g, o = both(cfg, parts, fields)
    g.step(4)
    o.step(4)
    compare_fields(g, o, cfg, 1e-10, "ballistic")
    compare_particles(g, o, 1e-10, 0.0, "ballistic")
    g2, o2 = both(cfg, None, fields)
    g2.step(5)
    o2.step(5)
    compare_fields(g2, o2, cfg, 1e-10, "no particles")
    assert g2.diagnose()["n_particles"] == 0


def test_particles_leaving_are_removed_and_counted():
    cfg = W.SimConfig(dim=2, n=(20, 20, 1), pml=((4, 4), (4, 4), (0, 0)), dt=0.6, shape_order=2,
                      push=0, precision=64)
    x = np.array([[23.8, 10.0], [-3.9, 5.0], [10.0, 23.95], [10.0, 10.0]])
    u = np.array([[5.0, 0, 0], [-5.0, 0, 0], [0, 5.0, 0], [0.1, 0.2, 0.0]])
    parts = W.Particles(x=x, u=u, w=np.ones(4))
    g, o = both(cfg, parts)
    g.step(1)
    o.step(1)
    assert o.num_particles == 1 and g.num_particles == 1
    compare_fields(g, o, cfg, 1e-10, "leaving")
    d = g.diagnose()
    assert d["n_pushes"] == 4


def test_add_particles_after_steps_and_capacity():
    cfg, parts, fields = _random_case(2, 1, seed=9, n_particles=50)
    g, o = both(cfg, parts, fields, max_particles=80)
    g.step(3)
    o.step(3)
    more = W.random_particles(cfg, 30, seed=10, margin=2.0)
    g.add_particles(more.x, more.u, more.w)
    o.add_particles(more.x, more.u, more.w)
    g.step(3)
    o.step(3)
    compare_fields(g, o, cfg, 1e-10, "added")
    compare_particles(g, o, 1e-10, 1e-10, "added")
    np.testing.assert_allclose(g.rho_static(), o.rho_static(), rtol=0, atol=1e-12)
    extra = W.random_particles(cfg, 10, seed=11, margin=2.0)
    with pytest.raises(B.PmlPicError) as e:
        g.add_particles(extra.x, extra.u, extra.w)
    assert e.value.code == -6


def test_diagnostics_match_oracle():
    cfg, parts, fields = _random_case(3, 2, seed=21, n_particles=120)
    g, o = both(cfg, parts, fields)
    g.step(2)
    o.step(2)
    dg, do = g.diagnose(), o.diagnose()
    for k in ("u_interior", "u_pml", "gauss_max", "rho_max"):
        assert abs(dg[k] - do[k]) <= 1e-10 * max(abs(do[k]), 1e-30), (k, dg[k], do[k])
    assert abs(dg["gauss_l2"] - do["gauss_l2"]) <= 1e-9 * do["gauss_l2"]
    assert dg["n_particles"] == do["n_particles"]


def test_nonfinite_is_reported():
    cfg = W.single_particle_config(precision=32, n=32, pml=4)
    g = B.PmlPic(cfg, max_particles=1)
    F = np.zeros((12,) + tuple(reversed(cfg.nodes())))
    F[0, 0, 10, 10] = np.nan
    g.set_split_fields(F)
    with pytest.raises(B.PmlPicError) as e:
        g.diagnose()
    assert e.value.code == -5


@pytest.mark.parametrize("dim,order", [(2, 1), (2, 2), (2, 3), (3, 1), (3, 2)])
@pytest.mark.parametrize("precision", [64, 32])
def test_dense_clusters_lds_path(dim, order, precision):
    """Dense clusters (hundreds of particles per cell, as in the beams) whose chunks
    fit the LDS box, plus sparse particles that take the global-atomic fallback."""
    cfg64, _, fields = _random_case(dim, order, seed=70 + dim * 3 + order, n_particles=10)
    rng = np.random.default_rng(80 + dim + order)
    n_dense = 3000
    centre = np.array([(cfg64.n[d] * 0.5) * cfg64.dx[d] for d in range(dim)])
    x = centre + rng.normal(0.0, 1.2, (n_dense, dim)) * np.array(cfg64.dx[:dim])
    u = rng.normal(0.0, 0.8, (n_dense, 3))
    sparse = W.random_particles(cfg64, 400, seed=90 + dim, margin=1.5, umax=2.0)
    parts = W.Particles(x=np.concatenate([x, sparse.x]), u=np.concatenate([u, sparse.u]),
                        w=np.concatenate([rng.uniform(0.5, 1.5, n_dense), sparse.w]))
    cfg = cfg64.replace(precision=precision)
    g, _ = both(cfg, parts, fields)
    _, o = both(cfg64, parts, fields)
    g.step(6)
    o.step(6)
    if precision == 64:
        compare_fields(g, o, cfg64, 1e-10, "dense fp64")
        compare_particles(g, o, 1e-10, 1e-10, "dense fp64")
    else:
        compare_fields(g, o, cfg64, 1e-5, "dense fp32", l2=True)
        compare_particles(g, o, 1e-4, 1e-4, "dense fp32")


@pytest.mark.parametrize("dim", [2, 3])
def test_chunks_drifting_far_from_their_sort_tile(dim):
    """Fast particles in random directions and a long sort interval: a chunk's cells
    spread beyond what its LDS box can hold, so the box is clipped to the tile and the
    particles outside it deposit to global memory."""
    if dim == 2:
        cfg = W.SimConfig(dim=2, n=(96, 80, 1), pml=((8, 8), (8, 8), (0, 0)), dt=0.7, shape_order=2,
                          alpha_mode=W.ALPHA_DAMPED, sigma_coef=W.cubic_profile(3.2), push=1, precision=64,
                          tile=(16, 16, 1), sort_interval=40)
        steps = 26
    else:
        cfg = W.SimConfig(dim=3, n=(30, 28, 26), pml=((4, 4), (4, 4), (4, 4)), dt=0.5, shape_order=1,
                          alpha_mode=W.ALPHA_DAMPED, sigma_coef=W.cubic_profile(3.2), push=1, precision=64,
                          tile=(8, 8, 8), sort_interval=40)
        steps = 14
    rng = np.random.default_rng(300 + dim)
    n = 4000
    x = rng.uniform(0.2, 0.8, (n, dim)) * np.array([cfg.n[d] * cfg.dx[d] for d in range(dim)])
    u = rng.normal(0.0, 1.0, (n, 3))
    u *= (4.0 / np.linalg.norm(u, axis=1))[:, None]
    parts = W.Particles(x=x, u=u, w=rng.uniform(0.5, 1.5, n))
    g, o = both(cfg, parts)
    g.step(steps)
    o.step(steps)
    compare_fields(g, o, cfg, 1e-9, "drifting chunks")
    compare_particles(g, o, 1e-9, 1e-9, "drifting chunks")


@pytest.mark.parametrize("precision", [64, 32])
def test_removed_particles_stay_removed_in_3d_tile_push(precision):
    """Particles that reach the PEC walls are removed at once and stay in the arrays until
    the next sort (the sort interval here is longer than the run), so the 3D tile push meets
    them at every later step: they must deposit nothing, stay removed and not count as pushes.
    Half the particles start within 1.5 cells of a wall moving outwards (most leave in the
    first steps), the rest anywhere.  Every 2 steps: the push tally equals the live particles
    the steps began with, and fields and live particles (ids, positions, momenta) match the
    FP64 oracle."""
    cfg64 = W.SimConfig(dim=3, n=(20, 18, 22), pml=((4, 4), (4, 4), (4, 4)), dt=0.5, shape_order=1,
                        alpha_mode=W.ALPHA_DAMPED, sigma_coef=W.cubic_profile(3.2), push=1, precision=64,
                        tile=(8, 8, 8), sort_interval=100)
    rng = np.random.default_rng(4242)
    lo = np.array([-cfg64.pml[d][0] * cfg64.dx[d] for d in range(3)])
    hi = np.array([(cfg64.n[d] + cfg64.pml[d][1]) * cfg64.dx[d] for d in range(3)])
    n_wall = 1500
    axis = rng.integers(0, 3, n_wall)
    side = rng.integers(0, 2, n_wall)
    x = lo + (hi - lo) * rng.uniform(0.1, 0.9, (n_wall, 3))
    depth = rng.uniform(0.2, 1.5, n_wall)
    u = rng.normal(0.0, 0.5, (n_wall, 3))
    for k in range(n_wall):
        a = axis[k]
        x[k, a] = lo[a] + depth[k] if side[k] == 0 else hi[a] - depth[k]
        u[k, a] = (-1.0 if side[k] == 0 else 1.0) * rng.uniform(1.5, 4.0)
    rest = W.random_particles(cfg64, 1500, seed=4243, margin=1.0, umax=2.0)
    parts = W.Particles(x=np.concatenate([x, rest.x]), u=np.concatenate([u, rest.u]),
                        w=np.concatenate([rng.uniform(0.5, 1.5, n_wall), rest.w]))
    cfg = cfg64.replace(precision=precision)
    g, _ = both(cfg, parts)
    _, o = both(cfg64, parts)
    pushes = 0
    for _ in range(4):
        for _ in range(2):
            pushes += len(g.particles()[0])   # the live particles the step pushes
            g.step(1)
            o.step(1)
        assert g.diagnose()["n_pushes"] == pushes
        if precision == 64:
            compare_fields(g, o, cfg64, 1e-10, "removed particles fp64")
            compare_particles(g, o, 1e-10, 1e-10, "removed particles fp64")
        else:
            # FP32 could decide a wall crossing differently for a particle that ends a step
            # within rounding of the wall: the live sets may differ by such a particle
            compare_fields(g, o, cfg64, 1e-5, "removed particles fp32", l2=True)
            assert len(set(g.particles()[0]) ^ set(o.particles()[0])) <= 2
    live = len(o.particles()[0])
    say("removed particles: live", live, "of", len(parts.w), "pushes", pushes)
    assert live < len(parts.w) - n_wall // 2   # most of the wall particles left


@pytest.mark.parametrize("precision", [64, 32])
@pytest.mark.parametrize("order", [1, 3])
def test_one_pass_3d_field_update_equals_three_sweeps(precision, order):
    """The one-pass 3D update_yee_pml (strips of 61 columns, 14 rows, chunks of planes, halo
    lanes, rows and planes recomputed, y neighbours through LDS) gives the same bits as the
    B / E / B sweeps, on a ragged grid with uneven layers on every face (split parts in faces,
    edges and corners) and enough planes for several chunks.  A few particles far apart, so
    that the current has no order-dependent sums."""
    cfg = W.SimConfig(dim=3, n=(70, 23, 41), pml=((5, 7), (4, 6), (6, 5)), dx=(1.0, 0.9, 1.1), dt=0.45,
                      shape_order=order, alpha_mode=W.ALPHA_DAMPED, damping_scale=1.2,
                      sigma_coef=((0.1, 0.0, 0.5, 2.5), (0.0, 0.3, 2.0), (0.2, 0.0, 0.0, 3.0)), push=1,
                      precision=precision)
    fields = W.random_split_fields(cfg, seed=500 + order, amp=0.3)
    x = np.array([[3.3, 5.1, 2.2], [35.7, 12.2, 20.5], [66.4, 20.9, 38.1], [70.5, 2.5, 40.6]])
    u = np.array([[0.5, -0.3, 0.2], [-0.8, 0.4, 0.0], [0.3, 0.9, -0.1], [1.5, 0.2, 0.3]])
    parts = W.Particles(x=x, u=u, w=np.array([1.0, 0.7, 1.3, 0.9]))
    runs = []
    for flags in (0, B.FLAG_SEPARATE_FIELDS):
        g = B.PmlPic(cfg, max_particles=4, flags=flags)
        g.set_split_fields(fields)
        g.add_particles(parts.x, parts.u, parts.w)
        g.step(6)
        runs.append(g.split_fields())
    diff = np.max(np.abs(runs[0] - runs[1]))
    say("3D one pass vs three sweeps, max |diff|", diff)
    assert np.array_equal(runs[0], runs[1])


@pytest.mark.parametrize("precision", [64, 32])
@pytest.mark.parametrize("order", [1, 3])
def test_one_pass_field_update_equals_three_sweeps(precision, order):
    """The one-pass 2D update_yee_pml (strips of 61 columns, segments of rows, halo
    lanes and rows recomputed) gives the same bits as the B / E / B sweeps.  A few
    particles far apart, so that the current has no order-dependent sums."""
    cfg = W.SimConfig(dim=2, n=(150, 47, 1), pml=((9, 7), (6, 10), (0, 0)), dx=(1.0, 0.8, 1.0), dt=0.55,
                      shape_order=order, alpha_mode=W.ALPHA_DAMPED, damping_scale=1.2,
                      sigma_coef=((0.1, 0.0, 0.5, 2.5), (0.0, 0.3, 2.0), (0.0,)), push=1, precision=precision)
    fields = W.random_split_fields(cfg, seed=400 + order, amp=0.3)
    x = np.array([[3.3, 5.1], [60.7, 20.2], [120.4, 40.9], [150.5, 2.5]])
    u = np.array([[0.5, -0.3, 0.2], [-0.8, 0.4, 0.0], [0.3, 0.9, -0.1], [1.5, 0.2, 0.0]])
    parts = W.Particles(x=x, u=u, w=np.array([1.0, 0.7, 1.3, 0.9]))
    runs = []
    for flags in (0, B.FLAG_SEPARATE_FIELDS | B.FLAG_KEEP_CURRENT):
        g = B.PmlPic(cfg, max_particles=4, flags=flags)
        g.set_split_fields(fields)
        g.add_particles(parts.x, parts.u, parts.w)
        g.step(6)
        runs.append((g.split_fields(), g.current()))
    assert np.array_equal(runs[0][1], runs[1][1])
    diff = np.max(np.abs(runs[0][0] - runs[1][0]))
    say("one pass vs three sweeps, max |diff|", diff)
    assert np.array_equal(runs[0][0], runs[1][0])


@pytest.mark.parametrize("precision", [64, 32])
@pytest.mark.parametrize("flags", [0, B.FLAG_UNFUSED, B.FLAG_NO_SORT])
@pytest.mark.parametrize("dim", [2, 3])
def test_weight_damping_matches_oracle(dim, flags, precision):
    """Per-particle weight damping (alpha mode 3): many particles crossing faces,
    edges and corners of the layers over several steps, in every kernel form.  The
    current depends on each particle's accumulated damping integral."""
    cfg64, parts, fields = _random_case(dim, 2 if dim == 2 else 1, seed=500 + dim, n_particles=400,
                                        alpha_mode=W.ALPHA_WEIGHT)
    cfg = cfg64.replace(precision=precision)
    g, _ = both(cfg, parts, fields, flags=flags | B.FLAG_KEEP_CURRENT)
    _, o = both(cfg64, parts, fields)
    for k in range(3):
        g.step(3)
        o.step(3)
        if precision == 64:
            compare_fields(g, o, cfg64, 1e-10, "step %d" % (3 * k + 3))
            compare_current(g, o, 1e-10, "J")
            compare_particles(g, o, 1e-10, 1e-10, "step %d" % (3 * k + 3))
        else:
            compare_fields(g, o, cfg64, 2e-5, "fp32 step %d" % (3 * k + 3), l2=True)
    dg, do = g.diagnose(), o.diagnose()
    tol = 1e-10 if precision == 64 else 1e-4
    assert abs(dg["rho_max"] - do["rho_max"]) <= tol * do["rho_max"]


def test_dense_and_sparse_ranges_2d():
    """A dense cluster (ranges of 1024 sorted particles whose node box fits in LDS) next
    to a sparse population (ranges whose box does not: split into eight pieces that
    deposit to global memory, listed last), over several sort intervals."""
    cfg = W.SimConfig(dim=2, n=(120, 100, 1), pml=((10, 10), (10, 10), (0, 0)), dt=0.7, shape_order=2,
                      alpha_mode=W.ALPHA_DAMPED, sigma_coef=W.cubic_profile(3.2), push=1, precision=64,
                      tile=(16, 16, 1), sort_interval=4)
    rng = np.random.default_rng(77)
    n_dense, n_sparse = 5000, 3000
    xd = np.array([60.0, 50.0]) + rng.normal(0.0, 1.5, (n_dense, 2))
    xs = rng.uniform([-8.0, -8.0], [128.0, 108.0], (n_sparse, 2))
    x = np.vstack([xd, xs])
    u = rng.normal(0.0, 0.8, (n_dense + n_sparse, 3))
    parts = W.Particles(x=x, u=u, w=rng.uniform(0.5, 1.5, n_dense + n_sparse))
    g, o = both(cfg, parts, flags=B.FLAG_KEEP_CURRENT)
    for k in range(3):
        g.step(5)
        o.step(5)
        compare_fields(g, o, cfg, 1e-10, "step %d" % (5 * k + 5))
        compare_current(g, o, 1e-10, "step %d" % (5 * k + 5))
        compare_particles(g, o, 1e-10, 1e-10, "step %d" % (5 * k + 5))


@pytest.mark.parametrize("dim,order,precision", [(2, 2, 64), (3, 1, 64), (3, 1, 32)])
def test_restart_from_exported_state(dim, order, precision):
    """Checkpoint and resume through the state calls: 9 steps in one run equal 4 steps, an
    export of the fields (every split part), the particles (ids, positions, momenta, weights)
    and the partner density, an import into a new run and 5 more steps.  The runs differ only
    in the order of their atomic adds (the new run sorts at its first step), so FP64 agrees to
    relative 1e-12 and FP32 to its rounding (relative L2 1e-6 per component)."""
    cfg, parts, fields = _random_case(dim, order, seed=900 + dim, n_particles=400, precision=precision)
    def fresh():
        g = B.PmlPic(cfg, max_particles=len(parts.w))
        g.set_split_fields(fields)
        g.add_particles(parts.x, parts.u, parts.w)
        return g
    a, b = fresh(), fresh()
    a.step(9)
    b.step(4)
    F, (ids, X, u, w), rho = b.split_fields(), b.particles(), b.rho_static()
    c = B.PmlPic(cfg, max_particles=len(parts.w))
    c.set_split_fields(F)
    c.set_particles(ids, X, u, w)
    c.set_rho_static(rho)
    c.step(5)
    Fa, Fc = a.fields(), c.fields()
    if precision == 64:
        worst = max(rel_err(Fc[k], Fa[k]) for k in range(6) if np.max(np.abs(Fa[k])) > 0)
        assert worst <= 1e-12, worst
    else:
        worst = max(rel_l2(Fc[k], Fa[k]) for k in range(6) if np.max(np.abs(Fa[k])) > 0)
        assert worst <= 1e-6, worst
    ia, Xa, ua, _ = a.particles()
    ic, Xc, uc, _ = c.particles()
    assert np.array_equal(ia, ic)
    tol = 1e-10 if precision == 64 else 1e-4
    assert np.max(np.abs(Xa - Xc)) <= tol and np.max(np.abs(ua - uc)) <= tol
    da, dc = a.diagnose(), c.diagnose()
    assert da["n_particles"] == dc["n_particles"]
    assert abs(da["u_interior"] - dc["u_interior"]) <= (1e-12 if precision == 64 else 1e-5) * abs(da["u_interior"])
    say("restart", dim, precision, "worst field difference", worst)


def test_particle_ids_out_of_range_are_rejected():
    """Ids index per-particle arrays (the pushed adjoint's): set_particles rejects a negative id
    and one beyond 32 bits, and leaves the run as it was."""
    cfg, parts, fields = _random_case(2, 1, seed=31, n_particles=4)
    g = B.PmlPic(cfg, max_particles=8)
    g.add_particles(parts.x, parts.u, parts.w)
    ids, X, u, w = g.particles()
    for bad in (-1, 2 ** 31):
        with pytest.raises(B.PmlPicError):
            g.set_particles(np.array([bad, 1, 2, 3]), X, u, w)
    assert np.array_equal(g.particles()[0], ids)
    g.set_particles(np.array([7, 1, 2, 3]), X, u, w)
    assert sorted(g.particles()[0].tolist()) == [1, 2, 3, 7]
