"""Pins of the oracle's Cole-Karkkainen Faraday update and binomial current filter (the
numerics of the paper's single-particle runs, App. A), against closed forms: the Fourier
multiplier of each discrete operator on a plane wave, the filter's stencil, and the
stability of the CK scheme at a time step where 3D Yee is unstable."""
import numpy as np
import pytest

import oracle
from paper_2201_09084_amd import workloads as W


def _cfg(n=14, solver=1, dt=0.5, filter_passes=0, pml=0):
    return W.SimConfig(dim=3, n=(n, n, n), pml=((pml, pml),) * 3, dx=(1.0, 1.0, 1.0), dt=dt, shape_order=1,
                       alpha_mode=W.ALPHA_ONE, sigma_coef=W.cubic_profile(3.2), push=0, precision=64,
                       solver=solver, filter_passes=filter_passes)


def _positions(shape, comp):
    """grid coordinates (x, y, z) of the samples of component comp (0..2 E, 3..5 B)"""
    nz, ny, nx = shape
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    X = [i.astype(float), j.astype(float), k.astype(float)]
    a = comp % 3
    for d in range(3):
        half = (d == a) if comp < 3 else (d != a)
        if half:
            X[d] = X[d] + 0.5
    return X


def _ck_multiplier(kv, b):
    t1, t2 = (b + 1) % 3, (b + 2) % 3
    c1, c2 = np.cos(kv[t1]), np.cos(kv[t2])
    return 7.0 / 12.0 + (2.0 * c1 + 2.0 * c2) / 12.0 + 4.0 * c1 * c2 / 48.0


@pytest.mark.parametrize("solver", [0, 1])
def test_faraday_half_step_is_the_fourier_multiplier(solver):
    """E = E0 cos(k.x) (random k off the axes), B = 0: after one B advance by tau, B_a at
    interior samples is -tau (D*_b E_c - D*_c E_b), with D*_b = A_b(k) (-2 sin(k_b/2))
    sin(k.x); A_b = 1 for Yee, the CK transverse average 7/12 + (cos k_t1 + cos k_t2)/6 +
    cos k_t1 cos k_t2 / 12 otherwise."""
    cfg = _cfg(solver=solver)
    o = oracle.OracleSim(cfg)
    shape = tuple(o.split_fields().shape[1:])
    rng = np.random.default_rng(5 + solver)
    kv = rng.uniform(0.3, 2.6, 3) * rng.choice([-1.0, 1.0], 3)
    E0 = rng.uniform(0.5, 1.5, 3)
    F = np.zeros((12,) + shape)
    for c in range(3):
        X = _positions(shape, c)
        F[2 * c] = E0[c] * np.cos(kv[0] * X[0] + kv[1] * X[1] + kv[2] * X[2])
    o.set_split_fields(F)
    tau = 0.37
    o.advance_B(tau)
    B = o.fields()[3:]
    sl = (slice(2, -3),) * 3
    worst = 0.0
    for a in range(3):
        b, c = (a + 1) % 3, (a + 2) % 3
        X = _positions(shape, 3 + a)
        ph = np.sin(kv[0] * X[0] + kv[1] * X[1] + kv[2] * X[2])
        Ab = _ck_multiplier(kv, b) if solver else 1.0
        Ac = _ck_multiplier(kv, c) if solver else 1.0
        dbEc = Ab * (-2.0 * np.sin(kv[b] / 2.0)) * E0[c] * ph
        dcEb = Ac * (-2.0 * np.sin(kv[c] / 2.0)) * E0[b] * ph
        want = -tau * (dbEc - dcEb)
        err = np.max(np.abs(B[a][sl] - want[sl]))
        worst = max(worst, err)
        assert err <= 1e-13, (a, err)
    assert worst <= 1e-13


def test_ck_differs_from_yee_off_axis():
    """The same field after one B advance with the two solvers: identical for a wave along
    an axis (transverse averages of a uniform difference), different off the axes."""
    out = {}
    for kv in ((1.1, 0.0, 0.0), (1.1, 0.9, 0.4)):
        for solver in (0, 1):
            o = oracle.OracleSim(_cfg(solver=solver))
            shape = tuple(o.split_fields().shape[1:])
            F = np.zeros((12,) + shape)
            for c in (1, 2):
                X = _positions(shape, c)
                F[2 * c] = np.cos(kv[0] * X[0] + kv[1] * X[1] + kv[2] * X[2])
            o.set_split_fields(F)
            o.advance_B(0.5)
            out[(kv, solver)] = o.fields()[3:][(slice(None),) + (slice(2, -3),) * 3]
    on_axis = np.max(np.abs(out[((1.1, 0.0, 0.0), 0)] - out[((1.1, 0.0, 0.0), 1)]))
    off_axis = np.max(np.abs(out[((1.1, 0.9, 0.4), 0)] - out[((1.1, 0.9, 0.4), 1)]))
    assert on_axis <= 1e-14
    assert off_axis >= 1e-3


def test_ck_stable_where_yee_is_not():
    """c dt = 0.95 dx: beyond the 3D Yee limit 1/sqrt(3) but within the CK limit dx.  A
    random magnetic field and E = 0 in a PEC box (no charge, so E has no longitudinal
    part): the CK energy oscillates without growing between steps 600 and 1200, Yee's
    diverges."""
    ratios = {}
    for solver in (0, 1):
        cfg = _cfg(n=10, solver=solver, dt=0.95)
        o = oracle.OracleSim(cfg)
        F = W.random_split_fields(cfg, seed=9, amp=1.0)
        F[:6] = 0.0
        o.set_split_fields(F)
        e0 = np.sum(o.fields() ** 2)
        o.step(600)
        with np.errstate(over="ignore", invalid="ignore"):
            e1 = np.sum(o.fields() ** 2) / e0
            o.step(600)
            e2 = np.sum(o.fields() ** 2) / e0
        ratios[solver] = (e1, e2)
    e1, e2 = ratios[1]
    assert e1 < 10.0 and e2 < 10.0 and e2 < 1.2 * e1, ratios
    assert not np.isfinite(ratios[0][1]) or ratios[0][1] > 1e6, ratios


def test_filter_is_the_binomial_multiplier():
    """J = cos(k.x): one pass gives prod_d cos^2(k_d/2) J at interior samples."""
    cfg = _cfg(filter_passes=1)
    o = oracle.OracleSim(cfg)
    shape = tuple(o.split_fields().shape[1:])
    kv = np.array([0.7, -1.9, 2.3])
    J = np.zeros((3,) + shape)
    for a in range(3):
        X = _positions(shape, a)
        J[a] = (a + 1.0) * np.cos(kv[0] * X[0] + kv[1] * X[1] + kv[2] * X[2] + 0.3 * a)
    o.set_current(J)
    o.filter_current()
    got = o.current()
    m = np.prod(np.cos(kv / 2.0) ** 2)
    sl = (slice(2, -3),) * 3
    for a in range(3):
        assert np.max(np.abs(got[a][sl] - m * J[a][sl])) <= 1e-14


def test_filter_spreads_a_point_over_the_binomial_stencil():
    """A single interior sample: the 27 weights (1/4, 1/2, 1/4)^3 (sum 1); two passes give
    (1, 4, 6, 4, 1)/16 per axis."""
    for passes, w1 in ((1, [0.25, 0.5, 0.25]), (2, [1 / 16, 4 / 16, 6 / 16, 4 / 16, 1 / 16])):
        cfg = _cfg(filter_passes=passes)
        o = oracle.OracleSim(cfg)
        shape = tuple(o.split_fields().shape[1:])
        J = np.zeros((3,) + shape)
        J[1][6, 7, 5] = 2.0
        o.set_current(J)
        o.filter_current()
        got = o.current()[1]
        w1 = np.array(w1)
        h = len(w1) // 2
        want = np.zeros(shape)
        want[6 - h:6 + h + 1, 7 - h:7 + h + 1, 5 - h:5 + h + 1] = 2.0 * np.einsum("i,j,k->ijk", w1, w1, w1)
        assert np.max(np.abs(got - want)) <= 1e-15
        assert abs(got.sum() - 2.0) <= 1e-14


def test_step_filters_the_deposited_current():
    """A step with the filter on leaves J equal to the filtered J of the same step without
    it (alpha = 1, so the damping is the identity); the fields differ only through J."""
    base = _cfg(n=12, solver=1, dt=0.9, pml=3)
    x = np.array([[6.3, 5.7, 6.1], [2.2, 8.9, 4.4]])
    u = np.array([[0.8, -0.3, 0.5], [-0.2, 0.6, 0.9]])
    w = np.array([1.0, 0.7])
    runs = {}
    for fp in (0, 1):
        o = oracle.OracleSim(base.replace(filter_passes=fp))
        o.add_particles(x, u, w)
        o.step(1)
        runs[fp] = o
    ref = oracle.OracleSim(base.replace(filter_passes=1))
    ref.set_current(runs[0].current())
    ref.filter_current()
    J1 = runs[1].current()
    assert np.max(np.abs(J1 - ref.current())) <= 1e-15 * max(1.0, np.max(np.abs(J1)))
    assert np.max(np.abs(J1 - runs[0].current())) > 1e-6
