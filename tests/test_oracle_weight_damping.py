"""Per-particle weight damping (alpha mode 3; Sec. II.C, discussion and limitations):
alpha = 1 in the field equations and each macroparticle's weight multiplied by
exp(-int sigma/eps0 dt) along its path.  Pins of the oracle against closed forms."""
import math

import numpy as np
import pytest

import oracle
from paper_2201_09084_amd import workloads as W

COEF = (0.2, 0.5, 0.0, 3.0)


def _phi(delta, L, coef=COEF):
    """int_0^delta sum_k a_k (z/L)^k dz, by numpy's polynomial antiderivative"""
    if delta <= 0.0:
        return 0.0
    p = np.polynomial.Polynomial(coef)
    return float(L * p.integ()(delta / L))


def _cfg(pml=((10, 12), (8, 14), (0, 0)), push=0):
    return W.SimConfig(dim=2, n=(40, 36, 1), pml=pml, dt=0.6, shape_order=2, alpha_mode=W.ALPHA_WEIGHT,
                       damping_scale=1.0, sigma_coef=(COEF, COEF, (0.0,)), push=push)


def _one(cfg, x, beta, theta_deg):
    g = 1.0 / math.sqrt(1.0 - beta * beta)
    th = math.radians(theta_deg)
    u = np.array([[g * beta * math.cos(th), g * beta * math.sin(th), 0.0]])
    o = oracle.OracleSim(cfg)
    o.add_particles(np.array([x]), u, np.array([1.0]))
    return o, beta * math.cos(th), beta * math.sin(th)


def _depths(cfg, X):
    """signed depths into the low and high layers of x and y (grid coordinates X)"""
    out = []
    for d in range(2):
        lo, hi = cfg.pml[d][0], cfg.pml[d][0] + cfg.n[d]
        out.append(((lo - X[d]) * cfg.dx[d], cfg.pml[d][0] * cfg.dx[d],
                    (X[d] - hi) * cfg.dx[d], cfg.pml[d][1] * cfg.dx[d]))
    return out


@pytest.mark.parametrize("theta,x0", [(0.0, (37.5, 18.0)), (180.0, (2.5, 18.0)), (35.0, (36.0, 33.0)),
                                      (-120.0, (3.0, 4.0))])
def test_lambda_is_phi_over_velocity(theta, x0):
    """A ballistic particle entering a layer at constant velocity: the integral of
    sigma over time telescopes to Phi(depth) / v_normal per axis (corners: the sum)."""
    cfg = _cfg()
    o, vx, vy = _one(cfg, x0, 0.8, theta)
    v = (vx, vy)
    checked = 0
    for _ in range(40):
        o.step(1)
        if o.num_particles == 0:
            break
        X = o.particles()[1][0]
        expect = 0.0
        for d, (dlo, Llo, dhi, Lhi) in enumerate(_depths(cfg, X)):
            if abs(v[d]) > 1e-12:
                expect += (_phi(dlo, Llo) + _phi(dhi, Lhi)) / abs(v[d])
        lam = o.lam()[0]
        assert abs(lam - expect) <= 1e-12 * max(1.0, expect), (lam, expect)
        checked += expect > 0.0
    assert checked >= 5


def test_deposit_uses_the_weight_at_mid_step():
    """Esirkepov's total current of a move is q w v; in mode 3 the weight is
    w exp(-Lambda(t^{n+1/2}))."""
    cfg = _cfg(pml=((10, 10), (10, 10), (0, 0)))
    beta = 0.7
    o, vx, _ = _one(cfg, (38.0, 18.0), beta, 0.0)
    o.step(6)                                   # now a few cells into the +x layer
    lam0 = o.lam()[0]
    X0 = o.particles()[1][0]
    o.step(1)
    J = o.current()
    hi = cfg.pml[0][0] + cfg.n[0]
    d0 = (X0[0] - hi) * cfg.dx[0]
    dh = d0 + vx * cfg.dt / 2.0
    lam_h = lam0 + (_phi(dh, 10.0) - _phi(d0, 10.0)) / vx
    total = J[0].sum() * cfg.dx[0] * cfg.dx[1]
    expect = cfg.charge * math.exp(-lam_h) * vx
    assert d0 > 0.0 and lam0 > 0.0
    assert abs(total - expect) <= 1e-12 * abs(expect), (total, expect)


def test_fields_see_no_alpha():
    cfg = _cfg()
    o = oracle.OracleSim(cfg)
    for X in ((1.0, 20.0), (55.0, 3.0), (30.0, 30.0)):
        assert o.alpha(X) == 1.0


def test_path_integral_crossing_the_interface():
    """A move that starts inside the box and ends in the layer integrates sigma only
    over the part of the path in the layer."""
    cfg = _cfg(pml=((10, 10), (10, 10), (0, 0)))
    o = oracle.OracleSim(cfg)
    hi = 50.0
    X0, X1, tau = (hi - 0.3, 20.0), (hi + 0.5, 20.0), 0.8
    v = (X1[0] - X0[0]) / tau
    expect = _phi(0.5, 10.0) / v
    assert abs(o.path_sigma(X0, X1, tau) - expect) <= 1e-13 * expect
    assert o.path_sigma((20.0, 20.0), (20.5, 20.0), tau) == 0.0


def test_weight_damping_lifts_the_velocity_assumption():
    """A beta = 0.5 particle: Eq. (alpha) assumes v = c, weight damping uses the
    particle's own path.  Error of Eq. (error) after exit (Sec. III protocol):
    weight damping no worse than the current damping and well below alpha = 1.
    Thresholds are ours: the paper prints no values."""
    import test_oracle_physics as P
    beta, nx, ny, L, tc, extra = 0.5, 64, 96, 10, 50, 60
    for theta in (0.0, 30.0):
        ref = P._exit_run(W.ALPHA_DAMPED, theta, beta, 3, 1.0)
        ref.step(tc + extra)
        errs = {}
        for mode in (W.ALPHA_ONE, W.ALPHA_DAMPED, W.ALPHA_WEIGHT):
            a = P._exit_run(mode, theta, beta, 1, 1.0)
            a.step(tc + extra)
            errs[mode] = P._energy_error(a, ref, nx, ny, L)
        assert errs[W.ALPHA_WEIGHT] <= 1.02 * errs[W.ALPHA_DAMPED], (theta, errs)
        assert errs[W.ALPHA_WEIGHT] < 0.7 * errs[W.ALPHA_ONE], (theta, errs)
