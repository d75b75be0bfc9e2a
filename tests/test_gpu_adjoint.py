"""Adjoint of the step.

Ballistic particles (push = 0): the transposed update checked by the dot-product identity,
the gradient of the interior field energy against the oracle's central differences, FP32
against FP64, checkpoint segment invariance, the torch.autograd.Function wrapper.

Pushed particles (push = 1, the whole step: gather, Boris push and Esirkepov deposit
reversed too): from random initial fields (so the particles' response to the fields is
large), the profile gradient, the particles' dU/dx0 and dU/du0 and the adjoint of the
initial fields in a random direction, each against the FP64 oracle's Richardson-extrapolated
central differences, in 2D and 3D for shape orders 1-3; FP32 against FP64; segment
invariance.

The full-size workload (2D 512^2, 16-cell PML, 4096-particle bunch, 500 steps,
checkpoints every 50, sigma/eps0 = 3.2 r^3, s = 1): ballistic and pushed, FP32 against
FP64, and the pushed FP64 gradient against the oracle's differences stored in
tests/golden/adjoint_c5_pushed_fd.json.

A finite-difference reference carries its own error: the tolerance on each comparison is
a small relative slack plus four times the difference between the estimates at h and h/2
(which bounds the error of the extrapolated value)."""
import json
import os

import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import say
from paper_2201_09084_amd import adjoint as A
from paper_2201_09084_amd import binding as B
from paper_2201_09084_amd import workloads as W

pytestmark = pytest.mark.gpu


def _grad(cfg, p, steps, seg, seed=None, want_lambda=False, fields=None):
    sim = A.make_sim(cfg, A.theta_of(cfg), p, steps, seg)
    if fields is not None:
        sim.set_split_fields(fields)
    U = sim.forward_ckpt(steps)
    g, lam = sim.backward(seed=seed, want_lambda=want_lambda)
    return U, g, lam, sim


@pytest.mark.parametrize("dim", [2, 3])
def test_dot_product_identity_fp64(dim):
    """With the particles fixed the map from the initial to the final fields is affine,
    so seed . (S_n(S0 + d) - S_n(S0)) must equal lambda_0 . d."""
    cfg = W.adjoint_small_config(n=24 if dim == 2 else 12, pml=6 if dim == 2 else 4, dim=dim)
    p = W.adjoint_small_particles(cfg, 4)
    steps = 40 if dim == 2 else 24
    S0 = W.random_split_fields(cfg, 31, amp=0.1)
    seed = W.random_split_fields(cfg, 32)
    d = W.random_split_fields(cfg, 33)
    say("dot-product test dim", dim, "steps", steps)
    _, _, lam, _ = _grad(cfg, p, steps, 9, seed=seed, want_lambda=True, fields=S0)
    runs = []
    for F in (S0, S0 + d):
        s = B.PmlPic(cfg, max_particles=len(p.w))
        s.set_split_fields(F)
        s.add_particles(p.x, p.u, p.w)
        s.step(steps)
        runs.append(s.split_fields())
    lhs = float(np.sum(seed * (runs[1] - runs[0])))
    rhs = float(np.sum(lam * d))
    say("  seed.dS", lhs, "lambda.d", rhs)
    assert abs(lhs - rhs) <= 1e-11 * max(abs(lhs), 1e-30)


@pytest.mark.parametrize("dim", [2, 3])
def test_energy_gradient_matches_oracle_differences(dim):
    if dim == 2:
        cfg = W.adjoint_small_config()
        steps, idx = 80, [0, 1, 2, 3, 5, 9, 15, 16, 18, 19, 24, 32]
    else:
        cfg = W.adjoint_small_config(n=12, pml=4, dim=3)
        steps, idx = 36, [0, 3, 19, 35, 48]
    p = W.adjoint_small_particles(cfg, 4)
    U, g, _, _ = _grad(cfg, p, steps, 10)
    Uo = oracle.interior_energy(cfg, p.x, p.u, p.w, steps)
    say("dim", dim, "U gpu", U, "oracle", Uo)
    assert abs(U - Uo) <= 1e-12 * abs(Uo)
    ref = oracle.fd_gradient(cfg, p.x, p.u, p.w, steps, idx=idx)
    scale = np.nanmax(np.abs(ref))
    err = np.max(np.abs(g[idx] - ref[idx])) / scale
    say("  max |adjoint - differences| / max |dU/dtheta| =", err)
    assert err <= 1e-6


def test_fp32_gradient_close_to_fp64():
    cfg = W.adjoint_small_config(n=64, pml=12)
    p = W.adjoint_small_particles(cfg, 64)
    _, g64, _, _ = _grad(cfg, p, 120, 20)
    _, g32, _, _ = _grad(cfg.replace(precision=32), p, 120, 20)
    err = np.max(np.abs(g32 - g64)) / np.max(np.abs(g64))
    say("FP32 vs FP64 gradient, max-norm relative", err)
    assert err <= 1e-3


def test_segment_length_does_not_change_the_gradient():
    cfg = W.adjoint_small_config()
    p = W.adjoint_small_particles(cfg, 4)
    U1, g1, _, _ = _grad(cfg, p, 60, 7)
    U2, g2, _, _ = _grad(cfg, p, 60, 60)
    assert abs(U1 - U2) <= 1e-13 * abs(U1)
    assert np.max(np.abs(g1 - g2)) <= 1e-11 * np.max(np.abs(g1))


def test_parameters_without_effect_get_zero():
    cfg = W.adjoint_small_config(n=24, pml=6).replace(alpha_mode=W.ALPHA_ONE, pml=((6, 6), (0, 0), (0, 0)))
    p = W.adjoint_small_particles(cfg, 4)
    _, g, _, _ = _grad(cfg, p, 40, 10)
    assert g[32] == 0.0
    assert np.all(g[16:32] == 0.0)
    assert np.any(g[:16] != 0.0)


def test_backward_leaves_the_final_state():
    cfg = W.adjoint_small_config(n=24, pml=6)
    p = W.adjoint_small_particles(cfg, 4)
    sim = A.make_sim(cfg, A.theta_of(cfg), p, 30, 8)
    sim.forward_ckpt(30)
    F = sim.split_fields()
    ids = sim.particles()[0]
    sim.backward()
    assert np.array_equal(sim.split_fields(), F)
    assert np.array_equal(sim.particles()[0], ids)
    g1, _ = sim.backward()                 # a second reverse pass gives the same gradient
    g2, _ = sim.backward()
    assert np.max(np.abs(g1 - g2)) <= 1e-12 * np.max(np.abs(g1))


def test_invalid_uses_are_rejected():
    cfg = W.adjoint_small_config(n=24, pml=6)
    p = W.adjoint_small_particles(cfg, 2)
    sim = A.make_sim(cfg, A.theta_of(cfg), p, 20, 10)
    with pytest.raises(B.PmlPicError):
        sim.backward()                     # nothing to reverse yet
    with pytest.raises(B.PmlPicError):
        sim.forward_ckpt(21)               # more than checkpoints x segment
    plain = B.PmlPic(cfg, max_particles=2)
    with pytest.raises(B.PmlPicError):
        plain.forward_ckpt(5)              # no adjoint storage
    with pytest.raises(B.PmlPicError):
        A.make_sim(cfg.replace(alpha_mode=W.ALPHA_WEIGHT), A.theta_of(cfg), p, 20, 10).forward_ckpt(5)
    sim.forward_ckpt(10)
    sim.backward()
    with pytest.raises(B.PmlPicError):
        sim.particle_adjoint(2)            # a ballistic reverse pass has no particle adjoint
    pushed = A.make_sim(cfg.replace(push=1), A.theta_of(cfg), p, 20, 10)
    pushed.forward_ckpt(10)
    with pytest.raises(B.PmlPicError):
        pushed.particle_adjoint(2)         # not reversed yet
    pushed.backward()
    with pytest.raises(B.PmlPicError):
        pushed.particle_adjoint(3)         # more ids than particles added
    assert pushed.particle_adjoint(2)[1].shape == (2, 3)


def test_autograd_function():
    cfg = W.adjoint_small_config(n=24, pml=6)
    p = W.adjoint_small_particles(cfg, 4)
    theta = torch.tensor(A.theta_of(cfg), dtype=torch.float64, requires_grad=True)
    U = A.interior_energy(theta, cfg, p, 40, segment=10)
    (2.0 * U).backward()
    _, g, _, _ = _grad(cfg, p, 40, 10)
    assert np.max(np.abs(theta.grad.numpy() - 2.0 * g)) <= 1e-12 * np.max(np.abs(g))


def test_full_size_workload_fp32_against_fp64_and_differences():
    """Ballistic: 2D 512 x 512, 16-cell layer, 4096-particle bunch, 500 steps, checkpoints
    every 50, sigma/eps0 = 3.2 r^3: FP32 gradient against the FP64 gradient, and the FP64
    gradient against central differences of the FP64 forward run on the GPU for the
    parameters that are non-zero at this profile."""
    cfg64 = W.adjoint_config(precision=64)
    p = W.adjoint_particles(cfg64)
    steps, seg = 500, 50
    U64, g64, _, _ = _grad(cfg64, p, steps, seg)
    U32, g32, _, _ = _grad(cfg64.replace(precision=32), p, steps, seg)
    err = np.max(np.abs(g32 - g64)) / np.max(np.abs(g64))
    say("C5: U fp64", U64, "fp32", U32, "gradient rel diff", err)
    assert abs(U32 - U64) <= 1e-4 * abs(U64)
    assert err <= 1e-3
    th0 = A.theta_of(cfg64)
    for i in (3, 19, 32):
        h = 1e-3 * abs(th0[i])
        D = []
        for hh in (h, 0.5 * h):
            Us = []
            for sgn in (1, -1):
                th = th0.copy()
                th[i] += sgn * hh
                s = B.PmlPic(A.with_theta(cfg64, th), max_particles=len(p.w))
                s.add_particles(p.x, p.u, p.w)
                s.step(steps)
                Us.append(s.diagnose()["u_interior"])
            D.append((Us[0] - Us[1]) / (2 * hh))
        fd = (4 * D[1] - D[0]) / 3
        say("  theta", i, "adjoint", g64[i], "differences", fd)
        assert abs(g64[i] - fd) <= 1e-6 * np.max(np.abs(g64))


# ---------------------------------------------------------------- pushed particles
def _pushed_case(dim, order):
    if dim == 2:
        cfg = W.adjoint_small_config().replace(push=1, shape_order=order)
        steps = 60
    else:
        cfg = W.adjoint_small_config(n=12, pml=4, dim=3).replace(push=1, shape_order=order)
        steps = 30
    p = W.adjoint_small_particles(cfg, 4)
    S0 = W.random_split_fields(cfg, 41, amp=0.05)
    return cfg, p, steps, S0


def _oracle_U(cfg, p, steps, S0, theta=None, x=None, u=None):
    c = cfg if theta is None else oracle.with_theta(cfg, theta)
    return oracle.interior_energy(c, p.x if x is None else x, p.u if u is None else u, p.w, steps, fields=S0)


def _richardson(f, h):
    """Central differences at h and h/2, extrapolated; and |D(h) - D(h/2)|."""
    D = [(f(hh) - f(-hh)) / (2.0 * hh) for hh in (h, 0.5 * h)]
    return (4.0 * D[1] - D[0]) / 3.0, abs(D[1] - D[0])


def _check(name, got, ref, err, scale, rel=1e-7):
    tol = rel * scale + 1e-6 * abs(ref) + 4.0 * err
    say("  %-10s adjoint % .10e differences % .10e |diff| %.2e tol %.2e" % (name, got, ref, abs(got - ref), tol))
    assert abs(got - ref) <= tol, name


@pytest.mark.parametrize("dim,order", [(2, 1), (2, 2), (2, 3), (3, 1), (3, 2)])
def test_pushed_adjoint_matches_oracle_differences(dim, order):
    """Profile gradient, particle adjoints and the initial-field adjoint of a pushed run."""
    cfg, p, steps, S0 = _pushed_case(dim, order)
    sim = A.make_sim(cfg, A.theta_of(cfg), p, steps, 7)
    sim.set_split_fields(S0)
    U = sim.forward_ckpt(steps)
    g, lam = sim.backward(want_lambda=True)
    gx, gu = sim.particle_adjoint(len(p.w))
    Uo = _oracle_U(cfg, p, steps, S0)
    say("dim", dim, "order", order, "U gpu", U, "oracle", Uo)
    assert abs(U - Uo) <= 1e-12 * abs(Uo)
    th0 = oracle.theta_vector(cfg)
    idx = [0, 3, 5, 16, 19, 32] if dim == 2 else [0, 3, 19, 35, 48]
    refs = {}
    for i in idx:
        def f(e, i=i):
            th = th0.copy()
            th[i] += e
            return _oracle_U(cfg, p, steps, S0, theta=th)
        refs[i] = _richardson(f, 1e-3 * max(abs(th0[i]), 0.1))
    scale = max(abs(r[0]) for r in refs.values())
    for i in idx:
        _check("theta %d" % i, g[i], refs[i][0], refs[i][1], scale)
    prefs = []
    for j in range(2):
        for c in range(dim + 3):
            def f(e, j=j, c=c):
                x, u = p.x.copy(), p.u.copy()
                if c < dim:
                    x[j, c] += e
                else:
                    u[j, c - dim] += e
                return _oracle_U(cfg, p, steps, S0, x=x, u=u)
            got = gx[j, c] if c < dim else gu[j, c - dim]
            prefs.append(("%s[%d,%d]" % ("x" if c < dim else "u", j, c if c < dim else c - dim), got)
                         + _richardson(f, 1e-5))
    scale = max(abs(r[2]) for r in prefs)
    for name, got, ref, err in prefs:
        _check(name, got, ref, err, scale)
    d = W.random_split_fields(cfg, 43)
    ref, err = _richardson(lambda e: _oracle_U(cfg, p, steps, S0 + e * d), 1e-4)
    _check("fields.d", float(np.sum(lam * d)), ref, err, abs(ref))


def test_pushed_segment_length_does_not_change_the_gradient():
    cfg, p, steps, S0 = _pushed_case(2, 2)
    out = []
    for seg in (7, 60):
        sim = A.make_sim(cfg, A.theta_of(cfg), p, steps, seg)
        sim.set_split_fields(S0)
        U = sim.forward_ckpt(steps)
        g, _ = sim.backward()
        out.append((U, g, sim.particle_adjoint(len(p.w))[1]))
    assert abs(out[0][0] - out[1][0]) <= 1e-13 * abs(out[0][0])
    assert np.max(np.abs(out[0][1] - out[1][1])) <= 1e-11 * np.max(np.abs(out[0][1]))
    assert np.max(np.abs(out[0][2] - out[1][2])) <= 1e-11 * np.max(np.abs(out[0][2]))


def test_pushed_fp32_gradient_close_to_fp64():
    cfg = W.adjoint_small_config(n=64, pml=12).replace(push=1)
    p = W.adjoint_small_particles(cfg, 64)
    _, g64, _, _ = _grad(cfg, p, 120, 20)
    _, g32, _, _ = _grad(cfg.replace(precision=32), p, 120, 20)
    err = np.max(np.abs(g32 - g64)) / np.max(np.abs(g64))
    say("pushed FP32 vs FP64 gradient, max-norm relative", err)
    assert err <= 1e-3


def test_full_size_pushed_workload_against_oracle_differences():
    """Pushed: the full-size workload at sigma/eps0 = 3.2 r^3, s = 1 (the bunch crosses the
    +x layer and leaves through the outer wall by step ~150; U after 500 steps).  FP64 U
    and gradient against the oracle's stored values, FP32 against FP64."""
    with open(os.path.join(os.path.dirname(__file__), "golden", "adjoint_c5_pushed_fd.json")) as fh:
        ref = json.load(fh)
    cfg64 = W.adjoint_config(precision=64).replace(push=1)
    p = W.adjoint_particles(cfg64)
    steps, seg = 500, 50
    U64, g64, _, sim = _grad(cfg64, p, steps, seg)
    gx, gu = sim.particle_adjoint(len(p.w))
    U32, g32, _, _ = _grad(cfg64.replace(precision=32), p, steps, seg)
    err = np.max(np.abs(g32 - g64)) / np.max(np.abs(g64))
    say("C5 pushed: U fp64", U64, "oracle", ref["U"], "fp32", U32, "gradient fp32 vs fp64", err)
    say("  |dU/du0| max", np.max(np.abs(gu)), "|dU/dx0| max", np.max(np.abs(gx)))
    assert abs(U64 - ref["U"]) <= 1e-10 * abs(ref["U"])
    assert abs(U32 - U64) <= 1e-4 * abs(U64)
    assert err <= 1e-3
    scale = np.max(np.abs(g64))
    for i, r in ref["derivatives"].items():
        _check("theta " + i, g64[int(i)], r["value"], r["error_estimate"], scale, rel=1e-10)
