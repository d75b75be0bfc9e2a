"""The single-particle exit error of Sec. III (Figs. 2 and 3) with the numerics of App. A.

A macroparticle starts near the middle of the 3D box moving toward the +x PML at angle theta
(in the x-y plane) and crosses the interface at t = 65 dt; at t = 125 dt its fields are
compared with those of a reference run in a box doubled along x (the particle never meets a
PML there) through Eq. (error), an FP64 reduction on the GPU (pml_pic_field_error):

    E = sum over samples in the physical box of (E - E_ref)^2 + (B - B_ref)^2
        / sum of E_ref^2 + B_ref^2.

Fields start at zero; the motionless opposite-charge partner of App. A.1 is implicit (the
charge-conserving deposit makes E consistent with the moving charge plus its partner).  The
particle moves at its initial velocity (push = 0): the error then measures the fields' PML
artefacts alone, and slow particles are not pulled back by their partner before they reach
the PML (a reading; the paper does not say how its particle was pushed).
"""
import math

import numpy as np

from . import binding as B
from . import workloads as W

T_CROSS, T_END = 65, 125


def _config(mode, n, pml, precision, extend_x=1, damping_scale=1.0):
    return W.SimConfig(dim=3, n=(n * extend_x, n, n), pml=((pml, pml),) * 3, dt=1.0, shape_order=3,
                       alpha_mode=mode, damping_scale=damping_scale,
                       sigma_coef=W.paper_conductivity_profile(pml), push=0, precision=precision,
                       solver=1, filter_passes=1)


def _start(n, theta, beta):
    """Start so that the particle crosses x = n at T_CROSS, at mid-height in y then."""
    v = beta
    x0 = n - T_CROSS * v * math.cos(theta)
    y0 = n / 2.0 - T_CROSS * v * math.sin(theta)
    return np.array([[x0, y0, n / 2.0]])


def _run(cfg, x0, u):
    sim = B.PmlPic(cfg, max_particles=1)
    sim.add_particles(x0, u, np.array([1.0]))
    sim.step(T_END)
    return sim


def exit_errors(theta_deg=0.0, gamma_beta=math.sqrt(99.0), modes=(0, 1, 2), n=128, pml=8, precision=64):
    """{mode: Eq. (error)} for a particle with momentum u = gamma beta c at angle theta."""
    th = math.radians(theta_deg)
    gam = math.sqrt(1.0 + gamma_beta ** 2)
    beta = gamma_beta / gam
    x0 = _start(n, th, beta)
    u = np.array([[gamma_beta * math.cos(th), gamma_beta * math.sin(th), 0.0]])
    ref = _run(_config(W.ALPHA_DAMPED, n, pml, precision, extend_x=2), x0, u)
    out = {}
    for mode in modes:
        out[mode] = _run(_config(mode, n, pml, precision), x0, u).field_error(ref)
    return out
