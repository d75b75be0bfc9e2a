"""The beam-deflection measurement of the cavity run (Sec. IV.A, Fig. 5) on top of the
library's slab moments.

<u_x> = <p_x>/mc of the beam is recorded where the beam crosses four z-planes (54 and 35 mm
before and after the box centre).  Every particle of the gamma = 479 beam moves at the same
v_z, so the slab of width v_z dt just past a plane holds exactly the particles that crossed
it during the last step; summing that slab's moments over the steps gives the crossing
averages.  The unphysical deflection near each PML is the change of <u_x> between the outer
and inner plane on that side minus the same change in a reference run whose box is twice as
long (its PMLs far from the planes); the physical deflection is the reference change between
the two outer planes.
"""
import math

import numpy as np

from . import binding as B
from . import workloads as W

# per-face damping of the z faces (entries 1 + mode): the schemes of Fig. 4-5 and the
# combination suggested at the end of Sec. IV.A
SCHEMES = {
    "standard": ((0, 0), (0, 0), (1, 1)),        # alpha = 0 in both PMLs
    "undamped": ((0, 0), (0, 0), (2, 2)),        # alpha = 1
    "damped": ((0, 0), (0, 0), (3, 3)),          # Eq. (alpha), v = c
    "undamped_entry": ((0, 0), (0, 0), (2, 3)),  # alpha = 1 where the beam enters, Eq. (alpha) where it leaves
}


def crossing_ux(faces, nz=108, cavity=(34.0, 74.0), n_macro=1 << 18, precision=64, gamma=479.0, seed=1006):
    """Runs one transit of the cavity and returns (planes, <u_x> at each plane, count)."""
    cfg = W.cavity_config(precision=precision, n=(64, 64, nz), max_source=n_macro, alpha_face=faces)
    beam = W.cavity_beam(cfg, n_macro=n_macro, seed=seed, gamma=gamma)
    sim = B.PmlPic(cfg, max_particles=n_macro)
    sim.set_conductor(W.cavity_conductor(cfg, cavity=cavity))
    sim.set_source(beam.x, beam.u, beam.w, axis=2)
    planes = W.deflection_planes(cfg)
    vz = math.sqrt(gamma * gamma - 1.0) / gamma
    width = vz * cfg.dt
    edges = np.ravel([[p, p + width] for p in planes])
    tail = np.min(beam.x[:, 2])
    nsteps = int(math.ceil((planes[-1] + width - tail) / width)) + 2
    acc = np.zeros((len(planes), 5))
    for _ in range(nsteps):
        sim.step(1)
        acc += sim.slab_moments(2, edges)[0::2]
    return planes, acc[:, 2] / acc[:, 1], acc[:, 0]


def unphysical_deflection(n_macro=1 << 18, precision=64, schemes=None):
    """{scheme: (left, right)} unphysical deflections and the physical one (reference run)."""
    ref_planes, ref, _ = crossing_ux(SCHEMES["damped"], nz=216, cavity=(88.0, 128.0), n_macro=n_macro,
                                     precision=precision)
    physical = ref[3] - ref[0]
    out = {}
    for name in (schemes or SCHEMES):
        _, u, _ = crossing_ux(SCHEMES[name], n_macro=n_macro, precision=precision)
        out[name] = ((u[1] - u[0]) - (ref[1] - ref[0]), (u[3] - u[2]) - (ref[3] - ref[2]))
    return out, physical
