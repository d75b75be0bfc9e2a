"""Shared helpers for the GPU parity tests: run the HIP path and the FP64 oracle on the
same seeded inputs and compare."""
import sys

import numpy as np

import oracle
from paper_2201_09084_amd import binding as B
from paper_2201_09084_amd import workloads as W


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def both(cfg, particles=None, fields=None, max_particles=None, flags=0, X_ids=None, parallel=False):
    """Creates a GPU simulation and an oracle with the same configuration and inputs
    (parallel: the oracle's all-cores build, for the largest cases)."""
    n = len(particles) if particles is not None else 0
    cap = max_particles if max_particles is not None else max(n, 1)
    g = B.PmlPic(cfg, max_particles=cap, flags=flags)
    o = oracle.OracleSim(cfg, parallel=parallel)
    if fields is not None:
        g.set_split_fields(fields)
        o.set_split_fields(fields)
    if particles is not None and n:
        g.add_particles(particles.x, particles.u, particles.w)
        o.add_particles(particles.x, particles.u, particles.w)
    return g, o


def rel_err(a, b):
    """max |a - b| / max |b| (0 if both are zero)"""
    scale = np.max(np.abs(b))
    d = np.max(np.abs(a - b))
    if scale == 0.0:
        return d
    return d / scale


def rel_l2(a, b):
    nb = np.linalg.norm(b)
    if nb == 0.0:
        return np.linalg.norm(a)
    return np.linalg.norm(a - b) / nb


def split_active_mask(cfg, comp):
    """Samples where component comp (0..5) keeps two split parts on the GPU."""
    o = oracle.OracleSim(cfg)
    nn = cfg.nodes()
    a = comp % 3
    b, c = (a + 1) % 3, (a + 2) % 3
    if cfg.dim == 2 and (b == 2 or c == 2):
        return np.zeros((nn[2], nn[1], nn[0]), bool)
    off = 0.0 if comp < 3 else 0.5
    sb = np.array([o.sigma(b, i + off) for i in range(nn[b])])
    sc = np.array([o.sigma(c, i + off) for i in range(nn[c])])
    shape = [1, 1, 1]
    shape[2 - b] = nn[b]
    sbv = sb.reshape(shape)
    shape = [1, 1, 1]
    shape[2 - c] = nn[c]
    scv = sc.reshape(shape)
    return np.broadcast_to((sbv + scv) > 0, (nn[2], nn[1], nn[0]))


def compare_fields(g, o, cfg, tol, what="", l2=False):
    Fg = g.split_fields()
    Fo = o.split_fields()
    tg = Fg[0::2] + Fg[1::2]
    to = Fo[0::2] + Fo[1::2]
    worst = 0.0
    for c in range(6):
        e = rel_l2(tg[c], to[c]) if l2 else rel_err(tg[c], to[c])
        if np.max(np.abs(to[c])) == 0.0:
            assert np.max(np.abs(tg[c])) <= 1e-12, (what, c, np.max(np.abs(tg[c])))
            continue
        worst = max(worst, e)
        assert e <= tol, (what, "component", c, e)
        m = split_active_mask(cfg, c)
        if m.any():
            e2 = rel_err(Fg[2 * c][m], Fo[2 * c][m]) if not l2 else rel_l2(Fg[2 * c][m], Fo[2 * c][m])
            if np.max(np.abs(Fo[2 * c][m])) > 0:
                assert e2 <= max(tol, 1e-12) * 10, (what, "split part", c, e2)
    return worst


def compare_current(g, o, tol, what=""):
    """J of the last step, component by component, over the edges inside the box: J_a
    at the last node index along axis a is padding beyond the outer wall (a particle
    leaving the box may deposit there on the GPU, the oracle drops it)."""
    Jg, Jo = g.current(), o.current()
    for a in range(3):
        sl = [slice(None)] * 3
        if Jg[a].shape[2 - a] > 1:        # J_z of a 2D run has no staggered axis
            sl[2 - a] = slice(0, -1)
        jg, jo = Jg[a][tuple(sl)], Jo[a][tuple(sl)]
        s = np.max(np.abs(jo))
        err = np.max(np.abs(jg - jo))
        assert err <= tol * max(s, 1e-30), (what, "J", a, err, s)


def compare_particles(g, o, tol_x, tol_u, what=""):
    ig, Xg, ug, wg = g.particles()
    io, Xo, uo, wo = o.particles()
    order = np.argsort(io, kind="stable")
    io, Xo, uo, wo = io[order], Xo[order], uo[order], wo[order]
    assert np.array_equal(ig, io), (what, "particle ids differ", len(ig), len(io))
    if len(ig) == 0:
        return 0.0, 0.0
    ex = np.max(np.abs(Xg - Xo))
    eu = np.max(np.abs(ug - uo)) / max(1.0, np.max(np.abs(uo)))
    assert ex <= tol_x, (what, "position", ex)
    assert eu <= tol_u, (what, "momentum", eu)
    return ex, eu
