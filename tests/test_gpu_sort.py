"""sort_particles checked bit for bit (integer work): after pml_pic_sort_particles the live
particles sit in non-decreasing order of their cell's tile-major key, key_start is the
exclusive prefix sum of the host histogram of those keys (then the live count), every id
appears exactly once, removed particles are gone, and every particle's state is unchanged.
Cases: 2D and 3D ragged grids with uneven PMLs, dense clusters mixed with sparse particles
over box and PML, particles removed at the outer wall, the default and odd tile shapes."""
import numpy as np
import pytest

from gpu_helpers import say
from paper_2201_09084_amd import binding as B
from paper_2201_09084_amd import workloads as W

pytestmark = pytest.mark.gpu


def _keys(cfg, X, tile):
    """Host reference of the documented tile-major key of each particle's cell."""
    M = [cfg.n[d] + cfg.pml[d][0] + cfg.pml[d][1] if d < cfg.dim else 1 for d in range(3)]
    ntile = [(M[d] + tile[d] - 1) // tile[d] for d in range(3)]
    cell = np.floor(X).astype(np.int64)
    cell[:, cfg.dim:] = 0
    t = cell // np.array(tile)
    loc = cell - t * np.array(tile)
    tid = (t[:, 2] * ntile[1] + t[:, 1]) * ntile[0] + t[:, 0]
    lid = (loc[:, 2] * tile[1] + loc[:, 1]) * tile[0] + loc[:, 0]
    return tid * (tile[0] * tile[1] * tile[2]) + lid, int(np.prod([ntile[d] * tile[d] for d in range(3)]))


def _cluster(cfg, n, centre, rms, seed):
    rng = np.random.default_rng(seed)
    x = np.asarray(centre, float) + rms * rng.standard_normal((n, cfg.dim))
    return W.Particles(x=x, u=rng.uniform(-0.5, 0.5, (n, 3)), w=rng.uniform(0.5, 1.5, n))


def _shuffled(parts, seed):
    o = np.random.default_rng(seed).permutation(len(parts.w))
    return W.Particles(x=parts.x[o], u=parts.u[o], w=parts.w[o])


def _check_sort(g, cfg, what):
    ids0, X0, u0, w0 = g.particles()                 # by id
    tile, ks = g.sort_particles()
    ids, X, u, w = g.particles(device_order=True)
    n = len(ids)
    say(what, "tile", tile, "live", n, "keys", len(ks) - 1)
    assert n == len(ids0) and n > 0
    assert np.array_equal(np.sort(ids), ids0), "ids are not the same set"
    assert len(np.unique(ids)) == n
    o = np.argsort(ids, kind="stable")
    assert np.array_equal(X[o], X0) and np.array_equal(u[o], u0) and np.array_equal(w[o], w0)
    keys, nkeys = _keys(cfg, X, tile)
    assert nkeys == len(ks) - 1
    assert np.all(np.diff(keys) >= 0), "keys decrease in device order"
    hist = np.bincount(keys, minlength=nkeys)
    start = np.concatenate(([0], np.cumsum(hist)[:-1]))
    assert np.array_equal(ks[:nkeys].astype(np.int64), start)
    assert int(ks[nkeys]) == n
    return n


@pytest.mark.parametrize("dim,tile", [(2, (0, 0, 0)), (2, (5, 3, 1)), (3, (0, 0, 0)), (3, (3, 5, 2))])
def test_sort_particles_bit_exact(dim, tile):
    if dim == 2:
        cfg = W.SimConfig(dim=2, n=(37, 29, 1), pml=((6, 9), (7, 5), (0, 0)), dx=(1.0, 0.9, 1.0), dt=0.6,
                          shape_order=2, push=1, precision=32, tile=tile)
        dense = _cluster(cfg, 3000, (12.0, 10.0), 0.7, 1)
    else:
        cfg = W.SimConfig(dim=3, n=(13, 11, 9), pml=((4, 5), (3, 4), (5, 3)), dx=(1.0, 0.9, 1.1), dt=0.45,
                          shape_order=1, push=1, precision=32, tile=tile)
        dense = _cluster(cfg, 3000, (6.0, 5.0, 4.0), 0.6, 1)
    sparse = W.random_particles(cfg, 2000, seed=2, margin=0.05, umax=3.0)
    parts = _shuffled(W.Particles(x=np.concatenate([dense.x, sparse.x]), u=np.concatenate([dense.u, sparse.u]),
                                  w=np.concatenate([dense.w, sparse.w])), 3)
    g = B.PmlPic(cfg, max_particles=len(parts.w))
    g.add_particles(parts.x, parts.u, parts.w)
    n0 = _check_sort(g, cfg, "after add")
    assert n0 == len(parts.w)
    # steps: particles move (some across tiles), those past the outer walls are removed
    g.step(3)
    n1 = _check_sort(g, cfg, "after 3 steps")
    assert n1 < n0, "no particle left through the walls"
    assert n1 == g.num_particles
