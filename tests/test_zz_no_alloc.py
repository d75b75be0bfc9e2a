"""pml_pic_field_error_noalloc (partial sums in the library's static device scratch, no
allocation) against pml_pic_field_error (partials in the handle's workspace): the same
FP64 sums of Eq. (error) (Sec. III) up to the order of the additions, on two calls in a
row, the second on a smaller grid, and once more on the first."""
import numpy as np
import pytest

from gpu_helpers import say
from paper_2201_09084_amd import binding as B
from paper_2201_09084_amd import workloads as W

pytestmark = pytest.mark.gpu

# FP64 sums of up to ~1e8 non-negative terms in two different orders
TOL = 1e-12


def _random_pair(cfg, seed):
    """A run and a reference run with the same grid, seeded random split fields."""
    rng = np.random.default_rng(seed)
    g = B.PmlPic(cfg, max_particles=1)
    r = B.PmlPic(cfg, max_particles=1)
    shape = (12, g.nsamp)
    g.set_split_fields(rng.standard_normal(shape))
    r.set_split_fields(rng.standard_normal(shape))
    return g, r


def _check(g, r, what):
    a = g.field_error_sums(r)
    b = g.field_error_sums(r, noalloc=True)
    say(what, "workspace", a, "static scratch", b)
    assert a[0] > 0 and a[1] > 0
    assert abs(b[0] - a[0]) <= TOL * a[0], (what, a, b)
    assert abs(b[1] - a[1]) <= TOL * a[1], (what, a, b)
    assert g.field_error_sums(g, noalloc=True)[0] == 0.0


def test_noalloc_field_error_matches_workspace_form():
    # 200^3 nodes: 4 x 51 x 201 workgroups in the workspace form, more than the static
    # scratch's 32768, so the no-allocation form folds planes onto its workgroups
    big = W.SimConfig(dim=3, n=(180, 180, 180), pml=((10, 10), (10, 10), (10, 10)), dt=0.5,
                      precision=32, push=0)
    small = W.SimConfig(dim=2, n=(70, 50, 1), pml=((8, 8), (6, 6), (0, 0)), precision=64, push=0)
    g, r = _random_pair(big, 7)
    _check(g, r, "3D 200^3 FP32")
    del g, r
    g2, r2 = _random_pair(small, 8)
    _check(g2, r2, "2D 86x62 FP64")
    g3, r3 = _random_pair(big.replace(n=(60, 40, 30)), 9)
    _check(g3, r3, "3D 80x60x50 FP32")
