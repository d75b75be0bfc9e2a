"""Host-only checks of the C ABI: the library loads, exports every function that
include/pml_pic.h declares, and rejects bad parameters with the documented status
codes (pml_pic_workspace_size validates without touching a GPU)."""
import ctypes as C
import os
import re

import pytest

from paper_2201_09084_amd import binding as B
from paper_2201_09084_amd import workloads as W

HDR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "pml_pic.h")


def _declared_functions():
    text = open(HDR).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pml_pic_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(B.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return B.load_library()


def test_every_declared_function_is_exported(lib):
    names = _declared_functions()
    assert len(names) >= 17
    for n in names:
        assert hasattr(lib, n), n
    assert set(B.EXPORTED) == set(names)


def _size(cfg, **kw):
    p = B.make_params(cfg, max_particles=kw.pop("max_particles", 16))
    for k, v in kw.items():
        setattr(p, k, v)
    n = C.c_size_t(0)
    rc = B.load_library().pml_pic_workspace_size(C.byref(p), C.byref(n))
    return rc, n.value


def test_workspace_size_valid_configs(lib):
    rc, n = _size(W.single_particle_config())
    assert rc == 0 and n > 0
    rc2, n2 = _size(W.single_particle_config(precision=32))
    assert rc2 == 0 and n2 < n
    rc3, n3 = _size(W.beam3d_config(), max_particles=17 << 20)
    assert rc3 == 0 and n3 > 3e9


def test_parameter_validation_codes(lib):
    cfg = W.single_particle_config()
    assert _size(cfg, dt=0.71)[0] == -2                  # beyond the 2D Yee CFL limit 1/sqrt(2)
    assert _size(cfg, dim=4)[0] == -1
    assert _size(cfg, shape_order=4)[0] == -1
    assert _size(cfg, alpha_mode=4)[0] == -1
    assert _size(cfg, alpha_mode=3)[0] == 0                # per-particle weight damping
    assert _size(cfg, precision=16)[0] == -1
    assert _size(cfg, max_particles=-1)[0] == -1
    p = B.make_params(cfg)
    p.pml[0][1] = 200                                     # thicker than the 128-cell box
    n = C.c_size_t()
    assert lib.pml_pic_workspace_size(C.byref(p), C.byref(n)) == -1
    p = B.make_params(cfg)
    p.sigma_coef[0][3] = -1.0                             # negative conductivity
    assert lib.pml_pic_workspace_size(C.byref(p), C.byref(n)) == -1
    assert b"negative" in lib.pml_pic_last_error(None)
    p = B.make_params(cfg)
    p.dx[0] = 0.0
    assert lib.pml_pic_workspace_size(C.byref(p), C.byref(n)) == -1


def test_grid_size_limits(lib):
    """Grids whose padded arrays pass 2^31 samples (2D: 32-bit sample offsets) or whose
    tile-rounded cell count passes 2^31 (the sort's keys) are rejected before anything is
    allocated; the largest grids inside both limits are accepted."""
    def size2(n, pml=0):
        cfg = W.SimConfig(dim=2, n=(n, n), pml=((pml, pml),) * 2, dt=0.5, max_particles=4)
        return _size(cfg)

    assert size2(46000)[0] == 0                           # 46016 x 46009 samples < 2^31
    rc, _ = size2(46400)                                  # 46464 x 46409 > 2^31
    assert rc == -1 and b"32-bit sample offsets" in lib.pml_pic_last_error(None)

    def size3(nz, tile=(0, 0, 0)):
        cfg = W.SimConfig(dim=3, n=(2045, 2045, nz), pml=((0, 0),) * 3, dt=0.5, max_particles=4)
        p = B.make_params(cfg, max_particles=4)
        for d in range(3):
            p.tile[d] = tile[d]
        n = C.c_size_t()
        return lib.pml_pic_workspace_size(C.byref(p), C.byref(n))

    assert size3(504) == 0                                # 2048 x 2048 x 504 keys < 2^31
    assert size3(505) == -1                               # 2048 x 2048 x 512 = 2^31
    assert b"sort keys" in lib.pml_pic_last_error(None)
    assert size3(100, tile=(1 << 20, 8, 8)) == -1         # a huge tile rounds the key range up


def test_ck_solver_and_filter_validation(lib):
    """The Cole-Karkkainen solver is 3D with cubic cells and c dt <= dx (App. A); the
    binomial current filter is 3D with 0..4 passes."""
    cfg3 = W.SimConfig(dim=3, n=(16, 16, 16), pml=((4, 4),) * 3, dx=(1.0, 1.0, 1.0), dt=0.9,
                       sigma_coef=W.cubic_profile(3.2), max_particles=4)
    assert _size(cfg3, dt=0.9)[0] == -2                   # beyond the 3D Yee limit 1/sqrt(3)
    assert _size(cfg3, solver=1)[0] == 0
    assert _size(cfg3, solver=1, dt=1.0)[0] == 0          # the CK limit c dt = dx
    assert _size(cfg3, solver=1, dt=1.01)[0] == -2
    assert _size(cfg3, solver=2)[0] == -1
    p = B.make_params(cfg3, max_particles=4)
    p.solver = 1
    p.dx[2] = 1.1                                         # not cubic
    n = C.c_size_t()
    assert lib.pml_pic_workspace_size(C.byref(p), C.byref(n)) == -1
    assert b"cubic" in lib.pml_pic_last_error(None)
    cfg2 = W.single_particle_config()
    assert _size(cfg2, solver=1)[0] == -1                 # 2D
    assert _size(cfg2, filter_passes=1)[0] == -1          # 2D
    assert _size(cfg3, dt=0.5, filter_passes=5)[0] == -1
    sep = B.FLAG_SEPARATE_FIELDS
    rc0, n0 = _size(cfg3, dt=0.5, flags=sep)
    rc1, n1 = _size(cfg3, dt=0.5, filter_passes=1, flags=sep)
    assert rc0 == 0 and rc1 == 0 and n1 > n0              # the filter's scratch copy of J
    rc2, n2 = _size(cfg3, dt=0.5)                         # the one-pass update's second field set
    assert rc2 == 0 and n2 > n0


def test_beam_transport_validation(lib):
    """Per-face alpha entries 0..3 and not with weight damping; conductors 3D; the cavity
    run's Yee time step at the CFL limit itself is accepted."""
    cav = W.cavity_config(precision=32, max_source=1000)
    assert _size(cav, max_particles=1000)[0] == 0                     # c dt = dz / sqrt(3)
    rc0, n0 = _size(cav.replace(conductor=0, max_source=0), max_particles=1000)
    rc1, n1 = _size(cav, max_particles=1000)
    assert rc0 == 0 and n1 > n0                            # mask and source storage
    p = B.make_params(cav, max_particles=1000)
    p.dt = 1.0001 / 3 ** 0.5
    n = C.c_size_t()
    assert lib.pml_pic_workspace_size(C.byref(p), C.byref(n)) == -2
    cfg2 = W.single_particle_config()
    assert _size(cfg2, conductor=1)[0] == -1               # conductors are 3D
    p = B.make_params(cfg2)
    p.alpha_face[0][1] = 4
    assert lib.pml_pic_workspace_size(C.byref(p), C.byref(n)) == -1
    p = B.make_params(cfg2.replace(alpha_mode=W.ALPHA_WEIGHT))
    p.alpha_face[0][1] = 2
    assert lib.pml_pic_workspace_size(C.byref(p), C.byref(n)) == -1
    assert b"WEIGHT" in lib.pml_pic_last_error(None)
    p = B.make_params(cfg2)
    p.alpha_face[1][0] = 3
    assert lib.pml_pic_workspace_size(C.byref(p), C.byref(n)) == 0
    assert _size(cfg2, max_source=-1)[0] == -1


def test_create_rejects_small_or_missing_workspace(lib):
    p = B.make_params(W.single_particle_config(), max_particles=4)
    h = C.c_void_p()
    assert lib.pml_pic_create(C.byref(p), None, C.c_size_t(0), None, C.byref(h)) == -3
    assert lib.pml_pic_create(C.byref(p), C.c_void_p(256), C.c_size_t(10), None, C.byref(h)) == -3
    assert not h.value


_BAD_ALLOC_CHILD = r"""
import ctypes as C, sys
sys.path.insert(0, %r)
from paper_2201_09084_amd import binding as B
from paper_2201_09084_amd import workloads as W
L = B.load_library()
p = B.make_params(W.single_particle_config(), max_particles=16)
n = C.c_size_t(0)
# 2^31 - 1 runs: the per-run layout table alone would need terabytes of host memory;
# only the first run is read before that allocation
rc = L.pml_pic_batch_workspace_size(C.byref(p), 2**31 - 1, C.byref(n))
print("rc", rc, L.pml_pic_batch_last_error(None).decode(), flush=True)
"""


def test_host_allocation_failure_is_a_status_code(lib):
    """A host allocation sized by the caller's arguments that fails (std::bad_alloc) is
    caught inside the call and returned as PML_PIC_E_HOST with a message; without the
    guard the exception would cross the C ABI and abort the process (run in a child)."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, "-c", _BAD_ALLOC_CHILD % root], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 0, (r.returncode, r.stdout, r.stderr[-2000:])
    assert "rc -7 out of host memory" in r.stdout, r.stdout


def test_deterministic_mode_layout_and_batch_rejection(lib):
    """The deterministic debug mode takes the unfused, unsorted layout (no tile work
    lists), and batches refuse it."""
    cfg = W.SimConfig(dim=3, n=(13, 11, 9), pml=((4, 5), (3, 4), (5, 3)), dt=0.45, shape_order=1, precision=32)
    det = B.workspace_size(B.make_params(cfg, 1000, B.FLAG_DETERMINISTIC))
    plain = B.workspace_size(B.make_params(cfg, 1000, B.FLAG_UNFUSED | B.FLAG_NO_SORT))
    assert det == plain
    with pytest.raises(B.PmlPicError) as e:
        B.batch_workspace_size([B.make_params(cfg, 1, B.FLAG_DETERMINISTIC)] * 2)
    assert "single runs" in str(e.value)


def test_checked_build_exports_every_declared_function():
    """The bounds-checked debug build (libpmlpic_check.so) loads and exports the same calls."""
    path = os.path.join(os.path.dirname(B.__file__), "libpmlpic_check.so")
    assert os.path.exists(path), "build it with __graft_entry__.build()"
    L = C.CDLL(path)
    names = _declared_functions()
    assert len(names) >= 17
    for n in names:
        assert hasattr(L, n), n



def test_atomic_rates_rejects_null_output_without_a_gpu(lib):
    # the argument check comes before any HIP call
    assert lib.pml_pic_atomic_rates(C.POINTER(C.c_double)()) == B.PML_PIC_E_INVALID_ARG
    assert b"rates is NULL" in lib.pml_pic_last_error(None)
