"""FP64 CPU oracle of the damped-current PML particle-in-cell step.

TEST INFRASTRUCTURE ONLY.  The test suite, the smoke check and the CPU-baseline leg
of the benchmark may use this package; the product library never does.  It wraps the
plain C implementation in ``pml_oracle.c`` (built by ``oracle/build.py`` with gcc) via
ctypes, and shares no code with the HIP library.

A simulation is configured from any object with the attributes ``dim, n, pml, dx,
dt, shape_order, alpha_mode, damping_scale, sigma_coef, push, charge, mass``.
Functions whose result has no independent pin say so in their docstring
("parity unpinned").
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_LIB_OMP_PATH = os.path.join(_HERE, "liboracle_omp.so")
_lib = None
_lib_omp = None

NPARTS = 12
PART_NAMES = ["Exy", "Exz", "Eyz", "Eyx", "Ezx", "Ezy",
              "Bxy", "Bxz", "Byz", "Byx", "Bzx", "Bzy"]


class OrcParams(C.Structure):
    _fields_ = [
        ("dim", C.c_int), ("n", C.c_int * 3), ("pml", (C.c_int * 2) * 3),
        ("dx", C.c_double * 3), ("dt", C.c_double), ("shape_order", C.c_int),
        ("alpha_mode", C.c_int), ("damping_scale", C.c_double), ("n_sigma_coef", C.c_int),
        ("sigma_coef", (C.c_double * 16) * 3), ("push", C.c_int),
        ("charge", C.c_double), ("mass", C.c_double),
        ("solver", C.c_int), ("filter_passes", C.c_int), ("alpha_face", (C.c_int * 2) * 3),
    ]


def build_library(force: bool = False) -> str:
    """Compiles liboracle.so and liboracle_omp.so with gcc (oracle/build.py)."""
    from . import build as _b
    return _b.build(force=force)


def lib():
    """The single-threaded build (liboracle.so)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build_library()
        _lib = _load(_LIB_PATH)
    return _lib


def lib_parallel():
    """The all-cores build of the same source (liboracle_omp.so, gcc -fopenmp)."""
    global _lib_omp
    if _lib_omp is None:
        if not os.path.exists(_LIB_OMP_PATH):
            build_library()
        _lib_omp = _load(_LIB_OMP_PATH)
    return _lib_omp


def num_threads() -> int:
    """Threads the all-cores build uses (OpenMP's default: OMP_NUM_THREADS or the cores)."""
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.strip().split(",")[0].isdigit():
        return int(env.strip().split(",")[0])
    return len(os.sched_getaffinity(0))


def _load(path):
    """Loads one build and declares the C signatures."""
    L = C.CDLL(path)
    P = C.POINTER
    d, vp, i, l, sz = C.c_double, C.c_void_p, C.c_int, C.c_long, C.c_size_t
    dp = P(C.c_double)
    lp = P(C.c_long)
    sig = {
        "orc_shape": (d, [i, d]),
        "orc_sigma": (d, [vp, i, d]),
        "orc_alpha_axis": (d, [vp, i, d]),
        "orc_alpha": (d, [vp, dp]),
        "orc_create": (vp, [P(OrcParams)]),
        "orc_destroy": (None, [vp]),
        "orc_num_samples": (sz, [vp]),
        "orc_num_particles": (l, [vp]),
        "orc_step_count": (l, [vp]),
        "orc_add_particles": (i, [vp, l, dp, dp, dp]),
        "orc_set_particles": (i, [vp, l, lp, dp, dp, dp]),
        "orc_get_particles": (None, [vp, lp, dp, dp, dp]),
        "orc_get_fields": (None, [vp, dp]),
        "orc_set_fields": (None, [vp, dp]),
        "orc_get_current": (None, [vp, dp]),
        "orc_set_current": (None, [vp, dp]),
        "orc_get_rho_static": (None, [vp, dp]),
        "orc_set_rho_static": (None, [vp, dp]),
        "orc_gather": (None, [vp, dp, dp]),
        "orc_filter_current": (None, [vp]),
        "orc_boris": (None, [d, dp, dp, dp]),
        "orc_deposit_into": (None, [vp, dp, dp, d, d]),
        "orc_zero_current": (None, [vp]),
        "orc_damp_current": (None, [vp]),
        "orc_advance_B": (None, [vp, d]),
        "orc_advance_E": (None, [vp, d]),
        "orc_step": (None, [vp, i]),
        "orc_diagnose": (None, [vp, dp]),
        "orc_rho": (None, [vp, dp]),
        "orc_get_lambda": (None, [vp, dp]),
        "orc_path_sigma": (d, [vp, dp, dp, d]),
        "orc_set_conductor": (i, [vp, P(C.c_ubyte)]),
        "orc_sample_in_conductor": (i, [vp, i, i, i, i]),
        "orc_set_source": (i, [vp, l, dp, dp, dp, i]),
        "orc_slab_moments": (None, [vp, i, i, dp, dp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    return L


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _pad3(X) -> np.ndarray:
    v = np.zeros(3)
    a = np.asarray(X, dtype=np.float64).reshape(-1)
    v[: len(a)] = a
    return v


def _lp(a: np.ndarray):
    assert a.dtype == np.int64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_long))


def shape(order: int, d: float) -> float:
    """Centred B-spline shape factor of the given order at distance d (cells)."""
    return lib().orc_shape(order, float(d))


def boris(qdt_2m: float, E, B, u) -> np.ndarray:
    """One relativistic Boris update of u = gamma v in fields E, B."""
    E = np.ascontiguousarray(E, dtype=np.float64)
    B = np.ascontiguousarray(B, dtype=np.float64)
    uu = np.array(u, dtype=np.float64)
    lib().orc_boris(float(qdt_2m), _dp(E), _dp(B), _dp(uu))
    return uu


def make_params(cfg) -> OrcParams:
    p = OrcParams()
    p.dim = int(cfg.dim)
    for d in range(3):
        p.n[d] = int(cfg.n[d]) if d < cfg.dim else 0
        p.pml[d][0] = int(cfg.pml[d][0]) if d < cfg.dim else 0
        p.pml[d][1] = int(cfg.pml[d][1]) if d < cfg.dim else 0
        p.dx[d] = float(cfg.dx[d]) if d < cfg.dim else 1.0
    p.dt = float(cfg.dt)
    p.shape_order = int(cfg.shape_order)
    p.alpha_mode = int(cfg.alpha_mode)
    p.damping_scale = float(cfg.damping_scale)
    coef = np.zeros((3, 16))
    for d, row in enumerate(cfg.sigma_coef):
        coef[d, : len(row)] = row
    p.n_sigma_coef = 16
    for d in range(3):
        for k in range(16):
            p.sigma_coef[d][k] = coef[d, k]
    p.push = int(cfg.push)
    p.charge = float(cfg.charge)
    p.mass = float(cfg.mass)
    p.solver = int(getattr(cfg, "solver", 0))
    p.filter_passes = int(getattr(cfg, "filter_passes", 0))
    faces = getattr(cfg, "alpha_face", ((0, 0), (0, 0), (0, 0)))
    for d in range(3):
        for side in range(2):
            p.alpha_face[d][side] = int(faces[d][side])
    return p


class OracleSim:
    """Plain FP64 simulation (split fields everywhere, absolute grid coordinates)."""

    def __init__(self, cfg, parallel: bool = False):
        """parallel: the all-cores build (OpenMP over cell loops and particles, per-thread
        current buffers summed in thread order); the same arithmetic up to the order of
        the current sums."""
        self.cfg = cfg
        self._L = lib_parallel() if parallel else lib()
        self._p = make_params(cfg)
        self._h = self._L.orc_create(C.byref(self._p))
        if not self._h:
            raise ValueError("oracle: invalid parameters")
        self.dim = int(cfg.dim)
        self.M = [int(cfg.n[d]) + int(cfg.pml[d][0]) + int(cfg.pml[d][1]) if d < cfg.dim else 0
                  for d in range(3)]
        self.nn = [m + 1 if d < cfg.dim else 1 for d, m in enumerate(self.M)]
        self.nsamp = int(self._L.orc_num_samples(self._h))

    def __del__(self):
        h = getattr(self, "_h", None)
        L = getattr(self, "_L", None)
        if h and L is not None:
            L.orc_destroy(h)
            self._h = None

    # ---- particles
    def add_particles(self, x, u, w):
        x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, self.dim)
        u = np.ascontiguousarray(u, dtype=np.float64).reshape(-1, 3)
        w = np.ascontiguousarray(w, dtype=np.float64).reshape(-1)
        self._L.orc_add_particles(self._h, len(w), _dp(x), _dp(u), _dp(w))

    def set_particles(self, ids, X, u, w):
        ids = np.ascontiguousarray(ids, dtype=np.int64)
        X = np.ascontiguousarray(X, dtype=np.float64).reshape(-1, 3)
        u = np.ascontiguousarray(u, dtype=np.float64).reshape(-1, 3)
        w = np.ascontiguousarray(w, dtype=np.float64).reshape(-1)
        self._L.orc_set_particles(self._h, len(w), _lp(ids), _dp(X), _dp(u), _dp(w))

    def set_conductor(self, cells):
        """Conductor cells: uint8 array of shape (M_z, M_y, M_x) (cells including the PML),
        nonzero = conductor; the fields inside are zeroed now and after every update."""
        if cells is None:
            rc = self._L.orc_set_conductor(self._h, None)
        else:
            c = np.ascontiguousarray(cells, dtype=np.uint8).reshape(self.M[2], self.M[1], self.M[0])
            self._cond = c
            rc = self._L.orc_set_conductor(self._h, c.ctypes.data_as(C.POINTER(C.c_ubyte)))
        if rc:
            raise ValueError("oracle: conductors are 3D")

    def sample_in_conductor(self, comp, i, j, k) -> bool:
        return bool(self._L.orc_sample_in_conductor(self._h, int(comp), int(i), int(j), int(k)))

    def set_source(self, x, u, w, axis=2):
        """Beam source: particles at the present time (physical x, u, w) injected when their
        ballistic path reaches the outer wall of the low layer of `axis`."""
        x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, self.dim)
        u = np.ascontiguousarray(u, dtype=np.float64).reshape(-1, 3)
        w = np.ascontiguousarray(w, dtype=np.float64).reshape(-1)
        if self._L.orc_set_source(self._h, len(w), _dp(x), _dp(u), _dp(w), int(axis)):
            raise ValueError("oracle: a source particle never enters the box")

    def slab_moments(self, axis, edges) -> np.ndarray:
        """(nslab, 5): count, sum w, sum w u_x, sum w u_y, sum w u_z per slab of `axis`."""
        e = np.ascontiguousarray(edges, dtype=np.float64)
        out = np.zeros((len(e) - 1, 5))
        self._L.orc_slab_moments(self._h, int(axis), len(e) - 1, _dp(e), _dp(out))
        return out

    @property
    def num_particles(self) -> int:
        return int(self._L.orc_num_particles(self._h))

    @property
    def step_count(self) -> int:
        return int(self._L.orc_step_count(self._h))

    def particles(self):
        """(ids, X grid coordinates n x 3, u n x 3, w n)."""
        n = self.num_particles
        ids = np.zeros(n, np.int64)
        X = np.zeros((n, 3))
        u = np.zeros((n, 3))
        w = np.zeros(n)
        if n:
            self._L.orc_get_particles(self._h, _lp(ids), _dp(X), _dp(u), _dp(w))
        return ids, X, u, w

    def lam(self) -> np.ndarray:
        """Per particle (order of particles()): the integral of sigma/eps0 over time
        along its path, whose exponential damps its weight in alpha mode 3."""
        n = self.num_particles
        out = np.zeros(n)
        if n:
            self._L.orc_get_lambda(self._h, _dp(out))
        return out

    def path_sigma(self, X0, X1, tau: float) -> float:
        """Integral of sigma/eps0 over time along the straight move X0 -> X1 (grid
        coordinates) taking tau."""
        return self._L.orc_path_sigma(self._h, _dp(_pad3(X0)), _dp(_pad3(X1)), float(tau))

    # ---- fields
    def _shape(self):
        return (self.nn[2], self.nn[1], self.nn[0])

    def split_fields(self) -> np.ndarray:
        """(12, nz, ny, nx) split parts in the order of PART_NAMES."""
        out = np.zeros((NPARTS, self.nsamp))
        self._L.orc_get_fields(self._h, _dp(out))
        return out.reshape((NPARTS,) + self._shape())

    def set_split_fields(self, F: np.ndarray):
        F = np.ascontiguousarray(F, dtype=np.float64).reshape(NPARTS, self.nsamp)
        self._L.orc_set_fields(self._h, _dp(F))

    def fields(self) -> np.ndarray:
        """(6, nz, ny, nx) totals Ex Ey Ez Bx By Bz (Eq. MaxwellSum)."""
        F = self.split_fields()
        return F[0::2] + F[1::2]

    def current(self) -> np.ndarray:
        out = np.zeros((3, self.nsamp))
        self._L.orc_get_current(self._h, _dp(out))
        return out.reshape((3,) + self._shape())

    def set_current(self, J):
        J = np.ascontiguousarray(J, dtype=np.float64).reshape(3, self.nsamp)
        self._L.orc_set_current(self._h, _dp(J))

    def rho_static(self):
        out = np.zeros(self.nsamp)
        self._L.orc_get_rho_static(self._h, _dp(out))
        return out.reshape(self._shape())

    def set_rho_static(self, r):
        r = np.ascontiguousarray(r, dtype=np.float64).reshape(-1)
        self._L.orc_set_rho_static(self._h, _dp(r))

    def rho(self):
        out = np.zeros(self.nsamp)
        self._L.orc_rho(self._h, _dp(out))
        return out.reshape(self._shape())

    # ---- phases
    def gather(self, X) -> np.ndarray:
        X = _pad3(X)
        out = np.zeros(6)
        self._L.orc_gather(self._h, _dp(X), _dp(out))
        return out

    def deposit(self, X0, X1, vz, qw):
        X0 = _pad3(X0)
        X1 = _pad3(X1)
        self._L.orc_deposit_into(self._h, _dp(X0), _dp(X1), float(vz), float(qw))

    def zero_current(self):
        self._L.orc_zero_current(self._h)

    def damp_current(self):
        self._L.orc_damp_current(self._h)

    def filter_current(self):
        """filter_passes binomial passes over the current (App. A)"""
        self._L.orc_filter_current(self._h)

    def advance_B(self, tau):
        self._L.orc_advance_B(self._h, float(tau))

    def advance_E(self, tau):
        self._L.orc_advance_E(self._h, float(tau))

    def step(self, n: int = 1):
        self._L.orc_step(self._h, int(n))

    def sigma(self, d: int, X: float) -> float:
        return self._L.orc_sigma(self._h, d, float(X))

    def alpha_axis(self, d: int, X: float) -> float:
        return self._L.orc_alpha_axis(self._h, d, float(X))

    def alpha(self, X) -> float:
        X = _pad3(X)
        return self._L.orc_alpha(self._h, _dp(X))

    def diagnose(self) -> dict:
        out = np.zeros(7)
        self._L.orc_diagnose(self._h, _dp(out))
        return {"u_interior": out[0], "u_pml": out[1], "gauss_max": out[2],
                "gauss_l2": out[3], "rho_max": out[4], "n_particles": int(out[5]),
                "step": int(out[6])}


# ---------------------------------------------------------------- reference gradient
# Parameters of the PML: the per-axis conductivity polynomial sigma/eps0 = sum_k
# a_{d,k} (depth/L)^k (16 coefficients per axis, Sec. II.C and Sec. III) and the scale s
# of the current damping alpha = exp(-s Phi) (Sec. II.C), packed as
# (a_{0,0..15}, ..., a_{dim-1,0..15}, s).

def theta_vector(cfg) -> np.ndarray:
    th = np.zeros(16 * cfg.dim + 1)
    for d in range(cfg.dim):
        row = list(cfg.sigma_coef[d])
        th[16 * d:16 * d + len(row)] = row
    th[-1] = cfg.damping_scale
    return th


def with_theta(cfg, theta):
    import dataclasses
    th = np.asarray(theta, dtype=np.float64)
    rows = [tuple(th[16 * d:16 * d + 16]) for d in range(cfg.dim)]
    rows += [tuple(cfg.sigma_coef[d]) for d in range(cfg.dim, 3)]
    return dataclasses.replace(cfg, sigma_coef=tuple(rows), damping_scale=float(th[-1]))


def interior_energy(cfg, x, u, w, n_steps: int, fields=None) -> float:
    """Field energy inside the physical box after n_steps (the energy norm of Sec. III)."""
    o = OracleSim(cfg)
    if fields is not None:
        o.set_split_fields(fields)
    if len(w):
        o.add_particles(x, u, w)
    o.step(n_steps)
    return o.diagnose()["u_interior"]


def fd_gradient(cfg, x, u, w, n_steps: int, idx=None, rel_h: float = 1e-3) -> np.ndarray:
    """dU/dtheta by central differences, Richardson-extrapolated from steps h and h/2
    (truncation O(h^4)); h = rel_h * max(|theta_i|, 0.1).  Entries not in idx are NaN."""
    th0 = theta_vector(cfg)
    idx = range(th0.size) if idx is None else idx
    g = np.full(th0.size, np.nan)

    def U(th):
        return interior_energy(with_theta(cfg, th), x, u, w, n_steps)

    for i in idx:
        h = rel_h * max(abs(th0[i]), 0.1)
        D = []
        for hh in (h, 0.5 * h):
            tp, tm = th0.copy(), th0.copy()
            tp[i] += hh
            tm[i] -= hh
            D.append((U(tp) - U(tm)) / (2.0 * hh))
        g[i] = (4.0 * D[1] - D[0]) / 3.0
    return g
