"""Thin ctypes binding of the C ABI in include/pml_pic.h.

Argument marshalling only: every step of the particle-in-cell path runs in the HIP
kernels of libpmlpic.so.  PyTorch provides the device workspace (one uint8 tensor)
and the stream.  There is no CPU fallback: if the library or a GPU is missing,
constructing a simulation raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# PMLPIC_LIB may name another build of the library (the bounds-checked libpmlpic_check.so)
LIB_PATH = os.environ.get("PMLPIC_LIB") or os.path.join(HERE, "libpmlpic.so")

PML_PIC_OK = 0
PML_PIC_E_INVALID_ARG = -1
STATUS = {0: "OK", -1: "E_INVALID_ARG", -2: "E_CFL", -3: "E_WORKSPACE", -4: "E_HIP",
          -5: "E_NONFINITE", -6: "E_CAPACITY", -7: "E_HOST"}
FLAG_UNFUSED, FLAG_NO_SORT, FLAG_SEPARATE_DAMP, FLAG_KEEP_CURRENT, FLAG_SEPARATE_FIELDS = 1, 2, 4, 8, 16
FLAG_DETERMINISTIC = 32

EXPORTED = [
    "pml_pic_workspace_size", "pml_pic_create", "pml_pic_add_particles", "pml_pic_step",
    "pml_pic_diagnose", "pml_pic_grid_shape", "pml_pic_get_fields", "pml_pic_set_fields",
    "pml_pic_get_current", "pml_pic_get_rho_static", "pml_pic_set_rho_static",
    "pml_pic_num_particles", "pml_pic_get_particles", "pml_pic_set_particles",
    "pml_pic_last_error", "pml_pic_destroy", "pml_pic_step_profiled",
    "pml_pic_batch_workspace_size", "pml_pic_batch_create", "pml_pic_batch_run",
    "pml_pic_batch_set_launch", "pml_pic_batch_step", "pml_pic_batch_last_error",
    "pml_pic_batch_destroy", "pml_pic_batch_step_profiled", "pml_pic_forward_ckpt",
    "pml_pic_backward", "pml_pic_set_conductor", "pml_pic_set_source", "pml_pic_slab_moments",
    "pml_pic_field_error", "pml_pic_field_error_noalloc", "pml_pic_sort_particles",
    "pml_pic_particle_adjoint", "pml_pic_atomic_rates",
]
PHASES = ["sort_particles", "clear_current", "gather_push", "deposit_current", "damp_pml_current",
          "update_yee_pml_B", "update_yee_pml_E", "update_yee_pml", "filter_current"]


class Params(C.Structure):
    _fields_ = [
        ("dim", C.c_int32), ("n", C.c_int32 * 3), ("pml", (C.c_int32 * 2) * 3),
        ("dx", C.c_double * 3), ("dt", C.c_double), ("shape_order", C.c_int32),
        ("alpha_mode", C.c_int32), ("damping_scale", C.c_double), ("n_sigma_coef", C.c_int32),
        ("sigma_coef", (C.c_double * 16) * 3), ("precision", C.c_int32), ("push", C.c_int32),
        ("sort_interval", C.c_int32), ("tile", C.c_int32 * 3), ("max_particles", C.c_int64),
        ("charge", C.c_double), ("mass", C.c_double), ("flags", C.c_int32),
        ("adjoint_segment", C.c_int32), ("adjoint_checkpoints", C.c_int32),
        ("solver", C.c_int32), ("filter_passes", C.c_int32),
        ("alpha_face", (C.c_int32 * 2) * 3), ("conductor", C.c_int32), ("max_source", C.c_int64),
    ]


class Diag(C.Structure):
    _fields_ = [
        ("u_interior", C.c_double), ("u_pml", C.c_double), ("gauss_max", C.c_double),
        ("gauss_l2", C.c_double), ("rho_max", C.c_double), ("n_particles", C.c_int64),
        ("step", C.c_int64), ("n_pushes", C.c_int64), ("nonfinite", C.c_int32),
    ]


class PmlPicError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (STATUS.get(code, "?"), code, msg))
        self.code = code


_lib = None


def load_library():
    """Loads libpmlpic.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("%s is not built; run __graft_entry__.build()" % os.path.basename(LIB_PATH))
        L = C.CDLL(LIB_PATH)
        P = C.POINTER
        vp, i32, i64, dp = C.c_void_p, C.c_int32, C.c_int64, P(C.c_double)
        sig = {
            "pml_pic_workspace_size": (C.c_int, [P(Params), P(C.c_size_t)]),
            "pml_pic_create": (C.c_int, [P(Params), vp, C.c_size_t, vp, P(vp)]),
            "pml_pic_add_particles": (C.c_int, [vp, i64, dp, dp, dp]),
            "pml_pic_step": (C.c_int, [vp, i32]),
            "pml_pic_step_profiled": (C.c_int, [vp, i32, dp, P(C.c_int64)]),
            "pml_pic_diagnose": (C.c_int, [vp, P(Diag)]),
            "pml_pic_grid_shape": (C.c_int, [vp, P(C.c_int32), P(C.c_int64)]),
            "pml_pic_get_fields": (C.c_int, [vp, dp, i64]),
            "pml_pic_set_fields": (C.c_int, [vp, dp, i64]),
            "pml_pic_get_current": (C.c_int, [vp, dp, i64]),
            "pml_pic_get_rho_static": (C.c_int, [vp, dp, i64]),
            "pml_pic_set_rho_static": (C.c_int, [vp, dp, i64]),
            "pml_pic_num_particles": (C.c_int, [vp, P(C.c_int64)]),
            "pml_pic_get_particles": (C.c_int, [vp, i64, P(C.c_int64), dp, dp, dp, P(C.c_int64)]),
            "pml_pic_set_particles": (C.c_int, [vp, i64, P(C.c_int64), dp, dp, dp]),
            "pml_pic_last_error": (C.c_char_p, [vp]),
            "pml_pic_destroy": (None, [vp]),
            "pml_pic_batch_workspace_size": (C.c_int, [P(Params), i32, P(C.c_size_t)]),
            "pml_pic_batch_create": (C.c_int, [P(Params), i32, vp, C.c_size_t, vp, i32, P(vp)]),
            "pml_pic_batch_run": (vp, [vp, i32]),
            "pml_pic_batch_set_launch": (C.c_int, [vp, i32, i32]),
            "pml_pic_batch_step": (C.c_int, [vp, i32]),
            "pml_pic_batch_step_profiled": (C.c_int, [vp, i32, dp, P(C.c_int64)]),
            "pml_pic_batch_last_error": (C.c_char_p, [vp]),
            "pml_pic_batch_destroy": (None, [vp]),
            "pml_pic_forward_ckpt": (C.c_int, [vp, i32, dp]),
            "pml_pic_backward": (C.c_int, [vp, dp, i64, dp, dp, i32]),
            "pml_pic_particle_adjoint": (C.c_int, [vp, i64, dp, dp]),
            "pml_pic_set_conductor": (C.c_int, [vp, P(C.c_uint8)]),
            "pml_pic_set_source": (C.c_int, [vp, i64, dp, dp, dp, i32]),
            "pml_pic_slab_moments": (C.c_int, [vp, i32, i32, dp, dp]),
            "pml_pic_field_error": (C.c_int, [vp, vp, dp, dp]),
            "pml_pic_field_error_noalloc": (C.c_int, [vp, vp, dp, dp]),
            "pml_pic_sort_particles": (C.c_int, [vp, P(C.c_int32), P(C.c_uint32), i64, P(C.c_int64)]),
            "pml_pic_atomic_rates": (C.c_int, [dp]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def make_params(cfg, max_particles=None, flags=0, adjoint=(0, 0)) -> Params:
    """C parameter block from a workloads.SimConfig-like object."""
    p = Params()
    p.dim = int(cfg.dim)
    for d in range(3):
        p.n[d] = int(cfg.n[d]) if d < cfg.dim else 1
        p.pml[d][0] = int(cfg.pml[d][0]) if d < cfg.dim else 0
        p.pml[d][1] = int(cfg.pml[d][1]) if d < cfg.dim else 0
        p.dx[d] = float(cfg.dx[d]) if d < cfg.dim else 1.0
        p.tile[d] = int(cfg.tile[d]) if hasattr(cfg, "tile") else 0
    p.dt = float(cfg.dt)
    p.shape_order = int(cfg.shape_order)
    p.alpha_mode = int(cfg.alpha_mode)
    p.damping_scale = float(cfg.damping_scale)
    p.n_sigma_coef = 16
    for d, row in enumerate(cfg.sigma_coef):
        for k, v in enumerate(row):
            p.sigma_coef[d][k] = float(v)
    p.precision = int(cfg.precision)
    p.push = int(cfg.push)
    p.sort_interval = int(getattr(cfg, "sort_interval", 0))
    mp = max_particles if max_particles is not None else int(getattr(cfg, "max_particles", 0))
    p.max_particles = int(mp)
    p.charge = float(cfg.charge)
    p.mass = float(cfg.mass)
    p.flags = int(flags)
    p.adjoint_segment = int(adjoint[0])
    p.adjoint_checkpoints = int(adjoint[1])
    p.solver = int(getattr(cfg, "solver", 0))
    p.filter_passes = int(getattr(cfg, "filter_passes", 0))
    faces = getattr(cfg, "alpha_face", ((0, 0), (0, 0), (0, 0)))
    for d in range(3):
        for side in range(2):
            p.alpha_face[d][side] = int(faces[d][side])
    p.conductor = int(getattr(cfg, "conductor", 0))
    p.max_source = int(getattr(cfg, "max_source", 0))
    return p


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _lp(a):
    return a.ctypes.data_as(C.POINTER(C.c_int64))


def workspace_size(params: Params) -> int:
    n = C.c_size_t(0)
    rc = load_library().pml_pic_workspace_size(C.byref(params), C.byref(n))
    if rc != PML_PIC_OK:
        raise PmlPicError(rc, load_library().pml_pic_last_error(None).decode())
    return int(n.value)


def atomic_rates() -> dict:
    """pml_pic_atomic_rates on the current GPU: lane additions per second of FP64 / FP32
    atomic adds into LDS and into global memory (distinct consecutive addresses)."""
    r = (C.c_double * 4)()
    rc = load_library().pml_pic_atomic_rates(r)
    if rc != PML_PIC_OK:
        raise PmlPicError(rc, load_library().pml_pic_last_error(None).decode())
    return {"lds_f64": r[0], "lds_f32": r[1], "global_f32": r[2], "global_f64": r[3]}


class PmlPic:
    """One simulation on the current GPU (names follow the C ABI)."""

    def __init__(self, cfg, max_particles=None, flags=0, stream=None, _borrowed=None, adjoint=(0, 0)):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("PmlPic needs a ROCm GPU; there is no CPU fallback")
        L = load_library()
        self.cfg = cfg
        self.params = make_params(cfg, max_particles, flags, adjoint)
        if _borrowed is not None:        # a run owned by a PmlPicBatch
            self._h, self._owned, self.stream = C.c_void_p(_borrowed), False, stream
            self._init_shape()
            return
        self._owned = True
        nbytes = workspace_size(self.params)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
        base = self.workspace.data_ptr()
        aligned = (base + 255) // 256 * 256
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = C.c_void_p()
        rc = L.pml_pic_create(C.byref(self.params), C.c_void_p(aligned), C.c_size_t(nbytes),
                              C.c_void_p(self.stream.cuda_stream), C.byref(h))
        if rc != PML_PIC_OK:
            raise PmlPicError(rc, L.pml_pic_last_error(None).decode())
        self._h = h
        self._init_shape()

    def _init_shape(self):
        L = load_library()
        nn = (C.c_int32 * 3)()
        ns = C.c_int64()
        self._check(L.pml_pic_grid_shape(self._h, nn, C.byref(ns)))
        self.nn = [int(nn[0]), int(nn[1]), int(nn[2])]
        self.nsamp = int(ns.value)

    def _check(self, rc):
        if rc != PML_PIC_OK:
            raise PmlPicError(rc, load_library().pml_pic_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            if getattr(self, "_owned", True):
                load_library().pml_pic_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------- particles
    def add_particles(self, x, u, w):
        x = np.ascontiguousarray(x, dtype=np.float64)
        u = np.ascontiguousarray(u, dtype=np.float64)
        w = np.ascontiguousarray(w, dtype=np.float64)
        self._check(load_library().pml_pic_add_particles(self._h, len(w), _dp(x), _dp(u), _dp(w)))

    def set_conductor(self, cells):
        """Conductor cells: uint8 array of shape (M_z, M_y, M_x), nonzero = conductor (None
        removes them)."""
        L = load_library()
        if cells is None:
            self._check(L.pml_pic_set_conductor(self._h, None))
            return
        M = [self.nn[d] - 1 for d in range(3)]
        c = np.ascontiguousarray(cells, dtype=np.uint8).reshape(M[2], M[1], M[0])
        self._check(L.pml_pic_set_conductor(self._h, c.ctypes.data_as(C.POINTER(C.c_uint8))))

    def set_source(self, x, u, w, axis=2):
        """Beam source: particles at the present time, injected when their ballistic path
        reaches the outer wall of the low layer of `axis`."""
        x = np.ascontiguousarray(x, dtype=np.float64)
        u = np.ascontiguousarray(u, dtype=np.float64)
        w = np.ascontiguousarray(w, dtype=np.float64)
        self._check(load_library().pml_pic_set_source(self._h, len(w), _dp(x), _dp(u), _dp(w), int(axis)))

    def sort_particles(self):
        """Sorts the particles now; returns (tile shape, key_start of n_keys + 1 entries:
        the first slot of every key, then the particle count)."""
        L = load_library()
        tile = (C.c_int32 * 3)()
        nk = C.c_int64()
        self._check(L.pml_pic_sort_particles(self._h, tile, None, 0, C.byref(nk)))
        ks = np.zeros(int(nk.value) + 1, dtype=np.uint32)
        self._check(L.pml_pic_sort_particles(self._h, tile, ks.ctypes.data_as(C.POINTER(C.c_uint32)), ks.size,
                                             C.byref(nk)))
        return (int(tile[0]), int(tile[1]), int(tile[2])), ks

    def field_error(self, ref) -> float:
        """Eq. (error) against the reference run `ref` over this run's physical box."""
        num, den = self.field_error_sums(ref)
        return num / den if den > 0 else num

    def field_error_sums(self, ref, noalloc=False):
        """(sum (F - F_ref)^2, sum F_ref^2) of Eq. (error); noalloc: through
        pml_pic_field_error_noalloc (partials in the library's static device scratch)."""
        num, den = C.c_double(), C.c_double()
        L = load_library()
        f = L.pml_pic_field_error_noalloc if noalloc else L.pml_pic_field_error
        self._check(f(self._h, ref._h, C.byref(num), C.byref(den)))
        return num.value, den.value

    def slab_moments(self, axis, edges) -> np.ndarray:
        """(nslab, 5): count, sum w, sum w u_x, sum w u_y, sum w u_z per slab of `axis`."""
        e = np.ascontiguousarray(edges, dtype=np.float64)
        out = np.zeros((len(e) - 1, 5))
        self._check(load_library().pml_pic_slab_moments(self._h, int(axis), len(e) - 1, _dp(e), _dp(out)))
        return out

    def set_particles(self, ids, X, u, w):
        ids = np.ascontiguousarray(ids, dtype=np.int64)
        X = np.ascontiguousarray(X, dtype=np.float64).reshape(-1, 3)
        u = np.ascontiguousarray(u, dtype=np.float64).reshape(-1, 3)
        w = np.ascontiguousarray(w, dtype=np.float64)
        self._check(load_library().pml_pic_set_particles(self._h, len(w), _lp(ids), _dp(X), _dp(u), _dp(w)))

    def particles(self, cap=None, device_order=False):
        """(ids, X grid coordinates n x 3, u n x 3, w) of the live particles, sorted by id
        (device_order: in their order on the device)."""
        if cap is None:
            cap = max(1, int(self.params.max_particles))
        ids = np.zeros(cap, np.int64)
        X = np.zeros((cap, 3))
        u = np.zeros((cap, 3))
        w = np.zeros(cap)
        n = C.c_int64()
        self._check(load_library().pml_pic_get_particles(self._h, cap, _lp(ids), _dp(X), _dp(u), _dp(w),
                                                         C.byref(n)))
        n = int(n.value)
        if device_order:
            return ids[:n], X[:n], u[:n], w[:n]
        o = np.argsort(ids[:n], kind="stable")
        return ids[:n][o], X[:n][o], u[:n][o], w[:n][o]

    @property
    def num_particles(self) -> int:
        n = C.c_int64()
        self._check(load_library().pml_pic_num_particles(self._h, C.byref(n)))
        return int(n.value)

    # ---------------------------------------------------------------- stepping
    def step(self, n: int = 1):
        self._check(load_library().pml_pic_step(self._h, int(n)))

    def step_profiled(self, n: int = 1):
        """Steps with HIP events around every kernel phase: {phase: (total ms, launches)}."""
        ms = np.zeros(len(PHASES))
        calls = np.zeros(len(PHASES), np.int64)
        self._check(load_library().pml_pic_step_profiled(self._h, int(n), _dp(ms), _lp(calls)))
        return {PHASES[k]: (float(ms[k]), int(calls[k])) for k in range(len(PHASES)) if calls[k] > 0}

    # ---------------------------------------------------------------- adjoint
    def forward_ckpt(self, n: int) -> float:
        """n steps keeping checkpoints; returns the interior field energy after them."""
        U = C.c_double()
        self._check(load_library().pml_pic_forward_ckpt(self._h, int(n), C.byref(U)))
        return float(U.value)

    def backward(self, seed=None, want_lambda=False):
        """Reverse pass of the last forward_ckpt.  seed: None (interior energy) or a
        12-part array shaped like split_fields().  Returns (grad_theta, lambda or None)."""
        L = load_library()
        n_theta = 16 * int(self.params.dim) + 1
        grad = np.zeros(n_theta)
        lam = np.zeros(12 * self.nsamp) if want_lambda else None
        if seed is not None:
            seed = np.ascontiguousarray(seed, dtype=np.float64).reshape(-1)
            sp, sc = _dp(seed), seed.size
        else:
            sp, sc = None, 0
        self._check(L.pml_pic_backward(self._h, sp, sc, _dp(lam) if lam is not None else None, _dp(grad),
                                       n_theta))
        return grad, (lam.reshape((12,) + self._shape()) if lam is not None else None)

    def particle_adjoint(self, n: int):
        """After backward() of a pushed run: (dU/dx of shape (n, dim) in the physical
        coordinates of add_particles, dU/du of shape (n, 3)) for particle ids 0..n-1."""
        dim = int(self.params.dim)
        gx = np.zeros(n * dim)
        gu = np.zeros(n * 3)
        self._check(load_library().pml_pic_particle_adjoint(self._h, int(n), _dp(gx), _dp(gu)))
        return gx.reshape(n, dim), gu.reshape(n, 3)

    def diagnose(self, allow_nonfinite=False) -> dict:
        d = Diag()
        rc = load_library().pml_pic_diagnose(self._h, C.byref(d))
        if rc != PML_PIC_OK and not (allow_nonfinite and rc == -5):
            self._check(rc)
        return {k: getattr(d, k) for k, _ in Diag._fields_}

    # ---------------------------------------------------------------- fields
    def _shape(self):
        return (self.nn[2], self.nn[1], self.nn[0])

    def split_fields(self) -> np.ndarray:
        out = np.zeros(12 * self.nsamp)
        self._check(load_library().pml_pic_get_fields(self._h, _dp(out), out.size))
        return out.reshape((12,) + self._shape())

    def set_split_fields(self, F):
        F = np.ascontiguousarray(F, dtype=np.float64).reshape(-1)
        self._check(load_library().pml_pic_set_fields(self._h, _dp(F), F.size))

    def fields(self) -> np.ndarray:
        F = self.split_fields()
        return F[0::2] + F[1::2]

    def current(self) -> np.ndarray:
        out = np.zeros(3 * self.nsamp)
        self._check(load_library().pml_pic_get_current(self._h, _dp(out), out.size))
        return out.reshape((3,) + self._shape())

    def rho_static(self) -> np.ndarray:
        out = np.zeros(self.nsamp)
        self._check(load_library().pml_pic_get_rho_static(self._h, _dp(out), out.size))
        return out.reshape(self._shape())

    def set_rho_static(self, r):
        r = np.ascontiguousarray(r, dtype=np.float64).reshape(-1)
        self._check(load_library().pml_pic_set_rho_static(self._h, _dp(r), r.size))


def batch_workspace_size(params_list) -> int:
    arr = (Params * len(params_list))(*params_list)
    n = C.c_size_t(0)
    rc = load_library().pml_pic_batch_workspace_size(arr, len(params_list), C.byref(n))
    if rc != PML_PIC_OK:
        raise PmlPicError(rc, load_library().pml_pic_batch_last_error(None).decode())
    return int(n.value)


class PmlPicBatch:
    """Many independent runs stepped together (pml_pic_batch_*).  ``runs[r]`` is a PmlPic
    view of run r (owned by the batch).  Uses its own torch stream so that the step can
    be captured as a HIP graph."""

    def __init__(self, cfgs, particles_per_run=1, use_graph=True, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("PmlPicBatch needs a ROCm GPU; there is no CPU fallback")
        L = load_library()
        self.cfgs = list(cfgs)
        caps = particles_per_run if isinstance(particles_per_run, (list, tuple)) else [particles_per_run] * len(cfgs)
        self.params = [make_params(c, max_particles=m) for c, m in zip(self.cfgs, caps)]
        arr = (Params * len(self.params))(*self.params)
        nbytes = batch_workspace_size(self.params)
        self.stream = stream if stream is not None else torch.cuda.Stream()
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
        aligned = (self.workspace.data_ptr() + 255) // 256 * 256
        h = C.c_void_p()
        rc = L.pml_pic_batch_create(arr, len(self.params), C.c_void_p(aligned), C.c_size_t(nbytes),
                                    C.c_void_p(self.stream.cuda_stream), int(bool(use_graph)), C.byref(h))
        if rc != PML_PIC_OK:
            raise PmlPicError(rc, L.pml_pic_batch_last_error(None).decode())
        self._h = h
        self.runs = [PmlPic(c, max_particles=m, stream=self.stream,
                            _borrowed=L.pml_pic_batch_run(self._h, r))
                     for r, (c, m) in enumerate(zip(self.cfgs, caps))]
        self.launch = (64, 0)

    def _check(self, rc):
        if rc != PML_PIC_OK:
            raise PmlPicError(rc, load_library().pml_pic_batch_last_error(self._h).decode())

    def step(self, n: int = 1):
        self._check(load_library().pml_pic_batch_step(self._h, int(n)))

    def step_profiled(self, n: int = 1):
        """Eager steps with HIP events around every kernel: {phase: (total ms, launches)}."""
        ms = np.zeros(len(PHASES))
        calls = np.zeros(len(PHASES), np.int64)
        self._check(load_library().pml_pic_batch_step_profiled(self._h, int(n), _dp(ms), _lp(calls)))
        return {PHASES[k]: (float(ms[k]), int(calls[k])) for k in range(len(PHASES)) if calls[k] > 0}

    def set_launch(self, block_x: int, grid_blocks: int = 0):
        self._check(load_library().pml_pic_batch_set_launch(self._h, int(block_x), int(grid_blocks)))
        self.launch = (block_x, grid_blocks)

    def synchronize(self):
        self.stream.synchronize()

    def timed_steps(self, n: int) -> float:
        """Seconds for n steps, from HIP events recorded on the batch's stream."""
        import torch
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(self.stream)
        self.step(n)
        b.record(self.stream)
        b.synchronize()
        return a.elapsed_time(b) / 1e3

    def close(self):
        if getattr(self, "_h", None):
            for r in self.runs:
                r._h = None
            load_library().pml_pic_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
