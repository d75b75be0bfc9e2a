/*
 * pml_pic.h -- C ABI of the MI355X (gfx950) damped-current PML particle-in-cell step.
 *
 * Method: Lehe, Blelly, Giacomel, Jambunathan, Vay, "Absorption of charged particles
 * in Perfectly-Matched-Layers by optimal damping of the deposited current".
 *   - split-field Maxwell equations with the source -alpha j/eps0 in the PML:
 *     Sec. II.A, Eqs. (MaxwellE), (MaxwellB), (MaxwellSum);
 *   - damping coefficient alpha(z) = exp(-int_0^z sigma/(eps0 v) dz'): Sec. II.A,
 *     Eq. (alpha), evaluated in closed form at nodes and cell centres (Sec. II.B);
 *   - alpha = 0 (standard PML) and alpha = 1 (undamped deposition) comparison
 *     schemes: Sec. I, Fig. 1 caption;
 *   - Yee FDTD, Esirkepov charge-conserving deposition with B-spline shapes,
 *     motionless opposite-charge partner, E = B = 0 at t = 0: Sec. II.B, App. A.
 *
 * Units are normalised: c = eps0 = mu0 = 1.  Node i along axis d sits at physical
 * coordinate (i - pml[d][0]) * dx[d]; the physical box is [0, n[d] dx[d]] and the PML
 * lies outside it, closed by PEC walls (tangential E = 0).  In 2D the grid is the x-y
 * plane and fields/momenta keep all three components (2D3V).
 *
 * Memory ownership: the caller allocates ONE device buffer of at least
 * pml_pic_workspace_size() bytes (256-byte aligned) and a HIP stream, and passes both
 * to pml_pic_create.  The calls of a simulation never allocate device memory (only the
 * measurement aid pml_pic_atomic_rates allocates, and frees, buffers of its own); the
 * handle borrows the buffer and the stream, which must outlive it.  Host arrays passed to the calls
 * below are read or written before the call returns (the call synchronises the
 * stream when it copies to or from the host) and stay owned by the caller.
 *
 * Errors: every call returns a pml_pic_status; no C++ exception crosses the ABI (one
 * thrown inside a call, e.g. std::bad_alloc from a host buffer sized by the caller's
 * arguments, is caught there and returned as PML_PIC_E_HOST with a message).
 * pml_pic_last_error() gives a message for the last failure on a handle.  A handle is
 * used by one host thread at a time.  Particles that leave through the outer PEC walls
 * are removed and counted; that is not an error.
 */
#ifndef PML_PIC_H
#define PML_PIC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PML_PIC_OK = 0,
    PML_PIC_E_INVALID_ARG = -1,   /* bad parameter, size or pointer */
    PML_PIC_E_CFL = -2,           /* c dt >= 1/sqrt(sum_d 1/dx_d^2) */
    PML_PIC_E_WORKSPACE = -3,     /* workspace smaller than pml_pic_workspace_size or misaligned */
    PML_PIC_E_HIP = -4,           /* a HIP runtime call failed (message has the HIP error) */
    PML_PIC_E_NONFINITE = -5,     /* pml_pic_diagnose found NaN/Inf in the fields */
    PML_PIC_E_CAPACITY = -6,      /* more particles than max_particles */
    PML_PIC_E_HOST = -7           /* host-side failure: out of host memory, or another C++
                                     exception caught at the ABI (the message says which) */
} pml_pic_status;

/* current-damping scheme in the PML (the alpha of Eq. MaxwellE) */
enum {
    PML_ALPHA_ZERO = 0,    /* alpha = 0 in the PML: no current there (standard PML)          */
    PML_ALPHA_ONE = 1,     /* alpha = 1: undamped current                                      */
    PML_ALPHA_DAMPED = 2,  /* Eq. (alpha) at each current sample, assumed velocity 1/damping_scale */
    PML_ALPHA_WEIGHT = 3   /* alpha = 1 in the field equations; instead each particle's weight is
                              damped by exp(-int sigma/eps0 dt) along its own path (Sec. II.C,
                              discussion of the velocity limitation) */
};

/* pml_pic_params.flags */
enum {
    PML_PIC_FLAG_UNFUSED = 1,      /* gather_push and deposit_current as separate launches */
    PML_PIC_FLAG_NO_SORT = 2,      /* never sort; deposit with global atomics only */
    PML_PIC_FLAG_SEPARATE_DAMP = 4,/* damp_pml_current as its own pass over the PML */
    PML_PIC_FLAG_KEEP_CURRENT = 8, /* keep J after the step (for pml_pic_get_current); by
                                      default the E update consumes J and zeroes it */
    PML_PIC_FLAG_SEPARATE_FIELDS = 16,/* update_yee_pml as three sweeps (B half, E, B half);
                                      by default 2D runs make one pass over the fields,
                                      which keeps J after the step */
    PML_PIC_FLAG_DETERMINISTIC = 32 /* debug mode: implies UNFUSED and NO_SORT, and one thread
                                      adds the particles' currents in slot order with plain
                                      loads and stores, so that a run repeats bit for bit and
                                      equals the atomic deposit to rounding (slow: meant for
                                      runs of a few thousand particles; single runs only) */
};

typedef struct {
    int32_t dim;                /* 2 (x-y plane, 2D3V) or 3 */
    int32_t n[3];               /* physical cells per axis (ignored beyond dim).  Limits, with
                                   M = n + both PML thicknesses: 2D M <= 65533 per axis and
                                   (M_x + 9 rounded up to 64) (M_y + 9) < 2^31 samples; 3D
                                   M <= 2045, 2045, 1021; the grid rounded up to whole sort
                                   tiles < 2^31 cells */
    int32_t pml[3][2];          /* PML cells per axis, low / high face; 0 = bare PEC wall */
    double dx[3];               /* cell sizes */
    double dt;                  /* time step; c dt < 1/sqrt(sum 1/dx_d^2) (Yee), c dt <= dx (CK) */
    int32_t shape_order;        /* particle shape: 1 linear, 2 quadratic, 3 cubic */
    int32_t alpha_mode;         /* PML_ALPHA_ZERO / ONE / DAMPED / WEIGHT */
    double damping_scale;       /* 1/v of Eq. (alpha): alpha = exp(-damping_scale * int sigma/eps0) */
    int32_t n_sigma_coef;       /* K <= 16 */
    double sigma_coef[3][16];   /* sigma_d/eps0 = sum_k coef[d][k] (depth/L_d)^k, depth > 0 */
    int32_t precision;          /* 32 (fields and particles in FP32) or 64 */
    int32_t push;               /* 1: gather + Boris push; 0: momenta held fixed (ballistic) */
    int32_t sort_interval;      /* steps between particle sorts; 0 = default */
    int32_t tile[3];            /* deposit tile in cells; 0 = default */
    int64_t max_particles;      /* particle capacity of the workspace */
    double charge, mass;        /* species charge and mass per unit weight */
    int32_t flags;              /* PML_PIC_FLAG_* */
    int32_t adjoint_segment;    /* steps per checkpoint segment of the adjoint; 0 = no adjoint storage */
    int32_t adjoint_checkpoints;/* checkpoints kept by pml_pic_forward_ckpt (segments per run) */
    int32_t solver;             /* PML_PIC_SOLVER_YEE, or PML_PIC_SOLVER_CK: the Cole-Karkkainen
                                   solver the paper's single-particle runs use (App. A): 3D,
                                   cubic cells, c dt <= dx; Faraday's law takes the Yee
                                   difference averaged over its transverse neighbours with
                                   weights 7/12 (itself), 1/12 (the four side neighbours), 1/48
                                   (the four diagonal ones); Ampere's law stays Yee */
    int32_t filter_passes;      /* 3D: passes of the binomial filter (App. A) over the deposited
                                   current before the field update: each sample becomes the
                                   (1/4, 1/2, 1/4)^3-weighted sum of its 27 neighbours (samples
                                   outside the component's extent count as 0); 0..4 */
    int32_t alpha_face[3][2];   /* per-face damping mode (low / high side of each axis):
                                   0 = alpha_mode; 1 + PML_ALPHA_ZERO / ONE / DAMPED for that
                                   face's layer.  The paper's suggestion for a beam entering
                                   through one PML and leaving through the other (end of Sec.
                                   IV.A): undamped where it enters, Eq. (alpha) where it
                                   leaves.  A sample in an edge or corner takes the product of
                                   its faces' factors.  Not with PML_ALPHA_WEIGHT. */
    int32_t conductor;          /* 1: reserve a conductor mask (pml_pic_set_conductor); 3D */
    int64_t max_source;         /* capacity of the beam source (pml_pic_set_source), particles */
} pml_pic_params;

enum { PML_PIC_SOLVER_YEE = 0, PML_PIC_SOLVER_CK = 1 };

typedef struct {
    double u_interior;   /* 1/2 sum (E^2 + B^2) dV over samples inside the physical box (FP64 sum) */
    double u_pml;        /* same over the remaining samples */
    double gauss_max;    /* max |div E - rho| over nodes strictly inside the physical box */
    double gauss_l2;     /* RMS of the same residual */
    double rho_max;      /* max |rho| of the live particles (partners excluded) */
    int64_t n_particles; /* live particles */
    int64_t step;        /* steps taken */
    int64_t n_pushes;    /* particle pushes performed since creation */
    int32_t nonfinite;   /* 1 if a field value is NaN or Inf */
} pml_pic_diag;

typedef struct pml_pic_handle pml_pic_handle;

/* Bytes of device workspace needed for these parameters.  Validates them first
 * (returns PML_PIC_E_INVALID_ARG or PML_PIC_E_CFL on bad input). */
int pml_pic_workspace_size(const pml_pic_params *params, size_t *bytes);

/* Creates a simulation on the current HIP device.  device_workspace: caller-owned
 * device buffer of `bytes` bytes, 256-byte aligned; stream: a hipStream_t (may be
 * NULL for the default stream).  Fields start at zero, there are no particles.  A 3D
 * run with the linear shape and sorting also gets a stream and two events of its own
 * (default priority, released by pml_pic_destroy): with 2^22 particle slots or more,
 * part of its push runs there, forked from `stream` and joined back to it within each
 * step, so that work queued on `stream` after a step still follows all of it. */
int pml_pic_create(const pml_pic_params *params, void *device_workspace, size_t bytes,
                   void *stream, pml_pic_handle **out);

/* Adds n particles from host arrays: x (n x dim, physical coordinates with origin at
 * the physical-box corner), u = gamma v (n x 3), w (n weights).  Each particle also
 * gets a motionless opposite-charge partner at its initial position, which enters
 * only the charge density of the diagnostics (App. A.1).  Positions outside the PEC
 * box give PML_PIC_E_INVALID_ARG; exceeding max_particles gives PML_PIC_E_CAPACITY.
 * Particle ids are assigned consecutively from the number added so far. */
int pml_pic_add_particles(pml_pic_handle *h, int64_t n, const double *x, const double *u,
                          const double *w);

/* Advances n_steps time steps, asynchronously on the handle's stream. */
int pml_pic_step(pml_pic_handle *h, int32_t n_steps);

/* Kernel phases timed by pml_pic_step_profiled */
enum {
    PML_PIC_PHASE_SORT = 0,        /* sort_particles */
    PML_PIC_PHASE_CLEAR_J = 1,     /* clearing the current arrays */
    PML_PIC_PHASE_PUSH = 2,        /* gather_push (fused with deposit_current unless UNFUSED) */
    PML_PIC_PHASE_DEPOSIT = 3,     /* deposit_current when UNFUSED */
    PML_PIC_PHASE_DAMP = 4,        /* damp_pml_current when SEPARATE_DAMP */
    PML_PIC_PHASE_UPDATE_B = 5,    /* update_yee_pml, the two B half steps */
    PML_PIC_PHASE_UPDATE_E = 6,    /* update_yee_pml, the E step (with alpha J) */
    PML_PIC_PHASE_UPDATE_FIELDS = 7, /* update_yee_pml in one pass (2D default) */
    PML_PIC_PHASE_FILTER_J = 8,    /* the binomial filter of the deposited current (3D) */
    PML_PIC_NUM_PHASES = 9
};

/* Same work as pml_pic_step, with a pair of HIP events on the handle's stream around
 * every kernel phase.  Adds the elapsed milliseconds of phase p to phase_ms[p] and
 * the number of timed launches to phase_calls[p] (arrays of PML_PIC_NUM_PHASES
 * entries, caller-owned).  Synchronises the stream before returning. */
int pml_pic_step_profiled(pml_pic_handle *h, int32_t n_steps, double *phase_ms, int64_t *phase_calls);

/* FP64 diagnostics on the device (energies, Gauss residual with an FP64 charge
 * deposit, counts); synchronises the stream.  Returns PML_PIC_E_NONFINITE (with
 * *out filled) if a field value is not finite. */
int pml_pic_diagnose(pml_pic_handle *h, pml_pic_diag *out);

/* Eq. (error) of Sec. III against a reference run `ref` (same dim, precision, cell size and
 * low-side PML, covering h's physical box; e.g. the box extended beyond the face the particle
 * leaves through): *num = sum over the E and B samples inside h's physical box of
 * (F - F_ref)^2, *den = sum of F_ref^2 (FP64 device reductions); the relative error is
 * num / den.  Both handles must live on the current device.  Synchronises both streams. */
int pml_pic_field_error(pml_pic_handle *h, pml_pic_handle *ref, double *num, double *den);

/* pml_pic_field_error for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): the same sums,
 * with the per-workgroup partials and the result in a static device array of the library
 * (513 KiB per GPU, held until the process ends) instead of the handle's workspace.  It
 * calls no hipMalloc/hipFree and allocates nothing on the device.  At most 32768
 * workgroups hold partials (each covers several rows and planes on larger grids); a grid
 * whose single row of 64-sample x-blocks needs more gives PML_PIC_E_INVALID_ARG (no grid
 * within the limits of pml_pic_params does).  All calls on one GPU share the array:
 * calls that overlap on one GPU (other streams, other threads) race and must be
 * serialised by the caller.  The sums may differ from pml_pic_field_error's in the
 * order of the FP64 additions.  Synchronises both streams. */
int pml_pic_field_error_noalloc(pml_pic_handle *h, pml_pic_handle *ref, double *num, double *den);

/* Number of sample positions per field component: nn[d] = cells + 1 along each
 * in-plane axis, 1 along the invariant axis; n_samples = nn0 * nn1 * nn2. */
int pml_pic_grid_shape(const pml_pic_handle *h, int32_t nn[3], int64_t *n_samples);

/* Fields as 12 FP64 split parts of n_samples each, x fastest, in the order
 * E_xy E_xz E_yz E_yx E_zx E_zy B_xy B_xz B_yz B_yx B_zx B_zy (F_ab is the part of
 * F_a driven by the derivative along b, Eqs. MaxwellE/MaxwellB).  Sample (i,j,k) of
 * E_a sits half a cell up along a, of B_a half a cell up along the other two axes.
 * Where a component is stored unsplit its whole value is reported in one part.
 * `count` is the number of doubles in `host` (>= 12 n_samples).  Synchronises. */
int pml_pic_get_fields(pml_pic_handle *h, double *host, int64_t count);
int pml_pic_set_fields(pml_pic_handle *h, const double *host, int64_t count);

/* The current J_x J_y J_z (3 x n_samples doubles) deposited and damped by the last
 * step, at E's sample positions; needs PML_PIC_FLAG_KEEP_CURRENT or the one-pass 2D
 * field update (otherwise the arrays are zero after every step).  J_a at node index
 * M_a along its own axis a (the edge half a cell beyond the outer wall) is padding: a
 * particle leaving the box may deposit there, nothing reads it, and its value is
 * unspecified.  Synchronises. */
int pml_pic_get_current(pml_pic_handle *h, double *host, int64_t count);

/* Static partner charge density at the nodes (n_samples doubles). */
int pml_pic_get_rho_static(pml_pic_handle *h, double *host, int64_t count);
int pml_pic_set_rho_static(pml_pic_handle *h, const double *host, int64_t count);

/* ------------------------------------------------------------------ beam transport
 * The pieces of the paper's cavity run (Sec. IV.A, App. A.2): conductor cells, a beam
 * injected continuously through the entry PML, and the beam's momentum moments per slab
 * (the <u_x> deflection diagnostic). */

/* Conductor cells (3D; needs params.conductor = 1).  cells: host array of M_0 M_1 M_2
 * bytes (cells including the PML, x fastest), nonzero = conductor, or NULL to remove
 * them.  The paper models the cavity walls by setting E and B to zero in the cells they
 * cover; here every field sample lying in the closed extent of a conductor cell (on a
 * wall between a vacuum and a conductor cell too) is set to zero now and after each field
 * update, which on a wall zeroes the tangential E and the normal B.  Particles are not
 * affected by conductors.  Synchronises. */
int pml_pic_set_conductor(pml_pic_handle *h, const uint8_t *cells);

/* Beam source (Sec. IV.A: a long beam injected on one side of the box through that
 * side's PML).  x (n x dim, physical), u (n x 3), w (n): host arrays giving each
 * particle's state at the present time; it moves ballistically until the first step
 * start t = (step + m) dt, m >= 0, at which x + m dt v lies at or beyond the outer wall
 * of the low layer of `axis`, and is added then at that position (no static partner;
 * ids follow those already given, in the order given).  Replaces an earlier source.
 * Needs n <= params.max_source and room for n more particles (max_particles).  Returns
 * PML_PIC_E_INVALID_ARG if a particle never reaches the wall or reaches it outside the
 * box along another axis.  Synchronises. */
int pml_pic_set_source(pml_pic_handle *h, int64_t n, const double *x, const double *u, const double *w,
                       int32_t axis);

/* Beam moments per slab along `axis`: edges (n_slabs + 1 increasing physical
 * coordinates, host); out (host, n_slabs x 5 doubles) receives for each slab
 * [edges[k], edges[k+1]) the number of live particles in it, sum w, sum w u_x,
 * sum w u_y and sum w u_z (FP64 sums).  <u_x> = out[2] / out[1] per slab gives the
 * deflection diagnostic of Sec. IV.A.  1 <= n_slabs <= 64.  Synchronises. */
int pml_pic_slab_moments(pml_pic_handle *h, int32_t axis, int32_t n_slabs, const double *edges, double *out);

/* sort_particles as its own call (the step also runs it every sort_interval steps and
 * after particles are added).  Counting sort of the live particles by their cell's
 * tile-major key, into the other particle buffer; removed particles are dropped.  With
 * tiles of tile[0] x tile[1] x tile[2] cells (pml_pic_params.tile, or the default: 16 x 16
 * in 2D, 8 x 8 x 8 in 3D), numbered x fastest over ntile_d = ceil(M_d / tile[d]) tiles per
 * axis, the key of cell (i, j, k) is
 *   ((tz ntile_1 + ty) ntile_0 + tx) (tile[0] tile[1] tile[2]) + (lz tile[1] + ly) tile[0] + lx
 * with t = index / tile and l = index - t tile per axis.  Particles of equal key keep no
 * particular order.  tile (3 ints, may be NULL) receives the tile shape; *n_keys (may be
 * NULL) the number of keys; key_start (host, may be NULL, then cap is ignored; else cap >=
 * n_keys + 1) the first sorted slot of every key followed by the live particle count.
 * Synchronises.  Not available with PML_PIC_FLAG_NO_SORT. */
int pml_pic_sort_particles(pml_pic_handle *h, int32_t tile[3], uint32_t *key_start, int64_t cap, int64_t *n_keys);

/* Live particle count (synchronises). */
int pml_pic_num_particles(pml_pic_handle *h, int64_t *n);

/* Copies the live particles to host arrays of capacity `cap`: ids, grid coordinates
 * X (n x 3; node-index units, X = x/dx + pml_lo), u (n x 3), w (n).  Order is the
 * device order (sorted by cell), not the insertion order.  Synchronises. */
int pml_pic_get_particles(pml_pic_handle *h, int64_t cap, int64_t *ids, double *X, double *u,
                          double *w, int64_t *n_out);

/* Replaces all particles by the given ones (grid coordinates as above); the static
 * partner density is left as it is; with PML_ALPHA_WEIGHT their damping integrals
 * restart at zero.  Ids must lie in [0, 2^31) (PML_PIC_E_INVALID_ARG otherwise); the
 * pushed adjoint needs them below max_particles. */
int pml_pic_set_particles(pml_pic_handle *h, int64_t n, const int64_t *ids, const double *X,
                          const double *u, const double *w);

/* ------------------------------------------------------------------ adjoint
 * Gradient of the interior field energy U = 1/2 sum (E^2 + B^2) dV (samples inside the
 * physical box) after n steps with respect to the PML profile parameters
 * theta = (sigma_coef[d][k] for d < dim, k < 16; then damping_scale; entries with
 * k >= n_sigma_coef are not part of the profile and get 0), by a hand-written
 * reverse-mode pass through the whole step: update_yee_pml and the alpha damping (Sec.
 * II.A-II.C) and, with push = 1, gather_push and the Esirkepov deposit_current (the
 * particles' response to the fields, and the fields' to the particles' paths).  With
 * push = 0 the paths, and so the undamped current, do not depend on the fields.
 * alpha_mode must be PML_ALPHA_ONE or PML_ALPHA_DAMPED; no current filter, conductors or
 * beam source; pushed runs need every particle id below max_particles.  Needs
 * params.adjoint_segment > 0 and adjoint_checkpoints * adjoint_segment >= n_steps.  The
 * objective is a function of the final fields only; a particle leaving through the outer
 * wall ends its path there, so U is piecewise smooth in theta and the gradient is that
 * of the piece holding theta. */

/* Runs n_steps from the current state, keeping the state every adjoint_segment steps
 * and the final state; writes U (FP64 reduction) to *U.  Synchronises. */
int pml_pic_forward_ckpt(pml_pic_handle *h, int32_t n_steps, double *U);

/* Reverse pass of the last pml_pic_forward_ckpt: restores each checkpoint, recomputes
 * its segment, and runs the transposed step.  seed: NULL for dU/dfields of the
 * interior energy, else a 12-part field array (as pml_pic_get_fields) used as the
 * adjoint of the final state.  lambda_out (12 parts, may be NULL) receives the adjoint
 * of the initial state (for split samples per part; elsewhere the same value in both
 * parts).  grad_theta (n_theta = 16 dim + 1 doubles) receives d(seed . state)/d(theta).
 * The final state of the forward run is restored afterwards.  Synchronises. */
int pml_pic_backward(pml_pic_handle *h, const double *seed, int64_t seed_count, double *lambda_out,
                     double *grad_theta, int32_t n_theta);

/* After pml_pic_backward of a pushed run: the adjoint of the initial particle state, by
 * particle id 0..n-1 (the order of pml_pic_add_particles): dU/dx (n x dim, per unit of
 * the physical coordinates given to pml_pic_add_particles) and dU/du (n x 3, u = gamma v)
 * of the seed's objective.  Ids of particles that were never live hold 0.  Host buffers,
 * caller-owned.  PML_PIC_E_INVALID_ARG if the last reverse pass was not of a pushed run
 * or n exceeds the particles added.  Synchronises. */
int pml_pic_particle_adjoint(pml_pic_handle *h, int64_t n, double *dU_dx, double *dU_du);

/* ------------------------------------------------------------------ batches
 * Many independent runs advanced together: each run has its own grid, PML, profile,
 * alpha mode and particles (all runs share dim, shape_order and precision).  One
 * step of every run is a fixed set of launches (particles, then B, E, B over a work
 * list of (run, block) items walked by a persistent grid); with use_graph the step is
 * captured once as a HIP graph and replayed.  Batched runs deposit with global atomics
 * (no sorting), the form meant for few particles per run, as in single-particle exit
 * studies (Sec. III). */
typedef struct pml_pic_batch pml_pic_batch;

/* Workspace bytes for n_runs runs with the given parameters (validated as for one run). */
int pml_pic_batch_workspace_size(const pml_pic_params *runs, int32_t n_runs, size_t *bytes);

/* Creates the batch in one caller-owned, 256-byte aligned device workspace.  stream
 * must be a non-default hipStream_t when use_graph is 1 (graphs cannot be captured on
 * the legacy default stream). */
int pml_pic_batch_create(const pml_pic_params *runs, int32_t n_runs, void *device_workspace, size_t bytes,
                         void *stream, int32_t use_graph, pml_pic_batch **out);

/* Handle of run `run`, owned by the batch (valid until pml_pic_batch_destroy; never
 * pass it to pml_pic_destroy).  Every single-run call works on it: add particles,
 * diagnose, get/set fields; pml_pic_step on it advances that run alone. */
pml_pic_handle *pml_pic_batch_run(pml_pic_batch *b, int32_t run);

/* Launch shape of the batched field kernels, block_x in 32, 64, 128, 256: in 2D the
 * rows per wavefront segment of the one-pass field update (each wavefront owns 61
 * columns), in 3D blocks of block_x x (256/block_x) nodes; grid_blocks persistent
 * 256-thread workgroups (0 = 8 per compute unit).  Drops the captured graphs. */
int pml_pic_batch_set_launch(pml_pic_batch *b, int32_t block_x, int32_t grid_blocks);

/* Advances every run by n_steps, asynchronously on the batch's stream. */
int pml_pic_batch_step(pml_pic_batch *b, int32_t n_steps);

/* Same work launched eagerly (no graph) with HIP events around every kernel; adds
 * milliseconds and launch counts per phase as pml_pic_step_profiled does
 * (PUSH = particles of all runs, UPDATE_B = both B half steps, UPDATE_E).
 * Synchronises the stream. */
int pml_pic_batch_step_profiled(pml_pic_batch *b, int32_t n_steps, double *phase_ms, int64_t *phase_calls);

const char *pml_pic_batch_last_error(const pml_pic_batch *b);
void pml_pic_batch_destroy(pml_pic_batch *b);

/* A measurement aid, not a step of the method: the throughput of the float atomic additions
 * a deposit can accumulate with, on the current device, in lane additions per second:
 * rates[0] FP64 and rates[1] FP32 atomic adds into LDS (the lanes of a wavefront on consecutive
 * words of a workgroup's box), rates[2] FP32 and rates[3] FP64 atomic adds into global memory
 * at distinct consecutive addresses (the pattern of a box's flush to J).  For benchmarks and
 * design work: which precision an LDS box should hold, and what a flush costs.  Allocates and
 * frees 72 MiB of device memory and a stream of its own; synchronises that stream.
 * PML_PIC_E_INVALID_ARG if rates is NULL, PML_PIC_E_HIP (message via
 * pml_pic_last_error(NULL)) if a HIP call fails. */
int pml_pic_atomic_rates(double rates[4]);

/* Message of the last failed call on h (or of the last failed create if h is NULL). */
const char *pml_pic_last_error(const pml_pic_handle *h);

/* Releases the host-side handle; the caller frees the workspace afterwards. */
void pml_pic_destroy(pml_pic_handle *h);

#ifdef __cplusplus
}
#endif
#endif /* PML_PIC_H */
