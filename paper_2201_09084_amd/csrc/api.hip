// Host side of the C ABI declared in include/pml_pic.h: parameter validation,
// workspace layout, per-axis coefficient tables (built in FP64, stored in the run
// precision), kernel launches on the caller's stream, and state I/O.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdint>
#include <cstring>
#include <new>
#include <stdexcept>
#include <string>
#include <vector>

#include "common.h"
#include "pml_pic.h"

using namespace pmlpic;

namespace {

thread_local std::string g_create_error;

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

struct Layout {
  int dim = 2, M[3] = {0, 0, 0}, ext[3] = {1, 1, 1}, nn[3] = {1, 1, 1};
  long sy = 0, sz = 0, base = 0, nelem = 0;
  int ntab = 0;
  size_t esz = 4;
  int64_t cap = 0;
  size_t off_field[15] = {};   // E0-2, B0-2, Ea0-2, Ba0-2, J0-2
  size_t off_alt[12] = {};     // second set of E, B, Ea, Ba for the out-of-place 2D update
  size_t off_altj[3] = {};     // second current buffer (2D one-pass runs, by step parity)
  size_t off_jtmp = 0;         // 3D current filter: scratch copy of the three J arrays
  bool has_alt = false;
  size_t off_tab = 0;
  size_t off_cell[2] = {}, off_f[2][3] = {}, off_u[2][3] = {}, off_w[2] = {}, off_lam[2] = {}, off_id[2] = {};
  size_t off_oldcell = 0, off_oldf[3] = {};
  bool tile_push3 = false;                  // 3D linear shape: push by sort tile (push3d.hip)
  size_t off_count = 0, off_pushes = 0;
  size_t off_counts = 0, off_rank = 0, off_blocksums = 0, off_tprefix = 0, off_tpartial = 0, off_tblocks = 0;
  size_t off_tdense = 0;
  int ntiles = 1;
  size_t off_items = 0, max_items = 0, off_jbox = 0, off_jslot = 0;
  size_t off_rflags = 0, off_nitems = 0, max_ranges = 0;
  size_t off_rho = 0, off_rho_static = 0, off_partial = 0, off_result = 0, off_flags = 0;
  size_t off_cmask = 0;                     // conductor flags per node (params.conductor)
  size_t off_src_cell = 0, off_src_f[3] = {}, off_src_u[3] = {}, off_src_w = 0, off_src_id = 0;
  int64_t src_cap = 0;                      // beam source entries (params.max_source)
  size_t off_slab = 0;                      // slab moments: edges and sums (FP64)
  int nkeys = 0, tile[3] = {1, 1, 1}, ntile[3] = {1, 1, 1}, nscan = 0, diag_blocks = 0;
  // adjoint storage (present when adjoint_segment > 0)
  int seg = 0, nckpt = 0;            // segment length, checkpoint slots (incl. the final state)
  size_t fields_bytes = 0;           // the 12 E/B arrays (totals and split parts), contiguous
  size_t parts_bytes = 0;            // one particle buffer (cell .. id), contiguous
  size_t off_ckpt = 0, ckpt_stride = 0;
  size_t off_seg_state = 0, off_seg_J = 0, J_bytes = 0;
  size_t off_adj = 0, off_bh = 0, off_grad = 0;
  // pushed runs: the particle buffer and live count at each step of a segment, the
  // adjoint of one step's current, and the particle adjoints (offsets, momenta) by id
  size_t off_seg_parts = 0, off_seg_count = 0, off_lj = 0, off_padj = 0;
  size_t off_check = 0;                     // bounds-checked builds: the CHECK_* word
  size_t total = 0;
};

int fail(std::string *err, int code, const std::string &msg) {
  if (err) *err = msg;
  return code;
}

// Runs the body of an exported call.  A C++ exception (std::bad_alloc from a host vector
// sized by the caller or the grid, or anything else the standard library throws) becomes
// PML_PIC_E_HOST with a message instead of crossing the C ABI; setting the message may
// itself run out of memory, in which case the code alone is returned.
template <class Body>
int abi_guard(std::string *err, Body &&body) noexcept {
  const char *what = "unknown C++ exception";
  try {
    return body();
  } catch (const std::bad_alloc &) {
    what = "out of host memory";
  } catch (const std::exception &e) {
    try {
      if (err) *err = std::string("C++ exception: ") + e.what();
    } catch (...) {
    }
    return PML_PIC_E_HOST;
  } catch (...) {
  }
  try {
    if (err) *err = what;
  } catch (...) {
  }
  return PML_PIC_E_HOST;
}

// depth inside the PML of axis d at grid coordinate X (0 in the physical box) and the
// thickness of that side (physical lengths)
double pml_depth(const pml_pic_params &p, int d, double X, double *thick) {
  const double lo = p.pml[d][0], hi = (double)p.pml[d][0] + p.n[d];
  *thick = 0.0;
  if (X < lo) { *thick = p.pml[d][0] * p.dx[d]; return (lo - X) * p.dx[d]; }
  if (X > hi) { *thick = p.pml[d][1] * p.dx[d]; return (X - hi) * p.dx[d]; }
  return 0.0;
}

// sigma/eps0 = sum_k a_k (depth/L)^k and its exact integral Phi over depth
void profile(const pml_pic_params &p, int d, double X, double *sigma, double *phi) {
  double L;
  const double dep = pml_depth(p, d, X, &L);
  *sigma = 0.0;
  *phi = 0.0;
  if (dep <= 0.0 || L <= 0.0) return;
  const double r = dep / L;
  double pw = 1.0;
  for (int k = 0; k < p.n_sigma_coef; ++k) {
    *sigma += p.sigma_coef[d][k] * pw;
    *phi += p.sigma_coef[d][k] * L * pw * r / (k + 1);
    pw *= r;
  }
}

// The mode the kernels apply: with per-face modes the alpha tables carry each face's
// factor (0, 1 or Eq. alpha), so the kernels multiply by the tables as in mode 2.
int kernel_alpha_mode(const pml_pic_params &p) {
  for (int d = 0; d < 3; ++d)
    for (int side = 0; side < 2; ++side)
      if (p.alpha_face[d][side] != 0) return PML_ALPHA_DAMPED;
  return p.alpha_mode;
}

// the flags a run works with: the deterministic debug mode implies the unfused, unsorted form
int effective_flags(int flags) {
  return (flags & PML_PIC_FLAG_DETERMINISTIC) ? (flags | PML_PIC_FLAG_UNFUSED | PML_PIC_FLAG_NO_SORT) : flags;
}

int validate(const pml_pic_params *p, std::string *err) {
  if (!p) return fail(err, PML_PIC_E_INVALID_ARG, "params is NULL");
  if (p->dim != 2 && p->dim != 3) return fail(err, PML_PIC_E_INVALID_ARG, "dim must be 2 or 3");
  double s2 = 0.0;
  for (int d = 0; d < p->dim; ++d) {
    if (p->n[d] < 1) return fail(err, PML_PIC_E_INVALID_ARG, "n[d] must be >= 1");
    if (p->pml[d][0] < 0 || p->pml[d][1] < 0) return fail(err, PML_PIC_E_INVALID_ARG, "negative PML thickness");
    if (p->pml[d][0] > p->n[d] || p->pml[d][1] > p->n[d])
      return fail(err, PML_PIC_E_INVALID_ARG, "PML thicker than the physical box");
    if (!(p->dx[d] > 0.0) || !std::isfinite(p->dx[d])) return fail(err, PML_PIC_E_INVALID_ARG, "dx must be > 0");
    s2 += 1.0 / (p->dx[d] * p->dx[d]);
  }
  const int M0 = p->n[0] + p->pml[0][0] + p->pml[0][1];
  const int M1 = p->n[1] + p->pml[1][0] + p->pml[1][1];
  const int M2 = p->dim == 3 ? p->n[2] + p->pml[2][0] + p->pml[2][1] : 0;
  if (p->dim == 2 && (M0 > 65533 || M1 > 65533)) return fail(err, PML_PIC_E_INVALID_ARG, "2D grid too large");
  if (p->dim == 3 && (M0 > 2045 || M1 > 2045 || M2 > 1021)) return fail(err, PML_PIC_E_INVALID_ARG, "3D grid too large");
  if (!(p->dt > 0.0) || !std::isfinite(p->dt)) return fail(err, PML_PIC_E_INVALID_ARG, "dt must be > 0");
  if (p->solver != PML_PIC_SOLVER_YEE && p->solver != PML_PIC_SOLVER_CK)
    return fail(err, PML_PIC_E_INVALID_ARG, "solver must be PML_PIC_SOLVER_YEE or PML_PIC_SOLVER_CK");
  if (p->solver == PML_PIC_SOLVER_CK) {
    if (p->dim != 3) return fail(err, PML_PIC_E_INVALID_ARG, "the CK solver is 3D");
    if (std::fabs(p->dx[1] - p->dx[0]) > 1e-12 * p->dx[0] || std::fabs(p->dx[2] - p->dx[0]) > 1e-12 * p->dx[0])
      return fail(err, PML_PIC_E_INVALID_ARG, "the CK solver needs cubic cells");
    if (!(p->dt <= p->dx[0] * (1.0 + 1e-12))) return fail(err, PML_PIC_E_CFL, "c dt exceeds the CK limit dx");
  } else if (!(p->dt <= (1.0 + 1e-12) / std::sqrt(s2))) {
    return fail(err, PML_PIC_E_CFL, "c dt violates the Yee CFL limit");
  }
  if (p->filter_passes < 0 || p->filter_passes > 4) return fail(err, PML_PIC_E_INVALID_ARG, "filter_passes must be in [0,4]");
  if (p->filter_passes > 0 && p->dim != 3) return fail(err, PML_PIC_E_INVALID_ARG, "the current filter is 3D");
  bool faces = false;
  for (int d = 0; d < 3; ++d)
    for (int side = 0; side < 2; ++side) {
      const int f = p->alpha_face[d][side];
      if (f < 0 || f > 3) return fail(err, PML_PIC_E_INVALID_ARG, "alpha_face entries must be 0 (global) or 1 + mode 0..2");
      faces = faces || f != 0;
    }
  if (faces && p->alpha_mode == PML_ALPHA_WEIGHT)
    return fail(err, PML_PIC_E_INVALID_ARG, "per-face alpha modes do not combine with PML_ALPHA_WEIGHT");
  if (p->conductor != 0 && p->conductor != 1) return fail(err, PML_PIC_E_INVALID_ARG, "conductor must be 0 or 1");
  if (p->conductor && p->dim != 3) return fail(err, PML_PIC_E_INVALID_ARG, "conductors are 3D");
  if (p->max_source < 0) return fail(err, PML_PIC_E_INVALID_ARG, "max_source < 0");
  if (p->shape_order < 1 || p->shape_order > 3) return fail(err, PML_PIC_E_INVALID_ARG, "shape_order must be 1, 2 or 3");
  if (p->alpha_mode < 0 || p->alpha_mode > 3) return fail(err, PML_PIC_E_INVALID_ARG, "alpha_mode must be 0, 1, 2 or 3");
  if (!(p->damping_scale >= 0.0) || !std::isfinite(p->damping_scale))
    return fail(err, PML_PIC_E_INVALID_ARG, "damping_scale must be >= 0");
  if (p->n_sigma_coef < 0 || p->n_sigma_coef > 16) return fail(err, PML_PIC_E_INVALID_ARG, "n_sigma_coef must be in [0,16]");
  for (int d = 0; d < p->dim; ++d) {
    for (int k = 0; k < p->n_sigma_coef; ++k)
      if (!std::isfinite(p->sigma_coef[d][k])) return fail(err, PML_PIC_E_INVALID_ARG, "non-finite sigma coefficient");
    const int M = d == 0 ? M0 : (d == 1 ? M1 : M2);
    for (int h = 0; h <= 2 * M; ++h) {
      double s, ph;
      profile(*p, d, 0.5 * h, &s, &ph);
      if (s < 0.0) return fail(err, PML_PIC_E_INVALID_ARG, "sigma profile is negative somewhere in the PML");
    }
  }
  if (p->precision != 32 && p->precision != 64) return fail(err, PML_PIC_E_INVALID_ARG, "precision must be 32 or 64");
  if (p->push != 0 && p->push != 1) return fail(err, PML_PIC_E_INVALID_ARG, "push must be 0 or 1");
  if (p->max_particles < 0 || p->max_particles > (int64_t)1 << 30)
    return fail(err, PML_PIC_E_INVALID_ARG, "max_particles must be in [0, 2^30]");
  if (p->sort_interval < 0) return fail(err, PML_PIC_E_INVALID_ARG, "sort_interval must be >= 0");
  for (int d = 0; d < 3; ++d)
    if (p->tile[d] < 0) return fail(err, PML_PIC_E_INVALID_ARG, "tile must be >= 0");
  {
    // the 2D kernels address samples with 32-bit offsets, and the sort counts cell keys
    // (the grid rounded up to whole tiles) in 32-bit integers
    const int64_t Ms[3] = {M0, M1, M2};
    const int64_t px = ((int64_t)M0 + 1 + 2 * G + 63) / 64 * 64;
    if (p->dim == 2 && px * ((int64_t)M1 + 1 + 2 * G) > (int64_t)INT32_MAX)
      return fail(err, PML_PIC_E_INVALID_ARG, "2D grid too large for 32-bit sample offsets");
    int64_t keys = 1;
    for (int d = 0; d < p->dim; ++d) {
      const int64_t t = p->tile[d] > 0 ? p->tile[d] : (p->dim == 2 ? 16 : 8);
      keys *= (Ms[d] + t - 1) / t * t;
      if (keys > (int64_t)INT32_MAX) return fail(err, PML_PIC_E_INVALID_ARG, "grid too large for 32-bit sort keys");
    }
  }
  if (!(p->mass > 0.0) || !std::isfinite(p->charge)) return fail(err, PML_PIC_E_INVALID_ARG, "need mass > 0, finite charge");
  return PML_PIC_OK;
}

void make_layout(const pml_pic_params &p_in, Layout &L) {
  pml_pic_params p = p_in;
  p.flags = effective_flags(p.flags);
  L.dim = p.dim;
  L.esz = p.precision == 64 ? 8 : 4;
  for (int d = 0; d < 3; ++d) {
    if (d < p.dim) {
      L.M[d] = p.n[d] + p.pml[d][0] + p.pml[d][1];
      L.nn[d] = L.M[d] + 1;
      L.ext[d] = L.M[d] + 1 + 2 * G;
    } else { L.M[d] = 0; L.nn[d] = 1; L.ext[d] = 1; }
  }
  const long px = (long)align_up((size_t)L.ext[0], 64);
  L.sy = px;
  L.sz = (p.dim == 3) ? px * L.ext[1] : 0;
  L.base = G + G * L.sy + (p.dim == 3 ? G * L.sz : 0);
  L.nelem = px * L.ext[1] * L.ext[2];
  L.ntab = *std::max_element(L.M, L.M + 3) + 1 + 2 * G;
  L.cap = p.max_particles;
  const int deft[3] = {p.dim == 2 ? 16 : 8, p.dim == 2 ? 16 : 8, p.dim == 2 ? 1 : 8};
  L.nkeys = 1;
  for (int d = 0; d < 3; ++d) {
    L.tile[d] = d < p.dim ? (p.tile[d] > 0 ? p.tile[d] : deft[d]) : 1;
    L.ntile[d] = d < p.dim ? (L.M[d] + L.tile[d] - 1) / L.tile[d] : 1;
    L.nkeys *= L.ntile[d] * L.tile[d];
  }
  L.nscan = (L.nkeys + 4095) / 4096;
  L.diag_blocks = ((L.M[0] + 1 + 63) / 64) * ((L.M[1] + 1 + 3) / 4) * (p.dim == 3 ? L.M[2] + 1 : 1);

  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes, 256); return o; };
  for (int a = 0; a < 15; ++a) L.off_field[a] = take(L.esz * (size_t)L.nelem);
  // the one-pass field update reads one set of arrays and writes the other; in 3D it
  // covers the Yee solver without current filter, conductors or adjoint storage
  const bool one3 = p.dim == 3 && !(p.flags & PML_PIC_FLAG_SEPARATE_FIELDS) && p.solver == PML_PIC_SOLVER_YEE &&
                    p.filter_passes == 0 && !p.conductor && p.adjoint_segment == 0;
  L.has_alt = (p.dim == 2 && !(p.flags & PML_PIC_FLAG_SEPARATE_FIELDS)) || one3;
  if (p.filter_passes > 0) L.off_jtmp = take(3 * L.esz * (size_t)L.nelem);
  if (L.has_alt) {
    for (int a = 0; a < 12; ++a) L.off_alt[a] = take(L.esz * (size_t)L.nelem);
    for (int a = 0; a < 3; ++a) L.off_altj[a] = take(L.esz * (size_t)L.nelem);
  }
  L.off_tab = take(L.esz * (3 * T_NKIND * (size_t)L.ntab + 3 * PROF_N));
  const size_t cap = (size_t)std::max<int64_t>(L.cap, 1);
  for (int b = 0; b < 2; ++b) {
    L.off_cell[b] = take(4 * cap);
    for (int d = 0; d < 3; ++d) L.off_f[b][d] = d < p.dim ? take(L.esz * cap) : 0;
    for (int d = 0; d < 3; ++d) L.off_u[b][d] = take(L.esz * cap);
    L.off_w[b] = take(L.esz * cap);
    L.off_lam[b] = p.alpha_mode == PML_ALPHA_WEIGHT ? take(L.esz * cap) : 0;
    L.off_id[b] = take(4 * cap);
  }
  L.off_oldcell = take(4 * cap);
  for (int d = 0; d < 3; ++d) L.off_oldf[d] = d < p.dim ? take(L.esz * cap) : 0;
  L.tile_push3 = !(p.flags & (PML_PIC_FLAG_UNFUSED | PML_PIC_FLAG_NO_SORT)) && push3d_applies(p.dim, p.shape_order, L.tile, L.sz);
  L.off_count = take(8);
  L.off_check = take(4);
  L.off_pushes = take(8 * N_PUSH_COUNTERS);
  L.off_counts = take(4 * ((size_t)L.nkeys + 1));
  L.off_rank = take(4 * cap);
  L.off_blocksums = take(4 * ((size_t)L.nscan + 2));
  L.ntiles = L.ntile[0] * L.ntile[1] * L.ntile[2];
  L.off_tprefix = take(4 * ((size_t)L.ntiles + 1));
  L.off_tpartial = take(4 * ((size_t)L.ntiles + 1));
  L.off_tdense = take(4 * ((size_t)L.ntiles + 1));
  L.off_tblocks = take(4 * ((size_t)(L.ntiles + 4095) / 4096 + 2));
  // chunks of the tiled step: 3D, at most one partial chunk per tile beyond cap / chunk;
  // 2D, fixed ranges of the sorted array, each split into at most RANGE_SPLIT_MAX items
  L.max_ranges = (cap + tiled_chunk(p.dim) - 1) / tiled_chunk(p.dim);
  L.max_items = std::max((size_t)L.ntiles + L.max_ranges, RANGE_SPLIT_MAX * L.max_ranges);
  L.off_items = take(16 * L.max_items);
  L.off_rflags = take(4 * L.max_ranges + 4);
  L.off_nitems = take(16);
  L.off_rho = take(8 * (size_t)L.nelem);
  L.off_rho_static = take(8 * (size_t)L.nelem);
  L.off_partial = take(8 * (4 * (size_t)L.diag_blocks + 1024));
  L.off_result = take(8 * 8);
  L.off_flags = take(4 * 4);
  L.off_jbox = take(4 * 8);   // two boxes of nodes with current, by step parity
  // slots of the boxes of nodes given current by the 2D deposits, three sets in rotation
  // (this step's, the last step's being cleared, the next step's being emptied)
  L.off_jslot = take(3 * 16 * JSLOTS);
  if (p.conductor) L.off_cmask = take((size_t)L.nelem);
  L.src_cap = p.max_source;
  if (p.max_source > 0) {
    const size_t ns = (size_t)p.max_source;
    L.off_src_cell = take(4 * ns);
    for (int d = 0; d < p.dim; ++d) L.off_src_f[d] = take(L.esz * ns);
    for (int d = 0; d < 3; ++d) L.off_src_u[d] = take(L.esz * ns);
    L.off_src_w = take(L.esz * ns);
    L.off_src_id = take(4 * ns);
  }
  L.off_slab = take(8 * (6 * (size_t)SLAB_MAX + 1));
  if (p.adjoint_segment > 0) {
    const size_t fb = L.esz * (size_t)L.nelem;          // one field array (multiple of 256 bytes)
    L.seg = p.adjoint_segment;
    L.nckpt = std::max(p.adjoint_checkpoints, 1) + 1;
    L.fields_bytes = 12 * fb;
    L.parts_bytes = L.off_id[0] + align_up(4 * cap, 256) - L.off_cell[0];
    L.ckpt_stride = align_up(L.fields_bytes + L.parts_bytes + 256 + 8 * N_PUSH_COUNTERS, 256);
    L.off_ckpt = take(L.ckpt_stride * L.nckpt);
    L.off_seg_state = take(L.fields_bytes * (size_t)(L.seg + 1));
    L.J_bytes = 3 * fb;
    L.off_seg_J = take(L.J_bytes * (size_t)L.seg);
    L.off_adj = take(12 * fb);
    L.off_bh = take(6 * fb);
    L.off_grad = take(8 * 3 * 8 * (size_t)L.ntab);
    if (p.push) {
      L.off_seg_parts = take(L.parts_bytes * (size_t)L.seg);
      L.off_seg_count = take(4 * (size_t)L.seg);
      L.off_lj = take(3 * fb);
      L.off_padj = take(6 * L.esz * cap);
    }
  }
  L.total = off;
}

}  // namespace

// particle slots from which the dense tiles' push of a 3D tiled step runs on the handle's side
// stream beside the tile-box push (below it, one after the other on the caller's stream)
constexpr int64_t SIDE_PUSH_MIN_SLOTS = int64_t(1) << 22;

struct pml_pic_handle {
  pml_pic_params p;
  Layout L;
  char *ws = nullptr;
  hipStream_t stream = nullptr;
  std::string err;
  int cur = 0;               // active particle buffer
  int jphase = 0;            // 2D one-pass: steps taken (rotation of the box slots)
  int fset = 0;              // active set of field arrays
  int64_t n_slots = 0;       // upper bound of used particle slots
  int64_t n_added = 0;
  int64_t step = 0;
  int sort_interval = 8;
  int since_sort = 0;
  bool sort_pending = false;
  // FP64 host copies of the per-axis tables: [axis][kind][ntab]
  std::vector<double> tab64;
  // adjoint bookkeeping: host metadata of each checkpoint, steps of the last forward
  struct CkptMeta { int cur; int64_t n_slots, n_added, step; int since_sort; bool sort_pending; };
  std::vector<CkptMeta> ckpt_meta;
  int64_t fwd_steps = -1;
  // while set, step k of step_t copies the 12 field arrays before the step to
  // snap_state[k] and the undamped current after the deposit to snap_J[k]
  std::vector<char *> snap_state, snap_J;
  // pushed runs: the particle buffer and count as step k's push reads them go to
  // snap_parts[k] and snap_count[k], the host's slot bound to snap_ns[k]
  std::vector<char *> snap_parts, snap_count;
  std::vector<int64_t> snap_ns;
  bool padj_valid = false;   // particle adjoints hold the last pml_pic_backward's result
  // the last step's filtered current lives in the filter's scratch arrays (odd passes)
  bool j_in_tmp = false;
  bool has_cond = false;                 // conductor mask set
  std::vector<int64_t> src_steps;        // injection step of each source entry (sorted)
  int64_t src_next = 0;                  // first entry not injected yet
  int64_t tail_n = 0;                    // particles injected since the last sort (unsorted tail)
  // 3D tiled push of a single run: the dense tiles' kernel runs on `side` beside the tile-box
  // kernel on `stream` (forked after and joined before with the two events); default priority
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;

  pml_pic_handle() = default;
  pml_pic_handle(const pml_pic_handle &) = delete;
  pml_pic_handle &operator=(const pml_pic_handle &) = delete;
  ~pml_pic_handle() {
    if (ev_join) (void)hipEventDestroy(ev_join);
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (side) (void)hipStreamDestroy(side);
  }

  template <typename X> X *at(size_t off) const { return reinterpret_cast<X *>(ws + off); }
  double tab(int axis, int kind, int i) const { return tab64[((size_t)axis * T_NKIND + kind) * L.ntab + i + G]; }

  template <typename T> Grid<T> grid() const {
    Grid<T> g;
    g.dim = p.dim; g.order = p.shape_order;
    for (int d = 0; d < 3; ++d) {
      g.M[d] = L.M[d];
      g.lo[d] = d < p.dim ? p.pml[d][0] : 0;
      g.n[d] = d < p.dim ? p.n[d] : 0;
      g.ext[d] = L.ext[d];
      g.inv_dx[d] = (T)(1.0 / (d < p.dim ? p.dx[d] : 1.0));
    }
    g.sy = L.sy; g.sz = L.sz; g.base = L.base; g.nelem = L.nelem;
    g.dt = (T)p.dt;
    g.qdt_2m = (T)(p.charge * p.dt / (2.0 * p.mass));
    g.solver = p.solver;
    for (int a = 0; a < 3; ++a) {
      const int b = (a + 1) % 3, c = (a + 2) % 3;
      const double ib = b < p.dim ? 1.0 / p.dx[b] : 1.0, ic = c < p.dim ? 1.0 / p.dx[c] : 1.0;
      g.jcoef[a] = (T)(ib * ic / p.dt);
    }
    g.charge = (T)p.charge;
    g.tab = at<T>(L.off_tab);
    g.ntab = L.ntab;
    g.wdamp = p.alpha_mode == PML_ALPHA_WEIGHT ? 1 : 0;
    g.prof = at<T>(L.off_tab) + 3 * T_NKIND * (size_t)L.ntab;
    g.cmask = has_cond ? at<uint8_t>(L.off_cmask) : nullptr;
#ifdef PMLPIC_CHECK
    g.check = at<uint32_t>(L.off_check);
#else
    g.check = nullptr;
#endif
    return g;
  }
  // offset of field array idx (0..11: E, B, Ea, Ba) of set `set`
  size_t foff_set(int set, int idx) const { return (set && L.has_alt) ? L.off_alt[idx] : L.off_field[idx]; }
  size_t foff(int idx) const { return foff_set(fset, idx); }
  template <typename T> Fields<T> fields_set(int set) const {
    Fields<T> F;
    for (int a = 0; a < 3; ++a) {
      F.E[a] = at<T>(foff_set(set, a));
      F.B[a] = at<T>(foff_set(set, 3 + a));
      F.Ea[a] = at<T>(foff_set(set, 6 + a));
      F.Ba[a] = at<T>(foff_set(set, 9 + a));
      F.J[a] = at<T>(L.off_field[12 + a]);
    }
    return F;
  }
  template <typename T> Fields<T> fields() const { return fields_set<T>(fset); }
  // the current buffer of parity k (2D one-pass runs keep two)
  template <typename T> T *jbuf(int k, int a) const {
    return at<T>((k && L.has_alt) ? L.off_altj[a] : L.off_field[12 + a]);
  }
  template <typename T> Parts<T> parts(int b) const {
    Parts<T> P;
    P.cell = at<uint32_t>(L.off_cell[b]);
    for (int d = 0; d < 3; ++d) {
      P.f[d] = d < p.dim ? at<T>(L.off_f[b][d]) : nullptr;
      P.u[d] = at<T>(L.off_u[b][d]);
    }
    P.w = at<T>(L.off_w[b]);
    P.lam = p.alpha_mode == PML_ALPHA_WEIGHT ? at<T>(L.off_lam[b]) : nullptr;
    P.id = at<int32_t>(L.off_id[b]);
    return P;
  }
  // the beam source entries, in the particle format (no damping integral)
  template <typename T> Parts<T> src_parts() const {
    Parts<T> P;
    P.cell = at<uint32_t>(L.off_src_cell);
    for (int d = 0; d < 3; ++d) {
      P.f[d] = d < p.dim ? at<T>(L.off_src_f[d]) : nullptr;
      P.u[d] = at<T>(L.off_src_u[d]);
    }
    P.w = at<T>(L.off_src_w);
    P.lam = nullptr;
    P.id = at<int32_t>(L.off_src_id);
    return P;
  }
  template <typename T> Parts<T> old_parts() const {
    Parts<T> P = parts<T>(0);
    P.cell = at<uint32_t>(L.off_oldcell);
    for (int d = 0; d < 3; ++d) P.f[d] = d < p.dim ? at<T>(L.off_oldf[d]) : nullptr;
    return P;
  }
  StepCtl ctl() const {
    StepCtl c;
    c.count = at<int32_t>(L.off_count);
    c.pushes = at<unsigned long long>(L.off_pushes);
    c.jslot = nullptr;
    return c;
  }
  SortWork sortwork() const {
    SortWork s;
    s.counts = at<uint32_t>(L.off_counts);
    s.rank = at<uint32_t>(L.off_rank);
    s.blocksums = at<uint32_t>(L.off_blocksums);
    s.nkeys = L.nkeys;
    for (int d = 0; d < 3; ++d) { s.tile[d] = L.tile[d]; s.ntile[d] = L.ntile[d]; }
#ifdef PMLPIC_CHECK
    s.check = at<uint32_t>(L.off_check);
#else
    s.check = nullptr;
#endif
    return s;
  }
  TileWork tilework() const {
    TileWork w;
    w.key_start = at<uint32_t>(L.off_counts);
    w.prefix = at<uint32_t>(L.off_tprefix);
    w.pprefix = at<uint32_t>(L.off_tpartial);
    w.dprefix = at<uint32_t>(L.off_tdense);
    w.blocksums = at<uint32_t>(L.off_tblocks);
    w.items = at<int4>(L.off_items);
    w.sel = 0;
    w.flags = at<uint32_t>(L.off_rflags);
    w.n_items = at<uint32_t>(L.off_nitems);
    w.ntiles = L.ntiles;
    w.tilecells = L.tile[0] * L.tile[1] * L.tile[2];
    w.chunk = tiled_chunk(p.dim);
    for (int d = 0; d < 3; ++d) { w.tile[d] = L.tile[d]; w.ntile[d] = L.ntile[d]; }
    // 3D: a fixed range of the sorted array straddles tiles whose joint box is too big
    // for LDS, so chunks follow the tiles; 2D: fixed ranges keep every chunk full
    w.by_tile = p.dim == 3 ? 1 : 0;
    // widest margin (<= 2 cells) whose box (tile + 2 margin + deposit window per axis)
    // fits in LDS twice (two replicas), else once
    const int win = p.shape_order == 1 ? 4 : 6;
    w.margin = 0;
    bool found = false;
    for (int copies = 2; copies >= 1 && !found; --copies)
      for (int m = 2; m >= 0; --m) {
        long nodes = 1;
        for (int d = 0; d < p.dim; ++d) nodes *= L.tile[d] + 2 * m + win - 1;
        if (copies * ((3 * nodes) | 1) <= 3L * tiled_nodes(p.dim)) { w.margin = m; found = true; break; }
      }
    return w;
  }
  DiagWork diagwork() const {
    DiagWork w;
    w.rho = at<double>(L.off_rho);
    w.rho_static = at<double>(L.off_rho_static);
    w.partial = at<double>(L.off_partial);
    w.result = at<double>(L.off_result);
    w.flags = at<int32_t>(L.off_flags);
    w.max_blocks = L.diag_blocks;
    return w;
  }
};

#define HIPCHK(h, expr)                                                                     \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess) {                                                                  \
      (h)->err = std::string("HIP error in " #expr ": ") + hipGetErrorString(e_);            \
      return PML_PIC_E_HIP;                                                                  \
    }                                                                                        \
  } while (0)

namespace {

void build_tables(pml_pic_handle *h) {
  const pml_pic_params &p = h->p;
  const Layout &L = h->L;
  h->tab64.assign((size_t)3 * T_NKIND * L.ntab + 3 * PROF_N, 0.0);
  for (int d = 0; d < p.dim; ++d) {   // profile block of the per-particle weight damping
    double *pr = h->tab64.data() + (size_t)3 * T_NKIND * L.ntab + d * PROF_N;
    pr[PROF_LO] = p.pml[d][0];
    pr[PROF_HI] = p.pml[d][0] + p.n[d];
    pr[PROF_LLO] = p.pml[d][0] * p.dx[d];
    pr[PROF_LHI] = p.pml[d][1] * p.dx[d];
    pr[PROF_DX] = p.dx[d];
    for (int k = 0; k < p.n_sigma_coef; ++k) pr[PROF_C + k] = p.sigma_coef[d][k] / (k + 1);
  }
  auto put = [&](int axis, int kind, int i, double v) { h->tab64[((size_t)axis * T_NKIND + kind) * L.ntab + i + G] = v; };
  for (int d = 0; d < 3; ++d) {
    for (int i = -G; i <= L.M[d] + G; ++i) {
      for (int centre = 0; centre < 2; ++centre) {
        const double X = i + 0.5 * centre;
        const bool in_grid = d < p.dim && X >= 0.0 && X <= (double)L.M[d];
        double sig = 0.0, phi = 0.0;
        if (in_grid) profile(p, d, X, &sig, &phi);
        double L_;
        const double dep = (d < p.dim) ? pml_depth(p, d, X, &L_) : 0.0;
        const double taus[2] = {p.dt, 0.5 * p.dt};
        double ev[2], gv[2];
        for (int t = 0; t < 2; ++t) {
          if (sig > 0.0) { ev[t] = std::exp(-sig * taus[t]); gv[t] = -std::expm1(-sig * taus[t]) / sig; }
          else { ev[t] = 1.0; gv[t] = taus[t]; }
        }
        double alpha = 1.0;
        // the layer's mode: that of its face when one is set, else the global one
        const int face = d < 3 ? p.alpha_face[d][X < (double)p.pml[d][0] ? 0 : 1] : 0;
        const int mode = face ? face - 1 : p.alpha_mode;
        if (dep > 0.0 && mode == PML_ALPHA_ZERO) alpha = 0.0;
        else if (mode == PML_ALPHA_DAMPED) alpha = std::exp(-p.damping_scale * phi);
        if (d < p.dim && !in_grid) alpha = 0.0;   // guard samples: no current
        const int k0 = centre ? T_SIG_C : T_SIG_N;
        const double inv_dx = 1.0 / (d < p.dim ? p.dx[d] : 1.0);
        put(d, centre ? T_GHK_C : T_GK_N, i, (centre ? gv[1] : gv[0]) * inv_dx);
        put(d, k0 + 0, i, sig);
        put(d, k0 + 1, i, ev[0]);
        put(d, k0 + 2, i, gv[0]);
        put(d, k0 + 3, i, ev[1]);
        put(d, k0 + 4, i, gv[1]);
        put(d, k0 + 5, i, alpha);
      }
    }
  }
}

template <typename T>
int upload_tables(pml_pic_handle *h) {
  std::vector<T> t(h->tab64.size());
  for (size_t i = 0; i < t.size(); ++i) t[i] = (T)h->tab64[i];
  HIPCHK(h, hipMemcpyAsync(h->at<T>(h->L.off_tab), t.data(), sizeof(T) * t.size(), hipMemcpyHostToDevice, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  return PML_PIC_OK;
}

// storage rule of component c (0..5 = Ex..Bz): unsplit in-plane part index, or -1 if split
int unsplit_part(const pml_pic_params &p, int c) {
  const int a = c % 3, b = (a + 1) % 3, cc = (a + 2) % 3;
  if (p.dim == 2 && (b == 2 || cc == 2)) return (b == 2) ? 1 : 0;
  return -1;
}

// is the split of component c active at sample (i,j,k)?
bool split_active(const pml_pic_handle *h, int c, const int id[3]) {
  const int a = c % 3, b = (a + 1) % 3, cc = (a + 2) % 3;
  const int kind = c < 3 ? T_SIG_N : T_SIG_C;
  return h->tab(b, kind, id[b]) + h->tab(cc, kind, id[cc]) > 0.0;
}

template <typename T>
int get_fields_t(pml_pic_handle *h, double *out) {
  const Layout &L = h->L;
  const size_t ns = (size_t)L.nn[0] * L.nn[1] * L.nn[2];
  std::vector<T> tot(L.nelem), aux(L.nelem);
  HIPCHK(h, hipStreamSynchronize(h->stream));
  for (int c = 0; c < 6; ++c) {
    const int a = c % 3;
    HIPCHK(h, hipMemcpy(tot.data(), h->at<T>(h->foff(c < 3 ? a : 3 + a)), sizeof(T) * L.nelem, hipMemcpyDeviceToHost));
    const int up = unsplit_part(h->p, c);
    if (up < 0)
      HIPCHK(h, hipMemcpy(aux.data(), h->at<T>(h->foff(c < 3 ? 6 + a : 9 + a)), sizeof(T) * L.nelem, hipMemcpyDeviceToHost));
    double *p0 = out + (size_t)(2 * c) * ns, *p1 = out + (size_t)(2 * c + 1) * ns;
    for (int k = 0; k < L.nn[2]; ++k)
      for (int j = 0; j < L.nn[1]; ++j)
        for (int i = 0; i < L.nn[0]; ++i) {
          const size_t o = ((size_t)k * L.nn[1] + j) * L.nn[0] + i;
          const long q = L.base + i + j * L.sy + k * L.sz;
          const int id[3] = {i, j, k};
          const double t = (double)tot[q];
          if (up == 0) { p0[o] = t; p1[o] = 0.0; }
          else if (up == 1) { p0[o] = 0.0; p1[o] = t; }
          else if (split_active(h, c, id)) { p0[o] = (double)aux[q]; p1[o] = t - (double)aux[q]; }
          else { p0[o] = t; p1[o] = 0.0; }
        }
  }
  return PML_PIC_OK;
}

template <typename T>
int set_fields_t(pml_pic_handle *h, const double *in) {
  const Layout &L = h->L;
  const size_t ns = (size_t)L.nn[0] * L.nn[1] * L.nn[2];
  std::vector<T> tot(L.nelem), aux(L.nelem);
  HIPCHK(h, hipStreamSynchronize(h->stream));
  for (int c = 0; c < 6; ++c) {
    const int a = c % 3;
    std::fill(tot.begin(), tot.end(), T(0));
    std::fill(aux.begin(), aux.end(), T(0));
    const int up = unsplit_part(h->p, c);
    const double *p0 = in + (size_t)(2 * c) * ns, *p1 = in + (size_t)(2 * c + 1) * ns;
    for (int k = 0; k < L.nn[2]; ++k)
      for (int j = 0; j < L.nn[1]; ++j)
        for (int i = 0; i < L.nn[0]; ++i) {
          const size_t o = ((size_t)k * L.nn[1] + j) * L.nn[0] + i;
          const long q = L.base + i + j * L.sy + k * L.sz;
          const int id[3] = {i, j, k};
          tot[q] = (T)(p0[o] + p1[o]);
          if (up < 0 && split_active(h, c, id)) aux[q] = (T)p0[o];
        }
    HIPCHK(h, hipMemcpy(h->at<T>(h->foff(c < 3 ? a : 3 + a)), tot.data(), sizeof(T) * L.nelem, hipMemcpyHostToDevice));
    if (up < 0)
      HIPCHK(h, hipMemcpy(h->at<T>(h->foff(c < 3 ? 6 + a : 9 + a)), aux.data(), sizeof(T) * L.nelem, hipMemcpyHostToDevice));
  }
  return PML_PIC_OK;
}

template <typename T>
int get_current_t(pml_pic_handle *h, double *out) {
  const Layout &L = h->L;
  const size_t ns = (size_t)L.nn[0] * L.nn[1] * L.nn[2];
  std::vector<T> buf(L.nelem);
  const bool alpha_in_update = !(h->p.flags & PML_PIC_FLAG_SEPARATE_DAMP) && current_alpha(kernel_alpha_mode(h->p));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  for (int a = 0; a < 3; ++a) {
    // 2D one-pass runs: the buffer of the last step (the parity flipped after it)
    T *src = L.has_alt ? h->jbuf<T>(1 - h->fset, a)
                       : (h->j_in_tmp ? h->at<T>(L.off_jtmp) + (size_t)a * L.nelem : h->at<T>(L.off_field[12 + a]));
    HIPCHK(h, hipMemcpy(buf.data(), src, sizeof(T) * L.nelem, hipMemcpyDeviceToHost));
    for (int k = 0; k < L.nn[2]; ++k)
      for (int j = 0; j < L.nn[1]; ++j)
        for (int i = 0; i < L.nn[0]; ++i) {
          const size_t o = ((size_t)k * L.nn[1] + j) * L.nn[0] + i;
          const long q = L.base + i + j * L.sy + k * L.sz;
          double v = (double)buf[q];
          if (alpha_in_update) {
            const int id[3] = {i, j, k};
            for (int d = 0; d < h->p.dim; ++d) v *= h->tab(d, d == a ? T_A_C : T_A_N, id[d]);
          }
          out[(size_t)a * ns + o] = v;
        }
  }
  return PML_PIC_OK;
}

// grid coordinate -> (cell, offset) in precision T; false if outside [0, M)
template <typename T>
bool to_cell(const Layout &L, int dim, const double *X, int id[3], T f[3]) {
  for (int d = 0; d < 3; ++d) { id[d] = 0; f[d] = T(0); }
  for (int d = 0; d < dim; ++d) {
    if (!std::isfinite(X[d])) return false;
    double fl = std::floor(X[d]);
    int i = (int)fl;
    T ff = (T)(X[d] - fl);
    if (ff >= T(1)) { ff = T(0); i += 1; }
    if (i < 0 || i >= L.M[d]) return false;
    id[d] = i;
    f[d] = ff;
  }
  return true;
}

template <typename T>
int write_particles(pml_pic_handle *h, int64_t at_slot, int64_t n, const int64_t *ids, const double *X3,
                    const double *xphys, const double *u, const double *w) {
  const Layout &L = h->L;
  const int dim = h->p.dim;
  std::vector<uint32_t> cell(n);
  std::vector<T> f[3], uu[3], ww(n);
  std::vector<int32_t> id(n);
  for (int d = 0; d < 3; ++d) { f[d].resize(n); uu[d].resize(n); }
  for (int64_t t = 0; t < n; ++t) {
    double X[3] = {0, 0, 0};
    for (int d = 0; d < dim; ++d)
      X[d] = X3 ? X3[3 * t + d] : xphys[dim * t + d] / h->p.dx[d] + h->p.pml[d][0];
    int ic[3];
    T ff[3];
    if (!to_cell<T>(L, dim, X, ic, ff)) {
      h->err = "particle " + std::to_string(t) + " lies outside the PEC box";
      return PML_PIC_E_INVALID_ARG;
    }
    if (!std::isfinite(u[3 * t]) || !std::isfinite(u[3 * t + 1]) || !std::isfinite(u[3 * t + 2]) || !std::isfinite(w[t])) {
      h->err = "particle " + std::to_string(t) + " has a non-finite momentum or weight";
      return PML_PIC_E_INVALID_ARG;
    }
    cell[t] = pack_cell(dim, ic[0], ic[1], ic[2]);
    for (int d = 0; d < 3; ++d) { f[d][t] = ff[d]; uu[d][t] = (T)u[3 * t + d]; }
    ww[t] = (T)w[t];
    if (ids && (ids[t] < 0 || ids[t] > INT32_MAX)) {
      h->err = "particle " + std::to_string(t) + " has an id outside [0, 2^31)";
      return PML_PIC_E_INVALID_ARG;
    }
    id[t] = ids ? (int32_t)ids[t] : (int32_t)(h->n_added + t);
  }
  const int b = h->cur;
  hipStream_t s = h->stream;
  HIPCHK(h, hipMemcpyAsync(h->at<uint32_t>(L.off_cell[b]) + at_slot, cell.data(), 4 * n, hipMemcpyHostToDevice, s));
  for (int d = 0; d < dim; ++d)
    HIPCHK(h, hipMemcpyAsync(h->at<T>(L.off_f[b][d]) + at_slot, f[d].data(), sizeof(T) * n, hipMemcpyHostToDevice, s));
  for (int d = 0; d < 3; ++d)
    HIPCHK(h, hipMemcpyAsync(h->at<T>(L.off_u[b][d]) + at_slot, uu[d].data(), sizeof(T) * n, hipMemcpyHostToDevice, s));
  HIPCHK(h, hipMemcpyAsync(h->at<T>(L.off_w[b]) + at_slot, ww.data(), sizeof(T) * n, hipMemcpyHostToDevice, s));
  HIPCHK(h, hipMemcpyAsync(h->at<int32_t>(L.off_id[b]) + at_slot, id.data(), 4 * n, hipMemcpyHostToDevice, s));
  if (h->p.alpha_mode == PML_ALPHA_WEIGHT) {   // damping integrals start at zero
    std::vector<T> zero(n, T(0));
    HIPCHK(h, hipMemcpyAsync(h->at<T>(L.off_lam[b]) + at_slot, zero.data(), sizeof(T) * n, hipMemcpyHostToDevice, s));
  }
  HIPCHK(h, hipStreamSynchronize(s));
  return PML_PIC_OK;
}

int read_count(pml_pic_handle *h, int32_t *n) {
  HIPCHK(h, hipMemcpyAsync(n, h->at<int32_t>(h->L.off_count), 4, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  return PML_PIC_OK;
}

int write_count(pml_pic_handle *h, int32_t n) {
  HIPCHK(h, hipMemcpyAsync(h->at<int32_t>(h->L.off_count), &n, 4, hipMemcpyHostToDevice, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  return PML_PIC_OK;
}

// Timing hooks around each phase (no-ops unless profiling).
struct PhaseTimer {
  pml_pic_handle *h = nullptr;
  bool on = false;
  std::vector<hipEvent_t> ev;
  std::vector<int> phase;
  hipError_t err = hipSuccess;
  void begin(hipStream_t s) {
    if (!on) return;
    hipEvent_t e;
    if (err == hipSuccess) err = hipEventCreate(&e);
    if (err == hipSuccess) err = hipEventRecord(e, s);
    if (err == hipSuccess) ev.push_back(e);
  }
  void end(hipStream_t s, int p) {
    if (!on) return;
    begin(s);
    phase.push_back(p);
  }
};

// sort_particles: counting sort of the live particles by tile-major cell key into the
// other particle buffer (removed ones dropped), then the work list of the tiled push
template <typename T>
void sort_now(pml_pic_handle *h, const StepCtl &ctl, int ns) {
  const Grid<T> g = h->grid<T>();
  hipStream_t s = h->stream;
  const bool fused = !(h->p.flags & PML_PIC_FLAG_UNFUSED);
  launch_sort<T>(g, h->parts<T>(h->cur), h->parts<T>(1 - h->cur), h->sortwork(), ctl, ns, s);
  if (fused && h->p.dim == 3) launch_tile_chunks(h->tilework(), ctl.count, s);

  if (fused && h->p.dim == 2)
    launch_range_items(h->tilework(), h->parts<T>(1 - h->cur).cell, ctl.count, h->p.shape_order,
                       (int)h->L.max_ranges, std::min(h->sort_interval - 1, 2), s);
  h->cur = 1 - h->cur;
  h->since_sort = 0;
  h->sort_pending = false;
  h->tail_n = 0;
}

template <typename T>
int step_t(pml_pic_handle *h, int nsteps, PhaseTimer &pt) {
  const Grid<T> g = h->grid<T>();
  const int fl = h->p.flags;
  const bool use_sort = !(fl & PML_PIC_FLAG_NO_SORT);
  const bool fused = !(fl & PML_PIC_FLAG_UNFUSED);
  const bool sep_damp = (fl & PML_PIC_FLAG_SEPARATE_DAMP) != 0;
  const bool one_pass = h->L.has_alt;
  // The E update zeroes J only where it updates E; the filter also reads the samples on
  // the PEC walls, so with the filter J is cleared before every deposit instead.
  const bool keep_j = (fl & PML_PIC_FLAG_KEEP_CURRENT) != 0 || one_pass || h->p.filter_passes > 0;
  const int amode = kernel_alpha_mode(h->p);
  hipStream_t s = h->stream;
  const size_t jbytes = sizeof(T) * (size_t)h->L.nelem;
  int *jslot = h->at<int>(h->L.off_jslot);
  for (int it = 0; it < nsteps; ++it) {
    Fields<T> F = h->fields<T>();
    StepCtl ctl = h->ctl();
    // beam source: the entries due at this step join the particles (sorted in below)
    int64_t due = 0;
    while (h->src_next + due < (int64_t)h->src_steps.size() && h->src_steps[h->src_next + due] == h->step) ++due;
    if (due > 0) {
      if (h->n_slots + due > h->L.cap)
        return fail(&h->err, PML_PIC_E_CAPACITY, "max_particles exceeded by the beam source");
      // appended after the live particles; until the next sort they form an unsorted tail
      // that the tiled push leaves to the per-particle kernel
      launch_inject<T>(h->p.dim, h->parts<T>(h->cur), h->src_parts<T>(), ctl.count, h->src_next, (int)due,
                       ctl.count + 1, h->tail_n == 0, s);
      h->src_next += due;
      h->n_slots += due;
      h->tail_n += due;
      // a beam's injected particles crowd few cells, where the per-particle kernel's global
      // atomics collide: past a few thousand it is cheaper to sort them in right away
      if (h->tail_n > 4096) h->sort_pending = true;
    }
    const int ns = (int)h->n_slots;
    const int ph = h->jphase % 3;
    int *slot_cur = jslot + 4 * JSLOTS * ph;                 // this step's boxes
    JClear<T> jc{{nullptr, nullptr, nullptr}, nullptr, nullptr};
    JZero<T> jz{{nullptr, nullptr, nullptr}};
    if (one_pass && h->p.dim == 3) {   // deposit into this step's buffer, the field pass clears the other
      for (int a = 0; a < 3; ++a) {
        F.J[a] = h->jbuf<T>(h->fset, a);
        jz.J[a] = h->jbuf<T>(1 - h->fset, a);
      }
    } else if (one_pass) {
      ctl.jslot = slot_cur;
      for (int a = 0; a < 3; ++a) {
        F.J[a] = h->jbuf<T>(h->fset, a);        // deposited this step
        jc.J[a] = h->jbuf<T>(1 - h->fset, a);   // the last step's, cleared during this step
      }
      jc.prev = jslot + 4 * JSLOTS * ((ph + 2) % 3);
      jc.next = jslot + 4 * JSLOTS * ((ph + 1) % 3);
    }
    if (it < (int)h->snap_state.size())
      HIPCHK(h, hipMemcpyAsync(h->snap_state[it], F.E[0], h->L.fields_bytes, hipMemcpyDeviceToDevice, s));
    if (use_sort && ns > 0 && (h->sort_pending || h->since_sort >= h->sort_interval)) {
      pt.begin(s);
      sort_now<T>(h, ctl, ns);
      pt.end(s, PML_PIC_PHASE_SORT);
    }
    const bool tiled = fused && use_sort && ns > 0;
    if (one_pass && h->p.dim == 2 && !tiled) {   // the tiled deposit clears the other buffer itself
      pt.begin(s);
      launch_jbox_clear<T>(g, jc, s);
      pt.end(s, PML_PIC_PHASE_CLEAR_J);
    } else if (!one_pass && keep_j) {   // J survives the step; clear it before depositing (the three arrays are adjacent)
      pt.begin(s);
      HIPCHK(h, hipMemsetAsync(F.J[0], 0, 3 * jbytes, s));
      pt.end(s, PML_PIC_PHASE_CLEAR_J);
    }
    const Parts<T> P = h->parts<T>(h->cur);
    if (it < (int)h->snap_parts.size()) {
      HIPCHK(h, hipMemcpyAsync(h->snap_parts[it], P.cell, h->L.parts_bytes, hipMemcpyDeviceToDevice, s));
      HIPCHK(h, hipMemcpyAsync(h->snap_count[it], ctl.count, 4, hipMemcpyDeviceToDevice, s));
      h->snap_ns[it] = ns;
    }
    pt.begin(s);
    if (fused && use_sort && h->L.tile_push3) {
      // dense tiles (a cell with many particles: a beam whose LDS adds would meet on a few
      // nodes) take the kernel with chunk-sized replicated boxes, the others the tile-box one.
      // The two touch disjoint particles and add into J with atomics, so the dense kernel (a
      // few workgroups busy for tens of microseconds on a beam) runs on the handle's side
      // stream beside the tile-box kernel instead of before it.
      // (the fork and the join cost more than they hide on runs of a few hundred thousand
      // particles: the cavity's step took 0.145 against 0.133 ms with them)
      TileWork tw = h->tilework();
      const bool beside = h->side && ns >= SIDE_PUSH_MIN_SLOTS;
      hipStream_t sd = s;
      if (beside) {
        HIPCHK(h, hipEventRecord(h->ev_fork, s));
        HIPCHK(h, hipStreamWaitEvent(h->side, h->ev_fork, 0));
        sd = h->side;
      }
      tw.sel = 1;
      launch_push_deposit_tiles<T>(g, F, P, ctl, jc, tw, ns, h->p.push, sd);
      tw.sel = 2;
      launch_push3d<T>(g, F, P, ctl, tw, ns, h->p.push, s);
      // the particles injected since the sort (their own slots) also before the join
      if (h->tail_n > 0) launch_gather_push_tail<T>(g, F, P, ctl, ctl.count + 1, (int)h->tail_n, ns, h->p.push, s);
      if (beside) {
        HIPCHK(h, hipEventRecord(h->ev_join, h->side));
        HIPCHK(h, hipStreamWaitEvent(s, h->ev_join, 0));
      }
    } else if (fused && use_sort) {
      launch_push_deposit_tiles<T>(g, F, P, ctl, jc, h->tilework(), ns, h->p.push, s);
      if (h->tail_n > 0) launch_gather_push_tail<T>(g, F, P, ctl, ctl.count + 1, (int)h->tail_n, ns, h->p.push, s);
    } else {
      launch_gather_push<T>(g, F, P, h->old_parts<T>(), ctl, ns, h->p.push, fused, s);
    }
    pt.end(s, PML_PIC_PHASE_PUSH);
    if (!fused) {
      pt.begin(s);
      launch_deposit<T>(g, F, P, h->old_parts<T>(), ctl, ns, (fl & PML_PIC_FLAG_DETERMINISTIC) != 0, s);
      pt.end(s, PML_PIC_PHASE_DEPOSIT);
    }
    if (h->p.filter_passes > 0) {
      pt.begin(s);
      T *jf = launch_filter_current<T>(g, F.J[0], h->at<T>(h->L.off_jtmp), h->p.filter_passes, s);
      for (int a = 0; a < 3; ++a) F.J[a] = jf + (size_t)a * h->L.nelem;   // the rest of the step reads it
      h->j_in_tmp = jf != h->at<T>(h->L.off_field[12]);
      pt.end(s, PML_PIC_PHASE_FILTER_J);
    }
    if (it < (int)h->snap_J.size())
      HIPCHK(h, hipMemcpyAsync(h->snap_J[it], F.J[0], h->L.J_bytes, hipMemcpyDeviceToDevice, s));
    if (sep_damp && current_alpha(amode)) {
      pt.begin(s);
      launch_damp_current<T>(g, F, s);
      pt.end(s, PML_PIC_PHASE_DAMP);
    }
    if (one_pass) {
      pt.begin(s);
      if (h->p.dim == 3)
        launch_fused_fields_3d<T>(g, F, h->fields_set<T>(1 - h->fset), jz, !sep_damp && current_alpha(amode), s);
      else
        launch_fused_fields<T>(g, F, h->fields_set<T>(1 - h->fset), slot_cur,
                               !sep_damp && current_alpha(amode), s);
      pt.end(s, PML_PIC_PHASE_UPDATE_FIELDS);
      h->fset = 1 - h->fset;
      h->jphase++;
    } else {
      pt.begin(s);
      launch_update_B<T>(g, F, true, s);
      pt.end(s, PML_PIC_PHASE_UPDATE_B);
      pt.begin(s);
      launch_update_E<T>(g, F, !sep_damp, amode, !keep_j, s);
      pt.end(s, PML_PIC_PHASE_UPDATE_E);
      pt.begin(s);
      launch_update_B<T>(g, F, true, s);
      pt.end(s, PML_PIC_PHASE_UPDATE_B);
    }
    h->step++;
    h->since_sort++;
  }
  HIPCHK(h, hipGetLastError());
  if (pt.err != hipSuccess) {
    h->err = std::string("HIP event error: ") + hipGetErrorString(pt.err);
    return PML_PIC_E_HIP;
  }
  return PML_PIC_OK;
}

template <typename T>
int diagnose_t(pml_pic_handle *h, pml_pic_diag *out) {
  const Grid<T> g = h->grid<T>();
  const DiagWork dw = h->diagwork();
  launch_diag<T>(g, h->fields<T>(), h->parts<T>(h->cur), h->ctl(), (int)h->n_slots, dw, h->stream);
  HIPCHK(h, hipGetLastError());
  double res[8];
  int32_t flags[2];
  unsigned long long pushv[N_PUSH_COUNTERS];
  unsigned long long pushes = 0;
  HIPCHK(h, hipMemcpyAsync(res, dw.result, sizeof(double) * 5, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipMemcpyAsync(flags, dw.flags, sizeof(int32_t) * 2, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipMemcpyAsync(pushv, h->ctl().pushes, sizeof(pushv), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  for (int k = 0; k < N_PUSH_COUNTERS; ++k) pushes += pushv[k];
  long inner = 1;
  for (int d = 0; d < h->p.dim; ++d) inner *= std::max(0, h->p.n[d] - 1);
  out->u_interior = res[0];
  out->u_pml = res[1];
  out->gauss_max = res[2];
  out->gauss_l2 = inner > 0 ? std::sqrt(res[3] / (double)inner) : 0.0;
  out->rho_max = res[4];
  out->n_particles = flags[1];
  out->step = h->step;
  out->n_pushes = (int64_t)pushes;
  out->nonfinite = flags[0];
  if (flags[0]) { h->err = "non-finite value in the fields"; return PML_PIC_E_NONFINITE; }
  return PML_PIC_OK;
}

template <typename T>
int get_particles_t(pml_pic_handle *h, int64_t cap, int64_t *ids, double *X, double *u, double *w, int64_t *n_out) {
  int32_t cnt;
  int rc = read_count(h, &cnt);
  if (rc) return rc;
  const int64_t n = std::min<int64_t>(cnt, h->n_slots);
  const Layout &L = h->L;
  const int b = h->cur, dim = h->p.dim;
  std::vector<uint32_t> cell(n);
  std::vector<T> f[3], uu[3], ww(n);
  std::vector<int32_t> id(n);
  for (int d = 0; d < 3; ++d) { f[d].resize(n); uu[d].resize(n); }
  if (n > 0) {
    HIPCHK(h, hipMemcpy(cell.data(), h->at<uint32_t>(L.off_cell[b]), 4 * n, hipMemcpyDeviceToHost));
    for (int d = 0; d < dim; ++d) HIPCHK(h, hipMemcpy(f[d].data(), h->at<T>(L.off_f[b][d]), sizeof(T) * n, hipMemcpyDeviceToHost));
    for (int d = 0; d < 3; ++d) HIPCHK(h, hipMemcpy(uu[d].data(), h->at<T>(L.off_u[b][d]), sizeof(T) * n, hipMemcpyDeviceToHost));
    HIPCHK(h, hipMemcpy(ww.data(), h->at<T>(L.off_w[b]), sizeof(T) * n, hipMemcpyDeviceToHost));
    HIPCHK(h, hipMemcpy(id.data(), h->at<int32_t>(L.off_id[b]), 4 * n, hipMemcpyDeviceToHost));
  }
  int64_t m = 0;
  for (int64_t t = 0; t < n; ++t) {
    if (cell[t] == DEAD) continue;
    if (m >= cap) { h->err = "particle output capacity too small"; return PML_PIC_E_CAPACITY; }
    int ic[3];
    unpack_cell(dim, cell[t], ic[0], ic[1], ic[2]);
    ids[m] = id[t];
    for (int d = 0; d < 3; ++d) {
      X[3 * m + d] = d < dim ? (double)ic[d] + (double)f[d][t] : 0.0;
      u[3 * m + d] = (double)uu[d][t];
    }
    w[m] = (double)ww[t];
    ++m;
  }
  *n_out = m;
  return PML_PIC_OK;
}

}  // namespace

static int create_handle(const pml_pic_params *params, void *device_workspace, size_t bytes, void *stream,
                         pml_pic_handle **out, std::string *err) {
  if (!out) return fail(err, PML_PIC_E_INVALID_ARG, "out is NULL");
  *out = nullptr;
  int rc = validate(params, err);
  if (rc) return rc;
  Layout L;
  make_layout(*params, L);
  if (!device_workspace || bytes < L.total)
    return fail(err, PML_PIC_E_WORKSPACE, "workspace smaller than pml_pic_workspace_size()");
  if (((uintptr_t)device_workspace) % 256 != 0)
    return fail(err, PML_PIC_E_WORKSPACE, "workspace must be 256-byte aligned");
  pml_pic_handle *h = new pml_pic_handle();
  h->p = *params;
  h->p.flags = effective_flags(params->flags);
  h->L = L;
  h->ws = (char *)device_workspace;
  h->stream = (hipStream_t)stream;
  h->sort_interval = params->sort_interval > 0 ? params->sort_interval : 8;
  build_tables(h);
  hipError_t e = hipMemsetAsync(h->ws, 0, L.total, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e == hipSuccess) {   // current-box slots start empty
    std::vector<int> empty(3 * 4 * JSLOTS);
    for (int k = 0; k < 3 * JSLOTS; ++k) {
      empty[4 * k] = 0x7FFFFFFF; empty[4 * k + 1] = -0x7FFFFFFF;
      empty[4 * k + 2] = 0x7FFFFFFF; empty[4 * k + 3] = -0x7FFFFFFF;
    }
    e = hipMemcpy(h->ws + L.off_jslot, empty.data(), sizeof(int) * empty.size(), hipMemcpyHostToDevice);
  }
  if (e != hipSuccess) {
    *err = std::string("HIP error while clearing the workspace: ") + hipGetErrorString(e);
    delete h;
    return PML_PIC_E_HIP;
  }
  rc = params->precision == 64 ? upload_tables<double>(h) : upload_tables<float>(h);
  if (rc) {
    *err = h->err;
    delete h;
    return rc;
  }
  *out = h;
  return PML_PIC_OK;
}

// ===================================================================== batches
struct pml_pic_batch {
  std::vector<pml_pic_handle *> runs;
  std::vector<int64_t> slots_seen;
  char *ws = nullptr;
  hipStream_t stream = nullptr;
  std::string err;
  int dim = 2, order = 1, prec = 32;
  size_t off_desc = 0, off_items = 0, max_items = 0;
  int n_items = 0, bdx = 64, grid_blocks = 0;
  int parity = 0;               // 2D: field set holding the current state
  bool use_graph = false;
  hipGraph_t graph[2] = {nullptr, nullptr};        // one step from each field set
  hipGraphExec_t exec[2] = {nullptr, nullptr};
};

namespace {

const int BATCH_BDX[4] = {32, 64, 128, 256};

// Work items of a batched step.  2D: (run, strip of FW columns, first row, end row)
// for the one-pass field update, `bdx` rows per segment.  3D: (run, bx, by, z) blocks
// of bdx x (256 / bdx) nodes for the in-place sweeps.
size_t batch_items(const std::vector<Layout> &Ls, int dim, int bdx) {
  size_t n = 0;
  if (dim == 2) {
    for (const Layout &L : Ls) n += (size_t)((L.M[0] + FW) / FW) * ((L.M[1] + bdx) / bdx);
    return n;
  }
  const int bdy = 256 / bdx;
  for (const Layout &L : Ls)
    n += (size_t)((L.M[0] + bdx) / bdx) * ((L.M[1] + bdy) / bdy) * (L.M[2] + 1);
  return n;
}

// a batched run: particles deposit with global atomics; in 3D the fields advance in
// place, in 2D out of place between two sets
pml_pic_params batch_run_params(const pml_pic_params &p) {
  pml_pic_params pr = p;
  pr.flags |= PML_PIC_FLAG_NO_SORT;
  if (p.dim == 3) pr.flags |= PML_PIC_FLAG_SEPARATE_FIELDS;
  else pr.flags &= ~PML_PIC_FLAG_SEPARATE_FIELDS;
  pr.flags &= ~(PML_PIC_FLAG_UNFUSED | PML_PIC_FLAG_SEPARATE_DAMP | PML_PIC_FLAG_KEEP_CURRENT);
  return pr;
}

int batch_layout(const pml_pic_params *runs, int32_t n, std::vector<Layout> &Ls, std::vector<size_t> &offs,
                 size_t &off_desc, size_t &off_items, size_t &max_items, size_t &total, std::string *err) {
  if (!runs || n < 1) return fail(err, PML_PIC_E_INVALID_ARG, "need at least one run");
  Ls.assign(n, Layout());
  for (int r = 0; r < n; ++r) {
    const int rc = validate(&runs[r], err);
    if (rc) {
      if (err) *err = "run " + std::to_string(r) + ": " + *err;
      return rc;
    }
    if (runs[r].conductor || runs[r].max_source > 0)
      return fail(err, PML_PIC_E_INVALID_ARG, "batched runs have neither conductors nor sources");
    if (runs[r].flags & PML_PIC_FLAG_DETERMINISTIC)
      return fail(err, PML_PIC_E_INVALID_ARG, "the deterministic debug mode is for single runs");
    if (runs[r].solver != PML_PIC_SOLVER_YEE || runs[r].filter_passes > 0)
      return fail(err, PML_PIC_E_INVALID_ARG, "batched runs use the Yee solver without current filter");
    if (runs[r].dim != runs[0].dim || runs[r].shape_order != runs[0].shape_order ||
        runs[r].precision != runs[0].precision)
      return fail(err, PML_PIC_E_INVALID_ARG, "all runs of a batch need the same dim, shape_order and precision");
    make_layout(batch_run_params(runs[r]), Ls[r]);
  }
  max_items = 0;
  for (int k = 0; k < 4; ++k) max_items = std::max(max_items, batch_items(Ls, runs[0].dim, BATCH_BDX[k]));
  const size_t dsz = runs[0].precision == 64 ? sizeof(RunDesc<double>) : sizeof(RunDesc<float>);
  off_desc = 0;
  off_items = align_up(dsz * n, 256);
  size_t off = align_up(off_items + sizeof(int4) * max_items, 256);
  offs.resize(n);
  for (int r = 0; r < n; ++r) {
    offs[r] = off;
    off = align_up(off + Ls[r].total, 256);
  }
  total = off;
  return PML_PIC_OK;
}

template <typename T>
int batch_upload_descs(pml_pic_batch *b) {
  std::vector<RunDesc<T>> d(b->runs.size());
  for (size_t r = 0; r < b->runs.size(); ++r) {
    pml_pic_handle *h = b->runs[r];
    d[r].g = h->grid<T>();
    d[r].F = h->fields_set<T>(0);
    d[r].F2 = h->fields_set<T>(1);
    d[r].jbox = h->at<int>(h->L.off_jbox);
    d[r].pad2[0] = d[r].pad2[1] = 0;
    d[r].P = h->parts<T>(h->cur);
    d[r].ctl = h->ctl();
    d[r].n_slots = (int)h->n_slots;
    d[r].push = h->p.push;
    d[r].alpha_mode = kernel_alpha_mode(h->p);
    d[r].pad = 0;
    b->slots_seen[r] = h->n_slots;
  }
  HIPCHK(b, hipMemcpyAsync(b->ws + b->off_desc, d.data(), sizeof(RunDesc<T>) * d.size(), hipMemcpyHostToDevice, b->stream));
  HIPCHK(b, hipStreamSynchronize(b->stream));
  return PML_PIC_OK;
}

int batch_build_items(pml_pic_batch *b, int bdx) {
  const int bdy = 256 / bdx;
  std::vector<int4> it;
  it.reserve(b->max_items);
  for (size_t r = 0; r < b->runs.size(); ++r) {
    const Layout &L = b->runs[r]->L;
    if (b->dim == 2) {
      const int ns = (L.M[0] + FW) / FW;
      for (int y0 = 0; y0 <= L.M[1]; y0 += bdx)
        for (int st = 0; st < ns; ++st) it.push_back(make_int4((int)r, st, y0, std::min(y0 + bdx, L.M[1] + 1)));
      continue;
    }
    const int nbx = (L.M[0] + bdx) / bdx, nby = (L.M[1] + bdy) / bdy, nbz = L.M[2] + 1;
    for (int bz = 0; bz < nbz; ++bz)
      for (int by = 0; by < nby; ++by)
        for (int bx = 0; bx < nbx; ++bx) it.push_back(make_int4((int)r, bx, by, bz));
  }
  if (it.size() > b->max_items) return fail(&b->err, PML_PIC_E_INVALID_ARG, "work list overflow");
  HIPCHK(b, hipMemcpyAsync(b->ws + b->off_items, it.data(), sizeof(int4) * it.size(), hipMemcpyHostToDevice, b->stream));
  HIPCHK(b, hipStreamSynchronize(b->stream));
  b->n_items = (int)it.size();
  b->bdx = bdx;
  return PML_PIC_OK;
}

void batch_drop_graph(pml_pic_batch *b) {
  for (int k = 0; k < 2; ++k) {
    if (b->exec[k]) (void)hipGraphExecDestroy(b->exec[k]);
    if (b->graph[k]) (void)hipGraphDestroy(b->graph[k]);
    b->exec[k] = nullptr;
    b->graph[k] = nullptr;
  }
}

// One step of every run, the order of the single-run step.  2D: J cleared over the
// previous step's box, particles, one-pass fields from set `parity` to the other.  3D: particles, B half step, E
// step (consuming J), B half step, in place.
template <typename T>
void batch_launch(pml_pic_batch *b, int parity, PhaseTimer *pt = nullptr) {
  const RunDesc<T> *runs = (const RunDesc<T> *)(b->ws + b->off_desc);
  const int4 *items = (const int4 *)(b->ws + b->off_items);
  if (b->dim == 2) {
    if (pt) pt->begin(b->stream);
    launch_batch_clear_j<T>(runs, (int)b->runs.size(), parity, b->stream);
    if (pt) pt->end(b->stream, PML_PIC_PHASE_CLEAR_J);
    if (pt) pt->begin(b->stream);
    launch_batch_phase<T>(0, b->dim, b->order, runs, (int)b->runs.size(), items, b->n_items, b->bdx, b->grid_blocks,
                          parity, b->stream);
    if (pt) pt->end(b->stream, PML_PIC_PHASE_PUSH);
    if (pt) pt->begin(b->stream);
    launch_batch_fused<T>(runs, items, b->n_items, parity, b->grid_blocks, b->stream);
    if (pt) pt->end(b->stream, PML_PIC_PHASE_UPDATE_FIELDS);
    return;
  }
  static const int order_of_phases[4] = {0, 1, 2, 1};
  static const int timer_phase[3] = {PML_PIC_PHASE_PUSH, PML_PIC_PHASE_UPDATE_B, PML_PIC_PHASE_UPDATE_E};
  for (int k = 0; k < 4; ++k) {
    const int ph = order_of_phases[k];
    if (pt) pt->begin(b->stream);
    launch_batch_phase<T>(ph, b->dim, b->order, runs, (int)b->runs.size(), items, b->n_items, b->bdx,
                          b->grid_blocks, 0, b->stream);
    if (pt) pt->end(b->stream, timer_phase[ph]);
  }
}

template <typename T>
int batch_step_t(pml_pic_batch *b, int n, PhaseTimer *pt = nullptr) {
  bool changed = false;
  for (size_t r = 0; r < b->runs.size(); ++r) changed = changed || b->runs[r]->n_slots != b->slots_seen[r];
  if (changed) {
    const int rc = batch_upload_descs<T>(b);
    if (rc) return rc;
  }
  const int flip = b->dim == 2 ? 1 : 0;   // 2D steps alternate between the field sets
  if (pt) {
    for (int it = 0; it < n; ++it) {
      batch_launch<T>(b, b->parity, pt);
      b->parity ^= flip;
    }
    HIPCHK(b, hipGetLastError());
  } else if (b->use_graph) {
    for (int it = 0; it < n; ++it) {
      const int k = b->parity;
      if (!b->exec[k]) {
        HIPCHK(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
        batch_launch<T>(b, k);
        hipGraph_t g = nullptr;
        HIPCHK(b, hipStreamEndCapture(b->stream, &g));
        b->graph[k] = g;
        HIPCHK(b, hipGraphInstantiate(&b->exec[k], b->graph[k], nullptr, nullptr, 0));
      }
      HIPCHK(b, hipGraphLaunch(b->exec[k], b->stream));
      b->parity ^= flip;
    }
  } else {
    for (int it = 0; it < n; ++it) {
      batch_launch<T>(b, b->parity);
      b->parity ^= flip;
    }
    HIPCHK(b, hipGetLastError());
  }
  for (pml_pic_handle *h : b->runs) {
    h->step += n;
    h->fset = b->parity;
  }
  return PML_PIC_OK;
}

}  // namespace

extern "C" {

static int pml_pic_batch_workspace_size_impl(const pml_pic_params *runs, int32_t n_runs, size_t *bytes) {
  if (!bytes) return PML_PIC_E_INVALID_ARG;
  std::vector<Layout> Ls;
  std::vector<size_t> offs;
  size_t od, oi, mi, total;
  const int rc = batch_layout(runs, n_runs, Ls, offs, od, oi, mi, total, &g_create_error);
  if (rc) return rc;
  *bytes = total;
  return PML_PIC_OK;
}

static int pml_pic_batch_create_impl(const pml_pic_params *runs, int32_t n_runs, void *device_workspace, size_t bytes,
                         void *stream, int32_t use_graph, pml_pic_batch **out) {
  if (!out) return fail(&g_create_error, PML_PIC_E_INVALID_ARG, "out is NULL");
  *out = nullptr;
  std::vector<Layout> Ls;
  std::vector<size_t> offs;
  size_t od, oi, mi, total;
  int rc = batch_layout(runs, n_runs, Ls, offs, od, oi, mi, total, &g_create_error);
  if (rc) return rc;
  if (!device_workspace || bytes < total || ((uintptr_t)device_workspace) % 256 != 0)
    return fail(&g_create_error, PML_PIC_E_WORKSPACE, "batch workspace too small or misaligned");
  if (use_graph && !stream)
    return fail(&g_create_error, PML_PIC_E_INVALID_ARG, "graphs need a non-default stream");
  pml_pic_batch *b = new pml_pic_batch();
  b->ws = (char *)device_workspace;
  b->stream = (hipStream_t)stream;
  b->dim = runs[0].dim;
  b->order = runs[0].shape_order;
  b->prec = runs[0].precision;
  b->off_desc = od;
  b->off_items = oi;
  b->max_items = mi;
  b->use_graph = use_graph != 0;
  for (int r = 0; r < n_runs; ++r) {
    pml_pic_params pr = batch_run_params(runs[r]);
    pml_pic_handle *h = nullptr;
    rc = create_handle(&pr, b->ws + offs[r], Ls[r].total, stream, &h, &g_create_error);
    if (rc) {
      for (pml_pic_handle *x : b->runs) delete x;
      delete b;
      return rc;
    }
    b->runs.push_back(h);
  }
  b->slots_seen.assign(n_runs, -1);
  int dev = 0, n_cu = 256;
  if (hipGetDevice(&dev) == hipSuccess) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess && prop.multiProcessorCount > 0) n_cu = prop.multiProcessorCount;
  }
  b->grid_blocks = 8 * n_cu;
  rc = b->prec == 64 ? batch_upload_descs<double>(b) : batch_upload_descs<float>(b);
  if (rc == PML_PIC_OK) rc = batch_build_items(b, 64);
  if (rc) {
    g_create_error = b->err;
    for (pml_pic_handle *x : b->runs) delete x;
    delete b;
    return rc;
  }
  *out = b;
  return PML_PIC_OK;
}

pml_pic_handle *pml_pic_batch_run(pml_pic_batch *b, int32_t run) {
  if (!b || run < 0 || run >= (int32_t)b->runs.size()) return nullptr;
  return b->runs[run];
}

static int pml_pic_batch_set_launch_impl(pml_pic_batch *b, int32_t block_x, int32_t grid_blocks) {
  if (!b) return PML_PIC_E_INVALID_ARG;
  if (block_x != 32 && block_x != 64 && block_x != 128 && block_x != 256)
    return fail(&b->err, PML_PIC_E_INVALID_ARG, "block_x must be 32, 64, 128 or 256");
  if (grid_blocks < 0) return fail(&b->err, PML_PIC_E_INVALID_ARG, "grid_blocks must be >= 0");
  HIPCHK(b, hipStreamSynchronize(b->stream));
  batch_drop_graph(b);
  if (grid_blocks > 0) b->grid_blocks = grid_blocks;
  return batch_build_items(b, block_x);
}

static int pml_pic_batch_step_impl(pml_pic_batch *b, int32_t n_steps) {
  if (!b) return PML_PIC_E_INVALID_ARG;
  if (n_steps < 0) return fail(&b->err, PML_PIC_E_INVALID_ARG, "n_steps < 0");
  return b->prec == 64 ? batch_step_t<double>(b, n_steps) : batch_step_t<float>(b, n_steps);
}

static int pml_pic_batch_step_profiled_impl(pml_pic_batch *b, int32_t n_steps, double *phase_ms, int64_t *phase_calls) {
  if (!b || !phase_ms || !phase_calls) return PML_PIC_E_INVALID_ARG;
  if (n_steps < 0) return fail(&b->err, PML_PIC_E_INVALID_ARG, "n_steps < 0");
  PhaseTimer pt;
  pt.on = true;
  int rc = b->prec == 64 ? batch_step_t<double>(b, n_steps, &pt) : batch_step_t<float>(b, n_steps, &pt);
  hipError_t e = hipStreamSynchronize(b->stream);
  if (rc == PML_PIC_OK && (e != hipSuccess || pt.err != hipSuccess)) {
    b->err = std::string("HIP error: ") + hipGetErrorString(e != hipSuccess ? e : pt.err);
    rc = PML_PIC_E_HIP;
  }
  for (size_t k = 0; k < pt.phase.size() && 2 * k + 1 < pt.ev.size(); ++k) {
    float ms = 0.f;
    if (rc == PML_PIC_OK && hipEventElapsedTime(&ms, pt.ev[2 * k], pt.ev[2 * k + 1]) == hipSuccess) {
      phase_ms[pt.phase[k]] += ms;
      phase_calls[pt.phase[k]] += 1;
    }
  }
  for (hipEvent_t ev : pt.ev) (void)hipEventDestroy(ev);
  return rc;
}

const char *pml_pic_batch_last_error(const pml_pic_batch *b) { return b ? b->err.c_str() : g_create_error.c_str(); }

void pml_pic_batch_destroy(pml_pic_batch *b) {
  if (!b) return;
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  else (void)hipDeviceSynchronize();
  batch_drop_graph(b);
  for (pml_pic_handle *h : b->runs) delete h;
  delete b;
}

}  // extern "C"

// ===================================================================== C ABI
extern "C" {

static int pml_pic_workspace_size_impl(const pml_pic_params *params, size_t *bytes) {
  if (!bytes) return PML_PIC_E_INVALID_ARG;
  const int rc = validate(params, &g_create_error);
  if (rc) return rc;
  Layout L;
  make_layout(*params, L);
  *bytes = L.total;
  return PML_PIC_OK;
}

static int pml_pic_create_impl(const pml_pic_params *params, void *device_workspace, size_t bytes, void *stream,
                   pml_pic_handle **out) {
  const int rc = create_handle(params, device_workspace, bytes, stream, out, &g_create_error);
  if (rc != PML_PIC_OK || !(*out)->L.tile_push3) return rc;
  // the stream and events on which the dense tiles' push runs beside the tile-box push
  pml_pic_handle *h = *out;
  hipError_t e = hipStreamCreateWithFlags(&h->side, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&h->ev_fork, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&h->ev_join, hipEventDisableTiming);
  if (e != hipSuccess) {
    g_create_error = std::string("HIP error while creating the push stream: ") + hipGetErrorString(e);
    delete h;
    *out = nullptr;
    return PML_PIC_E_HIP;
  }
  return PML_PIC_OK;
}

static int pml_pic_add_particles_impl(pml_pic_handle *h, int64_t n, const double *x, const double *u, const double *w) {
  if (!h) return PML_PIC_E_INVALID_ARG;
  if (n < 0 || (n > 0 && (!x || !u || !w))) return fail(&h->err, PML_PIC_E_INVALID_ARG, "bad particle arrays");
  if (n == 0) return PML_PIC_OK;
  int32_t cnt;
  int rc = read_count(h, &cnt);
  if (rc) return rc;
  const int64_t first = h->sort_pending ? h->n_slots : std::min<int64_t>(cnt, h->n_slots);
  if (first + n > h->L.cap) return fail(&h->err, PML_PIC_E_CAPACITY, "max_particles exceeded");
  rc = h->p.precision == 64 ? write_particles<double>(h, first, n, nullptr, nullptr, x, u, w)
                            : write_particles<float>(h, first, n, nullptr, nullptr, x, u, w);
  if (rc) return rc;
  h->n_added += n;
  h->n_slots = first + n;
  rc = write_count(h, (int32_t)h->n_slots);
  if (rc) return rc;
  double *rs = h->at<double>(h->L.off_rho_static);
  if (h->p.precision == 64)
    launch_rho<double>(h->grid<double>(), h->parts<double>(h->cur), h->ctl(), (int)first, (int)h->n_slots, rs, -1.0, h->stream);
  else
    launch_rho<float>(h->grid<float>(), h->parts<float>(h->cur), h->ctl(), (int)first, (int)h->n_slots, rs, -1.0, h->stream);
  HIPCHK(h, hipGetLastError());
  HIPCHK(h, hipStreamSynchronize(h->stream));
  h->sort_pending = true;
  return PML_PIC_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ beam transport
namespace {

// Conductor flags per node: bit c (E_x, E_y, E_z, B_x, B_y, B_z) when sample c at that
// node index lies in the closed extent of a conductor cell -- along each axis the one cell
// a half-integer coordinate is inside, or the cells an integer coordinate borders.
void conductor_bits(const Layout &L, const uint8_t *cells, std::vector<uint8_t> &bits) {
  bits.assign((size_t)L.nelem, 0);
  auto cell_at = [&](int x, int y, int z) { return cells[((size_t)z * L.M[1] + y) * L.M[0] + x] != 0; };
  for (int k = 0; k <= L.M[2]; ++k)
    for (int j = 0; j <= L.M[1]; ++j)
      for (int i = 0; i <= L.M[0]; ++i) {
        const int id[3] = {i, j, k};
        uint8_t m = 0;
        for (int c = 0; c < 6; ++c) {
          const int a = c % 3;
          int lo[3], hi[3];
          bool any_cell = true;
          for (int d = 0; d < 3; ++d) {
            const bool half = c < 3 ? d == a : d != a;   // E_a half-integer along a, B_a across a
            lo[d] = half ? id[d] : id[d] - 1;
            hi[d] = id[d];
            lo[d] = std::max(lo[d], 0);
            hi[d] = std::min(hi[d], L.M[d] - 1);
            if (lo[d] > hi[d]) any_cell = false;
          }
          if (!any_cell) continue;
          bool in = false;
          for (int z = lo[2]; z <= hi[2] && !in; ++z)
            for (int y = lo[1]; y <= hi[1] && !in; ++y)
              for (int x = lo[0]; x <= hi[0] && !in; ++x) in = cell_at(x, y, z);
          if (in) m |= (uint8_t)(1u << c);
        }
        bits[(size_t)(L.base + i + (long)j * L.sy + (long)k * L.sz)] = m;
      }
}

template <typename T>
int upload_source(pml_pic_handle *h, const std::vector<int64_t> &order, const std::vector<double> &X,
                  const double *u, const double *w, int64_t first_id) {
  const Layout &L = h->L;
  const int dim = h->p.dim;
  const size_t n = order.size();
  std::vector<uint32_t> cell(n);
  std::vector<T> f[3], uu[3], ww(n);
  std::vector<int32_t> id(n);
  for (int d = 0; d < 3; ++d) { f[d].resize(n); uu[d].resize(n); }
  for (size_t q = 0; q < n; ++q) {
    const int64_t t = order[q];
    int ic[3];
    T ff[3];
    if (!to_cell<T>(L, dim, &X[3 * t], ic, ff)) {
      h->err = "source particle " + std::to_string(t) + " enters the box outside it along another axis";
      return PML_PIC_E_INVALID_ARG;
    }
    cell[q] = pack_cell(dim, ic[0], ic[1], ic[2]);
    for (int d = 0; d < 3; ++d) { f[d][q] = ff[d]; uu[d][q] = (T)u[3 * t + d]; }
    ww[q] = (T)w[t];
    id[q] = (int32_t)(first_id + t);
  }
  hipStream_t s = h->stream;
  HIPCHK(h, hipMemcpyAsync(h->at<uint32_t>(L.off_src_cell), cell.data(), 4 * n, hipMemcpyHostToDevice, s));
  for (int d = 0; d < dim; ++d)
    HIPCHK(h, hipMemcpyAsync(h->at<T>(L.off_src_f[d]), f[d].data(), sizeof(T) * n, hipMemcpyHostToDevice, s));
  for (int d = 0; d < 3; ++d)
    HIPCHK(h, hipMemcpyAsync(h->at<T>(L.off_src_u[d]), uu[d].data(), sizeof(T) * n, hipMemcpyHostToDevice, s));
  HIPCHK(h, hipMemcpyAsync(h->at<T>(L.off_src_w), ww.data(), sizeof(T) * n, hipMemcpyHostToDevice, s));
  HIPCHK(h, hipMemcpyAsync(h->at<int32_t>(L.off_src_id), id.data(), 4 * n, hipMemcpyHostToDevice, s));
  HIPCHK(h, hipStreamSynchronize(s));
  return PML_PIC_OK;
}

}  // namespace

extern "C" {

static int pml_pic_set_conductor_impl(pml_pic_handle *h, const uint8_t *cells) {
  if (!h) return PML_PIC_E_INVALID_ARG;
  if (!h->p.conductor) return fail(&h->err, PML_PIC_E_INVALID_ARG, "created without params.conductor");
  HIPCHK(h, hipStreamSynchronize(h->stream));
  if (!cells) {
    h->has_cond = false;
    return PML_PIC_OK;
  }
  std::vector<uint8_t> bits;
  conductor_bits(h->L, cells, bits);
  HIPCHK(h, hipMemcpy(h->at<uint8_t>(h->L.off_cmask), bits.data(), bits.size(), hipMemcpyHostToDevice));
  h->has_cond = true;
  if (h->p.precision == 64) launch_apply_conductor<double>(h->grid<double>(), h->fields<double>(), h->stream);
  else launch_apply_conductor<float>(h->grid<float>(), h->fields<float>(), h->stream);
  HIPCHK(h, hipGetLastError());
  HIPCHK(h, hipStreamSynchronize(h->stream));
  return PML_PIC_OK;
}

static int pml_pic_set_source_impl(pml_pic_handle *h, int64_t n, const double *x, const double *u, const double *w, int32_t axis) {
  if (!h) return PML_PIC_E_INVALID_ARG;
  const int dim = h->p.dim;
  if (n < 0 || (n > 0 && (!x || !u || !w))) return fail(&h->err, PML_PIC_E_INVALID_ARG, "bad source arrays");
  if (axis < 0 || axis >= dim) return fail(&h->err, PML_PIC_E_INVALID_ARG, "axis out of range");
  if (n > h->L.src_cap) return fail(&h->err, PML_PIC_E_CAPACITY, "more source particles than params.max_source");
  if (h->n_slots + n > h->L.cap) return fail(&h->err, PML_PIC_E_CAPACITY, "max_particles too small for the source");
  // injection step and position of each particle (FP64): the first step start m >= 0 at
  // which its ballistic position lies at or beyond the outer wall of the low layer
  const double wall = -(double)h->p.pml[axis][0] * h->p.dx[axis];
  const double dt = h->p.dt;
  std::vector<int64_t> m(n);
  std::vector<double> X(3 * (size_t)n, 0.0);
  for (int64_t t = 0; t < n; ++t) {
    const double *ut = u + 3 * t;
    const double gam = std::sqrt(1.0 + ut[0] * ut[0] + ut[1] * ut[1] + ut[2] * ut[2]);
    const double va = ut[axis] / gam, xa = x[dim * t + axis];
    if (!std::isfinite(xa) || !std::isfinite(gam) || !std::isfinite(w[t]))
      return fail(&h->err, PML_PIC_E_INVALID_ARG, "non-finite source particle");
    int64_t k = 0;
    if (xa < wall) {
      if (!(va > 0.0)) return fail(&h->err, PML_PIC_E_INVALID_ARG, "a source particle never reaches the box");
      const double need = (wall - xa) / (va * dt);
      if (!(need < 1e15)) return fail(&h->err, PML_PIC_E_INVALID_ARG, "a source particle never reaches the box");
      k = std::max<int64_t>(1, (int64_t)std::ceil(need));
      while (xa + (double)k * dt * va < wall) ++k;
      while (k > 1 && xa + (double)(k - 1) * dt * va >= wall) --k;
    }
    m[t] = k;
    for (int d = 0; d < dim; ++d) {
      const double xd = x[dim * t + d] + (double)k * dt * (ut[d] / gam);
      X[3 * t + d] = xd / h->p.dx[d] + h->p.pml[d][0];
    }
  }
  std::vector<int64_t> order(n);
  for (int64_t t = 0; t < n; ++t) order[t] = t;
  std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) { return m[a] < m[b]; });
  HIPCHK(h, hipStreamSynchronize(h->stream));
  const int rc = n == 0 ? 0
                        : (h->p.precision == 64 ? upload_source<double>(h, order, X, u, w, h->n_added)
                                                : upload_source<float>(h, order, X, u, w, h->n_added));
  if (rc) return rc;
  h->src_steps.resize(n);
  for (int64_t q = 0; q < n; ++q) h->src_steps[q] = h->step + m[order[q]];
  h->src_next = 0;
  h->n_added += n;
  return PML_PIC_OK;
}

static int pml_pic_slab_moments_impl(pml_pic_handle *h, int32_t axis, int32_t n_slabs, const double *edges, double *out) {
  if (!h) return PML_PIC_E_INVALID_ARG;
  if (axis < 0 || axis >= h->p.dim) return fail(&h->err, PML_PIC_E_INVALID_ARG, "axis out of range");
  if (n_slabs < 1 || n_slabs > SLAB_MAX) return fail(&h->err, PML_PIC_E_INVALID_ARG, "n_slabs must be in [1,64]");
  if (!edges || !out) return fail(&h->err, PML_PIC_E_INVALID_ARG, "edges and out are required");
  for (int k = 0; k < n_slabs; ++k)
    if (!(edges[k] < edges[k + 1])) return fail(&h->err, PML_PIC_E_INVALID_ARG, "edges must increase");
  double *dev = h->at<double>(h->L.off_slab);
  double *dsum = dev + SLAB_MAX + 1;
  hipStream_t s = h->stream;
  HIPCHK(h, hipMemcpyAsync(dev, edges, sizeof(double) * (n_slabs + 1), hipMemcpyHostToDevice, s));
  if (h->p.precision == 64)
    launch_slab_moments<double>(h->grid<double>(), h->parts<double>(h->cur), h->ctl().count, (int)h->n_slots, axis,
                                h->p.dx[axis], n_slabs, dev, dsum, s);
  else
    launch_slab_moments<float>(h->grid<float>(), h->parts<float>(h->cur), h->ctl().count, (int)h->n_slots, axis,
                               h->p.dx[axis], n_slabs, dev, dsum, s);
  HIPCHK(h, hipGetLastError());
  HIPCHK(h, hipMemcpyAsync(out, dsum, sizeof(double) * 5 * n_slabs, hipMemcpyDeviceToHost, s));
  HIPCHK(h, hipStreamSynchronize(s));
  return PML_PIC_OK;
}

static int pml_pic_set_particles_impl(pml_pic_handle *h, int64_t n, const int64_t *ids, const double *X, const double *u,
                          const double *w) {
  if (!h) return PML_PIC_E_INVALID_ARG;
  if (n < 0 || (n > 0 && (!ids || !X || !u || !w))) return fail(&h->err, PML_PIC_E_INVALID_ARG, "bad particle arrays");
  if (n > h->L.cap) return fail(&h->err, PML_PIC_E_CAPACITY, "max_particles exceeded");
  HIPCHK(h, hipStreamSynchronize(h->stream));
  int rc = n == 0 ? 0
                  : (h->p.precision == 64 ? write_particles<double>(h, 0, n, ids, X, nullptr, u, w)
                                          : write_particles<float>(h, 0, n, ids, X, nullptr, u, w));
  if (rc) return rc;
  h->n_slots = n;
  h->tail_n = 0;   // the sort below takes every particle
  for (int64_t t = 0; t < n; ++t) h->n_added = std::max<int64_t>(h->n_added, ids[t] + 1);
  rc = write_count(h, (int32_t)n);
  if (rc) return rc;
  h->sort_pending = true;
  return PML_PIC_OK;
}

// Bounds-checked builds: after a call that ran kernels, any CHECK_* bit the kernels set
// becomes PML_PIC_E_HIP with a message (and the word is cleared); other builds return rc.
static int report_checks(pml_pic_handle *h, int rc) {
#ifdef PMLPIC_CHECK
  if (!h) return rc;
  uint32_t bits = 0;
  if (hipStreamSynchronize(h->stream) != hipSuccess ||
      hipMemcpy(&bits, h->ws + h->L.off_check, 4, hipMemcpyDeviceToHost) != hipSuccess)
    return fail(&h->err, PML_PIC_E_HIP, "bounds-check word unreadable");
  if (bits) {
    (void)hipMemset(h->ws + h->L.off_check, 0, 4);
    char msg[160];
    snprintf(msg, sizeof msg, "bounds check failed (bits 0x%x: 1 sample index, 2 global current, 4 LDS box, 8 sort key)",
             bits);
    return fail(&h->err, PML_PIC_E_HIP, msg);
  }
#endif
  return rc;
}

static int pml_pic_step_impl(pml_pic_handle *h, int32_t n_steps) {
  if (!h) return PML_PIC_E_INVALID_ARG;
  if (n_steps < 0) return fail(&h->err, PML_PIC_E_INVALID_ARG, "n_steps < 0");
  PhaseTimer pt;
  return h->p.precision == 64 ? step_t<double>(h, n_steps, pt) : step_t<float>(h, n_steps, pt);
}

static int pml_pic_step_profiled_impl(pml_pic_handle *h, int32_t n_steps, double *phase_ms, int64_t *phase_calls) {
  if (!h || !phase_ms || !phase_calls) return PML_PIC_E_INVALID_ARG;
  if (n_steps < 0) return fail(&h->err, PML_PIC_E_INVALID_ARG, "n_steps < 0");
  PhaseTimer pt;
  pt.h = h;
  pt.on = true;
  int rc = h->p.precision == 64 ? step_t<double>(h, n_steps, pt) : step_t<float>(h, n_steps, pt);
  hipError_t e = hipStreamSynchronize(h->stream);
  if (rc == PML_PIC_OK && e != hipSuccess) {
    h->err = std::string("HIP error: ") + hipGetErrorString(e);
    rc = PML_PIC_E_HIP;
  }
  for (size_t k = 0; k < pt.phase.size() && 2 * k + 1 < pt.ev.size(); ++k) {
    float ms = 0.f;
    if (rc == PML_PIC_OK && hipEventElapsedTime(&ms, pt.ev[2 * k], pt.ev[2 * k + 1]) == hipSuccess) {
      phase_ms[pt.phase[k]] += ms;
      phase_calls[pt.phase[k]] += 1;
    }
  }
  for (hipEvent_t ev : pt.ev) (void)hipEventDestroy(ev);
  return rc;
}

static int field_error_check(pml_pic_handle *h, pml_pic_handle *ref, double *num, double *den) {
  if (!h || !ref || !num || !den) return PML_PIC_E_INVALID_ARG;
  const pml_pic_params &a = h->p, &b = ref->p;
  if (a.dim != b.dim || a.precision != b.precision)
    return fail(&h->err, PML_PIC_E_INVALID_ARG, "the reference needs the same dim and precision");
  for (int d = 0; d < a.dim; ++d)
    if (a.dx[d] != b.dx[d] || a.pml[d][0] != b.pml[d][0] || b.n[d] + b.pml[d][1] < a.n[d])
      return fail(&h->err, PML_PIC_E_INVALID_ARG,
                  "the reference needs the same cells and low PML and must cover the physical box");
  return PML_PIC_OK;
}

static int pml_pic_field_error_impl(pml_pic_handle *h, pml_pic_handle *ref, double *num, double *den) {
  const int rc = field_error_check(h, ref, num, den);
  if (rc) return rc;
  HIPCHK(h, hipStreamSynchronize(ref->stream));
  const DiagWork dw = h->diagwork();
  if (h->p.precision == 64)
    launch_field_error<double>(h->grid<double>(), h->fields<double>(), ref->grid<double>(), ref->fields<double>(),
                               dw.partial, dw.result, h->stream);
  else
    launch_field_error<float>(h->grid<float>(), h->fields<float>(), ref->grid<float>(), ref->fields<float>(),
                              dw.partial, dw.result, h->stream);
  HIPCHK(h, hipGetLastError());
  double r[2];
  HIPCHK(h, hipMemcpyAsync(r, dw.result, sizeof(r), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  *num = r[0];
  *den = r[1];
  return PML_PIC_OK;
}

// The same reduction with its partial sums in the library's static device scratch (no
// workspace, no allocation of any kind on the device).
static int pml_pic_field_error_noalloc_impl(pml_pic_handle *h, pml_pic_handle *ref, double *num, double *den) {
  const int rc = field_error_check(h, ref, num, den);
  if (rc) return rc;
  double *sc = nullptr;
  HIPCHK(h, field_error_scratch(&sc));
  HIPCHK(h, hipStreamSynchronize(ref->stream));
  const bool ok = h->p.precision == 64
                      ? launch_field_error_scratch<double>(h->grid<double>(), h->fields<double>(), ref->grid<double>(),
                                                           ref->fields<double>(), sc, h->stream)
                      : launch_field_error_scratch<float>(h->grid<float>(), h->fields<float>(), ref->grid<float>(),
                                                          ref->fields<float>(), sc, h->stream);
  if (!ok)
    return fail(&h->err, PML_PIC_E_INVALID_ARG,
                "grid too wide for the static scratch of pml_pic_field_error_noalloc (" +
                    std::to_string(field_error_scratch_pairs()) + " partial sums)");
  HIPCHK(h, hipGetLastError());
  double r[2];
  HIPCHK(h, hipMemcpyAsync(r, sc, sizeof(r), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  *num = r[0];
  *den = r[1];
  return PML_PIC_OK;
}

static int pml_pic_diagnose_impl(pml_pic_handle *h, pml_pic_diag *out) {
  if (!h || !out) return PML_PIC_E_INVALID_ARG;
  return h->p.precision == 64 ? diagnose_t<double>(h, out) : diagnose_t<float>(h, out);
}

static int pml_pic_grid_shape_impl(const pml_pic_handle *h, int32_t nn[3], int64_t *n_samples) {
  if (!h || !nn || !n_samples) return PML_PIC_E_INVALID_ARG;
  for (int d = 0; d < 3; ++d) nn[d] = h->L.nn[d];
  *n_samples = (int64_t)h->L.nn[0] * h->L.nn[1] * h->L.nn[2];
  return PML_PIC_OK;
}

static int64_t n_samples_of(const pml_pic_handle *h) { return (int64_t)h->L.nn[0] * h->L.nn[1] * h->L.nn[2]; }

static int pml_pic_get_fields_impl(pml_pic_handle *h, double *host, int64_t count) {
  if (!h || !host) return PML_PIC_E_INVALID_ARG;
  if (count < 12 * n_samples_of(h)) return fail(&h->err, PML_PIC_E_INVALID_ARG, "field buffer too small");
  return h->p.precision == 64 ? get_fields_t<double>(h, host) : get_fields_t<float>(h, host);
}

static int pml_pic_set_fields_impl(pml_pic_handle *h, const double *host, int64_t count) {
  if (!h || !host) return PML_PIC_E_INVALID_ARG;
  if (count < 12 * n_samples_of(h)) return fail(&h->err, PML_PIC_E_INVALID_ARG, "field buffer too small");
  return h->p.precision == 64 ? set_fields_t<double>(h, host) : set_fields_t<float>(h, host);
}

static int pml_pic_get_current_impl(pml_pic_handle *h, double *host, int64_t count) {
  if (!h || !host) return PML_PIC_E_INVALID_ARG;
  if (count < 3 * n_samples_of(h)) return fail(&h->err, PML_PIC_E_INVALID_ARG, "current buffer too small");
  return h->p.precision == 64 ? get_current_t<double>(h, host) : get_current_t<float>(h, host);
}

static int pml_pic_get_rho_static_impl(pml_pic_handle *h, double *host, int64_t count) {
  if (!h || !host) return PML_PIC_E_INVALID_ARG;
  const Layout &L = h->L;
  if (count < n_samples_of(h)) return fail(&h->err, PML_PIC_E_INVALID_ARG, "buffer too small");
  std::vector<double> buf(L.nelem);
  HIPCHK(h, hipStreamSynchronize(h->stream));
  HIPCHK(h, hipMemcpy(buf.data(), h->at<double>(L.off_rho_static), 8 * L.nelem, hipMemcpyDeviceToHost));
  for (int k = 0; k < L.nn[2]; ++k)
    for (int j = 0; j < L.nn[1]; ++j)
      for (int i = 0; i < L.nn[0]; ++i)
        host[((size_t)k * L.nn[1] + j) * L.nn[0] + i] = buf[L.base + i + j * L.sy + k * L.sz];
  return PML_PIC_OK;
}

static int pml_pic_set_rho_static_impl(pml_pic_handle *h, const double *host, int64_t count) {
  if (!h || !host) return PML_PIC_E_INVALID_ARG;
  const Layout &L = h->L;
  if (count < n_samples_of(h)) return fail(&h->err, PML_PIC_E_INVALID_ARG, "buffer too small");
  std::vector<double> buf(L.nelem, 0.0);
  for (int k = 0; k < L.nn[2]; ++k)
    for (int j = 0; j < L.nn[1]; ++j)
      for (int i = 0; i < L.nn[0]; ++i)
        buf[L.base + i + j * L.sy + k * L.sz] = host[((size_t)k * L.nn[1] + j) * L.nn[0] + i];
  HIPCHK(h, hipStreamSynchronize(h->stream));
  HIPCHK(h, hipMemcpy(h->at<double>(L.off_rho_static), buf.data(), 8 * L.nelem, hipMemcpyHostToDevice));
  return PML_PIC_OK;
}

static int pml_pic_sort_particles_impl(pml_pic_handle *h, int32_t tile[3], uint32_t *key_start, int64_t cap,
                                       int64_t *n_keys) {
  if (!h) return PML_PIC_E_INVALID_ARG;
  if (key_start && cap < (int64_t)h->L.nkeys + 1)
    return fail(&h->err, PML_PIC_E_INVALID_ARG, "key_start needs n_keys + 1 entries");
  if (h->p.flags & PML_PIC_FLAG_NO_SORT)
    return fail(&h->err, PML_PIC_E_INVALID_ARG, "the run was created with PML_PIC_FLAG_NO_SORT");
  if (tile)
    for (int d = 0; d < 3; ++d) tile[d] = h->L.tile[d];
  if (n_keys) *n_keys = h->L.nkeys;
  const int ns = (int)h->n_slots;
  if (ns > 0) {
    if (h->p.precision == 64) sort_now<double>(h, h->ctl(), ns);
    else sort_now<float>(h, h->ctl(), ns);
    HIPCHK(h, hipGetLastError());
  }
  if (key_start) {
    const Layout &L = h->L;
    if (ns > 0) {
      HIPCHK(h, hipMemcpyAsync(key_start, h->at<uint32_t>(L.off_counts), 4 * ((size_t)L.nkeys + 1),
                               hipMemcpyDeviceToHost, h->stream));
    } else {
      std::fill(key_start, key_start + L.nkeys + 1, 0u);
    }
  }
  HIPCHK(h, hipStreamSynchronize(h->stream));
  return PML_PIC_OK;
}

static int pml_pic_num_particles_impl(pml_pic_handle *h, int64_t *n) {
  if (!h || !n) return PML_PIC_E_INVALID_ARG;
  pml_pic_diag d;
  const int rc = pml_pic_diagnose(h, &d);
  if (rc && rc != PML_PIC_E_NONFINITE) return rc;
  *n = d.n_particles;
  return PML_PIC_OK;
}

static int pml_pic_get_particles_impl(pml_pic_handle *h, int64_t cap, int64_t *ids, double *X, double *u, double *w,
                          int64_t *n_out) {
  if (!h || !n_out || (cap > 0 && (!ids || !X || !u || !w))) return PML_PIC_E_INVALID_ARG;
  return h->p.precision == 64 ? get_particles_t<double>(h, cap, ids, X, u, w, n_out)
                              : get_particles_t<float>(h, cap, ids, X, u, w, n_out);
}

const char *pml_pic_last_error(const pml_pic_handle *h) {
  return h ? h->err.c_str() : g_create_error.c_str();
}

void pml_pic_destroy(pml_pic_handle *h) {
  if (!h) return;
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  else (void)hipDeviceSynchronize();
  delete h;
}

}  // extern "C"

// ===================================================================== adjoint (host side)
namespace {

template <typename T>
Fields<T> fields_at(const pml_pic_handle *h, char *base) {
  const size_t fb = sizeof(T) * (size_t)h->L.nelem;
  Fields<T> F;
  for (int a = 0; a < 3; ++a) {
    F.E[a] = (T *)(base + a * fb);
    F.B[a] = (T *)(base + (3 + a) * fb);
    F.Ea[a] = (T *)(base + (6 + a) * fb);
    F.Ba[a] = (T *)(base + (9 + a) * fb);
    F.J[a] = nullptr;
  }
  return F;
}

char *ckpt_ptr(pml_pic_handle *h, int c) { return h->ws + h->L.off_ckpt + (size_t)c * h->L.ckpt_stride; }

int save_ckpt(pml_pic_handle *h, int c) {
  const Layout &L = h->L;
  char *dst = ckpt_ptr(h, c);
  hipStream_t s = h->stream;
  HIPCHK(h, hipMemcpyAsync(dst, h->ws + h->foff(0), L.fields_bytes, hipMemcpyDeviceToDevice, s));
  HIPCHK(h, hipMemcpyAsync(dst + L.fields_bytes, h->ws + L.off_cell[h->cur], L.parts_bytes, hipMemcpyDeviceToDevice, s));
  HIPCHK(h, hipMemcpyAsync(dst + L.fields_bytes + L.parts_bytes, h->ws + L.off_count, 4, hipMemcpyDeviceToDevice, s));
  HIPCHK(h, hipMemcpyAsync(dst + L.fields_bytes + L.parts_bytes + 256, h->ws + L.off_pushes, 8 * N_PUSH_COUNTERS,
                           hipMemcpyDeviceToDevice, s));
  if ((int)h->ckpt_meta.size() < L.nckpt) h->ckpt_meta.resize(L.nckpt);
  h->ckpt_meta[c] = {h->cur, h->n_slots, h->n_added, h->step, h->since_sort, h->sort_pending};
  return PML_PIC_OK;
}

int restore_ckpt(pml_pic_handle *h, int c) {
  const Layout &L = h->L;
  const pml_pic_handle::CkptMeta m = h->ckpt_meta[c];
  h->cur = m.cur; h->n_slots = m.n_slots; h->n_added = m.n_added; h->step = m.step;
  // the tiled step needs the key ranges of the sort that ordered the restored buffer
  h->since_sort = m.since_sort; h->sort_pending = true;
  const char *src = ckpt_ptr(h, c);
  hipStream_t s = h->stream;
  HIPCHK(h, hipMemcpyAsync(h->ws + h->foff(0), src, L.fields_bytes, hipMemcpyDeviceToDevice, s));
  HIPCHK(h, hipMemcpyAsync(h->ws + L.off_cell[h->cur], src + L.fields_bytes, L.parts_bytes, hipMemcpyDeviceToDevice, s));
  HIPCHK(h, hipMemcpyAsync(h->ws + L.off_count, src + L.fields_bytes + L.parts_bytes, 4, hipMemcpyDeviceToDevice, s));
  HIPCHK(h, hipMemcpyAsync(h->ws + L.off_pushes, src + L.fields_bytes + L.parts_bytes + 256, 8 * N_PUSH_COUNTERS,
                           hipMemcpyDeviceToDevice, s));
  return PML_PIC_OK;
}

int check_adjoint(pml_pic_handle *h) {
  if (h->L.seg <= 0) return fail(&h->err, PML_PIC_E_INVALID_ARG, "created without adjoint_segment");
  if (h->p.push != 0 && h->n_added > h->L.cap)
    return fail(&h->err, PML_PIC_E_INVALID_ARG, "the pushed adjoint needs particle ids below max_particles");
  if (h->p.alpha_mode == PML_ALPHA_ZERO)
    return fail(&h->err, PML_PIC_E_INVALID_ARG, "alpha_mode 0 is not differentiable in the profile");
  if (h->p.alpha_mode == PML_ALPHA_WEIGHT)
    return fail(&h->err, PML_PIC_E_INVALID_ARG, "the adjoint does not cover per-particle weight damping");
  if (h->p.solver != PML_PIC_SOLVER_YEE || h->p.filter_passes > 0)
    return fail(&h->err, PML_PIC_E_INVALID_ARG, "the adjoint covers the Yee solver without current filter");
  if (kernel_alpha_mode(h->p) != h->p.alpha_mode || h->p.conductor || h->p.max_source > 0)
    return fail(&h->err, PML_PIC_E_INVALID_ARG, "the adjoint covers neither per-face modes, conductors nor sources");
  return PML_PIC_OK;
}

template <typename T>
int forward_ckpt_t(pml_pic_handle *h, int n, double *U) {
  int rc = check_adjoint(h);
  if (rc) return rc;
  const int seg = h->L.seg;
  if (n < 1 || (n + seg - 1) / seg > h->L.nckpt - 1)
    return fail(&h->err, PML_PIC_E_INVALID_ARG, "n_steps exceeds adjoint_checkpoints * adjoint_segment");
  PhaseTimer pt;
  for (int c = 0; c * seg < n; ++c) {
    if ((rc = save_ckpt(h, c))) return rc;
    if ((rc = step_t<T>(h, std::min(seg, n - c * seg), pt))) return rc;
  }
  if ((rc = save_ckpt(h, h->L.nckpt - 1))) return rc;
  h->fwd_steps = n;
  h->padj_valid = false;
  pml_pic_diag d;
  rc = diagnose_t<T>(h, &d);
  if (rc && rc != PML_PIC_E_NONFINITE) return rc;
  *U = d.u_interior;
  return rc;
}

// dg/dsigma for g = (1 - exp(-sigma tau))/sigma, stable for small sigma tau
double dg_dsigma(double sig, double tau) {
  const double x = sig * tau;
  if (x < 1e-3) return tau * tau * (-0.5 + x / 3.0 - x * x / 8.0 + x * x * x / 30.0);
  const double e = std::exp(-x);
  return (tau * e - (-std::expm1(-x)) / sig) / sig;
}

void chain_rule(const pml_pic_handle *h, const std::vector<double> &Gv, double *grad) {
  const pml_pic_params &p = h->p;
  const Layout &L = h->L;
  const int NK = 8;   // gradient kinds, in the order of adjoint.hip
  auto Gat = [&](int axis, int kind, int i) { return Gv[((size_t)axis * NK + kind) * L.ntab + i + G]; };
  for (int k = 0; k < 16 * p.dim + 1; ++k) grad[k] = 0.0;
  for (int d = 0; d < p.dim; ++d) {
    for (int i = -G; i <= L.M[d] + G; ++i) {
      for (int centre = 0; centre < 2; ++centre) {
        const double X = i + 0.5 * centre;
        if (X < 0.0 || X > (double)L.M[d]) continue;
        double thick;
        const double dep = pml_depth(p, d, X, &thick);
        if (dep <= 0.0 || thick <= 0.0) continue;
        double sig, phi;
        profile(p, d, X, &sig, &phi);
        const double r = dep / thick;
        double dUdsig, dUdalpha;
        if (!centre) {
          const double tau = p.dt, e = std::exp(-sig * tau);
          const double dg = dg_dsigma(sig, tau);
          dUdsig = Gat(d, 0, i) * (-tau * e) + Gat(d, 1, i) * dg + Gat(d, 2, i) * dg / p.dx[d] + Gat(d, 7, i);
          dUdalpha = Gat(d, 5, i);
        } else {
          const double tau = 0.5 * p.dt, e = std::exp(-sig * tau);
          const double dg = dg_dsigma(sig, tau);
          dUdsig = Gat(d, 3, i) * (-tau * e) + Gat(d, 4, i) * dg / p.dx[d];
          dUdalpha = Gat(d, 6, i);
        }
        double alpha = 1.0;
        if (p.alpha_mode == PML_ALPHA_DAMPED) alpha = std::exp(-p.damping_scale * phi);
        else dUdalpha = 0.0;
        double rk = 1.0;
        for (int k = 0; k < p.n_sigma_coef; ++k) {
          const double dphi = thick * rk * r / (k + 1);
          grad[16 * d + k] += dUdsig * rk + dUdalpha * (-p.damping_scale * alpha * dphi);
          rk *= r;
        }
        grad[16 * p.dim] += dUdalpha * (-phi * alpha);
      }
    }
  }
}

template <typename T>
int backward_t(pml_pic_handle *h, const double *seed, double *lambda_out, double *grad) {
  int rc = check_adjoint(h);
  if (rc) return rc;
  if (h->fwd_steps < 1) return fail(&h->err, PML_PIC_E_INVALID_ARG, "no pml_pic_forward_ckpt run to reverse");
  const Layout &L = h->L;
  const Grid<T> g = h->grid<T>();
  hipStream_t s = h->stream;
  const size_t fb = sizeof(T) * (size_t)L.nelem;
  const int n = (int)h->fwd_steps, seg = L.seg;
  double *Gacc = h->at<double>(L.off_grad);
  HIPCHK(h, hipMemsetAsync(Gacc, 0, 8 * 3 * 8 * (size_t)L.ntab, s));
  AdjFields<T> A;
  for (int c = 0; c < 6; ++c) {
    A.LT[c] = (T *)(h->ws + L.off_adj + c * fb);
    A.LA[c] = (T *)(h->ws + L.off_adj + (6 + c) * fb);
  }
  HIPCHK(h, hipMemsetAsync(h->ws + L.off_adj, 0, 12 * fb, s));
  const bool pushed = h->p.push != 0;
  T *LJ[3] = {nullptr, nullptr, nullptr};
  PartAdj<T> PA{};
  if (pushed) {   // the current's adjoint is 0 outside the samples E updates; particles start at 0
    const size_t cap = (size_t)std::max<int64_t>(L.cap, 1);
    for (int a = 0; a < 3; ++a) LJ[a] = (T *)(h->ws + L.off_lj + a * fb);
    for (int d = 0; d < 3; ++d) {
      PA.lf[d] = (T *)(h->ws + L.off_padj + d * sizeof(T) * cap);
      PA.lu[d] = (T *)(h->ws + L.off_padj + (3 + d) * sizeof(T) * cap);
    }
    HIPCHK(h, hipMemsetAsync(h->ws + L.off_lj, 0, 3 * fb, s));
    HIPCHK(h, hipMemsetAsync(h->ws + L.off_padj, 0, 6 * sizeof(T) * cap, s));
  }
  h->padj_valid = false;
  if ((rc = restore_ckpt(h, L.nckpt - 1))) return rc;
  const size_t ns = (size_t)L.nn[0] * L.nn[1] * L.nn[2];
  if (!seed) {
    launch_adj_seed_energy<T>(g, h->fields<T>(), A, s);
  } else {   // 12-part seed -> LT / LA
    std::vector<T> lt(L.nelem), la(L.nelem);
    for (int c = 0; c < 6; ++c) {
      std::fill(lt.begin(), lt.end(), T(0));
      std::fill(la.begin(), la.end(), T(0));
      const int up = unsplit_part(h->p, c);
      const double *s0 = seed + (size_t)(2 * c) * ns, *s1 = seed + (size_t)(2 * c + 1) * ns;
      for (int k = 0; k < L.nn[2]; ++k)
        for (int j = 0; j < L.nn[1]; ++j)
          for (int i = 0; i < L.nn[0]; ++i) {
            const size_t o = ((size_t)k * L.nn[1] + j) * L.nn[0] + i;
            const long q = L.base + i + j * L.sy + k * L.sz;
            const int id[3] = {i, j, k};
            if (up < 0 && split_active(h, c, id)) { lt[q] = (T)s1[o]; la[q] = (T)(s0[o] - s1[o]); }
            else lt[q] = (T)(up == 1 ? s1[o] : s0[o]);
          }
      HIPCHK(h, hipMemcpyAsync(A.LT[c], lt.data(), fb, hipMemcpyHostToDevice, s));
      HIPCHK(h, hipMemcpyAsync(A.LA[c], la.data(), fb, hipMemcpyHostToDevice, s));
      HIPCHK(h, hipStreamSynchronize(s));
    }
  }
  char *seg_state = h->ws + L.off_seg_state;
  char *seg_J = h->ws + L.off_seg_J;
  char *bh = h->ws + L.off_bh;
  const int nseg = (n + seg - 1) / seg;
  PhaseTimer pt;
  for (int c = nseg - 1; c >= 0; --c) {
    if ((rc = restore_ckpt(h, c))) return rc;
    const int len = std::min(seg, n - c * seg);
    h->snap_state.clear();
    h->snap_J.clear();
    for (int k = 0; k < len; ++k) {
      h->snap_state.push_back(seg_state + (size_t)k * L.fields_bytes);
      h->snap_J.push_back(seg_J + (size_t)k * L.J_bytes);
      if (pushed) {
        h->snap_parts.push_back(h->ws + L.off_seg_parts + (size_t)k * L.parts_bytes);
        h->snap_count.push_back(h->ws + L.off_seg_count + 4 * (size_t)k);
        h->snap_ns.push_back(0);
      }
    }
    rc = step_t<T>(h, len, pt);
    const std::vector<int64_t> seg_ns = h->snap_ns;
    h->snap_state.clear();
    h->snap_J.clear();
    h->snap_parts.clear();
    h->snap_count.clear();
    h->snap_ns.clear();
    if (rc) return rc;
    HIPCHK(h, hipMemcpyAsync(seg_state + (size_t)len * L.fields_bytes, h->ws + h->foff(0), L.fields_bytes,
                             hipMemcpyDeviceToDevice, s));
    for (int k = len - 1; k >= 0; --k) {
      const Fields<T> Fn = fields_at<T>(h, seg_state + (size_t)k * L.fields_bytes);
      const Fields<T> Fn1 = fields_at<T>(h, seg_state + (size_t)(k + 1) * L.fields_bytes);
      // B^{n+1/2} from the stored B^n, E^n
      HIPCHK(h, hipMemcpyAsync(bh, Fn.B[0], 3 * fb, hipMemcpyDeviceToDevice, s));
      HIPCHK(h, hipMemcpyAsync(bh + 3 * fb, Fn.Ba[0], 3 * fb, hipMemcpyDeviceToDevice, s));
      Fields<T> FH = Fn;
      for (int a = 0; a < 3; ++a) { FH.B[a] = (T *)(bh + a * fb); FH.Ba[a] = (T *)(bh + (3 + a) * fb); }
      launch_update_B<T>(g, FH, true, s);
      T *J[3];
      for (int a = 0; a < 3; ++a) J[a] = (T *)(seg_J + (size_t)k * L.J_bytes + a * fb);
      Fields<T> F3 = FH;        // second B half step: B^{n+1/2} -> B^{n+1} with E^{n+1}
      for (int a = 0; a < 3; ++a) F3.E[a] = Fn1.E[a];
      launch_adj_B_half<T>(g, A, F3, Gacc, s);
      launch_adj_E<T>(g, A, FH, J, h->p.alpha_mode, Gacc, pushed ? LJ : nullptr, s);   // E^n -> E^{n+1}
      launch_adj_B_half<T>(g, A, Fn, Gacc, s);                 // first half step: B^n, E^n
      if (pushed) {   // gather_push and deposit_current of step k, from its particles and E^n, B^n
        const size_t rel = (size_t)k * L.parts_bytes - L.off_cell[0] + L.off_seg_parts;
        Parts<T> Pk = h->parts<T>(0);
        Pk.cell = (uint32_t *)(h->ws + rel + L.off_cell[0]);
        for (int d = 0; d < 3; ++d) {
          Pk.f[d] = d < h->p.dim ? (T *)(h->ws + rel + L.off_f[0][d]) : nullptr;
          Pk.u[d] = (T *)(h->ws + rel + L.off_u[0][d]);
        }
        Pk.w = (T *)(h->ws + rel + L.off_w[0]);
        Pk.lam = nullptr;
        Pk.id = (int32_t *)(h->ws + rel + L.off_id[0]);
        launch_adj_particles<T>(g, Fn, Pk, (const int32_t *)(h->ws + L.off_seg_count + 4 * (size_t)k),
                                (int)seg_ns[k], (int)L.cap, A, LJ, PA, s);
      }
    }
    HIPCHK(h, hipGetLastError());
  }
  if ((rc = restore_ckpt(h, L.nckpt - 1))) return rc;
  h->padj_valid = pushed;
  std::vector<double> Gv((size_t)3 * 8 * L.ntab);
  HIPCHK(h, hipMemcpyAsync(Gv.data(), Gacc, 8 * Gv.size(), hipMemcpyDeviceToHost, s));
  HIPCHK(h, hipStreamSynchronize(s));
  chain_rule(h, Gv, grad);
  if (lambda_out) {
    std::vector<T> lt(L.nelem), la(L.nelem);
    for (int c = 0; c < 6; ++c) {
      HIPCHK(h, hipMemcpy(lt.data(), A.LT[c], fb, hipMemcpyDeviceToHost));
      HIPCHK(h, hipMemcpy(la.data(), A.LA[c], fb, hipMemcpyDeviceToHost));
      const int up = unsplit_part(h->p, c);
      double *o0 = lambda_out + (size_t)(2 * c) * ns, *o1 = lambda_out + (size_t)(2 * c + 1) * ns;
      for (int k = 0; k < L.nn[2]; ++k)
        for (int j = 0; j < L.nn[1]; ++j)
          for (int i = 0; i < L.nn[0]; ++i) {
            const size_t o = ((size_t)k * L.nn[1] + j) * L.nn[0] + i;
            const long q = L.base + i + j * L.sy + k * L.sz;
            const int id[3] = {i, j, k};
            const double vt = (double)lt[q];
            if (up < 0 && split_active(h, c, id)) { o0[o] = vt + (double)la[q]; o1[o] = vt; }
            else { o0[o] = vt; o1[o] = vt; }
          }
    }
  }
  return PML_PIC_OK;
}

}  // namespace

extern "C" {

static int pml_pic_forward_ckpt_impl(pml_pic_handle *h, int32_t n_steps, double *U) {
  if (!h || !U) return PML_PIC_E_INVALID_ARG;
  return h->p.precision == 64 ? forward_ckpt_t<double>(h, n_steps, U) : forward_ckpt_t<float>(h, n_steps, U);
}

static int pml_pic_backward_impl(pml_pic_handle *h, const double *seed, int64_t seed_count, double *lambda_out,
                     double *grad_theta, int32_t n_theta) {
  if (!h || !grad_theta) return PML_PIC_E_INVALID_ARG;
  if (n_theta != 16 * h->p.dim + 1) return fail(&h->err, PML_PIC_E_INVALID_ARG, "n_theta must be 16 dim + 1");
  const int64_t ns = (int64_t)h->L.nn[0] * h->L.nn[1] * h->L.nn[2];
  if (seed && seed_count < 12 * ns) return fail(&h->err, PML_PIC_E_INVALID_ARG, "seed buffer too small");
  return h->p.precision == 64 ? backward_t<double>(h, seed, lambda_out, grad_theta)
                              : backward_t<float>(h, seed, lambda_out, grad_theta);
}

static int pml_pic_particle_adjoint_impl(pml_pic_handle *h, int64_t n, double *dU_dx, double *dU_du) {
  if (!h || !dU_dx || !dU_du || n < 0) return PML_PIC_E_INVALID_ARG;
  if (!h->padj_valid)
    return fail(&h->err, PML_PIC_E_INVALID_ARG, "no pml_pic_backward of a pushed run to read particle adjoints from");
  if (n > h->n_added || n > h->L.cap) return fail(&h->err, PML_PIC_E_INVALID_ARG, "n exceeds the particles added");
  const Layout &L = h->L;
  const size_t cap = (size_t)std::max<int64_t>(L.cap, 1), esz = L.esz;
  std::vector<char> buf(6 * esz * cap);
  HIPCHK(h, hipMemcpy(buf.data(), h->ws + L.off_padj, buf.size(), hipMemcpyDeviceToHost));
  auto val = [&](int arr, int64_t i) {
    const char *q = buf.data() + ((size_t)arr * cap + (size_t)i) * esz;
    return esz == 8 ? *(const double *)q : (double)*(const float *)q;
  };
  const int dim = h->p.dim;
  for (int64_t i = 0; i < n; ++i) {
    for (int d = 0; d < dim; ++d) dU_dx[dim * i + d] = val(d, i) / h->p.dx[d];   // offsets are in cells
    for (int d = 0; d < 3; ++d) dU_du[3 * i + d] = val(3 + d, i);
  }
  return PML_PIC_OK;
}

}  // extern "C"

// ===================================================================== exported entry points
// Every call runs its body under abi_guard: no C++ exception crosses the C ABI.
extern "C" {

int pml_pic_batch_workspace_size(const pml_pic_params *runs, int32_t n_runs, size_t *bytes) {
  return abi_guard(&g_create_error, [&] { return pml_pic_batch_workspace_size_impl(runs, n_runs, bytes); });
}

int pml_pic_batch_create(const pml_pic_params *runs, int32_t n_runs, void *device_workspace, size_t bytes, void *stream, int32_t use_graph, pml_pic_batch **out) {
  return abi_guard(&g_create_error, [&] { return pml_pic_batch_create_impl(runs, n_runs, device_workspace, bytes, stream, use_graph, out); });
}

int pml_pic_batch_set_launch(pml_pic_batch *b, int32_t block_x, int32_t grid_blocks) {
  return abi_guard(b ? &b->err : &g_create_error, [&] { return pml_pic_batch_set_launch_impl(b, block_x, grid_blocks); });
}

int pml_pic_batch_step(pml_pic_batch *b, int32_t n_steps) {
  return abi_guard(b ? &b->err : &g_create_error, [&] { return pml_pic_batch_step_impl(b, n_steps); });
}

int pml_pic_batch_step_profiled(pml_pic_batch *b, int32_t n_steps, double *phase_ms, int64_t *phase_calls) {
  return abi_guard(b ? &b->err : &g_create_error, [&] { return pml_pic_batch_step_profiled_impl(b, n_steps, phase_ms, phase_calls); });
}

int pml_pic_workspace_size(const pml_pic_params *params, size_t *bytes) {
  return abi_guard(&g_create_error, [&] { return pml_pic_workspace_size_impl(params, bytes); });
}

int pml_pic_create(const pml_pic_params *params, void *device_workspace, size_t bytes, void *stream, pml_pic_handle **out) {
  return abi_guard(&g_create_error, [&] { return pml_pic_create_impl(params, device_workspace, bytes, stream, out); });
}

int pml_pic_add_particles(pml_pic_handle *h, int64_t n, const double *x, const double *u, const double *w) {
  return abi_guard(h ? &h->err : &g_create_error, [&] { return pml_pic_add_particles_impl(h, n, x, u, w); });
}

int pml_pic_set_conductor(pml_pic_handle *h, const uint8_t *cells) {
  return abi_guard(h ? &h->err : &g_create_error, [&] { return pml_pic_set_conductor_impl(h, cells); });
}

int pml_pic_set_source(pml_pic_handle *h, int64_t n, const double *x, const double *u, const double *w, int32_t axis) {
  return abi_guard(h ? &h->err : &g_create_error, [&] { return pml_pic_set_source_impl(h, n, x, u, w, axis); });
}

int pml_pic_slab_moments(pml_pic_handle *h, int32_t axis, int32_t n_slabs, const double *edges, double *out) {
  return abi_guard(h ? &h->err : &g_create_error, [&] { return pml_pic_slab_moments_impl(h, axis, n_slabs, edges, out); });
}

int pml_pic_set_particles(pml_pic_handle *h, int64_t n, const int64_t *ids, const double *X, const double *u, const double *w) {
  return abi_guard(h ? &h->err : &g_create_error, [&] { return pml_pic_set_particles_impl(h, n, ids, X, u, w); });
}

int pml_pic_step(pml_pic_handle *h, int32_t n_steps) {
  return abi_guard(h ? &h->err : &g_create_error, [&] { return report_checks(h, pml_pic_step_impl(h, n_steps)); });
}

int pml_pic_step_profiled(pml_pic_handle *h, int32_t n_steps, double *phase_ms, int64_t *phase_calls) {
  return abi_guard(h ? &h->err : &g_create_error, [&] { return report_checks(h, pml_pic_step_profiled_impl(h, n_steps, phase_ms, phase_calls)); });
}

int pml_pic_field_error(pml_pic_handle *h, pml_pic_handle *ref, double *num, double *den) {
  return abi_guard(h ? &h->err : &g_create_error, [&] { return pml_pic_field_error_impl(h, ref, num, den); });
}

int pml_pic_field_error_noalloc(pml_pic_handle *h, pml_pic_handle *ref, double *num, double *den) {
  return abi_guard(h ? &h->err : &g_create_error, [&] { return pml_pic_field_error_noalloc_impl(h, ref, num, den); });
}

int pml_pic_diagnose(pml_pic_handle *h, pml_pic_diag *out) {
  return abi_guard(h ? &h->err : &g_create_error, [&] { return report_checks(h, pml_pic_diagnose_impl(h, out)); });
}

int pml_pic_grid_shape(const pml_pic_handle *h, int32_t nn[3], int64_t *n_samples) {
  return abi_guard(&g_create_error, [&] { return pml_pic_grid_shape_impl(h, nn, n_samples); });
}

int pml_pic_get_fields(pml_pic_handle *h, double *host, int64_t count) {
  return abi_guard(h ? &h->err : &g_create_error, [&] { return pml_pic_get_fields_impl(h, host, count); });
}

int pml_pic_set_fields(pml_pic_handle *h, const double *host, int64_t count) {
  return abi_guard(h ? &h->err : &g_create_error, [&] { return pml_pic_set_fields_impl(h, host, count); });
}

int pml_pic_get_current(pml_pic_handle *h, double *host, int64_t count) {
  return abi_guard(h ? &h->err : &g_create_error, [&] { return pml_pic_get_current_impl(h, host, count); });
}

int pml_pic_get_rho_static(pml_pic_handle *h, double *host, int64_t count) {
  return abi_guard(h ? &h->err : &g_create_error, [&] { return pml_pic_get_rho_static_impl(h, host, count); });
}

int pml_pic_set_rho_static(pml_pic_handle *h, const double *host, int64_t count) {
  return abi_guard(h ? &h->err : &g_create_error, [&] { return pml_pic_set_rho_static_impl(h, host, count); });
}

int pml_pic_sort_particles(pml_pic_handle *h, int32_t tile[3], uint32_t *key_start, int64_t cap, int64_t *n_keys) {
  return abi_guard(h ? &h->err : &g_create_error, [&] { return report_checks(h, pml_pic_sort_particles_impl(h, tile, key_start, cap, n_keys)); });
}

int pml_pic_num_particles(pml_pic_handle *h, int64_t *n) {
  return abi_guard(h ? &h->err : &g_create_error, [&] { return pml_pic_num_particles_impl(h, n); });
}

int pml_pic_get_particles(pml_pic_handle *h, int64_t cap, int64_t *ids, double *X, double *u, double *w, int64_t *n_out) {
  return abi_guard(h ? &h->err : &g_create_error, [&] { return pml_pic_get_particles_impl(h, cap, ids, X, u, w, n_out); });
}

int pml_pic_forward_ckpt(pml_pic_handle *h, int32_t n_steps, double *U) {
  return abi_guard(h ? &h->err : &g_create_error, [&] { return report_checks(h, pml_pic_forward_ckpt_impl(h, n_steps, U)); });
}

int pml_pic_backward(pml_pic_handle *h, const double *seed, int64_t seed_count, double *lambda_out, double *grad_theta, int32_t n_theta) {
  return abi_guard(h ? &h->err : &g_create_error, [&] { return report_checks(h, pml_pic_backward_impl(h, seed, seed_count, lambda_out, grad_theta, n_theta)); });
}

int pml_pic_particle_adjoint(pml_pic_handle *h, int64_t n, double *dU_dx, double *dU_du) {
  return abi_guard(h ? &h->err : &g_create_error, [&] { return pml_pic_particle_adjoint_impl(h, n, dU_dx, dU_du); });
}

}  // extern "C"

namespace pmlpic {
// Lane additions per second of FP64 and FP32 atomic adds into LDS (rates[0], rates[1]) and
// into global memory at distinct consecutive addresses (rates[2], rates[3]) on the current
// device (probe.hip); 0 or PML_PIC_E_HIP with the failing call in err.
int atomic_rates(double rates[4], std::string *err);
}  // namespace pmlpic

extern "C" {

int pml_pic_atomic_rates(double *rates) {
  return abi_guard(&g_create_error, [&] {
    if (!rates) return fail(&g_create_error, PML_PIC_E_INVALID_ARG, "rates is NULL");
    return atomic_rates(rates, &g_create_error);
  });
}

}  // extern "C"
