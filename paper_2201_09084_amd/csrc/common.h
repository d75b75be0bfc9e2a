// Device-side views and helpers shared by the HIP kernels of the PML PIC library.
//
// Layout in HBM (all arrays live in one caller-owned workspace):
//   * field arrays (E, B totals, one split part per component, J) are 3D blocks with
//     G guard layers on every side of every in-plane axis, x fastest, row pitch padded
//     to a multiple of 64 elements; sample (i,j,k) of a component is at
//     base + i + j*sy + k*sz.  Guard and out-of-extent samples hold 0 and are never
//     updated, so stencils near the PEC walls read zeros without bounds checks;
//   * per-axis 1D coefficient tables (sigma, exponential factors, alpha) at nodes and
//     cell centres, built in FP64 on the host;
//   * particles as structure-of-arrays: packed cell index (int per axis, +1 offset),
//     offsets in [0,1) within the cell, u = gamma v, weight, id.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pmlpic {

constexpr int G = 4;                 // guard layers per side
constexpr uint32_t DEAD = 0xFFFFFFFFu;

// kinds of per-axis table entries; node tables then centre tables
// (T_GK_N = g * (1/dx) of that axis at nodes for a full step; T_GHK_C = the same at
// centres for a half step: the factors that multiply a raw neighbour difference)
enum TabKind {
  T_SIG_N = 0, T_E_N, T_G_N, T_EH_N, T_GH_N, T_A_N,
  T_SIG_C, T_E_C, T_G_C, T_EH_C, T_GH_C, T_A_C,
  T_GK_N, T_GHK_C,
  T_NKIND
};

// The same pointer in the global address space.  Field arrays reached through a
// descriptor in device memory (batched runs) are otherwise accessed with flat
// instructions, which also tie up the LDS counters.
template <typename T>
__host__ __device__ __forceinline__ const __attribute__((address_space(1))) T *gptr(const T *p) {
  return (const __attribute__((address_space(1))) T *)p;
}
template <typename T>
__host__ __device__ __forceinline__ __attribute__((address_space(1))) T *gptr(T *p) {
  return (__attribute__((address_space(1))) T *)p;
}

// Per axis, the profile block used by the per-particle weight damping: low and high
// layer edges (grid units), their thicknesses (physical), then a_k / (k + 1) for the
// 16 coefficients of sigma/eps0 = sum_k a_k (depth/L)^k.
enum { PROF_LO = 0, PROF_HI, PROF_LLO, PROF_LHI, PROF_DX, PROF_C, PROF_N = PROF_C + 16 };

// alpha applied to the current in the field update (modes 0 and 2)
__host__ __device__ __forceinline__ bool current_alpha(int alpha_mode) { return alpha_mode == 0 || alpha_mode == 2; }

// Bounds-checked debug builds (compiled with -DPMLPIC_CHECK into libpmlpic_check.so): the
// particle kernels' index computations are checked before each access; a failed check sets a
// bit in a word of the workspace and the access is skipped (or redirected to sample 0), so
// the kernel still ends normally, and the host turns the bits into an error.
enum CheckBits : uint32_t {
  CHECK_SAMPLE = 1u,      // a field / current sample index outside its array
  CHECK_GLOBAL_J = 2u,    // a deposit to global J outside the array
  CHECK_LDS_BOX = 4u,     // a deposit into a workgroup's LDS current box outside the box
  CHECK_SORT_KEY = 8u     // a particle's sort key outside the key range
};
__device__ __forceinline__ void check_failed(uint32_t *check, uint32_t bit) {
  if (check) atomicOr(check, bit);
}

template <typename T>
struct Grid {
  int dim, order;
  int M[3];            // cells per axis including the PML (0 on the invariant axis)
  int lo[3], n[3];     // PML cells on the low side, physical cells
  long sy, sz;         // strides of y and z (x stride is 1)
  long base;           // offset of sample (0,0,0)
  long nelem;          // elements per field array
  int ext[3];          // allocated extent per axis (incl. guards)
  T dt;
  T inv_dx[3];
  T qdt_2m;            // charge dt / (2 mass)
  int solver;          // PML_PIC_SOLVER_YEE / _CK (Faraday's law)
  T jcoef[3];          // Esirkepov factor of J_a: (1/dx_b)(1/dx_c)/dt over the other two axes
                       // (1/dx = 1 on the invariant axis of a 2D run)
  T charge;
  const T *tab;        // [3][T_NKIND][ntab], entry i + G for index i in [-G, M+G]
  int ntab;
  int wdamp;           // 1: per-particle weight damping (alpha mode 3)
  const T *prof;       // [3][PROF_N]: layer edges, thicknesses and sigma coefficients
  const uint8_t *cmask;  // conductor: per node, bit c set when sample c (E_x..E_z, B_x..B_z)
                         // at that node index lies in a conductor cell; null without conductors
  uint32_t *check;       // bounds-checked builds (PMLPIC_CHECK): CHECK_* bits of failed
                         // checks, read by the host after each call; null otherwise

  __host__ __device__ long at(int i, int j, int k) const {
    const long q = base + i + j * sy + k * sz;
#if defined(PMLPIC_CHECK) && defined(__HIP_DEVICE_COMPILE__)
    if (q < 0 || q >= nelem) { check_failed(check, CHECK_SAMPLE); return 0; }
#endif
    return q;
  }
  __device__ T tb(int axis, int kind, int i) const {
    return gptr(tab)[(axis * T_NKIND + kind) * ntab + i + G];
  }
  // the same entry read through the constant address space: with an index that is the same
  // in every lane it becomes a scalar load (a scalar register, not counted with the vector
  // loads); the tables are not written while a kernel runs
  __device__ T tb_uniform(int axis, int kind, int i) const {
    return ((const __attribute__((address_space(4))) T *)tab)[(axis * T_NKIND + kind) * ntab + i + G];
  }
};

template <typename T>
struct Fields {
  T *E[3];
  T *B[3];
  T *Ea[3];   // split part E_ab, b = a+1 (valid where the component is split)
  T *Ba[3];   // split part B_ab, b = a+1
  T *J[3];
};

template <typename T>
struct Parts {
  uint32_t *cell;     // packed (i+1) per axis; DEAD for removed particles
  T *f[3];            // offsets in [0,1)
  T *u[3];            // gamma v
  T *w;               // weight
  T *lam;             // alpha mode 3: int sigma/eps0 dt along the path (else null)
  int32_t *id;
};

// --------------------------------------------------------------- packed cells
// 2D: 16 bits per axis; 3D: 11 / 11 / 10 bits.  Stored value is index + 1, so a
// particle one cell outside the grid (just before removal) is representable.
__host__ __device__ inline uint32_t pack_cell(int dim, int i, int j, int k) {
  if (dim == 2) return (uint32_t)(i + 1) | ((uint32_t)(j + 1) << 16);
  return (uint32_t)(i + 1) | ((uint32_t)(j + 1) << 11) | ((uint32_t)(k + 1) << 22);
}
__host__ __device__ inline void unpack_cell(int dim, uint32_t c, int &i, int &j, int &k) {
  if (dim == 2) { i = (int)(c & 0xFFFFu) - 1; j = (int)(c >> 16) - 1; k = 0; return; }
  i = (int)(c & 0x7FFu) - 1; j = (int)((c >> 11) & 0x7FFu) - 1; k = (int)(c >> 22) - 1;
}

// --------------------------------------------------------------- shapes
// Centred B-spline weights of order ORDER (1 linear, 2 quadratic, 3 cubic) for a point
// at offset f in [0,1) from node i: the stencil is nodes i+start .. i+start+ORDER.
template <int ORDER, typename T>
__device__ __forceinline__ int shape_weights(T f, T (&w)[ORDER + 1]) {
  if constexpr (ORDER == 1) {
    w[0] = T(1) - f;
    w[1] = f;
    return 0;
  } else if constexpr (ORDER == 2) {
    const int up = f >= T(0.5);
    const T d = f - T(up);                 // distance to the nearest node, [-1/2, 1/2)
    const T a = T(0.5) - d, b = T(0.5) + d;
    w[0] = T(0.5) * a * a;
    w[1] = T(0.75) - d * d;
    w[2] = T(0.5) * b * b;
    return up - 1;
  } else {
    const T g = T(1) - f;
    const T f2 = f * f, g2 = g * g;
    w[0] = g2 * g * T(1.0 / 6.0);
    w[1] = (T(4) - T(6) * f2 + T(3) * f2 * f) * T(1.0 / 6.0);
    w[2] = (T(4) - T(6) * g2 + T(3) * g2 * g) * T(1.0 / 6.0);
    w[3] = f2 * f * T(1.0 / 6.0);
    return -1;
  }
}

// Same for the half-integer sample positions (index s refers to s + 1/2).
template <int ORDER, typename T>
__device__ __forceinline__ int shape_weights_stag(int i, T f, T (&w)[ORDER + 1]) {
  if constexpr (sizeof(T) == 4) {   // selects instead of branches (the same arithmetic)
    const bool hi = f >= T(0.5);
    const T a = f - T(0.5), b = f + T(0.5);
    const bool fix = !hi && b >= T(1);
    return ((hi || fix) ? i : i - 1) + shape_weights<ORDER>(hi ? a : (fix ? T(0) : b), w);
  } else {
    int ii;
    T ff;
    if (f >= T(0.5)) { ii = i; ff = f - T(0.5); }
    else { ii = i - 1; ff = f + T(0.5); if (ff >= T(1)) { ff = T(0); ii = i; } }
    return ii + shape_weights<ORDER>(ff, w);
  }
}

// The array of three for a component known only at run time (per lane): a select between
// the three pointers.  Indexing the kernel argument's array with it makes the compiler load
// the pointer from memory, and each wait for that load also waits for every store and
// atomic issued before it.
template <typename T>
__device__ __forceinline__ T *pick3(T *const (&a)[3], int c) {
  return c == 0 ? a[0] : (c == 1 ? a[1] : a[2]);
}

// --------------------------------------------------------------- atomics
__device__ __forceinline__ void atomic_add(float *p, float v) { unsafeAtomicAdd(p, v); }
__device__ __forceinline__ void atomic_add(double *p, double v) { unsafeAtomicAdd(p, v); }

// --------------------------------------------------------------- launch wrappers
constexpr int N_PUSH_COUNTERS = 256;   // push tallies are spread over this many words

struct StepCtl {
  int32_t *count;                 // device: live particle slots in use
  unsigned long long *pushes;     // N_PUSH_COUNTERS partial push counts
  int *jslot;                     // 2D one-pass runs: JSLOTS boxes of nodes given current this
                                  // step (x lo, x hi, y lo, y hi each); workgroup b merges its
                                  // box into slot b mod JSLOTS; else null
};
// Slots of the boxes of nodes that received current: workgroups merge into different
// slots (atomics on one word from every workgroup serialise across the chip), and a
// wavefront reads all of them (one slot per lane) to form the union.
constexpr int JSLOTS = 64;
__device__ __forceinline__ void jslot_merge(int *slots, int xlo, int xhi, int ylo, int yhi) {
  if (xlo > xhi) return;
  int *s = slots + 4 * (int)(blockIdx.x % JSLOTS);
  atomicMin(&s[0], xlo); atomicMax(&s[1], xhi); atomicMin(&s[2], ylo); atomicMax(&s[3], yhi);
}
// union of the slots, uniform over the wavefront (every lane calls it)
__device__ __forceinline__ int4 jslot_union(const int *slots) {
  const int l = (int)(threadIdx.x & 63);
  int4 b = make_int4(0x7FFFFFFF, -0x7FFFFFFF, 0x7FFFFFFF, -0x7FFFFFFF);
  if (l < JSLOTS) {
    const auto *p = gptr(slots) + 4 * l;
    b = make_int4(p[0], p[1], p[2], p[3]);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    b.x = min(b.x, __shfl_xor(b.x, off)); b.y = max(b.y, __shfl_xor(b.y, off));
    b.z = min(b.z, __shfl_xor(b.z, off)); b.w = max(b.w, __shfl_xor(b.w, off));
  }
  return make_int4(__builtin_amdgcn_readfirstlane(b.x), __builtin_amdgcn_readfirstlane(b.y),
                   __builtin_amdgcn_readfirstlane(b.z), __builtin_amdgcn_readfirstlane(b.w));
}

// 2D one-pass runs keep J in two buffers by step parity: while the deposit of a step
// fills one, the other (consumed by the previous step's field update) is cleared over
// that step's node box, and the slots of the next step are emptied.  prev = null: none.
template <typename T>
struct JClear {
  T *J[3];
  const int *prev;   // JSLOTS boxes of the step whose current is cleared
  int *next;         // JSLOTS boxes of the next step, emptied
};
// inside a kernel: every workgroup clears its share (grid-stride), workgroup 0 empties
// `next`; all threads of the workgroup call it
template <typename T>
__device__ __forceinline__ void jclear_share(const Grid<T> &g, const JClear<T> &jc) {
  if (blockIdx.x == 0 && threadIdx.x < JSLOTS) {
    auto *p = gptr(jc.next) + 4 * threadIdx.x;
    p[0] = 0x7FFFFFFF; p[1] = -0x7FFFFFFF; p[2] = 0x7FFFFFFF; p[3] = -0x7FFFFFFF;
  }
  const int4 b = jslot_union(jc.prev);
  const int x0 = max(b.x, -G), x1 = min(b.y, g.M[0] + G);
  const int y0 = max(b.z, -G), y1 = min(b.w, g.M[1] + G);
  if (x0 > x1 || y0 > y1) return;
  const int w = x1 - x0 + 1, n = w * (y1 - y0 + 1);
  const int sy = (int)g.sy, q0 = (int)g.base;
  for (int e = (int)(blockIdx.x * blockDim.x + threadIdx.x); e < n; e += (int)(gridDim.x * blockDim.x)) {
    const int q = q0 + x0 + e % w + (y0 + e / w) * sy;
    gptr(jc.J[0])[q] = T(0);
    gptr(jc.J[1])[q] = T(0);
    gptr(jc.J[2])[q] = T(0);
  }
}

template <typename T>
void launch_update_B(const Grid<T> &g, const Fields<T> &F, bool half, hipStream_t s);
template <typename T>
void launch_update_E(const Grid<T> &g, const Fields<T> &F, bool fuse_alpha, int alpha_mode, bool consume,
                     hipStream_t s);
// `passes` binomial filter passes over J (3D), alternating between J and tmp (three
// adjacent arrays of nelem each); returns the one holding the filtered current
template <typename T>
T *launch_filter_current(const Grid<T> &g, T *J, T *tmp, int passes, hipStream_t s);
template <typename T>
void launch_damp_current(const Grid<T> &g, const Fields<T> &F, hipStream_t s);
// beam transport: conductor mask applied to the fields, source injection, slab moments
constexpr int SLAB_MAX = 64;
template <typename T>
void launch_apply_conductor(const Grid<T> &g, const Fields<T> &F, hipStream_t s);
template <typename T>
void launch_inject(int dim, const Parts<T> &P, const Parts<T> &S, int32_t *count, int64_t first, int n,
                   int32_t *tail_start, bool mark, hipStream_t s);
template <typename T>
void launch_slab_moments(const Grid<T> &g, const Parts<T> &P, const int32_t *count, int n_slots, int axis, double dxa,
                         int nslab, const double *edges, double *out, hipStream_t s);
template <typename T>
void launch_gather_push(const Grid<T> &g, const Fields<T> &F, const Parts<T> &P, Parts<T> old,
                        StepCtl ctl, int n_slots, int push, bool fused, hipStream_t s);
// the same over slots [*start, count) (the unsorted tail of a tiled run), n_upper >= its length
template <typename T>
void launch_gather_push_tail(const Grid<T> &g, const Fields<T> &F, const Parts<T> &P, StepCtl ctl,
                             const int32_t *start, int n_upper, int n_slots, int push, hipStream_t s);
// Work decomposition of the tiled particle step: after every sort, each tile's range
// of cell-sorted particles is cut into chunks of at most `chunk` particles, listed as
// work items (full chunks first, then each tile's partial chunk).
struct TileWork {
  const uint32_t *key_start;   // sort counts: first slot of every cell key at the last sort
  uint32_t *dprefix;           // ntiles + 1: exclusive prefix of the chunks of dense tiles (a cell
                               // holding more than DENSE_CELL particles), total last
  uint32_t *prefix;            // ntiles + 1: the same for the full chunks of the other tiles
  uint32_t *pprefix;           // ntiles + 1: the same for their last partial chunk
  uint32_t *blocksums;         // scan scratch
  int4 *items;                 // per chunk: first slot, end slot, tile
  uint32_t *flags;             // 2D: per fixed range, 1 if its node box does not fit in LDS
  uint32_t *n_items;           // 2D: number of items in `items`
  int ntiles, tilecells, chunk, margin;
  int tile[3], ntile[3];
  int by_tile;                 // 1: tile items; 0: ranges of the sorted array (2D list)
  int sel;                     // tile items a launch takes: 0 all, 1 the chunks of dense tiles,
                               // 2 the chunks of the other tiles
};
void launch_tile_chunks(const TileWork &tw, const int32_t *count, hipStream_t s);
// 2D work list after a sort: cell = the sorted particles' cells, max_ranges = ranges of
// `chunk` particles at full capacity, drift = cells a particle may move per side before
// the next sort (allowance in the LDS fit test)
void launch_range_items(const TileWork &tw, const uint32_t *cell, const int32_t *count, int order, int max_ranges,
                        int drift, hipStream_t s);
constexpr int RANGE_SPLIT_MAX = 8;                      // items per range at most
int tiled_chunk(int dim);   // particles per chunk of the tiled step
int tiled_nodes(int dim);   // LDS nodes per current component of one chunk's box
template <typename T>
void launch_push_deposit_tiles(const Grid<T> &g, const Fields<T> &F, const Parts<T> &P, StepCtl ctl, JClear<T> jc,
                               const TileWork &tw, int n_slots, int push, hipStream_t s);
template <typename T>
void launch_deposit(const Grid<T> &g, const Fields<T> &F, const Parts<T> &P, Parts<T> old,
                    StepCtl ctl, int n_slots, bool serial, hipStream_t s);

// 3D linear-shape runs (push3d.hip): gather_push + deposit_current, one workgroup per chunk
// of a sort tile (the work items of launch_tile_chunks), its current summed in an LDS box of
// the tile's nodes (tile + 3 per axis) and added to J with global atomics.  Applies to tiles
// of at least three cells whose box fits in LDS and spans less than 2^32 samples of the grid
// (plane: the grid's z stride).
bool push3d_applies(int dim, int order, const int tile[3], long plane);
template <typename T>
void launch_push3d(const Grid<T> &g, const Fields<T> &F, const Parts<T> &P, StepCtl ctl, const TileWork &tw,
                   int n_slots, int push, hipStream_t s);

struct SortWork {
  uint32_t *counts;      // nkeys + 1
  uint32_t *rank;        // per particle
  uint32_t *blocksums;   // scan scratch
  int nkeys;
  int tile[3];
  int ntile[3];
  uint32_t *check;       // bounds-checked builds: as Grid::check
};
template <typename T>
void launch_sort(const Grid<T> &g, const Parts<T> &src, const Parts<T> &dst, SortWork sw,
                 StepCtl ctl, int n_slots, hipStream_t s);

// Eq. (error) sums against a reference run (out[0] = sum (F - F_ref)^2, out[1] = sum F_ref^2
// over g's physical box); partial holds two doubles per workgroup of g's node grid
template <typename T>
void launch_field_error(const Grid<T> &g, const Fields<T> &F, const Grid<T> &gr, const Fields<T> &R, double *partial,
                        double *out, hipStream_t s);
// The same sums with the partials and the result in the file-scope device array of
// diag.hip (no workspace): field_error_scratch gives its device address on the current
// device; the launch returns false (launching nothing) when the grid needs more partial
// pairs per row of x-blocks than the array holds (field_error_scratch_pairs()).
hipError_t field_error_scratch(double **ptr);
int field_error_scratch_pairs();
template <typename T>
bool launch_field_error_scratch(const Grid<T> &g, const Fields<T> &F, const Grid<T> &gr, const Fields<T> &R,
                                double *sc, hipStream_t s);
struct DiagWork {
  double *rho;           // nelem
  const double *rho_static;
  double *partial;       // per block scratch
  double *result;        // 8 doubles
  int32_t *flags;        // [0] nonfinite, [1] live count
  int max_blocks;
};
template <typename T>
void launch_diag(const Grid<T> &g, const Fields<T> &F, const Parts<T> &P, StepCtl ctl,
                 int n_slots, DiagWork dw, hipStream_t s);
template <typename T>
void launch_rho(const Grid<T> &g, const Parts<T> &P, StepCtl ctl, int first, int n_slots, double *rho,
                double sign, hipStream_t s);

// adjoint of the fields: LT[c] (part driven along a+2, or the whole component where it
// is not split), LA[c] (part driven along a+1 minus LT), c = E_x .. B_z
// the clear of a JClear as its own launch (steps whose deposit is not the tiled kernel)
template <typename T>
void launch_jbox_clear(const Grid<T> &g, const JClear<T> &jc, hipStream_t s);
// workgroups of the deposit launch of a step
template <typename T>
int deposit_blocks(const Grid<T> &g, const TileWork &tw, int n_slots, bool tiled);

// output columns per wavefront strip of the one-pass 2D field update (64 lanes less
// one halo column on the left and two on the right)
constexpr int FW = 61;

// update_yee_pml in one pass over the fields (2D): reads F (and its J, not cleared, inside
// the union of the slots `jslot`), writes the new E, B (and split parts) to D
template <typename T>
void launch_fused_fields(const Grid<T> &g, const Fields<T> &F, const Fields<T> &D, const int *jslot, bool fuse_alpha,
                         hipStream_t s);

// update_yee_pml in one pass over 3D fields (fused3d.hip): reads F (and its J, not
// cleared), writes the new E, B (and split parts) to D, and clears the other current
// buffer jz (read by the previous step) over the samples it owns
template <typename T>
struct JZero {
  T *J[3];
};
template <typename T>
void launch_fused_fields_3d(const Grid<T> &g, const Fields<T> &F, const Fields<T> &D, const JZero<T> &jz,
                            bool fuse_alpha, hipStream_t s);

template <typename T>
struct AdjFields {
  T *LT[6];
  T *LA[6];
};
template <typename T>
void launch_adj_seed_energy(const Grid<T> &g, const Fields<T> &F, const AdjFields<T> &L, hipStream_t s);
template <typename T>
void launch_adj_B_half(const Grid<T> &g, const AdjFields<T> &L, const Fields<T> &Fb, double *Gacc, hipStream_t s);
template <typename T>
void launch_adj_E(const Grid<T> &g, const AdjFields<T> &L, const Fields<T> &Fe, T *const J[3], int alpha_mode,
                  double *Gacc, T *const *LJ, hipStream_t s);
// adjoint of each particle's offset (cell units, per axis) and momentum, indexed by id
template <typename T>
struct PartAdj {
  T *lf[3];
  T *lu[3];
};
// reverse of one step's gather_push and deposit_current (adjoint_particles.hip): Fn holds
// the fields at the start of the step, P the particles as that step's push read them
template <typename T>
void launch_adj_particles(const Grid<T> &g, const Fields<T> &Fn, const Parts<T> &P, const int32_t *count, int ns,
                          int cap, const AdjFields<T> &L, T *const LJ[3], const PartAdj<T> &A, hipStream_t s);

// one run of a batch: everything its kernels need, in device memory
template <typename T>
struct RunDesc {
  Grid<T> g;
  Fields<T> F;    // field set 0 (and J)
  Fields<T> F2;   // field set 1 of the out-of-place 2D update (same J)
  int *jbox;      // 2D: two boxes of nodes with current (by step parity)
  int pad2[2];
  Parts<T> P;
  StepCtl ctl;
  int n_slots;
  int push;
  int alpha_mode;
  int pad;
};

// 2D batches: one-pass field update of every run, reading set `parity` and writing
// the other (items: run, strip, first row, end row), then J cleared over the same items
template <typename T>
void launch_batch_fused(const RunDesc<T> *runs, const int4 *items, int n_items, int parity, int grid_blocks,
                        hipStream_t s);
template <typename T>
void launch_batch_clear_j(const RunDesc<T> *runs, int n_runs, int parity, hipStream_t s);

// one phase of a batched step: 0 particles, 1 B half step, 2 E step
template <typename T>
void launch_batch_phase(int phase, int dim, int order, const RunDesc<T> *runs, int n_runs, const int4 *items,
                        int n_items, int bdx, int grid_blocks, int parity, hipStream_t s);

}  // namespace pmlpic
