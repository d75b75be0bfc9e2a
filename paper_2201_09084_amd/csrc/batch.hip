// Batched form of the step: many independent runs (their own grids, PML thicknesses,
// profiles and particles, one precision, dimension and shape order) advanced by one
// set of launches.  Each run is described by a RunDesc in device memory; the field
// kernels walk a work list of (run, block) items with a persistent grid-stride loop,
// so every run's nodes are spread over the whole GPU whatever their sizes.  The
// per-sample and per-particle arithmetic is the single-run code (field_core.h,
// particle_core.h), so a batched run reproduces the same run stepped alone.
#include "field_core.h"
#include "fused2d.h"
#include "particle_core.h"

namespace pmlpic {

// 2D: one wavefront per work item (run, strip, y0, y1), persistent over the list
template <typename T>
__global__ void __launch_bounds__(256) k_batch_fused_2d(const RunDesc<T> *__restrict__ runs,
                                                        const int4 *__restrict__ items, int n_items, int parity) {
  const int lane = threadIdx.x & 63;
  // the wavefront's index, made visibly uniform so that the run's descriptor lands in
  // scalar registers
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  // Workgroups go to the 8 XCDs in turn (workgroup b on XCD b mod 8).  Each XCD takes
  // one contiguous eighth of the item list, so neighbouring strips, which share the
  // cache lines at their edges, mostly meet in the same L2.
  int first = 0, last = n_items, slot = blockIdx.x, nslots = gridDim.x;
  if ((gridDim.x & 7) == 0) {
    const int x = blockIdx.x & 7;
    first = (int)((long)n_items * x / 8);
    last = (int)((long)n_items * (x + 1) / 8);
    slot = blockIdx.x >> 3;
    nslots = gridDim.x >> 3;
  }
  for (int it = first + slot * 4 + wave; it < last; it += nslots * 4) {
    const int4 w = items[it];
    const Grid<T> g = runs[w.x].g;
    const Fields<T> src = parity ? runs[w.x].F2 : runs[w.x].F;
    const Fields<T> dst = parity ? runs[w.x].F : runs[w.x].F2;
    const int *jb = runs[w.x].jbox + 4 * parity;
    const int4 box = make_int4(__builtin_amdgcn_readfirstlane(jb[0]), __builtin_amdgcn_readfirstlane(jb[1]),
                               __builtin_amdgcn_readfirstlane(jb[2]), __builtin_amdgcn_readfirstlane(jb[3]));
    fused_segment_2d(g, src, dst, box, w.y, w.z, w.w, current_alpha(runs[w.x].alpha_mode), lane);
  }
}

// per run: J <- 0 over the previous step's box, this step's box reset to empty
template <typename T>
__global__ void __launch_bounds__(256) k_batch_clear_j(const RunDesc<T> *__restrict__ runs, int n_runs, int parity) {
  for (int r = blockIdx.x; r < n_runs; r += gridDim.x) {
    const Grid<T> g = runs[r].g;
    const Fields<T> F = runs[r].F;
    const int *prev = runs[r].jbox + 4 * (1 - parity);
    int *cur = runs[r].jbox + 4 * parity;
    const int x0 = max(prev[0], -G), x1 = min(prev[1], g.M[0] + G);
    const int y0 = max(prev[2], -G), y1 = min(prev[3], g.M[1] + G);
    if (x0 <= x1 && y0 <= y1) {
      const int w = x1 - x0 + 1, n = w * (y1 - y0 + 1);
      for (int e = threadIdx.x; e < n; e += blockDim.x) {
        const long q = g.at(x0 + e % w, y0 + e / w, 0);
        gptr(F.J[0])[q] = T(0);
        gptr(F.J[1])[q] = T(0);
        gptr(F.J[2])[q] = T(0);
      }
    }
    if (threadIdx.x == 0) {
      cur[0] = 0x7FFFFFFF; cur[1] = -0x7FFFFFFF; cur[2] = 0x7FFFFFFF; cur[3] = -0x7FFFFFFF;
    }
  }
}

template <typename T>
void launch_batch_fused(const RunDesc<T> *runs, const int4 *items, int n_items, int parity, int grid_blocks,
                        hipStream_t s) {
  hipLaunchKernelGGL((k_batch_fused_2d<T>), dim3(grid_blocks), dim3(256), 0, s, runs, items, n_items, parity);
}
template <typename T>
void launch_batch_clear_j(const RunDesc<T> *runs, int n_runs, int parity, hipStream_t s) {
  hipLaunchKernelGGL((k_batch_clear_j<T>), dim3(n_runs), dim3(256), 0, s, runs, n_runs, parity);
}
template void launch_batch_fused<float>(const RunDesc<float> *, const int4 *, int, int, int, hipStream_t);
template void launch_batch_fused<double>(const RunDesc<double> *, const int4 *, int, int, int, hipStream_t);
template void launch_batch_clear_j<float>(const RunDesc<float> *, int, int, hipStream_t);
template void launch_batch_clear_j<double>(const RunDesc<double> *, int, int, hipStream_t);

template <typename T, int DIM>
__global__ void __launch_bounds__(256) k_batch_update_B(const RunDesc<T> *__restrict__ runs, const int4 *__restrict__ items,
                                                        int n_items, int bdx) {
  const int tx = threadIdx.x % bdx, ty = threadIdx.x / bdx, bdy = blockDim.x / bdx;
  for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
    const int4 w = items[it];
    const Grid<T> g = runs[w.x].g;
    const Fields<T> F = runs[w.x].F;
    const int i = w.y * bdx + tx, j = w.z * bdy + ty, k = w.w;
    if (i > g.M[0] || j > g.M[1]) continue;
    const int id[3] = {i, j, k};
    const long q = g.at(i, j, k);
    update_B_comp<T, DIM, 0>(g, F, id, q);
    update_B_comp<T, DIM, 1>(g, F, id, q);
    update_B_comp<T, DIM, 2>(g, F, id, q);
  }
}

template <typename T, int DIM>
__global__ void __launch_bounds__(256) k_batch_update_E(const RunDesc<T> *__restrict__ runs, const int4 *__restrict__ items,
                                                        int n_items, int bdx) {
  const int tx = threadIdx.x % bdx, ty = threadIdx.x / bdx, bdy = blockDim.x / bdx;
  for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
    const int4 w = items[it];
    const Grid<T> g = runs[w.x].g;
    const Fields<T> F = runs[w.x].F;
    const bool fuse_alpha = current_alpha(runs[w.x].alpha_mode);
    const int i = w.y * bdx + tx, j = w.z * bdy + ty, k = w.w;
    if (i > g.M[0] || j > g.M[1]) continue;
    const int id[3] = {i, j, k};
    const long q = g.at(i, j, k);
    update_E_comp<T, DIM, 0>(g, F, id, q, fuse_alpha, true);
    update_E_comp<T, DIM, 1>(g, F, id, q, fuse_alpha, true);
    update_E_comp<T, DIM, 2>(g, F, id, q, fuse_alpha, true);
  }
}

// one workgroup per run: its threads take the run's particle slots in turn
template <typename T, int DIM, int ORDER>
__global__ void __launch_bounds__(64) k_batch_push(const RunDesc<T> *__restrict__ runs, int parity) {
  const RunDesc<T> &R = runs[blockIdx.x];
  const Grid<T> g = R.g;
  const Fields<T> F = parity ? R.F2 : R.F;   // the set holding the current fields
  const Parts<T> P = R.P;
  const int n = min(*R.ctl.count, R.n_slots);
  int lo0 = 0x7FFFFFFF, hi0 = -0x7FFFFFFF, lo1 = 0x7FFFFFFF, hi1 = -0x7FFFFFFF;
  for (int base = 0; base < n; base += blockDim.x) {
    const int p = base + threadIdx.x;
    bool active = false;
    int rng[4] = {0, -1, 0, -1};
    if (p < n) active = push_one<T, DIM, ORDER>(g, F, P, P, p, R.push, true, rng);
    count_pushes(R.ctl.pushes, active);
    if (rng[0] <= rng[1]) { lo0 = min(lo0, rng[0]); hi0 = max(hi0, rng[1]); lo1 = min(lo1, rng[2]); hi1 = max(hi1, rng[3]); }
  }
  if (DIM == 2) jbox_grow(R.jbox + 4 * parity, lo0, hi0, lo1, hi1);
}

// phase 0: particles of all runs; 1: B half step; 2: E step
template <typename T>
void launch_batch_phase(int phase, int dim, int order, const RunDesc<T> *runs, int n_runs, const int4 *items,
                        int n_items, int bdx, int grid_blocks, int parity, hipStream_t s) {
  const dim3 blk(256), grd(grid_blocks);
  const dim3 pblk(64), pgrd(n_runs);
  if (phase == 0) {
#define PMLPIC_BPUSH(DIMV, ORD) hipLaunchKernelGGL((k_batch_push<T, DIMV, ORD>), pgrd, pblk, 0, s, runs, parity)
    if (dim == 2) {
      if (order == 1) PMLPIC_BPUSH(2, 1); else if (order == 2) PMLPIC_BPUSH(2, 2); else PMLPIC_BPUSH(2, 3);
    } else {
      if (order == 1) PMLPIC_BPUSH(3, 1); else if (order == 2) PMLPIC_BPUSH(3, 2); else PMLPIC_BPUSH(3, 3);
    }
#undef PMLPIC_BPUSH
  } else if (phase == 1) {
    if (dim == 2) hipLaunchKernelGGL((k_batch_update_B<T, 2>), grd, blk, 0, s, runs, items, n_items, bdx);
    else hipLaunchKernelGGL((k_batch_update_B<T, 3>), grd, blk, 0, s, runs, items, n_items, bdx);
  } else {
    if (dim == 2) hipLaunchKernelGGL((k_batch_update_E<T, 2>), grd, blk, 0, s, runs, items, n_items, bdx);
    else hipLaunchKernelGGL((k_batch_update_E<T, 3>), grd, blk, 0, s, runs, items, n_items, bdx);
  }
}

template void launch_batch_phase<float>(int, int, int, const RunDesc<float> *, int, const int4 *, int, int, int,
                                        int, hipStream_t);
template void launch_batch_phase<double>(int, int, int, const RunDesc<double> *, int, const int4 *, int, int, int,
                                         int, hipStream_t);

}  // namespace pmlpic
