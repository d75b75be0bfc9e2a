// Batched form of the step: many independent runs (their own grids, PML thicknesses,
// profiles and particles, one precision, dimension and shape order) advanced by one
// set of launches.  Each run is described by a RunDesc in device memory; the field
// kernels walk a work list of (run, block) items with a persistent grid-stride loop,
// so every run's nodes are spread over the whole GPU whatever their sizes.  The
// per-sample and per-particle arithmetic is the single-run code (field_core.h,
// particle_core.h), so a batched run reproduces the same run stepped alone.
#include "field_core.h"
#include "particle_core.h"

namespace pmlpic {

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
    const bool fuse_alpha = runs[w.x].alpha_mode != 1;
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
__global__ void __launch_bounds__(64) k_batch_push(const RunDesc<T> *__restrict__ runs) {
  const RunDesc<T> &R = runs[blockIdx.x];
  const Grid<T> g = R.g;
  const Fields<T> F = R.F;
  const Parts<T> P = R.P;
  const int n = min(*R.ctl.count, R.n_slots);
  for (int base = 0; base < n; base += blockDim.x) {
    const int p = base + threadIdx.x;
    bool active = false;
    if (p < n) active = push_one<T, DIM, ORDER>(g, F, P, P, p, R.push, true);
    count_pushes(R.ctl.pushes, active);
  }
}

// phase 0: particles of all runs; 1: B half step; 2: E step
template <typename T>
void launch_batch_phase(int phase, int dim, int order, const RunDesc<T> *runs, int n_runs, const int4 *items,
                        int n_items, int bdx, int grid_blocks, hipStream_t s) {
  const dim3 blk(256), grd(grid_blocks);
  const dim3 pblk(64), pgrd(n_runs);
  if (phase == 0) {
#define PMLPIC_BPUSH(DIMV, ORD) hipLaunchKernelGGL((k_batch_push<T, DIMV, ORD>), pgrd, pblk, 0, s, runs)
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
                                        hipStream_t);
template void launch_batch_phase<double>(int, int, int, const RunDesc<double> *, int, const int4 *, int, int, int,
                                         hipStream_t);

}  // namespace pmlpic
