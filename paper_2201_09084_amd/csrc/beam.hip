// Beam-transport pieces of the cavity run (Sec. IV.A, App. A.2): conductor cells,
// injection of a beam source through the entry PML, and the beam's momentum moments per
// slab (the <u_x> deflection diagnostic).
#include <algorithm>

#include "common.h"

namespace pmlpic {

// ------------------------------------------------------------------ conductors
// Zeroes both parts of every E and B sample flagged in the conductor mask (used when the
// mask is set; afterwards the field kernels zero the flagged samples after each update).
template <typename T>
__global__ void __launch_bounds__(256) k_apply_conductor(Grid<T> g, Fields<T> F) {
  const int i = (int)(blockIdx.x * 64 + (threadIdx.x & 63));
  const int j = (int)(blockIdx.y * 4 + (threadIdx.x >> 6));
  const int k = (int)blockIdx.z;
  if (i > g.M[0] || j > g.M[1] || k > g.M[2]) return;
  const long q = g.at(i, j, k);
  const unsigned m = gptr(g.cmask)[q];
  if (!m) return;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if ((m >> a) & 1) { F.E[a][q] = T(0); F.Ea[a][q] = T(0); }
    if ((m >> (3 + a)) & 1) { F.B[a][q] = T(0); F.Ba[a][q] = T(0); }
  }
}

template <typename T>
void launch_apply_conductor(const Grid<T> &g, const Fields<T> &F, hipStream_t s) {
  if (!g.cmask || g.dim != 3) return;
  dim3 blk(256), grd((g.M[0] + 1 + 63) / 64, (g.M[1] + 1 + 3) / 4, g.M[2] + 1);
  hipLaunchKernelGGL((k_apply_conductor<T>), grd, blk, 0, s, g, F);
}
template void launch_apply_conductor<float>(const Grid<float> &, const Fields<float> &, hipStream_t);
template void launch_apply_conductor<double>(const Grid<double> &, const Fields<double> &, hipStream_t);

// ------------------------------------------------------------------ beam source
// Appends entries [first, first + n) of the source (already in the particle format, at
// their injection positions) after the live slots: slot count + t for entry first + t.
// Every thread reads the count before any thread of the next launch changes it; the
// count itself is raised by k_count_add afterwards, which on the first injection since
// the last sort also records where the unsorted tail starts.
template <typename T>
__global__ void __launch_bounds__(256) k_inject(int dim, Parts<T> P, Parts<T> S, const int32_t *count, int64_t first,
                                                int n) {
  const int t = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (t >= n) return;
  const int64_t src = first + t;
  const int64_t dst = (int64_t)*count + t;
  P.cell[dst] = S.cell[src];
  for (int d = 0; d < dim; ++d) P.f[d][dst] = S.f[d][src];
  for (int d = 0; d < 3; ++d) P.u[d][dst] = S.u[d][src];
  P.w[dst] = S.w[src];
  P.id[dst] = S.id[src];
  if (P.lam) P.lam[dst] = T(0);
}

__global__ void k_count_add(int32_t *count, int n, int32_t *tail_start, int mark) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    const int32_t c = *count;
    if (mark) *tail_start = c;
    *count = c + n;
  }
}

template <typename T>
void launch_inject(int dim, const Parts<T> &P, const Parts<T> &S, int32_t *count, int64_t first, int n,
                   int32_t *tail_start, bool mark, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL((k_inject<T>), dim3((n + 255) / 256), dim3(256), 0, s, dim, P, S, count, first, n);
  hipLaunchKernelGGL(k_count_add, dim3(1), dim3(64), 0, s, count, n, tail_start, mark ? 1 : 0);
}
template void launch_inject<float>(int, const Parts<float> &, const Parts<float> &, int32_t *, int64_t, int,
                                   int32_t *, bool, hipStream_t);
template void launch_inject<double>(int, const Parts<double> &, const Parts<double> &, int32_t *, int64_t, int,
                                    int32_t *, bool, hipStream_t);

// ------------------------------------------------------------------ slab moments
// Per slab [edges[k], edges[k+1]) of physical coordinate along `axis`: number of live
// particles, sum w, sum w u_x, sum w u_y, sum w u_z.  Each workgroup sums into FP64 LDS
// accumulators, then adds them to out (FP64 global atomics, one per slab entry and
// workgroup).
template <typename T>
__global__ void __launch_bounds__(256) k_slab_moments(Grid<T> g, Parts<T> P, const int32_t *count, int n_slots,
                                                      int axis, double dxa, int nslab, const double *edges,
                                                      double *out) {
  __shared__ double acc[5 * SLAB_MAX];
  __shared__ double e[SLAB_MAX + 1];
  for (int t = threadIdx.x; t < 5 * nslab; t += blockDim.x) acc[t] = 0.0;
  for (int t = threadIdx.x; t <= nslab; t += blockDim.x) e[t] = edges[t];
  __syncthreads();
  const int n = min(*count, n_slots);
  for (int p = (int)(blockIdx.x * blockDim.x + threadIdx.x); p < n; p += (int)(gridDim.x * blockDim.x)) {
    const uint32_t c = P.cell[p];
    if (c == DEAD) continue;
    int ic[3];
    unpack_cell(g.dim, c, ic[0], ic[1], ic[2]);
    const double X = (double)ic[axis] + (double)P.f[axis][p];
    const double x = (X - (double)g.lo[axis]) * dxa;
    if (!(x >= e[0] && x < e[nslab])) continue;
    int lo = 0, hi = nslab;   // e[lo] <= x < e[hi]
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (x >= e[mid]) lo = mid;
      else hi = mid;
    }
    const double w = (double)P.w[p];
    atomicAdd(&acc[5 * lo + 0], 1.0);
    atomicAdd(&acc[5 * lo + 1], w);
    atomicAdd(&acc[5 * lo + 2], w * (double)P.u[0][p]);
    atomicAdd(&acc[5 * lo + 3], w * (double)P.u[1][p]);
    atomicAdd(&acc[5 * lo + 4], w * (double)P.u[2][p]);
  }
  __syncthreads();
  for (int t = threadIdx.x; t < 5 * nslab; t += blockDim.x)
    if (acc[t] != 0.0) atomicAdd(&out[t], acc[t]);
}

template <typename T>
void launch_slab_moments(const Grid<T> &g, const Parts<T> &P, const int32_t *count, int n_slots, int axis, double dxa,
                         int nslab, const double *edges, double *out, hipStream_t s) {
  (void)hipMemsetAsync(out, 0, sizeof(double) * 5 * (size_t)nslab, s);
  if (n_slots <= 0) return;
  const int blocks = std::min(1024, (n_slots + 255) / 256);
  hipLaunchKernelGGL((k_slab_moments<T>), dim3(blocks), dim3(256), 0, s, g, P, count, n_slots, axis, dxa, nslab,
                     edges, out);
}
template void launch_slab_moments<float>(const Grid<float> &, const Parts<float> &, const int32_t *, int, int, double,
                                         int, const double *, double *, hipStream_t);
template void launch_slab_moments<double>(const Grid<double> &, const Parts<double> &, const int32_t *, int, int,
                                          double, int, const double *, double *, hipStream_t);

}  // namespace pmlpic
