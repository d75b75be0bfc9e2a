// update_yee_pml and damp_pml_current: the split-field Yee/PML update with the damped
// current source (Sec. II.A, Eqs. MaxwellE / MaxwellB / MaxwellSum; Yee centring of
// Sec. II.B) and the current damping J <- alpha J (Eq. alpha).
//
// Storage: each component keeps its total F_a everywhere and, where it is split, the
// part F_ab (b = a+1) in a second array; the other part is F_a - F_ab.  A sample is
// split where sigma_b + sigma_c > 0 at its position; elsewhere both parts are
// undamped and only the total evolves.  In 2D the parts driven by z derivatives never
// change, so E_x, E_y, B_x, B_y are stored unsplit with the one in-plane rate.
//
// Time integration of dF/dt = -sigma F + rhs over tau: F <- e F + g rhs with
// e = exp(-sigma tau), g = (1 - e)/sigma (g = tau where sigma = 0), read from the
// per-axis tables (Berenger's exponential differencing).
//
// Memory-bound stencils: one thread per node, x fastest, coalesced rows.
#include <algorithm>

#include "pml_pic.h"
#include "field_core.h"
#include "fused2d.h"

namespace pmlpic {

// one-pass update_yee_pml in 2D: one wavefront per (strip of FW columns, segment of rows)
template <typename T>
__global__ void __launch_bounds__(256) k_fused_2d(Grid<T> g, Fields<T> F, Fields<T> D, const int *jslot, int nstrips,
                                                  int rows, int nseg, bool fuse_alpha) {
  // workgroup b runs on XCD b mod 8: give each XCD a contiguous eighth of the
  // wavefronts so that neighbouring strips share its L2 (gridDim is a multiple of 8)
  const int per = (int)(gridDim.x >> 3);
  const int b = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
  const int w = b * 4 + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  if (w >= nstrips * nseg) return;   // whole wavefront
  const int strip = w % nstrips, seg = w / nstrips;
  const int y0 = seg * rows, y1 = min(y0 + rows, g.M[1] + 1);
  fused_segment_2d(g, F, D, jslot_union(jslot), strip, y0, y1, fuse_alpha, (int)(threadIdx.x & 63));
}

template <typename T>
__global__ void __launch_bounds__(256) k_jbox_clear(Grid<T> g, JClear<T> jc) {
  jclear_share(g, jc);
}

template <typename T>
void launch_jbox_clear(const Grid<T> &g, const JClear<T> &jc, hipStream_t s) {
  const long n = (long)(g.M[0] + 1 + 2 * G) * (g.M[1] + 1 + 2 * G);
  const int blocks = (int)std::min<long>(1024, (n + 255) / 256);
  hipLaunchKernelGGL((k_jbox_clear<T>), dim3(blocks), dim3(256), 0, s, g, jc);
}
template void launch_jbox_clear<float>(const Grid<float> &, const JClear<float> &, hipStream_t);
template void launch_jbox_clear<double>(const Grid<double> &, const JClear<double> &, hipStream_t);

template <typename T, int DIM, bool CK = false>
__global__ void __launch_bounds__(256) k_update_B(Grid<T> g, Fields<T> F) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
  const int k = (DIM == 3) ? (int)blockIdx.z : 0;
  if (i > g.M[0] || j > g.M[1]) return;
  const int id[3] = {i, j, k};
  const long q = g.at(i, j, k);
  update_B_comp<T, DIM, 0, CK>(g, F, id, q);
  update_B_comp<T, DIM, 1, CK>(g, F, id, q);
  update_B_comp<T, DIM, 2, CK>(g, F, id, q);
}

template <typename T, int DIM>
__global__ void __launch_bounds__(256) k_update_E(Grid<T> g, Fields<T> F, bool fuse_alpha, bool consume) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
  const int k = (DIM == 3) ? (int)blockIdx.z : 0;
  if (i > g.M[0] || j > g.M[1]) return;
  const int id[3] = {i, j, k};
  const long q = g.at(i, j, k);
  update_E_comp<T, DIM, 0>(g, F, id, q, fuse_alpha, consume);
  update_E_comp<T, DIM, 1>(g, F, id, q, fuse_alpha, consume);
  update_E_comp<T, DIM, 2>(g, F, id, q, fuse_alpha, consume);
}

// damp_pml_current: J_A <- alpha J_A at every sample where alpha != 1 (the PML).
template <typename T, int DIM>
__global__ void __launch_bounds__(256) k_damp(Grid<T> g, Fields<T> F) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
  const int k = (DIM == 3) ? (int)blockIdx.z : 0;
  if (i > g.M[0] || j > g.M[1]) return;
  const int id[3] = {i, j, k};
  const long q = g.at(i, j, k);
  const T a0 = alpha_at<T, DIM, 0>(g, id);
  const T a1 = alpha_at<T, DIM, 1>(g, id);
  const T a2 = alpha_at<T, DIM, 2>(g, id);
  if (a0 != T(1)) F.J[0][q] *= a0;
  if (a1 != T(1)) F.J[1][q] *= a1;
  if (a2 != T(1)) F.J[2][q] *= a2;
}

template <typename T>
static dim3 node_grid(const Grid<T> &g, dim3 &blk) {
  blk = dim3(64, 4, 1);
  return dim3((g.M[0] + 1 + 63) / 64, (g.M[1] + 1 + 3) / 4, g.dim == 3 ? g.M[2] + 1 : 1);
}

// rows per segment: enough wavefronts to fill the GPU (about 4096), 8 to 64 rows
void fused_2d_shape(int M0, int M1, int &nstrips, int &rows, int &nseg) {
  nstrips = (M0 + 1 + FW - 1) / FW;
  const long want = 4096;
  rows = (int)std::min<long>(64, std::max<long>(8, (long)nstrips * (M1 + 1) / want));
  nseg = (M1 + 1 + rows - 1) / rows;
}

template <typename T>
void launch_fused_fields(const Grid<T> &g, const Fields<T> &F, const Fields<T> &D, const int *jslot, bool fuse_alpha,
                         hipStream_t s) {
  int nstrips, rows, nseg;
  fused_2d_shape(g.M[0], g.M[1], nstrips, rows, nseg);
  const int waves = nstrips * nseg;
  const int blocks = ((waves + 3) / 4 + 7) / 8 * 8;
  hipLaunchKernelGGL((k_fused_2d<T>), dim3(blocks), dim3(256), 0, s, g, F, D, jslot, nstrips, rows, nseg,
                     fuse_alpha);
}
template void launch_fused_fields<float>(const Grid<float> &, const Fields<float> &, const Fields<float> &,
                                         const int *, bool, hipStream_t);
template void launch_fused_fields<double>(const Grid<double> &, const Fields<double> &, const Fields<double> &,
                                          const int *, bool, hipStream_t);

// B is only ever advanced by half steps (B^n -> B^{n+1/2} -> B^{n+1})
template <typename T>
void launch_update_B(const Grid<T> &g, const Fields<T> &F, bool /*half*/, hipStream_t s) {
  dim3 blk, grd = node_grid(g, blk);
  if (g.dim == 2) hipLaunchKernelGGL((k_update_B<T, 2>), grd, blk, 0, s, g, F);
  else if (g.solver == PML_PIC_SOLVER_CK) hipLaunchKernelGGL((k_update_B<T, 3, true>), grd, blk, 0, s, g, F);
  else hipLaunchKernelGGL((k_update_B<T, 3>), grd, blk, 0, s, g, F);
}

template <typename T>
void launch_update_E(const Grid<T> &g, const Fields<T> &F, bool fuse_alpha, int alpha_mode, bool consume,
                     hipStream_t s) {
  dim3 blk, grd = node_grid(g, blk);
  const bool fa = fuse_alpha && current_alpha(alpha_mode);
  if (g.dim == 2) hipLaunchKernelGGL((k_update_E<T, 2>), grd, blk, 0, s, g, F, fa, consume);
  else hipLaunchKernelGGL((k_update_E<T, 3>), grd, blk, 0, s, g, F, fa, consume);
}

// Binomial filter of the deposited current (App. A), 3D, one pass: dst_A(i,j,k) = sum
// over the 27 neighbours o of w(o_x) w(o_y) w(o_z) src_A(i+o), w = (1/4, 1/2, 1/4), with
// neighbours outside J_A's extent (M_A samples along A, M + 1 across) counting as 0.  The
// weights factor per axis, so each thread owns one (i, j) column of a chunk of kz planes
// and keeps the x-y filtered value of three consecutive planes in registers: a plane is
// read once per chunk (with one halo plane on each side), and only samples of the extent
// are written.  kz is 16 on large grids and shrinks on small ones so that the launch
// still has a few thousand workgroups.
template <typename T>
__global__ void __launch_bounds__(256) k_filter_J(Grid<T> g, const T *src, T *dst, int nchunk, int kz) {
  const int A = (int)blockIdx.z / nchunk, chunk = (int)blockIdx.z % nchunk;
  const int ext0 = g.M[0] + (A != 0), ext1 = g.M[1] + (A != 1), ext2 = g.M[2] + (A != 2);
  const int i = (int)(blockIdx.x * 64 + (threadIdx.x & 63));
  const int j = (int)(blockIdx.y * 4 + (threadIdx.x >> 6));
  const int k0 = chunk * kz, k1 = min(k0 + kz, ext2);
  if (i >= ext0 || j >= ext1 || k0 >= k1) return;
  const T *J = src + (size_t)A * g.nelem;
  T *out = dst + (size_t)A * g.nelem;
  const bool xl = i > 0, xr = i + 1 < ext0, yl = j > 0, yr = j + 1 < ext1;
  auto row = [&](long q) {
    T r = T(0.5) * J[q];
    if (xl) r += T(0.25) * J[q - 1];
    if (xr) r += T(0.25) * J[q + 1];
    return r;
  };
  auto plane = [&](int k) {
    if (k < 0 || k >= ext2) return T(0);
    const long q = g.at(i, j, k);
    T p = T(0.5) * row(q);
    if (yl) p += T(0.25) * row(q - g.sy);
    if (yr) p += T(0.25) * row(q + g.sy);
    return p;
  };
  T pm = plane(k0 - 1), p0 = plane(k0);
  for (int k = k0; k < k1; ++k) {
    const T pp = plane(k + 1);
    out[g.at(i, j, k)] = T(0.25) * pm + T(0.5) * p0 + T(0.25) * pp;
    pm = p0;
    p0 = pp;
  }
}

// passes alternate between J and tmp (the three components of each are adjacent); returns
// the one that holds the result.  Samples outside the extents of tmp are never written
// (the workspace starts zeroed).
template <typename T>
T *launch_filter_current(const Grid<T> &g, T *J, T *tmp, int passes, hipStream_t s) {
  if (g.dim != 3 || passes <= 0) return J;
  const int gx = (g.M[0] + 1 + 63) / 64, gy = (g.M[1] + 1 + 3) / 4;
  const int want = (4096 + 3 * gx * gy - 1) / (3 * gx * gy);   // chunks for ~4096 workgroups
  const int kz = std::max(2, std::min(16, (g.M[2] + 1 + want - 1) / want));
  const int nchunk = (g.M[2] + 1 + kz - 1) / kz;
  dim3 blk(256), grd(gx, gy, 3 * nchunk);
  T *a = J, *b = tmp;
  for (int p = 0; p < passes; ++p) {
    hipLaunchKernelGGL((k_filter_J<T>), grd, blk, 0, s, g, a, b, nchunk, kz);
    std::swap(a, b);
  }
  return a;
}
template float *launch_filter_current<float>(const Grid<float> &, float *, float *, int, hipStream_t);
template double *launch_filter_current<double>(const Grid<double> &, double *, double *, int, hipStream_t);

template <typename T>
void launch_damp_current(const Grid<T> &g, const Fields<T> &F, hipStream_t s) {
  dim3 blk, grd = node_grid(g, blk);
  if (g.dim == 2) hipLaunchKernelGGL((k_damp<T, 2>), grd, blk, 0, s, g, F);
  else hipLaunchKernelGGL((k_damp<T, 3>), grd, blk, 0, s, g, F);
}

template void launch_update_B<float>(const Grid<float> &, const Fields<float> &, bool, hipStream_t);
template void launch_update_B<double>(const Grid<double> &, const Fields<double> &, bool, hipStream_t);
template void launch_update_E<float>(const Grid<float> &, const Fields<float> &, bool, int, bool, hipStream_t);
template void launch_update_E<double>(const Grid<double> &, const Fields<double> &, bool, int, bool, hipStream_t);
template void launch_damp_current<float>(const Grid<float> &, const Fields<float> &, hipStream_t);
template void launch_damp_current<double>(const Grid<double> &, const Fields<double> &, hipStream_t);

}  // namespace pmlpic
