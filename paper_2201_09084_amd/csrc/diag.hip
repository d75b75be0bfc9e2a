// reduce_diag_fp64: FP64 diagnostics over FP32 or FP64 state.
//   * field energy 1/2 sum (E^2 + B^2) dV split into samples inside the physical box
//     and the rest (the energy norm of Eq. error, Sec. III);
//   * charge density of the live particles deposited in FP64 at the nodes (same
//     B-spline as the current) and the Gauss residual div E - rho - rho_partner over
//     nodes strictly inside the physical box (App. A.1: the partner makes
//     div E = rho hold from t = 0);
//   * live particle count and a non-finite flag.
// Deterministic two-pass reductions: per-block partials, then one block.
#include <algorithm>
#include <mutex>

#include "common.h"

namespace pmlpic {

constexpr int RB = 256;

__device__ __forceinline__ double block_sum(double v, double *sh) {
  const int t = threadIdx.x + threadIdx.y * blockDim.x;
  const int n = blockDim.x * blockDim.y;
  sh[t] = v;
  __syncthreads();
  for (int off = n / 2; off > 0; off >>= 1) {
    if (t < off) sh[t] += sh[t + off];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

__device__ __forceinline__ double block_max(double v, double *sh) {
  const int t = threadIdx.x + threadIdx.y * blockDim.x;
  const int n = blockDim.x * blockDim.y;
  sh[t] = v;
  __syncthreads();
  for (int off = n / 2; off > 0; off >>= 1) {
    if (t < off) sh[t] = fmax(sh[t], sh[t + off]);
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

template <typename T>
__device__ __forceinline__ bool in_box(const Grid<T> &g, double X, int d) {
  return X >= (double)g.lo[d] && X <= (double)(g.lo[d] + g.n[d]);
}

// energy partials: partial[4*b + 0] interior, +1 pml; non-finite flag
template <typename T, int DIM>
__global__ void __launch_bounds__(RB) k_energy(Grid<T> g, Fields<T> F, double *partial, int32_t *flags) {
  __shared__ double sh[RB];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
  const int k = (DIM == 3) ? (int)blockIdx.z : 0;
  double ui = 0.0, up = 0.0;
  bool bad = false;
  if (i <= g.M[0] && j <= g.M[1]) {
    const long q = g.at(i, j, k);
    const int id[3] = {i, j, k};
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      const int a = c % 3;
      bool valid = true, phys = true;
#pragma unroll
      for (int d = 0; d < DIM; ++d) {
        const bool stag = (c < 3) ? (d == a) : (d != a);
        if (id[d] > g.M[d] - (stag ? 1 : 0)) valid = false;
        phys = phys && in_box(g, id[d] + (stag ? 0.5 : 0.0), d);
      }
      if (!valid) continue;
      const T *arr = c < 3 ? F.E[a] : F.B[a];
      const double v = (double)arr[q];
      if (!isfinite(v)) bad = true;
      if (phys) ui += 0.5 * v * v; else up += 0.5 * v * v;
    }
  }
  double dV = 1.0;
  for (int d = 0; d < DIM; ++d) dV /= (double)g.inv_dx[d];
  const int b = (blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
  const double si = block_sum(ui * dV, sh);
  const double sp = block_sum(up * dV, sh);
  if (threadIdx.x == 0 && threadIdx.y == 0) { partial[4 * b] = si; partial[4 * b + 1] = sp; }
  if (bad) flags[0] = 1;
}

// FP64 charge density of live particles (sign * q w S / dV) at the nodes
template <typename T, int DIM, int ORDER>
__global__ void __launch_bounds__(256) k_rho(Grid<T> g, Parts<T> P, const int32_t *count, int first,
                                              int n_slots, double *rho, double sign) {
  const int p = first + blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n_slots || p >= *count) return;
  const uint32_t c = P.cell[p];
  if (c == DEAD) return;
  int id[3];
  unpack_cell(DIM, c, id[0], id[1], id[2]);
  double wts[3][ORDER + 1];
  int st[3] = {0, 0, 0};
  for (int d = 0; d < DIM; ++d) st[d] = id[d] + shape_weights<ORDER>((double)P.f[d][p], wts[d]);
  double dV = 1.0;
  for (int d = 0; d < DIM; ++d) dV /= (double)g.inv_dx[d];
  double w = (double)P.w[p];
  if (g.wdamp) w *= exp(-(double)P.lam[p]);   // weight damping: the particle's present charge
  const double qw = sign * (double)g.charge * w / dV;
  const int nz = DIM == 3 ? ORDER + 1 : 1;
  for (int cz = 0; cz < nz; ++cz)
    for (int b = 0; b <= ORDER; ++b)
      for (int a = 0; a <= ORDER; ++a) {
        double wv = wts[0][a] * wts[1][b] * (DIM == 3 ? wts[2][cz] : 1.0);
        if (wv == 0.0) continue;
        atomicAdd(&rho[g.at(st[0] + a, st[1] + b, DIM == 3 ? st[2] + cz : 0)], qw * wv);
      }
}

// Gauss residual partials: partial[4*b + 2] max|r|, +3 sum r^2; rho max in a separate pass
template <typename T, int DIM>
__global__ void __launch_bounds__(RB) k_gauss(Grid<T> g, Fields<T> F, const double *rho, const double *rho_static,
                                              double *partial) {
  __shared__ double sh[RB];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
  const int k = (DIM == 3) ? (int)blockIdx.z : 0;
  double rmax = 0.0, rsum = 0.0;
  if (i <= g.M[0] && j <= g.M[1]) {
    const int id[3] = {i, j, k};
    bool inner = true;
    for (int d = 0; d < DIM; ++d) inner = inner && id[d] > g.lo[d] && id[d] < g.lo[d] + g.n[d];
    if (inner) {
      const long q = g.at(i, j, k);
      const long st[3] = {1L, g.sy, g.sz};
      double div = 0.0;
      for (int d = 0; d < DIM; ++d) div += ((double)F.E[d][q] - (double)F.E[d][q - st[d]]) * (double)g.inv_dx[d];
      const double r = div - rho[q] - rho_static[q];
      rmax = fabs(r);
      rsum = r * r;
    }
  }
  const int b = (blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
  const double m = block_max(rmax, sh);
  const double s2 = block_sum(rsum, sh);
  if (threadIdx.x == 0 && threadIdx.y == 0) { partial[4 * b + 2] = m; partial[4 * b + 3] = s2; }
}

__global__ void __launch_bounds__(RB) k_rho_max(const double *rho, long n, double *partial_rmax) {
  __shared__ double sh[RB];
  double m = 0.0;
  for (long q = (long)blockIdx.x * RB + threadIdx.x; q < n; q += (long)gridDim.x * RB) m = fmax(m, fabs(rho[q]));
  m = block_max(m, sh);
  if (threadIdx.x == 0) partial_rmax[blockIdx.x] = m;
}

template <typename T>
__global__ void __launch_bounds__(RB) k_count_live(Parts<T> P, const int32_t *count, int n_slots, int32_t *live) {
  __shared__ double sh[RB];
  const int p = blockIdx.x * RB + threadIdx.x;
  const double v = (p < n_slots && p < *count && P.cell[p] != DEAD) ? 1.0 : 0.0;
  const double s = block_sum(v, sh);
  if (threadIdx.x == 0 && s > 0) atomicAdd(live, (int32_t)s);
}

// result: [0] U interior, [1] U pml, [2] gauss max, [3] gauss sum sq, [4] rho max
__global__ void __launch_bounds__(RB) k_final(const double *partial, int nb, const double *rmaxp, int nrb,
                                              double *result) {
  __shared__ double sh[RB];
  double a = 0, b = 0, c = 0, d = 0, e = 0;
  for (int t = threadIdx.x; t < nb; t += RB) {
    a += partial[4 * t]; b += partial[4 * t + 1];
    c = fmax(c, partial[4 * t + 2]); d += partial[4 * t + 3];
  }
  for (int t = threadIdx.x; t < nrb; t += RB) e = fmax(e, rmaxp[t]);
  a = block_sum(a, sh); b = block_sum(b, sh); d = block_sum(d, sh);
  c = block_max(c, sh); e = block_max(e, sh);
  if (threadIdx.x == 0) { result[0] = a; result[1] = b; result[2] = c; result[3] = d; result[4] = e; }
}

template <typename T>
static dim3 diag_grid(const Grid<T> &g, dim3 &blk) {
  blk = dim3(64, 4, 1);
  return dim3((g.M[0] + 1 + 63) / 64, (g.M[1] + 1 + 3) / 4, g.dim == 3 ? g.M[2] + 1 : 1);
}

template <typename T>
void launch_rho(const Grid<T> &g, const Parts<T> &P, StepCtl ctl, int first, int n_slots, double *rho,
                double sign, hipStream_t s) {
  const int n = n_slots - first;
  if (n <= 0) return;
  dim3 blk(256), grd((n + 255) / 256);
#define PMLPIC_RHO(DIMV, ORD) hipLaunchKernelGGL((k_rho<T, DIMV, ORD>), grd, blk, 0, s, g, P, ctl.count, first, n_slots, rho, sign)
  if (g.dim == 2) {
    if (g.order == 1) PMLPIC_RHO(2, 1); else if (g.order == 2) PMLPIC_RHO(2, 2); else PMLPIC_RHO(2, 3);
  } else {
    if (g.order == 1) PMLPIC_RHO(3, 1); else if (g.order == 2) PMLPIC_RHO(3, 2); else PMLPIC_RHO(3, 3);
  }
#undef PMLPIC_RHO
}

template <typename T>
void launch_diag(const Grid<T> &g, const Fields<T> &F, const Parts<T> &P, StepCtl ctl, int n_slots,
                 DiagWork dw, hipStream_t s) {
  dim3 blk, grd = diag_grid(g, blk);
  const int nb = grd.x * grd.y * grd.z;
  hipMemsetAsync(dw.flags, 0, 2 * sizeof(int32_t), s);
  hipMemsetAsync(dw.rho, 0, sizeof(double) * (size_t)g.nelem, s);
  if (g.dim == 2) hipLaunchKernelGGL((k_energy<T, 2>), grd, blk, 0, s, g, F, dw.partial, dw.flags);
  else hipLaunchKernelGGL((k_energy<T, 3>), grd, blk, 0, s, g, F, dw.partial, dw.flags);
  launch_rho<T>(g, P, ctl, 0, n_slots, dw.rho, 1.0, s);
  if (g.dim == 2) hipLaunchKernelGGL((k_gauss<T, 2>), grd, blk, 0, s, g, F, dw.rho, dw.rho_static, dw.partial);
  else hipLaunchKernelGGL((k_gauss<T, 3>), grd, blk, 0, s, g, F, dw.rho, dw.rho_static, dw.partial);
  const int nrb = 1024;
  double *rmaxp = dw.partial + 4 * (size_t)nb;
  hipLaunchKernelGGL(k_rho_max, dim3(nrb), dim3(RB), 0, s, dw.rho, g.nelem, rmaxp);
  if (n_slots > 0)
    hipLaunchKernelGGL((k_count_live<T>), dim3((n_slots + RB - 1) / RB), dim3(RB), 0, s, P, ctl.count, n_slots,
                       dw.flags + 1);
  hipLaunchKernelGGL(k_final, dim3(1), dim3(RB), 0, s, dw.partial, nb, rmaxp, nrb, dw.result);
}

// Eq. (error) of Sec. III against a reference run: partial[2*b] = sum over the samples of
// g's physical box of (F - F_ref)^2, partial[2*b + 1] = sum of F_ref^2 (E and B, the six
// totals).  The reference grid has the same cell size and low PML and covers g's physical
// box, so a sample has the same index in both.  Workgroup (bx, by, bz) covers x-block bx
// and the (y-block, plane) pairs by + m gridDim.y, bz + n gridDim.z (one pair when the
// grid spans every block); then one block sums the partials.
template <typename T, int DIM>
__global__ void __launch_bounds__(RB) k_field_error(Grid<T> g, Fields<T> F, Grid<T> gr, Fields<T> R,
                                                    double *partial) {
  __shared__ double sh[RB];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int kmax = DIM == 3 ? g.M[2] : 0;
  double num = 0.0, den = 0.0;
  for (int k = (DIM == 3) ? (int)blockIdx.z : 0; k <= kmax; k += (int)gridDim.z) {
    for (int jb = (int)blockIdx.y; jb * (int)blockDim.y <= g.M[1]; jb += (int)gridDim.y) {
      const int j = jb * (int)blockDim.y + (int)threadIdx.y;
      if (i > g.M[0] || j > g.M[1]) continue;
      const long q = g.at(i, j, k), qr = gr.at(i, j, k);
      const int id[3] = {i, j, k};
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        const int a = c % 3;
        bool phys = true;
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
          const bool stag = (c < 3) ? (d == a) : (d != a);
          phys = phys && in_box(g, id[d] + (stag ? 0.5 : 0.0), d);
        }
        if (!phys) continue;
        const double v = (double)(c < 3 ? F.E[a] : F.B[a])[q];
        const double r = (double)(c < 3 ? R.E[a] : R.B[a])[qr];
        num += (v - r) * (v - r);
        den += r * r;
      }
    }
  }
  const int b = (blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
  const double sn = block_sum(num, sh);
  const double sd = block_sum(den, sh);
  if (threadIdx.x == 0 && threadIdx.y == 0) { partial[2 * b] = sn; partial[2 * b + 1] = sd; }
}

__global__ void __launch_bounds__(RB) k_sum_pairs(const double *partial, int nb, double *out) {
  __shared__ double sh[RB];
  double a = 0.0, c = 0.0;
  for (int b = threadIdx.x; b < nb; b += RB) { a += partial[2 * b]; c += partial[2 * b + 1]; }
  a = block_sum(a, sh);
  c = block_sum(c, sh);
  if (threadIdx.x == 0) { out[0] = a; out[1] = c; }
}

// one workgroup per (x-block, y-block, plane), partial pairs in the handle's workspace
template <typename T>
void launch_field_error(const Grid<T> &g, const Fields<T> &F, const Grid<T> &gr, const Fields<T> &R, double *partial,
                        double *out, hipStream_t s) {
  dim3 blk(64, 4, 1), grd((g.M[0] + 1 + 63) / 64, (g.M[1] + 1 + 3) / 4, g.dim == 3 ? g.M[2] + 1 : 1);
  if (g.dim == 2) hipLaunchKernelGGL((k_field_error<T, 2>), grd, blk, 0, s, g, F, gr, R, partial);
  else hipLaunchKernelGGL((k_field_error<T, 3>), grd, blk, 0, s, g, F, gr, R, partial);
  hipLaunchKernelGGL(k_sum_pairs, dim3(1), dim3(RB), 0, s, partial, (int)(grd.x * grd.y * grd.z), out);
}

// ------------------------------------------------ Eq. (error) without allocation
// For callers that cannot allocate (code under HIP graph capture, tight serving loops):
// the partial sums and the result live in this file-scope device array instead of the
// handle's workspace.  Every GPU the library runs on holds one copy (513 KiB) until the
// process ends; every call on that GPU shares it, so calls that overlap on one GPU
// race.  Nothing in it needs to start at zero: each call writes every partial it reads.
constexpr int FE_SCRATCH_PAIRS = 32768;                 // partial (num, den) pairs
constexpr int FE_SCRATCH_RESULT = 64;                   // doubles before the partials
static __device__ __align__(256) double scratch[FE_SCRATCH_RESULT + 2 * FE_SCRATCH_PAIRS];

namespace {
constexpr int FE_MAX_DEVICES = 64;
double *g_scratch_ptr[FE_MAX_DEVICES] = {};
std::mutex g_scratch_mu;
}  // namespace

// Device address of `scratch` on the current device, looked up once per device (in
// host code the array's name is only a stand-in for that address).
hipError_t field_error_scratch(double **ptr) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= FE_MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = (double *)p;
  }
  *ptr = g_scratch_ptr[dev];
  return hipSuccess;
}

int field_error_scratch_pairs() { return FE_SCRATCH_PAIRS; }

// The same sums with at most FE_SCRATCH_PAIRS workgroups (each covers several y-blocks
// and planes when the grid is larger), partials and result in `sc` (the device address
// of `scratch`); returns false, launching nothing, if one row of x-blocks alone needs
// more workgroups than that (no grid within the library's size limits does).
template <typename T>
bool launch_field_error_scratch(const Grid<T> &g, const Fields<T> &F, const Grid<T> &gr, const Fields<T> &R,
                                double *sc, hipStream_t s) {
  const long gx = (g.M[0] + 1 + 63) / 64, gy = (g.M[1] + 1 + 3) / 4, gz = g.dim == 3 ? g.M[2] + 1 : 1;
  if (gx > FE_SCRATCH_PAIRS) return false;
  long cy = std::min<long>(gy, FE_SCRATCH_PAIRS / gx);
  long cz = std::min<long>(gz, FE_SCRATCH_PAIRS / (gx * cy));
  dim3 blk(64, 4, 1), grd((unsigned)gx, (unsigned)cy, (unsigned)cz);
  double *partial = sc + FE_SCRATCH_RESULT;
  if (g.dim == 2) hipLaunchKernelGGL((k_field_error<T, 2>), grd, blk, 0, s, g, F, gr, R, partial);
  else hipLaunchKernelGGL((k_field_error<T, 3>), grd, blk, 0, s, g, F, gr, R, partial);
  hipLaunchKernelGGL(k_sum_pairs, dim3(1), dim3(RB), 0, s, partial, (int)(gx * cy * cz), sc);
  return true;
}
template bool launch_field_error_scratch<float>(const Grid<float> &, const Fields<float> &, const Grid<float> &,
                                                const Fields<float> &, double *, hipStream_t);
template bool launch_field_error_scratch<double>(const Grid<double> &, const Fields<double> &, const Grid<double> &,
                                                 const Fields<double> &, double *, hipStream_t);
template void launch_field_error<float>(const Grid<float> &, const Fields<float> &, const Grid<float> &,
                                        const Fields<float> &, double *, double *, hipStream_t);
template void launch_field_error<double>(const Grid<double> &, const Fields<double> &, const Grid<double> &,
                                         const Fields<double> &, double *, double *, hipStream_t);

template void launch_diag<float>(const Grid<float> &, const Fields<float> &, const Parts<float> &, StepCtl, int,
                                 DiagWork, hipStream_t);
template void launch_diag<double>(const Grid<double> &, const Fields<double> &, const Parts<double> &, StepCtl,
                                  int, DiagWork, hipStream_t);
template void launch_rho<float>(const Grid<float> &, const Parts<float> &, StepCtl, int, int, double *, double,
                                hipStream_t);
template void launch_rho<double>(const Grid<double> &, const Parts<double> &, StepCtl, int, int, double *, double,
                                 hipStream_t);

}  // namespace pmlpic
