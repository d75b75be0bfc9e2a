// Reverse mode of update_yee_pml and of the alpha damping.  For given current the field
// update is linear in the state:  B' = eh B + ghk D(E) (half step),
// E' = e E + gk D(B') - g w alpha J, then B'' from B' and E'.  (Pushed runs also reverse
// the particles, adjoint_particles.hip, from the current's adjoint written here.)  Its
// transpose runs backwards with
//   * curl-transpose kernels: the adjoint of every neighbour difference, written as a
//     gather over the samples that read a given sample (no atomics);
//   * self kernels: lambda <- e lambda per split part, and the FP64 derivatives of the
//     objective with respect to every per-axis table entry (e, g, g/dx at nodes; e, g/dx
//     for half steps at centres; alpha at nodes and centres; sigma through the current's
//     split weights), reduced inside each workgroup before one atomic per entry.
// Adjoint storage per component: LT (adjoint of the part driven along a+2, equal to the
// adjoint of the total where the component is not split) and LA (adjoint of the part
// driven along a+1 minus LT, used only where the component is split).
#include "field_core.h"

namespace pmlpic {

enum GradKind { G_E_N = 0, G_G_N, G_GK_N, G_EH_C, G_GHK_C, G_A_N, G_A_C, G_SIG_N, G_NKIND };

template <typename T, int DIM>
__device__ __forceinline__ bool is_split(const Grid<T> &g, bool isE, int A, const int (&id)[3]) {
  const int Bx = (A + 1) % 3, Cx = (A + 2) % 3;
  if (DIM == 2 && (Bx == 2 || Cx == 2)) return false;
  const int kind = isE ? T_SIG_N : T_SIG_C;
  return g.tb(Bx, kind, id[Bx]) + g.tb(Cx, kind, id[Cx]) > T(0);
}

// valid extent of a sample; for E also off the PEC walls (samples the E update changes)
template <typename T, int DIM>
__device__ __forceinline__ bool e_updated(const Grid<T> &g, int A, const int (&id)[3]) {
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    if (d == A) { if (id[d] < 0 || id[d] > g.M[d] - 1) return false; }
    else if (id[d] < 1 || id[d] > g.M[d] - 1) return false;
  }
  return true;
}
template <typename T, int DIM>
__device__ __forceinline__ bool b_valid(const Grid<T> &g, int A, const int (&id)[3]) {
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    if (d == A) { if (id[d] < 0 || id[d] > g.M[d]) return false; }
    else if (id[d] < 0 || id[d] > g.M[d] - 1) return false;
  }
  return true;
}

template <typename T, int DIM>
__device__ __forceinline__ long stride_ax(const Grid<T> &g, int axis) {
  return axis == 0 ? 1L : (axis == 1 ? g.sy : g.sz);
}

// ---------------------------------------------------------------- gradient reduction
// Per-thread contributions acc[axis][kind] at this thread's index along each axis are
// summed over the workgroup (64 x 4 threads: x varies along lanes, y along waves) and
// added to G[(axis * G_NKIND + kind) * ntab + index + G] with one FP64 atomic per
// distinct index.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

template <int DIM>
__device__ void flush_grads(double (&acc)[3][G_NKIND], const int (&id)[3], double *Gacc, int ntab) {
  __shared__ double colsum[G_NKIND][64];
  __shared__ double plane[G_NKIND][4];
  const int tx = threadIdx.x, ty = threadIdx.y;
  // axis 0: sum over the 4 rows sharing tx
  for (int k = 0; k < G_NKIND; ++k) {
    if (ty == 0) colsum[k][tx] = 0.0;
  }
  __syncthreads();
  for (int k = 0; k < G_NKIND; ++k)
    if (acc[0][k] != 0.0) atomicAdd(&colsum[k][tx], acc[0][k]);
  __syncthreads();
  if (ty == 0) {
    for (int k = 0; k < G_NKIND; ++k) {
      const double v = colsum[k][tx];
      if (v != 0.0) atomicAdd(&Gacc[(0 * G_NKIND + k) * ntab + id[0] + G], v);
    }
  }
  // axis 1: sum over the 64 lanes of a row (one wavefront)
  for (int k = 0; k < G_NKIND; ++k) {
    const double v = wave_sum(acc[1][k]);
    if (tx == 0 && v != 0.0) atomicAdd(&Gacc[(1 * G_NKIND + k) * ntab + id[1] + G], v);
  }
  if (DIM == 3) {   // axis 2: one z index per workgroup
    for (int k = 0; k < G_NKIND; ++k) {
      const double v = wave_sum(acc[2][k]);
      if (tx == 0) plane[k][ty] = v;
    }
    __syncthreads();
    if (tx == 0 && ty == 0) {
      for (int k = 0; k < G_NKIND; ++k) {
        const double v = plane[k][0] + plane[k][1] + plane[k][2] + plane[k][3];
        if (v != 0.0) atomicAdd(&Gacc[(2 * G_NKIND + k) * ntab + id[2] + G], v);
      }
    }
  }
}

// ---------------------------------------------------------------- seeds
// lambda of the interior energy U = 1/2 sum (E^2 + B^2) dV over samples in the box
template <typename T, int DIM>
__global__ void __launch_bounds__(256) k_adj_seed_energy(Grid<T> g, Fields<T> F, AdjFields<T> L) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
  const int k = (DIM == 3) ? (int)blockIdx.z : 0;
  if (i > g.M[0] || j > g.M[1]) return;
  const int id[3] = {i, j, k};
  const long q = g.at(i, j, k);
  T dV = T(1);
#pragma unroll
  for (int d = 0; d < DIM; ++d) dV /= g.inv_dx[d];
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    const int a = c % 3;
    bool valid = true, inside = true;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      const bool stag = (c < 3) ? (d == a) : (d != a);
      if (id[d] > g.M[d] - (stag ? 1 : 0)) valid = false;
      const T X = T(id[d]) + (stag ? T(0.5) : T(0));
      inside = inside && X >= T(g.lo[d]) && X <= T(g.lo[d] + g.n[d]);
    }
    const T *arr = c < 3 ? F.E[a] : F.B[a];
    L.LT[c][q] = (valid && inside) ? arr[q] * dV : T(0);
    L.LA[c][q] = T(0);
  }
}

// ---------------------------------------------------------------- B half step
// lambda_E += (d B_half / d E)^T lambda_B
template <typename T, int DIM>
__global__ void __launch_bounds__(256) k_adj_B_curl(Grid<T> g, AdjFields<T> L) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
  const int k = (DIM == 3) ? (int)blockIdx.z : 0;
  if (i > g.M[0] || j > g.M[1]) return;
  const int id[3] = {i, j, k};
  const long q = g.at(i, j, k);
#pragma unroll
  for (int C = 0; C < 3; ++C) {
    // E_C is read by B_{C+1} (part driven along C+2) and B_{C+2} (part driven along C+1)
    bool ok = true;
#pragma unroll
    for (int d = 0; d < DIM; ++d) ok = ok && id[d] <= g.M[d] - (d == C ? 1 : 0);
    if (!ok) continue;
    T acc = T(0);
    const int A1 = (C + 1) % 3, b1 = (C + 2) % 3;   // B_{A1}, its part b = A1+1 = C+2
    if (b1 < DIM) {
      const long s = stride_ax<T, DIM>(g, b1);
      int idm[3] = {id[0], id[1], id[2]};
      idm[b1] -= 1;
      T l0 = L.LT[3 + A1][q], l1 = L.LT[3 + A1][q - s];
      if (is_split<T, DIM>(g, false, A1, id)) l0 += L.LA[3 + A1][q];
      if (idm[b1] >= 0 && is_split<T, DIM>(g, false, A1, idm)) l1 += L.LA[3 + A1][q - s];
      acc += g.tb(b1, T_GHK_C, id[b1]) * l0 - g.tb(b1, T_GHK_C, idm[b1]) * l1;
    }
    const int A2 = (C + 2) % 3, c2 = (C + 1) % 3;   // B_{A2}, its part c = A2+2 = C+1
    if (c2 < DIM) {
      const long s = stride_ax<T, DIM>(g, c2);
      int idm[3] = {id[0], id[1], id[2]};
      idm[c2] -= 1;
      const T l0 = L.LT[3 + A2][q], l1 = L.LT[3 + A2][q - s];
      acc += -g.tb(c2, T_GHK_C, id[c2]) * l0 + g.tb(c2, T_GHK_C, idm[c2]) * l1;
    }
    L.LT[C][q] += acc;
  }
}

// lambda_B <- (d B_half / d B)^T lambda_B, gradients of eh and ghk
template <typename T, int DIM>
__global__ void __launch_bounds__(256) k_adj_B_self(Grid<T> g, AdjFields<T> L, Fields<T> Fb, double *Gacc) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
  const int k = (DIM == 3) ? (int)blockIdx.z : 0;
  const int id[3] = {i, j, k};
  double acc[3][G_NKIND];
#pragma unroll
  for (int d = 0; d < 3; ++d)
#pragma unroll
    for (int kk = 0; kk < G_NKIND; ++kk) acc[d][kk] = 0.0;
  if (i <= g.M[0] && j <= g.M[1]) {
    const long q = g.at(i, j, k);
#pragma unroll
    for (int A = 0; A < 3; ++A) {
      if (!b_valid<T, DIM>(g, A, id)) continue;
      const int Bx = (A + 1) % 3, Cx = (A + 2) % 3;
      T Db = T(0), Dc = T(0);
      if (Bx < DIM) Db = Fb.E[Cx][q + stride_ax<T, DIM>(g, Bx)] - Fb.E[Cx][q];
      if (Cx < DIM) Dc = Fb.E[Bx][q + stride_ax<T, DIM>(g, Cx)] - Fb.E[Bx][q];
      const T lt = L.LT[3 + A][q];
      if (DIM == 2 && (Bx == 2 || Cx == 2)) {
        const int P = (Bx == 2) ? Cx : Bx;
        const T e = g.tb(P, T_EH_C, id[P]);
        acc[P][G_EH_C] += (double)lt * (double)Fb.B[A][q];
        acc[P][G_GHK_C] += (double)lt * (double)(P == Bx ? -Db : Dc);
        L.LT[3 + A][q] = e * lt;
      } else if (is_split<T, DIM>(g, false, A, id)) {
        const T lb = lt + L.LA[3 + A][q], lc = lt;
        const T p1 = Fb.Ba[A][q], p2 = Fb.B[A][q] - p1;
        acc[Bx][G_EH_C] += (double)lb * (double)p1;
        acc[Cx][G_EH_C] += (double)lc * (double)p2;
        acc[Bx][G_GHK_C] += (double)lb * (double)(-Db);
        acc[Cx][G_GHK_C] += (double)lc * (double)Dc;
        const T nb = g.tb(Bx, T_EH_C, id[Bx]) * lb, nc = g.tb(Cx, T_EH_C, id[Cx]) * lc;
        L.LT[3 + A][q] = nc;
        L.LA[3 + A][q] = nb - nc;
      }
    }
  }
  flush_grads<DIM>(acc, id, Gacc, g.ntab);
}

// ---------------------------------------------------------------- E step
// lambda_B += (d E' / d B)^T lambda_E
template <typename T, int DIM>
__global__ void __launch_bounds__(256) k_adj_E_curl(Grid<T> g, AdjFields<T> L) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
  const int k = (DIM == 3) ? (int)blockIdx.z : 0;
  if (i > g.M[0] || j > g.M[1]) return;
  const int id[3] = {i, j, k};
  const long q = g.at(i, j, k);
#pragma unroll
  for (int C = 0; C < 3; ++C) {
    if (!b_valid<T, DIM>(g, C, id)) continue;
    T acc = T(0);
    // B_C is read by E_{C+1} (part driven along C+2, +d) and E_{C+2} (part driven along C+1, -d)
    const int A1 = (C + 1) % 3, b1 = (C + 2) % 3;
    if (b1 < DIM) {
      int idp[3] = {id[0], id[1], id[2]};
      idp[b1] += 1;
      const long s = stride_ax<T, DIM>(g, b1);
      T l0 = T(0), l1 = T(0);
      if (e_updated<T, DIM>(g, A1, id)) {
        l0 = L.LT[A1][q];
        if (is_split<T, DIM>(g, true, A1, id)) l0 += L.LA[A1][q];
      }
      if (e_updated<T, DIM>(g, A1, idp)) {
        l1 = L.LT[A1][q + s];
        if (is_split<T, DIM>(g, true, A1, idp)) l1 += L.LA[A1][q + s];
      }
      acc += g.tb(b1, T_GK_N, id[b1]) * l0 - g.tb(b1, T_GK_N, idp[b1]) * l1;
    }
    const int A2 = (C + 2) % 3, c2 = (C + 1) % 3;
    if (c2 < DIM) {
      int idp[3] = {id[0], id[1], id[2]};
      idp[c2] += 1;
      const long s = stride_ax<T, DIM>(g, c2);
      const T l0 = e_updated<T, DIM>(g, A2, id) ? L.LT[A2][q] : T(0);
      const T l1 = e_updated<T, DIM>(g, A2, idp) ? L.LT[A2][q + s] : T(0);
      acc += -g.tb(c2, T_GK_N, id[c2]) * l0 + g.tb(c2, T_GK_N, idp[c2]) * l1;
    }
    L.LT[3 + C][q] += acc;
  }
}

// lambda_E <- (d E' / d E)^T lambda_E; gradients of e, g, g/dx, alpha and sigma (through
// the split weights of the current); J is the undamped current of the step.  With LJ0
// set (pushed runs) also writes the adjoint of that current, dU/dJ = -(g alpha)^T lambda_E,
// to LJ0..LJ2 (0 where E is not updated)
template <typename T, int DIM>
__global__ void __launch_bounds__(256) k_adj_E_self(Grid<T> g, AdjFields<T> L, Fields<T> Fe, const T *J0,
                                                   const T *J1, const T *J2, int alpha_mode, double *Gacc,
                                                   T *LJ0, T *LJ1, T *LJ2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
  const int k = (DIM == 3) ? (int)blockIdx.z : 0;
  const int id[3] = {i, j, k};
  double acc[3][G_NKIND];
#pragma unroll
  for (int d = 0; d < 3; ++d)
#pragma unroll
    for (int kk = 0; kk < G_NKIND; ++kk) acc[d][kk] = 0.0;
  if (i <= g.M[0] && j <= g.M[1]) {
    const long q = g.at(i, j, k);
    const T *Js[3] = {J0, J1, J2};
    T *LJ[3] = {LJ0, LJ1, LJ2};
#pragma unroll
    for (int A = 0; A < 3; ++A) {
      if (!e_updated<T, DIM>(g, A, id)) {
        if (LJ0) LJ[A][q] = T(0);
        continue;
      }
      const int Bx = (A + 1) % 3, Cx = (A + 2) % 3;
      T Db = T(0), Dc = T(0);
      if (Bx < DIM) Db = Fe.B[Cx][q] - Fe.B[Cx][q - stride_ax<T, DIM>(g, Bx)];
      if (Cx < DIM) Dc = Fe.B[Bx][q] - Fe.B[Bx][q - stride_ax<T, DIM>(g, Cx)];
      const T jr = Js[A][q];
      T al = T(1), axis_al[3] = {T(1), T(1), T(1)};
      if (alpha_mode != 1) {
#pragma unroll
        for (int d = 0; d < DIM; ++d) { axis_al[d] = g.tb(d, d == A ? T_A_C : T_A_N, id[d]); al *= axis_al[d]; }
      }
      const T lt = L.LT[A][q];
      double dU_daj = 0.0;   // dU/d(alpha J) at this sample
      if (DIM == 2 && (Bx == 2 || Cx == 2)) {
        const int P = (Bx == 2) ? Cx : Bx;
        const T e = g.tb(P, T_E_N, id[P]), gg = g.tb(P, T_G_N, id[P]);
        acc[P][G_E_N] += (double)lt * (double)Fe.E[A][q];
        acc[P][G_GK_N] += (double)lt * (double)(P == Bx ? Db : -Dc);
        acc[P][G_G_N] += (double)lt * (double)(-al * jr);
        dU_daj = -(double)lt * (double)gg;
        L.LT[A][q] = e * lt;
      } else if (is_split<T, DIM>(g, true, A, id)) {
        const T lb = lt + L.LA[A][q], lc = lt;
        const T p1 = Fe.Ea[A][q], p2 = Fe.E[A][q] - p1;
        const double sb = g.tb(Bx, T_SIG_N, id[Bx]), sc = g.tb(Cx, T_SIG_N, id[Cx]);
        const double S = sb + sc, wb = sb / S, wc = sc / S;
        const double gb = g.tb(Bx, T_G_N, id[Bx]), gc = g.tb(Cx, T_G_N, id[Cx]);
        const double aj = (double)al * (double)jr;
        acc[Bx][G_E_N] += (double)lb * (double)p1;
        acc[Cx][G_E_N] += (double)lc * (double)p2;
        acc[Bx][G_GK_N] += (double)lb * (double)Db;
        acc[Cx][G_GK_N] += (double)lc * (double)(-Dc);
        acc[Bx][G_G_N] += (double)lb * (-wb * aj);
        acc[Cx][G_G_N] += (double)lc * (-wc * aj);
        acc[Bx][G_SIG_N] += -aj * (sc / (S * S)) * ((double)lb * gb - (double)lc * gc);
        acc[Cx][G_SIG_N] += -aj * (sb / (S * S)) * ((double)lc * gc - (double)lb * gb);
        dU_daj = -((double)lb * gb * wb + (double)lc * gc * wc);
        const T nb = g.tb(Bx, T_E_N, id[Bx]) * lb, nc = g.tb(Cx, T_E_N, id[Cx]) * lc;
        L.LT[A][q] = nc;
        L.LA[A][q] = nb - nc;
      } else {
        dU_daj = -(double)lt * (double)g.dt;
      }
      if (LJ0) LJ[A][q] = (T)(dU_daj * (double)al);
      const double dU_dalpha = dU_daj * (double)jr;
      if (alpha_mode != 1 && dU_dalpha != 0.0) {
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
          double other = 1.0;
#pragma unroll
          for (int e2 = 0; e2 < DIM; ++e2) if (e2 != d) other *= (double)axis_al[e2];
          acc[d][d == A ? G_A_C : G_A_N] += dU_dalpha * other;
        }
      }
    }
  }
  flush_grads<DIM>(acc, id, Gacc, g.ntab);
}

// ---------------------------------------------------------------- launchers
template <typename T>
static dim3 adj_grid(const Grid<T> &g, dim3 &blk) {
  blk = dim3(64, 4, 1);
  return dim3((g.M[0] + 1 + 63) / 64, (g.M[1] + 1 + 3) / 4, g.dim == 3 ? g.M[2] + 1 : 1);
}

template <typename T>
void launch_adj_seed_energy(const Grid<T> &g, const Fields<T> &F, const AdjFields<T> &L, hipStream_t s) {
  dim3 blk, grd = adj_grid(g, blk);
  if (g.dim == 2) hipLaunchKernelGGL((k_adj_seed_energy<T, 2>), grd, blk, 0, s, g, F, L);
  else hipLaunchKernelGGL((k_adj_seed_energy<T, 3>), grd, blk, 0, s, g, F, L);
}

// transpose of one B half step whose input was Fb (B before, E used by the curl)
template <typename T>
void launch_adj_B_half(const Grid<T> &g, const AdjFields<T> &L, const Fields<T> &Fb, double *Gacc, hipStream_t s) {
  dim3 blk, grd = adj_grid(g, blk);
  if (g.dim == 2) {
    hipLaunchKernelGGL((k_adj_B_curl<T, 2>), grd, blk, 0, s, g, L);
    hipLaunchKernelGGL((k_adj_B_self<T, 2>), grd, blk, 0, s, g, L, Fb, Gacc);
  } else {
    hipLaunchKernelGGL((k_adj_B_curl<T, 3>), grd, blk, 0, s, g, L);
    hipLaunchKernelGGL((k_adj_B_self<T, 3>), grd, blk, 0, s, g, L, Fb, Gacc);
  }
}

// transpose of the E step whose input was Fe (E before, B^{n+1/2} used by the curl), J raw
// (LJ: null, or the three arrays that receive the adjoint of the step's current)
template <typename T>
void launch_adj_E(const Grid<T> &g, const AdjFields<T> &L, const Fields<T> &Fe, T *const J[3], int alpha_mode,
                  double *Gacc, T *const *LJ, hipStream_t s) {
  dim3 blk, grd = adj_grid(g, blk);
  T *l0 = LJ ? LJ[0] : nullptr, *l1 = LJ ? LJ[1] : nullptr, *l2 = LJ ? LJ[2] : nullptr;
  if (g.dim == 2) {
    hipLaunchKernelGGL((k_adj_E_curl<T, 2>), grd, blk, 0, s, g, L);
    hipLaunchKernelGGL((k_adj_E_self<T, 2>), grd, blk, 0, s, g, L, Fe, J[0], J[1], J[2], alpha_mode, Gacc, l0, l1, l2);
  } else {
    hipLaunchKernelGGL((k_adj_E_curl<T, 3>), grd, blk, 0, s, g, L);
    hipLaunchKernelGGL((k_adj_E_self<T, 3>), grd, blk, 0, s, g, L, Fe, J[0], J[1], J[2], alpha_mode, Gacc, l0, l1, l2);
  }
}

template void launch_adj_seed_energy<float>(const Grid<float> &, const Fields<float> &, const AdjFields<float> &, hipStream_t);
template void launch_adj_seed_energy<double>(const Grid<double> &, const Fields<double> &, const AdjFields<double> &, hipStream_t);
template void launch_adj_B_half<float>(const Grid<float> &, const AdjFields<float> &, const Fields<float> &, double *, hipStream_t);
template void launch_adj_B_half<double>(const Grid<double> &, const AdjFields<double> &, const Fields<double> &, double *, hipStream_t);
template void launch_adj_E<float>(const Grid<float> &, const AdjFields<float> &, const Fields<float> &, float *const[3], int,
                                  double *, float *const *, hipStream_t);
template void launch_adj_E<double>(const Grid<double> &, const AdjFields<double> &, const Fields<double> &, double *const[3],
                                   int, double *, double *const *, hipStream_t);

}  // namespace pmlpic
