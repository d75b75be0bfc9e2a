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
#include "common.h"

namespace pmlpic {

template <typename T, int DIM>
__device__ __forceinline__ long stride_of(const Grid<T> &g, int axis) {
  return axis == 0 ? 1L : (axis == 1 ? g.sy : g.sz);
}

// B_A half step at node (i,j,k) -> sample B_A(i,j,k).  Written as FMA chains on the
// raw neighbour differences so that each part takes three roundings per update.
template <typename T, int DIM, int A>
__device__ __forceinline__ void update_B_comp(const Grid<T> &g, const Fields<T> &F, const int (&id)[3],
                                              long q) {
  constexpr int Bx = (A + 1) % 3, Cx = (A + 2) % 3;
  // extent: along A up to M_A (node), across up to M-1 (centre)
  if (A < DIM && id[A] > g.M[A]) return;
  if (Bx < DIM && id[Bx] > g.M[Bx] - 1) return;
  if (Cx < DIM && id[Cx] > g.M[Cx] - 1) return;
  // part b: -d_b E_c ; part c: +d_c E_b
  T Db = T(0), Dc = T(0);
  if (Bx < DIM) Db = F.E[Cx][q + stride_of<T, DIM>(g, Bx)] - F.E[Cx][q];
  if (Cx < DIM) Dc = F.E[Bx][q + stride_of<T, DIM>(g, Cx)] - F.E[Bx][q];
  if constexpr (DIM == 2 && (Bx == 2 || Cx == 2)) {
    constexpr int P = (Bx == 2) ? Cx : Bx;   // the in-plane derivative (and damping) axis
    const T e = g.tb(P, T_EH_C, id[P]), gk = g.tb(P, T_GHK_C, id[P]);
    if constexpr (P == Bx) F.B[A][q] = fma(-gk, Db, e * F.B[A][q]);
    else F.B[A][q] = fma(gk, Dc, e * F.B[A][q]);
  } else {
    const T sb = g.tb(Bx, T_SIG_C, id[Bx]), sc = g.tb(Cx, T_SIG_C, id[Cx]);
    const T gkb = g.tb(Bx, T_GHK_C, id[Bx]), gkc = g.tb(Cx, T_GHK_C, id[Cx]);
    if (sb + sc > T(0)) {
      T p1 = F.Ba[A][q];
      T p2 = F.B[A][q] - p1;
      p1 = fma(-gkb, Db, g.tb(Bx, T_EH_C, id[Bx]) * p1);
      p2 = fma(gkc, Dc, g.tb(Cx, T_EH_C, id[Cx]) * p2);
      F.B[A][q] = p1 + p2;
      F.Ba[A][q] = p1;
    } else {
      F.B[A][q] = fma(-gkb, Db, fma(gkc, Dc, F.B[A][q]));
    }
  }
}

// alpha at J_A's sample (i,j,k): product of per-axis factors (centre along A)
template <typename T, int DIM, int A>
__device__ __forceinline__ T alpha_at(const Grid<T> &g, const int (&id)[3]) {
  T a = T(1);
#pragma unroll
  for (int d = 0; d < DIM; ++d) a *= g.tb(d, d == A ? T_A_C : T_A_N, id[d]);
  return a;
}

template <typename T, int DIM, int A>
__device__ __forceinline__ void update_E_comp(const Grid<T> &g, const Fields<T> &F, const int (&id)[3],
                                              long q, bool fuse_alpha, bool consume) {
  constexpr int Bx = (A + 1) % 3, Cx = (A + 2) % 3;
  if (A < DIM && id[A] > g.M[A] - 1) return;
  if (Bx < DIM && (id[Bx] < 1 || id[Bx] > g.M[Bx] - 1)) return;   // PEC: tangential E = 0
  if (Cx < DIM && (id[Cx] < 1 || id[Cx] > g.M[Cx] - 1)) return;
  // part b: +d_b B_c ; part c: -d_c B_b ; source -alpha J split by the damping rates
  T Db = T(0), Dc = T(0);
  if (Bx < DIM) Db = F.B[Cx][q] - F.B[Cx][q - stride_of<T, DIM>(g, Bx)];
  if (Cx < DIM) Dc = F.B[Bx][q] - F.B[Bx][q - stride_of<T, DIM>(g, Cx)];
  T j = F.J[A][q];
  if (consume && j != T(0)) F.J[A][q] = T(0);   // leaves J zero for the next deposit
  if (fuse_alpha) j *= alpha_at<T, DIM, A>(g, id);
  if constexpr (DIM == 2 && (Bx == 2 || Cx == 2)) {
    constexpr int P = (Bx == 2) ? Cx : Bx;
    const T e = g.tb(P, T_E_N, id[P]), gg = g.tb(P, T_G_N, id[P]), gk = g.tb(P, T_GK_N, id[P]);
    const T base = fma(-gg, j, e * F.E[A][q]);
    if constexpr (P == Bx) F.E[A][q] = fma(gk, Db, base);
    else F.E[A][q] = fma(-gk, Dc, base);
  } else {
    const T sb = g.tb(Bx, T_SIG_N, id[Bx]), sc = g.tb(Cx, T_SIG_N, id[Cx]);
    const T gkb = g.tb(Bx, T_GK_N, id[Bx]), gkc = g.tb(Cx, T_GK_N, id[Cx]);
    if (sb + sc > T(0)) {
      const T inv = T(1) / (sb + sc);
      T p1 = F.Ea[A][q];
      T p2 = F.E[A][q] - p1;
      p1 = fma(gkb, Db, fma(-g.tb(Bx, T_G_N, id[Bx]) * (sb * inv), j, g.tb(Bx, T_E_N, id[Bx]) * p1));
      p2 = fma(-gkc, Dc, fma(-g.tb(Cx, T_G_N, id[Cx]) * (sc * inv), j, g.tb(Cx, T_E_N, id[Cx]) * p2));
      F.E[A][q] = p1 + p2;
      F.Ea[A][q] = p1;
    } else {
      F.E[A][q] = fma(gkb, Db, fma(-gkc, Dc, fma(-g.dt, j, F.E[A][q])));
    }
  }
}

template <typename T, int DIM>
__global__ void __launch_bounds__(256) k_update_B(Grid<T> g, Fields<T> F) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
  const int k = (DIM == 3) ? (int)blockIdx.z : 0;
  if (i > g.M[0] || j > g.M[1]) return;
  const int id[3] = {i, j, k};
  const long q = g.at(i, j, k);
  update_B_comp<T, DIM, 0>(g, F, id, q);
  update_B_comp<T, DIM, 1>(g, F, id, q);
  update_B_comp<T, DIM, 2>(g, F, id, q);
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

// B is only ever advanced by half steps (B^n -> B^{n+1/2} -> B^{n+1})
template <typename T>
void launch_update_B(const Grid<T> &g, const Fields<T> &F, bool /*half*/, hipStream_t s) {
  dim3 blk, grd = node_grid(g, blk);
  if (g.dim == 2) hipLaunchKernelGGL((k_update_B<T, 2>), grd, blk, 0, s, g, F);
  else hipLaunchKernelGGL((k_update_B<T, 3>), grd, blk, 0, s, g, F);
}

template <typename T>
void launch_update_E(const Grid<T> &g, const Fields<T> &F, bool fuse_alpha, int alpha_mode, bool consume,
                     hipStream_t s) {
  dim3 blk, grd = node_grid(g, blk);
  const bool fa = fuse_alpha && alpha_mode != 1;
  if (g.dim == 2) hipLaunchKernelGGL((k_update_E<T, 2>), grd, blk, 0, s, g, F, fa, consume);
  else hipLaunchKernelGGL((k_update_E<T, 3>), grd, blk, 0, s, g, F, fa, consume);
}

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
