// Per-sample device functions of update_yee_pml and damp_pml_current, shared by the
// single-run kernels (fields.hip) and the batched kernels (batch.hip).
//
// The split-field Yee/PML update with the damped current source (Sec. II.A, Eqs.
// MaxwellE / MaxwellB / MaxwellSum; Yee centring of Sec. II.B).  Each component keeps
// its total F_a everywhere and, where it is split (sigma_b + sigma_c > 0 at the
// sample), the part F_ab (b = a+1) in a second array; the other part is F_a - F_ab.
// In 2D the parts driven by z derivatives never change, so E_x, E_y, B_x, B_y are
// stored unsplit with the one in-plane rate.  dF/dt = -sigma F + rhs advances over tau
// as F <- e F + g rhs, e = exp(-sigma tau), g = (1 - e)/sigma (g = tau where sigma = 0).
#pragma once
#include "common.h"

namespace pmlpic {

template <typename T, int DIM>
__device__ __forceinline__ long stride_of(const Grid<T> &g, int axis) {
  return axis == 0 ? 1L : (axis == 1 ? g.sy : g.sz);
}

// The rest of the B_A half step at sample B_A(i,j,k) once its two differences are known
// (part b: -Db, the difference along b = A+1 of E_c; part c: +Dc, along c = A+2 of E_b);
// returns at samples outside B_A's extent.  FMA chains on the raw differences so that each
// part takes three roundings per update.
template <typename T, int DIM, int A>
__device__ __forceinline__ void update_B_apply(const Grid<T> &g, const Fields<T> &F, const int (&id)[3], long q,
                                               T Db, T Dc) {
  constexpr int Bx = (A + 1) % 3, Cx = (A + 2) % 3;
  // extent: along A up to M_A (node), across up to M-1 (centre)
  if (A < DIM && id[A] > g.M[A]) return;
  if (Bx < DIM && id[Bx] > g.M[Bx] - 1) return;
  if (Cx < DIM && id[Cx] > g.M[Cx] - 1) return;
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
  if (DIM == 3 && g.cmask && ((gptr(g.cmask)[q] >> (3 + A)) & 1)) {   // inside a conductor
    F.B[A][q] = T(0);
    F.Ba[A][q] = T(0);
  }
}

// B_A half step at node (i,j,k) -> sample B_A(i,j,k) with the Yee differences (the
// Cole-Karkkainen form is k_update_B_ck in fields.hip).
template <typename T, int DIM, int A>
__device__ __forceinline__ void update_B_comp(const Grid<T> &g, const Fields<T> &F, const int (&id)[3],
                                              long q) {
  constexpr int Bx = (A + 1) % 3, Cx = (A + 2) % 3;
  if (A < DIM && id[A] > g.M[A]) return;
  if (Bx < DIM && id[Bx] > g.M[Bx] - 1) return;
  if (Cx < DIM && id[Cx] > g.M[Cx] - 1) return;
  T Db = T(0), Dc = T(0);
  if (Bx < DIM) Db = F.E[Cx][q + stride_of<T, DIM>(g, Bx)] - F.E[Cx][q];
  if (Cx < DIM) Dc = F.E[Bx][q + stride_of<T, DIM>(g, Cx)] - F.E[Bx][q];
  update_B_apply<T, DIM, A>(g, F, id, q, Db, Dc);
}

// alpha at J_A's sample (i,j,k): product of per-axis factors (centre along A)
template <typename T, int DIM, int A>
__device__ __forceinline__ T alpha_at(const Grid<T> &g, const int (&id)[3]) {
  T a = T(1);
#pragma unroll
  for (int d = 0; d < DIM; ++d) a *= g.tb(d, d == A ? T_A_C : T_A_N, id[d]);
  return a;
}

// The rest of the E_A step at sample E_A(i,j,k) once its two differences are known (part
// b: +Db, the difference along b = A+1 of B_c; part c: -Dc, along c = A+2 of B_b), with the
// source -alpha J; returns at samples outside E_A's extent and on the PEC walls.
template <typename T, int DIM, int A>
__device__ __forceinline__ void update_E_apply(const Grid<T> &g, const Fields<T> &F, const int (&id)[3], long q,
                                               T Db, T Dc, bool fuse_alpha, bool consume) {
  constexpr int Bx = (A + 1) % 3, Cx = (A + 2) % 3;
  if (A < DIM && id[A] > g.M[A] - 1) return;
  if (Bx < DIM && (id[Bx] < 1 || id[Bx] > g.M[Bx] - 1)) return;   // PEC: tangential E = 0
  if (Cx < DIM && (id[Cx] < 1 || id[Cx] > g.M[Cx] - 1)) return;
  // source -alpha J split by the damping rates
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
  if (DIM == 3 && g.cmask && ((gptr(g.cmask)[q] >> A) & 1)) {   // inside a conductor
    F.E[A][q] = T(0);
    F.Ea[A][q] = T(0);
  }
}

template <typename T, int DIM, int A>
__device__ __forceinline__ void update_E_comp(const Grid<T> &g, const Fields<T> &F, const int (&id)[3],
                                              long q, bool fuse_alpha, bool consume) {
  constexpr int Bx = (A + 1) % 3, Cx = (A + 2) % 3;
  if (A < DIM && id[A] > g.M[A] - 1) return;
  if (Bx < DIM && (id[Bx] < 1 || id[Bx] > g.M[Bx] - 1)) return;
  if (Cx < DIM && (id[Cx] < 1 || id[Cx] > g.M[Cx] - 1)) return;
  T Db = T(0), Dc = T(0);
  if (Bx < DIM) Db = F.B[Cx][q] - F.B[Cx][q - stride_of<T, DIM>(g, Bx)];
  if (Cx < DIM) Dc = F.B[Bx][q] - F.B[Bx][q - stride_of<T, DIM>(g, Cx)];
  update_E_apply<T, DIM, A>(g, F, id, q, Db, Dc, fuse_alpha, consume);
}

}  // namespace pmlpic
