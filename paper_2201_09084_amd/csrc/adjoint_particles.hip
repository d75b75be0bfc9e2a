// Reverse mode of gather_push and deposit_current for one step (pushed runs).
//
// Forward, per particle (state at the start of step n: cell i0, offset f0 in cell units,
// momentum u0 = u^{n-1/2}, weight w):
//   EB = gather(E^n, B^n at x0)              B-spline of the run's order, Yee-staggered
//   u1 = Boris(u0, EB)                       u^{n+1/2}
//   x1 = x0 + dt u1 / gamma(u1)              per axis, in cell units dt/dx u1/gamma
//   J += Esirkepov(x0 -> x1, q w)            (2D: J_z from v_z = u1_z / gamma)
// The step's field update reads J only through E' = ... - g alpha J, so the adjoint of J
// at each node (lambda_J, written by the transposed E update) is all the deposit's
// reverse needs.  Each thread reverses one particle: it recomputes the forward values
// from the stored start-of-step state, then
//   * the deposit's reverse is a gather of lambda_J over the move's window (no atomics),
//     giving dU/dx0 and dU/dx1 through the derivatives of the shape weights;
//   * the drift's reverse adds dU/dx1 to dU/dx0 and (d v / d u1)^T dt/dx dU/dx1 to dU/du1;
//   * the Boris rotation's reverse gives dU/du0 and dU/dEB;
//   * the gather's reverse scatters dU/dEB times the shape weights into the adjoint of
//     the total fields (atomics: several particles share nodes) and adds the
//     field-gradient term to dU/dx0.
// Particle adjoints are kept by particle id (the sort permutes the slots between steps).
#include "common.h"

namespace pmlpic {

// B-spline weights of order ORDER and their derivatives with respect to the offset f
// (same node placement as shape_weights: the return value is the first node's offset)
template <int ORDER, typename T>
__device__ __forceinline__ int shape_wd(T f, T (&w)[ORDER + 1], T (&dw)[ORDER + 1]) {
  if constexpr (ORDER == 1) {
    w[0] = T(1) - f; w[1] = f;
    dw[0] = T(-1); dw[1] = T(1);
    return 0;
  } else if constexpr (ORDER == 2) {
    const int up = f >= T(0.5);
    const T d = f - T(up);
    const T a = T(0.5) - d, b = T(0.5) + d;
    w[0] = T(0.5) * a * a; w[1] = T(0.75) - d * d; w[2] = T(0.5) * b * b;
    dw[0] = -a; dw[1] = T(-2) * d; dw[2] = b;
    return up - 1;
  } else {
    const T g = T(1) - f;
    const T f2 = f * f, g2 = g * g;
    w[0] = g2 * g * T(1.0 / 6.0);
    w[1] = (T(4) - T(6) * f2 + T(3) * f2 * f) * T(1.0 / 6.0);
    w[2] = (T(4) - T(6) * g2 + T(3) * g2 * g) * T(1.0 / 6.0);
    w[3] = f2 * f * T(1.0 / 6.0);
    dw[0] = T(-0.5) * g2;
    dw[1] = T(-2) * f + T(1.5) * f2;
    dw[2] = T(2) * g - T(1.5) * g2;
    dw[3] = T(0.5) * f2;
    return -1;
  }
}
// at the half-integer samples (index s stands for s + 1/2); the shifted offset moves
// with f, so the derivatives are those of shape_wd
template <int ORDER, typename T>
__device__ __forceinline__ int shape_wd_stag(int i, T f, T (&w)[ORDER + 1], T (&dw)[ORDER + 1]) {
  int ii;
  T ff;
  if (f >= T(0.5)) { ii = i; ff = f - T(0.5); }
  else { ii = i - 1; ff = f + T(0.5); if (ff >= T(1)) { ff = T(0); ii = i; } }
  return ii + shape_wd<ORDER>(ff, w, dw);
}

// both shapes of a move on the (ORDER+2)-node window of the forward deposit, with their
// derivatives; returns the window's first node
template <int ORDER, typename T>
__device__ __forceinline__ int window_wd(int i0, T f0, int i1, T f1, T (&S0)[ORDER + 2], T (&S1)[ORDER + 2],
                                         T (&D0)[ORDER + 2], T (&D1)[ORDER + 2]) {
  T w0[ORDER + 1], w1[ORDER + 1], d0[ORDER + 1], d1[ORDER + 1];
  const int s0 = i0 + shape_wd<ORDER>(f0, w0, d0);
  const int s1 = i1 + shape_wd<ORDER>(f1, w1, d1);
  const int st = s0 < s1 ? s0 : s1;
  const int o0 = s0 - st, o1 = s1 - st;   // 0 or 1
#pragma unroll
  for (int k = 0; k < ORDER + 2; ++k) {
    const int k0 = k - o0, k1 = k - o1;
    S0[k] = (k0 >= 0 && k0 <= ORDER) ? w0[k0 >= 0 && k0 <= ORDER ? k0 : 0] : T(0);
    D0[k] = (k0 >= 0 && k0 <= ORDER) ? d0[k0 >= 0 && k0 <= ORDER ? k0 : 0] : T(0);
    S1[k] = (k1 >= 0 && k1 <= ORDER) ? w1[k1 >= 0 && k1 <= ORDER ? k1 : 0] : T(0);
    D1[k] = (k1 >= 0 && k1 <= ORDER) ? d1[k1 >= 0 && k1 <= ORDER ? k1 : 0] : T(0);
  }
  return st;
}

// Reverse of the Esirkepov deposit of charge qw along (i0,f0) -> (i1,f1): adds
// dU/df0, dU/df1 (per axis) and, in 2D, dU/dvz, given lambda_J at the window's nodes.
template <typename T, int DIM, int ORDER>
__device__ __forceinline__ void deposit_reverse(const Grid<T> &g, const T *const (&LJ)[3], const int (&i0)[3],
                                                const T (&f0)[3], const int (&i1)[3], const T (&f1)[3], T vz,
                                                T qw, T (&gf0)[3], T (&gf1)[3], T &gvz) {
  constexpr int W = ORDER + 2;
  T S0[3][W], S1[3][W], D0[3][W], D1[3][W];
  T g0[3][W], g1[3][W];   // dU/dS0, dU/dS1
  int ws[3] = {0, 0, 0};
#pragma unroll
  for (int d = 0; d < 3; ++d)
#pragma unroll
    for (int k = 0; k < W; ++k) { g0[d][k] = T(0); g1[d][k] = T(0); }
#pragma unroll
  for (int d = 0; d < DIM; ++d) ws[d] = window_wd<ORDER>(i0[d], f0[d], i1[d], f1[d], S0[d], S1[d], D0[d], D1[d]);
  const long q0 = g.at(ws[0], ws[1], ws[2]);
  if constexpr (DIM == 2) {
    const T cx = qw * g.jcoef[0], cy = qw * g.jcoef[1];
    const T kz = qw * g.inv_dx[0] * g.inv_dx[1];
    // J_x[a][b] = -cx/2 R_a (S0y_b + S1y_b), R_a = sum_{a' <= a} (S1x - S0x)_{a'}
#pragma unroll
    for (int b = 0; b < W; ++b) {
      const T sy = S0[1][b] + S1[1][b];
      T R = T(0), gsy = T(0), lam[W - 1];
#pragma unroll
      for (int a = 0; a < W - 1; ++a) {
        lam[a] = LJ[0][q0 + a + b * g.sy];
        R += S1[0][a] - S0[0][a];
        gsy -= cx * T(0.5) * R * lam[a];
      }
      T suf = T(0);
#pragma unroll
      for (int a = W - 2; a >= 0; --a) {
        suf -= cx * T(0.5) * sy * lam[a];
        g1[0][a] += suf;
        g0[0][a] -= suf;
      }
      g0[1][b] += gsy;
      g1[1][b] += gsy;
    }
#pragma unroll
    for (int a = 0; a < W; ++a) {
      const T sx = S0[0][a] + S1[0][a];
      T R = T(0), gsx = T(0), lam[W - 1];
#pragma unroll
      for (int b = 0; b < W - 1; ++b) {
        lam[b] = LJ[1][q0 + a + b * g.sy];
        R += S1[1][b] - S0[1][b];
        gsx -= cy * T(0.5) * R * lam[b];
      }
      T suf = T(0);
#pragma unroll
      for (int b = W - 2; b >= 0; --b) {
        suf -= cy * T(0.5) * sx * lam[b];
        g1[1][b] += suf;
        g0[1][b] -= suf;
      }
      g0[0][a] += gsx;
      g1[0][a] += gsx;
    }
    // J_z[a][b] = kz vz ((S0x S0y + S1x S1y)/3 + (S1x S0y + S0x S1y)/6)
    T gcz = T(0);
    const T cz = kz * vz;
#pragma unroll
    for (int b = 0; b < W; ++b)
#pragma unroll
      for (int a = 0; a < W; ++a) {
        const T lam = LJ[2][q0 + a + b * g.sy];
        const T wz = (S0[0][a] * S0[1][b] + S1[0][a] * S1[1][b]) * T(1.0 / 3.0) +
                     (S1[0][a] * S0[1][b] + S0[0][a] * S1[1][b]) * T(1.0 / 6.0);
        gcz += lam * wz;
        const T gw = lam * cz;
        g0[0][a] += gw * (S0[1][b] * T(1.0 / 3.0) + S1[1][b] * T(1.0 / 6.0));
        g1[0][a] += gw * (S1[1][b] * T(1.0 / 3.0) + S0[1][b] * T(1.0 / 6.0));
        g0[1][b] += gw * (S0[0][a] * T(1.0 / 3.0) + S1[0][a] * T(1.0 / 6.0));
        g1[1][b] += gw * (S1[0][a] * T(1.0 / 3.0) + S0[0][a] * T(1.0 / 6.0));
      }
    gvz += gcz * kz;
  } else {
    // J_A[a][b][c] = -coef R_a avg(b, c) over the window, R_a = running sum along A
#pragma unroll
    for (int A = 0; A < 3; ++A) {
      const int Bx = (A + 1) % 3, Cx = (A + 2) % 3;
      const T coef = qw * g.jcoef[A];
      const long st[3] = {1, g.sy, g.sz};
#pragma unroll
      for (int c = 0; c < W; ++c)
#pragma unroll
        for (int b = 0; b < W; ++b) {
          const T avg = (S0[Bx][b] * S0[Cx][c] + S1[Bx][b] * S1[Cx][c]) * T(1.0 / 3.0) +
                        (S1[Bx][b] * S0[Cx][c] + S0[Bx][b] * S1[Cx][c]) * T(1.0 / 6.0);
          const long qb = q0 + b * st[Bx] + c * st[Cx];
          T R = T(0), gavg = T(0), lam[W - 1];
#pragma unroll
          for (int a = 0; a < W - 1; ++a) {
            lam[a] = LJ[A][qb + a * st[A]];
            R += S1[A][a] - S0[A][a];
            gavg -= coef * R * lam[a];
          }
          T suf = T(0);
#pragma unroll
          for (int a = W - 2; a >= 0; --a) {
            suf -= coef * avg * lam[a];
            g1[A][a] += suf;
            g0[A][a] -= suf;
          }
          g0[Bx][b] += gavg * (S0[Cx][c] * T(1.0 / 3.0) + S1[Cx][c] * T(1.0 / 6.0));
          g1[Bx][b] += gavg * (S1[Cx][c] * T(1.0 / 3.0) + S0[Cx][c] * T(1.0 / 6.0));
          g0[Cx][c] += gavg * (S0[Bx][b] * T(1.0 / 3.0) + S1[Bx][b] * T(1.0 / 6.0));
          g1[Cx][c] += gavg * (S1[Bx][b] * T(1.0 / 3.0) + S0[Bx][b] * T(1.0 / 6.0));
        }
    }
  }
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    T a0 = T(0), a1 = T(0);
#pragma unroll
    for (int k = 0; k < W; ++k) { a0 += g0[d][k] * D0[d][k]; a1 += g1[d][k] * D1[d][k]; }
    gf0[d] += a0;
    gf1[d] += a1;
  }
}

// Shape weights (and derivatives) of one staggered component at x0, per axis
template <typename T, int ORDER>
struct CompShape {
  T w[3][ORDER + 1], dw[3][ORDER + 1];
  int s[3];
};
template <typename T, int DIM, int ORDER>
__device__ __forceinline__ void comp_shape(int mask, const int (&id)[3], const T (&f)[3], CompShape<T, ORDER> &S) {
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    if (d >= DIM) {
#pragma unroll
      for (int k = 0; k <= ORDER; ++k) { S.w[d][k] = k == 0 ? T(1) : T(0); S.dw[d][k] = T(0); }
      S.s[d] = 0;
    } else if (mask & (1 << d)) {
      S.s[d] = shape_wd_stag<ORDER>(id[d], f[d], S.w[d], S.dw[d]);
    } else {
      S.s[d] = id[d] + shape_wd<ORDER>(f[d], S.w[d], S.dw[d]);
    }
  }
}

// stagger bits of E_x, E_y, E_z, B_x, B_y, B_z (bit d: half-integer along d)
__device__ __forceinline__ int comp_mask(int c) {
  return c == 0 ? 1 : c == 1 ? 2 : c == 2 ? 4 : c == 3 ? 6 : c == 4 ? 5 : 3;
}

// forward gather of the total field component `arr` at x0
template <typename T, int DIM, int ORDER>
__device__ __forceinline__ T gather_value(const Grid<T> &g, const T *arr, const CompShape<T, ORDER> &S) {
  constexpr int NZ = DIM == 3 ? ORDER + 1 : 1;
  T acc = T(0);
#pragma unroll
  for (int c = 0; c < NZ; ++c) {
    T pl = T(0);
#pragma unroll
    for (int b = 0; b <= ORDER; ++b) {
      T row = T(0);
      const long q = g.at(S.s[0], S.s[1] + b, S.s[2] + c);
#pragma unroll
      for (int a = 0; a <= ORDER; ++a) row += S.w[0][a] * arr[q + a];
      pl += S.w[1][b] * row;
    }
    acc += S.w[2][c] * pl;
  }
  return acc;
}

// reverse of the gather of one component: lam_out += lam * weights (atomics), and the
// field-gradient term lam * dEB/dx0 added to gf
template <typename T, int DIM, int ORDER>
__device__ __forceinline__ void gather_reverse(const Grid<T> &g, const T *arr, T *lam_out, T lam,
                                               const CompShape<T, ORDER> &S, T (&gf)[3]) {
  constexpr int NZ = DIM == 3 ? ORDER + 1 : 1;
  T gx = T(0), gy = T(0), gz = T(0);
#pragma unroll
  for (int c = 0; c < NZ; ++c) {
#pragma unroll
    for (int b = 0; b <= ORDER; ++b) {
      const long q = g.at(S.s[0], S.s[1] + b, S.s[2] + c);
#pragma unroll
      for (int a = 0; a <= ORDER; ++a) {
        const T v = arr[q + a];
        const T wyz = S.w[1][b] * S.w[2][c];
        gx += S.dw[0][a] * wyz * v;
        gy += S.w[0][a] * S.dw[1][b] * S.w[2][c] * v;
        if (DIM == 3) gz += S.w[0][a] * S.w[1][b] * S.dw[2][c] * v;
        const T wt = S.w[0][a] * wyz * lam;
        if (wt != T(0)) atomic_add(&lam_out[q + a], wt);
      }
    }
  }
  gf[0] += lam * gx;
  gf[1] += lam * gy;
  if (DIM == 3) gf[2] += lam * gz;
}

template <typename T>
__device__ __forceinline__ void cross(const T (&a)[3], const T (&b)[3], T (&o)[3]) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}

template <typename T, int DIM, int ORDER>
__global__ void __launch_bounds__(256) k_adj_particles(Grid<T> g, Fields<T> Fn, Parts<T> P, const int32_t *count,
                                                      int ns, int cap, AdjFields<T> L, const T *LJx, const T *LJy,
                                                      const T *LJz, PartAdj<T> A) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= ns || p >= *count) return;
  const uint32_t cell = P.cell[p];
  if (cell == DEAD) return;
  const int pid = P.id[p];
  if (pid < 0 || pid >= cap) return;   // ids are below the capacity (checked by the host)
  int i0[3];
  unpack_cell(DIM, cell, i0[0], i0[1], i0[2]);
  const T f0[3] = {P.f[0][p], P.f[1][p], DIM == 3 ? P.f[2][p] : T(0)};
  const T u0[3] = {P.u[0][p], P.u[1][p], P.u[2][p]};
  const T qw = g.charge * P.w[p];
  const T k = g.qdt_2m;

  // ---- forward recompute
  const T *arr[6] = {Fn.E[0], Fn.E[1], Fn.E[2], Fn.B[0], Fn.B[1], Fn.B[2]};
  T EB[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    CompShape<T, ORDER> S;
    comp_shape<T, DIM, ORDER>(comp_mask(c), i0, f0, S);
    EB[c] = gather_value<T, DIM, ORDER>(g, arr[c], S);
  }
  T m[3], tv[3], pv[3], av[3], u1[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) m[d] = u0[d] + k * EB[d];
  const T igm = T(1) / sqrt(T(1) + m[0] * m[0] + m[1] * m[1] + m[2] * m[2]);
#pragma unroll
  for (int d = 0; d < 3; ++d) tv[d] = k * EB[3 + d] * igm;
  const T sfac = T(2) / (T(1) + tv[0] * tv[0] + tv[1] * tv[1] + tv[2] * tv[2]);
  cross(m, tv, pv);
#pragma unroll
  for (int d = 0; d < 3; ++d) pv[d] += m[d];
  cross(pv, tv, av);
#pragma unroll
  for (int d = 0; d < 3; ++d) u1[d] = m[d] + sfac * av[d] + k * EB[d];
  const T ig1 = T(1) / sqrt(T(1) + u1[0] * u1[0] + u1[1] * u1[1] + u1[2] * u1[2]);
  int i1[3] = {i0[0], i0[1], i0[2]};
  T f1[3] = {f0[0], f0[1], f0[2]};
#pragma unroll
  for (int d = 0; d < DIM; ++d) {   // the forward move's re-basing of the offset
    T nf = f1[d] + (g.dt * g.inv_dx[d]) * (u1[d] * ig1);
    if (nf >= T(1)) { nf -= T(1); i1[d] += 1; }
    else if (nf < T(0)) {
      nf += T(1); i1[d] -= 1;
      if (nf >= T(1)) { nf = T(0); i1[d] += 1; }
    }
    f1[d] = nf;
  }

  // ---- reverse
  T lf1[3] = {T(0), T(0), T(0)}, lu1[3];
#pragma unroll
  for (int d = 0; d < DIM; ++d) lf1[d] = A.lf[d][pid];
#pragma unroll
  for (int d = 0; d < 3; ++d) lu1[d] = A.lu[d][pid];
  T gf0[3] = {T(0), T(0), T(0)}, gvz = T(0);
  const T *const LJ[3] = {LJx, LJy, LJz};
  deposit_reverse<T, DIM, ORDER>(g, LJ, i0, f0, i1, f1, u1[2] * ig1, qw, gf0, lf1, gvz);
  // drift: f1 = f0 + dt/dx u1/gamma1
  T lf0[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) lf0[d] = lf1[d] + gf0[d];
  T lv[3] = {T(0), T(0), gvz};   // dU/d(u1/gamma1)
#pragma unroll
  for (int d = 0; d < DIM; ++d) lv[d] += lf1[d] * g.dt * g.inv_dx[d];
  {
    const T uv = lv[0] * u1[0] + lv[1] * u1[1] + lv[2] * u1[2];
#pragma unroll
    for (int d = 0; d < 3; ++d) lu1[d] += ig1 * lv[d] - ig1 * ig1 * ig1 * u1[d] * uv;
  }
  // Boris: u1 = m + s (p x t) + kE, p = m + m x t, s = 2/(1+t.t), t = k B igm, m = u0 + kE
  T lE[3], lB[3], lm[3], lt[3], lp[3], tmp[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) { lm[d] = lu1[d]; lE[d] = k * lu1[d]; }
  const T ls = lu1[0] * av[0] + lu1[1] * av[1] + lu1[2] * av[2];
  T la[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) la[d] = sfac * lu1[d];
  cross(tv, la, lp);              // a = p x t
  cross(la, pv, lt);
  cross(tv, lp, tmp);             // p = m + m x t
#pragma unroll
  for (int d = 0; d < 3; ++d) lm[d] += lp[d] + tmp[d];
  cross(lp, m, tmp);
#pragma unroll
  for (int d = 0; d < 3; ++d) lt[d] += tmp[d] - ls * sfac * sfac * tv[d];   // ds/dt = -s^2 t
  const T lig = k * (EB[3] * lt[0] + EB[4] * lt[1] + EB[5] * lt[2]);
  {
    const T ig3 = igm * igm * igm;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      lB[d] = k * igm * lt[d];
      lm[d] -= lig * ig3 * m[d];
      lE[d] += k * lm[d];
    }
  }
  // gather: scatter into the adjoint of the total fields, field-gradient term into lf0
  const T lEB[6] = {lE[0], lE[1], lE[2], lB[0], lB[1], lB[2]};
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    if (lEB[c] == T(0)) continue;
    CompShape<T, ORDER> S;
    comp_shape<T, DIM, ORDER>(comp_mask(c), i0, f0, S);
    gather_reverse<T, DIM, ORDER>(g, arr[c], L.LT[c], lEB[c], S, lf0);
  }
#pragma unroll
  for (int d = 0; d < DIM; ++d) A.lf[d][pid] = lf0[d];
#pragma unroll
  for (int d = 0; d < 3; ++d) A.lu[d][pid] = lm[d];
}

template <typename T>
void launch_adj_particles(const Grid<T> &g, const Fields<T> &Fn, const Parts<T> &P, const int32_t *count, int ns,
                          int cap, const AdjFields<T> &L, T *const LJ[3], const PartAdj<T> &A, hipStream_t s) {
  if (ns <= 0) return;
  const dim3 blk(256), grd((ns + 255) / 256);
#define PMLPIC_ADJP(D, O) \
  hipLaunchKernelGGL((k_adj_particles<T, D, O>), grd, blk, 0, s, g, Fn, P, count, ns, cap, L, LJ[0], LJ[1], LJ[2], A)
  if (g.dim == 2) {
    if (g.order == 1) PMLPIC_ADJP(2, 1);
    else if (g.order == 2) PMLPIC_ADJP(2, 2);
    else PMLPIC_ADJP(2, 3);
  } else {
    if (g.order == 1) PMLPIC_ADJP(3, 1);
    else if (g.order == 2) PMLPIC_ADJP(3, 2);
    else PMLPIC_ADJP(3, 3);
  }
#undef PMLPIC_ADJP
}

template void launch_adj_particles<float>(const Grid<float> &, const Fields<float> &, const Parts<float> &,
                                          const int32_t *, int, int, const AdjFields<float> &, float *const[3],
                                          const PartAdj<float> &, hipStream_t);
template void launch_adj_particles<double>(const Grid<double> &, const Fields<double> &, const Parts<double> &,
                                           const int32_t *, int, int, const AdjFields<double> &, double *const[3],
                                           const PartAdj<double> &, hipStream_t);

}  // namespace pmlpic
