// Per-particle device functions of gather_push and deposit_current, shared by the
// single-run kernels (particles.hip) and the batched kernels (batch.hip).
//
// gather: the six total field components (sum of the split parts, Eq. MaxwellSum) are
// interpolated with the same-order B-spline at each component's staggered Yee sample;
// boris: relativistic Boris rotation of u = gamma v; move: x += dt u/gamma with the
// offset re-based into [0,1); deposit: Esirkepov's charge-conserving scheme (used in
// App. A) on the (order+2)-node window that covers both shapes of the move.
#pragma once
#include "common.h"

namespace pmlpic {

template <int ORDER, typename T>
struct Shape3 {
  T wn[3][ORDER + 1];
  T wc[3][ORDER + 1];
  int sn[3], sc[3];
};

template <typename T, int DIM, int ORDER>
__device__ __forceinline__ void shape_all(const int (&id)[3], const T (&f)[3], Shape3<ORDER, T> &S) {
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    S.sn[d] = id[d] + shape_weights<ORDER>(f[d], S.wn[d]);
    S.sc[d] = shape_weights_stag<ORDER>(id[d], f[d], S.wc[d]);
  }
}

// interpolate one component whose stagger bits are MASK (bit d: half-integer along d)
template <typename T, int DIM, int ORDER, int MASK>
__device__ __forceinline__ T gather_comp(const Grid<T> &g, const T *__restrict__ arr,
                                         const Shape3<ORDER, T> &S) {
  constexpr bool hx = MASK & 1, hy = MASK & 2, hz = MASK & 4;
  const int x0 = hx ? S.sc[0] : S.sn[0];
  const int y0 = hy ? S.sc[1] : S.sn[1];
  T acc = T(0);
  if constexpr (DIM == 2) {
    const long q0 = g.at(x0, y0, 0);
#pragma unroll
    for (int b = 0; b <= ORDER; ++b) {
      T row = T(0);
#pragma unroll
      for (int a = 0; a <= ORDER; ++a) row += (hx ? S.wc[0][a] : S.wn[0][a]) * arr[q0 + b * g.sy + a];
      acc += (hy ? S.wc[1][b] : S.wn[1][b]) * row;
    }
  } else {
    const int z0 = hz ? S.sc[2] : S.sn[2];
    const long q0 = g.at(x0, y0, z0);
#pragma unroll
    for (int c = 0; c <= ORDER; ++c) {
      T pl = T(0);
#pragma unroll
      for (int b = 0; b <= ORDER; ++b) {
        T row = T(0);
#pragma unroll
        for (int a = 0; a <= ORDER; ++a)
          row += (hx ? S.wc[0][a] : S.wn[0][a]) * arr[q0 + c * g.sz + b * g.sy + a];
        pl += (hy ? S.wc[1][b] : S.wn[1][b]) * row;
      }
      acc += (hz ? S.wc[2][c] : S.wn[2][c]) * pl;
    }
  }
  return acc;
}

// 2D: every stencil load is issued before the first product, with 32-bit offsets
// (left to itself the compiler interleaved loads and waits in the register-heavy
// fused kernel: one memory round trip per stencil row)
template <typename T, int ORDER, int MASK>
__device__ __forceinline__ void load_stencil_2d(const Grid<T> &g, const T *arr, const Shape3<ORDER, T> &S,
                                                T (&v)[ORDER + 1][ORDER + 1]) {
  constexpr bool hx = MASK & 1, hy = MASK & 2;
  const int sy = (int)g.sy;
  const int q0 = (int)g.base + (hx ? S.sc[0] : S.sn[0]) + (hy ? S.sc[1] : S.sn[1]) * sy;
  const auto *a = gptr(arr) + q0;
#pragma unroll
  for (int b = 0; b <= ORDER; ++b)
#pragma unroll
    for (int c = 0; c <= ORDER; ++c) v[b][c] = a[b * sy + c];
}
template <typename T, int ORDER, int MASK>
__device__ __forceinline__ T interp_2d(const Shape3<ORDER, T> &S, const T (&v)[ORDER + 1][ORDER + 1]) {
  constexpr bool hx = MASK & 1, hy = MASK & 2;
  T acc = T(0);
#pragma unroll
  for (int b = 0; b <= ORDER; ++b) {
    T row = T(0);
#pragma unroll
    for (int c = 0; c <= ORDER; ++c) row += (hx ? S.wc[0][c] : S.wn[0][c]) * v[b][c];
    acc += (hy ? S.wc[1][b] : S.wn[1][b]) * row;
  }
  return acc;
}

template <typename T, int DIM, int ORDER>
__device__ __forceinline__ void gather(const Grid<T> &g, const Fields<T> &F, const int (&id)[3],
                                       const T (&f)[3], T (&EB)[6]) {
  Shape3<ORDER, T> S;
  shape_all<T, DIM, ORDER>(id, f, S);
  if constexpr (DIM == 2) {   // E, then B: two memory round trips
    T v[3][ORDER + 1][ORDER + 1];
    load_stencil_2d<T, ORDER, 1>(g, F.E[0], S, v[0]);
    load_stencil_2d<T, ORDER, 2>(g, F.E[1], S, v[1]);
    load_stencil_2d<T, ORDER, 0>(g, F.E[2], S, v[2]);
    __builtin_amdgcn_sched_barrier(0);
    EB[0] = interp_2d<T, ORDER, 1>(S, v[0]);
    EB[1] = interp_2d<T, ORDER, 2>(S, v[1]);
    EB[2] = interp_2d<T, ORDER, 0>(S, v[2]);
    load_stencil_2d<T, ORDER, 2>(g, F.B[0], S, v[0]);
    load_stencil_2d<T, ORDER, 1>(g, F.B[1], S, v[1]);
    load_stencil_2d<T, ORDER, 3>(g, F.B[2], S, v[2]);
    __builtin_amdgcn_sched_barrier(0);
    EB[3] = interp_2d<T, ORDER, 2>(S, v[0]);
    EB[4] = interp_2d<T, ORDER, 1>(S, v[1]);
    EB[5] = interp_2d<T, ORDER, 3>(S, v[2]);
    return;
  }
  EB[0] = gather_comp<T, DIM, ORDER, 1>(g, F.E[0], S);
  EB[1] = gather_comp<T, DIM, ORDER, 2>(g, F.E[1], S);
  EB[2] = gather_comp<T, DIM, ORDER, 4>(g, F.E[2], S);
  EB[3] = gather_comp<T, DIM, ORDER, 6>(g, F.B[0], S);
  EB[4] = gather_comp<T, DIM, ORDER, 5>(g, F.B[1], S);
  EB[5] = gather_comp<T, DIM, ORDER, 3>(g, F.B[2], S);
}

// relativistic Boris rotation (Boris 1970)
template <typename T>
__device__ __forceinline__ void boris(T k, const T (&EB)[6], T (&u)[3]) {
  const T mx = u[0] + k * EB[0], my = u[1] + k * EB[1], mz = u[2] + k * EB[2];
  const T ig = T(1) / sqrt(T(1) + mx * mx + my * my + mz * mz);
  const T tx = k * EB[3] * ig, ty = k * EB[4] * ig, tz = k * EB[5] * ig;
  const T s = T(2) / (T(1) + tx * tx + ty * ty + tz * tz);
  const T px = mx + (my * tz - mz * ty);
  const T py = my + (mz * tx - mx * tz);
  const T pz = mz + (mx * ty - my * tx);
  u[0] = mx + s * (py * tz - pz * ty) + k * EB[0];
  u[1] = my + s * (pz * tx - px * tz) + k * EB[1];
  u[2] = mz + s * (px * ty - py * tx) + k * EB[2];
}

// x^{n+1} = x^n + dt u/gamma; returns true if the particle is still inside the PEC box
template <typename T, int DIM>
__device__ __forceinline__ bool move(const Grid<T> &g, int (&id)[3], T (&f)[3], const T (&u)[3], T &inv_gamma) {
  inv_gamma = T(1) / sqrt(T(1) + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
  bool inside = true;
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    const T disp = (g.dt * g.inv_dx[d]) * (u[d] * inv_gamma);
    T nf = f[d] + disp;
    if constexpr (sizeof(T) == 4) {
      // the same arithmetic with selects instead of branches (FP32: fewer scalar and exec-mask
      // instructions per particle; in FP64 the extra live values make the push kernel spill)
      const bool hi = nf >= T(1), lo = nf < T(0);
      const T up = nf - T(1), dn = nf + T(1);
      const bool fix = lo && dn >= T(1);   // a step just below 0 that rounds to 1 after the wrap
      nf = hi ? up : (lo ? (fix ? T(0) : dn) : nf);
      id[d] += hi ? 1 : ((lo && !fix) ? -1 : 0);
    } else {
      if (nf >= T(1)) { nf -= T(1); id[d] += 1; }
      else if (nf < T(0)) {
        nf += T(1); id[d] -= 1;
        if (nf >= T(1)) { nf = T(0); id[d] += 1; }
      }
    }
    f[d] = nf;
    inside = inside && id[d] >= 0 && id[d] < g.M[d];
  }
  return inside;
}

// Where deposited current goes: straight to the global J arrays (hardware float
// atomics at L2), or to a workgroup's LDS copy of a box of nodes that is flushed to
// global memory once at the end.
template <typename T>
struct GlobalSink {
  T *J[3];
  long q0, sy, sz;
  long nelem = 0;
  uint32_t *check = nullptr;
  __device__ __forceinline__ void origin(const Grid<T> &g, const int (&ws)[3]) {
    q0 = g.at(ws[0], ws[1], ws[2]);
    sy = g.sy;
    sz = g.sz;
    nelem = g.nelem;
    check = g.check;
  }
  __device__ __forceinline__ void add(int comp, int a, int b, int c, T v) {
    const long q = q0 + a + b * sy + c * sz;
#ifdef PMLPIC_CHECK
    if (q < 0 || q >= nelem) { check_failed(check, CHECK_GLOBAL_J); return; }
#endif
    atomic_add(&J[comp][q], v);
  }
};

// The LDS box is replicated: lane L adds into copy L mod R, so lanes of a wave that
// hit the same node (dense beams: whole waves share a cell) meet in R different words
// and banks (the copy stride is odd).  The flush sums the copies.  The box holds FP64
// sums whatever the run's precision: on gfx950 the LDS FP64 add runs about twenty
// times faster than the FP32 one, and the sums round once, at the flush.
template <typename T>
struct LdsSink {
  double *lds;
  int lo[3];
  int e0, e01, total;
  int q0;
  uint32_t *check = nullptr;
  __device__ __forceinline__ void origin(const Grid<T> &g, const int (&ws)[3]) {
    q0 = (ws[0] - lo[0]) + (ws[1] - lo[1]) * e0 + (ws[2] - lo[2]) * e01;
    check = g.check;
  }
  __device__ __forceinline__ void add(int comp, int a, int b, int c, T v) {
    const int q = q0 + a + b * e0 + c * e01;
#ifdef PMLPIC_CHECK
    if (q < 0 || q >= total) { check_failed(check, CHECK_LDS_BOX); return; }
#endif
    atomicAdd(&lds[comp * total + q], (double)v);
  }
};

// the (ORDER+2)-node window holding both shapes of a move, per axis: S0, S1 and start
template <typename T, int ORDER>
__device__ __forceinline__ int move_window(int i0, T f0, int i1, T f1, T (&S0)[ORDER + 2], T (&S1)[ORDER + 2]) {
  T w0[ORDER + 1], w1[ORDER + 1];
  const int s0 = i0 + shape_weights<ORDER>(f0, w0);
  const int s1 = i1 + shape_weights<ORDER>(f1, w1);
  const int st = s0 < s1 ? s0 : s1;
  const bool sh0 = s0 != st, sh1 = s1 != st;     // shape shifted one node up in the window
#pragma unroll
  for (int k = 0; k < ORDER + 2; ++k) {
    const T a0 = k <= ORDER ? w0[k <= ORDER ? k : 0] : T(0);
    const T b0 = k >= 1 ? w0[k >= 1 ? k - 1 : 0] : T(0);
    const T a1 = k <= ORDER ? w1[k <= ORDER ? k : 0] : T(0);
    const T b1 = k >= 1 ? w1[k >= 1 ? k - 1 : 0] : T(0);
    S0[k] = sh0 ? b0 : a0;
    S1[k] = sh1 ? b1 : a1;
  }
  return st;
}

// Esirkepov deposit of charge qw moving (i0,f0) -> (i1,f1) into `sink`; vz is used in
// 2D only (current along the invariant axis)
template <typename T, int DIM, int ORDER, class Sink>
__device__ __forceinline__ void deposit(const Grid<T> &g, Sink &sink, const int (&i0)[3], const T (&f0)[3],
                                        const int (&i1)[3], const T (&f1)[3], T vz, T qw) {
  constexpr int W = ORDER + 2;
  T S0[3][W], S1[3][W];
  int ws[3] = {0, 0, 0};
#pragma unroll
  for (int d = 0; d < DIM; ++d) ws[d] = move_window<T, ORDER>(i0[d], f0[d], i1[d], f1[d], S0[d], S1[d]);
  sink.origin(g, ws);
  if constexpr (DIM == 2) {
    const T cx = qw * g.jcoef[0];
    const T cy = qw * g.jcoef[1];
    const T cz = qw * vz * g.inv_dx[0] * g.inv_dx[1];
#pragma unroll
    for (int b = 0; b < W; ++b) {            // J_x: running sum along x
      const T sy = S0[1][b] + S1[1][b];
      T acc = T(0);
#pragma unroll
      for (int a = 0; a < W - 1; ++a) {
        acc -= cx * T(0.5) * (S1[0][a] - S0[0][a]) * sy;
        if (acc != T(0)) sink.add(0, a, b, 0, acc);
      }
    }
#pragma unroll
    for (int a = 0; a < W; ++a) {            // J_y: running sum along y
      const T sx = S0[0][a] + S1[0][a];
      T acc = T(0);
#pragma unroll
      for (int b = 0; b < W - 1; ++b) {
        acc -= cy * T(0.5) * (S1[1][b] - S0[1][b]) * sx;
        if (acc != T(0)) sink.add(1, a, b, 0, acc);
      }
    }
    if (cz != T(0)) {
#pragma unroll
      for (int b = 0; b < W; ++b)
#pragma unroll
        for (int a = 0; a < W; ++a) {
          const T wz = (S0[0][a] * S0[1][b] + S1[0][a] * S1[1][b]) * T(1.0 / 3.0) +
                       (S1[0][a] * S0[1][b] + S0[0][a] * S1[1][b]) * T(1.0 / 6.0);
          if (wz != T(0)) sink.add(2, a, b, 0, cz * wz);
        }
    }
  } else {
#pragma unroll
    for (int A = 0; A < 3; ++A) {
      const int Bx = (A + 1) % 3, Cx = (A + 2) % 3;
      const T coef = qw * g.jcoef[A];
#pragma unroll
      for (int c = 0; c < W; ++c)
#pragma unroll
        for (int b = 0; b < W; ++b) {
          const T avg = (S0[Bx][b] * S0[Cx][c] + S1[Bx][b] * S1[Cx][c]) * T(1.0 / 3.0) +
                        (S1[Bx][b] * S0[Cx][c] + S0[Bx][b] * S1[Cx][c]) * T(1.0 / 6.0);
          if (avg == T(0)) continue;
          T acc = T(0);
#pragma unroll
          for (int a = 0; a < W - 1; ++a) {
            acc -= coef * (S1[A][a] - S0[A][a]) * avg;
            if (acc != T(0)) {
              int ii[3];
              ii[A] = a; ii[Bx] = b; ii[Cx] = c;
              sink.add(A, ii[0], ii[1], ii[2], acc);
            }
          }
        }
    }
  }
}


// Per-particle weight damping (Sec. II.C, discussion of the velocity limitation): the
// weight is w exp(-Lambda), Lambda = int sigma/eps0 dt along the particle's path.
// For one layer face, with the signed depth s into the layer at the start and end of
// a straight move taking tau, a = max(s0, 0), b = max(s1, 0), the integral is
// tau (b - a) / (s1 - s0) times the divided difference (Phi(b) - Phi(a)) / (b - a) of
// the antiderivative of the polynomial profile, evaluated as sum_k c_k h_k with
// c_k = a_k / (k + 1), h_0 = 1, h_k = (b/L) h_{k-1} + (a/L)^k (no cancellation when b
// is close to a; it is sigma(a) when b = a).
template <typename T>
__device__ __forceinline__ T face_sigma_integral(const T *pc, T L, T s0, T s1, T tau) {
  if (!(s0 > T(0)) && !(s1 > T(0))) return T(0);
  const T a = s0 > T(0) ? s0 : T(0), b = s1 > T(0) ? s1 : T(0);
  const T frac = (s1 == s0) ? T(1) : (b - a) / (s1 - s0);
  const T ra = a / L, rb = b / L;
  T h = T(1), pa = T(1), dd = pc[0];
#pragma unroll
  for (int k = 1; k < 16; ++k) {
    pa *= ra;
    h = fma(rb, h, pa);
    dd = fma(pc[k], h, dd);
  }
  return tau * frac * dd;
}

// Lambda gained over the first half of the move (i0, f0) -> (i1, f1) and over the
// whole move (summed over the layers of every axis)
template <typename T, int DIM>
__device__ __forceinline__ void path_lambda(const Grid<T> &g, const int (&i0)[3], const T (&f0)[3],
                                            const int (&i1)[3], const T (&f1)[3], T &half, T &full) {
  half = T(0);
  full = T(0);
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    const T *pr = g.prof + d * PROF_N;
    const T h = pr[PROF_DX];
    const int lo = (int)pr[PROF_LO], hi = (int)pr[PROF_HI];
    // signed depths into the low and high layers (exact integer parts)
    const T l0 = ((T)(lo - i0[d]) - f0[d]) * h, l1 = ((T)(lo - i1[d]) - f1[d]) * h;
    const T u0 = ((T)(i0[d] - hi) + f0[d]) * h, u1 = ((T)(i1[d] - hi) + f1[d]) * h;
    const T lm = T(0.5) * (l0 + l1), um = T(0.5) * (u0 + u1);
    if (pr[PROF_LLO] > T(0)) {
      half += face_sigma_integral(pr + PROF_C, pr[PROF_LLO], l0, lm, T(0.5) * g.dt);
      full += face_sigma_integral(pr + PROF_C, pr[PROF_LLO], l0, l1, g.dt);
    }
    if (pr[PROF_LHI] > T(0)) {
      half += face_sigma_integral(pr + PROF_C, pr[PROF_LHI], u0, um, T(0.5) * g.dt);
      full += face_sigma_integral(pr + PROF_C, pr[PROF_LHI], u0, u1, g.dt);
    }
  }
}

// charge times weight w of particle p for the deposit of the move (i0, f0) -> (i1, f1);
// with weight damping also updates its Lambda
template <typename T, int DIM>
__device__ __forceinline__ T deposit_charge_w(const Grid<T> &g, const Parts<T> &P, int p, T w, const int (&i0)[3],
                                              const T (&f0)[3], const int (&i1)[3], const T (&f1)[3]) {
  T qw = g.charge * w;
  if (g.wdamp) {
    T half, full;
    path_lambda<T, DIM>(g, i0, f0, i1, f1, half, full);
    const T lam = P.lam[p];
    qw *= exp(-(lam + half));
    P.lam[p] = lam + full;
  }
  return qw;
}
template <typename T, int DIM>
__device__ __forceinline__ T deposit_charge(const Grid<T> &g, const Parts<T> &P, int p, const int (&i0)[3],
                                            const T (&f0)[3], const int (&i1)[3], const T (&f1)[3]) {
  return deposit_charge_w<T, DIM>(g, P, p, P.w[p], i0, f0, i1, f1);
}

// Nodes along one axis that a deposit moving from cell i0 to cell i1 can touch
template <int ORDER>
__device__ __forceinline__ void dep_range(int i0, int i1, int &lo, int &hi) {
  lo = min(i0, i1) + (ORDER == 1 ? -1 : -2);
  hi = max(i0, i1) + (ORDER == 1 ? 2 : 3);
}

// Union of the threads' node boxes (x lo, x hi, y lo, y hi; empty when lo > hi) over
// the workgroup, valid in thread 0.  Every thread of the workgroup calls it.
__device__ __forceinline__ int4 block_box(int xlo, int xhi, int ylo, int yhi) {
  __shared__ int sb[4];
  if (threadIdx.x == 0) { sb[0] = 0x7FFFFFFF; sb[1] = -0x7FFFFFFF; sb[2] = 0x7FFFFFFF; sb[3] = -0x7FFFFFFF; }
  __syncthreads();
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    xlo = min(xlo, __shfl_xor(xlo, off));
    xhi = max(xhi, __shfl_xor(xhi, off));
    ylo = min(ylo, __shfl_xor(ylo, off));
    yhi = max(yhi, __shfl_xor(yhi, off));
  }
  if ((threadIdx.x & 63) == 0 && xlo <= xhi) {
    atomicMin(&sb[0], xlo); atomicMax(&sb[1], xhi); atomicMin(&sb[2], ylo); atomicMax(&sb[3], yhi);
  }
  __syncthreads();
  return make_int4(sb[0], sb[1], sb[2], sb[3]);
}

// A batched run's box of nodes given current this step, grown by one workgroup
__device__ __forceinline__ void jbox_grow(int *jbox, int xlo, int xhi, int ylo, int yhi) {
  const int4 b = block_box(xlo, xhi, ylo, yhi);
  if (threadIdx.x == 0 && b.x <= b.y) {
    atomicMin(&jbox[0], b.x); atomicMax(&jbox[1], b.y); atomicMin(&jbox[2], b.z); atomicMax(&jbox[3], b.w);
  }
}

// One particle of the fused step (fused = true: gather, Boris, move, Esirkepov deposit
// into global J, removal) or of the first half of the unfused step (fused = false: the
// old position goes to `old`, the deposit follows in k_deposit).  Returns whether
// the slot held a live particle.
template <typename T, int DIM, int ORDER>
__device__ __forceinline__ bool push_one(const Grid<T> &g, const Fields<T> &F, const Parts<T> &P, const Parts<T> &old,
                                         int p, int push, bool fused, int *rng = nullptr) {
  const uint32_t c = P.cell[p];
  if (c == DEAD) return false;
  int id[3];
  unpack_cell(DIM, c, id[0], id[1], id[2]);
  T f[3] = {P.f[0][p], P.f[1][p], DIM == 3 ? P.f[2][p] : T(0)};
  T u[3] = {P.u[0][p], P.u[1][p], P.u[2][p]};
  if (push) {
    T EB[6];
    gather<T, DIM, ORDER>(g, F, id, f, EB);
    boris(g.qdt_2m, EB, u);
  }
  const int id0[3] = {id[0], id[1], id[2]};
  const T f0[3] = {f[0], f[1], f[2]};
  T ig;
  const bool inside = move<T, DIM>(g, id, f, u, ig);
  P.u[0][p] = u[0]; P.u[1][p] = u[1]; P.u[2][p] = u[2];
#pragma unroll
  for (int d = 0; d < DIM; ++d) P.f[d][p] = f[d];
  if (fused) {
    GlobalSink<T> sink{{F.J[0], F.J[1], F.J[2]}, 0, 0, 0};
    deposit<T, DIM, ORDER>(g, sink, id0, f0, id, f, u[2] * ig, deposit_charge<T, DIM>(g, P, p, id0, f0, id, f));
    if (rng) {
      dep_range<ORDER>(id0[0], id[0], rng[0], rng[1]);
      dep_range<ORDER>(id0[1], id[1], rng[2], rng[3]);
    }
    P.cell[p] = inside ? pack_cell(DIM, id[0], id[1], id[2]) : DEAD;
  } else {
    old.cell[p] = c;
#pragma unroll
    for (int d = 0; d < DIM; ++d) old.f[d][p] = f0[d];
    P.cell[p] = pack_cell(DIM, id[0], id[1], id[2]);
  }
  return true;
}

// Push tally of a wavefront, added to one of N_PUSH_COUNTERS words chosen by the
// wavefront (a single shared counter would serialise every wavefront of the grid).
__device__ __forceinline__ void count_pushes(unsigned long long *pushes, bool active) {
  const unsigned long long m = __ballot(active);
  if (m && (threadIdx.x & 63) == (unsigned)(__ffsll((long long)m) - 1)) {
    const unsigned slot = (blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) % N_PUSH_COUNTERS;
    atomicAdd(&pushes[slot], (unsigned long long)__popcll(m));
  }
}

}  // namespace pmlpic
