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

// ---------------------------------------------------------------- 3D sweeps
// The B half step and the E step of update_B_apply / update_E_apply (field_core.h) for the
// three components of one 3D node, with every load of the node requested up front (the
// conductor mask first, inside the one uniform branch; the neighbours of the far faces lie in
// the guard layers; a split part where the split is off reads the plain component, a value
// the update ignores): a memory round trip or two per node, where the per-component form
// waited on each load in turn.  Same arithmetic in the same order, so the same bits.
template <typename T>
struct NodeTabs {   // per-axis table entries at the node's index along each axis
  T sig[3], gk[3], eh[3];
};

// B_A at the node from its differences Db (along b = A + 1 of E_c) and Dc (along c = A + 2
// of E_b), the loaded B_A and split part, written back where the node holds a B_A sample
template <typename T, int A>
__device__ __forceinline__ void b_node(const Grid<T> &g, const Fields<T> &F, const int (&id)[3], long q,
                                       const NodeTabs<T> &t, T Db, T Dc, T b, T ba, uint32_t cm) {
  constexpr int Bx = (A + 1) % 3, Cx = (A + 2) % 3;
  if (id[A] > g.M[A] || id[Bx] > g.M[Bx] - 1 || id[Cx] > g.M[Cx] - 1) return;
  if (t.sig[Bx] + t.sig[Cx] > T(0)) {
    T p1 = ba;
    T p2 = b - p1;
    p1 = fma(-t.gk[Bx], Db, t.eh[Bx] * p1);
    p2 = fma(t.gk[Cx], Dc, t.eh[Cx] * p2);
    b = p1 + p2;
    ba = p1;
    gptr(F.Ba[A])[q] = ba;
  } else {
    b = fma(-t.gk[Bx], Db, fma(t.gk[Cx], Dc, b));
  }
  if ((cm >> (3 + A)) & 1) {   // inside a conductor
    b = T(0);
    gptr(F.Ba[A])[q] = T(0);
  }
  gptr(F.B[A])[q] = b;
}

template <typename T>
__global__ void __launch_bounds__(256) k_update_B3(Grid<T> g, Fields<T> F) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
  const int k = (int)blockIdx.z;
  if (i > g.M[0] || j > g.M[1]) return;
  const int id[3] = {i, j, k};
  const long q = g.at(i, j, k), sy = g.sy, sz = g.sz;
  uint32_t cm = 0;
  if (g.cmask) cm = gptr(g.cmask)[q];
  NodeTabs<T> t;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    t.sig[d] = g.tb(d, T_SIG_C, id[d]);
    t.gk[d] = g.tb(d, T_GHK_C, id[d]);
    t.eh[d] = g.tb(d, T_EH_C, id[d]);
  }
  const auto *E0 = gptr(F.E[0]), *E1 = gptr(F.E[1]), *E2 = gptr(F.E[2]);
  const T e0 = E0[q], e0y = E0[q + sy], e0z = E0[q + sz];
  const T e1 = E1[q], e1x = E1[q + 1], e1z = E1[q + sz];
  const T e2 = E2[q], e2x = E2[q + 1], e2y = E2[q + sy];
  const T b0 = gptr(F.B[0])[q], b1 = gptr(F.B[1])[q], b2 = gptr(F.B[2])[q];
  const T ba0 = gptr(t.sig[1] + t.sig[2] > T(0) ? F.Ba[0] : F.B[0])[q];
  const T ba1 = gptr(t.sig[2] + t.sig[0] > T(0) ? F.Ba[1] : F.B[1])[q];
  const T ba2 = gptr(t.sig[0] + t.sig[1] > T(0) ? F.Ba[2] : F.B[2])[q];
  b_node<T, 0>(g, F, id, q, t, e2y - e2, e1z - e1, b0, ba0, cm);   // B_x: d_y E_z, d_z E_y
  b_node<T, 1>(g, F, id, q, t, e0z - e0, e2x - e2, b1, ba1, cm);   // B_y: d_z E_x, d_x E_z
  b_node<T, 2>(g, F, id, q, t, e1x - e1, e0y - e0, b2, ba2, cm);   // B_z: d_x E_y, d_y E_x
}

template <typename T>
struct NodeTabsE {
  T sig[3], gk[3], gg[3], e[3], aC[3], aN[3];
};

// E_A at the node from Db (along b of B_c), Dc (along c of B_b) and the source J_A
template <typename T, int A>
__device__ __forceinline__ void e_node(const Grid<T> &g, const Fields<T> &F, const int (&id)[3], long q,
                                       const NodeTabsE<T> &t, T Db, T Dc, T e, T ea, T j, uint32_t cm,
                                       bool fuse_alpha, bool consume) {
  constexpr int Bx = (A + 1) % 3, Cx = (A + 2) % 3;
  if (id[A] > g.M[A] - 1) return;
  if (id[Bx] < 1 || id[Bx] > g.M[Bx] - 1) return;   // PEC: tangential E = 0
  if (id[Cx] < 1 || id[Cx] > g.M[Cx] - 1) return;
  if (consume && j != T(0)) gptr(F.J[A])[q] = T(0);   // leaves J zero for the next deposit
  if (fuse_alpha) {   // alpha_at: the product over the axes in order x, y, z
    T a = T(1);
#pragma unroll
    for (int d = 0; d < 3; ++d) a *= d == A ? t.aC[d] : t.aN[d];
    j *= a;
  }
  const T sb = t.sig[Bx], sc = t.sig[Cx];
  if (sb + sc > T(0)) {
    const T inv = T(1) / (sb + sc);
    T p1 = ea;
    T p2 = e - p1;
    p1 = fma(t.gk[Bx], Db, fma(-t.gg[Bx] * (sb * inv), j, t.e[Bx] * p1));
    p2 = fma(-t.gk[Cx], Dc, fma(-t.gg[Cx] * (sc * inv), j, t.e[Cx] * p2));
    e = p1 + p2;
    gptr(F.Ea[A])[q] = p1;
  } else {
    e = fma(t.gk[Bx], Db, fma(-t.gk[Cx], Dc, fma(-g.dt, j, e)));
  }
  if ((cm >> A) & 1) {   // inside a conductor
    e = T(0);
    gptr(F.Ea[A])[q] = T(0);
  }
  gptr(F.E[A])[q] = e;
}

template <typename T>
__global__ void __launch_bounds__(256) k_update_E3(Grid<T> g, Fields<T> F, bool fuse_alpha, bool consume) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
  const int k = (int)blockIdx.z;
  if (i > g.M[0] || j > g.M[1]) return;
  const int id[3] = {i, j, k};
  const long q = g.at(i, j, k), sy = g.sy, sz = g.sz;
  uint32_t cm = 0;
  if (g.cmask) cm = gptr(g.cmask)[q];
  NodeTabsE<T> t;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    t.sig[d] = g.tb(d, T_SIG_N, id[d]);
    t.gk[d] = g.tb(d, T_GK_N, id[d]);
    t.gg[d] = g.tb(d, T_G_N, id[d]);
    t.e[d] = g.tb(d, T_E_N, id[d]);
    t.aC[d] = g.tb(d, T_A_C, id[d]);
    t.aN[d] = g.tb(d, T_A_N, id[d]);
  }
  const auto *B0 = gptr(F.B[0]), *B1 = gptr(F.B[1]), *B2 = gptr(F.B[2]);
  const T b0 = B0[q], b0y = B0[q - sy], b0z = B0[q - sz];
  const T b1 = B1[q], b1x = B1[q - 1], b1z = B1[q - sz];
  const T b2 = B2[q], b2x = B2[q - 1], b2y = B2[q - sy];
  const T e0 = gptr(F.E[0])[q], e1 = gptr(F.E[1])[q], e2 = gptr(F.E[2])[q];
  const T j0 = gptr(F.J[0])[q], j1 = gptr(F.J[1])[q], j2 = gptr(F.J[2])[q];
  const T ea0 = gptr(t.sig[1] + t.sig[2] > T(0) ? F.Ea[0] : F.E[0])[q];
  const T ea1 = gptr(t.sig[2] + t.sig[0] > T(0) ? F.Ea[1] : F.E[1])[q];
  const T ea2 = gptr(t.sig[0] + t.sig[1] > T(0) ? F.Ea[2] : F.E[2])[q];
  // E_x: d_y B_z, d_z B_y; E_y: d_z B_x, d_x B_z; E_z: d_x B_y, d_y B_x
  e_node<T, 0>(g, F, id, q, t, b2 - b2y, b1 - b1z, e0, ea0, j0, cm, fuse_alpha, consume);
  e_node<T, 1>(g, F, id, q, t, b0 - b0z, b2 - b2x, e1, ea1, j1, cm, fuse_alpha, consume);
  e_node<T, 2>(g, F, id, q, t, b1 - b1x, b0 - b0y, e2, ea2, j2, cm, fuse_alpha, consume);
}

// Cole-Karkkainen B half step (3D), marching along z.  Each CK difference is a weighted
// sum over the plane normal to its axis: along z, the difference of the 9-point in-plane
// averages P(k) of two consecutive planes; along x or y, a 3-point row average of the Yee
// differences in plane k plus a lighter one in planes k - 1 and k + 1.  A thread owns one
// (i, j) column of a chunk of planes and keeps these per-plane sums for planes k - 1, k,
// k + 1 in registers, so each E plane is read once per chunk (27 loads per node and plane,
// neighbours from the same cache lines) instead of 108 scattered ones per node.
template <typename T>
struct CkPlane {
  T S0, S1;   // x-rows of d_y E_z (weights 1/12 7/12 1/12 in the plane, 1/48 1/12 1/48 beside it)
  T W0, W1;   // the same of d_y E_x
  T U0, U1;   // y-rows of d_x E_z
  T V0, V1;   // the same of d_x E_y
  T P, Q;     // 9-point averages of E_y and E_x (7/12 centre, 1/12 sides, 1/48 corners)
};

template <typename T>
__device__ __forceinline__ CkPlane<T> ck_plane(const Grid<T> &g, const Fields<T> &F, int i, int j, int k) {
  const T a0 = T(7.0 / 12.0), a1 = T(1.0 / 12.0), a2 = T(1.0 / 48.0);
  const long q = g.at(i, j, k);
  T ex[3][3], ey[3][3], ez[3][3];   // [y - j + 1][x - i + 1]
#pragma unroll
  for (int dy = 0; dy < 3; ++dy)
#pragma unroll
    for (int dx = 0; dx < 3; ++dx) {
      const long o = q + (dy - 1) * g.sy + (dx - 1);
      ex[dy][dx] = F.E[0][o];
      ey[dy][dx] = F.E[1][o];
      ez[dy][dx] = F.E[2][o];
    }
  CkPlane<T> r;
  auto xrows = [&](T (&e)[3][3], T &w0, T &w1) {   // d_y along the x-row of row j
    const T m = e[2][0] - e[1][0], c = e[2][1] - e[1][1], p = e[2][2] - e[1][2];
    w0 = a0 * c + a1 * (m + p);
    w1 = a1 * c + a2 * (m + p);
  };
  auto yrows = [&](T (&e)[3][3], T &w0, T &w1) {   // d_x along the y-column of column i
    const T m = e[0][2] - e[0][1], c = e[1][2] - e[1][1], p = e[2][2] - e[2][1];
    w0 = a0 * c + a1 * (m + p);
    w1 = a1 * c + a2 * (m + p);
  };
  auto nine = [&](T (&e)[3][3]) {
    return a0 * e[1][1] + a1 * ((e[0][1] + e[2][1]) + (e[1][0] + e[1][2])) +
           a2 * ((e[0][0] + e[0][2]) + (e[2][0] + e[2][2]));
  };
  xrows(ez, r.S0, r.S1);
  xrows(ex, r.W0, r.W1);
  yrows(ez, r.U0, r.U1);
  yrows(ey, r.V0, r.V1);
  r.P = nine(ey);
  r.Q = nine(ex);
  return r;
}

template <typename T>
__global__ void __launch_bounds__(256) k_update_B_ck(Grid<T> g, Fields<T> F, int kz) {
  const int i = (int)(blockIdx.x * 64 + (threadIdx.x & 63));
  const int j = (int)(blockIdx.y * 4 + (threadIdx.x >> 6));
  const int k0 = (int)blockIdx.z * kz, k1 = min(k0 + kz, g.M[2] + 1);
  if (i > g.M[0] || j > g.M[1] || k0 >= k1) return;
  NodeTabs<T> t;   // x and y entries fixed for the column; z entries per plane (scalar loads)
  t.sig[0] = g.tb(0, T_SIG_C, i);
  t.gk[0] = g.tb(0, T_GHK_C, i);
  t.eh[0] = g.tb(0, T_EH_C, i);
  t.sig[1] = g.tb(1, T_SIG_C, j);
  t.gk[1] = g.tb(1, T_GHK_C, j);
  t.eh[1] = g.tb(1, T_EH_C, j);
  CkPlane<T> pm = ck_plane(g, F, i, j, k0 - 1), p0 = ck_plane(g, F, i, j, k0);
  for (int k = k0; k < k1; ++k) {
    const int id[3] = {i, j, k};
    const long q = g.at(i, j, k);
    uint32_t cm = 0;
    if (g.cmask) cm = gptr(g.cmask)[q];
    t.sig[2] = g.tb_uniform(2, T_SIG_C, k);
    t.gk[2] = g.tb_uniform(2, T_GHK_C, k);
    t.eh[2] = g.tb_uniform(2, T_EH_C, k);
    const CkPlane<T> pp = ck_plane(g, F, i, j, k + 1);
    const T b0 = gptr(F.B[0])[q], b1 = gptr(F.B[1])[q], b2 = gptr(F.B[2])[q];
    const T ba0 = gptr(t.sig[1] + t.sig[2] > T(0) ? F.Ba[0] : F.B[0])[q];
    const T ba1 = gptr(t.sig[2] + t.sig[0] > T(0) ? F.Ba[1] : F.B[1])[q];
    const T ba2 = gptr(t.sig[0] + t.sig[1] > T(0) ? F.Ba[2] : F.B[2])[q];
    // B_x: b = y (E_z), c = z (E_y); B_y: b = z (E_x), c = x (E_z); B_z: b = x (E_y), c = y (E_x)
    b_node<T, 0>(g, F, id, q, t, p0.S0 + (pm.S1 + pp.S1), pp.P - p0.P, b0, ba0, cm);
    b_node<T, 1>(g, F, id, q, t, pp.Q - p0.Q, p0.U0 + (pm.U1 + pp.U1), b1, ba1, cm);
    b_node<T, 2>(g, F, id, q, t, p0.V0 + (pm.V1 + pp.V1), p0.W0 + (pm.W1 + pp.W1), b2, ba2, cm);
    pm = p0;
    p0 = pp;
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

// planes per chunk: 16 on large grids, fewer on small ones so that a launch keeps a few
// thousand workgroups
static int zchunk(const int M[3], int per_plane_groups_mult, int &nchunk) {
  const int gx = (M[0] + 1 + 63) / 64, gy = (M[1] + 1 + 3) / 4;
  const int mult = per_plane_groups_mult * gx * gy;
  const int want = (4096 + mult - 1) / mult;
  const int kz = std::max(2, std::min(16, (M[2] + 1 + want - 1) / want));
  nchunk = (M[2] + 1 + kz - 1) / kz;
  return kz;
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

// rows per segment: enough wavefronts to fill the GPU (about 8192), 4 to 64 rows
// (measured on the 1056^2 beam grid: 8 rows 24.9 us, 4 rows 20.3 us, 3 rows 23.8 us,
// 2 rows 23.3 us per pass)
void fused_2d_shape(int M0, int M1, int &nstrips, int &rows, int &nseg) {
  nstrips = (M0 + 1 + FW - 1) / FW;
  const long want = 8192;
  rows = (int)std::min<long>(64, std::max<long>(4, (long)nstrips * (M1 + 1) / want));
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
  else if (g.solver == PML_PIC_SOLVER_CK) {
    int nchunk;
    const int kz = zchunk(g.M, 1, nchunk);
    hipLaunchKernelGGL((k_update_B_ck<T>), dim3(grd.x, grd.y, nchunk), dim3(256), 0, s, g, F, kz);
  }
  else hipLaunchKernelGGL((k_update_B3<T>), grd, blk, 0, s, g, F);
}

template <typename T>
void launch_update_E(const Grid<T> &g, const Fields<T> &F, bool fuse_alpha, int alpha_mode, bool consume,
                     hipStream_t s) {
  dim3 blk, grd = node_grid(g, blk);
  const bool fa = fuse_alpha && current_alpha(alpha_mode);
  if (g.dim == 2) hipLaunchKernelGGL((k_update_E<T, 2>), grd, blk, 0, s, g, F, fa, consume);
  else hipLaunchKernelGGL((k_update_E3<T>), grd, blk, 0, s, g, F, fa, consume);
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
  // neighbour weights, zero outside the extents: all nine loads of a plane are issued on every
  // path (the neighbours lie in the guard layers or hold finite samples) and then combined, one
  // memory round trip per plane instead of one per load
  const T wl = i > 0 ? T(0.25) : T(0), wr = i + 1 < ext0 ? T(0.25) : T(0);
  const T wd = j > 0 ? T(0.25) : T(0), wu = j + 1 < ext1 ? T(0.25) : T(0);
  auto row = [&](long q) {
    const T c = gptr(J)[q], l = gptr(J)[q - 1], r = gptr(J)[q + 1];
    T v = T(0.5) * c;
    v += wl * l;
    v += wr * r;
    return v;
  };
  auto plane = [&](int k) {
    const long q = g.at(i, j, k);   // k in [-1, ext2]: inside the guard layers
    const T rd = row(q - g.sy), r0 = row(q), ru = row(q + g.sy);
    T p = T(0.5) * r0;
    p += wd * rd;
    p += wu * ru;
    return k >= 0 && k < ext2 ? p : T(0);
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
  int nchunk;
  const int kz = zchunk(g.M, 3, nchunk);
  dim3 blk(256), grd((g.M[0] + 1 + 63) / 64, (g.M[1] + 1 + 3) / 4, 3 * nchunk);
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
