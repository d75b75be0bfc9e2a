// update_yee_pml as one pass over 3D fields: B half step, E step, B half step (the split
// Yee/PML update of Sec. II.A, Eqs. MaxwellE / MaxwellB / MaxwellSum, with the damped
// source -alpha J), with the arithmetic of update_B_apply / update_E_apply in the same
// order, so the result equals the three in-place sweeps bit for bit.  Each field sample is
// read once from one set of arrays and written once to the other set (out of place: the
// halo reads of a workgroup must see the old values while its neighbour writes).
//
// A workgroup of 16 wavefronts owns a strip of FW = 61 columns (x), 14 rows (y) and a chunk
// of planes (z), and marches along z.  Wavefront w holds row j = y0 - 1 + w, lane l column
// i = x0 - 1 + l: x neighbours come from the adjacent lanes (shuffles), z neighbours from
// the previous plane kept in registers, y neighbours through LDS (each wavefront publishes
// its row of B^{n+1/2} and of E^{n+1}).  At plane k it computes B^{n+1/2}(k), E^{n+1}(k)
// and B^{n+1}(k - 1).  Halo work: lanes 0, 62, 63, the rows y0 - 1 and y0 + 14, and one
// plane before and after the chunk, computed and thrown away (the last plane's loads are
// issued twice, the second time unused).  Every owned sample in
// [0, M] is written (a sample the update leaves alone is copied); split parts wherever the
// split is active.  The current of this step is read (and not cleared); the other current
// buffer, read by the previous step, is cleared over the owned samples for the next deposit.
#include <algorithm>

#include "common.h"

namespace pmlpic {

// output rows per workgroup (with one halo row on each side, ROWS + 2 wavefronts): 14 in
// FP32; 6 in FP64, whose registers would not fit 16 wavefronts.  ITEMS: the number of
// workgroups the chunks of planes aim at (see fused_3d_shape)
template <typename T> struct F3Cfg {
  static constexpr int ROWS = 14;
  static constexpr long ITEMS = 1536;
};
template <> struct F3Cfg<double> {
  static constexpr int ROWS = 6;
  static constexpr long ITEMS = 2048;
};

template <typename T>
struct Tab9 {   // per-axis tables at one index: the kinds the B and E updates read
  T sigC, ghkC, ehC, sigN, gkN, eN, gN, aC, aN;
};
template <typename T>
__device__ __forceinline__ void load_tab9(const Grid<T> &g, int axis, int idx, Tab9<T> &t) {
  t.sigC = g.tb(axis, T_SIG_C, idx);
  t.ghkC = g.tb(axis, T_GHK_C, idx);
  t.ehC = g.tb(axis, T_EH_C, idx);
  t.sigN = g.tb(axis, T_SIG_N, idx);
  t.gkN = g.tb(axis, T_GK_N, idx);
  t.eN = g.tb(axis, T_E_N, idx);
  t.gN = g.tb(axis, T_G_N, idx);
  t.aC = g.tb(axis, T_A_C, idx);
  t.aN = g.tb(axis, T_A_N, idx);
}

// a value that is the same in every lane, moved to a scalar register
__device__ __forceinline__ float wave_uniform(float v) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}
__device__ __forceinline__ double wave_uniform(double v) {
  const long long b = __double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)b);
  const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(b >> 32));
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
template <typename T>
__device__ __forceinline__ Tab9<T> wave_uniform(const Tab9<T> &t) {
  return {wave_uniform(t.sigC), wave_uniform(t.ghkC), wave_uniform(t.ehC), wave_uniform(t.sigN), wave_uniform(t.gkN),
          wave_uniform(t.eN),   wave_uniform(t.gN),   wave_uniform(t.aC),  wave_uniform(t.aN)};
}

template <typename T>
struct Vec3S { T x, y, z, xa, ya, za; };   // three components and their split parts

// B half step of one component (update_B_apply): part b driven by -Db (rate along b),
// part c by +Dc (rate along c)
template <typename T>
__device__ __forceinline__ void bstep1(T &b, T &ba, const Tab9<T> &TB, const Tab9<T> &TC, T Db, T Dc) {
  if (TB.sigC + TC.sigC > T(0)) {
    T p1 = ba;
    T p2 = b - p1;
    p1 = fma(-TB.ghkC, Db, TB.ehC * p1);
    p2 = fma(TC.ghkC, Dc, TC.ehC * p2);
    b = p1 + p2;
    ba = p1;
  } else {
    b = fma(-TB.ghkC, Db, fma(TC.ghkC, Dc, b));
  }
}

// E step of one component (update_E_apply) with the source j (alpha already applied)
template <typename T>
__device__ __forceinline__ void estep1(T &e, T &ea, const Tab9<T> &TB, const Tab9<T> &TC, T Db, T Dc, T j, T dt) {
  const T sb = TB.sigN, sc = TC.sigN;
  if (sb + sc > T(0)) {
    const T inv = T(1) / (sb + sc);
    T p1 = ea;
    T p2 = e - p1;
    p1 = fma(TB.gkN, Db, fma(-TB.gN * (sb * inv), j, TB.eN * p1));
    p2 = fma(-TC.gkN, Dc, fma(-TC.gN * (sc * inv), j, TC.eN * p2));
    e = p1 + p2;
    ea = p1;
  } else {
    e = fma(TB.gkN, Db, fma(-TC.gkN, Dc, fma(-dt, j, e)));
  }
}

constexpr int F3_KZMAX = 64;   // planes per chunk at most

// Every load of the plane loop is issued whatever the lane's position, into the register
// that keeps it: an index outside the sample range is clamped to the range (such lanes and
// rows feed only samples the workgroup does not own), and a split part where the split is
// off reads the plain component at the same sample (a value the update then ignores).  With
// the z tables of the chunk's planes in LDS, the next plane's loads are a fixed count that
// the wave leaves in flight while it works on the current plane (a load skipped on some
// path, or a condition on a value just loaded, would make it wait for every load in flight).
template <typename T, int F3_ROWS = F3Cfg<T>::ROWS, int F3_WAVES = F3_ROWS + 2>
__global__ void __launch_bounds__(64 * F3_WAVES) k_fused_3d(Grid<T> g, Fields<T> F, Fields<T> D, JZero<T> jz,
                                                            int nstrips, int nrb, int kz, int nchunk, bool fuse_alpha) {
  // rows published through LDS, in two sets by plane parity: plane k writes set k & 1 and
  // reads set (k - 1) & 1 of the plane before, so that one barrier per plane orders them (a
  // set is rewritten two planes later, after every wavefront has passed the barrier between)
  __shared__ T sh_bx[2][F3_WAVES][64], sh_bz[2][F3_WAVES][64], sh_ex[2][F3_WAVES][64], sh_ez[2][F3_WAVES][64];
  __shared__ Tab9<T> sh_tz[F3_KZMAX + 3];   // z tables of planes k0 - 1 .. k1 + 1
  // workgroup b runs on XCD b mod 8: each XCD takes a contiguous eighth of the items, so
  // that neighbouring strips and rows (which read each other's halo) share its L2
  const int per = (int)(gridDim.x >> 3);
  const int item = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
  if (item >= nstrips * nrb * nchunk) return;   // whole workgroup
  const int strip = item % nstrips, rb = (item / nstrips) % nrb, chunk = item / (nstrips * nrb);
  const int lane = (int)(threadIdx.x & 63);
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int M0 = g.M[0], M1 = g.M[1], M2 = g.M[2];
  const int i = strip * FW - 1 + lane;
  const int j = rb * F3_ROWS - 1 + w;
  const int k0 = chunk * kz, k1 = min(k0 + kz, M2 + 1);
  for (int p = (int)threadIdx.x; p <= k1 - k0 + 2; p += 64 * F3_WAVES)
    load_tab9(g, 2, min(max(k0 - 1 + p, -G), M2 + G), sh_tz[p]);
  const bool own = lane >= 1 && lane <= FW && i <= M0 && w >= 1 && w <= F3_ROWS && j <= M1;
  Tab9<T> X, Y;   // x tables per lane, y tables per wavefront (scalar registers)
  load_tab9(g, 0, min(max(i, -G), M0 + G), X);
  load_tab9(g, 1, min(max(j, -G), M1 + G), Y);
  Y = wave_uniform(Y);
  // update extents: B_a at index <= M along a, <= M - 1 across; E_a at <= M - 1 along a,
  // in [1, M - 1] across (PEC walls); nothing below 0
  const bool bx_x = i >= 0 && i <= M0, bx_c = i >= 0 && i <= M0 - 1, ex_a = i >= 0 && i <= M0 - 1,
             ex_c = i >= 1 && i <= M0 - 1;
  const bool by_y = j >= 0 && j <= M1, by_c = j >= 0 && j <= M1 - 1, ey_a = j >= 0 && j <= M1 - 1,
             ey_c = j >= 1 && j <= M1 - 1;
  const long sz = g.sz;
  // sample offsets of plane 0 at the column and row clamped to the sample range (equal to
  // the lane's own where it owns a sample), and at the row above
  const int ic = min(max(i, -G), M0 + G);
  const long q0 = g.at(ic, min(max(j, -G), M1 + G), 0);
  const long q0r = g.at(ic, min(max(j + 1, -G), M1 + G), 0);
  auto ld = [&](const T *a, long q) -> T { return gptr(a)[q]; };
  auto ld_split = [&](const T *part, const T *plain, long q, bool on) -> T { return gptr(on ? part : plain)[q]; };
  const int wm = max(w - 1, 0), wp = min(w + 1, F3_WAVES - 1);   // LDS rows of j - 1, j + 1

  // inputs of plane k: E^n at k + 1, E^n at row j + 1, B^n, split parts, J
  struct In {
    T ex1, ey1, ez1;   // E^n(k + 1)
    T exr, ezr;        // E^n at row j + 1, plane k
    T exa, eya, eza;   // split parts of E^n(k)
    T bx, by, bz, bxa, bya, bza;
    T jx, jy, jz;
  };
  auto fetch = [&](int k, In &r) {
    const Tab9<T> Z = wave_uniform(sh_tz[k - k0 + 1]);
    const long q = q0 + (long)k * sz;
    r.ex1 = ld(F.E[0], q + sz);
    r.ey1 = ld(F.E[1], q + sz);
    r.ez1 = ld(F.E[2], q + sz);
    r.exr = ld(F.E[0], q0r + (long)k * sz);
    r.ezr = ld(F.E[2], q0r + (long)k * sz);
    r.exa = ld_split(F.Ea[0], F.E[0], q, Y.sigN + Z.sigN > T(0));
    r.eya = ld_split(F.Ea[1], F.E[1], q, Z.sigN + X.sigN > T(0));
    r.eza = ld_split(F.Ea[2], F.E[2], q, X.sigN + Y.sigN > T(0));
    r.bx = ld(F.B[0], q);
    r.by = ld(F.B[1], q);
    r.bz = ld(F.B[2], q);
    r.bxa = ld_split(F.Ba[0], F.B[0], q, Y.sigC + Z.sigC > T(0));
    r.bya = ld_split(F.Ba[1], F.B[1], q, Z.sigC + X.sigC > T(0));
    r.bza = ld_split(F.Ba[2], F.B[2], q, X.sigC + Y.sigC > T(0));
    r.jx = ld(F.J[0], q);
    r.jy = ld(F.J[1], q);
    r.jz = ld(F.J[2], q);
  };

  __syncthreads();   // the z tables
  int k = k0 - 1;
  T ecx = ld(F.E[0], q0 + (long)k * sz), ecy = ld(F.E[1], q0 + (long)k * sz),
    ecz = ld(F.E[2], q0 + (long)k * sz);   // E^n(k)
  In ia, ib;
  fetch(k, ia);
  Tab9<T> Zp, Zc = wave_uniform(sh_tz[0]);   // tables of planes k - 1, k
  Zp = Zc;
  Vec3S<T> bhp = {T(0), T(0), T(0), T(0), T(0), T(0)};   // B^{n+1/2}(k - 1)
  Vec3S<T> enp = {T(0), T(0), T(0), T(0), T(0), T(0)};   // E^{n+1}(k - 1)
  // the work at plane k from its inputs cur, then the advance to plane k + 1
  auto plane = [&](const int k, const In &cur) {
    const bool bz_z = k >= 0 && k <= M2, bz_c = k >= 0 && k <= M2 - 1, ez_a = k >= 0 && k <= M2 - 1,
               ez_c = k >= 1 && k <= M2 - 1;
    // B^{n+1/2}(k)
    Vec3S<T> bh = {cur.bx, cur.by, cur.bz, cur.bxa, cur.bya, cur.bza};
    {
      const T ez_r = __shfl_down(ecz, 1), ey_r = __shfl_down(ecy, 1);
      if (bx_x && by_c && bz_c) bstep1(bh.x, bh.xa, Y, Zc, cur.ezr - ecz, cur.ey1 - ecy);   // B_x: b = y, c = z
      if (bx_c && by_y && bz_c) bstep1(bh.y, bh.ya, Zc, X, cur.ex1 - ecx, ez_r - ecz);      // B_y: b = z, c = x
      if (bx_c && by_c && bz_z) bstep1(bh.z, bh.za, X, Y, ey_r - ecy, cur.exr - ecx);       // B_z: b = x, c = y
    }
    const int cb = k & 1, pb = cb ^ 1;   // LDS sets of this plane and of the one before
    sh_bx[cb][w][lane] = bh.x;
    sh_bz[cb][w][lane] = bh.z;
    __syncthreads();
    // E^{n+1}(k)
    Vec3S<T> en = {ecx, ecy, ecz, cur.exa, cur.eya, cur.eza};
    {
      const T bz_l = __shfl_up(bh.z, 1), by_l = __shfl_up(bh.y, 1);
      const T bxm = sh_bx[cb][wm][lane], bzm = sh_bz[cb][wm][lane];   // B^{n+1/2} at row j - 1
      T jx = cur.jx, jy = cur.jy, jzv = cur.jz;
      if (fuse_alpha) {   // alpha_at: the product over the axes in order x, y, z
        jx *= (T(1) * X.aC) * Y.aN * Zc.aN;
        jy *= (T(1) * X.aN) * Y.aC * Zc.aN;
        jzv *= (T(1) * X.aN) * Y.aN * Zc.aC;
      }
      if (ex_a && ey_c && ez_c) estep1(en.x, en.xa, Y, Zc, bh.z - bzm, bh.y - bhp.y, jx, g.dt);    // E_x: b = y, c = z
      if (ex_c && ey_a && ez_c) estep1(en.y, en.ya, Zc, X, bh.x - bhp.x, bh.z - bz_l, jy, g.dt);   // E_y: b = z, c = x
      if (ex_c && ey_c && ez_a) estep1(en.z, en.za, X, Y, bh.y - by_l, bh.x - bxm, jzv, g.dt);     // E_z: b = x, c = y
    }
    if (own && k >= k0 && k < k1) {
      const long q = q0 + (long)k * sz;
      gptr(D.E[0])[q] = en.x;
      gptr(D.E[1])[q] = en.y;
      gptr(D.E[2])[q] = en.z;
      if (Y.sigN + Zc.sigN > T(0)) gptr(D.Ea[0])[q] = en.xa;
      if (Zc.sigN + X.sigN > T(0)) gptr(D.Ea[1])[q] = en.ya;
      if (X.sigN + Y.sigN > T(0)) gptr(D.Ea[2])[q] = en.za;
      gptr(jz.J[0])[q] = T(0);
      gptr(jz.J[1])[q] = T(0);
      gptr(jz.J[2])[q] = T(0);
    }
    // B^{n+1}(k - 1) from B^{n+1/2}(k - 1) and E^{n+1} at planes k - 1, k
    if (k >= k0 + 1) {
      const int km = k - 1;
      const bool bz_zm = km <= M2, bz_cm = km <= M2 - 1;   // km >= k0 >= 0
      const T pz_r = __shfl_down(enp.z, 1), py_r = __shfl_down(enp.y, 1);
      const T exp1 = sh_ex[pb][wp][lane], ezp1 = sh_ez[pb][wp][lane];   // E^{n+1}(k - 1) at row j + 1
      Vec3S<T> b = bhp;
      if (bx_x && by_c && bz_cm) bstep1(b.x, b.xa, Y, Zp, ezp1 - enp.z, en.y - enp.y);
      if (bx_c && by_y && bz_cm) bstep1(b.y, b.ya, Zp, X, en.x - enp.x, pz_r - enp.z);
      if (bx_c && by_c && bz_zm) bstep1(b.z, b.za, X, Y, py_r - enp.y, exp1 - enp.x);
      if (own) {
        const long q = q0 + (long)km * sz;
        gptr(D.B[0])[q] = b.x;
        gptr(D.B[1])[q] = b.y;
        gptr(D.B[2])[q] = b.z;
        if (Y.sigC + Zp.sigC > T(0)) gptr(D.Ba[0])[q] = b.xa;
        if (Zp.sigC + X.sigC > T(0)) gptr(D.Ba[1])[q] = b.ya;
        if (X.sigC + Y.sigC > T(0)) gptr(D.Ba[2])[q] = b.za;
      }
    }
    sh_ex[cb][w][lane] = en.x;
    sh_ez[cb][w][lane] = en.z;
    // advance one plane
    bhp = bh;
    enp = en;
    Zp = Zc;
    Zc = wave_uniform(sh_tz[k - k0 + 2]);
    ecx = cur.ex1;
    ecy = cur.ey1;
    ecz = cur.ez1;
  };
  // the next plane's loads go out before this plane's arithmetic (at the last plane, those
  // of that plane again, cache hits and not used: a fixed load count on every path)
  for (; k <= k1; ++k) {
    fetch(min(k + 1, k1), ib);
    plane(k, ia);
    ia = ib;
  }
}

// planes per chunk, so that the launch holds about `want` workgroups: longer chunks re-read
// fewer halo planes, shorter ones balance the compute units better.  FP32 on the 281^3-sample
// beam grid (16-wavefront workgroups, one per compute unit): 9 planes 0.70 ms, 14 planes
// 0.685 ms, 19 planes 0.67 ms, 28 planes 0.70 ms, 38 planes 0.73 ms per pass
static void fused_3d_shape(const int M[3], int rows, long want, int &nstrips, int &nrb, int &kz, int &nchunk) {
  nstrips = (M[0] + 1 + FW - 1) / FW;
  nrb = (M[1] + 1 + rows - 1) / rows;
  const long per_plane = (long)nstrips * nrb;
  kz = (int)std::min<long>(F3_KZMAX, std::max<long>(8, (M[2] + 1) * per_plane / want));
  nchunk = (M[2] + 1 + kz - 1) / kz;
}

template <typename T>
void launch_fused_fields_3d(const Grid<T> &g, const Fields<T> &F, const Fields<T> &D, const JZero<T> &jz,
                            bool fuse_alpha, hipStream_t s) {
  constexpr int rows = F3Cfg<T>::ROWS;
  int nstrips, nrb, kz, nchunk;
  fused_3d_shape(g.M, rows, F3Cfg<T>::ITEMS, nstrips, nrb, kz, nchunk);
  const long items = (long)nstrips * nrb * nchunk;
  const unsigned blocks = (unsigned)((items + 7) / 8 * 8);
  hipLaunchKernelGGL((k_fused_3d<T>), dim3(blocks), dim3(64 * (rows + 2)), 0, s, g, F, D, jz, nstrips, nrb, kz,
                     nchunk, fuse_alpha);
}
template void launch_fused_fields_3d<float>(const Grid<float> &, const Fields<float> &, const Fields<float> &,
                                            const JZero<float> &, bool, hipStream_t);
template void launch_fused_fields_3d<double>(const Grid<double> &, const Fields<double> &, const Fields<double> &,
                                             const JZero<double> &, bool, hipStream_t);

}  // namespace pmlpic
