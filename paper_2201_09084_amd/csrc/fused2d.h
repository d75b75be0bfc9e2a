// update_yee_pml as one pass over 2D fields: B half step, E step, B half step (the
// same arithmetic as update_B_comp / update_E_comp, in the same order, so the result
// equals the three separate sweeps bit for bit), reading each field sample once from
// one set of arrays and writing it once to the other set (out of place: a wavefront's
// halo reads must see the old values while the neighbouring wavefront writes).
//
// A wavefront owns a strip of FW = 61 columns and a segment of rows.  Lane l holds
// column i = x0 - 1 + l; the x neighbours come from the adjacent lanes (shuffles), the
// y neighbours from the previous row kept in registers.  Marching up the rows, at row
// j it has E^n at rows j and j+1 and computes B^{n+1/2}(j), E^{n+1}(j) and
// B^{n+1}(j-1).  Halo work: the lanes 0, 62, 63 and one row before and after the
// segment, computed and thrown away.  Every owned sample in [0, M] is written (a
// sample the update leaves alone is copied); split parts wherever the split is active.
// The current is read, not cleared, and only inside the box of nodes the deposits of
// this step touched (it is zero elsewhere).
#pragma once
#include "common.h"

namespace pmlpic {

template <typename T>
struct XTab {            // per-lane tables along x at the lane's column
  T ehC, ghkC, sigC, eN, gN, gkN, sigN, aC, aN;
};
template <typename T>
struct YTab {            // tables along y at one row
  T ehC, ghkC, sigC, eN, gN, gkN, sigN, aC, aN;
};

template <typename T>
__device__ __forceinline__ void load_tabs(const Grid<T> &g, int axis, int idx, T &ehC, T &ghkC, T &sigC, T &eN,
                                          T &gN, T &gkN, T &sigN, T &aC, T &aN) {
  ehC = g.tb(axis, T_EH_C, idx);
  ghkC = g.tb(axis, T_GHK_C, idx);
  sigC = g.tb(axis, T_SIG_C, idx);
  eN = g.tb(axis, T_E_N, idx);
  gN = g.tb(axis, T_G_N, idx);
  gkN = g.tb(axis, T_GK_N, idx);
  sigN = g.tb(axis, T_SIG_N, idx);
  aC = g.tb(axis, T_A_C, idx);
  aN = g.tb(axis, T_A_N, idx);
}

template <typename T>
struct BRow { T x, y, z, za; };
template <typename T>
struct ERow { T x, y, z, za; };

// B half step at (i, j) from B (with its z split part) and the E differences.
// dEz_y = Ez(i,j+1) - Ez(i,j), dEz_x = Ez(i+1,j) - Ez(i,j), dEy_x = Ey(i+1,j) - Ey(i,j),
// dEx_y = Ex(i,j+1) - Ex(i,j).
template <typename T>
__device__ __forceinline__ void bhalf_2d(BRow<T> &b, const XTab<T> &X, const YTab<T> &Y, bool vx, bool vy, bool vz,
                                         T dEz_y, T dEz_x, T dEy_x, T dEx_y) {
  if (vx) b.x = fma(-Y.ghkC, dEz_y, Y.ehC * b.x);          // B_x: -d_y E_z, rate along y
  if (vy) b.y = fma(X.ghkC, dEz_x, X.ehC * b.y);           // B_y: +d_x E_z, rate along x
  if (vz) {                                                // B_z: -d_x E_y + d_y E_x
    if (X.sigC + Y.sigC > T(0)) {
      T p1 = b.za;
      T p2 = b.z - p1;
      p1 = fma(-X.ghkC, dEy_x, X.ehC * p1);
      p2 = fma(Y.ghkC, dEx_y, Y.ehC * p2);
      b.z = p1 + p2;
      b.za = p1;
    } else {
      b.z = fma(-X.ghkC, dEy_x, fma(Y.ghkC, dEx_y, b.z));
    }
  }
}

// E step at (i, j); dBz_y = Bz(i,j) - Bz(i,j-1), dBz_x = Bz(i,j) - Bz(i-1,j),
// dBy_x = By(i,j) - By(i-1,j), dBx_y = Bx(i,j) - Bx(i,j-1) (all at n+1/2)
template <typename T>
__device__ __forceinline__ void estep_2d(ERow<T> &e, const XTab<T> &X, const YTab<T> &Y, bool vx, bool vy, bool vz,
                                         T dBz_y, T dBz_x, T dBy_x, T dBx_y, T jx, T jy, T jz, bool fuse_alpha,
                                         T dt) {
  if (fuse_alpha) {
    jx *= X.aC * Y.aN;
    jy *= X.aN * Y.aC;
    jz *= X.aN * Y.aN;
  }
  if (vx) e.x = fma(Y.gkN, dBz_y, fma(-Y.gN, jx, Y.eN * e.x));     // E_x: +d_y B_z
  if (vy) e.y = fma(-X.gkN, dBz_x, fma(-X.gN, jy, X.eN * e.y));    // E_y: -d_x B_z
  if (vz) {                                                        // E_z: +d_x B_y - d_y B_x
    const T sb = X.sigN, sc = Y.sigN;
    if (sb + sc > T(0)) {
      const T inv = T(1) / (sb + sc);
      T p1 = e.za;
      T p2 = e.z - p1;
      p1 = fma(X.gkN, dBy_x, fma(-X.gN * (sb * inv), jz, X.eN * p1));
      p2 = fma(-Y.gkN, dBx_y, fma(-Y.gN * (sc * inv), jz, Y.eN * p2));
      e.z = p1 + p2;
      e.za = p1;
    } else {
      e.z = fma(X.gkN, dBy_x, fma(-Y.gkN, dBx_y, fma(-dt, jz, e.z)));
    }
  }
}

// Loads of one row j, issued one row ahead of their use: E_x, E_z at row j+1 and
// E_y, the split parts, B and J at row j.
template <typename T>
struct RowIn {
  T ex1, ez1, ey, eza, bx, by, bz, bza, jx, jy, jz;
};

// One wavefront: strip `strip`, output rows [y0, y1).  All 64 lanes run every
// iteration (the shuffles need them); only the lanes and rows owned are written.
template <typename T>
__device__ __forceinline__ void fused_segment_2d(const Grid<T> &g, const Fields<T> &F, const Fields<T> &D,
                                                 int4 jbox, int strip, int y0, int y1, bool fuse_alpha,
                                                 int lane) {
  const int M0 = g.M[0], M1 = g.M[1];
  const int i = strip * FW - 1 + lane;
  const bool colok = i >= -G && i <= M0 + G;
  const bool own = lane >= 1 && lane <= FW && i <= M0;
  const int ti = min(max(i, -G), M0 + G);
  XTab<T> X;
  load_tabs(g, 0, ti, X.ehC, X.ghkC, X.sigC, X.eN, X.gN, X.gkN, X.sigN, X.aC, X.aN);
  // update extents along x (0 <= i <= M0 - 1 or M0) per component
  const bool xi0 = i >= 0 && i <= M0, xi1 = i >= 0 && i <= M0 - 1, xe = i >= 1 && i <= M0 - 1;
  // 32-bit sample offsets from the arrays' (uniform) base pointers
  const int q0 = (int)(g.base + i), sy = (int)g.sy;
  auto ld = [&](const T *a, int j) -> T { return colok ? gptr(a)[q0 + j * sy] : T(0); };
  auto bsplit = [&](const YTab<T> &Y) { return X.sigC + Y.sigC > T(0); };
  auto esplit = [&](const YTab<T> &Y) { return X.sigN + Y.sigN > T(0); };
  auto ytab = [&](int j, YTab<T> &Y) {
    load_tabs(g, 1, min(max(j, -G), M1 + G), Y.ehC, Y.ghkC, Y.sigC, Y.eN, Y.gN, Y.gkN, Y.sigN, Y.aC, Y.aN);
  };
  const int jb0 = jbox.x, jb1 = jbox.y, jb2 = jbox.z, jb3 = jbox.w;   // wave-uniform
  const bool jcol = i >= jb0 && i <= jb1;
  auto fetch = [&](int j, const YTab<T> &Y, RowIn<T> &r) {
    r.ex1 = ld(F.E[0], j + 1);
    r.ez1 = ld(F.E[2], j + 1);
    r.ey = ld(F.E[1], j);
    r.eza = esplit(Y) ? ld(F.Ea[2], j) : T(0);
    r.bx = ld(F.B[0], j);
    r.by = ld(F.B[1], j);
    r.bz = ld(F.B[2], j);
    r.bza = bsplit(Y) ? ld(F.Ba[2], j) : T(0);
    const bool need_j = j >= y0 && jcol && j >= jb2 && j <= jb3;
    r.jx = need_j ? ld(F.J[0], j) : T(0);
    r.jy = need_j ? ld(F.J[1], j) : T(0);
    r.jz = need_j ? ld(F.J[2], j) : T(0);
  };

  YTab<T> Yp, Yc, Yn;   // tables of rows j-1, j, j+1
  int j = y0 - 1;
  ytab(j, Yc);
  ERow<T> ec;           // E^n at row j
  ec.x = ld(F.E[0], j);
  ec.z = ld(F.E[2], j);
  RowIn<T> cur, nxt;
  fetch(j, Yc, cur);
  BRow<T> bhp;          // B^{n+1/2} at row j-1
  ERow<T> enp;          // E^{n+1} at row j-1
  bhp.x = bhp.y = bhp.z = bhp.za = T(0);
  enp.x = enp.y = enp.z = enp.za = T(0);
  for (; j <= y1; ++j) {
    // next row's loads go out before this row's arithmetic
    ytab(j + 1, Yn);
    if (j < y1) fetch(j + 1, Yn, nxt);
    ec.y = cur.ey;
    ec.za = cur.eza;
    // B^{n+1/2}(j)
    BRow<T> bh;
    bh.x = cur.bx;
    bh.y = cur.by;
    bh.z = cur.bz;
    bh.za = cur.bza;
    const bool byj = j >= 0 && j <= M1, byj1 = j >= 0 && j <= M1 - 1;
    {
      const T ez_r = __shfl_down(ec.z, 1), ey_r = __shfl_down(ec.y, 1);
      bhalf_2d(bh, X, Yc, xi0 && byj1, xi1 && byj, xi1 && byj1, cur.ez1 - ec.z, ez_r - ec.z, ey_r - ec.y,
               cur.ex1 - ec.x);
    }
    ERow<T> en = ec;   // E^{n+1}(j)
    const T bz_l = __shfl_up(bh.z, 1), by_l = __shfl_up(bh.y, 1);
    if (j >= y0) {
      const bool eyj = j >= 1 && j <= M1 - 1;
      estep_2d(en, X, Yc, xi1 && eyj, xe && byj1, xe && eyj, bh.z - bhp.z, bh.z - bz_l, bh.y - by_l, bh.x - bhp.x,
               cur.jx, cur.jy, cur.jz, fuse_alpha, g.dt);
      if (own && j < y1) {
        const int q = q0 + j * sy;
        gptr(D.E[0])[q] = en.x;
        gptr(D.E[1])[q] = en.y;
        gptr(D.E[2])[q] = en.z;
        if (esplit(Yc)) gptr(D.Ea[2])[q] = en.za;
      }
    }
    // B^{n+1}(j-1) from B^{n+1/2}(j-1) and E^{n+1} at rows j-1, j
    const T pz_r = __shfl_down(enp.z, 1), py_r = __shfl_down(enp.y, 1);
    if (j >= y0 + 1) {
      const int jm = j - 1;
      BRow<T> b = bhp;
      const bool bm0 = jm <= M1, bm1 = jm <= M1 - 1;   // jm >= y0 >= 0
      bhalf_2d(b, X, Yp, xi0 && bm1, xi1 && bm0, xi1 && bm1, en.z - enp.z, pz_r - enp.z, py_r - enp.y,
               en.x - enp.x);
      if (own) {
        const int q = q0 + jm * sy;
        gptr(D.B[0])[q] = b.x;
        gptr(D.B[1])[q] = b.y;
        gptr(D.B[2])[q] = b.z;
        if (bsplit(Yp)) gptr(D.Ba[2])[q] = b.za;
      }
    }
    // advance one row
    bhp = bh;
    enp = en;
    Yp = Yc;
    Yc = Yn;
    ec.x = cur.ex1;
    ec.z = cur.ez1;
    cur = nxt;
  }
}

}  // namespace pmlpic
