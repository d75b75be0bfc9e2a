// gather_push + deposit_current for 3D runs with the linear shape, one workgroup per chunk of
// a sort tile.
//
// The step is the one of particles.hip (gather of the total fields, Eq. MaxwellSum;
// relativistic Boris; move; Esirkepov's charge-conserving current, used in App. A).  One
// workgroup takes one work item: a chunk of up to tw.chunk particles of one sort tile
// (tile[0] x tile[1] x tile[2] cells; a tile at one particle per cell is one item; tiles of a
// dense beam go to the replicated-box kernel of particles.hip), accumulates their current in an LDS box of the nodes (tile + 3 per
// axis) that particles in the tile or one cell beyond it can reach, and adds the box's
// non-zero entries to J with global atomics.  A move that stays in its cell along every axis (the thermal
// background: about 96%) takes a 12-value form of Esirkepov's current; moves across a cell
// face are queued in LDS and deposited after the loop with the general window, so that
// wavefronts do not run both forms side by side; a move that leaves the tile's one-cell
// margin (a particle that drifted since the last sort) deposits straight to J.
#include "particle_core.h"

namespace pmlpic {

constexpr int P3_TPB = 256;
constexpr int P3_NODES = 1344;   // LDS nodes per current component (FP64): 11^3 for 8^3 tiles
constexpr int P3_QCAP = 128;     // moves that cross a cell face, queued per workgroup

// Esirkepov's current of a linear-shape move that stays in its cell along every axis: J_a
// is non-zero only on the half node of that cell along a, times the four nodes of the cell
// across; with d = f1_a - f0_a and the two shapes S0 = (1 - f0, f0), S1 = (1 - f1, f1) on
// the cell's two nodes along the transverse axes b, c,
//   J_a = qw jcoef_a d [S0_b (2 S0_c + S1_c) + S1_b (S0_c + 2 S1_c)] / 6,
// which is Esirkepov's W_a = dS_a (S0_b S0_c / 3 + S1_b S0_c / 6 + S0_b S1_c / 6 + S1_b S1_c / 3)
// on the two-node window (twelve values instead of the 3 x 9 x 2 of the general window).
template <typename T>
__device__ __forceinline__ void deposit_incell_linear3(const Grid<T> &g, double *box, int q0, const int (&st)[3],
                                                       int total, const T (&f0)[3], const T (&f1)[3], T qw) {
#pragma unroll
  for (int A = 0; A < 3; ++A) {
    const int Bx = (A + 1) % 3, Cx = (A + 2) % 3;
    const T d = f1[A] - f0[A];
    if (d == T(0)) continue;
    const T coef = qw * g.jcoef[A] * d * T(1.0 / 6.0);
    const T b0[2] = {T(1) - f0[Bx], f0[Bx]}, b1[2] = {T(1) - f1[Bx], f1[Bx]};
    const T c0[2] = {T(1) - f0[Cx], f0[Cx]}, c1[2] = {T(1) - f1[Cx], f1[Cx]};
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const T u = T(2) * c0[c] + c1[c], v = c0[c] + T(2) * c1[c];
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const T val = coef * (b0[b] * u + b1[b] * v);
        const int q = q0 + b * st[Bx] + c * st[Cx];
#ifdef PMLPIC_CHECK
        if (q < 0 || q >= total) { check_failed(g.check, CHECK_LDS_BOX); continue; }
#endif
        atomicAdd(&box[A * total + q], (double)val);
      }
    }
  }
}

// The gather of the linear shape (the same products in the same order as gather_comp) with
// 32-bit byte offsets from each array's base: the loads take the base from scalar registers
// and one 32-bit offset per lane, and the six components' stencils differ from the node one
// by the staggered shift along each axis.  For arrays of fewer than 2^32 bytes.  In FP64 it
// takes the 3D beam's push from 1.76 to 1.28 ms (the 64-bit address arithmetic held the
// kernel at its register limit); FP32 keeps the 64-bit form (0.7% faster there).
template <typename T, int MASK>
__device__ __forceinline__ T gather_comp_off32(const T *arr, const Shape3<1, T> &S, uint32_t q0, uint32_t sy,
                                               uint32_t sz) {
  constexpr bool hx = MASK & 1, hy = MASK & 2, hz = MASK & 4;
  const auto *bp = (const __attribute__((address_space(1))) char *)gptr(arr);
  T v[2][2][2];
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const auto *rp = (const __attribute__((address_space(1))) T *)(bp + (size_t)((q0 + c * sz + b * sy) * (uint32_t)sizeof(T)));
      v[c][b][0] = rp[0];
      v[c][b][1] = rp[1];
    }
  T acc = T(0);
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    T pl = T(0);
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      T row = T(0);
#pragma unroll
      for (int a = 0; a < 2; ++a) row += (hx ? S.wc[0][a] : S.wn[0][a]) * v[c][b][a];
      pl += (hy ? S.wc[1][b] : S.wn[1][b]) * row;
    }
    acc += (hz ? S.wc[2][c] : S.wn[2][c]) * pl;
  }
  return acc;
}
template <typename T>
__device__ __forceinline__ void gather_linear3_off32(const Grid<T> &g, const Fields<T> &F, const int (&id)[3],
                                                     const T (&f)[3], T (&EB)[6]) {
  Shape3<1, T> S;
  shape_all<T, 3, 1>(id, f, S);
  // (indices wrap modulo 2^32 through the guard cells' negative coordinates and come back
  // into [0, nelem))
  const uint32_t sy = (uint32_t)g.sy, sz = (uint32_t)g.sz;
  const uint32_t qn = (uint32_t)g.base + (uint32_t)S.sn[0] + (uint32_t)S.sn[1] * sy + (uint32_t)S.sn[2] * sz;
  const uint32_t dx = (uint32_t)(S.sc[0] - S.sn[0]), dy = (uint32_t)(S.sc[1] - S.sn[1]) * sy,
                 dz = (uint32_t)(S.sc[2] - S.sn[2]) * sz;
#ifdef PMLPIC_CHECK
  const uint32_t qs[6] = {qn + dx, qn + dy, qn + dz, qn + dy + dz, qn + dx + dz, qn + dx + dy};
  for (int a = 0; a < 6; ++a)
    if ((long)qs[a] + (long)sz + (long)sy + 1 >= g.nelem) check_failed(g.check, CHECK_SAMPLE);
#endif
  EB[0] = gather_comp_off32<T, 1>(F.E[0], S, qn + dx, sy, sz);
  EB[1] = gather_comp_off32<T, 2>(F.E[1], S, qn + dy, sy, sz);
  EB[2] = gather_comp_off32<T, 4>(F.E[2], S, qn + dz, sy, sz);
  EB[3] = gather_comp_off32<T, 6>(F.B[0], S, qn + dy + dz, sy, sz);
  EB[4] = gather_comp_off32<T, 5>(F.B[1], S, qn + dx + dz, sy, sz);
  EB[5] = gather_comp_off32<T, 3>(F.B[2], S, qn + dx + dy, sy, sz);
}

// Wavefronts per SIMD the compiler must leave room for: FP64 registers otherwise grow past
// 128 and drop the kernel to 3 wavefronts (measured 2.34 against 1.94 ms on the 3D beam);
// FP32 is left to the compiler (asked for 4 it trades scheduling for registers: 1.44
// against 1.11 ms)
template <typename T> struct P3Occ { static constexpr int MIN_WAVES = 1; };
template <> struct P3Occ<double> { static constexpr int MIN_WAVES = 4; };

// Workgroup b takes work item b of the list built after the sort (with tw.sel == 2, of the
// part listing the tiles that are not dense: their full chunks, then their partial ones in
// tile order, x fastest; at one particle per cell every tile is one partial chunk and
// neighbouring workgroups take neighbouring tiles, sharing the cache lines of their fields
// and currents).  TS > 0: cubic tiles of TS cells known at compile time (the box
// strides become immediates); 0: the tile shape of tw.  OFF32: the gather with 32-bit
// offsets (field arrays of fewer than 2^32 bytes).
template <typename T, int TS, bool OFF32>
__global__ void __launch_bounds__(P3_TPB) __attribute__((amdgpu_waves_per_eu(P3Occ<T>::MIN_WAVES))) k_push3d_tiles(Grid<T> g, Fields<T> F, Parts<T> P, StepCtl ctl, TileWork tw,
                                                         int push) {
  __shared__ double box[3 * P3_NODES];
  __shared__ unsigned int n_pushed;
  // Moves that cross a cell face (or leave the box: q_glob) take the general Esirkepov
  // window; a few percent of the thermal particles do, so almost every wavefront would run
  // both forms side by side.  They are queued here and deposited together after the loop
  // (beyond the capacity, in place).
  __shared__ int q_n;
  __shared__ uint32_t q_c0[P3_QCAP], q_c1[P3_QCAP];
  __shared__ T q_f0[3][P3_QCAP], q_f1[3][P3_QCAP], q_qw[P3_QCAP];
  __shared__ unsigned char q_glob[P3_QCAP];
  const int tid = threadIdx.x;
  // the items of the last sort (particles injected since then form an unsorted tail pushed
  // by another kernel); the grid is an upper bound of their number.  With tw.sel == 2 only
  // the chunks of tiles that are not dense (dense tiles go to the kernel of particles.hip,
  // whose replicated LDS box fits the chunk instead of the tile: a dense beam's lanes would
  // otherwise meet on a few nodes of the tile box)
  const unsigned first = tw.sel == 2 ? tw.dprefix[tw.ntiles] : 0u;
  if (first + blockIdx.x >= tw.dprefix[tw.ntiles] + tw.prefix[tw.ntiles] + tw.pprefix[tw.ntiles]) return;
  const int4 item = tw.items[first + blockIdx.x];
  const int t = item.z;
  const int tc[3] = {t % tw.ntile[0], (t / tw.ntile[0]) % tw.ntile[1], t / (tw.ntile[0] * tw.ntile[1])};
  const uint32_t s = (uint32_t)item.x, e = (uint32_t)item.y;
  if (e <= s) return;   // whole workgroup (the work list holds no empty item)
  // cells [T0, T0 + tile) of the tile; particles in [T0 - 1, T0 + tile] at both ends of their
  // move deposit into the box of nodes [T0 - 1, T0 + tile + 1]
  int T0[3], ext[3], st[3], tl[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    tl[d] = TS > 0 ? TS : tw.tile[d];
    T0[d] = tc[d] * tl[d];
    ext[d] = tl[d] + 3;
  }
  st[0] = 1;
  st[1] = ext[0];
  st[2] = ext[0] * ext[1];
  const int total = st[2] * ext[2];
  // the first particle's state is requested before the box is cleared, the next one's
  // while the current one is processed
  struct PState {
    uint32_t c;
    T f[3], u[3], w;
  };
  auto load = [&](uint32_t p, PState &q) {
    q.c = P.cell[p];
#pragma unroll
    for (int d = 0; d < 3; ++d) { q.f[d] = P.f[d][p]; q.u[d] = P.u[d][p]; }
    q.w = P.w[p];
  };
  // (a slot past the item reads the item's last particle, unused: the same loads on every
  // path, which the wave then leaves in flight through the current particle's work)
  PState cur;
  uint32_t p = s + (uint32_t)tid;
  load(min(p, e - 1), cur);
  for (int q = tid; q < 3 * total; q += P3_TPB) box[q] = 0.0;
  if (tid == 0) { n_pushed = 0u; q_n = 0; }
  __syncthreads();
  LdsSink<T> lsink;
  lsink.lds = box;
  lsink.e0 = ext[0];
  lsink.e01 = st[2];
  lsink.total = total;
#pragma unroll
  for (int d = 0; d < 3; ++d) lsink.lo[d] = T0[d] - 1;
  unsigned int my_pushes = 0u;
  for (; p < e; p += P3_TPB) {
    // a removed particle (kept until the next sort drops it) runs the same code on a cell of
    // the tile, deposits nothing and is written back unchanged: every path issues the same
    // loads and stores, so the wave waits only for what it uses
    const bool live = cur.c != DEAD;
    const uint32_t c = live ? cur.c : pack_cell(3, T0[0], T0[1], T0[2]);
    my_pushes += live ? 1u : 0u;
    int id[3];
    unpack_cell(3, c, id[0], id[1], id[2]);
    T f[3] = {cur.f[0], cur.f[1], cur.f[2]};
    T u[3] = {cur.u[0], cur.u[1], cur.u[2]};
    if (push) {
      T EB[6];
      if constexpr (OFF32) gather_linear3_off32<T>(g, F, id, f, EB);
      else gather<T, 3, 1>(g, F, id, f, EB);
      boris(g.qdt_2m, EB, u);
    }
    // the next particle's state is requested after the gather's loads, not before them: the
    // wave's wait for the stencil then leaves it in flight (load counts complete in order),
    // and it arrives while this particle moves and deposits
    __builtin_amdgcn_sched_barrier(0);
    PState nxt;
    load(min(p + P3_TPB, e - 1), nxt);
    __builtin_amdgcn_sched_barrier(0);
    const int id0[3] = {id[0], id[1], id[2]};
    const T f0[3] = {f[0], f[1], f[2]};
    T ig;
    const bool inside = move<T, 3>(g, id, f, u, ig);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      P.u[d][p] = live ? u[d] : cur.u[d];
      P.f[d][p] = live ? f[d] : cur.f[d];
    }
    T qw = deposit_charge_w<T, 3>(g, P, p, cur.w, id0, f0, id, f);
    if (!live) qw = T(0);
    cur = nxt;
    bool inbox = true, incell = true;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const int lo = T0[d] - 1, hi = T0[d] + tl[d];
      inbox = inbox && id0[d] >= lo && id0[d] <= hi && id[d] >= lo && id[d] <= hi;
      incell = incell && id[d] == id0[d];
    }
    if (live && inbox && incell) {
      const int q0 = (id0[0] - lsink.lo[0]) + (id0[1] - lsink.lo[1]) * st[1] + (id0[2] - lsink.lo[2]) * st[2];
      deposit_incell_linear3<T>(g, box, q0, st, total, f0, f, qw);
    }
    const bool queued = live && !(inbox && incell);
    const unsigned long long mq = __ballot(queued);
    if (queued) {
      const int lane = tid & 63;
      const int leader = __ffsll((long long)mq) - 1;
      int base = 0;
      if (lane == leader) base = atomicAdd(&q_n, __popcll(mq));
      base = __shfl(base, leader);
      const int k = base + __popcll(mq & ((1ull << lane) - 1ull));
      if (k < P3_QCAP) {
        q_c0[k] = c;
        q_c1[k] = pack_cell(3, id[0], id[1], id[2]);
#pragma unroll
        for (int d = 0; d < 3; ++d) { q_f0[d][k] = f0[d]; q_f1[d][k] = f[d]; }
        q_qw[k] = qw;
        q_glob[k] = inbox ? 0 : 1;
      } else if (inbox) {
        deposit<T, 3, 1>(g, lsink, id0, f0, id, f, T(0), qw);
      } else {
        GlobalSink<T> gsink{{F.J[0], F.J[1], F.J[2]}, 0, 0, 0};
        deposit<T, 3, 1>(g, gsink, id0, f0, id, f, T(0), qw);
      }
    }
    P.cell[p] = live && inside ? pack_cell(3, id[0], id[1], id[2]) : DEAD;
  }
  __syncthreads();
  {   // the queued moves
    const int nq = min(q_n, P3_QCAP);
    for (int k = tid; k < nq; k += P3_TPB) {
      int i0[3], i1[3];
      unpack_cell(3, q_c0[k], i0[0], i0[1], i0[2]);
      unpack_cell(3, q_c1[k], i1[0], i1[1], i1[2]);
      const T f0[3] = {q_f0[0][k], q_f0[1][k], q_f0[2][k]};
      const T f1[3] = {q_f1[0][k], q_f1[1][k], q_f1[2][k]};
      if (q_glob[k]) {
        GlobalSink<T> gsink{{F.J[0], F.J[1], F.J[2]}, 0, 0, 0};
        deposit<T, 3, 1>(g, gsink, i0, f0, i1, f1, T(0), q_qw[k]);
      } else {
        deposit<T, 3, 1>(g, lsink, i0, f0, i1, f1, T(0), q_qw[k]);
      }
    }
  }
  // push tally: wavefront sums, then one atomic per workgroup
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) my_pushes += __shfl_xor(my_pushes, off);
  if ((tid & 63) == 0 && my_pushes) atomicAdd(&n_pushed, my_pushes);
  __syncthreads();
  if (tid == 0 && n_pushed) atomicAdd(&ctl.pushes[blockIdx.x % N_PUSH_COUNTERS], (unsigned long long)n_pushed);
  // flush: every non-zero entry of the box to J with one global atomic add; entry
  // q = ((comp ext2 + k) ext1 + j) ext0 + i, divided by multiply-shift (exact for q < 2^12)
  const uint32_t m0 = (1u << 20) / (uint32_t)ext[0] + 1u, m1 = (1u << 20) / (uint32_t)ext[1] + 1u,
                 m2 = (1u << 20) / (uint32_t)ext[2] + 1u;
  // (offsets from the box origin in 32 bits: push3d_applies admits a box only if it spans
  // less than 2^32 samples of the grid)
  const long qlo = g.at(lsink.lo[0], lsink.lo[1], lsink.lo[2]);
  const uint32_t sy = (uint32_t)g.sy, sz = (uint32_t)g.sz;
  for (int q = tid; q < 3 * total; q += P3_TPB) {
    const double v = box[q];
    if (v == 0.0) continue;
    const uint32_t uq = (uint32_t)q;
    const uint32_t r1 = (uq * m0) >> 20, i = uq - r1 * (uint32_t)ext[0];
    const uint32_t r2 = (r1 * m1) >> 20, j = r1 - r2 * (uint32_t)ext[1];
    const uint32_t comp = (r2 * m2) >> 20, k = r2 - comp * (uint32_t)ext[2];
#ifdef PMLPIC_CHECK
    const long qn = g.at(lsink.lo[0] + (int)i, lsink.lo[1] + (int)j, lsink.lo[2] + (int)k);
#else
    const long qn = qlo + (long)(i + j * sy + k * sz);
#endif
    atomic_add(pick3(F.J, (int)comp) + qn, (T)v);
  }
}

bool push3d_applies(int dim, int order, const int tile[3], long plane) {
  if (dim != 3 || order != 1) return false;
  long vol = 1;
  for (int d = 0; d < 3; ++d) {
    if (tile[d] < 3) return false;
    vol *= tile[d] + 3;
  }
  return vol <= P3_NODES && (tile[2] + 3) * plane < (1L << 32);
}

template <typename T>
void launch_push3d(const Grid<T> &g, const Fields<T> &F, const Parts<T> &P, StepCtl ctl, const TileWork &tw,
                   int n_slots, int push, hipStream_t s) {
  if (tw.ntiles <= 0 || n_slots <= 0) return;
  // items: at most one partial chunk per tile, plus the full chunks of the slots
  const unsigned nb = (unsigned)(tw.ntiles + (n_slots + tw.chunk - 1) / tw.chunk);
  const bool cube8 = tw.tile[0] == 8 && tw.tile[1] == 8 && tw.tile[2] == 8;
  if constexpr (sizeof(T) == 8) {
    if (g.nelem * (long)sizeof(T) < (1L << 32)) {
      if (cube8) hipLaunchKernelGGL((k_push3d_tiles<T, 8, true>), dim3(nb), dim3(P3_TPB), 0, s, g, F, P, ctl, tw, push);
      else hipLaunchKernelGGL((k_push3d_tiles<T, 0, true>), dim3(nb), dim3(P3_TPB), 0, s, g, F, P, ctl, tw, push);
      return;
    }
  }
  if (cube8) {
    hipLaunchKernelGGL((k_push3d_tiles<T, 8, false>), dim3(nb), dim3(P3_TPB), 0, s, g, F, P, ctl, tw, push);
  } else {
    hipLaunchKernelGGL((k_push3d_tiles<T, 0, false>), dim3(nb), dim3(P3_TPB), 0, s, g, F, P, ctl, tw, push);
  }
}

template void launch_push3d<float>(const Grid<float> &, const Fields<float> &, const Parts<float> &, StepCtl,
                                   const TileWork &, int, int, hipStream_t);
template void launch_push3d<double>(const Grid<double> &, const Fields<double> &, const Parts<double> &, StepCtl,
                                    const TileWork &, int, int, hipStream_t);

}  // namespace pmlpic
