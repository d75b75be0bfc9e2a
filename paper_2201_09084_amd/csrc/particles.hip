// gather_push, deposit_current and sort_particles.
//
// gather_push: the six total field components (sum of the split parts, Eq. MaxwellSum)
// are interpolated at the particle with the same-order B-spline at each component's
// staggered Yee position, then the relativistic Boris rotation advances u = gamma v,
// and the particle moves by dt u/gamma.  Positions are an integer cell per axis plus
// an offset in [0,1); the offset is re-based when it leaves [0,1).
//
// deposit_current: Esirkepov's charge-conserving scheme (used in App. A) for the move
// x^n -> x^{n+1} on the (order+2)-node window that covers both shapes; the running
// sums along each axis give J at E's staggered samples.  Accumulated with hardware
// float atomics (order-nondeterministic).  Particles that end outside the PEC box
// deposit this step and are then marked DEAD.
//
// The fused kernel does both for one particle in registers, so x^n and x^{n+1} are
// exactly the stored positions of consecutive steps (exact discrete continuity).
#include <algorithm>

#include "particle_core.h"

namespace pmlpic {

// fused (fused = true) or first half (fused = false) of the particle step, one thread
// per particle slot
template <typename T, int DIM, int ORDER>
__global__ void __launch_bounds__(256) k_gather_push(Grid<T> g, Fields<T> F, Parts<T> P, Parts<T> old,
                                                      StepCtl ctl, int n_slots, int push, bool fused,
                                                      const int32_t *start) {
  const int p = (start ? *start : 0) + (int)(blockIdx.x * blockDim.x + threadIdx.x);
  const int count = *ctl.count;
  bool active = false;
  int rng[4] = {0, -1, 0, -1};
  if (p < n_slots && p < count) active = push_one<T, DIM, ORDER>(g, F, P, old, p, push, fused, rng);
  count_pushes(ctl.pushes, active);
  if (DIM == 2 && fused && ctl.jslot) {
    const int4 b = block_box(rng[0], rng[1], rng[2], rng[3]);
    if (threadIdx.x == 0) jslot_merge(ctl.jslot, b.x, b.y, b.z, b.w);
  }
}

constexpr int TPB = 256;
// LDS nodes per current component (FP64 sums) and particles per thread.  2D: 36 KB,
// replicas of small boxes for dense beams.  3D: the 11^3-node box of one 8^3 tile with
// the linear-shape window (32 KB; a larger box costs more in occupancy than it gains).
template <int DIM> struct TileCfg;
template <> struct TileCfg<2> { static constexpr int NODES = 1536; static constexpr int PPT = 4; };
template <> struct TileCfg<3> { static constexpr int NODES = 1344; static constexpr int PPT = 4; };

// Fused gather_push + deposit_current over chunks of cell-sorted particles.  A
// workgroup takes one work item: a chunk of one sort tile (by_tile, 3D: the chunk's
// particles all belong to one tile) or a range of the sorted array (2D).  It
// accumulates Esirkepov's current in an LDS box, replicated R times with an odd
// stride so that lanes that share a node meet in different words and banks, and then
// adds every non-zero entry to global J once (distinct consecutive addresses).  The
// box is the bounding box of the chunk's old cells plus the deposit window; for a
// tile item whose particles spread since the sort, it may instead be that box
// clipped to the tile grown by `margin` cells per side (when the whole box does not
// fit, or when clipping buys more replicas at the cost of at most 1/16 of the chunk),
// and particles outside it deposit straight to global J.  A workgroup takes items
// blockIdx.x, blockIdx.x + gridDim.x, ...: one item when the grid covers the list, several
// when a short grid walks a list of unknown length (the dense tiles' chunks).
template <typename T, int DIM, int ORDER, int PPT, bool BY_TILE>
__global__ void __launch_bounds__(TPB) k_push_deposit_tiles(Grid<T> g, Fields<T> F, Parts<T> P, StepCtl ctl,
                                                            JClear<T> jc, TileWork tw, int push) {
  constexpr int WLO = ORDER == 1 ? -1 : -2;
  constexpr int WHI = ORDER == 1 ? 2 : 3;
  constexpr int NODES = TileCfg<DIM>::NODES;
  __shared__ double lds[3 * NODES];
  __shared__ int sbox[12];   // min[3], max[3] of the old cells; then the same clipped
  __shared__ unsigned int n_pushed, n_out;
  const int tid = threadIdx.x;
  if (DIM == 2 && jc.prev) jclear_share(g, jc);   // the other current buffer (a different array)
  // by tile: the items of the tiles; else the 2D list (heavy pieces last).  Uniform.
  // (Giving each XCD a contiguous eighth of the 3D list cut the fetched bytes by 3x
  // but ran 5% slower: the order below spreads the work of every region over all XCDs.)
  // (tw.sel == 1: the chunks of the dense tiles only, listed first)
  const unsigned n_items =
      BY_TILE ? tw.dprefix[tw.ntiles] + (tw.sel == 1 ? 0u : tw.prefix[tw.ntiles] + tw.pprefix[tw.ntiles])
              : *tw.n_items;
  for (unsigned it = blockIdx.x; it < n_items; it += gridDim.x) {
    int p0, p1, t = -1;
    {
      const int4 item = tw.items[it];
      p0 = __builtin_amdgcn_readfirstlane(item.x);
      p1 = __builtin_amdgcn_readfirstlane(item.y);
      if (BY_TILE) t = __builtin_amdgcn_readfirstlane(item.z);
    }
    if (p0 >= p1) continue;
    int clo[3] = {-0x3FFFFFFF, -0x3FFFFFFF, -0x3FFFFFFF}, chi[3] = {0x3FFFFFFF, 0x3FFFFFFF, 0x3FFFFFFF};
    if (t >= 0) {   // old cells of the tile grown by the margin
      const int tc[3] = {t % tw.ntile[0], (t / tw.ntile[0]) % tw.ntile[1], t / (tw.ntile[0] * tw.ntile[1])};
#pragma unroll
      for (int d = 0; d < DIM; ++d) {
        clo[d] = tc[d] * tw.tile[d] - tw.margin;
        chi[d] = tc[d] * tw.tile[d] + tw.tile[d] - 1 + tw.margin;
      }
    }
    if (tid == 0) { n_pushed = 0u; n_out = 0u; }
    if (tid < 3) {
      sbox[tid] = 0x7FFFFFFF; sbox[3 + tid] = -0x7FFFFFFF;
      sbox[6 + tid] = 0x7FFFFFFF; sbox[9 + tid] = -0x7FFFFFFF;
    }
    __syncthreads();
    int mn[6] = {0x7FFFFFFF, 0x7FFFFFFF, 0x7FFFFFFF, 0x7FFFFFFF, 0x7FFFFFFF, 0x7FFFFFFF};
    int mx[6] = {-0x7FFFFFFF, -0x7FFFFFFF, -0x7FFFFFFF, -0x7FFFFFFF, -0x7FFFFFFF, -0x7FFFFFFF};
    unsigned int out = 0u;
    // the cells of my particles requested together (a slot past the item reads its last one,
    // unused): one memory round trip, not one per particle
    uint32_t cs[PPT];
#pragma unroll
    for (int k = 0; k < PPT; ++k) cs[k] = P.cell[min(p0 + k * TPB + tid, p1 - 1)];
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
      const int p = p0 + k * TPB + tid;
      if (p < p1) {
        const uint32_t c = cs[k];
        if (c != DEAD) {
          int id[3];
          unpack_cell(DIM, c, id[0], id[1], id[2]);
          bool in = true;
#pragma unroll
          for (int d = 0; d < DIM; ++d) {
            mn[d] = min(mn[d], id[d]);
            mx[d] = max(mx[d], id[d]);
            if constexpr (BY_TILE) {
              const int v = min(max(id[d], clo[d]), chi[d]);
              in = in && v == id[d];
              mn[3 + d] = min(mn[3 + d], v);
              mx[3 + d] = max(mx[3 + d], v);
            }
          }
          out += in ? 0u : 1u;
        }
      }
    }
    // reduce over the wavefront first: 256 lanes updating the same few LDS words
    // serialise (measured: 8-17 us per workgroup in the dense 2D beam)
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
      for (int d = 0; d < DIM; ++d) {
        mn[d] = min(mn[d], __shfl_xor(mn[d], off));
        mx[d] = max(mx[d], __shfl_xor(mx[d], off));
        if constexpr (BY_TILE) {
          mn[3 + d] = min(mn[3 + d], __shfl_xor(mn[3 + d], off));
          mx[3 + d] = max(mx[3 + d], __shfl_xor(mx[3 + d], off));
        }
      }
      if constexpr (BY_TILE) out += __shfl_xor(out, off);
    }
    if ((tid & 63) == 0) {
#pragma unroll
      for (int d = 0; d < DIM; ++d) {
        if (mn[d] <= mx[d]) {
          atomicMin(&sbox[d], mn[d]); atomicMax(&sbox[3 + d], mx[d]);
          if constexpr (BY_TILE) { atomicMin(&sbox[6 + d], mn[3 + d]); atomicMax(&sbox[9 + d], mx[3 + d]); }
        }
      }
      if (BY_TILE && out) atomicAdd(&n_out, out);
    }
    __syncthreads();
    int sb[12];   // the box words, wave-uniform (scalar registers)
#pragma unroll
    for (int k = 0; k < 12; ++k) sb[k] = __builtin_amdgcn_readfirstlane(sbox[k]);
    if (DIM == 2 && ctl.jslot && tid == 0 && sb[0] <= sb[3])   // nodes this chunk can deposit to
      jslot_merge(ctl.jslot, sb[0] + WLO, sb[3] + WHI, sb[1] + WLO, sb[4] + WHI);
    LdsSink<T> lsink;
    const bool any = sb[0] <= sb[3];
    // replicas that fit for a box of n nodes per component (0: does not fit)
    auto reps = [&](long n) {
      const long st = (3 * n) | 1;
      int r = 0;
      while (r < 16 && (r ? 2 * r : 1) * st <= 3 * NODES) r = r ? 2 * r : 1;
      return r;
    };
    int o = 0;   // 0: whole bounding box; 6: clipped box, particles outside it go global
    if (BY_TILE && any) {
      long full = 1, clip = 1;
#pragma unroll
      for (int d = 0; d < DIM; ++d) {
        full *= sb[3 + d] - sb[d] + (WHI - WLO) + 1;
        clip *= sb[9 + d] - sb[6 + d] + (WHI - WLO) + 1;
      }
      const int rf = reps(full), rc = reps(clip);
      const unsigned nout = __builtin_amdgcn_readfirstlane(n_out);
      // the clipped box wins if the whole one does not fit, or if it allows more
      // replicas at the price of at most 1/16 of the chunk going to global memory
      if (rf == 0 || (rc > rf && 16u * nout <= (unsigned)(p1 - p0))) o = 6;
    }
    int ext[3] = {1, 1, 1}, bmn[3] = {0, 0, 0}, bmx[3] = {0, 0, 0};
    long total = 1;   // 64-bit: the box of a sparse range can exceed 2^31 nodes
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      if (d < DIM) {
        bmn[d] = o ? sb[6 + d] : sb[d];
        bmx[d] = o ? sb[9 + d] : sb[3 + d];
        lsink.lo[d] = bmn[d] + WLO;
        ext[d] = any ? bmx[d] - bmn[d] + (WHI - WLO) + 1 : 1;
      } else {
        lsink.lo[d] = 0;
      }
      total *= ext[d];
    }
    const long lstride = (3 * total) | 1;
    const bool use_lds = any && lstride <= 3 * NODES;
    // past this point the box sizes are used only when the box fits in LDS (int range)
    const int stride = use_lds ? (int)lstride : 1;
    int R = 1;
    while (use_lds && R < 16 && 2 * R * stride <= 3 * NODES) R *= 2;
    lsink.e0 = ext[0];
    lsink.e01 = use_lds ? ext[0] * ext[1] : 0;
    lsink.total = use_lds ? (int)total : 0;
    if (use_lds) {
      for (int e = tid; e < R * stride; e += TPB) lds[e] = 0.0;
    }
    lsink.lds = lds + (tid % R) * stride;
    __syncthreads();
    GlobalSink<T> gsink{{F.J[0], F.J[1], F.J[2]}, 0, 0, 0};
    // a particle's state is requested one particle ahead (a slot past the item reads its last
    // one, unused), so that its round trip overlaps the gather of the one before
    struct PState {
      uint32_t c;
      T f[3], u[3], w;
    };
    auto load = [&](int p, PState &st) {
      const int pc = min(p, p1 - 1);
      st.c = P.cell[pc];
#pragma unroll
      for (int d = 0; d < 3; ++d) st.f[d] = d < DIM ? P.f[d][pc] : T(0);
#pragma unroll
      for (int d = 0; d < 3; ++d) st.u[d] = P.u[d][pc];
      st.w = P.w[pc];
    };
    PState cur;
    load(p0 + tid, cur);
#pragma unroll 1
    for (int k = 0; k < PPT; ++k) {
      const int p = p0 + k * TPB + tid;
      PState nxt;
      load(p + TPB, nxt);
      bool active = false;
      if (p < p1) {
        const uint32_t c = cur.c;
        if (c != DEAD) {
          active = true;
          int id[3];
          unpack_cell(DIM, c, id[0], id[1], id[2]);
          bool inbox = use_lds;
#pragma unroll
          for (int d = 0; d < DIM; ++d) inbox = inbox && id[d] >= bmn[d] && id[d] <= bmx[d];
          T f[3] = {cur.f[0], cur.f[1], cur.f[2]};
          T u[3] = {cur.u[0], cur.u[1], cur.u[2]};
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
          const T qw = deposit_charge_w<T, DIM>(g, P, p, cur.w, id0, f0, id, f);
          if (inbox) deposit<T, DIM, ORDER>(g, lsink, id0, f0, id, f, u[2] * ig, qw);
          else deposit<T, DIM, ORDER>(g, gsink, id0, f0, id, f, u[2] * ig, qw);
          P.cell[p] = inside ? pack_cell(DIM, id[0], id[1], id[2]) : DEAD;
        }
      }
      const unsigned long long m = __ballot(active);
      if ((tid & 63) == 0 && m) atomicAdd(&n_pushed, (unsigned int)__popcll(m));
      cur = nxt;
    }
    __syncthreads();
    if (tid == 0 && n_pushed) atomicAdd(&ctl.pushes[blockIdx.x % N_PUSH_COUNTERS], (unsigned long long)n_pushed);
    if (use_lds) {
      const int ntot = lsink.total;
      for (int e = tid; e < 3 * ntot; e += TPB) {
        double acc = lds[e];
        for (int r = 1; r < R; ++r) acc += lds[r * stride + e];
        const T v = (T)acc;
        if (v == T(0)) continue;
        const int comp = e / ntot;
        int r = e - comp * ntot;
        const int i = r % ext[0];
        r /= ext[0];
        const int j = r % ext[1];
        const int kk = r / ext[1];
        atomic_add(pick3(F.J, comp) + g.at(lsink.lo[0] + i, lsink.lo[1] + j, lsink.lo[2] + kk), v);
      }
    }
    __syncthreads();   // the next item reuses the box and the counters
  }
}

// 2D work list, built after every sort: fixed ranges of `chunk` sorted particles.  A
// range whose node box does not fit in LDS (sparse particles: its deposits go to
// global memory, about forty atomics per particle) is split into RANGE_SPLIT items, so
// that no compute unit issues all of a range's global atomics and a piece whose own box
// fits uses LDS, and those items come last: the ranges that fit take the first round
// of workgroup slots, and the pieces, short, fill slots as they free up.  (Listed
// first, the pieces held slots that whole ranges then had to wait for.  A work queue
// with an atomic counter was slower: atomics on one word from every workgroup
// serialise across the chip.  On the 2D beam 8 pieces beat 1, 2, 4 and 16.)
constexpr int RANGE_SPLIT = RANGE_SPLIT_MAX;

// per range: 1 if its box (cells at the sort plus the deposit window and the drift
// allowance: win1 nodes wider than the cell span per axis) does not fit in `nodes`
// LDS nodes per component
__global__ void k_range_classify(TileWork tw, const uint32_t *cell, const int32_t *count, int win1, int nodes) {
  const int wave = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6), lane = threadIdx.x & 63;
  const int n = *count;
  const int nch = (n + tw.chunk - 1) / tw.chunk;
  if (wave >= nch) return;   // uniform over the wavefront
  const int p0 = wave * tw.chunk, p1 = min(p0 + tw.chunk, n);
  int xl = 0x7FFFFFFF, xh = -0x7FFFFFFF, yl = 0x7FFFFFFF, yh = -0x7FFFFFFF;
  for (int p = p0 + lane; p < p1; p += 64) {
    const uint32_t c = cell[p];
    if (c == DEAD) continue;
    int i, j, k;
    unpack_cell(2, c, i, j, k);
    xl = min(xl, i); xh = max(xh, i); yl = min(yl, j); yh = max(yh, j);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    xl = min(xl, __shfl_xor(xl, off)); xh = max(xh, __shfl_xor(xh, off));
    yl = min(yl, __shfl_xor(yl, off)); yh = max(yh, __shfl_xor(yh, off));
  }
  if (lane == 0) {
    bool heavy = false;
    if (xl <= xh) {
      const long total = (long)(xh - xl + win1) * (long)(yh - yl + win1);
      heavy = ((3 * total) | 1) > 3L * nodes;   // the kernel's LDS test
    }
    tw.flags[wave] = heavy ? 1u : 0u;
  }
}

// one workgroup: the ranges that fit in order, then the heavy ones (RANGE_SPLIT items each);
// the item count goes to *n_items
constexpr int ITEMS_TPB = 1024;
__global__ void __launch_bounds__(ITEMS_TPB) k_range_items(TileWork tw, const int32_t *count) {
  __shared__ uint32_t sh[ITEMS_TPB];
  __shared__ uint32_t carry_h, carry_l;
  const int tid = threadIdx.x;
  const int n = *count;
  const int nch = (n + tw.chunk - 1) / tw.chunk;
  const int piece = (tw.chunk + RANGE_SPLIT - 1) / RANGE_SPLIT;
  uint32_t h = 0;
  for (int c = tid; c < nch; c += ITEMS_TPB) h += tw.flags[c];
  sh[tid] = h;
  __syncthreads();
  for (int off = ITEMS_TPB / 2; off > 0; off >>= 1) {
    if (tid < off) sh[tid] += sh[tid + off];
    __syncthreads();
  }
  const uint32_t n_heavy = sh[0];
  if (tid == 0) { carry_h = 0u; carry_l = 0u; }
  __syncthreads();
  for (int start = 0; start < nch; start += ITEMS_TPB) {
    const int c = start + tid;
    const uint32_t f = c < nch ? tw.flags[c] : 0u;
    const uint32_t v = c < nch ? (f ? (1u << 16) : 1u) : 0u;   // heavy count high, light low
    sh[tid] = v;
    __syncthreads();
    for (int off = 1; off < ITEMS_TPB; off <<= 1) {   // inclusive scan
      const uint32_t add = tid >= off ? sh[tid - off] : 0u;
      __syncthreads();
      sh[tid] += add;
      __syncthreads();
    }
    const uint32_t ex = sh[tid] - v;
    if (c < nch) {
      const int p0 = c * tw.chunk, p1 = min(p0 + tw.chunk, n);
      if (f) {
        const int first = (int)((uint32_t)nch - n_heavy + (carry_h + (ex >> 16)) * RANGE_SPLIT);
        for (int k = 0; k < RANGE_SPLIT; ++k) {
          const int q0 = min(p0 + k * piece, p1), q1 = min(q0 + piece, p1);
          tw.items[first + k] = make_int4(q0, q1, 0, 0);
        }
      } else {
        tw.items[carry_l + (ex & 0xFFFFu)] = make_int4(p0, p1, 0, 0);
      }
    }
    __syncthreads();
    if (tid == ITEMS_TPB - 1) { carry_h += sh[tid] >> 16; carry_l += sh[tid] & 0xFFFFu; }
    __syncthreads();
  }
  if (tid == 0) *tw.n_items = n_heavy * RANGE_SPLIT + ((uint32_t)nch - n_heavy);
}

void launch_range_items(const TileWork &tw, const uint32_t *cell, const int32_t *count, int order, int max_ranges,
                        int drift, hipStream_t s) {
  if (max_ranges <= 0) return;
  // WHI - WLO + 1 of the deposit window, plus the cells the particles may drift per
  // side before the next sort
  const int win1 = (order == 1 ? 4 : 6) + 2 * drift;
  hipLaunchKernelGGL(k_range_classify, dim3((max_ranges + 3) / 4), dim3(256), 0, s, tw, cell, count, win1,
                     TileCfg<2>::NODES);
  hipLaunchKernelGGL(k_range_items, dim3(1), dim3(ITEMS_TPB), 0, s, tw, count);
}

// chunks per tile from the sorted key ranges (count: live slots after the sort)
__device__ __forceinline__ void tile_range(const TileWork &tw, int t, const int32_t *count, uint32_t &s, uint32_t &e) {
  s = tw.key_start[(size_t)t * tw.tilecells];
  e = t + 1 < tw.ntiles ? tw.key_start[(size_t)(t + 1) * tw.tilecells] : (uint32_t)*count;
}
// A tile is dense when one of its cells holds more than DENSE_CELL particles (a beam whose
// particles crowd a few cells: lanes of a wavefront would add into the same few nodes of a
// box spanning the whole tile).  Chunks are `chunk` particles of one tile's sorted range,
// the last one partial.  The list holds the chunks of the dense tiles first (dprefix counts
// them per tile), then the full chunks of the other tiles (prefix), then the other tiles'
// last partial chunks (pprefix): long items first, the short ones finish the launch.
constexpr uint32_t DENSE_CELL = 16;
// one wavefront per tile: its cells' counts from the key starts, reduced to the largest
__global__ void __launch_bounds__(256) k_tile_chunks(TileWork tw, const int32_t *count) {
  const int t = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  const int lane = threadIdx.x & 63;
  if (t >= tw.ntiles) return;   // uniform over the wavefront
  uint32_t s, e;
  tile_range(tw, t, count, s, e);
  const uint32_t n = e > s ? e - s : 0u;
  uint32_t big = 0;
  if (n > DENSE_CELL) {   // key_start[n_keys] is the sorted count
    const size_t k0 = (size_t)t * tw.tilecells;
    for (int c = lane; c < tw.tilecells; c += 64) big = max(big, tw.key_start[k0 + c + 1] - tw.key_start[k0 + c]);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) big = max(big, (uint32_t)__shfl_xor((int)big, off));
  }
  if (lane == 0) {
    const bool dense = big > DENSE_CELL;
    const uint32_t nfull = n / tw.chunk, part = n % tw.chunk ? 1u : 0u;
    tw.dprefix[t] = dense ? nfull + part : 0u;
    tw.prefix[t] = dense ? 0u : nfull;
    tw.pprefix[t] = dense ? 0u : part;
  }
}
// one work item per chunk, after the scans
__global__ void k_tile_items(TileWork tw, const int32_t *count) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= tw.ntiles) return;
  uint32_t s, e;
  tile_range(tw, t, count, s, e);
  const uint32_t nd = tw.dprefix[tw.ntiles], nf = tw.prefix[tw.ntiles];
  if (tw.dprefix[t + 1] > tw.dprefix[t]) {   // dense: every chunk in the first section
    for (uint32_t c = 0, p = s; p < e; ++c, p += tw.chunk)
      tw.items[tw.dprefix[t] + c] = make_int4((int)p, (int)min(e, p + (uint32_t)tw.chunk), t, 0);
    return;
  }
  const uint32_t nfull = e > s ? (e - s) / tw.chunk : 0u;
  for (uint32_t c = 0; c < nfull; ++c) {
    const uint32_t p = s + c * tw.chunk;
    tw.items[nd + tw.prefix[t] + c] = make_int4((int)p, (int)(p + tw.chunk), t, 0);
  }
  const uint32_t p = s + nfull * tw.chunk;
  if (p < e) tw.items[nd + nf + tw.pprefix[t]] = make_int4((int)p, (int)e, t, 0);
}

// second half of the unfused particle step: deposit from the saved x^n to x^{n+1}
template <typename T, int DIM, int ORDER>
__global__ void __launch_bounds__(256) k_deposit(Grid<T> g, Fields<T> F, Parts<T> P, Parts<T> old,
                                                  StepCtl ctl, int n_slots) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  int rng[4] = {0, -1, 0, -1};
  const uint32_t c = (p < n_slots && p < *ctl.count) ? P.cell[p] : DEAD;
  if (c != DEAD) {
    int i1[3], i0[3];
    unpack_cell(DIM, c, i1[0], i1[1], i1[2]);
    unpack_cell(DIM, old.cell[p], i0[0], i0[1], i0[2]);
    const T f1[3] = {P.f[0][p], P.f[1][p], DIM == 3 ? P.f[2][p] : T(0)};
    const T f0[3] = {old.f[0][p], old.f[1][p], DIM == 3 ? old.f[2][p] : T(0)};
    const T ux = P.u[0][p], uy = P.u[1][p], uz = P.u[2][p];
    const T ig = T(1) / sqrt(T(1) + ux * ux + uy * uy + uz * uz);
    GlobalSink<T> sink{{F.J[0], F.J[1], F.J[2]}, 0, 0, 0};
    deposit<T, DIM, ORDER>(g, sink, i0, f0, i1, f1, uz * ig, deposit_charge<T, DIM>(g, P, p, i0, f0, i1, f1));
    dep_range<ORDER>(i0[0], i1[0], rng[0], rng[1]);
    dep_range<ORDER>(i0[1], i1[1], rng[2], rng[3]);
    bool inside = true;
#pragma unroll
    for (int d = 0; d < DIM; ++d) inside = inside && i1[d] >= 0 && i1[d] < g.M[d];
    if (!inside) P.cell[p] = DEAD;
  }
  if (DIM == 2 && ctl.jslot) {
    const int4 b = block_box(rng[0], rng[1], rng[2], rng[3]);
    if (threadIdx.x == 0) jslot_merge(ctl.jslot, b.x, b.y, b.z, b.w);
  }
}

// Deterministic debug form of the unfused deposit: one thread adds every particle's current
// in slot order with plain loads and stores (the values of k_deposit, summed in a fixed
// order, so that a run repeats bit for bit; with sorting off the slot order never changes).
template <typename T>
struct PlainSink {
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
    J[comp][q] += v;
  }
};

template <typename T, int DIM, int ORDER>
__global__ void __launch_bounds__(64) k_deposit_serial(Grid<T> g, Fields<T> F, Parts<T> P, Parts<T> old,
                                                        StepCtl ctl, int n_slots) {
  if (threadIdx.x != 0) return;
  const int n = min(n_slots, *ctl.count);
  int box[4] = {0x7FFFFFFF, -0x7FFFFFFF, 0x7FFFFFFF, -0x7FFFFFFF};
  PlainSink<T> sink{{F.J[0], F.J[1], F.J[2]}, 0, 0, 0};
  for (int p = 0; p < n; ++p) {
    const uint32_t c = P.cell[p];
    if (c == DEAD) continue;
    int i1[3], i0[3];
    unpack_cell(DIM, c, i1[0], i1[1], i1[2]);
    unpack_cell(DIM, old.cell[p], i0[0], i0[1], i0[2]);
    const T f1[3] = {P.f[0][p], P.f[1][p], DIM == 3 ? P.f[2][p] : T(0)};
    const T f0[3] = {old.f[0][p], old.f[1][p], DIM == 3 ? old.f[2][p] : T(0)};
    const T ux = P.u[0][p], uy = P.u[1][p], uz = P.u[2][p];
    const T ig = T(1) / sqrt(T(1) + ux * ux + uy * uy + uz * uz);
    deposit<T, DIM, ORDER>(g, sink, i0, f0, i1, f1, uz * ig, deposit_charge<T, DIM>(g, P, p, i0, f0, i1, f1));
    int rng[4];
    dep_range<ORDER>(i0[0], i1[0], rng[0], rng[1]);
    dep_range<ORDER>(i0[1], i1[1], rng[2], rng[3]);
    box[0] = min(box[0], rng[0]); box[1] = max(box[1], rng[1]);
    box[2] = min(box[2], rng[2]); box[3] = max(box[3], rng[3]);
    bool inside = true;
#pragma unroll
    for (int d = 0; d < DIM; ++d) inside = inside && i1[d] >= 0 && i1[d] < g.M[d];
    if (!inside) P.cell[p] = DEAD;
  }
  if (DIM == 2 && ctl.jslot) jslot_merge(ctl.jslot, box[0], box[1], box[2], box[3]);
}

#define PMLPIC_DISPATCH_ORDER(DIMV, KERNEL, ...)                                         \
  switch (g.order) {                                                                    \
    case 1: hipLaunchKernelGGL((KERNEL<T, DIMV, 1>), grd, blk, 0, s, __VA_ARGS__); break; \
    case 2: hipLaunchKernelGGL((KERNEL<T, DIMV, 2>), grd, blk, 0, s, __VA_ARGS__); break; \
    default: hipLaunchKernelGGL((KERNEL<T, DIMV, 3>), grd, blk, 0, s, __VA_ARGS__); break; \
  }

template <typename T>
void launch_gather_push(const Grid<T> &g, const Fields<T> &F, const Parts<T> &P, Parts<T> old,
                        StepCtl ctl, int n_slots, int push, bool fused, hipStream_t s) {
  if (n_slots <= 0) return;
  dim3 blk(256), grd((n_slots + 255) / 256);
  const int32_t *start = nullptr;
  if (g.dim == 2) { PMLPIC_DISPATCH_ORDER(2, k_gather_push, g, F, P, old, ctl, n_slots, push, fused, start) }
  else { PMLPIC_DISPATCH_ORDER(3, k_gather_push, g, F, P, old, ctl, n_slots, push, fused, start) }
}

template <typename T>
void launch_gather_push_tail(const Grid<T> &g, const Fields<T> &F, const Parts<T> &P, StepCtl ctl,
                             const int32_t *start, int n_upper, int n_slots, int push, hipStream_t s) {
  if (n_upper <= 0 || n_slots <= 0) return;
  dim3 blk(256), grd((n_upper + 255) / 256);
  const Parts<T> old = P;   // not read by the fused form
  const bool fused = true;
  if (g.dim == 2) { PMLPIC_DISPATCH_ORDER(2, k_gather_push, g, F, P, old, ctl, n_slots, push, fused, start) }
  else { PMLPIC_DISPATCH_ORDER(3, k_gather_push, g, F, P, old, ctl, n_slots, push, fused, start) }
}
template void launch_gather_push_tail<float>(const Grid<float> &, const Fields<float> &, const Parts<float> &,
                                             StepCtl, const int32_t *, int, int, int, hipStream_t);
template void launch_gather_push_tail<double>(const Grid<double> &, const Fields<double> &, const Parts<double> &,
                                              StepCtl, const int32_t *, int, int, int, hipStream_t);

template <typename T>
void launch_push_deposit_tiles(const Grid<T> &g, const Fields<T> &F, const Parts<T> &P, StepCtl ctl, JClear<T> jc,
                               const TileWork &tw, int n_slots, int push, hipStream_t s) {
  if (n_slots <= 0) return;
  // an upper bound of the item count: by tile, every tile's last chunk may be partial;
  // else every range may be split
  // tw.sel == 1: the dense tiles' chunks, whose number only the device knows (none in most
  // runs): a grid of a few workgroups per compute unit walks them
  const long nb = tw.sel == 1 ? std::min<long>(1024, deposit_blocks<T>(g, tw, n_slots, true))
                              : deposit_blocks<T>(g, tw, n_slots, true);
  if (nb <= 0) return;
  dim3 blk(TPB), grd((unsigned)nb);
#define PMLPIC_TILES(DIMV, ORD)                                                                                \
  do {                                                                                                         \
    if (tw.by_tile)                                                                                            \
      hipLaunchKernelGGL((k_push_deposit_tiles<T, DIMV, ORD, TileCfg<DIMV>::PPT, true>), grd, blk, 0, s, g, F, \
                         P, ctl, jc, tw, push);                                                                \
    else                                                                                                       \
      hipLaunchKernelGGL((k_push_deposit_tiles<T, DIMV, ORD, TileCfg<DIMV>::PPT, false>), grd, blk, 0, s, g,   \
                         F, P, ctl, jc, tw, push);                                                             \
  } while (0)
  if (g.dim == 2) {
    if (g.order == 1) PMLPIC_TILES(2, 1); else if (g.order == 2) PMLPIC_TILES(2, 2); else PMLPIC_TILES(2, 3);
  } else {
    if (g.order == 1) PMLPIC_TILES(3, 1); else if (g.order == 2) PMLPIC_TILES(3, 2); else PMLPIC_TILES(3, 3);
  }
#undef PMLPIC_TILES
}

template <typename T>
void launch_deposit(const Grid<T> &g, const Fields<T> &F, const Parts<T> &P, Parts<T> old,
                    StepCtl ctl, int n_slots, bool serial, hipStream_t s) {
  if (n_slots <= 0) return;
  if (serial) {
    dim3 blk(64), grd(1);
    if (g.dim == 2) { PMLPIC_DISPATCH_ORDER(2, k_deposit_serial, g, F, P, old, ctl, n_slots) }
    else { PMLPIC_DISPATCH_ORDER(3, k_deposit_serial, g, F, P, old, ctl, n_slots) }
    return;
  }
  dim3 blk(256), grd((n_slots + 255) / 256);
  if (g.dim == 2) { PMLPIC_DISPATCH_ORDER(2, k_deposit, g, F, P, old, ctl, n_slots) }
  else { PMLPIC_DISPATCH_ORDER(3, k_deposit, g, F, P, old, ctl, n_slots) }
}

// ------------------------------------------------------------------ sort_particles
// Counting sort by a tile-major cell key: cells of one tile are contiguous in key
// space, so each tile's particles form one contiguous range, ordered by cell.
// Removed particles get no key and are dropped (compaction).

__device__ __forceinline__ uint32_t cell_key(int dim, const SortWork &sw, int i, int j, int k) {
  const int tx = i / sw.tile[0], lx = i - tx * sw.tile[0];
  const int ty = j / sw.tile[1], ly = j - ty * sw.tile[1];
  const int tz = k / sw.tile[2], lz = k - tz * sw.tile[2];
  const uint32_t tile = ((uint32_t)tz * sw.ntile[1] + ty) * sw.ntile[0] + tx;
  const uint32_t local = ((uint32_t)lz * sw.tile[1] + ly) * sw.tile[0] + lx;
  return tile * (uint32_t)(sw.tile[0] * sw.tile[1] * sw.tile[2]) + local;
}

// Runs of equal keys inside a wavefront (particles are nearly sorted from the previous
// sort): the first lane of my run and the first lane after it.
__device__ __forceinline__ void key_run(uint32_t key, int lane, int &first, int &next) {
  const uint32_t prev = __shfl_up(key, 1);
  const bool start = lane == 0 || prev != key;
  const unsigned long long starts = __ballot(start);
  const unsigned long long upto = (lane == 63) ? ~0ull : ((2ull << lane) - 1ull);
  first = 63 - __clzll((long long)(starts & upto));
  const unsigned long long after = starts & ~upto;
  next = after ? (__ffsll((long long)after) - 1) : 64;
}

// Histogram of the sort keys with the rank of every particle among equal keys.
// A workgroup takes a chunk of HIST_TPB*HIST_PPT consecutive particles (in the order
// of the previous sort) and counts in LDS: one block of tile-cells counters per sort
// tile its particles now occupy, the tiles entered in a small table (a chunk spans a
// few tiles, but their keys can lie far apart: the next row of tiles starts a whole
// row of tiles later).  Runs of equal keys in a wavefront take one counter update, and
// each distinct key costs one global atomic per chunk.  A chunk that meets more tiles
// than the table holds counts straight in global memory.
constexpr int HIST_TPB = 256;
constexpr int HIST_PPT = 4;
constexpr int HIST_LDS = 4096;
constexpr int HIST_MAX_TILES = 64;
constexpr uint32_t NO_TILE = 0xFFFFFFFFu;

template <typename T>
__global__ void __launch_bounds__(HIST_TPB) k_sort_hist(int dim, Parts<T> P, SortWork sw, StepCtl ctl, int n_slots) {
  __shared__ uint32_t cnt[HIST_LDS];
  __shared__ uint32_t stile[HIST_MAX_TILES];
  __shared__ int overflow;
  const int tid = threadIdx.x, lane = tid & 63;
  const int count = min(*ctl.count, n_slots);
  const int base = blockIdx.x * (HIST_TPB * HIST_PPT);
  const uint32_t tc = (uint32_t)(sw.tile[0] * sw.tile[1] * sw.tile[2]);
  const int nslot = (int)min((uint32_t)HIST_MAX_TILES, (uint32_t)HIST_LDS / tc);   // 0: no LDS counting
  if (tid < HIST_MAX_TILES) stile[tid] = NO_TILE;
  if (tid == 0) overflow = nslot == 0;
  __syncthreads();
  uint32_t key[HIST_PPT];
  int slot[HIST_PPT];
#pragma unroll
  for (int k = 0; k < HIST_PPT; ++k) {
    const int p = base + k * HIST_TPB + tid;
    key[k] = 0xFFFFFFFFu;
    slot[k] = -1;
    if (p < count) {
      const uint32_t c = P.cell[p];
      if (c != DEAD) {
        int i, j, kk;
        unpack_cell(dim, c, i, j, kk);
        key[k] = cell_key(dim, sw, i, j, kk);
#ifdef PMLPIC_CHECK
        if (key[k] >= (uint32_t)sw.nkeys) { check_failed(sw.check, CHECK_SORT_KEY); key[k] = 0xFFFFFFFFu; }
#endif
      }
    }
    // the table slot of my tile: the first lane of each run of equal tiles looks it up
    // (open addressing), the others take its answer
    const uint32_t t = key[k] != 0xFFFFFFFFu ? key[k] / tc : NO_TILE;
    int first, next;
    key_run(t, lane, first, next);
    int sl = -1;
    if (lane == first && t != NO_TILE && nslot > 0) {
      for (int a = 0; a < nslot; ++a) {
        const int h = (int)((t + (uint32_t)a) % (uint32_t)nslot);
        const uint32_t v = atomicCAS(&stile[h], NO_TILE, t);
        if (v == NO_TILE || v == t) { sl = h; break; }
      }
      if (sl < 0) overflow = 1;
    }
    slot[k] = __shfl(sl, first);
  }
  __syncthreads();
  const bool local = overflow == 0;   // uniform
  if (local)
    for (int e = tid; e < nslot * (int)tc; e += HIST_TPB) cnt[e] = 0u;
  __syncthreads();
  uint32_t r[HIST_PPT];
#pragma unroll
  for (int k = 0; k < HIST_PPT; ++k) {
    int first, next;
    key_run(key[k], lane, first, next);
    uint32_t b = 0;
    if (lane == first && key[k] != 0xFFFFFFFFu) {
      const uint32_t n = (uint32_t)(next - lane);
      b = local ? atomicAdd(&cnt[slot[k] * tc + key[k] % tc], n) : atomicAdd(&sw.counts[key[k]], n);
    }
    b = __shfl(b, first);
    r[k] = b + (uint32_t)(lane - first);
  }
  if (local) {
    __syncthreads();
    for (int e = tid; e < nslot * (int)tc; e += HIST_TPB) {
      const uint32_t t = stile[e / tc];
      if (t == NO_TILE) continue;
      const uint32_t c = cnt[e];
      if (c) cnt[e] = atomicAdd(&sw.counts[t * tc + e % tc], c);
    }
    __syncthreads();
  }
#pragma unroll
  for (int k = 0; k < HIST_PPT; ++k) {
    const int p = base + k * HIST_TPB + tid;
    if (key[k] != 0xFFFFFFFFu) sw.rank[p] = local ? cnt[slot[k] * tc + key[k] % tc] + r[k] : r[k];
  }
}

constexpr int SCAN_BLOCK = 1024;
constexpr int SCAN_ITEMS = 4;
constexpr int SCAN_TILE = SCAN_BLOCK * SCAN_ITEMS;

// Exclusive prefix of v over the SCAN_BLOCK threads of the workgroup, and their total:
// inclusive scans within each wavefront by lane shuffles, then one over the 16 wavefront
// totals (two barriers; wt holds SCAN_BLOCK / 64 words of LDS)
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t *wt, uint32_t &total) {
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  uint32_t x = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t y = __shfl_up(x, off);
    if (lane >= off) x += y;
  }
  if (lane == 63) wt[w] = x;
  __syncthreads();
  if (w == 0) {
    uint32_t z = lane < SCAN_BLOCK / 64 ? wt[lane] : 0u;
#pragma unroll
    for (int off = 1; off < SCAN_BLOCK / 64; off <<= 1) {
      const uint32_t y = __shfl_up(z, off);
      if (lane >= off) z += y;
    }
    if (lane < SCAN_BLOCK / 64) wt[lane] = z;   // inclusive prefix of the wavefront totals
  }
  __syncthreads();
  total = wt[SCAN_BLOCK / 64 - 1];
  return (w > 0 ? wt[w - 1] : 0u) + x - v;
}

// block-wide exclusive scan of SCAN_TILE counts; block totals to blocksums
__global__ void __launch_bounds__(SCAN_BLOCK) k_scan_local(uint32_t *counts, int n, uint32_t *blocksums) {
  __shared__ uint32_t wt[SCAN_BLOCK / 64];
  const int t = threadIdx.x;
  const long base = (long)blockIdx.x * SCAN_TILE + (long)t * SCAN_ITEMS;
  uint32_t v[SCAN_ITEMS];
  uint32_t sum = 0;
#pragma unroll
  for (int e = 0; e < SCAN_ITEMS; ++e) {
    v[e] = (base + e < n) ? counts[base + e] : 0u;
    sum += v[e];
  }
  uint32_t total;
  uint32_t run = block_exclusive_scan(sum, wt, total);   // exclusive prefix of this thread
#pragma unroll
  for (int e = 0; e < SCAN_ITEMS; ++e) {
    if (base + e < n) counts[base + e] = run;
    run += v[e];
  }
  if (t == 0) blocksums[blockIdx.x] = total;
}

// exclusive scan of the block totals in one block; writes the grand total to *total
__global__ void __launch_bounds__(SCAN_BLOCK) k_scan_blocks(uint32_t *blocksums, int nb, int32_t *total) {
  __shared__ uint32_t wt[SCAN_BLOCK / 64];
  const int t = threadIdx.x;
  uint32_t carry = 0;   // the same in every thread
  for (int start = 0; start < nb; start += SCAN_BLOCK) {
    const uint32_t v = (start + t < nb) ? blocksums[start + t] : 0u;
    uint32_t part;
    const uint32_t ex = block_exclusive_scan(v, wt, part);
    if (start + t < nb) blocksums[start + t] = carry + ex;
    carry += part;
    __syncthreads();   // wt is rewritten by the next pass
  }
  if (t == 0) *total = (int32_t)carry;
}

__global__ void __launch_bounds__(SCAN_BLOCK) k_scan_add(uint32_t *counts, int n, const uint32_t *blocksums) {
  const long base = (long)blockIdx.x * SCAN_TILE + (long)threadIdx.x * SCAN_ITEMS;
  const uint32_t add = blocksums[blockIdx.x];
#pragma unroll
  for (int e = 0; e < SCAN_ITEMS; ++e)
    if (base + e < n) counts[base + e] += add;
}

template <typename T>
__global__ void __launch_bounds__(256) k_sort_scatter(int dim, Parts<T> src, Parts<T> dst, SortWork sw,
                                                      const int32_t *old_count, int n_slots) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n_slots || p >= *old_count) return;
  const uint32_t c = src.cell[p];
  if (c == DEAD) return;
  int i, j, k;
  unpack_cell(dim, c, i, j, k);
  const uint32_t key = cell_key(dim, sw, i, j, k);
#ifdef PMLPIC_CHECK
  if (key >= (uint32_t)sw.nkeys) return;   // flagged by the histogram
#endif
  const uint32_t q = sw.counts[key] + sw.rank[p];
  dst.cell[q] = c;
  for (int d = 0; d < dim; ++d) dst.f[d][q] = src.f[d][p];
  dst.u[0][q] = src.u[0][p];
  dst.u[1][q] = src.u[1][p];
  dst.u[2][q] = src.u[2][p];
  dst.w[q] = src.w[p];
  if (src.lam) dst.lam[q] = src.lam[p];
  dst.id[q] = src.id[p];
}

// the live count after the sort: to the step's counter and after the last key start (the
// end of the last tile's range, which later injections past the count do not move)
__global__ void k_copy_count(const int32_t *src, int32_t *dst, uint32_t *key_end) {
  *dst = *src;
  *key_end = (uint32_t)*src;
}

template <typename T>
void launch_sort(const Grid<T> &g, const Parts<T> &src, const Parts<T> &dst, SortWork sw,
                 StepCtl ctl, int n_slots, hipStream_t s) {
  if (n_slots <= 0) return;
  const int nb = (sw.nkeys + SCAN_TILE - 1) / SCAN_TILE;
  hipMemsetAsync(sw.counts, 0, sizeof(uint32_t) * (size_t)sw.nkeys, s);
  dim3 blk(256), grd((n_slots + 255) / 256);
  const int hist_blocks = (n_slots + HIST_TPB * HIST_PPT - 1) / (HIST_TPB * HIST_PPT);
  hipLaunchKernelGGL((k_sort_hist<T>), dim3(hist_blocks), dim3(HIST_TPB), 0, s, g.dim, src, sw, ctl, n_slots);
  hipLaunchKernelGGL(k_scan_local, dim3(nb), dim3(SCAN_BLOCK), 0, s, sw.counts, sw.nkeys, sw.blocksums);
  // the new count goes to a scratch slot first: the scatter still needs the old one
  int32_t *new_count = (int32_t *)(sw.blocksums + nb);
  hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(SCAN_BLOCK), 0, s, sw.blocksums, nb, new_count);
  hipLaunchKernelGGL(k_scan_add, dim3(nb), dim3(SCAN_BLOCK), 0, s, sw.counts, sw.nkeys, sw.blocksums);
  hipLaunchKernelGGL((k_sort_scatter<T>), grd, blk, 0, s, g.dim, src, dst, sw, ctl.count, n_slots);
  hipLaunchKernelGGL(k_copy_count, dim3(1), dim3(1), 0, s, new_count, ctl.count, sw.counts + sw.nkeys);
}

template <typename T>
int deposit_blocks(const Grid<T> &g, const TileWork &tw, int n_slots, bool tiled) {
  if (n_slots <= 0) return 0;
  if (!tiled) return (n_slots + 255) / 256;
  const int ranges = (n_slots + tw.chunk - 1) / tw.chunk;
  return tw.by_tile ? tw.ntiles + ranges : RANGE_SPLIT * ranges;
}

template int deposit_blocks<float>(const Grid<float> &, const TileWork &, int, bool);
template int deposit_blocks<double>(const Grid<double> &, const TileWork &, int, bool);

int tiled_chunk(int dim) { return TPB * (dim == 2 ? TileCfg<2>::PPT : TileCfg<3>::PPT); }
int tiled_nodes(int dim) { return dim == 2 ? TileCfg<2>::NODES : TileCfg<3>::NODES; }

void launch_tile_chunks(const TileWork &tw, const int32_t *count, hipStream_t s) {
  hipLaunchKernelGGL(k_tile_chunks, dim3((tw.ntiles + 3) / 4), dim3(256), 0, s, tw, count);
  const int nb = (tw.ntiles + SCAN_TILE - 1) / SCAN_TILE;
  for (uint32_t *a : {tw.dprefix, tw.prefix, tw.pprefix}) {   // exclusive scans, totals last
    hipLaunchKernelGGL(k_scan_local, dim3(nb), dim3(SCAN_BLOCK), 0, s, a, tw.ntiles, tw.blocksums);
    hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(SCAN_BLOCK), 0, s, tw.blocksums, nb, (int32_t *)(a + tw.ntiles));
    hipLaunchKernelGGL(k_scan_add, dim3(nb), dim3(SCAN_BLOCK), 0, s, a, tw.ntiles, tw.blocksums);
  }
  hipLaunchKernelGGL(k_tile_items, dim3((tw.ntiles + 255) / 256), dim3(256), 0, s, tw, count);
}

template void launch_push_deposit_tiles<float>(const Grid<float> &, const Fields<float> &, const Parts<float> &,
                                               StepCtl, JClear<float>, const TileWork &, int, int, hipStream_t);
template void launch_push_deposit_tiles<double>(const Grid<double> &, const Fields<double> &, const Parts<double> &,
                                                StepCtl, JClear<double>, const TileWork &, int, int, hipStream_t);

template void launch_gather_push<float>(const Grid<float> &, const Fields<float> &, const Parts<float> &,
                                        Parts<float>, StepCtl, int, int, bool, hipStream_t);
template void launch_gather_push<double>(const Grid<double> &, const Fields<double> &, const Parts<double> &,
                                         Parts<double>, StepCtl, int, int, bool, hipStream_t);
template void launch_deposit<float>(const Grid<float> &, const Fields<float> &, const Parts<float> &,
                                    Parts<float>, StepCtl, int, bool, hipStream_t);
template void launch_deposit<double>(const Grid<double> &, const Fields<double> &, const Parts<double> &,
                                     Parts<double>, StepCtl, int, bool, hipStream_t);
template void launch_sort<float>(const Grid<float> &, const Parts<float> &, const Parts<float> &, SortWork,
                                 StepCtl, int, hipStream_t);
template void launch_sort<double>(const Grid<double> &, const Parts<double> &, const Parts<double> &, SortWork,
                                  StepCtl, int, hipStream_t);

}  // namespace pmlpic
