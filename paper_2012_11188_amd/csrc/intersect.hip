// Per-edge intersection |N(u) ∩ N(h)| and similarity (Algorithm 1 with its
// min-side rule), fused: the count c = t + 2 over closed neighbourhoods and
// the FP64 similarity are written into both CSR slots of the edge.
//
// Every undirected edge {u, h} is owned by its endpoint that is larger in the
// order (degree, id); the owner's row is the lookup structure and every lower
// neighbour u streams its own, shorter row through it, so an edge costs
// min-side work and no global atomics.
//
//   k_plan          per vertex, by degree: 1..small_max go to the small list,
//                   larger vertices are cut into chunks of `spc` row slots
//                   (block-scanned appends, one reservation per tile).
//   k_small_owner   one workgroup per small vertex: if it owns edges, its row
//                   goes into an LDS hash table and its wavefronts stream the
//                   lower neighbours' rows 64 ids at a time through it.
//   k_big_owner     persistent workgroups (1024 threads) holding a bitmap of an
//                   id window (2^wbits ids) in LDS: the owner's ids in the
//                   window are set, every lower neighbour's ids in the window
//                   are tested with one LDS read each, then the bits are
//                   cleared. Chunks are claimed from a global counter, edges
//                   inside a chunk by wavefronts from an LDS counter.
//   k_window_table  (ids spanning several windows) the first position of
//                   every window in every row, so that chunks read each lower
//                   neighbour's range in a window instead of searching it.
#include <hip/hip_runtime.h>

#include <climits>
#include <cstddef>

#include "index.h"

namespace scan {

__device__ __forceinline__ bool is_lower(int32_t u, int32_t du, int32_t h, int32_t dh) {
  return du < dh || (du == dh && u < h);
}

__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }
__device__ __forceinline__ uint64_t lanes_below() {
  return (1ull << lane_id()) - 1ull;
}

// Wave-uniform values. A value broadcast with __shfl or loaded from LDS lives
// in a vector register, and the compiler then treats a loop exit that depends
// on it as divergent; it may restructure such a loop so that lane 0 leaves it
// on a separate path from the other lanes, which breaks cross-lane operations
// inside it. readfirstlane puts the value in a scalar register, which makes the
// uniformity explicit (all lanes are active wherever these are used).
__device__ __forceinline__ int32_t uniform(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t uniform64(int64_t v) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)(uint32_t)v);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)(uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Sum over the wavefront with DPP row shifts and row broadcasts
// (register-path lane exchanges, no LDS crossbar): after row_shr 1, 2, 4, 8
// each row's last lane holds the row total, row_bcast 15 and 31 carry the
// totals to lane 63, which is read into a scalar. All lanes must be active.
__device__ __forceinline__ int32_t dpp_wave_sum(int32_t v) {
  v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, true);  // row_shr:1
  v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, true);  // row_shr:2
  v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, true);  // row_shr:4
  v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, true);  // row_shr:8
  v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, true);  // row_bcast:15 into rows 1, 3
  v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, true);  // row_bcast:31 into rows 2, 3
  return __builtin_amdgcn_readlane(v, kWave - 1);
}

__device__ __forceinline__ int32_t wave_incl_sum(int32_t v) {
  const int lane = lane_id();
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    int32_t t = __shfl_up(v, d, kWave);
    if (lane >= d) v += t;
  }
  return v;
}

struct BigChunk {
  int32_t h;
  int32_t k;  // slots [k*spc, (k+1)*spc) of row h
};

struct PlanCounts {
  int32_t small;       // vertices of degree 1..kLightDeg
  int32_t big;
  int32_t counter;     // work counter of k_big_owner
  int32_t heavy;       // vertices of degree kLightDeg+1..small_max
  int32_t heavy_next;  // work counter of the heavy small-vertex kernel
  int32_t pad[3];
};

constexpr int32_t kLightDeg = kWave;  // one wavefront per vertex up to this degree

// ---------------------------------------------------------------------------
// a2: ownership plan.

// Exclusive prefix sum over the workgroup (one value per thread, up to 1024
// threads); *total receives the sum. wsum holds one int per wavefront.
__device__ __forceinline__ int32_t block_excl_scan(int32_t v, int32_t *wsum, int32_t *total) {
  const int lane = lane_id(), wave = threadIdx.x / kWave, nw = blockDim.x / kWave;
  const int32_t incl = wave_incl_sum(v);
  if (lane == kWave - 1) wsum[wave] = incl;
  __syncthreads();
  if (wave == 0) {
    const int32_t w = lane < nw ? wsum[lane] : 0;
    const int32_t wi = wave_incl_sum(w);
    if (lane < nw) wsum[lane] = wi - w;
    if (lane == nw - 1) *total = wi;
  }
  __syncthreads();
  return incl - v + wsum[wave];
}

constexpr int kPlanThreads = 256;
constexpr int kPlanPer = 8;  // consecutive vertices per thread and tile

// Tiles of kPlanThreads * kPlanPer vertices: a vertex of degree 1..small_max
// goes to the small list, a larger one is cut into chunks of spc row slots.
// Whether a vertex owns any edge is left to the intersection kernels (they
// read the neighbour degrees anyway; a vertex that owns nothing costs one
// staging pass). The block scans its counts, reserves list space with one
// global atomic per list, and writes the entries in vertex order.
__global__ __launch_bounds__(kPlanThreads) void k_plan(const int32_t *deg, int64_t n, int small_max,
                                                       int spc, int32_t *small_list, int32_t *heavy_list,
                                                       BigChunk *big_list, PlanCounts *pc) {
  __shared__ int32_t wsum[kPlanThreads / kWave];
  __shared__ int32_t tot_small, tot_heavy, tot_big, base_small, base_heavy, base_big;
  constexpr int64_t kTile = (int64_t)kPlanThreads * kPlanPer;
  for (int64_t t0 = (int64_t)blockIdx.x * kTile; t0 < n; t0 += (int64_t)gridDim.x * kTile) {
    const int64_t v0 = t0 + (int64_t)threadIdx.x * kPlanPer;
    int32_t code[kPlanPer];  // 0 nothing, -1 light, -2 heavy small, else number of chunks
    int32_t ns = 0, nh = 0, nb = 0;
#pragma unroll
    for (int k = 0; k < kPlanPer; ++k) {
      const int32_t dh = v0 + k < n ? deg[v0 + k] : 0;
      code[k] = dh == 0 ? 0 : dh <= min(small_max, kLightDeg) ? -1 : dh <= small_max ? -2 : (dh + spc - 1) / spc;
      ns += code[k] == -1;
      nh += code[k] == -2;
      nb += code[k] > 0 ? code[k] : 0;
    }
    __syncthreads();  // wsum and the totals are reused across tiles
    const int32_t os = block_excl_scan(ns, wsum, &tot_small);
    const int32_t oh = block_excl_scan(nh, wsum, &tot_heavy);
    const int32_t ob = block_excl_scan(nb, wsum, &tot_big);
    if (threadIdx.x == 0) {
      base_small = tot_small ? atomicAdd(&pc->small, tot_small) : 0;
      base_heavy = tot_heavy ? atomicAdd(&pc->heavy, tot_heavy) : 0;
      base_big = tot_big ? atomicAdd(&pc->big, tot_big) : 0;
    }
    __syncthreads();
    int32_t ps = base_small + os, ph = base_heavy + oh, pb = base_big + ob;
#pragma unroll
    for (int k = 0; k < kPlanPer; ++k) {
      if (code[k] == -1) small_list[ps++] = (int32_t)(v0 + k);
      if (code[k] == -2) heavy_list[ph++] = (int32_t)(v0 + k);
      for (int32_t j = 0; j < code[k]; ++j) big_list[pb++] = BigChunk{(int32_t)(v0 + k), j};
    }
  }
}

// ---------------------------------------------------------------------------
// Writing one edge's result.

__device__ __forceinline__ void write_edge(int kind, int64_t s, int64_t mirror, int32_t t,
                                           int32_t du, int32_t dh, double *sims,
                                           int32_t *counts) {
  const int64_t c = (int64_t)t + 2;
  const double x = similarity(kind, c, (int64_t)du + 1, (int64_t)dh + 1);
  sims[s] = x;
  if (mirror >= 0) sims[mirror] = x;
  if (counts) {
    counts[s] = (int32_t)c;
    if (mirror >= 0) counts[mirror] = (int32_t)c;
  }
}

// ---------------------------------------------------------------------------
// Small owners (degree <= small_max): one workgroup per vertex, of one
// wavefront up to degree kLightDeg and of kSmallWaves wavefronts above. The
// vertex's lower neighbours are compacted into LDS; if there are any, its row
// goes into an LDS hash table (open addressing, load <= 1/2) and the lower
// neighbours' rows are streamed through it: with one wavefront, each group of
// kLightGroup lanes takes one lower neighbour (several rows per step, since
// these rows are short); with several, the wavefronts take them in turn, 64
// ids at a time.

constexpr int kSmallWaves = 4;
#ifndef SCAN_LIGHT_GROUP
#define SCAN_LIGHT_GROUP 16
#endif
constexpr int kLightGroup = SCAN_LIGHT_GROUP;  // lanes per lower neighbour in the one-wavefront kernel
#ifndef SCAN_HEAVY_GROUP
#define SCAN_HEAVY_GROUP 32
#endif
constexpr int kHeavyGroup = SCAN_HEAVY_GROUP;  // and in the kSmallWaves kernel
constexpr int32_t kEmpty = -1;

__device__ __forceinline__ uint32_t hash_slot(int32_t x, int tbits) {
  return ((uint32_t)x * 2654435761u) >> (32 - tbits);  // Fibonacci hashing
}

// Hash table slots per row entry (at least), the kernels' `spread`: the load
// factor is at most 1 / spread. A wavefront's probe loop runs as long as its
// longest chain, so sparse tables pay, up to the LDS they take from other
// workgroups. Builds of the 256-graph SBM batch (light owners, no bitmap
// kernel beside them) took 59.8, 53.0 and 50.8 ms with spreads of 2, 4 and 8;
// R-MAT-23 (heavy owners) 455.4, 452.6 and 454.9 ms. R-MAT-20, whose light
// owners run beside the bitmap kernel, took 7.06 ms per step with a light
// spread of 4 and 7.11 ms with 8. So the heavy kernel takes 4 (which also
// keeps small_max = 4096 within the LDS) and the light one 4 beside the
// bitmap kernel, else 8.
constexpr int kSpreadHeavy = 4, kSpreadLight = 4, kSpreadLightAlone = 8;

// LDS bytes of k_small_owner for a given small_max and spread.
static inline size_t small_lds_bytes(int small_max, int spread) {
  int tb = 6;
  while ((1 << tb) < spread * small_max) ++tb;
  return (size_t)small_max * 20 + ((size_t)4 << tb);
}

// One block per list entry, or (claim != nullptr) persistent blocks that
// claim entries from a counter. The count is read from device memory.
template <int WAVES>
__global__ __launch_bounds__(WAVES * kWave) void k_small_owner(
    const int32_t *list, const int32_t *countp, int32_t *claim, int small_max, int spread, const int64_t *off,
    const int32_t *deg, const int32_t *adj, int kind, double *sims, int32_t *counts, int32_t skip) {
  const int32_t count = *countp;
  __shared__ int32_t s_idx;
  extern __shared__ unsigned char smem[];
  int64_t *lou = (int64_t *)smem;               // [small_max] row offset of the j-th lower neighbour
  int32_t *row = (int32_t *)(lou + small_max);  // [small_max] the vertex's row
  int32_t *ldu = row + small_max;               // [small_max] degree of the j-th lower neighbour
  int32_t *le = ldu + small_max;                // [small_max] its slot in the vertex's row
  int32_t *tab = le + small_max;                // [2^tbits] hash table of the row
  __shared__ int32_t s_nlow;
  const int lane = lane_id(), wave = threadIdx.x / kWave;
  for (int64_t idx0 = blockIdx.x;; idx0 += gridDim.x) {
    int64_t idx = idx0;
    if (WAVES > 1 && claim) {
      __syncthreads();
      if (threadIdx.x == 0) s_idx = atomicAdd(claim, 1);
      __syncthreads();
      idx = uniform(s_idx);
    }
    if (idx >= count) break;  // uniform across the block
    const int32_t h = list[idx];
    const int32_t dh = deg[h];
    const int64_t oh = off[h];
    int tbits = 6;
    while ((1 << tbits) < spread * dh) ++tbits;
    const int32_t tsize = 1 << tbits;
    __syncthreads();
    if (threadIdx.x == 0) s_nlow = 0;
    __syncthreads();
    for (int32_t i0 = 0; i0 < dh; i0 += blockDim.x) {
      const int32_t i = i0 + (int32_t)threadIdx.x;
      int32_t u = 0, d = 0;
      if (i < dh) {
        u = adj[oh + i];
        d = deg[u];
        row[i] = u;
      }
      const bool low = i < dh && is_lower(u, d, h, dh) && d <= skip;
      const uint64_t m = __ballot(low);
      int32_t base = 0;
      if (m) {
        const int leader = __ffsll((unsigned long long)m) - 1;
        int32_t old = 0;
        if (lane == leader) old = atomicAdd(&s_nlow, __popcll(m));
        base = __builtin_amdgcn_readlane(old, leader);
      }
      if (low) {
        const int32_t j = base + __popcll(m & lanes_below());
        le[j] = i;
        ldu[j] = d;
        lou[j] = off[u];
      }
    }
    __syncthreads();
    const int32_t nlow = uniform(s_nlow);
    if (nlow == 0) continue;  // owns no edge (uniform across the block)
    for (int32_t i = threadIdx.x; i < tsize; i += blockDim.x) tab[i] = kEmpty;
    __syncthreads();
    for (int32_t i = threadIdx.x; i < dh; i += blockDim.x) {
      const int32_t x = row[i];
      uint32_t sl = hash_slot(x, tbits);
      while (atomicCAS(&tab[sl], kEmpty, x) != kEmpty) sl = (sl + 1) & (uint32_t)(tsize - 1);
    }
    __syncthreads();
    // Each group of G lanes takes one lower neighbour (NG per wavefront, the
    // wavefronts take successive sets) and streams its row G ids per step; a
    // missing row has length 0. Loads are clamped into the row.
    constexpr int G = WAVES == 1 ? kLightGroup : kHeavyGroup, NG = kWave / G;
    constexpr uint64_t gmask = G == 64 ? ~0ull : (1ull << G) - 1;
    const int grp = lane / G, gl = lane % G;
    for (int32_t j0 = wave * NG; j0 < nlow; j0 += WAVES * NG) {
      const int32_t j = j0 + grp;
      const bool has = j < nlow;
      const int32_t du = has ? ldu[j] : 0;
      const int64_t ou = has ? lou[j] : 0;
      int32_t dmaxg = 0;  // the longest of the NG rows
#pragma unroll
      for (int g = 0; g < NG; ++g)
        if (j0 + g < nlow) dmaxg = max(dmaxg, uniform(ldu[j0 + g]));
      int32_t t = 0;
      int64_t mpos = -1;
      for (int32_t k0 = 0; k0 < dmaxg; k0 += G) {
        const int32_t i = k0 + gl;
        const bool valid = i < du;
        const int32_t x = adj[ou + (valid ? i : (du > 0 ? du - 1 : 0))];
        uint32_t sl = hash_slot(x, tbits);
        bool hit = false;
        for (int32_t probe = 0; probe < tsize; ++probe) {  // ends at x or at an empty slot
          const int32_t v = tab[sl];
          if (v == x) {
            hit = true;
            break;
          }
          if (v == kEmpty) break;
          sl = (sl + 1) & (uint32_t)(tsize - 1);
        }
        const uint64_t m = __ballot(valid && hit), me = __ballot(valid && x == h);
        t += __popcll((m >> (grp * G)) & gmask);
        const uint64_t mine = (me >> (grp * G)) & gmask;
        if (mine) mpos = ou + k0 + (__ffsll((unsigned long long)mine) - 1);
      }
      if (has && gl == 0) write_edge(kind, oh + le[j], mpos, t, du, dh, sims, counts);
    }
  }
}

// ---------------------------------------------------------------------------
// Big owners: persistent workgroups with an LDS bitmap window.

constexpr int kBigThreads = 1024;
#ifndef SCAN_BIG_RUN
#define SCAN_BIG_RUN 4
#endif
constexpr int kUnroll = 4;   // ids per lane per probe group
constexpr int kSeg = 1024;   // most ids per work item (rows longer than this are split)

// Word of the owner bitmap holding bit y. The bitmap starts the kernel's
// dynamic LDS, which starts at LDS address 0 because the kernel has no
// static LDS (the host checks), so the byte address is (y / 32) * 4: two
// instructions, where a pointer to the bitmap costs a third (adding a base
// the compiler cannot fold).
__device__ __forceinline__ uint32_t bitmap_word(uint32_t y) {
  return *(const __attribute__((address_space(3))) uint32_t *)(size_t)((y >> 3) & ~3u);
}

struct BigShared {
  int32_t chunk;
  int32_t run_next, run_left;  // the rest of the workgroup's current run of chunks
  int32_t nlow;
  int32_t next;
  int32_t nextra;
  int32_t wsum[kBigThreads / kWave];
};

// First position in row[lo, hi) whose id is >= key, searched 64-wide by the
// whole wavefront (every lane returns the same value).
__device__ __forceinline__ int64_t wave_lower_bound(const int32_t *row, int64_t lo, int64_t hi,
                                                    int32_t key) {
  const int lane = lane_id();
  while (hi - lo > kWave) {
    const int64_t step = (hi - lo + kWave - 1) / kWave;
    const int64_t p = lo + (int64_t)lane * step;
    const bool less = p < hi && row[p] < key;
    const uint64_t m = __ballot(less);
    const int cnt = __popcll(m);  // positions lo, lo+step, ... below key are a prefix
    if (cnt == 0) return lo;
    const int64_t nlo = lo + (int64_t)(cnt - 1) * step + 1;
    const int64_t nhi = min(hi, lo + (int64_t)cnt * step);
    lo = nlo;
    hi = nhi;
  }
  const int64_t p = lo + lane;
  const bool less = p < hi && row[p] < key;
  return lo + __popcll(__ballot(less));
}

// One workgroup per chunk (owner h, up to spc row slots), persistent over a
// global chunk counter. Per id window: the owner's ids in the window are set
// in the LDS bitmap; each lower neighbour's ids in the window are cut into
// segments of kSeg ids, and wavefronts claim segments from an LDS counter
// (item j < nlow is the first segment of edge j; later items are the extra
// segments of long rows), so one long row cannot hold the workgroup at the
// barrier that ends the window. Partial counts meet in LDS.
template <bool kOneWindow>
__global__ __launch_bounds__(kBigThreads) void k_big_owner(
    const BigChunk *chunks, PlanCounts *pc, int spc, int wbits, int64_t n,
    const int64_t *off, const int32_t *deg, const int32_t *adj, const int32_t *wt, int32_t nwin, int kind,
    double *sims, int32_t *counts, int32_t skip) {
  extern __shared__ unsigned char smem[];
  const int64_t W = (int64_t)1 << wbits;
  const int nwords = (int)(W >> 5);
  uint32_t *bm = (uint32_t *)smem;
  int64_t *le_ou = (int64_t *)(bm + nwords);
  int32_t *le_lt = (int32_t *)(le_ou + spc);  // ids below h in the row (one window)
  int32_t *le_e = le_lt + spc;
  int32_t *le_du = le_e + spc;
  int32_t *le_cnt = le_du + spc;
  int32_t *le_b0 = le_cnt + spc;
  int32_t *le_b1 = le_b0 + spc;  // end of the range in the current window (cursor)
  int32_t *le_u = le_b1 + spc;    // the lower neighbour
  int32_t *le_xp = le_u + spc;    // [spc + 1] exclusive prefix of extra segments
  BigShared *sh = (BigShared *)(le_xp + spc + 1);
  const int tid = threadIdx.x, lane = lane_id();
  constexpr bool one_window = kOneWindow;  // the whole id space fits one window
  // Ids per work item: with several windows the per-window ranges are short
  // and half-size items measure faster (R-MAT-23: 0.57 against 0.62 s),
  // with one window full-size ones (R-MAT-20: 5.6 against 5.8 ms).
  constexpr int kItem = kOneWindow ? kSeg : kSeg / 2;
  constexpr int kItemLoads = kItem / kWave;
  constexpr int kGroups = kItem / (kWave * kUnroll);

  const int32_t nchunks = pc->big;  // written by k_plan: no host round trip
  for (int i = tid; i < nwords; i += blockDim.x) bm[i] = 0u;
  if (tid == 0) sh->run_left = 0;
  // With one window, chunks are claimed in runs of kRun consecutive ones:
  // a high-degree owner's chunks are consecutive, so a run often keeps one
  // owner, and the owner's bits stay in the bitmap from chunk to chunk
  // (they are cleared only when the next chunk has another owner).
  constexpr int32_t kRun = kOneWindow ? SCAN_BIG_RUN : 1;
  int32_t held = -1, held_dh = 0;  // the owner whose bits the bitmap holds
  int64_t held_oh = 0;
  for (;;) {
    __syncthreads();
    if (tid == 0) {
      if (sh->run_left == 0) {
        sh->run_next = atomicAdd(&pc->counter, kRun);
        sh->run_left = kRun;
      }
      sh->chunk = sh->run_next++;
      --sh->run_left;
      sh->nlow = 0;
    }
    __syncthreads();
    const int32_t ci = uniform(sh->chunk);
    if (ci >= nchunks) break;
    const BigChunk ch = chunks[ci];
    const int32_t h = ch.h;
    const int32_t dh = deg[h];
    const int64_t oh = off[h];
    const int64_t s0 = oh + (int64_t)ch.k * spc;
    const int m = (int)min((int64_t)spc, oh + dh - s0);
    // Stage the chunk's lower neighbours (wave-aggregated compaction).
    for (int e0 = 0; e0 < m; e0 += blockDim.x) {
      const int e = e0 + tid;
      int32_t u = 0, du = 0;
      bool low = false;
      if (e < m) {
        u = adj[s0 + e];
        du = deg[u];
        low = is_lower(u, du, h, dh) && du <= skip;
      }
      const uint64_t mk = __ballot(low);
      int32_t base = 0;
      if (mk) {
        const int leader = __ffsll((unsigned long long)mk) - 1;
        int32_t old = 0;
        if (lane == leader) old = atomicAdd(&sh->nlow, __popcll(mk));
        base = __builtin_amdgcn_readlane(old, leader);
      }
      if (low) {
        const int k = base + __popcll(mk & lanes_below());
        le_e[k] = e;
        le_u[k] = u;
        le_du[k] = du;
        le_ou[k] = off[u];
        le_cnt[k] = 0;
        le_lt[k] = 0;
        le_b0[k] = 0;
        le_b1[k] = one_window ? du : 0;
      }
    }
    __syncthreads();
    const int nlow = uniform(sh->nlow);
    if (nlow == 0) continue;
    if (one_window && h != held) {
      if (held >= 0) {
        for (int i = tid; i < held_dh; i += blockDim.x) bm[(uint32_t)adj[held_oh + i] >> 5] = 0u;
        __syncthreads();  // the new owner's bits may share words with the old one's
      }
      for (int i = tid; i < dh; i += blockDim.x) {
        const int32_t x = adj[oh + i];
        atomicOr(&bm[x >> 5], 1u << (x & 31));
      }
      held = h;
      held_oh = oh;
      held_dh = dh;
    }
    // Windows of ids [w0, w0 + W) that hold ids of N(h), in increasing order.
    // With the window table, thread i < nlow reads edge i's range in the
    // next window while the current window's items run (pf_w: the window
    // its prefetched pair belongs to).
    int64_t p = 0;
    int32_t pf0 = 0, pf1 = 0;
    int64_t pf_w = -1;
    while (p < dh) {
      const int64_t w0 = one_window ? 0 : ((int64_t)adj[oh + p] >> wbits) << wbits;
      const int64_t pe = one_window ? dh
                         : wt ? (int64_t)wt[(int64_t)h * (nwin + 1) + (w0 >> wbits) + 1]
                              : wave_lower_bound(adj + oh, p, dh, (int32_t)min(w0 + W, (int64_t)INT32_MAX));
      for (int64_t i = p + tid; !one_window && i < pe; i += blockDim.x) {
        const int32_t x = (int32_t)(adj[oh + i] - w0);
        atomicOr(&bm[x >> 5], 1u << (x & 31));
      }
      if (!one_window && wt) {
        // each lower neighbour's ids inside this window, from the table;
        // thread i reads back only its own edge's range before the scan's
        // barriers, so no barrier is needed here (nlow <= spc <= blockDim)
        const int64_t kw = w0 >> wbits;
        if (tid < nlow) {
          if (pf_w != kw) {
            const int32_t *t = wt + (int64_t)le_u[tid] * (nwin + 1) + kw;
            pf0 = t[0];
            pf1 = t[1];
          }
          le_b0[tid] = pf0;
          le_b1[tid] = pf1;
        }
      } else if (!one_window) {
        // each lower neighbour's ids inside this window, after the last one
        if (tid == 0) sh->next = 0;
        __syncthreads();
        for (;;) {
          int32_t old = 0;
          if (lane == 0) old = atomicAdd(&sh->next, 1);
          const int32_t i = __builtin_amdgcn_readlane(old, 0);
          if (i >= nlow) break;
          const int32_t du = uniform(le_du[i]);
          const int32_t *row = adj + uniform64(le_ou[i]);
          const int64_t b0 = wave_lower_bound(row, uniform(le_b1[i]), du, (int32_t)w0);
          const int64_t b1 = wave_lower_bound(row, b0, du, (int32_t)min(w0 + W, (int64_t)INT32_MAX));
          le_b0[i] = (int32_t)b0;
          le_b1[i] = (int32_t)b1;
        }
        __syncthreads();
      }
      // Extra segments of long ranges, as an exclusive prefix over the edges.
      int32_t ex = 0;
      if (tid < nlow) {
        const int32_t len = le_b1[tid] - le_b0[tid];
        ex = len > kItem ? (len - 1) / kItem : 0;
      }
      const int32_t xp = block_excl_scan(ex, sh->wsum, &sh->nextra);
      if (tid < nlow) le_xp[tid] = xp;
      if (tid == 0) sh->next = 0;
      __syncthreads();
      const int32_t nitems = nlow + uniform(sh->nextra);
      if (!one_window && wt && pe < dh && tid < nlow) {  // the next window's ranges, read during the items
        const int64_t kwn = (int64_t)adj[oh + pe] >> wbits;
        const int32_t *t = wt + (int64_t)le_u[tid] * (nwin + 1) + kwn;
        pf0 = t[0];
        pf1 = t[1];
        pf_w = kwn;
      }
      // Work items are claimed from the LDS counter, one lane adding 1.
      // A claim is split in two: take() issues the LDS atomic, resolve()
      // turns its result into an item. Between the two the wavefront probes
      // its current item, so the atomic's round trip is not on its path.
      auto take = [&]() -> int32_t {
        int32_t old = 0;
        if (lane == 0) old = atomicAdd(&sh->next, 1);
        return old;
      };
      auto resolve = [&](int32_t tok, int32_t &e, int32_t &lo, int32_t &hi, int64_t &ou) {
        const int32_t j = __builtin_amdgcn_readlane(tok, 0);
        if (j >= nitems) {
          e = -1;
          lo = hi = 0;
          ou = 0;
          return;
        }
        int32_t ee = j, sg = 0;
        if (j >= nlow) {
          // the last edge with le_xp[e] <= jj (le_xp is non-decreasing and
          // le_xp[0] = 0): a 64-way search, every lane sampling one edge
          const int32_t jj = j - nlow;
          int32_t a0 = 0, na = nlow;
          while (na > 1) {
            const int32_t step = (na + kWave - 1) / kWave;
            const int32_t q = a0 + lane * step;
            const int32_t c = __popcll(__ballot(q < a0 + na && le_xp[q] <= jj));  // >= 1: lane 0
            const int32_t nb = a0 + (c - 1) * step;
            na = min(step, a0 + na - nb);
            a0 = nb;
          }
          ee = a0;
          sg = 1 + jj - uniform(le_xp[a0]);
        }
        e = ee;
        ou = uniform64(le_ou[ee]);
        lo = uniform(le_b0[ee]) + sg * kItem;
        hi = min(uniform(le_b1[ee]), lo + kItem);
      };
      // Probes the group of kWave * kUnroll ids that starts at position g0
      // of an item of len ids. Per lane, acc counts the hits (low half) and
      // the ids below h (high half): rows are sorted, so with one window the
      // position of h in the lower neighbour's row is the sum of the latter
      // over the row's items. Both halves stay below 2^16 (<= kItem per item).
      auto probe_group = [&](const int32_t x[kUnroll], int32_t g0, int32_t len, uint32_t &acc) {
        if (g0 + kWave * kUnroll <= len) {
#pragma unroll
          for (int k = 0; k < kUnroll; ++k) {
            const uint32_t y = kOneWindow ? (uint32_t)x[k] : (uint32_t)(x[k] - (int32_t)w0);
            acc += __builtin_amdgcn_ubfe(bitmap_word(y), y, 1) + (x[k] < h ? 0x10000u : 0u);  // bit y & 31
          }
        } else {
#pragma unroll
          for (int k = 0; k < kUnroll; ++k) {
            if (g0 + k * kWave >= len) break;  // uniform
            const bool valid = g0 + k * kWave + lane < len;
            const uint32_t vm = 0u - (uint32_t)valid;
            // inside the item every id lies in the current window
            const uint32_t y = kOneWindow ? (uint32_t)x[k] : (uint32_t)(x[k] - (int32_t)w0);
            acc += (__builtin_amdgcn_ubfe(bitmap_word(y & vm), y, 1) + (x[k] < h ? 0x10000u : 0u)) & vm;
          }
        }
      };
      // Whole items are requested one item ahead, and the loop body is
      // unrolled twice so the two register sets swap roles without register
      // copies (a copy waits for its load). Every load of an item is
      // issued: a fixed count keeps the waits exact (the compiler waits for
      // an item's loads by counting the loads issued after them). The loads
      // are raw buffer loads over a resource of exactly the item's bytes, so
      // lanes past its end read 0 without touching memory (no line is
      // fetched for them, and no bound check or mask is needed; the probe
      // masks those lanes). Addressing is scalar base + lane offset +
      // immediate: no vector instruction per load.
      auto fetch_item = [&](int32_t x[kItemLoads], int64_t ou, int32_t lo, int32_t len) {
        // resource word 3: DATA_FORMAT 32 (a valid format enables the buffer)
        const __amdgpu_buffer_rsrc_t r =
            __builtin_amdgcn_make_buffer_rsrc((void *)(adj + ou + lo), (short)0, len * 4, 0x00020000);
#pragma unroll
        for (int j = 0; j < kItemLoads; ++j) x[j] = __builtin_amdgcn_raw_buffer_load_b32(r, lane * 4 + j * kWave * 4, 0, 0);
      };
      auto probe_item = [&](const int32_t x[kItemLoads], int32_t e, int32_t len) {
        uint32_t acc = 0;
#pragma unroll
        for (int c = 0; c < kGroups; ++c)
          if (c == 0 || len > c * kWave * kUnroll) probe_group(x + c * kUnroll, c * kWave * kUnroll, len, acc);
        const uint32_t t = (uint32_t)dpp_wave_sum((int32_t)acc);
        // t is wave-uniform: lane 0 records it (no return value is used, so
        // no lane waits on another)
        if (lane == 0) {
          atomicAdd(&le_cnt[e], (int32_t)(t & 0xffffu));
          if (kOneWindow) atomicAdd(&le_lt[e], (int32_t)(t >> 16));
        }
      };
      // Items are claimed one step further ahead: the claim's atomic goes
      // out before a probe and is resolved after it, when the probe has
      // freed its registers, so no claim waits on loads in flight.
      int32_t ea, loa, hia, eb, lob, hib;
      int64_t oua, oub;
      int32_t xa[kItemLoads], xb[kItemLoads];
      resolve(take(), ea, loa, hia, oua);
      fetch_item(xa, oua, loa, hia - loa);
      resolve(take(), eb, lob, hib, oub);
      while (ea >= 0) {
        fetch_item(xb, oub, lob, hib - lob);
        const int32_t ta = take();
        probe_item(xa, ea, hia - loa);
        resolve(ta, ea, loa, hia, oua);
        if (eb < 0) break;
        fetch_item(xa, oua, loa, hia - loa);
        const int32_t tb = take();
        probe_item(xb, eb, hib - lob);
        resolve(tb, eb, lob, hib, oub);
      }
      __syncthreads();
      for (int64_t i = p + tid; !one_window && i < pe; i += blockDim.x) {
        const int32_t x = (int32_t)(adj[oh + i] - w0);
        bm[x >> 5] = 0u;
      }
      p = pe;
      // the next window's bits may share words with the ones just cleared
      if (!one_window) __syncthreads();
    }
    __syncthreads();
    for (int i = tid; i < nlow; i += blockDim.x) {
      int64_t mir = -1;
      if (one_window) {
        // h sits after the ids below it (absent only from an asymmetric row)
        const int32_t lt = le_lt[i];
        if (lt < le_du[i] && adj[le_ou[i] + lt] == h) mir = le_ou[i] + lt;
      } else {
        // h may lie in a window that holds no id of N(h): locate it directly
        const int64_t ou = le_ou[i];
        int64_t lo = 0, hi = le_du[i];
        while (lo < hi) {
          const int64_t mid = (lo + hi) >> 1;
          if (adj[ou + mid] < h) lo = mid + 1;
          else hi = mid;
        }
        mir = (lo < le_du[i] && adj[ou + lo] == h) ? ou + lo : -1;
      }
      write_edge(kind, s0 + le_e[i], mir, le_cnt[i], le_du[i], dh, sims, counts);
    }
  }
}

// Window table of every row: wt[u * (nwin + 1) + k] = the first position in
// row u whose id is >= k * 2^wbits (k = 0..nwin), so that a lower
// neighbour's ids inside window k are positions [wt[k], wt[k + 1]) of its
// row. One wavefront per row; the next row's offsets are requested while a
// row is handled. Rows of up to kTableScan ids are streamed 64 ids per step:
// a lane whose id opens windows past its left neighbour's writes their
// starts (every entry is written once), and the step past the row's end
// closes the last windows. Longer rows find each window's start by a 64-way
// search (every lane samples one position, a few rounds per window), so that
// no wavefront walks a hub's whole row.
constexpr int32_t kTableScan = 2048;

__global__ __launch_bounds__(256) void k_window_table(const int64_t *off, const int32_t *adj, int64_t n,
                                                      int wbits, int32_t nwin, const PlanCounts *pc, int32_t *wt) {
  if (pc->big == 0) return;  // no bitmap owners: the table is not read
  const int lane = lane_id();
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / kWave;
  int64_t u = uniform64((blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kWave);
  int64_t o_next = 0, e_next = 0;  // offsets of the wavefront's next row
  if (u < n) {
    o_next = off[u];
    e_next = off[u + 1];
  }
  for (; u < n; u += nw) {
    const int64_t o = uniform64(o_next);
    const int32_t d = uniform((int32_t)(uniform64(e_next) - o));
    if (u + nw < n) {
      o_next = off[u + nw];
      e_next = off[u + nw + 1];
    }
    int32_t *t = wt + u * (nwin + 1);
    if (d > kTableScan) {
      int32_t lo = 0;  // window starts do not decrease with k
      for (int32_t k = 1; k < nwin; ++k) {
        const int64_t bound = (int64_t)k << wbits;
        int32_t hi = d;  // the start is in [lo, hi]; position d stands for the end of the row
        while (lo < hi) {
          // (kWave - 1) * step >= hi - lo: the last lane samples at or past hi
          const int32_t step = (hi - lo + kWave - 2) / (kWave - 1);
          const int64_t p = (int64_t)lo + (int64_t)lane * step;
          const bool at = p >= hi || adj[o + p] >= bound;
          const int f = __ffsll((unsigned long long)__ballot(at)) - 1;  // >= 0: the last lane is true
          if (f == 0) break;  // the start is lo
          const int32_t nlo = lo + (f - 1) * step + 1;
          hi = uniform((int32_t)min((int64_t)hi, (int64_t)lo + (int64_t)f * step));
          lo = uniform(nlo);
        }
        if (lane == 0) t[k] = lo;
      }
      if (lane == 0) {
        t[0] = 0;
        t[nwin] = d;
      }
      continue;
    }
    int32_t prev = -1;  // window of the id before this step (wave-uniform)
    for (int32_t i0 = 0; i0 <= d; i0 += kWave) {
      const int32_t i = i0 + lane;
      const int32_t w = i < d ? adj[o + i] >> wbits : nwin;  // past the end: window nwin
      int32_t wl = __shfl_up(w, 1, kWave);
      if (lane == 0) wl = prev;
      for (int32_t k = wl + 1; k <= w; ++k) t[k] = i;
      prev = __shfl(w, kWave - 1, kWave);
    }
  }
}

// ---------------------------------------------------------------------------
// Host side.

constexpr size_t kMaxWindowTable = (size_t)4 << 30;

static size_t big_lds_bytes(int wbits, int spc) {
  return ((size_t)1 << wbits) / 8 + (size_t)spc * (8 + 4 * 8) + 4 + sizeof(BigShared);
}

IntersectPlan::~IntersectPlan() {
  if (ready) {
    (void)hipEventSynchronize(ready);  // the copy into `host` is done
    (void)hipEventDestroy(ready);
  }
  pinned_put(host);
}

// The id window width of the large-owner kernel: cfg.wbits, no wider than
// the id space and narrowed until its LDS fits.
static int window_bits(const IntersectConfig &cfg, int64_t n, int lds_max) {
  int wbits = cfg.wbits;
  int nb = 0;
  while (((int64_t)1 << nb) < n) ++nb;
  if (nb < 10) nb = 10;
  if (wbits > nb) wbits = nb;
  while (wbits > 10 && big_lds_bytes(wbits, cfg.spc) > (size_t)lds_max) --wbits;
  return wbits;
}

scan_status intersect_plan(const IntersectConfig &cfg, int64_t n, int64_t nnz, const int64_t *off,
                           const int32_t *deg, const int32_t *adj, int device, DevArena &arena, hipStream_t s,
                           IntersectPlan &p) {
  static_assert(sizeof(PlanCounts) <= kPinnedBlock, "plan counts fit a pinned block");
  p.n = n;
  p.nnz = nnz;
  if (nnz == 0) return SCAN_OK;
  int lds_max = 65536;
  (void)hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, device);
  p.wbits = window_bits(cfg, n, lds_max);
  const int32_t nwin = (int32_t)((n + ((int64_t)1 << p.wbits) - 1) >> p.wbits);
  BigChunk *big_list;
  PlanCounts *pc;
  SCAN_TRY(arena.alloc(&p.small_list, n));
  SCAN_TRY(arena.alloc(&p.heavy_list, n));
  SCAN_TRY(arena.alloc(&big_list, nnz / cfg.spc + n + 1));
  SCAN_TRY(arena.alloc(&pc, 1));
  p.big_list = big_list;
  p.counts = pc;
  p.host = pinned_get();
  if (!p.host) return fail(SCAN_ENOMEM, "pinned host allocation failed");
  SCAN_HIP_TRY(hipEventCreateWithFlags(&p.ready, hipEventDisableTiming));
  SCAN_HIP_TRY(hipMemsetAsync(pc, 0, sizeof(PlanCounts), s));
  k_plan<<<grid_for(n, kPlanThreads * kPlanPer, 2048), kPlanThreads, 0, s>>>(deg, n, cfg.small_max, cfg.spc,
                                                                             p.small_list, p.heavy_list, big_list, pc);
  SCAN_HIP_TRY(hipMemcpyAsync(p.host, pc, sizeof(PlanCounts), hipMemcpyDeviceToHost, s));
  SCAN_HIP_TRY(hipEventRecord(p.ready, s));
  // Ids spanning several windows: the window table follows the plan (it
  // needs only the CSR, and nothing when there are no bitmap owners), so
  // that the large-owner kernel can start as soon as the host has read the
  // plan's counts.
  if (nwin > 1 && !cfg.search_windows && (size_t)(nwin + 1) * (size_t)n * 4 <= kMaxWindowTable) {
    SCAN_TRY(arena.alloc(&p.wt, (int64_t)(nwin + 1) * n));
    k_window_table<<<grid_for(n * kWave, 256), 256, 0, s>>>(off, adj, n, p.wbits, nwin, pc, p.wt);
  }
  return SCAN_OK;
}

scan_status intersect_all(const IntersectConfig &cfg, int64_t n, int64_t nnz, const int64_t *off,
                          const int32_t *deg, const int32_t *adj, int kind, double *sims,
                          int32_t *counts, int device, hipStream_t s, IntersectStats *stats,
                          const std::function<scan_status()> &after_launch, const IntersectPlan *plan) {
  if (nnz == 0) {
      return after_launch ? after_launch() : SCAN_OK;
  }
  int lds_max = 65536, cus = 256;
  (void)hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, device);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
  const int wbits = window_bits(cfg, n, lds_max);
  if (big_lds_bytes(wbits, cfg.spc) > (size_t)lds_max) return fail(SCAN_EINVAL, "chunk size too large for LDS");

  DevArena tmp(s);
  IntersectPlan own;
  if (!plan) {
    SCAN_TRY(intersect_plan(cfg, n, nnz, off, deg, adj, device, tmp, s, own));
    plan = &own;
  }
  if (plan->n != n || plan->nnz != nnz || !plan->ready || plan->wbits != wbits)
    return fail(SCAN_EINVAL, "plan made for another graph");
  const int32_t *small_list = plan->small_list, *heavy_list = plan->heavy_list;
  const BigChunk *big_list = (const BigChunk *)plan->big_list;
  PlanCounts *pc = (PlanCounts *)plan->counts;
  // The host reads the work counts to size the grids: one block per vertex
  // lets the hardware balance the uneven rows, which persistent grids with a
  // static split do not.
  SCAN_HIP_TRY(hipEventSynchronize(plan->ready));
  const PlanCounts h = *(const PlanCounts *)plan->host;
  if (stats) {
    stats->wbits = wbits;
    stats->launches = (h.small > 0) + (h.heavy > 0) + (h.big > 0);
    if (stats->host_counts) {
      stats->host_counts[0] = h.small;
      stats->host_counts[1] = h.big;
      stats->host_counts[3] = h.heavy;
    }
  }
  auto mark = [&](hipEvent_t e, hipStream_t st) -> scan_status {
    if (e) SCAN_HIP_TRY(hipEventRecord(e, st));
    return SCAN_OK;
  };
  SCAN_TRY(mark(stats ? stats->ev_plan_end : nullptr, s));
  // The large-owner kernel is persistent (one 1024-thread workgroup per CU,
  // most of the LDS) and leaves wavefront slots, registers and some LDS free
  // on every CU; the small-owner kernels, independent of it, run on the
  // helper stream and fill them. The large one is launched first so that its
  // workgroups are placed before the small ones take CUs.
  // The two small-owner kernels take helper streams of their own, so that
  // neither waits for the other.
  auto fork = [&](int k, bool used) -> hipStream_t {
    if (!used || !h.big) return s;
    if (plan->helper[k]) return plan->helper[k];  // ordered after the plan by the caller
    hipStream_t hs = helper_stream(k);
    if (!hs || stream_wait(hs, s) != SCAN_OK) return s;
    return hs;
  };
  const hipStream_t sh = fork(0, h.heavy > 0), sl = fork(1, h.small > 0);
  JoinOnExit join_sh{s, sh}, join_sl{s, sl};  // before the plan lists are released
  if (h.big) {
    size_t lds = big_lds_bytes(wbits, cfg.spc);
    const bool one = n <= ((int64_t)1 << wbits);
    // Several windows: each row's window starts come from the plan's table
    // unless it would exceed kMaxWindowTable bytes or the searched ranges are
    // asked for; then chunks search them per window.
    int32_t *wt = plan->wt;
    const int32_t nwin = (int32_t)((n + ((int64_t)1 << wbits) - 1) >> wbits);
    const void *fn = one ? (const void *)k_big_owner<true> : (const void *)k_big_owner<false>;
    hipFuncAttributes fa;
    SCAN_HIP_TRY(hipFuncGetAttributes(&fa, fn));
    if (fa.sharedSizeBytes != 0)  // bitmap_word assumes the dynamic LDS starts at address 0
      return fail(SCAN_EDEVICE, "k_big_owner has %zu bytes of static LDS", (size_t)fa.sharedSizeBytes);
    if (lds > 65536)
      SCAN_HIP_TRY(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    const int per_cu = (int)std::max<size_t>(1, std::min<size_t>(2, (size_t)lds_max / lds));
    const int grid = (int)std::min<int64_t>((int64_t)cus * per_cu, h.big);
    SCAN_TRY(mark(stats ? stats->ev_big_begin : nullptr, s));
    if (one)
      k_big_owner<true><<<grid, kBigThreads, lds, s>>>(big_list, pc, cfg.spc, wbits, n, off, deg, adj, nullptr,
                                                       nwin, kind, sims, counts, cfg.skip_deg);
    else
      k_big_owner<false><<<grid, kBigThreads, lds, s>>>(big_list, pc, cfg.spc, wbits, n, off, deg, adj, wt,
                                                        nwin, kind, sims, counts, cfg.skip_deg);
    SCAN_HIP_TRY(hipGetLastError());
    SCAN_TRY(mark(stats ? stats->ev_big_end : nullptr, s));
  } else {
    SCAN_TRY(mark(stats ? stats->ev_big_begin : nullptr, s));
    SCAN_TRY(mark(stats ? stats->ev_big_end : nullptr, s));
  }
  const hipStream_t ss = sh != s ? sh : sl;  // the small-owner events go on one of them
  SCAN_TRY(mark(stats ? stats->ev_small_begin : nullptr, ss));
  if (h.small || h.heavy) {
    const int cap = std::min<int>(cfg.small_max, kLightDeg);  // light rows: LDS sized for them
    const int spread1 = h.big ? kSpreadLight : kSpreadLightAlone;
    const size_t lds = small_lds_bytes(cfg.small_max, kSpreadHeavy), lds1 = small_lds_bytes(cap, spread1);
    if (lds > (size_t)lds_max || lds1 > (size_t)lds_max) return fail(SCAN_EINVAL, "small_max too large for LDS");
    if (lds > 65536)
      SCAN_HIP_TRY(hipFuncSetAttribute((const void *)k_small_owner<kSmallWaves>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    if (lds1 > 65536)
      SCAN_HIP_TRY(hipFuncSetAttribute((const void *)k_small_owner<1>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds1));
    if (h.heavy)  // the longer rows first
      k_small_owner<kSmallWaves><<<h.heavy, kSmallWaves * kWave, lds, sh>>>(
          heavy_list, &pc->heavy, nullptr, cfg.small_max, kSpreadHeavy, off, deg, adj, kind, sims, counts,
          cfg.skip_deg);
    if (h.small)
      k_small_owner<1><<<h.small, kWave, lds1, sl>>>(small_list, &pc->small, nullptr, cap, spread1, off, deg, adj,
                                                     kind, sims, counts, cfg.skip_deg);
    SCAN_HIP_TRY(hipGetLastError());
  }
  if (sl != ss) SCAN_TRY(stream_wait(ss, sl));  // the end event covers both
  SCAN_TRY(mark(stats ? stats->ev_small_end : nullptr, ss));
  if (after_launch) SCAN_TRY(after_launch());
  return SCAN_OK;
}

}  // namespace scan
