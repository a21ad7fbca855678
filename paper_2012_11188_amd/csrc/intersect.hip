// Per-edge intersection |N(u) ∩ N(h)| and similarity (Algorithm 1 with its
// min-side rule), fused: the count c = t + 2 over closed neighbourhoods and
// the FP64 similarity are written into both CSR slots of the edge.
//
// Every undirected edge {u, h} is owned by its endpoint that is larger in the
// order (degree, id); the owner's row is the lookup structure and every lower
// neighbour u streams its own, shorter row through it, so an edge costs
// min-side work and no global atomics.
//
//   k_plan          one thread per vertex: owners with degree <= small_max go
//                   to the small list, larger owners are cut into chunks of
//                   `spc` row slots (wave-aggregated appends).
//   k_small_owner   one wavefront per small owner: its row sits sorted in LDS;
//                   a lower neighbour's row is streamed 64 ids at a time and
//                   each id is located by a fixed-step binary search.
//   k_big_owner     persistent workgroups (1024 threads) holding a bitmap of an
//                   id window (2^wbits ids) in LDS: the owner's ids in the
//                   window are set, every lower neighbour's ids in the window
//                   are tested with one LDS read each, then the bits are
//                   cleared. Chunks are claimed from a global counter, edges
//                   inside a chunk by wavefronts from an LDS counter.
#include <hip/hip_runtime.h>

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

__device__ __forceinline__ int32_t wave_sum(int32_t v) {
#pragma unroll
  for (int m = kWave / 2; m > 0; m >>= 1) v += __shfl_xor(v, m, kWave);
  return v;
}

__device__ __forceinline__ int32_t wave_max(int32_t v) {
#pragma unroll
  for (int m = kWave / 2; m > 0; m >>= 1) v = max(v, __shfl_xor(v, m, kWave));
  return v;
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
  int32_t small;
  int32_t big;
  int32_t counter;  // work counter of k_big_owner
  int32_t pad;
};

// ---------------------------------------------------------------------------
// a2: ownership plan.

__global__ __launch_bounds__(256) void k_plan(const int64_t *off, const int32_t *deg,
                                              const int32_t *adj, int64_t n, int small_max,
                                              int spc, int32_t *small_list, BigChunk *big_list,
                                              PlanCounts *pc) {
  const int lane = lane_id();
  for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < n;
       base += (int64_t)gridDim.x * blockDim.x) {
    const int64_t h = base + threadIdx.x;
    bool own = false;
    int32_t dh = 0;
    if (h < n) {
      dh = deg[h];
      const int64_t b = off[h];
      for (int64_t s = b; s < b + dh; ++s) {
        const int32_t u = adj[s];
        if (is_lower(u, deg[u], (int32_t)h, dh)) {
          own = true;
          break;
        }
      }
    }
    const bool small = own && dh <= small_max;
    const uint64_t m = __ballot(small);
    if (m) {
      const int leader = __ffsll((unsigned long long)m) - 1;
      const int32_t sb =
          __builtin_amdgcn_readlane(atomicAdd(&pc->small, lane == leader ? __popcll(m) : 0), leader);
      if (small) small_list[sb + __popcll(m & lanes_below())] = (int32_t)h;
    }
    const int32_t nch = (own && !small) ? (dh + spc - 1) / spc : 0;
    const int32_t incl = wave_incl_sum(nch);
    const int32_t total = __shfl(incl, kWave - 1, kWave);
    if (total) {
      const int32_t bb = uniform(atomicAdd(&pc->big, lane == 0 ? total : 0));
      for (int32_t k = 0; k < nch; ++k) big_list[bb + incl - nch + k] = BigChunk{(int32_t)h, k};
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
// Small owners: one wavefront (workgroup of 64) per owner.

__global__ __launch_bounds__(64) void k_small_owner(const int32_t *list, int32_t count,
                                                    int small_max, const int64_t *off,
                                                    const int32_t *deg, const int32_t *adj,
                                                    int kind, double *sims, int32_t *counts) {
  extern __shared__ unsigned char smem[];
  int32_t *row = (int32_t *)smem;                  // [small_max]
  int32_t *rdu = row + small_max;                  // [small_max] degree, -1 if not lower
  int64_t *rou = (int64_t *)(rdu + small_max);     // [small_max]
  const int lane = lane_id();
  for (int32_t idx = blockIdx.x; idx < count; idx += gridDim.x) {
    const int32_t h = list[idx];
    const int32_t dh = deg[h];
    const int64_t oh = off[h];
    __syncthreads();
    for (int i = lane; i < dh; i += kWave) {
      const int32_t u = adj[oh + i];
      const int32_t d = deg[u];
      row[i] = u;
      rdu[i] = is_lower(u, d, h, dh) ? d : -1;
      rou[i] = off[u];
    }
    __syncthreads();
    int top = 1;
    while (top * 2 <= dh) top *= 2;
    for (int e = 0; e < dh; ++e) {
      const int32_t du = uniform(rdu[e]);
      if (du < 0) continue;
      const int64_t ou = uniform64(rou[e]);
      int32_t t = 0;
      int64_t mpos = -1;
      for (int32_t k0 = 0; k0 < du; k0 += kWave) {
        const int32_t i = k0 + lane;
        const bool valid = i < du;
        const int32_t x = valid ? adj[ou + i] : -1;
        int pos = -1;  // last index with row[pos] < x
        for (int step = top; step > 0; step >>= 1) {
          const int q = pos + step;
          if (q < dh && row[q] < x) pos = q;
        }
        const bool hit = valid && pos + 1 < dh && row[pos + 1] == x;
        t += __popcll(__ballot(hit));
        const uint64_t me = __ballot(valid && x == h);
        if (me) mpos = ou + k0 + (__ffsll((unsigned long long)me) - 1);
      }
      // wave-uniform result: every lane stores the same values
      write_edge(kind, oh + e, mpos, t, du, dh, sims, counts);
    }
  }
}

// ---------------------------------------------------------------------------
// Big owners: persistent workgroups with an LDS bitmap window.

constexpr int kBigThreads = 1024;
constexpr int kUnroll = 4;   // loads in flight per lane
constexpr int kSeg = 1024;   // ids per work item (rows longer than this are split)

struct BigShared {
  int32_t chunk;
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

// One workgroup per chunk (owner h, up to spc row slots), persistent over a
// global chunk counter. Per id window: the owner's ids in the window are set
// in the LDS bitmap; each lower neighbour's ids in the window are cut into
// segments of kSeg ids, and wavefronts claim segments from an LDS counter
// (item j < nlow is the first segment of edge j; later items are the extra
// segments of long rows), so one long row cannot hold the workgroup at the
// barrier that ends the window. Partial counts meet in LDS.
template <bool kOneWindow>
__global__ __launch_bounds__(kBigThreads) void k_big_owner(
    const BigChunk *chunks, int32_t nchunks, PlanCounts *pc, int spc, int wbits, int64_t n,
    const int64_t *off, const int32_t *deg, const int32_t *adj, int kind, double *sims,
    int32_t *counts) {
  extern __shared__ unsigned char smem[];
  const int64_t W = (int64_t)1 << wbits;
  const int nwords = (int)(W >> 5);
  uint32_t *bm = (uint32_t *)smem;
  int64_t *le_ou = (int64_t *)(bm + nwords);
  int64_t *le_mir = le_ou + spc;
  int32_t *le_e = (int32_t *)(le_mir + spc);
  int32_t *le_du = le_e + spc;
  int32_t *le_cnt = le_du + spc;
  int32_t *le_b0 = le_cnt + spc;
  int32_t *le_b1 = le_b0 + spc;  // end of the range in the current window (cursor)
  int32_t *le_xp = le_b1 + spc;  // [spc + 1] exclusive prefix of extra segments
  BigShared *sh = (BigShared *)(le_xp + spc + 1);
  const int tid = threadIdx.x, lane = lane_id();
  constexpr bool one_window = kOneWindow;  // the whole id space fits one window

  for (int i = tid; i < nwords; i += blockDim.x) bm[i] = 0u;
  for (;;) {
    __syncthreads();
    if (tid == 0) {
      sh->chunk = atomicAdd(&pc->counter, 1);
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
        low = is_lower(u, du, h, dh);
      }
      const uint64_t mk = __ballot(low);
      int32_t base = 0;
      if (mk) {
        const int leader = __ffsll((unsigned long long)mk) - 1;
        base = __builtin_amdgcn_readlane(atomicAdd(&sh->nlow, lane == leader ? __popcll(mk) : 0), leader);
      }
      if (low) {
        const int k = base + __popcll(mk & lanes_below());
        le_e[k] = e;
        le_du[k] = du;
        le_ou[k] = off[u];
        le_cnt[k] = 0;
        le_mir[k] = -1;
        le_b0[k] = 0;
        le_b1[k] = one_window ? du : 0;
      }
    }
    __syncthreads();
    const int nlow = uniform(sh->nlow);
    if (nlow == 0) continue;
    // Windows of ids [w0, w0 + W) that hold ids of N(h), in increasing order.
    int64_t p = 0;
    while (p < dh) {
      const int64_t w0 = one_window ? 0 : ((int64_t)adj[oh + p] >> wbits) << wbits;
      const int64_t pe = one_window ? dh : wave_lower_bound(adj + oh, p, dh, (int32_t)min(w0 + W, (int64_t)INT32_MAX));
      for (int64_t i = p + tid; i < pe; i += blockDim.x) {
        const int32_t x = (int32_t)(adj[oh + i] - w0);
        atomicOr(&bm[x >> 5], 1u << (x & 31));
      }
      if (!one_window) {
        // each lower neighbour's ids inside this window, after the last one
        if (tid == 0) sh->next = 0;
        __syncthreads();
        for (;;) {
          const int32_t i = uniform(atomicAdd(&sh->next, lane == 0 ? 1 : 0));
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
        ex = len > kSeg ? (len - 1) / kSeg : 0;
      }
      const int32_t xp = block_excl_scan(ex, sh->wsum, &sh->nextra);
      if (tid < nlow) le_xp[tid] = xp;
      if (tid == 0) sh->next = 0;
      __syncthreads();
      const int32_t nitems = nlow + uniform(sh->nextra);
      // Software pipeline over work items: the next item is claimed and its
      // first kWave*kUnroll ids are requested before the current item's ids
      // are probed, so two items' loads are in flight per wavefront.
      auto claim = [&](int32_t &e, int32_t &lo, int32_t &hi, int64_t &ou) {
        const int32_t j = uniform(atomicAdd(&sh->next, lane == 0 ? 1 : 0));
        if (j >= nitems) {
          e = -1;
          lo = hi = 0;
          ou = 0;
          return;
        }
        int32_t ee = j, sg = 0;
        if (j >= nlow) {
          const int32_t jj = j - nlow;
          int32_t a0 = 0, a1 = nlow;  // last edge with le_xp[e] <= jj
          while (a1 - a0 > 1) {
            const int32_t mid = (a0 + a1) >> 1;
            if (uniform(le_xp[mid]) <= jj) a0 = mid;
            else a1 = mid;
          }
          ee = a0;
          sg = 1 + jj - uniform(le_xp[a0]);
        }
        e = ee;
        ou = uniform64(le_ou[ee]);
        lo = uniform(le_b0[ee]) + sg * kSeg;
        hi = min(uniform(le_b1[ee]), lo + kSeg);
      };
      // Branch-free loads (a lane past the end reads adj[0] and discards it)
      // keep the loads unconditional, so the compiler waits only for the ones
      // it consumes.
      // Loads are branch-free (a lane past the end re-reads the row's first
      // id and discards it) and their values are only read by the probe, so
      // the compiler waits only for the loads it consumes. Hits and the
      // position of h are kept per lane and reduced once per item.
      // Validity is applied with masks, not branches (mask = all ones for a
      // lane inside the item, zero past its end).
      auto fetch = [&](int32_t x[kUnroll], const int32_t *row, uint32_t base, uint32_t hi) {
#pragma unroll
        for (int k = 0; k < kUnroll; ++k) {
          const uint32_t q = base + k * kWave + lane;
          const uint32_t vm = 0u - (uint32_t)(q < hi);
          x[k] = row[q & vm];
        }
      };
      auto probe = [&](const int32_t x[kUnroll], uint32_t base, uint32_t hi, int32_t &cnt,
                       int32_t &mpi) {
#pragma unroll
        for (int k = 0; k < kUnroll; ++k) {
          const uint32_t q = base + k * kWave + lane;
          const uint32_t vb = (uint32_t)(q < hi);
          const uint32_t vm = 0u - vb;
          // inside [lo, hi) every id lies in the current window
          const uint32_t y = kOneWindow ? (uint32_t)x[k] : (uint32_t)(x[k] - (int32_t)w0);
          const uint32_t word = bm[(y >> 5) & vm];
          cnt += (int32_t)((word >> (y & 31u)) & vb);
          const uint32_t eq = (uint32_t)(x[k] == h) & vb;
          mpi = eq ? (int32_t)q : mpi;
        }
      };
      int32_t ea, loa, hia;
      int64_t oua;
      int32_t xa[kUnroll];
      claim(ea, loa, hia, oua);
      fetch(xa, adj + oua, (uint32_t)loa, (uint32_t)hia);
      while (ea >= 0) {
        int32_t eb, lob, hib;
        int64_t oub;
        int32_t xb[kUnroll];
        claim(eb, lob, hib, oub);
        fetch(xb, adj + oub, (uint32_t)lob, (uint32_t)hib);
        int32_t cnt = 0, mpi = -1;
        probe(xa, (uint32_t)loa, (uint32_t)hia, cnt, mpi);
        for (int32_t base = loa + kWave * kUnroll; base < hia; base += kWave * kUnroll) {
          int32_t x[kUnroll];
          fetch(x, adj + oua, (uint32_t)base, (uint32_t)hia);
          probe(x, (uint32_t)base, (uint32_t)hia, cnt, mpi);
        }
        const int32_t t = wave_sum(cnt);
        const int32_t mp = wave_max(mpi);
        // t and mp are wave-uniform; lane 0 adds, every lane stores the mirror.
        atomicAdd(&le_cnt[ea], lane == 0 ? t : 0);
        if (mp >= 0) le_mir[ea] = oua + mp;
        ea = eb;
        loa = lob;
        hia = hib;
        oua = oub;
#pragma unroll
        for (int k = 0; k < kUnroll; ++k) xa[k] = xb[k];
      }
      __syncthreads();
      for (int64_t i = p + tid; i < pe; i += blockDim.x) {
        const int32_t x = (int32_t)(adj[oh + i] - w0);
        bm[x >> 5] = 0u;
      }
      p = pe;
      // the next window's bits may share words with the ones just cleared
      if (!one_window) __syncthreads();
    }
    __syncthreads();
    for (int i = tid; i < nlow; i += blockDim.x) {
      int64_t mir = le_mir[i];
      if (!one_window) {
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

// ---------------------------------------------------------------------------
// Host side.

static size_t big_lds_bytes(int wbits, int spc) {
  return ((size_t)1 << wbits) / 8 + (size_t)spc * (8 + 8 + 4 * 6) + 4 + sizeof(BigShared);
}

scan_status intersect_all(const IntersectConfig &cfg, int64_t n, int64_t nnz, const int64_t *off,
                          const int32_t *deg, const int32_t *adj, int kind, double *sims,
                          int32_t *counts, int device, hipStream_t s, IntersectStats *stats) {
  if (nnz == 0) return SCAN_OK;
  int lds_max = 65536, cus = 256;
  (void)hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, device);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
  int wbits = cfg.wbits;
  int nb = 0;
  while (((int64_t)1 << nb) < n) ++nb;
  if (nb < 10) nb = 10;
  if (wbits > nb) wbits = nb;  // no wider than the id space
  while (wbits > 10 && big_lds_bytes(wbits, cfg.spc) > (size_t)lds_max) --wbits;
  if (big_lds_bytes(wbits, cfg.spc) > (size_t)lds_max) return fail(SCAN_EINVAL, "chunk size too large for LDS");

  DevArena tmp(s);
  int32_t *small_list;
  BigChunk *big_list;
  PlanCounts *pc;
  const int64_t big_cap = nnz / cfg.spc + n + 1;
  SCAN_TRY(tmp.alloc(&small_list, n));
  SCAN_TRY(tmp.alloc(&big_list, big_cap));
  SCAN_TRY(tmp.alloc(&pc, 1));
  SCAN_HIP_TRY(hipMemsetAsync(pc, 0, sizeof(PlanCounts), s));
  k_plan<<<grid_for(n, 256, 8192), 256, 0, s>>>(off, deg, adj, n, cfg.small_max, cfg.spc,
                                                 small_list, big_list, pc);
  PlanCounts h;
  SCAN_HIP_TRY(hipMemcpyAsync(&h, pc, sizeof(h), hipMemcpyDeviceToHost, s));
  SCAN_HIP_TRY(hipStreamSynchronize(s));
  if (stats) {
    stats->owners_small = h.small;
    stats->chunks_big = h.big;
    stats->wbits = wbits;
    if (stats->ev_start) (void)hipEventRecord(stats->ev_start, s);
  }
  if (h.small) {
    size_t lds = (size_t)cfg.small_max * 16;
    k_small_owner<<<grid_for(h.small, 1, 1 << 20), kWave, lds, s>>>(
        small_list, h.small, cfg.small_max, off, deg, adj, kind, sims, counts);
    SCAN_HIP_TRY(hipGetLastError());
  }
  if (h.big) {
    size_t lds = big_lds_bytes(wbits, cfg.spc);
    const bool one = n <= ((int64_t)1 << wbits);
    const void *fn = one ? (const void *)k_big_owner<true> : (const void *)k_big_owner<false>;
    if (lds > 65536)
      SCAN_HIP_TRY(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    int per_cu = (int)std::max<size_t>(1, std::min<size_t>(2, (size_t)lds_max / lds));
    int grid = std::min<int64_t>((int64_t)cus * per_cu, h.big);
    if (one)
      k_big_owner<true><<<grid, kBigThreads, lds, s>>>(big_list, h.big, pc, cfg.spc, wbits, n, off,
                                                       deg, adj, kind, sims, counts);
    else
      k_big_owner<false><<<grid, kBigThreads, lds, s>>>(big_list, h.big, pc, cfg.spc, wbits, n, off,
                                                        deg, adj, kind, sims, counts);
    SCAN_HIP_TRY(hipGetLastError());
  }
  if (stats && stats->ev_end) (void)hipEventRecord(stats->ev_end, s);
  return SCAN_OK;
}

}  // namespace scan
