// Weighted cosine similarity (Section 3.1; Algorithm 1 is written for this
// measure). For adjacent u, v:
//   sigma(u, v) = D(u, v) / sqrt(S_u * S_v),
//   D(u, v) = sum over x in N[u] ∩ N[v] of w(u, x) w(v, x),
//   S_v     = sum over x in N[v] of w(v, x)^2,
// over closed neighbourhoods with w(x, x) = 1; w(u, x) is the weight stored in
// u's CSR slot for x. The paper leaves the order of these floating-point sums
// open. Here every sum adds its terms one at a time in ascending x, so each
// similarity is one fixed FP64 value (no FP contraction, IEEE sqrt and
// division); with all weights 1 the sums are the integers c, a_u and a_v and
// the result is the unweighted cosine bit for bit.
//
//   k_w_square_sums  one wavefront per vertex: the squares of its row, added
//                    in order with the self term 1 at its place.
//   k_w_unit_rows    the row holding the first slot of every kWUnit-slot unit
//                    of the CSR.
//   k_w_owner        one workgroup per unit. Each edge is handled once, by the
//                    endpoint larger in (degree, id) (the owner h, as in the
//                    unweighted path). The owner's ids and weights go into LDS
//                    in tiles of kWTile; every lower neighbour l streams its
//                    row through them in ascending order, a lane finds its id
//                    by binary search in its bucket of the tile (kWBuckets
//                    buckets of equal id width, indexed per tile), and the
//                    wavefront adds the products of the common ids in
//                    ascending id, inserting the terms of x = h (1 * w(l, h))
//                    and x = l (w(h, l) * 1).
#include <hip/hip_runtime.h>

#include <climits>

#include "index.h"

namespace scan {
namespace {

constexpr int kWUnit = 128;                  // CSR slots per workgroup
constexpr int kWThreads = 256;
constexpr int kWWaves = kWThreads / kWave;
constexpr int kWTile = 1024;                 // owner ids (and weights) per LDS tile
constexpr int kWBuckets = 512;               // id buckets per tile (a lookup's first guess)
constexpr int kWRows = 64;                   // row offsets staged at a time
#ifndef SCAN_W_CHUNKS
#define SCAN_W_CHUNKS 4
#endif
constexpr int kWChunks = SCAN_W_CHUNKS;      // 64-id chunks of a lower row loaded at once

__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }
__device__ __forceinline__ int32_t uniform(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t uniform64(int64_t v) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)(uint32_t)v);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)(uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}
// Lane k's double (k wave-uniform).
__device__ __forceinline__ double lane_f64(double v, int k) {
  const uint64_t b = (uint64_t)__double_as_longlong(v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int32_t)(uint32_t)b, k);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int32_t)(uint32_t)(b >> 32), k);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// Lanes past the end of a row re-read its last slot (clamped, so the id and
// weight loads need no branch and are issued together) and contribute +0.0,
// which leaves a non-negative running sum unchanged.
__global__ __launch_bounds__(256) void k_w_square_sums(const int64_t *off, const int32_t *adj, const double *w,
                                                       int64_t n, double *S) {
  const int lane = lane_id();
  const int64_t waves = (int64_t)gridDim.x * (blockDim.x / kWave);
  for (int64_t v = uniform64(((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave); v < n; v += waves) {
    const int64_t o = uniform64(off[v]), d = uniform64(off[v + 1]) - o;
    double acc = 0.0;
    bool self = false;
    int32_t xr = 0;  // raw loads of the chunk in flight (masked where used)
    double wr = 0.0;
    auto fetch = [&](int64_t c) {
      const int64_t p = c + lane;
      const int64_t q = o + (p < d ? p : d - 1);
      xr = adj[q];
      wr = w[q];
    };
    if (d > 0) fetch(0);
    for (int64_t c = 0; c < d; c += kWave) {
      const bool in = c + lane < d;
      const double wx = in ? wr : 0.0;
      const double sq = wx * wx;
      const uint64_t above = __ballot(in && xr > v);
      if (c + kWave < d) fetch(c + kWave);  // the next chunk's loads overlap this chunk's sum
      if (!self && above) {                 // the self term 1 goes before the first id above v
        const int fa = __ffsll((unsigned long long)above) - 1;
#pragma unroll
        for (int k = 0; k < kWave; ++k) {
          if (k == fa) acc += 1.0;
          acc += lane_f64(sq, k);
        }
        self = true;
      } else {
#pragma unroll
        for (int k = 0; k < kWave; ++k) acc += lane_f64(sq, k);
      }
    }
    if (!self) acc += 1.0;
    if (lane == 0) S[v] = acc;
  }
}

// row_of[k] = the row holding slot k * kWUnit (rows are non-empty there).
__global__ void k_w_unit_rows(const int64_t *off, int64_t n, int32_t *row_of) {
  for (int64_t h = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; h < n; h += (int64_t)gridDim.x * blockDim.x) {
    const int64_t a = off[h], b = off[h + 1];
    for (int64_t k = (a + kWUnit - 1) / kWUnit; k * kWUnit < b; ++k) row_of[k] = (int32_t)h;
  }
}

struct WShared {
  int32_t tid[kWTile];      // the owner's ids of the current tile
  double tw[kWTile];        // and their weights w(h, x)
  int32_t bst[kWBuckets + 1];  // first tile position of each id bucket (then tn)
  int64_t roff[kWRows + 1];  // off[base .. base + kWRows]
  int64_t lou[kWUnit];      // row offset of the j-th lower neighbour
  double acc[kWUnit];       // its running dot product
  double whl[kWUnit];       // w(h, l): the weight in h's slot for l
  int32_t le[kWUnit];       // that slot
  int32_t lid[kWUnit];      // l
  int32_t ldu[kWUnit];      // deg(l)
  int32_t cur[kWUnit];      // first position of l's row not yet streamed
  int32_t nxt[kWUnit];      // the id there (INT_MIN before the first tile)
  int32_t mpos[kWUnit];     // position of h in l's row (the mirror slot)
  int32_t ldone[kWUnit];    // 1 once the x = l term is added
  int32_t nlow;
};

__global__ __launch_bounds__(kWThreads) void k_w_owner(const int64_t *off, const int32_t *deg, const int32_t *adj,
                                                       const double *w, const double *S, const int32_t *row_of,
                                                       int64_t n, int64_t nnz, double *sims, int32_t skip) {
  __shared__ WShared sh;
  const int lane = lane_id(), wave = threadIdx.x / kWave;
  const int64_t s0 = (int64_t)blockIdx.x * kWUnit, s1 = s0 + kWUnit < nnz ? s0 + kWUnit : nnz;
  int64_t h = row_of[blockIdx.x], base = -1;
  for (;;) {
    if (base < 0 || h + 1 > base + kWRows) {  // stage the next kWRows row offsets
      __syncthreads();
      base = h;
      for (int i = threadIdx.x; i <= kWRows; i += blockDim.x) sh.roff[i] = off[base + i < n ? base + i : n];
      __syncthreads();
    }
    const int64_t ra = uniform64(sh.roff[h - base]), rb = uniform64(sh.roff[h + 1 - base]);
    if (ra >= s1) break;  // uniform across the block
    const int64_t a = ra > s0 ? ra : s0, b = rb < s1 ? rb : s1;
    if (a < b) {
      const int32_t dh = (int32_t)(rb - ra);
      if (threadIdx.x == 0) sh.nlow = 0;
      __syncthreads();
      // The lower neighbours among slots [a, b), compacted into LDS.
      {
        const int64_t slot = a + threadIdx.x;
        int32_t u = 0, du = 0;
        const bool in = slot < b;
        if (in) {
          u = adj[slot];
          du = deg[u];
        }
        const bool low = in && (du < dh || (du == dh && u < h)) && du <= skip;
        const uint64_t m = __ballot(low);
        int32_t j0 = 0;
        if (m) {
          const int leader = __ffsll((unsigned long long)m) - 1;
          j0 = __builtin_amdgcn_readlane(atomicAdd(&sh.nlow, lane == leader ? __popcll(m) : 0), leader);
        }
        if (low) {
          const int j = j0 + __popcll(m & ((1ull << lane) - 1ull));
          sh.le[j] = (int32_t)(slot - ra);
          sh.lid[j] = u;
          sh.ldu[j] = du;
          sh.lou[j] = off[u];
          sh.whl[j] = w[slot];
          sh.acc[j] = 0.0;
          sh.cur[j] = 0;
          sh.nxt[j] = INT_MIN;
          sh.mpos[j] = -1;
          sh.ldone[j] = 0;
        }
      }
      __syncthreads();
      const int32_t nlow = uniform(sh.nlow);
      for (int32_t t0 = 0; nlow > 0 && t0 < dh; t0 += kWTile) {
        const int32_t tn = dh - t0 < kWTile ? dh - t0 : kWTile;
        __syncthreads();  // the previous tile's readers are done
        for (int i = threadIdx.x; i < tn; i += blockDim.x) {
          sh.tid[i] = adj[ra + t0 + i];
          sh.tw[i] = w[ra + t0 + i];
        }
        __syncthreads();
        const int32_t tlo = uniform(sh.tid[0]), hi = uniform(sh.tid[tn - 1]);
        // Buckets of 2^tsh ids from tlo: bucket b holds positions
        // [bst[b], bst[b + 1]) (every entry written once, by the position
        // that opens it, or by the last position for the empty tail).
        int tsh = 0;
        while (((hi - tlo) >> tsh) >= kWBuckets) ++tsh;
        const int32_t nb = ((hi - tlo) >> tsh) + 1;
        for (int i = threadIdx.x; i < tn; i += blockDim.x) {
          const int32_t bi = (sh.tid[i] - tlo) >> tsh;
          const int32_t bp = i > 0 ? (sh.tid[i - 1] - tlo) >> tsh : -1;
          for (int32_t b = bp + 1; b <= bi; ++b) sh.bst[b] = i;
          if (i == tn - 1)
            for (int32_t b = bi + 1; b <= nb; ++b) sh.bst[b] = tn;
        }
        __syncthreads();
        const bool last = t0 + kWTile >= dh;
        for (int32_t j = wave; j < nlow; j += kWWaves) {
          if (!last && uniform(sh.nxt[j]) > hi) continue;  // nothing of l's row up to hi is left
          const int64_t ou = uniform64(sh.lou[j]);
          const int32_t du = uniform(sh.ldu[j]), l = uniform(sh.lid[j]);
          int32_t c = uniform(sh.cur[j]), mp = uniform(sh.mpos[j]), nx = INT_MAX;
          bool ldone = uniform(sh.ldone[j]) != 0;
          const double whl = sh.whl[j];
          double acc = sh.acc[j];
          // One chunk of 64 positions from c: returns how many were in
          // range (a prefix) and sets nx when the range ended inside it.
          auto chunk = [&](int32_t xq, double wq) {
            const bool in = c + lane < du;
            const int32_t x = in ? xq : INT_MAX;
            const double wl = in ? wq : 0.0;
            const bool valid = in && (last || x <= hi);
            // lower_bound of x in its bucket (x outside [tlo, hi]: no hit)
            const bool inr = x >= tlo && x <= hi;
            int32_t lo = 0, len = 0;
            if (inr) {
              const int32_t b = (x - tlo) >> tsh;
              lo = sh.bst[b];
              len = sh.bst[b + 1] - lo;
            }
            while (len > 0) {
              const int32_t half = len >> 1;
              if (sh.tid[lo + half] < x) {
                lo += half + 1;
                len -= half + 1;
              } else {
                len = half;
              }
            }
            const bool hit = valid && inr && lo < tn && sh.tid[lo] == x;
            const bool selfh = valid && x == (int32_t)h;
            const double prod = hit ? sh.tw[lo] * wl : wl;  // x = h: w(h, h) = 1
            const int cnt = __popcll(__ballot(valid));      // the valid lanes are a prefix
            const uint64_t hm = __ballot(selfh);
            if (hm) mp = c + __ffsll((unsigned long long)hm) - 1;
            // The products of the common ids, in lane (= ascending id)
            // order; the x = l term goes before the first of them above l.
            uint64_t cm = __ballot(hit || selfh);
            uint64_t after = 0;
            if (!ldone) {
              const uint64_t above = __ballot((hit || selfh) && x > l);
              if (above) {
                after = cm & ~((1ull << (__ffsll((unsigned long long)above) - 1)) - 1ull);
                cm &= ~after;
              }
            }
            for (; cm; cm &= cm - 1) acc += lane_f64(prod, __ffsll((unsigned long long)cm) - 1);
            if (after) {
              acc += whl;
              ldone = true;
              for (cm = after; cm; cm &= cm - 1) acc += lane_f64(prod, __ffsll((unsigned long long)cm) - 1);
            }
            if (cnt < kWave && c + cnt < du) nx = __builtin_amdgcn_readlane(x, cnt);
            return cnt;
          };
          // kWChunks chunks' loads are issued together (clamped into the
          // row, so unconditionally), then the chunks are taken in order.
          bool more = c < du;
          while (more) {
            int32_t xq[kWChunks];
            double wq[kWChunks];
#pragma unroll
            for (int u = 0; u < kWChunks; ++u) {
              const int32_t p = c + u * kWave + lane;
              const int64_t q = ou + (p < du ? p : du - 1);
              xq[u] = adj[q];
              wq[u] = w[q];
            }
#pragma unroll
            for (int u = 0; u < kWChunks; ++u) {
              if (more) {
                const int cnt = chunk(xq[u], wq[u]);
                c += cnt;
                more = cnt == kWave && c < du;
              }
            }
          }
          if (lane == 0) {
            sh.cur[j] = c;
            sh.nxt[j] = nx;
            sh.mpos[j] = mp;
            sh.ldone[j] = ldone ? 1 : 0;
            sh.acc[j] = acc;
          }
        }
      }
      __syncthreads();
      for (int32_t j = threadIdx.x; j < nlow; j += blockDim.x) {
        double acc = sh.acc[j];
        if (!sh.ldone[j]) acc += sh.whl[j];  // l is above every common id
        const int32_t l = sh.lid[j];
        const double x = acc / sqrt(S[h] * S[l]);
        sims[ra + sh.le[j]] = x;
        if (sh.mpos[j] >= 0) sims[sh.lou[j] + sh.mpos[j]] = x;
      }
      __syncthreads();  // before the next row reuses the arrays
    }
    ++h;
    if (h >= n) break;
  }
}

// err[0] = 1 if any weight is not finite.
__global__ void k_w_check(const double *w, int64_t nnz, int32_t *err) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nnz; i += (int64_t)gridDim.x * blockDim.x)
    if (!isfinite(w[i])) err[0] = 1;
}

}  // namespace

scan_status check_weights(const double *w, int64_t nnz, DevArena &tmp, hipStream_t s) {
  if (nnz == 0) return SCAN_OK;
  int32_t *d_err;
  SCAN_TRY(tmp.alloc(&d_err, 1));
  SCAN_HIP_TRY(hipMemsetAsync(d_err, 0, 4, s));
  k_w_check<<<grid_for(nnz, 256), 256, 0, s>>>(w, nnz, d_err);
  int32_t herr = 0;
  SCAN_HIP_TRY(hipMemcpyAsync(&herr, d_err, 4, hipMemcpyDeviceToHost, s));
  SCAN_HIP_TRY(hipStreamSynchronize(s));
  if (herr) return fail(SCAN_EGRAPH, "edge weights must be finite");
  return SCAN_OK;
}

scan_status weighted_similarity_all(int64_t n, int64_t nnz, const int64_t *off, const int32_t *deg,
                                    const int32_t *adj, const double *w, double *sims, DevArena &tmp,
                                    hipStream_t s, const IntersectStats *stats, int32_t skip_deg) {
  auto mark = [&](hipEvent_t e) -> scan_status {
    if (e) SCAN_HIP_TRY(hipEventRecord(e, s));
    return SCAN_OK;
  };
  SCAN_TRY(mark(stats ? stats->ev_small_begin : nullptr));
  if (nnz > 0) {
    const int64_t units = (nnz + kWUnit - 1) / kWUnit;
    if (units > INT_MAX) return fail(SCAN_EINVAL, "graph too large for the weighted path");
    double *S;
    int32_t *row_of;
    SCAN_TRY(tmp.alloc(&S, n));
    SCAN_TRY(tmp.alloc(&row_of, units));
    k_w_square_sums<<<grid_for(n * kWave, 256), 256, 0, s>>>(off, adj, w, n, S);
    k_w_unit_rows<<<grid_for(n, 256), 256, 0, s>>>(off, n, row_of);
    SCAN_HIP_TRY(hipGetLastError());
    SCAN_TRY(mark(stats ? stats->ev_small_end : nullptr));
    SCAN_TRY(mark(stats ? stats->ev_big_begin : nullptr));
    k_w_owner<<<(unsigned)units, kWThreads, 0, s>>>(off, deg, adj, w, S, row_of, n, nnz, sims, skip_deg);
    SCAN_HIP_TRY(hipGetLastError());
  } else {
    SCAN_TRY(mark(stats ? stats->ev_small_end : nullptr));
    SCAN_TRY(mark(stats ? stats->ev_big_begin : nullptr));
  }
  SCAN_TRY(mark(stats ? stats->ev_big_end : nullptr));
  return SCAN_OK;
}

}  // namespace scan
