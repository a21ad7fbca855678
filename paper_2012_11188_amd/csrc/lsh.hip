// Approximate similarities (Section 5) with the degree heuristic of Section
// 6.3: only edges between two high-degree vertices (degree > k for cosine,
// > 3k/2 for Jaccard) are approximated; every other edge keeps the exact
// similarity computed before this pass. The random draws are inputs.
//
//   SimHash (cosine, optionally weighted): bit i of v's sketch is 1 iff the
//   dot product of N[v] (weights w(v, x), w(v, v) = 1) with direction i,
//   gauss[x * k + i], is >= 0, the dot product summed term by term in
//   ascending x. Estimate cos(pi h / k) for h differing bits, read from a
//   table of the k + 1 values computed once on the host.
//   k-partition MinHash (Jaccard): bin(x) = floor(perm[x] * k / n); entry b of
//   v's sketch is the least perm[x] over x in N[v] in bin b (0xffffffff when
//   none). Estimate: matching non-empty bins / (k - bins empty in both).
//
//   k_simhash_big  workgroups resident on every CU claim (high vertex, group
//                of 64 directions) items from a counter; per item its
//                wavefronts gather the coordinates of kShChunk row entries
//                into LDS, then one of them adds them in ascending x (lane i:
//                direction g * 64 + i); the signs form one 64-bit word by
//                ballot.
//   k_minhash    one wavefront per high vertex: k bins in LDS, atomicMin of
//                perm[x] over N[v].
//   k_estimate   one wavefront per piece of 64 slots of a high vertex's row
//                (pieces numbered by a prefix over the vertices): the slots
//                whose other end is high too are overwritten.
#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>
#include <vector>

#include "index.h"

namespace scan {
namespace {

constexpr int kLshThreads = 256;
constexpr int kLshWaves = kLshThreads / kWave;
constexpr int kLshPiece = 64;  // row slots per estimate work item
constexpr int kShChunk = 64;     // row entries staged in LDS per round of the block kernel
constexpr int kShThreads = 256;
constexpr int kShUnroll = 8;     // entries whose LDS values the summing wave reads ahead
constexpr int kShWaves = kShThreads / kWave;
constexpr int kMhGroup = 16;   // lanes comparing one pair of MinHash sketches

__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }
__device__ __forceinline__ int32_t uniform(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t uniform64(int64_t v) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)(uint32_t)v);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)(uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ bool high(int kind, int64_t deg, int64_t k) {
  return kind == SCAN_SIM_JACCARD ? 2 * deg > 3 * k : deg > k;
}

// big[] = the high vertices, *nbig their number.
__global__ void k_simhash_list(const int64_t *off, int64_t n, int32_t k, int32_t *big, int32_t *nbig) {
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    const int64_t d = off[v + 1] - off[v];
    if (high(SCAN_SIM_COSINE, d, k)) big[atomicAdd(nbig, 1)] = (int32_t)v;
  }
}

// SimHash words, words[v * (k / 64) + g] with bit i for direction g * 64 + i:
// one item per (high vertex, group of 64 directions). The grid is what the
// CUs hold at once, and each workgroup claims its next item from *claim as
// soon as it is done (item sizes follow the degrees, so a static split would
// leave most workgroups idle behind the longest lists). Per round, all waves
// gather the coordinates of kShChunk row entries into LDS (a wave's gathers
// are issued back to back, so hundreds are in flight at once), then wave 0
// adds them in ascending order, lane i for direction g * 64 + i, with the
// self term at its place.
__global__ __launch_bounds__(kShThreads) void k_simhash_big(const int64_t *off, const int32_t *adj, const double *w,
                                                            const double *gauss, int32_t k, const int32_t *big,
                                                            const int32_t *nbig, unsigned long long *claim,
                                                            uint64_t *words) {
  extern __shared__ double st[];           // [kShChunk][64] coordinates
  __shared__ int32_t sid[kShChunk];        // the entries' ids
  __shared__ double sw[kShChunk];          // and weights
  __shared__ int64_t s_item;
  const int lane = lane_id(), wave = threadIdx.x / kWave;
  const int32_t groups = k / kWave;
  const int64_t items = (int64_t)uniform(*nbig) * groups;
  for (;;) {
    if (threadIdx.x == 0) s_item = (int64_t)atomicAdd(claim, 1ull);
    __syncthreads();
    const int64_t t = s_item;
    if (t >= items) break;  // uniform across the block
    const int64_t v = big[t / groups];
    const int32_t g = (int32_t)(t % groups);
    const int64_t o = uniform64(off[v]), d = uniform64(off[v + 1]) - o;
    const double *col = gauss + g * kWave + lane;
    double acc = 0.0;
    bool self = false;
    for (int64_t c = 0; c < d; c += kShChunk) {
      const int m = (int)(d - c < kShChunk ? d - c : kShChunk);
      __syncthreads();  // the previous round's readers are done
      // entries wave, wave + kShWaves, ...: ids first (one vector load), then
      // every gather of the wave, then the LDS stores
      constexpr int kPer = kShChunk / kShWaves;
      const int jl = wave + kShWaves * lane;  // the entry whose id this lane loads
      const int32_t xl = jl < m ? adj[o + c + jl] : 0;
      if (lane < kPer && jl < m) {
        sid[jl] = xl;
        sw[jl] = w ? w[o + c + jl] : 1.0;
      }
      double gv[kPer];
#pragma unroll
      for (int q = 0; q < kPer; ++q) gv[q] = col[(int64_t)__builtin_amdgcn_readlane(xl, q) * k];
#pragma unroll
      for (int q = 0; q < kPer; ++q)
        if (wave + kShWaves * q < m) st[(wave + kShWaves * q) * kWave + lane] = gv[q];
      __syncthreads();
      if (wave == 0) {
        for (int j0 = 0; j0 < m; j0 += kShUnroll) {
          int32_t xs[kShUnroll];
          double ws[kShUnroll], gs[kShUnroll];
#pragma unroll
          for (int u = 0; u < kShUnroll; ++u) {  // entries past m read stale LDS and are not added
            xs[u] = sid[j0 + u];
            ws[u] = sw[j0 + u];
            gs[u] = st[(j0 + u) * kWave + lane];
          }
#pragma unroll
          for (int u = 0; u < kShUnroll; ++u) {
            if (j0 + u < m) {
              if (!self && xs[u] > v) {
                acc += 1.0 * col[v * (int64_t)k];
                self = true;
              }
              acc += ws[u] * gs[u];
            }
          }
        }
      }
    }
    if (wave == 0) {
      if (!self) acc += 1.0 * col[v * (int64_t)k];
      const uint64_t bits = __ballot(acc >= 0.0);
      if (lane == 0) words[v * groups + g] = bits;
    }
    __syncthreads();  // every thread has read s_item before the next claim
  }
}

// sk[v * k + b]; the block's waves take one vertex each, bins in LDS.
__global__ __launch_bounds__(kLshThreads) void k_minhash(const int64_t *off, const int32_t *adj, const uint32_t *perm,
                                                         int64_t n, int32_t k, uint32_t *sk) {
  extern __shared__ uint32_t bins[];  // [kLshWaves][k]
  const int lane = lane_id(), wave = threadIdx.x / kWave;
  uint32_t *mine = bins + (size_t)wave * k;
  const int64_t waves = (int64_t)gridDim.x * kLshWaves;
  for (int64_t v = uniform64((int64_t)blockIdx.x * kLshWaves + wave); v < n; v += waves) {
    const int64_t o = uniform64(off[v]), d = uniform64(off[v + 1]) - o;
    if (!high(SCAN_SIM_JACCARD, d, k)) continue;
    for (int32_t b = lane; b < k; b += kWave) mine[b] = 0xffffffffu;
    for (int64_t c = -1; c < d; c += kWave) {  // position -1 is v itself
      const int64_t p = c + lane;
      if (p < d) {
        const int64_t x = p < 0 ? v : adj[o + p];
        const uint32_t px = perm[x];
        atomicMin(&mine[(uint64_t)px * (uint64_t)k / (uint64_t)n], px);
      }
    }
    for (int32_t b = lane; b < k; b += kWave) sk[v * k + b] = mine[b];
  }
}

// cnt[u] = pieces of kLshPiece slots of u's row when u is high, else 0.
__global__ void k_lsh_pieces(const int64_t *off, int64_t n, int kind, int32_t k, int32_t *cnt) {
  for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < n; u += (int64_t)gridDim.x * blockDim.x) {
    const int64_t d = off[u + 1] - off[u];
    cnt[u] = high(kind, d, k) ? (int32_t)((d + kLshPiece - 1) / kLshPiece) : 0;
  }
}

// One wavefront per piece (P = exclusive prefix of the pieces, P[n] their
// number): the piece's slots whose other end is high too get the estimate.
// SimHash: a lane per slot. MinHash: four groups of 16 lanes, a group per
// slot; lane l of a group compares bins 4 (l + 16 i) .. 4 (l + 16 i) + 3, so
// each load instruction of a group reads 256 contiguous bytes of a sketch.
__global__ __launch_bounds__(kLshThreads) void k_estimate(const int64_t *off, const int32_t *adj, int64_t n,
                                                          int kind, int32_t k, const int64_t *P,
                                                          const uint64_t *words, const uint32_t *sk,
                                                          const double *table, double *sims) {
  const int lane = lane_id();
  const int64_t waves = (int64_t)gridDim.x * kLshWaves;
  const int64_t T = uniform64(P[n]);
  for (int64_t t = uniform64(((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave); t < T; t += waves) {
    int64_t lo = 0, hi = n;  // the u with P[u] <= t < P[u + 1]
    while (hi - lo > 1) {
      const int64_t mid = (lo + hi) >> 1;
      if (uniform64(P[mid]) <= t) lo = mid;
      else hi = mid;
    }
    const int64_t u = lo, o = uniform64(off[u]), d = uniform64(off[u + 1]) - o;
    const int64_t p0 = (t - uniform64(P[u])) * kLshPiece;
    if (kind != SCAN_SIM_JACCARD) {
      const int64_t p = p0 + lane;
      if (p < d && p < p0 + kLshPiece) {
        const int64_t v = adj[o + p];
        if (high(kind, off[v + 1] - off[v], k)) {
          const int32_t groups = k / kWave;
          int32_t h = 0;
          for (int32_t i = 0; i < groups; ++i) h += __popcll(words[u * groups + i] ^ words[v * groups + i]);
          sims[o + p] = table[h];
        }
      }
      continue;
    }
    const int grp = lane / kMhGroup, gl = lane % kMhGroup;
    for (int r = 0; r < kLshPiece / (kWave / kMhGroup); ++r) {
      const int64_t p = p0 + r * (kWave / kMhGroup) + grp;
      bool on = p < d;
      int64_t v = 0;
      if (on) {
        v = adj[o + p];
        on = high(kind, off[v + 1] - off[v], k);
      }
      int32_t match = 0, empty = 0;
      if (on) {
        const uint4 *a = (const uint4 *)(sk + u * k), *b = (const uint4 *)(sk + v * k);
        for (int32_t i = gl; i < k / 4; i += kMhGroup) {
          const uint4 ea = a[i], eb = b[i];
          const uint32_t av[4] = {ea.x, ea.y, ea.z, ea.w}, bv[4] = {eb.x, eb.y, eb.z, eb.w};
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            if (av[j] == 0xffffffffu && bv[j] == 0xffffffffu) ++empty;
            else if (av[j] == bv[j]) ++match;
          }
        }
      }
      for (int m = kMhGroup / 2; m > 0; m >>= 1) {  // sums over the group (all lanes take part)
        match += __shfl_xor(match, m, kWave);
        empty += __shfl_xor(empty, m, kWave);
      }
      if (on && gl == 0) sims[o + p] = (double)match / (double)(k - empty);
    }
  }
}

// err[0] = 1 if some perm value is not below n.
__global__ void k_perm_check(const uint32_t *perm, int64_t n, int32_t *err) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    if ((int64_t)perm[i] >= n) err[0] = 1;
}

}  // namespace

scan_status lsh_overwrite(const LshSpec &spec, int64_t n, int64_t nnz, const int64_t *off, const int32_t *adj,
                          const double *w, int kind, double *sims, DevArena &tmp, hipStream_t s) {
  const int32_t k = spec.samples;
  if (n == 0 || nnz == 0) return SCAN_OK;
  uint64_t *words = nullptr;
  uint32_t *sk = nullptr;
  double *table = nullptr;
  if (kind == SCAN_SIM_JACCARD) {
    int32_t *d_err;
    SCAN_TRY(tmp.alloc(&d_err, 1));
    SCAN_HIP_TRY(hipMemsetAsync(d_err, 0, 4, s));
    k_perm_check<<<grid_for(n, 256), 256, 0, s>>>(spec.perm, n, d_err);
    int32_t herr = 0;
    SCAN_HIP_TRY(hipMemcpyAsync(&herr, d_err, 4, hipMemcpyDeviceToHost, s));
    SCAN_HIP_TRY(hipStreamSynchronize(s));
    if (herr) return fail(SCAN_EINVAL, "MinHash permutation values must lie in [0, n)");
    SCAN_TRY(tmp.alloc(&sk, n * (int64_t)k));
    const size_t lds = (size_t)kLshWaves * k * 4;
    if (lds > 65536)
      SCAN_HIP_TRY(hipFuncSetAttribute((const void *)k_minhash, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    k_minhash<<<grid_for(n, kLshWaves), kLshThreads, lds, s>>>(off, adj, spec.perm, n, k, sk);
  } else {
    std::vector<double> t(k + 1);
    for (int32_t h = 0; h <= k; ++h) t[h] = std::cos(M_PI * (double)h / (double)k);
    SCAN_TRY(tmp.alloc(&table, k + 1));
    SCAN_HIP_TRY(hipMemcpyAsync(table, t.data(), t.size() * 8, hipMemcpyHostToDevice, s));
    SCAN_TRY(tmp.alloc(&words, n * (int64_t)(k / kWave)));
    int32_t *big, *nbig;
    unsigned long long *claim;
    SCAN_TRY(tmp.alloc(&big, n));
    SCAN_TRY(tmp.alloc(&nbig, 1));
    SCAN_TRY(tmp.alloc(&claim, 1));
    SCAN_HIP_TRY(hipMemsetAsync(nbig, 0, 4, s));
    SCAN_HIP_TRY(hipMemsetAsync(claim, 0, 8, s));
    k_simhash_list<<<grid_for(n, 256), 256, 0, s>>>(off, n, k, big, nbig);
    const size_t lds = (size_t)kShChunk * kWave * 8;
    SCAN_HIP_TRY(hipFuncSetAttribute((const void *)k_simhash_big, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    int device = 0, cus = 256, per_cu = 0;
    (void)hipGetDevice(&device);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)k_simhash_big, kShThreads, lds) !=
            hipSuccess ||
        per_cu < 1) {
      (void)hipGetLastError();
      per_cu = 1;
    }
    k_simhash_big<<<cus * per_cu, kShThreads, lds, s>>>(off, adj, w, spec.gauss, k, big, nbig, claim, words);
  }
  int32_t *cnt;
  int64_t *P, *ws;
  SCAN_TRY(tmp.alloc(&cnt, n));
  SCAN_TRY(tmp.alloc(&P, n + 1));
  SCAN_TRY(tmp.alloc(&ws, scan_workspace_elems(n)));
  k_lsh_pieces<<<grid_for(n, 256), 256, 0, s>>>(off, n, kind, k, cnt);
  SCAN_TRY(exclusive_scan(cnt, P, n, ws, s));
  k_estimate<<<grid_for(n * kWave / 16, kLshThreads), kLshThreads, 0, s>>>(off, adj, n, kind, k, P, words, sk, table,
                                                                          sims);
  SCAN_HIP_TRY(hipGetLastError());
  if (kind != SCAN_SIM_JACCARD) SCAN_HIP_TRY(hipStreamSynchronize(s));  // the host table stays alive until here
  return SCAN_OK;
}

}  // namespace scan
