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
//   k_simhash    one wavefront per (high vertex, group of 64 directions):
//                lane i sums direction g * 64 + i over N[v] in ascending x;
//                the signs form one 64-bit word by ballot.
//   k_minhash    one wavefront per high vertex: k bins in LDS, atomicMin of
//                perm[x] over N[v].
//   k_estimate   one wavefront per high vertex: its lanes take the row's
//                slots and overwrite those whose other end is high too.
#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>
#include <vector>

#include "index.h"

namespace scan {
namespace {

constexpr int kLshThreads = 256;
constexpr int kLshWaves = kLshThreads / kWave;
constexpr int kLshBatch = 16;  // SimHash row entries whose coordinates are loaded together

__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }
__device__ __forceinline__ int32_t uniform(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t uniform64(int64_t v) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)(uint32_t)v);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)(uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Lane j's double (j wave-uniform).
__device__ __forceinline__ double lane_f64(double v, int j) {
  const uint64_t b = (uint64_t)__double_as_longlong(v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int32_t)(uint32_t)b, j);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int32_t)(uint32_t)(b >> 32), j);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

__device__ __forceinline__ bool high(int kind, int64_t deg, int64_t k) {
  return kind == SCAN_SIM_JACCARD ? 2 * deg > 3 * k : deg > k;
}

// words[v * (k / 64) + g]: bit i is direction g * 64 + i.
__global__ __launch_bounds__(kLshThreads) void k_simhash(const int64_t *off, const int32_t *adj, const double *w,
                                                         const double *gauss, int64_t n, int32_t k,
                                                         uint64_t *words) {
  const int lane = lane_id();
  const int32_t groups = k / kWave;
  const int64_t waves = (int64_t)gridDim.x * kLshWaves;
  for (int64_t t = uniform64(((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave); t < n * groups;
       t += waves) {
    const int64_t v = t / groups;
    const int32_t g = (int32_t)(t - v * groups);
    const int64_t o = uniform64(off[v]), d = uniform64(off[v + 1]) - o;
    if (!high(SCAN_SIM_COSINE, d, k)) continue;
    const double *col = gauss + g * kWave + lane;  // direction g * 64 + lane, row x at col[x * k]
    double acc = 0.0;
    bool self = false;
    for (int64_t c = 0; c < d; c += kWave) {
      const int64_t p = c + lane;
      const int64_t q = o + (p < d ? p : d - 1);
      const int32_t xr = adj[q];
      const double wr = w ? w[q] : 1.0;
      const int m = (int)(d - c < kWave ? d - c : kWave);
      // kLshBatch row entries at a time: their coordinates are loaded
      // together (entries past m re-read entry m - 1 and are not added), then
      // added in order.
      for (int j0 = 0; j0 < m; j0 += kLshBatch) {
        int32_t xs[kLshBatch];
        double gs[kLshBatch];
#pragma unroll
        for (int u = 0; u < kLshBatch; ++u) {
          const int j = j0 + u < m ? j0 + u : m - 1;
          xs[u] = __builtin_amdgcn_readlane(xr, j);
          gs[u] = col[(int64_t)xs[u] * k];
        }
#pragma unroll
        for (int u = 0; u < kLshBatch; ++u) {
          if (j0 + u < m) {
            if (!self && xs[u] > v) {  // the self term (w(v, v) = 1) at its place
              acc += 1.0 * col[v * (int64_t)k];
              self = true;
            }
            acc += lane_f64(wr, j0 + u) * gs[u];
          }
        }
      }
    }
    if (!self) acc += 1.0 * col[v * (int64_t)k];
    const uint64_t bits = __ballot(acc >= 0.0);
    if (lane == 0) words[v * groups + g] = bits;
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

__global__ __launch_bounds__(kLshThreads) void k_estimate(const int64_t *off, const int32_t *adj, int64_t n,
                                                          int kind, int32_t k, const uint64_t *words,
                                                          const uint32_t *sk, const double *table, double *sims) {
  const int lane = lane_id();
  const int64_t waves = (int64_t)gridDim.x * kLshWaves;
  for (int64_t u = uniform64(((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave); u < n; u += waves) {
    const int64_t o = uniform64(off[u]), d = uniform64(off[u + 1]) - o;
    if (!high(kind, d, k)) continue;
    for (int64_t p = lane; p < d; p += kWave) {
      const int64_t v = adj[o + p];
      if (!high(kind, off[v + 1] - off[v], k)) continue;
      double x;
      if (kind == SCAN_SIM_JACCARD) {
        const uint4 *a = (const uint4 *)(sk + u * k), *b = (const uint4 *)(sk + v * k);
        int32_t match = 0, empty = 0;
        for (int32_t i = 0; i < k / 4; ++i) {
          const uint4 ea = a[i], eb = b[i];
          const uint32_t av[4] = {ea.x, ea.y, ea.z, ea.w}, bv[4] = {eb.x, eb.y, eb.z, eb.w};
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            if (av[j] == 0xffffffffu && bv[j] == 0xffffffffu) ++empty;
            else if (av[j] == bv[j]) ++match;
          }
        }
        x = (double)match / (double)(k - empty);
      } else {
        const int32_t groups = k / kWave;
        int32_t h = 0;
        for (int32_t i = 0; i < groups; ++i) h += __popcll(words[u * groups + i] ^ words[v * groups + i]);
        x = table[h];
      }
      sims[o + p] = x;
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
    k_simhash<<<grid_for(n * (k / kWave) * kWave, kLshThreads), kLshThreads, 0, s>>>(off, adj, w, spec.gauss, n, k,
                                                                                    words);
  }
  k_estimate<<<grid_for(n * kWave, kLshThreads), kLshThreads, 0, s>>>(off, adj, n, kind, k, words, sk, table, sims);
  SCAN_HIP_TRY(hipGetLastError());
  if (kind != SCAN_SIM_JACCARD) SCAN_HIP_TRY(hipStreamSynchronize(s));  // the host table stays alive until here
  return SCAN_OK;
}

}  // namespace scan
