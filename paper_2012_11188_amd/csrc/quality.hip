// Clustering quality on the device: the modularity of Section 7.2 (Newman's
// definition) with every unclustered vertex in a cluster of its own, the
// score by which Section 7.3.4 selects (mu, eps).
//
//   Q = 1/(2m) * sum over ordered pairs (u, v) of (A_uv - d_u d_v / 2m) delta_uv
//     = (s_in - sd2 / 2m) / 2m,
//   s_in = ordered neighbour pairs inside one cluster (a count of CSR slots),
//   sd2  = sum over clusters of (sum of degrees in the cluster)^2.
//
// Both terms are integers and are accumulated exactly (int64 atomics), so the
// host's final FP64 step gives the same bits as any other exact evaluation.
#include <hip/hip_runtime.h>

#include "index.h"

namespace scan {

constexpr int kModThreads = 256;
constexpr int kModGroup = 8;          // lanes per vertex
constexpr int64_t kModGroupMax = 512;  // longer rows: the whole wavefront
constexpr int kModSteps = 8;

static __device__ __forceinline__ int64_t block_sum64(int64_t v, int64_t *wsum) {
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
#pragma unroll
  for (int m = kWave / 2; m > 0; m >>= 1) {
    const int32_t lo = __shfl_xor((int32_t)(uint32_t)v, m, kWave);
    const int32_t hi = __shfl_xor((int32_t)(v >> 32), m, kWave);
    v += (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
  }
  __syncthreads();
  if (lane == 0) wsum[wave] = v;
  __syncthreads();
  int64_t t = 0;
  if (threadIdx.x == 0)
    for (int w = 0; w < kModThreads / kWave; ++w) t += wsum[w];
  return t;  // thread 0
}

// s_in, and per cluster label the degree sum (dsum, zero on entry);
// unclustered vertices add their squared degree to terms[1] directly.
__global__ __launch_bounds__(kModThreads) void k_mod_rows(const int64_t *off, const int32_t *ids, int64_t n,
                                                          const int32_t *memb, int64_t *dsum, int64_t *terms) {
  __shared__ int64_t wsum[kModThreads / kWave];
  constexpr int kPerWave = kWave / kModGroup;
  const int lane = threadIdx.x & (kWave - 1), pos = lane % kModGroup;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / kWave;
  int64_t in = 0, sq = 0;  // this lane's shares
  for (int64_t v0 = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kWave * kPerWave; v0 < n;
       v0 += nw * kPerWave) {
    const int64_t v = v0 + lane / kModGroup;
    int64_t b = 0, e = 0;
    int32_t c = -1;
    if (v < n) {
      c = memb[v];
      if (c >= n || c < -1) {  // not a label of this graph: reported, counted as unclustered
        if (pos == 0) atomicAdd((unsigned long long *)&terms[2], 1ull);
        c = -1;
      }
      b = off[v];
      e = off[v + 1];
      if (pos == 0) {
        if (c >= 0) atomicAdd((unsigned long long *)&dsum[c], (unsigned long long)(e - b));
        else sq += (e - b) * (e - b);
      }
    }
    if (c >= 0 && e - b <= kModGroupMax)  // the same for every lane of the group
      for (int64_t k = b + pos; k < e; k += kModGroup) in += memb[ids[k]] == c ? 1 : 0;
    // long clustered rows: one at a time by the whole wavefront
    uint64_t longs = __ballot(c >= 0 && e - b > kModGroupMax && pos == 0);
    while (longs) {
      const int src = __ffsll((unsigned long long)longs) - 1;
      longs &= longs - 1;
      const int64_t rb = (int64_t)(uint32_t)__builtin_amdgcn_readlane((int32_t)b, src) |
                         ((int64_t)__builtin_amdgcn_readlane((int32_t)(b >> 32), src) << 32);
      const int64_t re = (int64_t)(uint32_t)__builtin_amdgcn_readlane((int32_t)e, src) |
                         ((int64_t)__builtin_amdgcn_readlane((int32_t)(e >> 32), src) << 32);
      const int32_t rc = __builtin_amdgcn_readlane(c, src);
      for (int64_t k0 = rb; k0 < re; k0 += kModSteps * kWave) {
        int32_t w[kModSteps];
#pragma unroll
        for (int j = 0; j < kModSteps; ++j) {
          const int64_t k = k0 + j * kWave + lane;
          w[j] = k < re ? ids[k] : -1;
        }
#pragma unroll
        for (int j = 0; j < kModSteps; ++j) in += (w[j] >= 0 && memb[w[j]] == rc) ? 1 : 0;
      }
    }
  }
  const int64_t bin = block_sum64(in, wsum);
  const int64_t bsq = block_sum64(sq, wsum);
  if (threadIdx.x == 0) {
    atomicAdd((unsigned long long *)&terms[0], (unsigned long long)bin);
    atomicAdd((unsigned long long *)&terms[1], (unsigned long long)bsq);
  }
}

// (terms[2] counts memberships outside [-1, n).)
// sd2 += dsum[c]^2 over every label, and dsum is cleared for the next call.
__global__ __launch_bounds__(kModThreads) void k_mod_squares(int64_t *dsum, int64_t n, int64_t *terms) {
  __shared__ int64_t wsum[kModThreads / kWave];
  int64_t sq = 0;
  for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < n; c += (int64_t)gridDim.x * blockDim.x) {
    const int64_t d = dsum[c];
    sq += d * d;
    dsum[c] = 0;
  }
  const int64_t b = block_sum64(sq, wsum);
  if (threadIdx.x == 0) atomicAdd((unsigned long long *)&terms[1], (unsigned long long)b);
}

__global__ void k_zero64(int64_t *p, int64_t count) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

void zero64(int64_t *p, int64_t count, hipStream_t s) {
  if (count > 0) k_zero64<<<grid_for(count, 256, 4096), 256, 0, s>>>(p, count);
}

void launch_modularity_terms(const scan_index *ix, const int32_t *memb, int64_t *dsum, int64_t *terms,
                             hipStream_t s) {
  const int64_t n = ix->n;
  const int64_t groups = (n + kWave / kModGroup - 1) / (kWave / kModGroup);
  k_mod_rows<<<grid_for(groups * kWave, kModThreads, 8192), kModThreads, 0, s>>>(ix->off, ix->no_ids, n, memb,
                                                                                 dsum, terms);
  k_mod_squares<<<grid_for(n, kModThreads, 2048), kModThreads, 0, s>>>(dsum, n, terms);
}

double modularity_value(int64_t s_in, int64_t sd2, int64_t nnz) {
  if (nnz == 0) return 0.0;
  const double two_m = (double)nnz;
  return ((double)s_in - (double)sd2 / two_m) / two_m;
}

}  // namespace scan
