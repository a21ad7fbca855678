// Prefix sums and the segmented (similarity desc, id asc) sort used for both
// the neighbour order (segments = CSR rows) and the core order (segments =
// CO[mu]). The paper sorts with a parallel integer sort over rational keys
// (Section 2.3 and Algorithm 2); here the key is the FP64 similarity itself,
// compared through its bit pattern, and segments are sorted by length class:
//   len <= 1      copy
//   len <= 64     one wavefront, bitonic network across lanes (registers)
//   len <= 4096   one workgroup, bitonic network in LDS
//   len >  4096   4096-element LDS tiles, then merge-path passes through HBM
#include <hip/hip_runtime.h>

#include "common.h"

namespace scan {

// ---------------------------------------------------------------------------
// Exclusive scan: int32 or int64 counts -> int64 offsets.

constexpr int kScanBlock = 256;
constexpr int kScanPer = 8;
constexpr int kScanTile = kScanBlock * kScanPer;

__device__ int64_t block_exclusive_sum(int64_t v, int64_t *sh, int64_t *total) {
  int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int d = 1; d < kScanBlock; d <<= 1) {
    int64_t x = t >= d ? sh[t - d] : 0;
    __syncthreads();
    sh[t] += x;
    __syncthreads();
  }
  int64_t incl = sh[t];
  *total = sh[kScanBlock - 1];
  __syncthreads();
  return incl - v;
}

template <class T>
__global__ __launch_bounds__(kScanBlock) void k_scan_reduce(const T *in, int64_t n, int64_t *bsum) {
  __shared__ int64_t sh[kScanBlock];
  int64_t base = (int64_t)blockIdx.x * kScanTile;
  int64_t s = 0;
  for (int k = 0; k < kScanPer; ++k) {
    int64_t i = base + (int64_t)k * kScanBlock + threadIdx.x;
    if (i < n) s += (int64_t)in[i];
  }
  int64_t total;
  block_exclusive_sum(s, sh, &total);
  if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

__global__ __launch_bounds__(kScanBlock) void k_scan_blocks(int64_t *bsum, int64_t nb) {
  __shared__ int64_t sh[kScanBlock];
  int64_t carry = 0;
  for (int64_t base = 0; base < nb; base += kScanBlock) {
    int64_t i = base + threadIdx.x;
    int64_t v = i < nb ? bsum[i] : 0;
    int64_t total;
    int64_t ex = block_exclusive_sum(v, sh, &total);
    if (i < nb) bsum[i] = carry + ex;
    carry += total;
  }
  if (threadIdx.x == 0) bsum[nb] = carry;
}

template <class T>
__global__ __launch_bounds__(kScanBlock) void k_scan_apply(const T *in, int64_t n, const int64_t *bsum,
                                                           int64_t nb, int64_t *out) {
  __shared__ int64_t sh[kScanBlock];
  int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanPer;
  T v[kScanPer];
  int64_t s = 0;
  for (int k = 0; k < kScanPer; ++k) {
    int64_t i = base + k;
    v[k] = i < n ? in[i] : (T)0;
    s += (int64_t)v[k];
  }
  int64_t total;
  int64_t run = bsum[blockIdx.x] + block_exclusive_sum(s, sh, &total);
  for (int k = 0; k < kScanPer; ++k) {
    int64_t i = base + k;
    if (i < n) out[i] = run;
    run += (int64_t)v[k];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = bsum[nb];
}

int64_t scan_workspace_elems(int64_t n) { return (n + kScanTile - 1) / kScanTile + 2; }

template <class T>
static scan_status scan_impl(const T *in, int64_t *out, int64_t n, int64_t *ws, hipStream_t s) {
  int64_t nb = (n + kScanTile - 1) / kScanTile;
  if (nb == 0) nb = 1;
  k_scan_reduce<T><<<(unsigned)nb, kScanBlock, 0, s>>>(in, n, ws);
  k_scan_blocks<<<1, kScanBlock, 0, s>>>(ws, nb);
  k_scan_apply<T><<<(unsigned)nb, kScanBlock, 0, s>>>(in, n, ws, nb, out);
  SCAN_HIP_TRY(hipGetLastError());
  return SCAN_OK;
}

scan_status exclusive_scan(const int32_t *in, int64_t *out, int64_t n, int64_t *ws, hipStream_t s) {
  return scan_impl<int32_t>(in, out, n, ws, s);
}
scan_status exclusive_scan64(const int64_t *in, int64_t *out, int64_t n, int64_t *ws,
                             hipStream_t s) {
  return scan_impl<int64_t>(in, out, n, ws, s);
}

// ---------------------------------------------------------------------------
// Segmented sort.

constexpr int kSortBlock = 256;
constexpr int kBigTile = 4096;
constexpr int kMergeItems = kBigTile / kSortBlock;  // 16
enum { kClsCopy = 0, kClsWave = 1, kClsSmall = 2, kClsMid = 3, kClsBig = 4, kNumCls = 5 };
constexpr int kSmallTile = 512;

struct SortStats {
  int32_t count[kNumCls];
  int32_t big_tiles;
  int32_t max_passes;
};

__device__ __forceinline__ int passes_for(int64_t len) {
  int64_t tiles = (len + kBigTile - 1) / kBigTile;
  int p = 0;
  while (((int64_t)1 << p) < tiles) ++p;
  return p;
}

// Wave-aggregated appends: one global atomic per (wavefront, class).
__global__ __launch_bounds__(256) void k_classify(const int64_t *seg_off, int64_t nseg,
                                                  int32_t *lists, int64_t cap, SortStats *st,
                                                  int32_t *big_tiles_of) {
  const int lane = threadIdx.x & (kWave - 1);
  const uint64_t below = (1ull << lane) - 1ull;
  for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < nseg;
       base += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = base + threadIdx.x;
    int c = -1;
    int64_t len = 0;
    if (i < nseg) {
      len = seg_off[i + 1] - seg_off[i];
      if (len > 0)
        c = len <= 1 ? kClsCopy : len <= kWave ? kClsWave : len <= kSmallTile ? kClsSmall
            : len <= kBigTile ? kClsMid : kClsBig;
    }
    int32_t tiles = c == kClsBig ? (int32_t)((len + kBigTile - 1) / kBigTile) : 0;
    for (int k = 0; k < kNumCls; ++k) {
      const uint64_t m = __ballot(c == k);
      if (!m) continue;
      const int leader = __ffsll((unsigned long long)m) - 1;
      int32_t b = 0;
      if (lane == leader) b = atomicAdd(&st->count[k], __popcll(m));
      b = __shfl(b, leader, kWave);
      if (c == k) {
        const int pos = b + __popcll(m & below);
        lists[k * cap + pos] = (int32_t)i;
        if (k == kClsBig) big_tiles_of[pos] = tiles;
      }
    }
    if (c == kClsBig) {
      atomicAdd(&st->big_tiles, tiles);
      atomicMax(&st->max_passes, passes_for(len));
    }
  }
}

__global__ void k_sort_copy(const int64_t *seg_off, const int32_t *list, int32_t count,
                            const double *kin, const int32_t *iin, double *kout, int32_t *iout) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x) {
    int64_t o = seg_off[list[i]];
    kout[o] = kin[o];
    iout[o] = iin[o];
  }
}

__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t v, int m) {
  uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
  lo = __shfl_xor(lo, m, kWave);
  hi = __shfl_xor(hi, m, kWave);
  return ((uint64_t)hi << 32) | lo;
}

// Bitonic sort of one (key, id) per lane across the 64 lanes, ascending.
__device__ __forceinline__ void wave_bitonic(uint64_t &k, int32_t &id, int lane) {
#pragma unroll
  for (int size = 2; size <= kWave; size <<= 1) {
#pragma unroll
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      uint64_t ok = shfl_xor_u64(k, stride);
      int32_t oid = __shfl_xor(id, stride, kWave);
      bool asc = (lane & size) == 0;
      bool lower = (lane & stride) == 0;
      bool other_less = key_less(ok, oid, k, id);
      bool take = (lower == asc) ? other_less : key_less(k, id, ok, oid);
      if (take) {
        k = ok;
        id = oid;
      }
    }
  }
}

__global__ __launch_bounds__(256) void k_sort_wave(const int64_t *seg_off, const int32_t *list,
                                                   int32_t count, const double *kin,
                                                   const int32_t *iin, double *kout,
                                                   int32_t *iout) {
  int lane = threadIdx.x & (kWave - 1);
  int64_t w = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kWave;
  int64_t nw = ((int64_t)gridDim.x * blockDim.x) / kWave;
  for (; w < count; w += nw) {
    int64_t o = seg_off[list[w]];
    int len = (int)(seg_off[list[w] + 1] - o);
    uint64_t k = kPadKey;
    int32_t id = kPadId;
    if (lane < len) {
      k = desc_key(kin[o + lane]);
      id = iin[o + lane];
    }
    wave_bitonic(k, id, lane);
    if (lane < len) {
      kout[o + lane] = key_to_sim(k);
      iout[o + lane] = id;
    }
  }
}

// Bitonic network over n_pad (power of two) LDS elements, ascending.
__device__ void block_bitonic(uint64_t *K, int32_t *I, int n_pad) {
  for (int size = 2; size <= n_pad; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      __syncthreads();
      for (int i = threadIdx.x; i < n_pad / 2; i += blockDim.x) {
        int lo = 2 * i - (i & (stride - 1));
        int hi = lo + stride;
        bool asc = (lo & size) == 0;
        uint64_t ka = K[lo], kb = K[hi];
        int32_t ia = I[lo], ib = I[hi];
        bool gt = key_less(kb, ib, ka, ia);
        if (gt == asc) {
          K[lo] = kb;
          K[hi] = ka;
          I[lo] = ib;
          I[hi] = ia;
        }
      }
    }
  }
  __syncthreads();
}

template <int TILE>
__global__ __launch_bounds__(kSortBlock) void k_sort_block(const int64_t *seg_off,
                                                           const int32_t *list, int32_t count,
                                                           const double *kin, const int32_t *iin,
                                                           double *kout, int32_t *iout) {
  __shared__ uint64_t K[TILE];
  __shared__ int32_t I[TILE];
  for (int64_t b = blockIdx.x; b < count; b += gridDim.x) {
    int64_t o = seg_off[list[b]];
    int len = (int)(seg_off[list[b] + 1] - o);
    int n_pad = 1;
    while (n_pad < len) n_pad <<= 1;
    __syncthreads();
    for (int i = threadIdx.x; i < n_pad; i += blockDim.x) {
      if (i < len) {
        K[i] = desc_key(kin[o + i]);
        I[i] = iin[o + i];
      } else {
        K[i] = kPadKey;
        I[i] = kPadId;
      }
    }
    block_bitonic(K, I, n_pad);
    for (int i = threadIdx.x; i < len; i += blockDim.x) {
      kout[o + i] = key_to_sim(K[i]);
      iout[o + i] = I[i];
    }
  }
}

// Big segments: tile_seg[t] = index into the big list; tile_first[b] = first
// global tile of big segment b.
__global__ void k_big_tiles(const int32_t *big_tiles_of, const int64_t *tile_first, int32_t nbig,
                            int32_t *tile_seg) {
  for (int64_t b = blockIdx.x; b < nbig; b += gridDim.x)
    for (int64_t t = threadIdx.x; t < big_tiles_of[b]; t += blockDim.x)
      tile_seg[tile_first[b] + t] = (int32_t)b;
}

__global__ __launch_bounds__(kSortBlock) void k_big_tile_sort(
    const int64_t *seg_off, const int32_t *big_list, const int32_t *tile_seg,
    const int64_t *tile_first, int64_t ntiles, const double *kin, const int32_t *iin,
    uint64_t *KA, int32_t *IA) {
  __shared__ uint64_t K[kBigTile];
  __shared__ int32_t I[kBigTile];
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    int32_t b = tile_seg[t];
    int64_t seg = big_list[b];
    int64_t o = seg_off[seg];
    int64_t len = seg_off[seg + 1] - o;
    int64_t start = (t - tile_first[b]) * kBigTile;
    int cnt = (int)min((int64_t)kBigTile, len - start);
    __syncthreads();
    for (int i = threadIdx.x; i < kBigTile; i += blockDim.x) {
      if (i < cnt) {
        K[i] = desc_key(kin[o + start + i]);
        I[i] = iin[o + start + i];
      } else {
        K[i] = kPadKey;
        I[i] = kPadId;
      }
    }
    block_bitonic(K, I, kBigTile);
    for (int i = threadIdx.x; i < cnt; i += blockDim.x) {
      KA[o + start + i] = K[i];
      IA[o + start + i] = I[i];
    }
  }
}

// Number of elements taken from A among the first `o` outputs of merging
// sorted A (la) and B (lb); elements are distinct.
__device__ __forceinline__ int64_t co_rank(const uint64_t *KA, const int32_t *IA, int64_t la,
                                           const uint64_t *KB, const int32_t *IB, int64_t lb,
                                           int64_t o) {
  int64_t lo = o > lb ? o - lb : 0, hi = o < la ? o : la;
  while (lo < hi) {
    int64_t mid = (lo + hi) >> 1;
    int64_t j = o - mid - 1;
    if (key_less(KB[j], IB[j], KA[mid], IA[mid]))
      hi = mid;
    else
      lo = mid + 1;
  }
  return lo;
}

// One merge-path pass for all big segments. Global pass q (1-based) of
// max_passes; a segment needing P passes does its pass i = q - (max_passes -
// P) when i >= 1, merging runs of width kBigTile << (i-1). Pass i reads A if
// i is odd, else B; writes B / A, or the final output when i == P.
__global__ __launch_bounds__(kSortBlock) void k_big_merge(
    const int64_t *seg_off, const int32_t *big_list, const int32_t *tile_seg,
    const int64_t *tile_first, int64_t ntiles, int q, int max_passes, uint64_t *KA, int32_t *IA,
    uint64_t *KB, int32_t *IB, double *kout, int32_t *iout) {
  __shared__ uint64_t K[kBigTile];
  __shared__ int32_t I[kBigTile];
  __shared__ int64_t bounds[4];
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    int32_t b = tile_seg[t];
    int64_t seg = big_list[b];
    int64_t o = seg_off[seg];
    int64_t len = seg_off[seg + 1] - o;
    int P = passes_for(len);
    int i = q - (max_passes - P);
    if (i < 1) continue;  // uniform across the block
    const uint64_t *sK = (i & 1) ? KA : KB;
    const int32_t *sI = (i & 1) ? IA : IB;
    uint64_t *dK = (i & 1) ? KB : KA;
    int32_t *dI = (i & 1) ? IB : IA;
    bool last = (i == P);
    int64_t w = (int64_t)kBigTile << (i - 1);
    int64_t tstart = (t - tile_first[b]) * kBigTile;
    int64_t pair = tstart / (2 * w);
    int64_t a0 = pair * 2 * w;
    int64_t la = min(w, len - a0);
    int64_t b0 = a0 + la;
    int64_t lb = max((int64_t)0, min(w, len - b0));
    const uint64_t *AK = sK + o + a0;
    const int32_t *AI = sI + o + a0;
    const uint64_t *BK = sK + o + b0;
    const int32_t *BI = sI + o + b0;
    int64_t ostart = tstart - a0;
    int cnt = (int)min((int64_t)kBigTile, len - tstart);
    __syncthreads();
    if (threadIdx.x == 0) {
      int64_t i0 = co_rank(AK, AI, la, BK, BI, lb, ostart);
      int64_t i1 = co_rank(AK, AI, la, BK, BI, lb, ostart + cnt);
      bounds[0] = i0;
      bounds[1] = i1;
      bounds[2] = ostart - i0;
      bounds[3] = ostart + cnt - i1;
    }
    __syncthreads();
    int64_t i0 = bounds[0], i1 = bounds[1], j0 = bounds[2], j1 = bounds[3];
    int na = (int)(i1 - i0), nb = (int)(j1 - j0);
    // Stage A[i0, i1) at K[0, na) and B[j0, j1) at K[na, na + nb).
    for (int x = threadIdx.x; x < na; x += blockDim.x) {
      K[x] = AK[i0 + x];
      I[x] = AI[i0 + x];
    }
    for (int x = threadIdx.x; x < nb; x += blockDim.x) {
      K[na + x] = BK[j0 + x];
      I[na + x] = BI[j0 + x];
    }
    __syncthreads();
    uint64_t rk[kMergeItems];
    int32_t ri[kMergeItems];
    int my0 = threadIdx.x * kMergeItems;
    if (my0 < cnt) {
      // merge-path split inside the staged tile
      int lo = my0 > nb ? my0 - nb : 0, hi = my0 < na ? my0 : na;
      while (lo < hi) {
        int mid = (lo + hi) >> 1;
        int j = my0 - mid - 1;
        if (key_less(K[na + j], I[na + j], K[mid], I[mid]))
          hi = mid;
        else
          lo = mid + 1;
      }
      int ia = lo, ib = my0 - lo;
#pragma unroll
      for (int x = 0; x < kMergeItems; ++x) {
        bool takeA = ib >= nb || (ia < na && key_less(K[ia], I[ia], K[na + ib], I[na + ib]));
        if (takeA) {
          rk[x] = K[ia];
          ri[x] = I[ia];
          ++ia;
        } else if (ib < nb) {
          rk[x] = K[na + ib];
          ri[x] = I[na + ib];
          ++ib;
        } else {
          rk[x] = kPadKey;
          ri[x] = kPadId;
        }
      }
    }
    __syncthreads();
    if (my0 < cnt) {
#pragma unroll
      for (int x = 0; x < kMergeItems; ++x) {
        K[my0 + x] = rk[x];
        I[my0 + x] = ri[x];
      }
    }
    __syncthreads();
    int64_t gbase = o + tstart;
    if (last) {
      for (int x = threadIdx.x; x < cnt; x += blockDim.x) {
        kout[gbase + x] = key_to_sim(K[x]);
        iout[gbase + x] = I[x];
      }
    } else {
      for (int x = threadIdx.x; x < cnt; x += blockDim.x) {
        dK[gbase + x] = K[x];
        dI[gbase + x] = I[x];
      }
    }
  }
}

scan_status segmented_sort(const int64_t *seg_off, int64_t nseg, int64_t total,
                           const double *key_in, const int32_t *id_in, double *key_out,
                           int32_t *id_out, hipStream_t s) {
  if (nseg <= 0 || total <= 0) return SCAN_OK;
  DevArena arena(s);
  int32_t *lists, *big_tiles_of;
  SortStats *st;
  SCAN_TRY(arena.alloc(&lists, kNumCls * nseg));
  SCAN_TRY(arena.alloc(&big_tiles_of, nseg));
  SCAN_TRY(arena.alloc(&st, 1));
  SCAN_HIP_TRY(hipMemsetAsync(st, 0, sizeof(SortStats), s));
  k_classify<<<grid_for(nseg, 256), 256, 0, s>>>(seg_off, nseg, lists, nseg, st, big_tiles_of);
  SortStats h;
  SCAN_HIP_TRY(hipMemcpyAsync(&h, st, sizeof(SortStats), hipMemcpyDeviceToHost, s));
  SCAN_HIP_TRY(hipStreamSynchronize(s));
  if (h.count[kClsCopy])
    k_sort_copy<<<grid_for(h.count[kClsCopy], 256), 256, 0, s>>>(
        seg_off, lists + kClsCopy * nseg, h.count[kClsCopy], key_in, id_in, key_out, id_out);
  if (h.count[kClsWave])
    k_sort_wave<<<grid_for((int64_t)h.count[kClsWave] * kWave, 256), 256, 0, s>>>(
        seg_off, lists + kClsWave * nseg, h.count[kClsWave], key_in, id_in, key_out, id_out);
  if (h.count[kClsSmall])
    k_sort_block<kSmallTile><<<grid_for(h.count[kClsSmall], 1), kSortBlock, 0, s>>>(
        seg_off, lists + kClsSmall * nseg, h.count[kClsSmall], key_in, id_in, key_out, id_out);
  if (h.count[kClsMid])
    k_sort_block<kBigTile><<<grid_for(h.count[kClsMid], 1), kSortBlock, 0, s>>>(
        seg_off, lists + kClsMid * nseg, h.count[kClsMid], key_in, id_in, key_out, id_out);
  if (h.count[kClsBig]) {
    int32_t nbig = h.count[kClsBig];
    int64_t ntiles = h.big_tiles;
    int64_t *tile_first, *scan_ws;
    int32_t *tile_seg, *IA, *IB;
    uint64_t *KA, *KB;
    SCAN_TRY(arena.alloc(&tile_first, nbig + 1));
    SCAN_TRY(arena.alloc(&scan_ws, scan_workspace_elems(nbig)));
    SCAN_TRY(arena.alloc(&tile_seg, ntiles));
    SCAN_TRY(arena.alloc(&KA, total));
    SCAN_TRY(arena.alloc(&KB, total));
    SCAN_TRY(arena.alloc(&IA, total));
    SCAN_TRY(arena.alloc(&IB, total));
    SCAN_TRY(exclusive_scan(big_tiles_of, tile_first, nbig, scan_ws, s));
    const int32_t *big_list = lists + kClsBig * nseg;
    k_big_tiles<<<grid_for(nbig, 1, 4096), 256, 0, s>>>(big_tiles_of, tile_first, nbig, tile_seg);
    k_big_tile_sort<<<grid_for(ntiles, 1), kSortBlock, 0, s>>>(
        seg_off, big_list, tile_seg, tile_first, ntiles, key_in, id_in, KA, IA);
    for (int q = 1; q <= h.max_passes; ++q)
      k_big_merge<<<grid_for(ntiles, 1), kSortBlock, 0, s>>>(seg_off, big_list, tile_seg,
                                                               tile_first, ntiles, q,
                                                               h.max_passes, KA, IA, KB, IB,
                                                               key_out, id_out);
  }
  SCAN_HIP_TRY(hipGetLastError());
  return SCAN_OK;
}

}  // namespace scan
