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
// Segment length classes: single elements are copied; up to 64 elements,
// lane groups of 8 / 16 / 32 / 64 sort one segment each (several segments
// per wavefront); up to 4096, one workgroup per segment with a block sort of
// the smallest fitting shape; longer segments are tiled and merged.
enum {
  kClsCopy = 0,
  kClsW8, kClsW16, kClsW32, kClsW64,
  kClsB128, kClsB256, kClsB512, kClsB1024, kClsB2048, kClsB4096,
  kClsBig,
  kNumCls
};
// Longest segment of a class (classes below kClsBig).
__host__ __device__ constexpr int class_cap(int c) {
  return c == kClsCopy ? 1 : c <= kClsW64 ? 8 << (c - kClsW8) : 128 << (c - kClsB128);
}

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

// Segments are classified in tiles of kClassTile: a block counts its tile's
// classes in LDS, reserves list space with one global atomic per class, then
// places the segments (wave-aggregated LDS cursors). Few global atomics: a
// per-wavefront reservation stalls on a handful of contended addresses.
constexpr int kClassTile = 4096;

__device__ __forceinline__ int seg_class(int64_t len) {
  if (len <= 0) return -1;
  if (len > kBigTile) return kClsBig;
  int c = kClsCopy;
  while (class_cap(c) < len) ++c;
  return c;
}

__global__ __launch_bounds__(256) void k_classify(const int64_t *seg_off, int64_t nseg,
                                                  int32_t *lists, int64_t cap, SortStats *st,
                                                  int32_t *big_tiles_of) {
  __shared__ int32_t cnt[kNumCls], base[kNumCls], cur[kNumCls];
  __shared__ int32_t tiles_sum, passes_max;
  const int lane = threadIdx.x & (kWave - 1);
  const uint64_t below = (1ull << lane) - 1ull;
  for (int64_t t0 = (int64_t)blockIdx.x * kClassTile; t0 < nseg; t0 += (int64_t)gridDim.x * kClassTile) {
    const int64_t t1 = min(nseg, t0 + kClassTile);
    __syncthreads();
    if (threadIdx.x < kNumCls) {
      cnt[threadIdx.x] = 0;
      cur[threadIdx.x] = 0;
    }
    if (threadIdx.x == 0) {
      tiles_sum = 0;
      passes_max = 0;
    }
    __syncthreads();
    for (int64_t i = t0 + threadIdx.x; i < t1; i += blockDim.x) {
      const int64_t len = seg_off[i + 1] - seg_off[i];
      const int c = seg_class(len);
      if (c >= 0) atomicAdd(&cnt[c], 1);
      if (c == kClsBig) {
        atomicAdd(&tiles_sum, (int32_t)((len + kBigTile - 1) / kBigTile));
        atomicMax(&passes_max, passes_for(len));
      }
    }
    __syncthreads();
    if (threadIdx.x < kNumCls && cnt[threadIdx.x]) base[threadIdx.x] = atomicAdd(&st->count[threadIdx.x], cnt[threadIdx.x]);
    if (threadIdx.x == 0 && tiles_sum) {
      atomicAdd(&st->big_tiles, tiles_sum);
      atomicMax(&st->max_passes, passes_max);
    }
    __syncthreads();
    for (int64_t b0 = t0; b0 < t1; b0 += blockDim.x) {
      const int64_t i = b0 + threadIdx.x;
      int64_t len = 0;
      if (i < t1) len = seg_off[i + 1] - seg_off[i];
      const int c = i < t1 ? seg_class(len) : -1;
      // One round per class present in the wavefront (the class of the
      // lowest pending lane, made uniform by readlane).
      bool pending = c >= 0;
      for (uint64_t act = __ballot(pending); act; act = __ballot(pending)) {
        const int k = __builtin_amdgcn_readlane(c, __ffsll((unsigned long long)act) - 1);
        const uint64_t m = __ballot(pending && c == k);
        const int leader = __ffsll((unsigned long long)m) - 1;
        const int32_t b = __builtin_amdgcn_readlane(atomicAdd(&cur[k], lane == leader ? __popcll(m) : 0), leader);
        if (pending && c == k) {
          const int32_t pos = base[k] + b + __popcll(m & below);
          lists[k * cap + pos] = (int32_t)i;
          if (k == kClsBig) big_tiles_of[pos] = (int32_t)((len + kBigTile - 1) / kBigTile);
          pending = false;
        }
      }
    }
  }
}

// Class kernels read their segment counts (written by k_classify) from
// device memory and run fixed grids, so the host never waits for them.
__global__ void k_sort_copy(const int64_t *seg_off, const int32_t *list, const int32_t *countp,
                            const double *kin, const int32_t *iin, double *kout, int32_t *iout) {
  const int32_t count = *countp;
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

// Bitonic sort of one (key, id) per lane within groups of S lanes, ascending
// (pos = lane within the group; every exchange stride is below S, so it stays
// inside the group).
template <int S>
__device__ __forceinline__ void group_bitonic(uint64_t &k, int32_t &id, int pos) {
#pragma unroll
  for (int size = 2; size <= S; size <<= 1) {
#pragma unroll
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      uint64_t ok = shfl_xor_u64(k, stride);
      int32_t oid = __shfl_xor(id, stride, kWave);
      bool asc = (pos & size) == 0;
      bool lower = (pos & stride) == 0;
      bool other_less = key_less(ok, oid, k, id);
      bool take = (lower == asc) ? other_less : key_less(k, id, ok, oid);
      if (take) {
        k = ok;
        id = oid;
      }
    }
  }
}

// Segments of at most S elements; a wavefront sorts kWave / S of them, one
// per group of S lanes.
template <int S>
__global__ __launch_bounds__(256) void k_sort_group(const int64_t *seg_off, const int32_t *list,
                                                    const int32_t *countp, const double *kin,
                                                    const int32_t *iin, double *kout, int32_t *iout) {
  constexpr int G = kWave / S;
  const int32_t count = *countp;
  const int lane = threadIdx.x & (kWave - 1), grp = lane / S, pos = lane % S;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / kWave;
  for (int64_t w = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kWave; w * G < count; w += nw) {
    const int64_t idx = w * G + grp;
    int64_t o = 0;
    int len = 0;
    if (idx < count) {
      const int32_t sg = list[idx];
      o = seg_off[sg];
      len = (int)(seg_off[sg + 1] - o);
    }
    uint64_t k = kPadKey;
    int32_t id = kPadId;
    if (pos < len) {
      k = desc_key(kin[o + pos]);
      id = iin[o + pos];
    }
    group_bitonic<S>(k, id, pos);
    if (pos < len) {
      kout[o + pos] = key_to_sim(k);
      iout[o + pos] = id;
    }
  }
}

// Block merge sort of up to THREADS * ITEMS (key, id) pairs, ascending by
// (key, id). Each thread sorts ITEMS pairs in registers (bitonic network),
// then log2(THREADS) merge stages through LDS: in each, every thread finds
// where its ITEMS outputs start on the merge path of its two input runs
// (binary search) and merges them serially. Global loads and stores are
// striped (coalesced) and pass through LDS. LDS indices are padded by one
// slot per 16 so that the blocked runs of consecutive threads start on
// different banks.
__device__ __forceinline__ int lds_pad(int i) { return i + (i >> 4); }

template <int THREADS, int ITEMS>
struct BlockSort {
  static constexpr int N = THREADS * ITEMS;
  static constexpr int NP = N + N / 16;
  struct Smem {
    uint64_t K[NP];
    int32_t I[NP];
  };

  __device__ static void thread_sort(uint64_t (&k)[ITEMS], int32_t (&id)[ITEMS]) {
#pragma unroll
    for (int size = 2; size <= ITEMS; size <<= 1) {
#pragma unroll
      for (int stride = size >> 1; stride > 0; stride >>= 1) {
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
          const int j = i ^ stride;
          if (j > i) {
            const bool asc = (i & size) == 0;
            const bool sw = asc ? key_less(k[j], id[j], k[i], id[i]) : key_less(k[i], id[i], k[j], id[j]);
            const uint64_t ki = k[i], kj = k[j];
            const int32_t ii = id[i], ij = id[j];
            k[i] = sw ? kj : ki;
            k[j] = sw ? ki : kj;
            id[i] = sw ? ij : ii;
            id[j] = sw ? ii : ij;
          }
        }
      }
    }
  }

  // Registers (blocked: thread t holds positions [t*ITEMS, (t+1)*ITEMS)) of
  // sorted runs of width ITEMS -> one sorted run of N, blocked.
  __device__ static void merge_stages(Smem &s, uint64_t (&k)[ITEMS], int32_t (&id)[ITEMS], int t) {
    const int o = t * ITEMS;
#pragma unroll 1
    for (int w = ITEMS; w < N; w <<= 1) {
#pragma unroll
      for (int x = 0; x < ITEMS; ++x) {
        s.K[lds_pad(o + x)] = k[x];
        s.I[lds_pad(o + x)] = id[x];
      }
      __syncthreads();
      const int a0 = o & ~(2 * w - 1), b0 = a0 + w, diag = o - a0;
      int lo = diag > w ? diag - w : 0, hi = diag < w ? diag : w;
      while (lo < hi) {  // A elements among the first diag outputs
        const int mid = (lo + hi) >> 1;
        const int jb = lds_pad(b0 + diag - mid - 1), ja = lds_pad(a0 + mid);
        if (key_less(s.K[jb], s.I[jb], s.K[ja], s.I[ja])) hi = mid;
        else lo = mid + 1;
      }
      // The heads of both runs stay in registers; after each output only
      // the consumed run's next element is read (two LDS reads per output).
      int ia = lo, ib = diag - lo;
      const int pa0 = lds_pad(a0 + min(ia, w - 1)), pb0 = lds_pad(b0 + min(ib, w - 1));
      uint64_t ka = s.K[pa0], kb = s.K[pb0];
      int32_t ra = s.I[pa0], rb = s.I[pb0];
#pragma unroll
      for (int x = 0; x < ITEMS; ++x) {
        const bool take_b = ib < w && (ia >= w || key_less(kb, rb, ka, ra));
        k[x] = take_b ? kb : ka;
        id[x] = take_b ? rb : ra;
        if (x + 1 < ITEMS) {
          ib += take_b ? 1 : 0;
          ia += take_b ? 0 : 1;
          const int pn = take_b ? lds_pad(b0 + min(ib, w - 1)) : lds_pad(a0 + min(ia, w - 1));
          const uint64_t kn = s.K[pn];
          const int32_t rn = s.I[pn];
          ka = take_b ? ka : kn;
          ra = take_b ? ra : rn;
          kb = take_b ? kn : kb;
          rb = take_b ? rn : rb;
        }
      }
      __syncthreads();
    }
  }

  // Sorts in[0, len) (len <= N; keys from load(i)), then store(i, key, id)
  // for i < len. Starts and ends with all threads past a barrier.
  template <class Load, class Store>
  __device__ static void run(Smem &s, int len, Load load, Store store) {
    // The thread index passes through an empty asm statement, so the
    // per-element addresses derived from it are computed per call: hoisted
    // out of a caller's loop they occupy over a hundred registers.
    int t = threadIdx.x;
    asm volatile("" : "+v"(t));
#pragma unroll
    for (int x = 0; x < ITEMS; ++x) {
      const int i = x * THREADS + t;
      uint64_t key = kPadKey;
      int32_t idv = kPadId;
      if (i < len) load(i, key, idv);
      s.K[lds_pad(i)] = key;
      s.I[lds_pad(i)] = idv;
    }
    __syncthreads();
    uint64_t k[ITEMS];
    int32_t id[ITEMS];
#pragma unroll
    for (int x = 0; x < ITEMS; ++x) {
      k[x] = s.K[lds_pad(t * ITEMS + x)];
      id[x] = s.I[lds_pad(t * ITEMS + x)];
    }
    __syncthreads();
    thread_sort(k, id);
    merge_stages(s, k, id, t);
#pragma unroll
    for (int x = 0; x < ITEMS; ++x) {
      s.K[lds_pad(t * ITEMS + x)] = k[x];
      s.I[lds_pad(t * ITEMS + x)] = id[x];
    }
    __syncthreads();
#pragma unroll
    for (int x = 0; x < ITEMS; ++x) {
      const int i = x * THREADS + t;
      if (i < len) store(i, s.K[lds_pad(i)], s.I[lds_pad(i)]);
    }
    __syncthreads();
  }
};

// One block per segment of the class (len <= THREADS * ITEMS).
template <int THREADS, int ITEMS>
__global__ __launch_bounds__(THREADS) void k_sort_block(const int64_t *seg_off, const int32_t *list,
                                                        const int32_t *countp, const double *kin,
                                                        const int32_t *iin, double *kout,
                                                        int32_t *iout) {
  const int32_t count = *countp;
  using BS = BlockSort<THREADS, ITEMS>;
  __shared__ typename BS::Smem sm;
  for (int64_t b = blockIdx.x; b < count; b += gridDim.x) {
    const int64_t o = seg_off[list[b]];
    const int len = (int)(seg_off[list[b] + 1] - o);
    BS::run(
        sm, len,
        [&](int i, uint64_t &k, int32_t &id) {
          k = desc_key(kin[o + i]);
          id = iin[o + i];
        },
        [&](int i, uint64_t k, int32_t id) {
          kout[o + i] = key_to_sim(k);
          iout[o + i] = id;
        });
  }
}

// Big segments: tile_seg[t] = index into the big list; tile_first[b] = first
// global tile of big segment b.
__global__ void k_big_tiles(const int32_t *big_tiles_of, const int64_t *tile_first, const int32_t *nbigp,
                            int32_t *tile_seg) {
  const int32_t nbig = *nbigp;
  for (int64_t b = blockIdx.x; b < nbig; b += gridDim.x)
    for (int64_t t = threadIdx.x; t < big_tiles_of[b]; t += blockDim.x)
      tile_seg[tile_first[b] + t] = (int32_t)b;
}

__global__ __launch_bounds__(kSortBlock) void k_big_tile_sort(
    const int64_t *seg_off, const int32_t *big_list, const int32_t *tile_seg,
    const int64_t *tile_first, const int32_t *ntilesp, const double *kin, const int32_t *iin,
    uint64_t *KA, int32_t *IA) {
  const int64_t ntiles = *ntilesp;
  using BS = BlockSort<kSortBlock, kBigTile / kSortBlock>;
  __shared__ typename BS::Smem sm;
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int32_t b = tile_seg[t];
    const int64_t seg = big_list[b];
    const int64_t o = seg_off[seg];
    const int64_t len = seg_off[seg + 1] - o;
    const int64_t start = o + (t - tile_first[b]) * kBigTile;
    const int cnt = (int)min((int64_t)kBigTile, len - (start - o));
    BS::run(
        sm, cnt,
        [&](int i, uint64_t &k, int32_t &id) {
          k = desc_key(kin[start + i]);
          id = iin[start + i];
        },
        [&](int i, uint64_t k, int32_t id) {
          KA[start + i] = k;
          IA[start + i] = id;
        });
  }
}

// Number of elements taken from A among the first `o` outputs of merging
// sorted A (la) and B (lb); elements are distinct. The smallest i with
// B[o-i-1] < A[i] (or the upper end of the range), found by one wavefront
// 64 candidates at a time; every lane returns it.
__device__ __forceinline__ int64_t wave_co_rank(const uint64_t *KA, const int32_t *IA, int64_t la,
                                                const uint64_t *KB, const int32_t *IB, int64_t lb,
                                                int64_t o) {
  const int lane = threadIdx.x & (kWave - 1);
  int64_t lo = o > lb ? o - lb : 0, hi = o < la ? o : la;
  while (lo < hi) {
    // (kWave - 1) * step >= hi - lo: the last lane samples at or past hi
    const int64_t step = (hi - lo + kWave - 2) / (kWave - 1);
    const int64_t p = lo + (int64_t)lane * step;
    bool t = true;  // positions at or past hi count as true
    if (p < hi) {
      const int64_t j = o - p - 1;
      t = key_less(KB[j], IB[j], KA[p], IA[p]);
    }
    const uint64_t m = __ballot(t);  // nonzero: the last lane samples at or past hi
    const int f = __ffsll((unsigned long long)m) - 1;
    if (f == 0) return lo;
    const int64_t nlo = lo + (int64_t)(f - 1) * step + 1;
    const int64_t nhi = min(hi, lo + (int64_t)f * step);
    lo = nlo;
    hi = nhi;
  }
  return lo;
}

// Where the merge of pass q places a big tile's pair: the pass-i run pair
// containing tile t of segment b (see k_big_merge for i and the runs).
struct MergePair {
  int i;            // the segment's own pass number (< 1: no pass now)
  bool last;        // its final pass
  int64_t o, len;   // segment
  int64_t a0, la, b0, lb, ostart;  // runs A = [a0, a0+la), B = [b0, b0+lb); tile's first output
  int cnt;          // outputs of the tile
};
__device__ __forceinline__ MergePair merge_pair(const int64_t *seg_off, const int32_t *big_list,
                                                const int32_t *tile_seg, const int64_t *tile_first,
                                                int64_t t, int q, int max_passes) {
  MergePair m;
  const int32_t b = tile_seg[t];
  const int64_t seg = big_list[b];
  m.o = seg_off[seg];
  m.len = seg_off[seg + 1] - m.o;
  const int P = passes_for(m.len);
  m.i = q - (max_passes - P);
  m.last = m.i == P;
  const int64_t w = (int64_t)kBigTile << (m.i >= 1 ? m.i - 1 : 0);
  const int64_t tstart = (t - tile_first[b]) * kBigTile;
  m.a0 = tstart / (2 * w) * 2 * w;
  m.la = min(w, m.len - m.a0);
  m.b0 = m.a0 + m.la;
  m.lb = max((int64_t)0, min(w, m.len - m.b0));
  m.ostart = tstart - m.a0;
  m.cnt = (int)min((int64_t)kBigTile, m.len - tstart);
  return m;
}

// Merge splits of pass q: split[t] = elements of run A among the outputs of
// its pair that precede tile t's first output. One wavefront per tile, so
// the dependent searches of all tiles run concurrently, ahead of the merge.
__global__ __launch_bounds__(256) void k_big_split(const int64_t *seg_off, const int32_t *big_list,
                                                   const int32_t *tile_seg, const int64_t *tile_first,
                                                   const int32_t *ntilesp, int q, const int32_t *max_passesp,
                                                   const uint64_t *KA, const int32_t *IA, const uint64_t *KB,
                                                   const int32_t *IB, int64_t *split) {
  const int max_passes = *max_passesp;
  if (q > max_passes) return;
  const int64_t ntiles = *ntilesp;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / kWave;
  for (int64_t t = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kWave; t < ntiles; t += nw) {
    const MergePair m = merge_pair(seg_off, big_list, tile_seg, tile_first, t, q, max_passes);
    if (m.i < 1) continue;  // uniform across the wavefront
    const uint64_t *sK = (m.i & 1) ? KA : KB;
    const int32_t *sI = (m.i & 1) ? IA : IB;
    const int64_t r = wave_co_rank(sK + m.o + m.a0, sI + m.o + m.a0, m.la, sK + m.o + m.b0, sI + m.o + m.b0,
                                   m.lb, m.ostart);
    if ((threadIdx.x & (kWave - 1)) == 0) split[t] = r;
  }
}

// One merge-path pass for all big segments. Global pass q (1-based) of
// max_passes; a segment needing P passes does its pass i = q - (max_passes -
// P) when i >= 1, merging runs of width kBigTile << (i-1). Pass i reads A if
// i is odd, else B; writes B / A, or the final output when i == P.
__global__ __launch_bounds__(kSortBlock) void k_big_merge(
    const int64_t *seg_off, const int32_t *big_list, const int32_t *tile_seg,
    const int64_t *tile_first, const int32_t *ntilesp, int q, const int32_t *max_passesp,
    const int64_t *split, uint64_t *KA, int32_t *IA, uint64_t *KB, int32_t *IB, double *kout,
    int32_t *iout) {
  const int max_passes = *max_passesp;
  if (q > max_passes) return;  // launched against an upper bound on the passes
  const int64_t ntiles = *ntilesp;
  __shared__ uint64_t K[kBigTile + kBigTile / 16];  // padded indices (lds_pad)
  __shared__ int32_t I[kBigTile + kBigTile / 16];
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const MergePair m = merge_pair(seg_off, big_list, tile_seg, tile_first, t, q, max_passes);
    if (m.i < 1) continue;  // uniform across the block
    int tid = threadIdx.x;  // opaque per tile: keeps per-element addresses out of registers
    asm volatile("" : "+v"(tid));
    const int64_t o = m.o, tstart = m.a0 + m.ostart;
    const int cnt = m.cnt;
    const bool last = m.last;
    const uint64_t *sK = (m.i & 1) ? KA : KB;
    const int32_t *sI = (m.i & 1) ? IA : IB;
    uint64_t *dK = (m.i & 1) ? KB : KA;
    int32_t *dI = (m.i & 1) ? IB : IA;
    const uint64_t *AK = sK + o + m.a0;
    const int32_t *AI = sI + o + m.a0;
    const uint64_t *BK = sK + o + m.b0;
    const int32_t *BI = sI + o + m.b0;
    // The tile's outputs take A[i0, i1) and B[j0, j1); the next tile of the
    // pair starts where this one ends.
    const int64_t i0 = split[t];
    const int64_t i1 = m.ostart + cnt == m.la + m.lb ? m.la : split[t + 1];
    const int64_t j0 = m.ostart - i0, j1 = m.ostart + cnt - i1;
    const int na = (int)(i1 - i0), nb = (int)(j1 - j0);
    __syncthreads();  // the previous tile's readers of K / I are done
    // Stage A[i0, i1) at K[0, na) and B[j0, j1) at K[na, na + nb): all of a
    // thread's loads are issued before its first LDS store.
    {
      uint64_t sk[kMergeItems];
      int32_t si[kMergeItems];
#pragma unroll
      for (int x = 0; x < kMergeItems; ++x) {
        const int e = x * kSortBlock + tid;
        if (e < cnt) {
          const bool in_a = e < na;
          const uint64_t *pk = in_a ? AK + i0 + e : BK + j0 + (e - na);
          const int32_t *pi = in_a ? AI + i0 + e : BI + j0 + (e - na);
          sk[x] = *pk;
          si[x] = *pi;
        }
      }
#pragma unroll
      for (int x = 0; x < kMergeItems; ++x) {
        const int e = x * kSortBlock + tid;
        if (e < cnt) {
          K[lds_pad(e)] = sk[x];
          I[lds_pad(e)] = si[x];
        }
      }
    }
    __syncthreads();
    uint64_t rk[kMergeItems];
    int32_t ri[kMergeItems];
    int my0 = tid * kMergeItems;
    if (my0 < cnt) {
      // merge-path split inside the staged tile
      int lo = my0 > nb ? my0 - nb : 0, hi = my0 < na ? my0 : na;
      while (lo < hi) {
        int mid = (lo + hi) >> 1;
        const int pj = lds_pad(na + my0 - mid - 1), pm = lds_pad(mid);
        if (key_less(K[pj], I[pj], K[pm], I[pm]))
          hi = mid;
        else
          lo = mid + 1;
      }
      // heads in registers; only the consumed side's next element is read
      // (positions clamped to staged entries; an exhausted side is not used)
      int ia = lo, ib = my0 - lo;
      const int pa0 = lds_pad(na > 0 ? min(ia, na - 1) : 0);
      const int pb0 = lds_pad(nb > 0 ? na + min(ib, nb - 1) : 0);
      uint64_t ka = K[pa0], kb = K[pb0];
      int32_t ra = I[pa0], rb = I[pb0];
#pragma unroll
      for (int x = 0; x < kMergeItems; ++x) {
        const bool has_a = ia < na, has_b = ib < nb;
        const bool take_a = has_a && (!has_b || key_less(ka, ra, kb, rb));
        rk[x] = take_a ? ka : has_b ? kb : kPadKey;
        ri[x] = take_a ? ra : has_b ? rb : kPadId;
        if (x + 1 < kMergeItems) {
          ia += take_a ? 1 : 0;
          ib += (!take_a && has_b) ? 1 : 0;
          const int pn = take_a ? lds_pad(na > 0 ? min(ia, na - 1) : 0) : lds_pad(nb > 0 ? na + min(ib, nb - 1) : 0);
          const uint64_t kn = K[pn];
          const int32_t rn = I[pn];
          ka = take_a ? kn : ka;
          ra = take_a ? rn : ra;
          kb = take_a ? kb : kn;
          rb = take_a ? rb : rn;
        }
      }
    }
    __syncthreads();
    if (my0 < cnt) {
#pragma unroll
      for (int x = 0; x < kMergeItems; ++x) {
        K[lds_pad(my0 + x)] = rk[x];
        I[lds_pad(my0 + x)] = ri[x];
      }
    }
    __syncthreads();
    int64_t gbase = o + tstart;
    if (last) {
      for (int x = tid; x < cnt; x += kSortBlock) {
        kout[gbase + x] = key_to_sim(K[lds_pad(x)]);
        iout[gbase + x] = I[lds_pad(x)];
      }
    } else {
      for (int x = tid; x < cnt; x += kSortBlock) {
        dK[gbase + x] = K[lds_pad(x)];
        dI[gbase + x] = I[lds_pad(x)];
      }
    }
  }
}

SortClasses::~SortClasses() {
  if (ready) {
    (void)hipEventSynchronize(ready);  // the copy into `host` is done
    (void)hipEventDestroy(ready);
  }
  pinned_put(host);
}

scan_status sort_classify(const int64_t *seg_off, int64_t nseg, DevArena &arena, hipStream_t s,
                          SortClasses &c) {
  static_assert(sizeof(SortStats) <= kPinnedBlock, "class sizes fit a pinned block");
  c.nseg = nseg;
  c.stream = s;
  if (nseg <= 0) return SCAN_OK;
  SortStats *st;
  SCAN_TRY(arena.alloc(&c.lists, kNumCls * nseg));
  SCAN_TRY(arena.alloc(&c.big_tiles_of, nseg));
  SCAN_TRY(arena.alloc(&st, 1));
  c.stats = st;
  c.host = pinned_get();
  if (!c.host) return fail(SCAN_ENOMEM, "pinned host allocation failed");
  SCAN_HIP_TRY(hipEventCreateWithFlags(&c.ready, hipEventDisableTiming));
  SCAN_HIP_TRY(hipMemsetAsync(st, 0, sizeof(SortStats), s));
  k_classify<<<grid_for(nseg, kClassTile, 2048), 256, 0, s>>>(seg_off, nseg, c.lists, nseg, st, c.big_tiles_of);
  SCAN_HIP_TRY(hipMemcpyAsync(c.host, st, sizeof(SortStats), hipMemcpyDeviceToHost, s));
  SCAN_HIP_TRY(hipEventRecord(c.ready, s));
  return SCAN_OK;
}

scan_status segmented_sort(const int64_t *seg_off, int64_t nseg, int64_t total,
                           const double *key_in, const int32_t *id_in, double *key_out,
                           int32_t *id_out, hipStream_t s) {
  if (nseg <= 0 || total <= 0) return SCAN_OK;
  DevArena arena(s);
  SortClasses c;
  SCAN_TRY(sort_classify(seg_off, nseg, arena, s, c));
  return sort_run(c, seg_off, total, key_in, id_in, key_out, id_out, s);
}

scan_status sort_run(const SortClasses &c, const int64_t *seg_off, int64_t total, const double *key_in,
                     const int32_t *id_in, double *key_out, int32_t *id_out, hipStream_t s) {
  const int64_t nseg = c.nseg;
  if (nseg <= 0 || total <= 0) return SCAN_OK;
  DevArena arena(s);
  // The host waits for the class sizes (they size each grid: one block or
  // wavefront per segment, which the hardware balances).
  SCAN_HIP_TRY(hipEventSynchronize(c.ready));
  const SortStats h = *(const SortStats *)c.host;
  if (c.stream != s) SCAN_HIP_TRY(hipStreamWaitEvent(s, c.ready, 0));  // the class lists
  SortStats *st = (SortStats *)c.stats;
  const int32_t *lists = c.lists, *big_tiles_of = c.big_tiles_of;
  const int32_t *cnt = st->count;  // device copies of the class sizes
  // The big segments' chain of launches (tile sorts, merge passes) and the
  // other classes' kernels run beside each other, the longer of the two on s
  // and the other on a helper stream (the join at the end then waits for the
  // shorter one, usually already done): the big chain goes on s when the big
  // segments hold at least half of the elements.
  hipStream_t bs = s, gs = s;
  if (h.count[kClsBig] && h.count[kClsBig] < nseg) {
    hipStream_t hs = helper_stream(0);
    if (hs && stream_wait(hs, s) == SCAN_OK) {
      if (2 * (int64_t)h.big_tiles * kBigTile >= total) gs = hs;
      else bs = hs;
    }
  }
  JoinOnExit join_bs{s, bs}, join_gs{s, gs};
  if (h.count[kClsCopy])
    k_sort_copy<<<grid_for(h.count[kClsCopy], 256), 256, 0, gs>>>(seg_off, lists + kClsCopy * nseg, cnt + kClsCopy,
                                                                  key_in, id_in, key_out, id_out);
#define SCAN_GROUP(S, C)                                                                      \
  if (h.count[C])                                                                              \
    k_sort_group<S><<<grid_for(((int64_t)h.count[C] + kWave / (S) - 1) / (kWave / (S)) * kWave, 256), 256, 0, \
                      gs>>>(seg_off, lists + (C) * nseg, cnt + (C), key_in, id_in, key_out, id_out);
  SCAN_GROUP(8, kClsW8)
  SCAN_GROUP(16, kClsW16)
  SCAN_GROUP(32, kClsW32)
  SCAN_GROUP(64, kClsW64)
#undef SCAN_GROUP
#define SCAN_BLOCK(T, I, C, ST)                                                                \
  static_assert((T) * (I) == class_cap(C), "block sort shape must match its class");          \
  if (h.count[C])                                                                              \
    k_sort_block<T, I><<<grid_for(h.count[C], 1), T, 0, ST>>>(seg_off, lists + (C) * nseg, cnt + (C), key_in, \
                                                              id_in, key_out, id_out);
  SCAN_BLOCK(64, 2, kClsB128, gs)
  SCAN_BLOCK(64, 4, kClsB256, gs)
  SCAN_BLOCK(64, 8, kClsB512, gs)
  SCAN_BLOCK(128, 8, kClsB1024, gs)
  SCAN_BLOCK(256, 8, kClsB2048, gs)
  SCAN_BLOCK(kSortBlock, kBigTile / kSortBlock, kClsB4096, gs)
#undef SCAN_BLOCK
  if (h.count[kClsBig]) {
    const int32_t nbig = h.count[kClsBig];
    const int64_t ntiles = h.big_tiles;
    int64_t *tile_first, *scan_ws, *split;
    int32_t *tile_seg, *IA, *IB;
    uint64_t *KA, *KB;
    SCAN_TRY(arena.alloc(&tile_first, nbig + 1));
    SCAN_TRY(arena.alloc(&scan_ws, scan_workspace_elems(nbig)));
    SCAN_TRY(arena.alloc(&tile_seg, ntiles));
    SCAN_TRY(arena.alloc(&split, ntiles));
    SCAN_TRY(arena.alloc(&KA, total));
    SCAN_TRY(arena.alloc(&KB, total));
    SCAN_TRY(arena.alloc(&IA, total));
    SCAN_TRY(arena.alloc(&IB, total));
    SCAN_TRY(exclusive_scan(big_tiles_of, tile_first, nbig, scan_ws, bs));
    const int32_t *big_list = lists + kClsBig * nseg;
    k_big_tiles<<<grid_for(nbig, 1, 4096), 256, 0, bs>>>(big_tiles_of, tile_first, cnt + kClsBig, tile_seg);
    k_big_tile_sort<<<grid_for(ntiles, 1), kSortBlock, 0, bs>>>(seg_off, big_list, tile_seg, tile_first,
                                                               &st->big_tiles, key_in, id_in, KA, IA);
    for (int q = 1; q <= h.max_passes; ++q) {
      k_big_split<<<grid_for(ntiles * kWave, 256), 256, 0, bs>>>(seg_off, big_list, tile_seg, tile_first,
                                                                &st->big_tiles, q, &st->max_passes, KA, IA, KB,
                                                                IB, split);
      k_big_merge<<<grid_for(ntiles, 1), kSortBlock, 0, bs>>>(seg_off, big_list, tile_seg, tile_first,
                                                             &st->big_tiles, q, &st->max_passes, split, KA, IA,
                                                             KB, IB, key_out, id_out);
    }
  }
  SCAN_HIP_TRY(hipGetLastError());
  return SCAN_OK;
}

scan_status segmented_sort_values(const int64_t *seg_off, int64_t nseg, const double *keys,
                                  const int32_t *ids, double *keys_out, int32_t *ids_out) {
  const int64_t total = seg_off[nseg];
  hipStream_t s = nullptr;
  DevArena tmp(s);
  int64_t *d_off;
  double *d_k, *d_ko;
  int32_t *d_i, *d_io;
  SCAN_TRY(tmp.alloc(&d_off, nseg + 1));
  SCAN_TRY(tmp.alloc(&d_k, std::max<int64_t>(total, 1)));
  SCAN_TRY(tmp.alloc(&d_ko, std::max<int64_t>(total, 1)));
  SCAN_TRY(tmp.alloc(&d_i, std::max<int64_t>(total, 1)));
  SCAN_TRY(tmp.alloc(&d_io, std::max<int64_t>(total, 1)));
  SCAN_HIP_TRY(hipMemcpyAsync(d_off, seg_off, (nseg + 1) * 8, hipMemcpyHostToDevice, s));
  if (total > 0) {
    SCAN_HIP_TRY(hipMemcpyAsync(d_k, keys, total * 8, hipMemcpyHostToDevice, s));
    SCAN_HIP_TRY(hipMemcpyAsync(d_i, ids, total * 4, hipMemcpyHostToDevice, s));
    SCAN_TRY(segmented_sort(d_off, nseg, total, d_k, d_i, d_ko, d_io, s));
    SCAN_HIP_TRY(hipMemcpyAsync(keys_out, d_ko, total * 8, hipMemcpyDeviceToHost, s));
    SCAN_HIP_TRY(hipMemcpyAsync(ids_out, d_io, total * 4, hipMemcpyDeviceToHost, s));
  }
  SCAN_HIP_TRY(hipStreamSynchronize(s));
  return SCAN_OK;
}

}  // namespace scan
