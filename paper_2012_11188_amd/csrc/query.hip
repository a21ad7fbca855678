// (mu, eps) clustering queries over the index (Section 4.2, Algorithms 3-5;
// connectivity by union-find as in Section 6.2; border vertices by the
// deterministic rule of Section 7.3.4).
//
// Per query, five grid-stride kernels over a batch (blockIdx.y = query). A
// byte per vertex (the slot's state array, all zero between queries) marks
// cores (2) and candidate borders (1):
//   a7  k_q_cores   K = length of the eps-prefix of CO[mu] (binary search);
//                   for the K cores: state = 2, parent = self
//   a8+a9 k_q_union for each core u, scan the eps-prefix of NO[u]; a core
//                   neighbour w is united with u (larger root hooked under the
//                   smaller, so every root is its component's smallest id); a
//                   non-core neighbour is marked as a candidate border
//   a9  k_q_jump    parent[u] = find(u) for every core
//   a10 k_q_output  memberships: cores -> root; marked non-cores -> root of
//                   the first core in their own NO row (NO is sorted by sim
//                   desc, id asc, so that is the most similar eps-similar core,
//                   ties to the lower id); others -1. Clears border marks.
//       k_q_reset   clears the core marks.
// A vertex w is a core iff deg(w) >= mu-1 and NO_SIM[off[w] + mu - 2] >= eps,
// which is exactly membership in the eps-prefix of CO[mu] (the CO entry of w
// for mu carries that same threshold value).
#include <hip/hip_runtime.h>

#include <climits>

#include <cmath>
#include <mutex>
#include <vector>

#include "index.h"

namespace scan {

constexpr uint8_t kCore = 2, kBorder = 1;
constexpr uint8_t kRoleClustered = SCAN_ROLE_CLUSTERED, kRoleHub = SCAN_ROLE_HUB, kRoleOutlier = SCAN_ROLE_OUTLIER;

struct IndexView {
  int64_t n, dmax;
  const int64_t *off;
  const int32_t *no_ids;
  const double *no_sim;
  const int64_t *co_off;
  const int32_t *co_ids;
  const double *co_thr;
};

// Length of the eps-prefix of CO[mu] (thresholds are sorted descending).
__device__ __forceinline__ void core_prefix(const IndexView &ix, int32_t mu, double eps, int64_t &base,
                                            int64_t &K) {
  K = 0;
  base = 0;
  if ((int64_t)mu > ix.dmax + 1) return;
  base = ix.co_off[mu];
  int64_t lo = 0, hi = ix.co_off[mu + 1] - base;
  while (lo < hi) {  // first position with thr < eps
    int64_t mid = (lo + hi) >> 1;
    if (ix.co_thr[base + mid] >= eps) lo = mid + 1;
    else hi = mid;
  }
  K = lo;
}

// parent[] entries of the query's cores form a forest (hooks go from a root
// to a smaller root, halving moves a pointer to an ancestor); the step cap
// only guards against a corrupt index.
__device__ __forceinline__ int32_t uf_find(int32_t *parent, int32_t x) {
  int32_t cur = x;
  for (int guard = 0; guard < (1 << 26); ++guard) {
    int32_t nxt = __atomic_load_n(&parent[cur], __ATOMIC_RELAXED);
    if (nxt == cur) return cur;
    int32_t nn = __atomic_load_n(&parent[nxt], __ATOMIC_RELAXED);
    if (nn != nxt) __atomic_store_n(&parent[cur], nn, __ATOMIC_RELAXED);  // path halving
    cur = nxt;
  }
  return cur;
}

// The root of x without writing: k_q_jump needs every core's final pointer to
// be its root, and a halving step of another thread, based on pointers read
// before this thread stored the root, could overwrite it with an ancestor.
__device__ __forceinline__ int32_t uf_root(const int32_t *parent, int32_t x) {
  int32_t cur = x;
  for (int guard = 0; guard < (1 << 26); ++guard) {
    const int32_t nxt = __atomic_load_n(&parent[cur], __ATOMIC_RELAXED);
    if (nxt == cur) return cur;
    cur = nxt;
  }
  return cur;
}

__device__ __forceinline__ void uf_union(int32_t *parent, int32_t a, int32_t b) {
  for (;;) {
    a = uf_find(parent, a);
    b = uf_find(parent, b);
    if (a == b) return;
    if (a < b) {
      int32_t t = a;
      a = b;
      b = t;
    }
    // hook root a (larger) under b (smaller)
    if (atomicCAS(&parent[a], a, b) == a) return;
  }
}

// A descriptor with memb == nullptr is an unused batch entry: every kernel
// skips it.
__global__ void k_q_cores(IndexView ix, QueryDesc *qd) {
  QueryDesc &q = qd[blockIdx.y];
  if (!q.memb) return;
  __shared__ int64_t sh[2];
  if (threadIdx.x == 0) {  // every block finds K itself (same addresses: cache hits)
    int64_t base, K;
    core_prefix(ix, q.mu, q.eps, base, K);
    sh[0] = base;
    sh[1] = K;
    if (blockIdx.x == 0) {
      q.K = K;
      q.base = base;
    }
  }
  __syncthreads();
  const int64_t base = sh[0], K = sh[1];
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < K;
       i += (int64_t)gridDim.x * blockDim.x) {
    int32_t u = ix.co_ids[base + i];
    q.parent[u] = u;
    q.flag[u] = kCore;
  }
}

// One wavefront per core; lanes stride the eps-prefix of its NO row.
__global__ void k_q_union(IndexView ix, const QueryDesc *qd) {
  const QueryDesc q = qd[blockIdx.y];
  if (!q.memb) return;
  int lane = threadIdx.x & (kWave - 1);
  int64_t w = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kWave;
  int64_t nw = ((int64_t)gridDim.x * blockDim.x) / kWave;
  for (int64_t i = w; i < q.K; i += nw) {
    int32_t u = ix.co_ids[q.base + i];
    int64_t b = ix.off[u], e = ix.off[u + 1];
    for (int64_t k0 = b; k0 < e; k0 += kWave) {
      int64_t k = k0 + lane;
      bool in = k < e && ix.no_sim[k] >= q.eps;
      if (in) {
        int32_t x = ix.no_ids[k];
        if (q.flag[x] == kCore) {
          if (x < u) uf_union(q.parent, u, x);
        } else {
          q.flag[x] = kBorder;
        }
      }
      if (!__all(in)) break;  // the prefix ended inside this chunk
    }
  }
}

__global__ void k_q_jump(IndexView ix, const QueryDesc *qd) {
  const QueryDesc q = qd[blockIdx.y];
  if (!q.memb) return;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < q.K;
       i += (int64_t)gridDim.x * blockDim.x) {
    int32_t u = ix.co_ids[q.base + i];
    __atomic_store_n(&q.parent[u], uf_root(q.parent, u), __ATOMIC_RELAXED);
  }
}

// Reads core marks of other vertices, so border marks (own vertex only) are
// the only ones it clears.
__global__ void k_q_output(IndexView ix, const QueryDesc *qd) {
  const QueryDesc q = qd[blockIdx.y];
  if (!q.memb) return;
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < ix.n;
       v += (int64_t)gridDim.x * blockDim.x) {
    const uint8_t st = q.flag[v];
    int32_t m = -1;
    if (st == kCore) {
      m = q.parent[v];
    } else if (st == kBorder) {
      q.flag[v] = 0;
      int64_t b = ix.off[v], e = ix.off[v + 1];
      for (int64_t k = b; k < e && ix.no_sim[k] >= q.eps; ++k) {
        int32_t x = ix.no_ids[k];
        if (q.flag[x] == kCore) {
          m = q.parent[x];
          break;
        }
      }
    }
    q.memb[v] = m;
    if (q.is_core) q.is_core[v] = st == kCore ? 1 : 0;
  }
}

__global__ void k_q_reset(IndexView ix, const QueryDesc *qd) {
  const QueryDesc q = qd[blockIdx.y];
  if (!q.memb) return;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < q.K;
       i += (int64_t)gridDim.x * blockDim.x)
    q.flag[ix.co_ids[q.base + i]] = 0;
}

void launch_query_kernels(const scan_index *ix, QueryDesc *d, int32_t count, hipStream_t s) {
  IndexView v{ix->n, ix->dmax, ix->off, ix->no_ids, ix->no_sim, ix->co_off, ix->co_ids, ix->co_thr};
  int64_t n = ix->n > 0 ? ix->n : 1;
  dim3 gc(grid_for(n, 256, 1024), count);
  dim3 gu(grid_for(n * kWave, 256, 2048), count);
  dim3 go(grid_for(n, 256, 2048), count);
  k_q_cores<<<gc, 256, 0, s>>>(v, d);
  k_q_union<<<gu, 256, 0, s>>>(v, d);
  k_q_jump<<<gc, 256, 0, s>>>(v, d);
  k_q_output<<<go, 256, 0, s>>>(v, d);
  k_q_reset<<<gc, 256, 0, s>>>(v, d);
}

// Hubs and outliers (Section 4.3): every unclustered vertex maps its
// neighbours to their clusters and checks whether two of them differ (the NO
// row holds the open neighbourhood). A wavefront takes kWave / kRoleGroup
// consecutive vertices, one per group of kRoleGroup lanes; a group scans its
// vertex's row kRoleGroup ids per step, reducing the step's smallest and
// largest cluster label within the group (lane exchanges stay inside the
// group, whose lanes are active together), and stops at a second cluster.
// Rows longer than kRoleGroupMax are scanned afterwards by the whole
// wavefront, kRoleSteps * 64 ids per step. A vertex in a cluster gets role 0
// without reading its row.
constexpr int kRoleGroup = 8;
constexpr int64_t kRoleGroupMax = 512;
constexpr int kRoleSteps = 8;

__device__ __forceinline__ int32_t group_min(int32_t x) {
#pragma unroll
  for (int m = kRoleGroup / 2; m > 0; m >>= 1) x = min(x, __shfl_xor(x, m, kWave));
  return x;
}
__device__ __forceinline__ int32_t group_max(int32_t x) {
#pragma unroll
  for (int m = kRoleGroup / 2; m > 0; m >>= 1) x = max(x, __shfl_xor(x, m, kWave));
  return x;
}

__global__ __launch_bounds__(256) void k_q_roles(IndexView ix, const int32_t *memb, uint8_t *roles) {
  constexpr int kPerWave = kWave / kRoleGroup;
  const int lane = threadIdx.x & (kWave - 1), pos = lane % kRoleGroup;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / kWave;
  for (int64_t v0 = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kWave * kPerWave; v0 < ix.n;
       v0 += nw * kPerWave) {
    const int64_t v = v0 + lane / kRoleGroup;
    int64_t b = 0, e = 0;
    bool unclustered = false;
    if (v < ix.n) {
      unclustered = memb[v] < 0;
      b = ix.off[v];
      e = ix.off[v + 1];
    }
    const bool group_row = unclustered && e - b <= kRoleGroupMax;
    uint8_t role = kRoleClustered;
    if (group_row) {  // the same for every lane of the group
      int32_t first = -1;
      bool hub = false;
      for (int64_t k0 = b; k0 < e && !hub; k0 += kRoleGroup) {
        const int64_t k = k0 + pos;
        const int32_t lab = k < e ? memb[ix.no_ids[k]] : -1;
        const int32_t lo = group_min(lab >= 0 ? lab : INT_MAX);
        const int32_t hi = group_max(lab);
        if (lo != INT_MAX) {
          if (first < 0) first = lo;
          hub = lo != first || hi != first;
        }
      }
      role = hub ? kRoleHub : kRoleOutlier;
    }
    // long unclustered rows: one at a time by the whole wavefront
    uint64_t longs = __ballot(unclustered && !group_row && pos == 0);
    while (longs) {
      const int src = __ffsll((unsigned long long)longs) - 1;
      longs &= longs - 1;
      const int64_t rb = (int64_t)(uint32_t)__builtin_amdgcn_readlane((int32_t)b, src) |
                         ((int64_t)__builtin_amdgcn_readlane((int32_t)(b >> 32), src) << 32);
      const int64_t re = (int64_t)(uint32_t)__builtin_amdgcn_readlane((int32_t)e, src) |
                         ((int64_t)__builtin_amdgcn_readlane((int32_t)(e >> 32), src) << 32);
      // kRoleSteps * kWave ids per iteration, all of their loads issued
      // before the labels are reduced (smallest and largest over the wave)
      int32_t first = -1;
      bool hub = false;
      for (int64_t k0 = rb; k0 < re && !hub; k0 += kRoleSteps * kWave) {  // uniform bounds and exit
        int32_t w[kRoleSteps];
#pragma unroll
        for (int j = 0; j < kRoleSteps; ++j) {
          const int64_t k = k0 + j * kWave + lane;
          w[j] = k < re ? ix.no_ids[k] : -1;
        }
        int32_t lo = INT_MAX, hi = -1;
#pragma unroll
        for (int j = 0; j < kRoleSteps; ++j) {
          const int32_t lab = w[j] >= 0 ? memb[w[j]] : -1;
          if (lab >= 0) {
            lo = min(lo, lab);
            hi = max(hi, lab);
          }
        }
#pragma unroll
        for (int m = kWave / 2; m > 0; m >>= 1) {
          lo = min(lo, __shfl_xor(lo, m, kWave));
          hi = max(hi, __shfl_xor(hi, m, kWave));
        }
        if (lo != INT_MAX) {
          if (first < 0) first = lo;
          hub = lo != first || hi != first;
        }
      }
      if (lane / kRoleGroup == src / kRoleGroup) role = hub ? kRoleHub : kRoleOutlier;
    }
    if (v < ix.n && pos == 0) roles[v] = role;
  }
}

void launch_roles(const scan_index *ix, const int32_t *memb, uint8_t *roles, hipStream_t s) {
  IndexView v{ix->n, ix->dmax, ix->off, ix->no_ids, ix->no_sim, ix->co_off, ix->co_ids, ix->co_thr};
  k_q_roles<<<grid_for((ix->n + kWave / kRoleGroup - 1) / (kWave / kRoleGroup) * kWave, 256), 256, 0, s>>>(
      v, memb, roles);
}

// ---------------------------------------------------------------------------
// Allocation-free query: the slot workspace and the descriptor live in a
// file-scope device array instead of allocated memory. Layout: the
// descriptor, then parent int32[n], then the state bytes uint8[n].

constexpr size_t kNoAllocDescBytes = 256;
constexpr int64_t kNoAllocMaxN = (int64_t)1 << 23;
constexpr size_t kNoAllocScratchBytes = kNoAllocDescBytes + (size_t)kNoAllocMaxN * 5;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

// The device address of `scratch` on each device, taken once per device with
// that device current (the host-side name of the array is not a device
// address).
static std::mutex g_scratch_mu;
static std::vector<void *> g_scratch_ptr;

static scan_status scratch_address(int device, unsigned char **out) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if ((int)g_scratch_ptr.size() <= device) g_scratch_ptr.resize(device + 1, nullptr);
  if (!g_scratch_ptr[device]) {
    int cur = 0;
    SCAN_HIP_TRY(hipGetDevice(&cur));
    if (cur != device) SCAN_HIP_TRY(hipSetDevice(device));
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != device) (void)hipSetDevice(cur);
    if (e != hipSuccess || !p)
      return fail(SCAN_EDEVICE, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
    g_scratch_ptr[device] = p;
  }
  *out = (unsigned char *)g_scratch_ptr[device];
  return SCAN_OK;
}

// Clears the state bytes (the query kernels expect them all zero) and writes
// the descriptor from kernel arguments: no host copy, no memset node.
__global__ void k_q_noalloc_init(QueryDesc *d, int32_t mu, double eps, int32_t *parent, uint8_t *flag,
                                 int64_t n, int32_t *memb, uint8_t *is_core) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    flag[i] = 0;
  if (blockIdx.x == 0 && threadIdx.x == 0) *d = QueryDesc{mu, 0, eps, 0, 0, parent, flag, memb, is_core};
}

scan_status query_noalloc(const scan_index *ix, int32_t mu, double eps, int32_t *memberships, uint8_t *is_core,
                          hipStream_t s) {
  if (ix->n > kNoAllocMaxN)
    return fail(SCAN_EINVAL, "scan_query_noalloc takes indexes of at most %lld vertices (this one has %lld)",
                (long long)kNoAllocMaxN, (long long)ix->n);
  unsigned char *base;
  SCAN_TRY(scratch_address(ix->device, &base));
  if (ix->n == 0) return SCAN_OK;
  QueryDesc *d = (QueryDesc *)base;
  int32_t *parent = (int32_t *)(base + kNoAllocDescBytes);
  uint8_t *flag = (uint8_t *)(parent + ix->n);
  k_q_noalloc_init<<<grid_for(ix->n, 256, 2048), 256, 0, s>>>(d, mu, eps, parent, flag, ix->n, memberships,
                                                               is_core);
  launch_query_kernels(ix, d, 1, s);
  SCAN_HIP_TRY(hipGetLastError());
  return SCAN_OK;
}

QueryDesc make_query_desc(int32_t mu, double eps, const QuerySlot &slot, int32_t *memb,
                          uint8_t *is_core) {
  return QueryDesc{mu, 0, eps, 0, 0, slot.parent, slot.flag, memb, is_core};
}

scan_status alloc_query_slot(const scan_index *ix, QuerySlot *slot, hipStream_t s) {
  size_t n = (size_t)(ix->n > 0 ? ix->n : 1);
  slot->bytes = n * 4 + n;
  slot->parent = (int32_t *)dev_alloc(n * 4, s);
  slot->flag = (uint8_t *)dev_alloc(n, s);
  if (!slot->parent || !slot->flag) {
    free_query_slot(slot, s);
    return fail(SCAN_ENOMEM, "query workspace allocation failed");
  }
  hipError_t e = hipMemsetAsync(slot->flag, 0, n, s);
  if (e != hipSuccess) return fail(SCAN_EDEVICE, "hipMemsetAsync: %s", hipGetErrorString(e));
  return SCAN_OK;
}

void free_query_slot(QuerySlot *slot, hipStream_t s) {
  size_t n = slot->bytes / 5;
  if (slot->parent) dev_free(slot->parent, n * 4, s);
  if (slot->flag) dev_free(slot->flag, n, s);
  slot->parent = nullptr;
  slot->flag = nullptr;
}

scan_status run_queries(const scan_index *ix, int32_t count, const int32_t *mu, const double *eps,
                        int32_t *const *memberships, uint8_t *const *is_core,
                        const QuerySlot *slots, hipStream_t s) {
  if (count <= 0) return SCAN_OK;
  std::vector<QueryDesc> h(count);
  for (int32_t i = 0; i < count; ++i) {
    h[i] = QueryDesc{mu[i], 0, eps[i], 0, 0, slots[i].parent, slots[i].flag, memberships[i],
                     is_core ? is_core[i] : nullptr};
  }
  QueryDesc *d = (QueryDesc *)dev_alloc(sizeof(QueryDesc) * count, s);
  if (!d) return fail(SCAN_ENOMEM, "query descriptor allocation failed");
  hipError_t e = hipMemcpyAsync(d, h.data(), sizeof(QueryDesc) * count, hipMemcpyHostToDevice, s);
  if (e != hipSuccess) {
    dev_free(d, sizeof(QueryDesc) * count, s);
    return fail(SCAN_EDEVICE, "hipMemcpyAsync: %s", hipGetErrorString(e));
  }
  // The descriptors are copied from pageable host memory: wait for the copy
  // before the host vector goes out of scope.
  e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail(SCAN_EDEVICE, "hipStreamSynchronize: %s", hipGetErrorString(e));
  launch_query_kernels(ix, d, count, s);
  e = hipGetLastError();
  dev_free(d, sizeof(QueryDesc) * count, s);
  if (e != hipSuccess) return fail(SCAN_EDEVICE, "query launch: %s", hipGetErrorString(e));
  return SCAN_OK;
}

}  // namespace scan
