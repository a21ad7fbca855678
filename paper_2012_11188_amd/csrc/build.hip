// Index construction (Section 4.1): per-edge similarity (Algorithm 1), the
// neighbour order and the core order (Algorithm 2), for one graph.
//
// GPU design (differs from the paper's 48-core CPU design, which merges
// degree-oriented sorted lists with atomic per-edge counters):
//   * Every undirected edge {u, h} is owned by its endpoint that is larger in
//     the order (degree, id). The owner's row N(h) is staged once in an LDS
//     hash table; each lower neighbour u streams its row N(u) (coalesced) and
//     probes it, so each edge costs min(|N[u]|, |N[h]|)-ish probes, the
//     min-side rule of Algorithm 1, with no global atomics.
//   * Owners are bucketed by degree into table-size classes (one launch each,
//     LDS sized to the class); rows of very high degree are split into id
//     ranges that fit the largest table and probed part by part.
//   * The count and the FP64 similarity are fused: the probing wave computes
//     c = t + 2 and writes the similarity into both CSR slots of the edge (the
//     mirror slot is the position of h found while streaming N(u)).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "index.h"

namespace scan {

// ---------------------------------------------------------------------------
// a1: degrees, int64 offsets, maximum degree.

template <class OffT>
__global__ void k_prepare(const OffT *off_in, int64_t n, int64_t *off, int32_t *deg,
                          unsigned long long *dmax) {
  unsigned long long local = 0;
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v <= n;
       v += (int64_t)gridDim.x * blockDim.x) {
    int64_t o = (int64_t)off_in[v];
    off[v] = o;
    if (v < n) {
      int64_t d = (int64_t)off_in[v + 1] - o;
      deg[v] = (int32_t)d;
      local = max(local, (unsigned long long)(d > 0 ? d : 0));
    }
  }
  for (int m = kWave / 2; m > 0; m >>= 1) local = max(local, __shfl_xor(local, m, kWave));
  if ((threadIdx.x & (kWave - 1)) == 0) atomicMax(dmax, local);
}

// Optional CSR validation (Section 2.2: simple undirected graph): offsets
// monotone from 0 to nnz, ids in range, no self-loops, rows strictly
// ascending, every edge present in both directions. err[0] = 1 on failure,
// err[1] = smallest offending row seen (atomicMin).
template <class OffT>
__global__ void k_validate(const OffT *off, const int32_t *adj, int64_t n, int64_t nnz,
                           int32_t *err) {
  int lane = threadIdx.x & (kWave - 1);
  int64_t w = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kWave;
  int64_t nw = ((int64_t)gridDim.x * blockDim.x) / kWave;
  for (int64_t v = w; v < n; v += nw) {
    int64_t b = (int64_t)off[v], e = (int64_t)off[v + 1];
    bool bad = b < 0 || e < b || e > nnz || (v == 0 && b != 0) || (v == n - 1 && e != nnz);
    if (!bad) {
      for (int64_t s = b + lane; s < e; s += kWave) {
        int64_t x = adj[s];
        bool ok = x >= 0 && x < n && x != v && (s == b || adj[s - 1] < x);
        if (ok) {
          int64_t lo = (int64_t)off[x], hi = (int64_t)off[x + 1];
          ok = lo >= 0 && hi >= lo && hi <= nnz;
          while (ok && lo < hi) {
            int64_t mid = (lo + hi) >> 1;
            if (adj[mid] < v) lo = mid + 1;
            else hi = mid;
          }
          ok = ok && lo < (int64_t)off[x + 1] && adj[lo] == v;
        }
        bad |= !ok;
      }
    }
    if (__any(bad) && lane == 0) {
      err[0] = 1;
      atomicMin(&err[1], (int32_t)v);
    }
  }
}

// ---------------------------------------------------------------------------
// a2: ownership and chunk planning.

__device__ __forceinline__ bool is_lower(int32_t u, int32_t du, int32_t h, int32_t dh) {
  return du < dh || (du == dh && u < h);
}

struct Chunk {
  int32_t h;  // owner
  int32_t k;  // chunk index within row h
};

constexpr int kNumClasses = 8;  // table classes small_log_t .. big_log_t

struct PlanStats {
  int32_t chunks[kNumClasses];
  int32_t owners;
};

// One wavefront per vertex h: counts its lower neighbours; if any, appends the
// chunks covering row h to the list of h's table class.
__global__ void k_plan(const int64_t *off, const int32_t *deg, const int32_t *adj, int64_t n,
                       int small_log_t, int big_log_t, int spc_small, int spc_big, Chunk *lists,
                       int64_t cap, PlanStats *st) {
  int lane = threadIdx.x & (kWave - 1);
  int64_t w = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kWave;
  int64_t nw = ((int64_t)gridDim.x * blockDim.x) / kWave;
  for (int64_t h = w; h < n; h += nw) {
    int32_t dh = deg[h];
    if (dh == 0) continue;
    int64_t b = off[h];
    bool any_lower = false;
    for (int64_t s = b + lane; s < b + dh && !any_lower; s += kWave) {
      int32_t u = adj[s];
      bool lw = is_lower(u, deg[u], (int32_t)h, dh);
      any_lower = __any(lw);
    }
    if (!any_lower) continue;
    int cls = 0;
    while (small_log_t + cls < big_log_t && (int64_t)dh > ((int64_t)1 << (small_log_t + cls - 1)))
      ++cls;
    int spc = (small_log_t + cls == big_log_t) ? spc_big : spc_small;
    int32_t nch = (dh + spc - 1) / spc;
    int32_t base = 0;
    if (lane == 0) {
      base = atomicAdd(&st->chunks[cls], nch);
      atomicAdd(&st->owners, 1);
    }
    base = __shfl(base, 0, kWave);
    for (int32_t k = lane; k < nch; k += kWave) lists[cls * cap + base + k] = Chunk{(int32_t)h, k};
  }
}

// ---------------------------------------------------------------------------
// a3 + a4: intersection and similarity.

__device__ __forceinline__ uint32_t hash_slot(int32_t x, int log_t) {
  return ((uint32_t)x * 0x9E3779B1u) >> (32 - log_t);
}

// One workgroup per chunk (owner h, row slots [s0, s1)). The row of h is
// inserted into the LDS table part by part (parts of at most 2^(LOG_T-1)
// ids, covering consecutive id ranges); for every lower neighbour u in the
// chunk one wavefront streams the part of N(u) inside the current id range
// and counts table hits.
template <int LOG_T>
__global__ __launch_bounds__(512) void k_intersect(const Chunk *chunks, int32_t nchunks, int spc,
                                                   const int64_t *off, const int32_t *deg,
                                                   const int32_t *adj, int kind, double *sims,
                                                   int32_t *counts) {
  constexpr int T = 1 << LOG_T;
  constexpr int CAP = T / 2;
  extern __shared__ unsigned char smem[];
  int32_t *tab = (int32_t *)smem;
  int32_t *cnt = tab + T;
  int64_t *mir = (int64_t *)(cnt + ((spc + 1) & ~1));
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
  const int nwaves = blockDim.x / kWave;

  for (int32_t ci = blockIdx.x; ci < nchunks; ci += gridDim.x) {
    const Chunk ch = chunks[ci];
    const int32_t h = ch.h;
    const int32_t dh = deg[h];
    const int64_t oh = off[h];
    const int64_t s0 = oh + (int64_t)ch.k * spc;
    const int m = (int)min((int64_t)spc, oh + dh - s0);
    const int parts = (dh + CAP - 1) / CAP;
    __syncthreads();
    for (int e = threadIdx.x; e < m; e += blockDim.x) {
      cnt[e] = 0;
      mir[e] = -1;
    }
    for (int p = 0; p < parts; ++p) {
      const int p0 = p * CAP, p1 = min(dh, p0 + CAP);
      const int32_t lo = p == 0 ? INT32_MIN : adj[oh + p0];
      const int32_t hi = p == parts - 1 ? INT32_MAX : adj[oh + p1];
      __syncthreads();
      for (int i = threadIdx.x; i < T; i += blockDim.x) tab[i] = -1;
      __syncthreads();
      for (int i = p0 + threadIdx.x; i < p1; i += blockDim.x) {
        int32_t x = adj[oh + i];
        uint32_t pos = hash_slot(x, LOG_T);
        while (atomicCAS(&tab[pos], -1, x) != -1) pos = (pos + 1) & (T - 1);
      }
      __syncthreads();
      for (int e = wave; e < m; e += nwaves) {
        const int32_t u = adj[s0 + e];
        const int32_t du = deg[u];
        if (!is_lower(u, du, h, dh)) continue;
        const int64_t ou = off[u];
        int64_t b0 = 0, b1 = du;
        if (parts > 1) {
          // positions in N(u) with lo <= x < hi (all lanes search alike)
          int64_t a = 0, z = du;
          while (a < z) {
            int64_t mid = (a + z) >> 1;
            if (adj[ou + mid] < lo) a = mid + 1;
            else z = mid;
          }
          b0 = a;
          z = du;
          while (a < z) {
            int64_t mid = (a + z) >> 1;
            if (adj[ou + mid] < hi) a = mid + 1;
            else z = mid;
          }
          b1 = a;
        }
        int32_t t = 0;
        int64_t mpos = -1;
        for (int64_t base = b0; base < b1; base += kWave) {
          int64_t i = base + lane;
          bool valid = i < b1;
          int32_t x = valid ? adj[ou + i] : -1;
          bool hit = false;
          if (valid) {
            uint32_t pos = hash_slot(x, LOG_T);
            for (;;) {
              int32_t y = tab[pos];
              if (y == x) { hit = true; break; }
              if (y == -1) break;
              pos = (pos + 1) & (T - 1);
            }
          }
          t += __popcll(__ballot(hit));
          unsigned long long own = __ballot(valid && x == h);
          if (own) mpos = ou + base + (__ffsll(own) - 1);
        }
        if (lane == 0) {
          cnt[e] += t;
          if (mpos >= 0) mir[e] = mpos;
        }
      }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < m; e += blockDim.x) {
      const int64_t s = s0 + e;
      const int32_t u = adj[s];
      const int32_t du = deg[u];
      if (!is_lower(u, du, h, dh)) continue;
      const int64_t c = (int64_t)cnt[e] + 2;
      const double x = similarity(kind, c, (int64_t)du + 1, (int64_t)dh + 1);
      sims[s] = x;
      if (mir[e] >= 0) sims[mir[e]] = x;
      if (counts) {
        counts[s] = (int32_t)c;
        if (mir[e] >= 0) counts[mir[e]] = (int32_t)c;
      }
    }
  }
}

template <int LOG_T>
static void launch_intersect(const Chunk *chunks, int32_t nchunks, int spc, int waves,
                             const int64_t *off, const int32_t *deg, const int32_t *adj, int kind,
                             double *sims, int32_t *counts, hipStream_t s) {
  size_t lds = (size_t)(1 << LOG_T) * 4 + (size_t)((spc + 1) & ~1) * 4 + (size_t)spc * 8;
  if (lds > 65536)
    (void)hipFuncSetAttribute((const void *)k_intersect<LOG_T>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  k_intersect<LOG_T><<<grid_for(nchunks, 1, 1 << 20), waves * kWave, lds, s>>>(
      chunks, nchunks, spc, off, deg, adj, kind, sims, counts);
}

static scan_status intersect_class(int log_t, const Chunk *chunks, int32_t nchunks, int spc,
                                   int waves, const int64_t *off, const int32_t *deg,
                                   const int32_t *adj, int kind, double *sims, int32_t *counts,
                                   hipStream_t s) {
  switch (log_t) {
#define SCAN_CASE(L) \
  case L: launch_intersect<L>(chunks, nchunks, spc, waves, off, deg, adj, kind, sims, counts, s); break;
    SCAN_CASE(7) SCAN_CASE(8) SCAN_CASE(9) SCAN_CASE(10) SCAN_CASE(11) SCAN_CASE(12)
    SCAN_CASE(13) SCAN_CASE(14) SCAN_CASE(15)
#undef SCAN_CASE
    default:
      return fail(SCAN_EINVAL, "unsupported table class 2^%d", log_t);
  }
  SCAN_HIP_TRY(hipGetLastError());
  return SCAN_OK;
}

// ---------------------------------------------------------------------------
// a6: core order placement. With E = exclusive prefix of the degree
// histogram, |CO[mu]| = n - E[mu-1]; vertex v gets a rank r(v) among the
// vertices of degree >= deg(v) (vertices of higher degree first), so its
// entry for mu = j + 2 lands at co_off[mu] + r(v), inside segment mu.

__global__ void k_degree_hist(const int32_t *deg, int64_t n, int32_t *hist) {
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x)
    atomicAdd(&hist[deg[v]], 1);
}

__global__ void k_co_sizes(const int64_t *E, int64_t n, int64_t dmax, int64_t *sizes) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < dmax;
       i += (int64_t)gridDim.x * blockDim.x)
    sizes[i] = n - E[i + 1];  // mu = i + 2: vertices with deg >= mu - 1 = i + 1
}

__global__ void k_co_finish_off(const int64_t *scan, int64_t dmax, int64_t *co_off) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i <= dmax + 2;
       i += (int64_t)gridDim.x * blockDim.x)
    co_off[i] = i < 2 ? 0 : scan[i - 2];
}

__global__ void k_co_place(const int64_t *off, const int32_t *deg, int64_t n, const int64_t *E,
                           int32_t *cursor, const int64_t *co_off, const double *no_sim,
                           double *co_key, int32_t *co_id) {
  int lane = threadIdx.x & (kWave - 1);
  int64_t w = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kWave;
  int64_t nw = ((int64_t)gridDim.x * blockDim.x) / kWave;
  for (int64_t v = w; v < n; v += nw) {
    int32_t d = deg[v];
    if (d == 0) continue;
    int64_t r = 0;
    if (lane == 0) r = (n - E[d + 1]) + atomicAdd(&cursor[d], 1);
    r = __shfl(r, 0, kWave);
    int64_t o = off[v];
    for (int32_t j = lane; j < d; j += kWave) {
      int64_t pos = co_off[j + 2] + r;
      co_key[pos] = no_sim[o + j];
      co_id[pos] = (int32_t)v;
    }
  }
}

__global__ void k_similarity_values(int kind, int64_t count, const int64_t *c, const int64_t *a,
                                   const int64_t *b, double *out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = similarity(kind, c[i], a[i], b[i]);
}

scan_status similarity_values(int32_t kind, int64_t count, const int64_t *c, const int64_t *a_u,
                              const int64_t *a_v, double *out) {
  hipStream_t s = nullptr;
  DevArena tmp(s);
  int64_t *dc, *da, *db;
  double *dout;
  SCAN_TRY(tmp.alloc(&dc, count));
  SCAN_TRY(tmp.alloc(&da, count));
  SCAN_TRY(tmp.alloc(&db, count));
  SCAN_TRY(tmp.alloc(&dout, count));
  SCAN_HIP_TRY(hipMemcpyAsync(dc, c, count * 8, hipMemcpyHostToDevice, s));
  SCAN_HIP_TRY(hipMemcpyAsync(da, a_u, count * 8, hipMemcpyHostToDevice, s));
  SCAN_HIP_TRY(hipMemcpyAsync(db, a_v, count * 8, hipMemcpyHostToDevice, s));
  k_similarity_values<<<grid_for(count, 256), 256, 0, s>>>(kind, count, dc, da, db, dout);
  SCAN_HIP_TRY(hipGetLastError());
  SCAN_HIP_TRY(hipMemcpyAsync(out, dout, count * 8, hipMemcpyDeviceToHost, s));
  SCAN_HIP_TRY(hipStreamSynchronize(s));
  return SCAN_OK;
}

// ---------------------------------------------------------------------------
// Host orchestration.

IntersectConfig default_config() { return IntersectConfig{}; }

scan_status index_alloc(scan_index *ix, void **p, size_t bytes) {
  if (bytes == 0) bytes = 8;
  void *q = dev_alloc(bytes, ix->stream);
  if (!q) return fail(SCAN_ENOMEM, "device allocation of %zu bytes failed", bytes);
  ix->allocs.push_back({q, bytes});
  ix->bytes += (int64_t)bytes;
  *p = q;
  return SCAN_OK;
}

void index_release(scan_index *ix) {
  for (auto &a : ix->allocs) dev_free(a.p, a.bytes, ix->stream);
  ix->allocs.clear();
}

namespace {

struct Staged {
  const void *offsets;
  const int32_t *adj;
};

scan_status check_csr(const scan_csr *g) {
  if (!g) return fail(SCAN_EINVAL, "null graph");
  if (g->n < 0 || g->nnz < 0) return fail(SCAN_EINVAL, "negative n or nnz");
  if (g->nnz % 2) return fail(SCAN_EINVAL, "odd nnz (%lld): an undirected CSR stores both directions", (long long)g->nnz);
  if (g->offset_bits != 32 && g->offset_bits != 64) return fail(SCAN_EINVAL, "offset_bits must be 32 or 64");
  if (g->n > 0x7fffffffLL) return fail(SCAN_EINVAL, "n exceeds int32 vertex ids");
  if (g->offset_bits == 32 && g->nnz > 0x7fffffffLL) return fail(SCAN_EINVAL, "nnz exceeds 32-bit offsets");
  if (g->n > 0 && !g->offsets) return fail(SCAN_EINVAL, "null offsets");
  if (g->nnz > 0 && !g->adj) return fail(SCAN_EINVAL, "null adj");
  return SCAN_OK;
}

}  // namespace

scan_status build_index(const scan_csr *g, int32_t kind, uint32_t flags, hipStream_t s,
                        const IntersectConfig &cfg, scan_index **out) {
  SCAN_TRY(check_csr(g));
  if (kind != SCAN_SIM_COSINE && kind != SCAN_SIM_JACCARD) return fail(SCAN_EINVAL, "unknown similarity kind %d", kind);
  if (flags & ~(uint32_t)(SCAN_VALIDATE | SCAN_KEEP_SIMS | SCAN_KEEP_COUNTS | SCAN_PROFILE)) return fail(SCAN_EINVAL, "unknown build flags 0x%x", flags);
  if (cfg.small_log_t < 7 || cfg.big_log_t > 15 || cfg.small_log_t > cfg.big_log_t ||
      cfg.big_log_t - cfg.small_log_t >= kNumClasses || cfg.spc_small < 1 || cfg.spc_big < 1 ||
      cfg.waves_big < 1 || cfg.waves_big > 8)
    return fail(SCAN_EINVAL, "bad intersection config");
  const int64_t n = g->n, nnz = g->nnz;
  const int osz = g->offset_bits / 8;

  scan_index *ix = new scan_index();
  ix->n = n;
  ix->nnz = nnz;
  ix->kind = kind;
  ix->flags = flags & (SCAN_KEEP_SIMS | SCAN_KEEP_COUNTS | SCAN_PROFILE);
  ix->stream = s;
  (void)hipGetDevice(&ix->device);
  const bool prof = (flags & SCAN_PROFILE) != 0;
  if (prof) {
    for (auto &e : ix->ev)
      if (hipEventCreate(&e) != hipSuccess) {
        delete ix;
        return fail(SCAN_EDEVICE, "hipEventCreate failed");
      }
  }
  auto mark = [&](int k) {
    if (prof) (void)hipEventRecord(ix->ev[k], s);
  };
  // The largest table class must fit the device's LDS per workgroup.
  IntersectConfig cf = cfg;
  {
    int lds_max = 65536;
    (void)hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, ix->device);
    auto lds_of = [&](int log_t) { return ((size_t)1 << log_t) * 4 + (size_t)((cf.spc_big + 1) & ~1) * 4 + (size_t)cf.spc_big * 8; };
    while (cf.big_log_t > cf.small_log_t && lds_of(cf.big_log_t) > (size_t)lds_max) --cf.big_log_t;
  }
  auto bail = [&](scan_status st) {
    index_release(ix);
    delete ix;
    return st;
  };
#define BTRY(expr)                      \
  do {                                  \
    scan_status st_ = (expr);           \
    if (st_ != SCAN_OK) return bail(st_); \
  } while (0)
#define BHIP(expr)                                                                      \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return bail(fail(SCAN_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)));   \
  } while (0)

  DevArena tmp(s);
  mark(0);
  Staged in{g->offsets, g->adj};
  if (!g->on_device && n > 0) {
    void *doff;
    int32_t *dadj;
    BTRY(tmp.alloc((unsigned char **)&doff, (n + 1) * osz));
    BTRY(tmp.alloc(&dadj, nnz));
    BHIP(hipMemcpyAsync(doff, g->offsets, (size_t)(n + 1) * osz, hipMemcpyHostToDevice, s));
    if (nnz) BHIP(hipMemcpyAsync(dadj, g->adj, (size_t)nnz * 4, hipMemcpyHostToDevice, s));
    in.offsets = doff;
    in.adj = dadj;
  }

  BTRY(index_alloc(ix, (void **)&ix->off, (size_t)(n + 1) * 8));
  int32_t *deg;
  unsigned long long *d_dmax;
  int32_t *d_err;
  BTRY(tmp.alloc(&deg, n));
  BTRY(tmp.alloc(&d_dmax, 1));
  BTRY(tmp.alloc(&d_err, 2));
  BHIP(hipMemsetAsync(d_dmax, 0, 8, s));
  if (n > 0) {
    if (osz == 4)
      k_prepare<int32_t><<<grid_for(n + 1, 256), 256, 0, s>>>((const int32_t *)in.offsets, n, ix->off, deg, d_dmax);
    else
      k_prepare<int64_t><<<grid_for(n + 1, 256), 256, 0, s>>>((const int64_t *)in.offsets, n, ix->off, deg, d_dmax);
  } else {
    BHIP(hipMemsetAsync(ix->off, 0, 8, s));
  }
  if ((flags & SCAN_VALIDATE) && n > 0) {
    int32_t init[2] = {0, 0x7fffffff};
    BHIP(hipMemcpyAsync(d_err, init, 8, hipMemcpyHostToDevice, s));
    if (osz == 4)
      k_validate<int32_t><<<grid_for(n * kWave, 256), 256, 0, s>>>((const int32_t *)in.offsets, in.adj, n, nnz, d_err);
    else
      k_validate<int64_t><<<grid_for(n * kWave, 256), 256, 0, s>>>((const int64_t *)in.offsets, in.adj, n, nnz, d_err);
    int32_t herr[2];
    BHIP(hipMemcpyAsync(herr, d_err, 8, hipMemcpyDeviceToHost, s));
    BHIP(hipStreamSynchronize(s));
    if (herr[0]) return bail(fail(SCAN_EGRAPH, "graph is not a simple undirected CSR with ascending rows (first bad row %d)", herr[1]));
  }
  unsigned long long hdmax = 0;
  BHIP(hipMemcpyAsync(&hdmax, d_dmax, 8, hipMemcpyDeviceToHost, s));
  BHIP(hipStreamSynchronize(s));
  const int64_t dmax = (int64_t)hdmax;
  ix->dmax = dmax;
  mark(1);

  BTRY(index_alloc(ix, (void **)&ix->no_ids, (size_t)nnz * 4));
  BTRY(index_alloc(ix, (void **)&ix->no_sim, (size_t)nnz * 8));
  BTRY(index_alloc(ix, (void **)&ix->co_off, (size_t)(dmax + 3) * 8));
  BTRY(index_alloc(ix, (void **)&ix->co_ids, (size_t)nnz * 4));
  BTRY(index_alloc(ix, (void **)&ix->co_thr, (size_t)nnz * 8));
  double *sims;
  if (flags & SCAN_KEEP_SIMS) {
    BTRY(index_alloc(ix, (void **)&ix->sims, (size_t)nnz * 8));
    sims = ix->sims;
  } else {
    BTRY(tmp.alloc(&sims, nnz));
  }
  if (flags & SCAN_KEEP_COUNTS) BTRY(index_alloc(ix, (void **)&ix->counts, (size_t)nnz * 4));

  if (nnz == 0) {
    BHIP(hipMemsetAsync(ix->co_off, 0, (size_t)(dmax + 3) * 8, s));
    for (int k = 2; k < 6; ++k) mark(k);
    *out = ix;
    return SCAN_OK;
  }

  // a2: plan chunks per table class.
  const int ncls = cf.big_log_t - cf.small_log_t + 1;
  const int64_t cap = n + nnz / std::min(cf.spc_small, cf.spc_big) + 1;
  Chunk *lists;
  PlanStats *d_plan;
  BTRY(tmp.alloc(&lists, cap * ncls));
  BTRY(tmp.alloc(&d_plan, 1));
  BHIP(hipMemsetAsync(d_plan, 0, sizeof(PlanStats), s));
  k_plan<<<grid_for(n * kWave, 256), 256, 0, s>>>(ix->off, deg, in.adj, n, cf.small_log_t, cf.big_log_t,
                                                  cf.spc_small, cf.spc_big, lists, cap, d_plan);
  PlanStats plan;
  BHIP(hipMemcpyAsync(&plan, d_plan, sizeof(plan), hipMemcpyDeviceToHost, s));
  BHIP(hipStreamSynchronize(s));
  ix->owners = plan.owners;
  mark(2);

  // a3 + a4: one launch per class.
  for (int c = 0; c < ncls; ++c) {
    if (!plan.chunks[c]) continue;
    int log_t = cf.small_log_t + c;
    bool big = log_t == cf.big_log_t;
    BTRY(intersect_class(log_t, lists + c * cap, plan.chunks[c], big ? cf.spc_big : cf.spc_small,
                         big ? cf.waves_big : 4, ix->off, deg, in.adj, kind, sims, ix->counts, s));
    ++ix->intersect_launches;
  }
  mark(3);

  // a5: neighbour order = rows sorted by (sim desc, id asc).
  BTRY(segmented_sort(ix->off, n, nnz, sims, in.adj, ix->no_sim, ix->no_ids, s));
  mark(4);

  // a6: core order.
  int32_t *hist, *cursor;
  int64_t *E, *sizes, *co_scan, *scan_ws;
  double *co_key;
  int32_t *co_id;
  BTRY(tmp.alloc(&hist, dmax + 1));
  BTRY(tmp.alloc(&cursor, dmax + 1));
  BTRY(tmp.alloc(&E, dmax + 2));
  BTRY(tmp.alloc(&sizes, dmax));
  BTRY(tmp.alloc(&co_scan, dmax + 1));
  BTRY(tmp.alloc(&scan_ws, scan_workspace_elems(std::max<int64_t>(n, dmax + 1))));
  BTRY(tmp.alloc(&co_key, nnz));
  BTRY(tmp.alloc(&co_id, nnz));
  BHIP(hipMemsetAsync(hist, 0, (size_t)(dmax + 1) * 4, s));
  BHIP(hipMemsetAsync(cursor, 0, (size_t)(dmax + 1) * 4, s));
  k_degree_hist<<<grid_for(n, 256), 256, 0, s>>>(deg, n, hist);
  BTRY(exclusive_scan(hist, E, dmax + 1, scan_ws, s));
  k_co_sizes<<<grid_for(dmax, 256), 256, 0, s>>>(E, n, dmax, sizes);
  BTRY(exclusive_scan64(sizes, co_scan, dmax, scan_ws, s));
  k_co_finish_off<<<grid_for(dmax + 3, 256), 256, 0, s>>>(co_scan, dmax, ix->co_off);
  k_co_place<<<grid_for(n * kWave, 256), 256, 0, s>>>(ix->off, deg, n, E, cursor, ix->co_off, ix->no_sim,
                                                     co_key, co_id);
  BTRY(segmented_sort(ix->co_off + 2, dmax, nnz, co_key, co_id, ix->co_thr, ix->co_ids, s));
  mark(5);
  BHIP(hipGetLastError());
  *out = ix;
  return SCAN_OK;
#undef BTRY
#undef BHIP
}

scan_status build_index_batch(const scan_csr *gs, int32_t count, int32_t kind, uint32_t flags,
                              hipStream_t s, const IntersectConfig &cfg, scan_index **outs) {
  if (count < 0 || (count > 0 && (!gs || !outs))) return fail(SCAN_EINVAL, "bad batch arguments");
  for (int32_t i = 0; i < count; ++i) {
    outs[i] = nullptr;
    SCAN_TRY(check_csr(&gs[i]));
  }
  for (int32_t i = 0; i < count; ++i) {
    scan_status st = build_index(&gs[i], kind, flags, s, cfg, &outs[i]);
    if (st != SCAN_OK) {
      for (int32_t j = 0; j < i; ++j) {
        index_release(outs[j]);
        delete outs[j];
        outs[j] = nullptr;
      }
      return st;
    }
  }
  return SCAN_OK;
}

}  // namespace scan
