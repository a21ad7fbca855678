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
// a6: core order placement. With E = exclusive prefix of the degree
// histogram, |CO[mu]| = n - E[mu-1]; vertex v gets a rank r(v) among the
// vertices of degree >= deg(v) (vertices of higher degree first), so its
// entry for mu = j + 2 lands at co_off[mu] + r(v), inside segment mu.

constexpr int kHistBins = 2048;  // degrees below this are binned in LDS first

__global__ __launch_bounds__(256) void k_degree_hist(const int32_t *deg, int64_t n, int64_t dmax,
                                                     int32_t *hist) {
  __shared__ int32_t lh[kHistBins];
  const int bins = (int)min((int64_t)kHistBins, dmax + 1);
  for (int i = threadIdx.x; i < bins; i += blockDim.x) lh[i] = 0;
  __syncthreads();
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x) {
    const int32_t d = deg[v];
    if (d < kHistBins) atomicAdd(&lh[d], 1);
    else atomicAdd(&hist[d], 1);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < bins; i += blockDim.x)
    if (lh[i]) atomicAdd(&hist[i], lh[i]);
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

// Rank of every non-isolated vertex in degree-descending order (ties in any
// order: each CO segment is sorted afterwards). One workgroup per tile of
// kRankTile consecutive vertices: LDS counters per degree plus one global
// reservation per (tile, degree). sv[r] = vertex of rank r.
constexpr int kRankTile = 1024;

__global__ __launch_bounds__(256) void k_co_rank(const int32_t *deg, int64_t n, int64_t dmax,
                                                 const int64_t *E, int32_t *cursor, int32_t *sv) {
  __shared__ int32_t lcnt[kHistBins];
  constexpr int kPer = kRankTile / 256;
  const int bins = (int)min((int64_t)kHistBins, dmax + 1);
  for (int64_t t0 = (int64_t)blockIdx.x * kRankTile; t0 < n; t0 += (int64_t)gridDim.x * kRankTile) {
    __syncthreads();
    for (int i = threadIdx.x; i < bins; i += blockDim.x) lcnt[i] = 0;
    __syncthreads();
    int32_t lr[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int64_t v = t0 + k * 256 + threadIdx.x;
      const int32_t d = v < n ? deg[v] : 0;
      lr[k] = -1;
      if (d > 0) lr[k] = d < kHistBins ? atomicAdd(&lcnt[d], 1) : atomicAdd(&cursor[d], 1);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < bins; i += blockDim.x)
      if (lcnt[i]) lcnt[i] = atomicAdd(&cursor[i], lcnt[i]);  // the tile's base within degree i
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int64_t v = t0 + k * 256 + threadIdx.x;
      if (v >= n || lr[k] < 0) continue;
      const int32_t d = deg[v];
      const int64_t r = (n - E[d + 1]) + (d < kHistBins ? lcnt[d] + lr[k] : lr[k]);
      sv[r] = (int32_t)v;
    }
  }
}

// CO[mu] is the prefix of ranks [0, |CO[mu]|) (ranks are degree-descending),
// and vertex v's entry in CO[mu] is no_sim[off[v] + mu - 2]. So the core order
// is a transpose of the neighbour-order rows taken in rank order: a tile of
// kFillRanks consecutive ranks x kFillMu consecutive mu is read row-contiguously
// into LDS and written segment-contiguously.
constexpr int kFillRanks = 64;
constexpr int kFillMu = 32;

__global__ void k_co_tiles(const int32_t *sv, const int32_t *deg, int64_t nz, int32_t *tiles_of) {
  const int64_t nt = (nz + kFillRanks - 1) / kFillRanks;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < nt;
       t += (int64_t)gridDim.x * blockDim.x)
    tiles_of[t] = (deg[sv[t * kFillRanks]] + kFillMu - 1) / kFillMu;  // first rank has the top degree
}

__global__ __launch_bounds__(256) void k_co_fill(const int32_t *sv, const int32_t *deg,
                                                 const int64_t *off, const double *no_sim,
                                                 const int64_t *co_off, int64_t nz,
                                                 const int64_t *tile_first, int64_t nrt,
                                                 double *co_key, int32_t *co_id) {
  __shared__ double tile[kFillMu][kFillRanks + 1];
  __shared__ int32_t vs[kFillRanks], vd[kFillRanks];
  __shared__ int64_t vo[kFillRanks];
  __shared__ int64_t s_t, s_k;
  const int64_t total = tile_first[nrt];
  for (int64_t b = blockIdx.x; b < total; b += gridDim.x) {
    __syncthreads();
    if (threadIdx.x == 0) {
      int64_t lo = 0, hi = nrt;  // last t with tile_first[t] <= b
      while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        if (tile_first[mid] <= b) lo = mid;
        else hi = mid;
      }
      s_t = lo;
      s_k = b - tile_first[lo];
    }
    __syncthreads();
    const int64_t r0 = s_t * kFillRanks;
    const int32_t j0 = (int32_t)(s_k * kFillMu);
    if (threadIdx.x < kFillRanks) {
      const int64_t r = r0 + threadIdx.x;
      int32_t v = 0, d = 0;
      int64_t o = 0;
      if (r < nz) {
        v = sv[r];
        d = deg[v];
        o = off[v];
      }
      vs[threadIdx.x] = v;
      vd[threadIdx.x] = d;
      vo[threadIdx.x] = o;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < kFillRanks * kFillMu; e += blockDim.x) {
      const int i = e / kFillMu, j = e % kFillMu;
      if (j0 + j < vd[i]) tile[j][i] = no_sim[vo[i] + j0 + j];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < kFillRanks * kFillMu; e += blockDim.x) {
      const int j = e / kFillRanks, i = e % kFillRanks;
      if (j0 + j < vd[i]) {
        const int64_t pos = co_off[j0 + j + 2] + r0 + i;
        co_key[pos] = tile[j][i];
        co_id[pos] = vs[i];
      }
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
  if (cfg.small_max < 1 || cfg.small_max > 4096 || cfg.spc < 1 || cfg.spc > 1024 || cfg.wbits < 10 ||
      cfg.wbits > 24)
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
  auto bail = [&](scan_status st) {
    for (auto &e : ix->ev)
      if (e) (void)hipEventDestroy(e);
    index_release(ix);
    delete ix;
    return st;
  };
#define BTRY(expr)                        \
  do {                                    \
    scan_status st_ = (expr);             \
    if (st_ != SCAN_OK) return bail(st_); \
  } while (0)
#define BHIP(expr)                                                                    \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess)                                                             \
      return bail(fail(SCAN_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_))); \
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

  // a2-a4: ownership plan, intersection and similarity.
  {
    IntersectStats ist;
    if (prof) {
      ist.ev_start = ix->ev[2];
      ist.ev_end = ix->ev[3];
    }
    BTRY(intersect_all(cfg, n, nnz, ix->off, deg, in.adj, kind, sims, ix->counts, ix->device, s,
                       &ist));
    ix->owners = ist.owners_small;
    ix->intersect_launches = (ist.owners_small > 0) + (ist.chunks_big > 0);
  }

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
  k_degree_hist<<<grid_for(n, 256, 1024), 256, 0, s>>>(deg, n, dmax, hist);
  BTRY(exclusive_scan(hist, E, dmax + 1, scan_ws, s));
  k_co_sizes<<<grid_for(dmax, 256), 256, 0, s>>>(E, n, dmax, sizes);
  BTRY(exclusive_scan64(sizes, co_scan, dmax, scan_ws, s));
  k_co_finish_off<<<grid_for(dmax + 3, 256), 256, 0, s>>>(co_scan, dmax, ix->co_off);
  int32_t *sv, *tiles_of;
  int64_t *tile_first;
  const int64_t nrt_max = (n + kFillRanks - 1) / kFillRanks;
  BTRY(tmp.alloc(&sv, n));
  BTRY(tmp.alloc(&tiles_of, nrt_max));
  BTRY(tmp.alloc(&tile_first, nrt_max + 1));
  k_co_rank<<<grid_for(n, kRankTile, 4096), 256, 0, s>>>(deg, n, dmax, E, cursor, sv);
  // nz = |CO[2]| = number of non-isolated vertices = co_off[3] - co_off[2]
  int64_t co23[2];
  BHIP(hipMemcpyAsync(co23, ix->co_off + 2, 16, hipMemcpyDeviceToHost, s));
  BHIP(hipStreamSynchronize(s));
  const int64_t nz = co23[1] - co23[0];
  const int64_t nrt = (nz + kFillRanks - 1) / kFillRanks;
  k_co_tiles<<<grid_for(nrt, 256), 256, 0, s>>>(sv, deg, nz, tiles_of);
  BTRY(exclusive_scan(tiles_of, tile_first, nrt, scan_ws, s));
  k_co_fill<<<grid_for(nnz / 512 + 1, 1, 1 << 16), 256, 0, s>>>(sv, deg, ix->off, ix->no_sim, ix->co_off, nz,
                                                                tile_first, nrt, co_key, co_id);
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
