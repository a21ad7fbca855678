// Index construction (Section 4.1): per-edge similarity (Algorithm 1), the
// neighbour order and the core order (Algorithm 2), for one graph or for a
// batch of graphs built together.
//
// A batch is processed as the disjoint union of its graphs (vertex ids and
// edge slots shifted by per-graph bases): degrees, the intersection and the
// neighbour-order sort run once over all graphs' edges, since no edge crosses
// two graphs. The core order is built per (graph, mu) segment. Every graph's
// index is a view into the shared buffers, with vertex ids local to the graph.
// A single graph is the batch of one (no shifting).
//
// Core order: CO[mu] of a graph is the prefix of its vertices ranked by
// degree, descending (ranks [0, |CO[mu]|)); vertex v's entry in CO[mu] is
// NO_SIM[off[v] + mu - 2]. So the core order is a transpose of the neighbour
// order taken in rank order, written tile by tile through LDS, then each
// segment is sorted by (threshold desc, id asc).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "index.h"

namespace scan {

SharedArena::~SharedArena() {
  if (!pinned.empty()) {  // staging copies may still be in flight
    if (done) (void)hipEventSynchronize(done);
    else (void)hipStreamSynchronize(stream);
    for (auto &b : pinned) pinned_give(b);
  }
  if (done) (void)hipEventDestroy(done);
  for (auto &a : allocs) dev_free(a.p, a.bytes, stream);
}

BuildProfileEvents::~BuildProfileEvents() {
  for (auto &e : ev)
    if (e) {
      (void)hipEventSynchronize(e);
      (void)hipEventDestroy(e);
    }
}

// Per-graph description of a batch member (device copy).
struct GraphDesc {
  const void *off;     // caller's offsets (device)
  const int32_t *adj;  // caller's adjacency (device)
  int64_t n, nnz;
  int64_t vbase, ebase;  // first vertex / slot in the union
  int64_t item_base;     // first work item of k_union_prepare
  int32_t off_bits;
  int32_t pad;
};

__device__ __forceinline__ int find_graph(const int64_t *base, int G, int64_t x) {
  int lo = 0, hi = G;  // last g with base[g] <= x
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (base[mid] <= x) lo = mid;
    else hi = mid;
  }
  return lo;
}

// ---------------------------------------------------------------------------
// a1: union CSR, degrees, per-graph maximum degree. Work items of graph g:
// its n+1 offsets, then (when the adjacency is copied) its nnz ids.

constexpr int kPrepThreads = 256;

// Work tiles of k_union_prepare: items [i0, i1) of graph g (its n+1 offsets,
// then, when the adjacency is copied, its nnz ids), planned on the host so
// that each tile lies in one graph.
struct PrepTile {
  int32_t g;
  int32_t pad;
  int64_t i0, i1;
};
constexpr int64_t kPrepTile = 4096;

__global__ __launch_bounds__(kPrepThreads) void k_union_prepare(const GraphDesc *gd, const PrepTile *tiles,
                                                                int64_t ntiles, int copy_adj, int64_t *off_u,
                                                                int32_t *deg_u, int32_t *adj_u, unsigned *dmax_g) {
  __shared__ unsigned wmax[kPrepThreads / kWave];
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const PrepTile tl = tiles[t];
    const GraphDesc d = gd[tl.g];
    unsigned ml = 0;  // the tile's maximum degree
    for (int64_t j = tl.i0 + threadIdx.x; j < tl.i1; j += blockDim.x) {
      if (j <= d.n) {
        int64_t o, o1 = 0;
        if (d.off_bits == 32) {
          o = ((const int32_t *)d.off)[j];
          if (j < d.n) o1 = ((const int32_t *)d.off)[j + 1];
        } else {
          o = ((const int64_t *)d.off)[j];
          if (j < d.n) o1 = ((const int64_t *)d.off)[j + 1];
        }
        off_u[d.vbase + j] = d.ebase + o;
        if (j < d.n) {
          const int64_t deg = o1 - o;
          deg_u[d.vbase + j] = (int32_t)deg;
          ml = max(ml, (unsigned)(deg > 0 ? deg : 0));
        }
      } else if (copy_adj) {
        const int64_t s = j - (d.n + 1);
        adj_u[d.ebase + s] = (int32_t)(d.vbase + d.adj[s]);
      }
    }
#pragma unroll
    for (int k = kWave / 2; k > 0; k >>= 1) ml = max(ml, (unsigned)__shfl_xor((int)ml, k, kWave));
    __syncthreads();  // wmax is reused across tiles
    if (lane == 0) wmax[wave] = ml;
    __syncthreads();
    if (threadIdx.x == 0) {
      unsigned m = 0;
      for (int w = 0; w < kPrepThreads / kWave; ++w) m = max(m, wmax[w]);
      if (m) atomicMax(&dmax_g[tl.g], m);
    }
  }
}

// Vertex ids in [lo, hi) slots of the union made local: id - vbase(g).
// A thread takes kLocalizePer consecutive slots: one search for the first
// slot's graph, then a step to the next graph where a slot passes its end.
constexpr int kLocalizePer = 16;

__global__ void k_localize_ids(int32_t *ids, const int64_t *ebase, const int64_t *vbase, int G,
                               int64_t nnz) {
  for (int64_t s0 = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) * kLocalizePer; s0 < nnz;
       s0 += (int64_t)gridDim.x * blockDim.x * kLocalizePer) {
    int g = find_graph(ebase, G, s0);
    int64_t end = ebase[g + 1];
    int32_t vb = (int32_t)vbase[g];
    const int64_t s1 = s0 + kLocalizePer < nnz ? s0 + kLocalizePer : nnz;
    for (int64_t s = s0; s < s1; ++s) {
      while (s >= end) {  // graphs without edges are stepped over
        ++g;
        end = ebase[g + 1];
        vb = (int32_t)vbase[g];
      }
      ids[s] -= vb;
    }
  }
}

// Per-graph local offsets: graph g's n+1 entries start at vbase(g) + g.
__global__ void k_local_offsets(const int64_t *off_u, const int64_t *obase, const int64_t *vbase,
                                const int64_t *ebase, int G, int64_t total, int64_t *off_local) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int g = find_graph(obase, G, i);
    off_local[i] = off_u[vbase[g] + (i - obase[g])] - ebase[g];
  }
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
// a6: core order.

constexpr int kHistBins = 2048;  // degrees below this are counted in LDS first
constexpr int kRankTile = 1024;  // vertices per rank tile (all in one graph)
constexpr int kFillRanks = 64;   // ranks per transpose tile
constexpr int kFillMu = 32;      // mu values per transpose tile

struct VTile {
  int32_t g;
  int32_t pad;
  int64_t v0, v1;  // union vertex ids [v0, v1), all in graph g
};

struct RTile {
  int32_t g;
  int32_t r0;  // first rank (local to graph g)
};
// A rank's vertex (union id), its degree and its row offset, written once by
// the rank pass so that the transpose reads one record per rank.
struct alignas(16) RankInfo {
  int32_t v, d;
  int64_t o;
};

// Per-graph degree histograms hist_all[hbase[g] + d].
__global__ __launch_bounds__(256) void k_graph_hist(const VTile *tiles, int64_t ntiles,
                                                    const int32_t *deg, const int64_t *hbase,
                                                    const unsigned *dmax_g, int32_t *hist_all) {
  __shared__ int32_t lh[kHistBins];
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const VTile tl = tiles[t];
    int32_t *hist = hist_all + hbase[tl.g];
    const int bins = (int)min((int64_t)kHistBins, (int64_t)dmax_g[tl.g] + 1);
    __syncthreads();
    for (int i = threadIdx.x; i < bins; i += blockDim.x) lh[i] = 0;
    __syncthreads();
    for (int64_t v = tl.v0 + threadIdx.x; v < tl.v1; v += blockDim.x) {
      const int32_t d = deg[v];
      if (d < kHistBins) atomicAdd(&lh[d], 1);
      else atomicAdd(&hist[d], 1);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < bins; i += blockDim.x)
      if (lh[i]) atomicAdd(&hist[i], lh[i]);
  }
}

// Core-order sizes from the degree histograms (P = exclusive scan of all
// graphs' histograms, so graph g's prefix is P[hbase[g] + d] - P[hbase[g]]):
//   E[d] = number of vertices of degree < d           (d = 0..dmax+1)
//   X[mu - 2] = |CO[mu]| = n - E[mu - 1]              (mu = 2..dmax+1)
// Flat over all graphs' entries.
__global__ void k_co_counts(const int64_t *P, const int64_t *hbase, const int64_t *Ebase,
                            const int64_t *segbase, const int64_t *n_g, int G, int64_t *E_all,
                            int64_t *X) {
  const int64_t total = Ebase[G];
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int g = find_graph(Ebase, G, i);
    const int64_t d = i - Ebase[g], dm = Ebase[g + 1] - Ebase[g] - 2;
    const int64_t e = P[hbase[g] + d] - P[hbase[g]];
    E_all[i] = e;
    if (d >= 1 && d <= dm) X[segbase[g] + d - 1] = n_g[g] - e;
  }
}

// Core-order offsets co[mu] = sum of |CO[m]| for 2 <= m < mu (XS = exclusive
// scan of X over all graphs), the union start of each segment for the sort
// (the end of the last one is the total), and the non-isolated counts.
__global__ void k_co_offsets(const int64_t *XS, const int64_t *cobase, const int64_t *segbase,
                             const int64_t *ebase, const int64_t *hbase, const int32_t *hist_all,
                             const int64_t *n_g, int G, int64_t *co_all, int64_t *seg_all,
                             int64_t *nz_g) {
  const int64_t total = cobase[G];
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int g = find_graph(cobase, G, i);
    const int64_t mu = i - cobase[g], dm = cobase[g + 1] - cobase[g] - 3;
    const int64_t co = mu < 2 ? 0 : XS[segbase[g] + mu - 2] - XS[segbase[g]];
    co_all[i] = co;
    if (mu >= 2 && mu <= dm + 1) seg_all[segbase[g] + mu - 2] = ebase[g] + co;
    if (mu == 0) nz_g[g] = dm > 0 ? n_g[g] - hist_all[hbase[g]] : 0;
    if (i == 0) seg_all[segbase[G]] = ebase[G];
  }
}

// Rank of every non-isolated vertex of its graph, degree-descending (ties in
// any order: each CO segment is sorted afterwards): r = #{deg > d} + the
// vertex's position among those of degree d, from LDS counters per tile plus
// one global reservation per (tile, degree). sv[svbase[g] + r] = union id.
__global__ __launch_bounds__(256) void k_co_rank(const VTile *tiles, int64_t ntiles,
                                                 const int32_t *deg, const int64_t *hbase,
                                                 const int64_t *Ebase, const unsigned *dmax_g,
                                                 const int64_t *E_all, int32_t *cursor_all,
                                                 const int64_t *n_g, const int64_t *svbase,
                                                 const int64_t *off, RankInfo *sv_all) {
  __shared__ int32_t lcnt[kHistBins];
  constexpr int kPer = kRankTile / 256;
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const VTile tl = tiles[t];
    const int g = tl.g;
    const int64_t *E = E_all + Ebase[g];
    int32_t *cursor = cursor_all + hbase[g];
    const int64_t n = n_g[g];
    const int bins = (int)min((int64_t)kHistBins, (int64_t)dmax_g[g] + 1);
    __syncthreads();
    for (int i = threadIdx.x; i < bins; i += blockDim.x) lcnt[i] = 0;
    __syncthreads();
    int32_t lr[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int64_t v = tl.v0 + k * 256 + threadIdx.x;
      const int32_t d = v < tl.v1 ? deg[v] : 0;
      lr[k] = -1;
      if (d > 0) lr[k] = d < kHistBins ? atomicAdd(&lcnt[d], 1) : atomicAdd(&cursor[d], 1);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < bins; i += blockDim.x)
      if (lcnt[i]) lcnt[i] = atomicAdd(&cursor[i], lcnt[i]);  // the tile's base within degree i
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int64_t v = tl.v0 + k * 256 + threadIdx.x;
      if (v >= tl.v1 || lr[k] < 0) continue;
      const int32_t d = deg[v];
      const int64_t r = (n - E[d + 1]) + (d < kHistBins ? lcnt[d] + lr[k] : lr[k]);
      sv_all[svbase[g] + r] = RankInfo{(int32_t)v, d, off[v]};
    }
  }
}

// Number of mu tiles of each rank tile (its first rank has the top degree).
// Rank tiles are planned from n (known on the host); those past the graph's
// non-isolated count get no mu tiles.
__global__ void k_co_tiles(const RTile *rt, int64_t nrt, const RankInfo *sv_all,
                           const int64_t *svbase, const int64_t *nz_g, int32_t *tiles_of) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < nrt;
       t += (int64_t)gridDim.x * blockDim.x)
    tiles_of[t] = rt[t].r0 < nz_g[rt[t].g]
                      ? (sv_all[svbase[rt[t].g] + rt[t].r0].d + kFillMu - 1) / kFillMu
                      : 0;
}

// One workgroup per (rank tile, mu tile): kFillRanks consecutive ranks x
// kFillMu consecutive mu, read row-contiguously from NO_SIM into LDS and
// written segment-contiguously into the unsorted core order. With one graph,
// rank tile t covers ranks [t kFillRanks, (t + 1) kFillRanks), and the last
// non-empty rank tiles (low degrees) have one mu tile each, so a block first
// tries the tile that assumption gives (one read confirms it) before
// searching.
__global__ __launch_bounds__(256) void k_co_fill(const RTile *rt, int64_t nrt, int32_t one_graph,
                                                 const int64_t *tile_first, const RankInfo *sv_all,
                                                 const int64_t *svbase, const int64_t *nz_g,
                                                 const double *no_sim, const int64_t *co_all,
                                                 const int64_t *cobase, const int64_t *ebase,
                                                 const int64_t *vbase,
                                                 double *co_key, int32_t *co_id) {
  __shared__ double tile[kFillMu][kFillRanks + 1];
  __shared__ int32_t vs[kFillRanks], vd[kFillRanks];
  __shared__ int64_t vo[kFillRanks];
  __shared__ int64_t s_t, s_k;
  const int64_t total = tile_first[nrt];
  const int64_t guess_end = one_graph ? (nz_g[0] + kFillRanks - 1) / kFillRanks : 0;
  for (int64_t b = blockIdx.x; b < total; b += gridDim.x) {
    __syncthreads();
    if (threadIdx.x < kWave) {
      const int lane = threadIdx.x;
      const int64_t guess = guess_end - (total - b);
      if (one_graph && guess >= 0 && guess < nrt && tile_first[guess] == b) {
        if (lane == 0) {
          s_t = guess;
          s_k = 0;
        }
      } else {
        // the last rank tile with tile_first <= b (tile_first[0] = 0): a
        // 64-way search by the first wavefront, every lane sampling one tile
        int64_t lo = 0, cnt = nrt;
        while (cnt > 1) {
          const int64_t step = (cnt + kWave - 1) / kWave;
          const int64_t q = lo + lane * step;
          const int c = __popcll(__ballot(q < lo + cnt && tile_first[q] <= b));  // >= 1: lane 0
          const int64_t nlo = lo + (c - 1) * step;
          cnt = min(step, lo + cnt - nlo);
          lo = nlo;
        }
        if (lane == 0) {
          s_t = lo;
          s_k = b - tile_first[lo];
        }
      }
    }
    __syncthreads();
    const int64_t t = s_t;
    const RTile r = one_graph ? RTile{0, (int32_t)(t * kFillRanks)} : rt[t];
    const int64_t r0 = r.r0;
    const int32_t j0 = (int32_t)(s_k * kFillMu);
    const int64_t *co = co_all + cobase[r.g];  // relative offsets of graph r.g
    const int64_t eb = ebase[r.g];
    const int32_t vb = (int32_t)vbase[r.g];
    if (threadIdx.x < kFillRanks) {
      const int64_t rr = r0 + threadIdx.x;
      RankInfo ri{0, 0, 0};
      if (rr < nz_g[r.g]) ri = sv_all[svbase[r.g] + rr];
      vs[threadIdx.x] = ri.v - vb;
      vd[threadIdx.x] = ri.d;
      vo[threadIdx.x] = ri.o;
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
        const int64_t pos = eb + co[j0 + j + 2] + r0 + i;
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

void index_release(scan_index *ix) {
  ix->arena.reset();
  ix->prof.reset();
}

namespace {

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

// A device allocation owned by the shared arena of the batch.
template <class T>
scan_status arena_alloc(SharedArena &a, T **p, int64_t count) {
  size_t bytes = (size_t)(count > 0 ? count : 1) * sizeof(T);
  void *q = dev_alloc(bytes, a.stream);
  if (!q) return fail(SCAN_ENOMEM, "device allocation of %zu bytes failed", bytes);
  a.allocs.push_back({q, bytes});
  a.bytes += (int64_t)bytes;
  *p = (T *)q;
  return SCAN_OK;
}

// Copies bytes from host memory to dst through a pinned block that the arena
// holds until the build's end has passed, so the call does not wait for the
// copy and src may go at once.
scan_status upload_pinned(SharedArena &a, void *dst, const void *src, size_t bytes, hipStream_t s) {
  if (!bytes) return SCAN_OK;
  const PinnedBlock b = pinned_take(bytes);
  if (!b.p) return fail(SCAN_ENOMEM, "pinned host allocation of %zu bytes failed", bytes);
  a.pinned.push_back(b);
  std::memcpy(b.p, src, bytes);
  SCAN_HIP_TRY(hipMemcpyAsync(dst, b.p, bytes, hipMemcpyHostToDevice, s));
  return SCAN_OK;
}

template <class T>
scan_status to_device(SharedArena &a, DevArena &tmp, T **dst, const std::vector<T> &src, hipStream_t s) {
  SCAN_TRY(tmp.alloc(dst, (int64_t)src.size()));
  return upload_pinned(a, *dst, src.data(), src.size() * sizeof(T), s);
}

// Host tables gathered into one buffer (each entry 16-byte aligned) and sent
// to the device with one copy.
class HostPack {
 public:
  template <class T>
  size_t add(const std::vector<T> &v) {
    const size_t at = (buf_.size() + 15) & ~(size_t)15;
    buf_.resize(at + v.size() * sizeof(T));
    if (!v.empty()) std::memcpy(buf_.data() + at, v.data(), v.size() * sizeof(T));
    return at;
  }
  scan_status upload(SharedArena &a, DevArena &tmp, hipStream_t s, unsigned char **dev) {
    SCAN_TRY(tmp.alloc(dev, (int64_t)std::max<size_t>(buf_.size(), 16)));
    return upload_pinned(a, *dev, buf_.data(), buf_.size(), s);
  }
  template <class T>
  static const T *at(const unsigned char *dev, size_t off) {
    return (const T *)(dev + off);
  }

 private:
  std::vector<unsigned char> buf_;
};

}  // namespace

scan_status build_index_batch(const scan_csr *gs, int32_t G, int32_t kind, uint32_t flags,
                              hipStream_t s, const IntersectConfig &cfg, scan_index **outs,
                              const double *weights, const LshSpec *lsh) {
  if (G < 0 || (G > 0 && (!gs || !outs))) return fail(SCAN_EINVAL, "bad batch arguments");
  for (int32_t g = 0; g < G; ++g) {
    outs[g] = nullptr;
    SCAN_TRY(check_csr(&gs[g]));
  }
  const bool weighted = kind == SCAN_SIM_WEIGHTED_COSINE;
  if (kind != SCAN_SIM_COSINE && kind != SCAN_SIM_JACCARD && !weighted)
    return fail(SCAN_EINVAL, "unknown similarity kind %d", kind);
  if (weighted && (G != 1 || (!weights && G > 0 && gs[0].nnz > 0)))
    return fail(SCAN_EINVAL, "the weighted cosine takes one graph and its edge weights (scan_build_index_weighted)");
  if (!weighted && weights) return fail(SCAN_EINVAL, "edge weights given for an unweighted similarity");
  if (weighted && (flags & SCAN_KEEP_COUNTS)) return fail(SCAN_EINVAL, "the weighted cosine has no intersection counts");
  if (lsh) {
    if (G != 1) return fail(SCAN_EINVAL, "approximate builds take one graph");
    if (lsh->samples < 64 || lsh->samples > 4096 || lsh->samples % 64)
      return fail(SCAN_EINVAL, "LSH samples must be a multiple of 64 in [64, 4096]");
    const bool need_gauss = kind != SCAN_SIM_JACCARD;
    if ((need_gauss && !lsh->gauss) || (!need_gauss && !lsh->perm))
      return fail(SCAN_EINVAL, "SimHash needs the Gaussian draws, MinHash the permutation");
    if (flags & SCAN_KEEP_COUNTS) return fail(SCAN_EINVAL, "approximate similarities have no intersection counts");
  }
  if (flags & ~(uint32_t)(SCAN_VALIDATE | SCAN_KEEP_SIMS | SCAN_KEEP_COUNTS | SCAN_PROFILE)) return fail(SCAN_EINVAL, "unknown build flags 0x%x", flags);
  if (cfg.small_max < 1 || cfg.small_max > 4096 || cfg.spc < 1 || cfg.spc > 1024 || cfg.wbits < 10 || cfg.wbits > 24)
    return fail(SCAN_EINVAL, "bad intersection config");
  if (G == 0) return SCAN_OK;

  std::vector<int64_t> vbase(G + 1, 0), ebase(G + 1, 0), item_base(G + 1, 0);
  const bool copy_adj = G > 1;
  for (int32_t g = 0; g < G; ++g) {
    vbase[g + 1] = vbase[g] + gs[g].n;
    ebase[g + 1] = ebase[g] + gs[g].nnz;
    item_base[g + 1] = item_base[g] + gs[g].n + 1 + (copy_adj ? gs[g].nnz : 0);
  }
  const int64_t N = vbase[G], NNZ = ebase[G];
  if (N > 0x7fffffffLL) return fail(SCAN_EINVAL, "batch has more than 2^31-1 vertices in total");
  int device = 0;
  (void)hipGetDevice(&device);

  auto arena = std::make_shared<SharedArena>();
  arena->stream = s;
  std::shared_ptr<BuildProfileEvents> prof;
  if (flags & SCAN_PROFILE) {
    prof = std::make_shared<BuildProfileEvents>();
    for (auto &e : prof->ev) SCAN_HIP_TRY(hipEventCreate(&e));
  }
  auto mark = [&](int k) {
    if (prof) (void)hipEventRecord(prof->ev[k], s);
  };
  DevArena tmp(s);
  mark(0);

  // Stage host-resident graphs.
  std::vector<GraphDesc> hd(G);
  for (int32_t g = 0; g < G; ++g) {
    const scan_csr &c = gs[g];
    const int osz = c.offset_bits / 8;
    hd[g] = GraphDesc{c.offsets, c.adj, c.n, c.nnz, vbase[g], ebase[g], item_base[g], c.offset_bits, 0};
    if (!c.on_device && c.n > 0) {
      unsigned char *doff;
      int32_t *dadj;
      SCAN_TRY(tmp.alloc(&doff, (c.n + 1) * osz));
      SCAN_TRY(tmp.alloc(&dadj, c.nnz));
      SCAN_HIP_TRY(hipMemcpyAsync(doff, c.offsets, (size_t)(c.n + 1) * osz, hipMemcpyHostToDevice, s));
      if (c.nnz) SCAN_HIP_TRY(hipMemcpyAsync(dadj, c.adj, (size_t)c.nnz * 4, hipMemcpyHostToDevice, s));
      hd[g].off = doff;
      hd[g].adj = dadj;
    } else if (c.n == 0) {
      hd[g].off = nullptr;
    }
  }

  // a1: union offsets (and adjacency), degrees, per-graph max degree.
  int64_t *off_u;
  int32_t *deg, *adj_u;
  unsigned *d_dmax;
  SCAN_TRY(arena_alloc(*arena, &off_u, N + 1));
  SCAN_TRY(tmp.alloc(&deg, N));
  SCAN_TRY(tmp.alloc(&d_dmax, G));
  if (copy_adj) SCAN_TRY(tmp.alloc(&adj_u, NNZ));
  else adj_u = const_cast<int32_t *>(hd[0].adj);
  GraphDesc *d_gd;
  PrepTile *d_ptiles;
  std::vector<PrepTile> ptiles;
  for (int32_t g = 0; g < G; ++g) {
    const int64_t items = item_base[g + 1] - item_base[g];
    for (int64_t i0 = 0; i0 < items; i0 += kPrepTile)
      ptiles.push_back(PrepTile{g, 0, i0, std::min(items, i0 + kPrepTile)});
  }
  {
    // graphs without vertices contribute only their (zero) end offset
    std::vector<GraphDesc> fix = hd;
    bool any_empty = false;
    for (int32_t g = 0; g < G; ++g)
      if (gs[g].n == 0) any_empty = true;
    if (any_empty) {
      int64_t *zero_off;
      SCAN_TRY(tmp.alloc(&zero_off, 1));
      SCAN_HIP_TRY(hipMemsetAsync(zero_off, 0, 8, s));
      for (int32_t g = 0; g < G; ++g)
        if (gs[g].n == 0) {
          fix[g].off = zero_off;
          fix[g].off_bits = 64;
        }
    }
    SCAN_TRY(to_device(*arena, tmp, &d_gd, fix, s));
  }
  SCAN_TRY(to_device(*arena, tmp, &d_ptiles, ptiles, s));
  SCAN_HIP_TRY(hipMemsetAsync(d_dmax, 0, (size_t)G * 4, s));
  SCAN_HIP_TRY(hipMemsetAsync(off_u, 0, 8, s));
  {
    const int64_t total = item_base[G];
    if (total > 0)
      k_union_prepare<<<grid_for((int64_t)ptiles.size(), 1, 4096), kPrepThreads, 0, s>>>(
          d_gd, d_ptiles, (int64_t)ptiles.size(), copy_adj ? 1 : 0, off_u, deg, adj_u, d_dmax);
  }
  if (flags & SCAN_VALIDATE) {
    int32_t *d_err;
    SCAN_TRY(tmp.alloc(&d_err, 2 * (int64_t)G));
    std::vector<int32_t> init(2 * G);
    for (int32_t g = 0; g < G; ++g) {
      init[2 * g] = 0;
      init[2 * g + 1] = 0x7fffffff;
    }
    SCAN_HIP_TRY(hipMemcpyAsync(d_err, init.data(), init.size() * 4, hipMemcpyHostToDevice, s));
    for (int32_t g = 0; g < G; ++g) {
      if (gs[g].n == 0) continue;
      if (gs[g].offset_bits == 32)
        k_validate<int32_t><<<grid_for(gs[g].n * kWave, 256), 256, 0, s>>>((const int32_t *)hd[g].off, hd[g].adj, gs[g].n, gs[g].nnz, d_err + 2 * g);
      else
        k_validate<int64_t><<<grid_for(gs[g].n * kWave, 256), 256, 0, s>>>((const int64_t *)hd[g].off, hd[g].adj, gs[g].n, gs[g].nnz, d_err + 2 * g);
    }
    std::vector<int32_t> herr(2 * G);
    SCAN_HIP_TRY(hipMemcpyAsync(herr.data(), d_err, herr.size() * 4, hipMemcpyDeviceToHost, s));
    SCAN_HIP_TRY(hipStreamSynchronize(s));
    for (int32_t g = 0; g < G; ++g)
      if (herr[2 * g])
        return fail(SCAN_EGRAPH, "graph %d is not a simple undirected CSR with ascending rows (first bad row %d)", g, herr[2 * g + 1]);
  }
  // The neighbour-order segments are the CSR rows: classified by length now,
  // on a helper stream, so their sizes are on the host when the sort starts.
  hipStream_t ns = NNZ > 0 ? helper_stream(2) : nullptr;
  if (ns && stream_wait(ns, s) != SCAN_OK) ns = nullptr;
  JoinOnExit join_ns{s, ns};
  SortClasses no_cls;
  if (NNZ > 0) SCAN_TRY(sort_classify(off_u, N, tmp, ns ? ns : s, no_cls));
  // a2: the ownership plan needs only the degrees; its counts come back with
  // the maximum degrees below.
  IntersectPlan plan;
  if (NNZ > 0 && !weighted) SCAN_TRY(intersect_plan(cfg, N, NNZ, off_u, deg, adj_u, device, tmp, s, plan));
  // The small-owner kernels' helper streams wait for the plan now, off the
  // path between the read-back and the first intersection launch.
  JoinOnExit join_h0{s, nullptr}, join_h1{s, nullptr};
  if (NNZ > 0 && !weighted) {
    for (int k = 0; k < 2; ++k) {
      hipStream_t hs = helper_stream(k);
      if (hs && stream_wait(hs, s) == SCAN_OK) plan.helper[k] = hs;
    }
    join_h0.helper = plan.helper[0];
    join_h1.helper = plan.helper[1];
  }
  const double *w_dev = weights;  // edge weights on the device (weighted cosine)
  if (weighted && NNZ > 0) {
    if (!gs[0].on_device) {
      double *dw;
      SCAN_TRY(tmp.alloc(&dw, NNZ));
      SCAN_HIP_TRY(hipMemcpyAsync(dw, weights, (size_t)NNZ * 8, hipMemcpyHostToDevice, s));
      w_dev = dw;
    }
    if (flags & SCAN_VALIDATE) SCAN_TRY(check_weights(w_dev, NNZ, tmp, s));
  }
  LshSpec lsh_dev;  // the draws on the device
  if (lsh && NNZ > 0) {
    lsh_dev.samples = lsh->samples;
    lsh_dev.gauss = lsh->gauss;
    lsh_dev.perm = lsh->perm;
    if (!gs[0].on_device) {
      if (kind == SCAN_SIM_JACCARD) {
        uint32_t *dp;
        SCAN_TRY(tmp.alloc(&dp, N));
        SCAN_HIP_TRY(hipMemcpyAsync(dp, lsh->perm, (size_t)N * 4, hipMemcpyHostToDevice, s));
        lsh_dev.perm = dp;
      } else {
        double *dg;
        SCAN_TRY(tmp.alloc(&dg, N * (int64_t)lsh->samples));
        SCAN_HIP_TRY(hipMemcpyAsync(dg, lsh->gauss, (size_t)N * lsh->samples * 8, hipMemcpyHostToDevice, s));
        lsh_dev.gauss = dg;
      }
    }
  }
  // Index arrays (their sizes do not depend on the degrees): allocated while
  // the device runs the kernels above, as one block carved into 256-byte
  // aligned arrays (each allocation may cross into the caller's allocator).
  int32_t *no_ids, *co_ids, *counts = nullptr;
  double *no_sim, *co_thr, *sims = nullptr;
  {
    size_t bytes = 0;
    auto take = [&](size_t b) {
      const size_t at = bytes;
      bytes += (b + 255) & ~(size_t)255;
      return at;
    };
    const size_t nz = (size_t)std::max<int64_t>(NNZ, 1);
    const size_t o_no_ids = take(nz * 4), o_no_sim = take(nz * 8), o_co_ids = take(nz * 4), o_co_thr = take(nz * 8);
    const size_t o_sims = (flags & SCAN_KEEP_SIMS) ? take(nz * 8) : 0;
    const size_t o_counts = (flags & SCAN_KEEP_COUNTS) ? take(nz * 4) : 0;
    unsigned char *block;
    SCAN_TRY(arena_alloc(*arena, &block, (int64_t)bytes));
    no_ids = (int32_t *)(block + o_no_ids);
    no_sim = (double *)(block + o_no_sim);
    co_ids = (int32_t *)(block + o_co_ids);
    co_thr = (double *)(block + o_co_thr);
    if (flags & SCAN_KEEP_SIMS) sims = (double *)(block + o_sims);
    if (flags & SCAN_KEEP_COUNTS) counts = (int32_t *)(block + o_counts);
  }
  if (!sims) SCAN_TRY(tmp.alloc(&sims, NNZ));

  // Tiles of the core-order kernels (they need no maximum degree): built
  // here, while the device runs the degree pass and the plan.
  std::vector<VTile> vt;
  std::vector<RTile> rt;
  for (int32_t g = 0; g < G; ++g) {
    for (int64_t v0 = vbase[g]; v0 < vbase[g + 1]; v0 += kRankTile)
      vt.push_back(VTile{g, 0, v0, std::min(vbase[g + 1], v0 + kRankTile)});
    for (int64_t r0 = 0; r0 < gs[g].n; r0 += kFillRanks) rt.push_back(RTile{g, (int32_t)r0});
  }
  // The one wait of the build that stalls the device: the maximum degrees
  // (with the plan counts) size everything after.
  std::vector<unsigned> hdmax(G);
  {
    const PinnedBlock hb = pinned_take((size_t)G * 4);
    if (!hb.p) return fail(SCAN_ENOMEM, "pinned host allocation failed");
    hipError_t e = hipMemcpyAsync(hb.p, d_dmax, (size_t)G * 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess) std::memcpy(hdmax.data(), hb.p, (size_t)G * 4);
    pinned_give(hb);
    SCAN_HIP_TRY(e);
  }
  SCAN_HIP_TRY(hipGetLastError());
  mark(1);

  // Host tables for the rest of the build; everything they hold is known once
  // the maximum degrees are (the core-order sizes themselves are computed on
  // the device).
  std::vector<int64_t> hbase(G + 1, 0), Ebase(G + 1, 0), cobase(G + 1, 0), segbase(G + 1, 0), ng(G),
      obase(G + 1, 0);
  for (int32_t g = 0; g < G; ++g) {
    hbase[g + 1] = hbase[g] + hdmax[g] + 1;
    Ebase[g + 1] = Ebase[g] + hdmax[g] + 2;
    cobase[g + 1] = cobase[g] + hdmax[g] + 3;
    segbase[g + 1] = segbase[g] + hdmax[g];  // segments mu = 2..dmax+1
    obase[g + 1] = obase[g] + gs[g].n + 1;
    ng[g] = gs[g].n;
  }
  HostPack pack;
  const size_t p_hbase = pack.add(hbase), p_Ebase = pack.add(Ebase), p_cobase = pack.add(cobase),
               p_segbase = pack.add(segbase), p_ng = pack.add(ng), p_obase = pack.add(obase),
               p_vbase = pack.add(vbase), p_ebase = pack.add(ebase), p_vt = pack.add(vt), p_rt = pack.add(rt);
  const int64_t *d_hbase = nullptr, *d_Ebase = nullptr, *d_cobase = nullptr, *d_segbase = nullptr,
                *d_ng = nullptr, *d_obase = nullptr, *d_vbase = nullptr, *d_ebase = nullptr;
  const VTile *d_vt = nullptr;
  const RTile *d_rt = nullptr;
  int64_t *d_corel = nullptr;  // per-graph core-order offsets (the indexes' co_off)
  // The tables go to the device in one copy on stream st, and the core-order
  // offsets are allocated: after the intersection is launched, so that
  // nothing stands between the read-back above and that launch.
  auto upload_tables = [&](hipStream_t st) -> scan_status {
    unsigned char *dpack;
    SCAN_TRY(pack.upload(*arena, tmp, st, &dpack));
    d_hbase = pack.at<int64_t>(dpack, p_hbase);
    d_Ebase = pack.at<int64_t>(dpack, p_Ebase);
    d_cobase = pack.at<int64_t>(dpack, p_cobase);
    d_segbase = pack.at<int64_t>(dpack, p_segbase);
    d_ng = pack.at<int64_t>(dpack, p_ng);
    d_obase = pack.at<int64_t>(dpack, p_obase);
    d_vbase = pack.at<int64_t>(dpack, p_vbase);
    d_ebase = pack.at<int64_t>(dpack, p_ebase);
    d_vt = pack.at<VTile>(dpack, p_vt);
    d_rt = pack.at<RTile>(dpack, p_rt);
    return arena_alloc(*arena, &d_corel, cobase[G]);
  };

  if (NNZ > 0) {
    // a6, first part: core-order sizes and offsets (from the degree
    // histograms, on the device) and the degree-rank list. These read only the
    // degrees, so they run on the helper stream that classified the rows (it
    // is ordered after the degree pass) while the intersection runs; the host
    // enqueues them once the intersection kernels are launched.
    const hipStream_t cs = ns ? ns : s;
    JoinOnExit join_cs{s, cs};
    int32_t *d_hist, *d_cursor, *d_tiles_of;
    RankInfo *d_sv;
    int64_t *d_E, *d_seg, *d_nz, *d_tile_first, *scan_ws;
    double *co_key;
    int32_t *co_id;
    SortClasses co_cls;
    const int64_t nrt = (int64_t)rt.size();
    auto co_prep = [&]() -> scan_status {  // cs is ordered after the degrees
      SCAN_TRY(upload_tables(cs));
      SCAN_TRY(tmp.alloc(&d_hist, hbase[G]));
      SCAN_TRY(tmp.alloc(&d_cursor, hbase[G]));
      SCAN_TRY(tmp.alloc(&d_E, Ebase[G]));
      SCAN_TRY(tmp.alloc(&d_seg, segbase[G] + 1));
      SCAN_TRY(tmp.alloc(&d_nz, G));
      SCAN_TRY(tmp.alloc(&d_sv, std::max<int64_t>(N, 1)));
      SCAN_TRY(tmp.alloc(&d_tiles_of, std::max<int64_t>(nrt, 1)));
      SCAN_TRY(tmp.alloc(&d_tile_first, nrt + 1));
      SCAN_TRY(tmp.alloc(&scan_ws, scan_workspace_elems(std::max<int64_t>(nrt, 1))));
      SCAN_TRY(tmp.alloc(&co_key, NNZ));
      SCAN_TRY(tmp.alloc(&co_id, NNZ));
      SCAN_HIP_TRY(hipMemsetAsync(d_hist, 0, (size_t)hbase[G] * 4, cs));
      SCAN_HIP_TRY(hipMemsetAsync(d_cursor, 0, (size_t)hbase[G] * 4, cs));
      if (!vt.empty())
        k_graph_hist<<<grid_for((int64_t)vt.size(), 1, 8192), 256, 0, cs>>>(d_vt, (int64_t)vt.size(), deg, d_hbase,
                                                                           d_dmax, d_hist);
      {
        int64_t *P, *X, *XS, *ws;
        SCAN_TRY(tmp.alloc(&P, hbase[G] + 1));
        SCAN_TRY(tmp.alloc(&X, std::max<int64_t>(segbase[G], 1)));
        SCAN_TRY(tmp.alloc(&XS, segbase[G] + 1));
        SCAN_TRY(tmp.alloc(&ws, scan_workspace_elems(std::max<int64_t>(hbase[G], segbase[G]))));
        SCAN_TRY(exclusive_scan(d_hist, P, hbase[G], ws, cs));
        k_co_counts<<<grid_for(Ebase[G], 256), 256, 0, cs>>>(P, d_hbase, d_Ebase, d_segbase, d_ng, G, d_E, X);
        SCAN_TRY(exclusive_scan64(X, XS, segbase[G], ws, cs));
        k_co_offsets<<<grid_for(cobase[G], 256), 256, 0, cs>>>(XS, d_cobase, d_segbase, d_ebase, d_hbase, d_hist, d_ng,
                                                              G, d_corel, d_seg, d_nz);
      }
      if (!vt.empty())
        k_co_rank<<<grid_for((int64_t)vt.size(), 1, 8192), 256, 0, cs>>>(d_vt, (int64_t)vt.size(), deg, d_hbase,
                                                                       d_Ebase, d_dmax, d_E, d_cursor, d_ng, d_vbase,
                                                                       off_u, d_sv);
      if (nrt > 0) {
        k_co_tiles<<<grid_for(nrt, 256), 256, 0, cs>>>(d_rt, nrt, d_sv, d_vbase, d_nz, d_tiles_of);
        SCAN_TRY(exclusive_scan(d_tiles_of, d_tile_first, nrt, scan_ws, cs));
      }
      return sort_classify(d_seg, segbase[G], tmp, cs, co_cls);  // the core-order segments
    };

    // a2-a4: ownership plan, intersection and similarity over the union.
    IntersectStats ist;
    if (prof) {
      ist.ev_small_begin = prof->ev[6];
      ist.ev_small_end = prof->ev[7];
      ist.ev_big_begin = prof->ev[8];
      ist.ev_big_end = prof->ev[9];
      ist.ev_plan_end = prof->ev[2];
      ist.host_counts = prof->plan_counts;
    }
    IntersectConfig icfg = cfg;
    if (lsh)  // the edges between two high-degree vertices are left to the approximate pass
      icfg.skip_deg = kind == SCAN_SIM_JACCARD ? 3 * lsh->samples / 2 : lsh->samples;
    if (weighted) {
      mark(2);  // no ownership plan
      if (cs != s) SCAN_TRY(stream_wait(cs, s));
      SCAN_TRY(co_prep());
      SCAN_TRY(weighted_similarity_all(N, NNZ, off_u, deg, adj_u, w_dev, sims, tmp, s, prof ? &ist : nullptr,
                                       icfg.skip_deg));
    } else {
      SCAN_TRY(intersect_all(icfg, N, NNZ, off_u, deg, adj_u, kind, sims, counts, device, s, &ist, co_prep, &plan));
    }
    if (lsh) SCAN_TRY(lsh_overwrite(lsh_dev, N, NNZ, off_u, adj_u, weighted ? w_dev : nullptr, kind, sims, tmp, s));
    mark(3);
    if (prof) {
      prof->window_bits = ist.wbits;
      prof->intersect_launches = ist.launches;
    }

    // a5: neighbour order, then ids made local to each graph (with the
    // tables, which came on the helper stream).
    SCAN_TRY(sort_run(no_cls, off_u, NNZ, sims, adj_u, no_sim, no_ids, s));
    if (cs != s) SCAN_TRY(stream_wait(s, cs));
    if (G > 1)
      k_localize_ids<<<grid_for(NNZ / kLocalizePer + 1, 256), 256, 0, s>>>(no_ids, d_ebase, d_vbase, G, NNZ);
    mark(4);

    // a6, second part: transposed fill, segmented sort (after the helper
    // stream's part above).
    if (nrt > 0) {
      k_co_fill<<<grid_for(NNZ / 512 + 1, 1, 1 << 16), 256, 0, s>>>(d_rt, nrt, G == 1 ? 1 : 0, d_tile_first, d_sv,
                                                                    d_vbase, d_nz, no_sim, d_corel, d_cobase,
                                                                    d_ebase, d_vbase, co_key, co_id);
    }
    SCAN_TRY(sort_run(co_cls, d_seg, NNZ, co_key, co_id, co_thr, co_ids, s));
    SCAN_HIP_TRY(hipGetLastError());
    mark(5);
  } else {
    // no edges: every co_off is zero
    SCAN_TRY(upload_tables(s));
    SCAN_HIP_TRY(hipMemsetAsync(d_corel, 0, (size_t)cobase[G] * 8, s));
    for (int k = 2; k < 10; ++k) mark(k);
  }

  // Per-graph offsets (local), then the index views.
  int64_t *off_local = off_u;
  if (G > 1) {
    SCAN_TRY(arena_alloc(*arena, &off_local, obase[G]));
    k_local_offsets<<<grid_for(obase[G], 256), 256, 0, s>>>(off_u, d_obase, d_vbase, d_ebase, G, obase[G],
                                                            off_local);
  }
  SCAN_HIP_TRY(hipGetLastError());
  // The build returns without waiting for the device: the temporaries are
  // released in stream order, and the pinned staging of the host tables
  // goes back to the pool once this event has passed.
  SCAN_HIP_TRY(hipEventCreateWithFlags(&arena->done, hipEventDisableTiming));
  SCAN_HIP_TRY(hipEventRecord(arena->done, s));

  for (int32_t g = 0; g < G; ++g) {
    scan_index *ix = new scan_index();
    ix->n = gs[g].n;
    ix->nnz = gs[g].nnz;
    ix->dmax = hdmax[g];
    ix->kind = kind;
    ix->flags = flags & (SCAN_KEEP_SIMS | SCAN_KEEP_COUNTS | SCAN_PROFILE);
    ix->stream = s;
    ix->device = device;
    ix->off = off_local + (G > 1 ? obase[g] : 0);
    ix->no_ids = no_ids + ebase[g];
    ix->no_sim = no_sim + ebase[g];
    ix->co_off = d_corel + cobase[g];
    ix->co_ids = co_ids + ebase[g];
    ix->co_thr = co_thr + ebase[g];
    if (flags & SCAN_KEEP_SIMS) ix->sims = sims + ebase[g];
    if (counts) ix->counts = counts + ebase[g];
    ix->arena = arena;
    ix->prof = prof;
    ix->bytes = (gs[g].n + 1) * 8 + gs[g].nnz * 24 + (int64_t)(hdmax[g] + 3) * 8 +
                ((flags & SCAN_KEEP_SIMS) ? gs[g].nnz * 8 : 0) + (counts ? gs[g].nnz * 4 : 0);
    outs[g] = ix;
  }
  return SCAN_OK;
}

scan_status build_index(const scan_csr *g, int32_t kind, uint32_t flags, hipStream_t s,
                        const IntersectConfig &cfg, scan_index **out) {
  if (!g) return fail(SCAN_EINVAL, "null graph");
  return build_index_batch(g, 1, kind, flags, s, cfg, out);
}

}  // namespace scan
