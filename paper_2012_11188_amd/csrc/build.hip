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

__global__ void k_union_prepare(const GraphDesc *gd, const int64_t *item_base, int G,
                                int64_t total, int copy_adj, int64_t *off_u, int32_t *deg_u,
                                int32_t *adj_u, unsigned *dmax_g) {
  // running maximum degree of the graph this thread last visited, flushed
  // with one atomic per wavefront when all its lanes saw the same graph
  int gl = -1;
  unsigned ml = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int g = find_graph(item_base, G, i);
    const GraphDesc d = gd[g];
    const int64_t j = i - d.item_base;
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
        if (g != gl) {
          if (gl >= 0) atomicMax(&dmax_g[gl], ml);
          gl = g;
          ml = 0;
        }
        ml = max(ml, (unsigned)(deg > 0 ? deg : 0));
      }
    } else if (copy_adj) {
      const int64_t s = j - (d.n + 1);
      adj_u[d.ebase + s] = (int32_t)(d.vbase + d.adj[s]);
    }
  }
  const int g0 = __builtin_amdgcn_readfirstlane(gl);
  if (__all(gl == g0)) {
    unsigned m = ml;
#pragma unroll
    for (int k = kWave / 2; k > 0; k >>= 1) m = max(m, (unsigned)__shfl_xor((int)m, k, kWave));
    if ((threadIdx.x & (kWave - 1)) == 0 && g0 >= 0) atomicMax(&dmax_g[g0], m);
  } else if (gl >= 0) {
    atomicMax(&dmax_g[gl], ml);
  }
}

// Vertex ids in [lo, hi) slots of the union made local: id - vbase(g).
__global__ void k_localize_ids(int32_t *ids, const int64_t *ebase, const int64_t *vbase, int G,
                               int64_t nnz) {
  for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < nnz;
       s += (int64_t)gridDim.x * blockDim.x) {
    const int g = find_graph(ebase, G, s);
    ids[s] -= (int32_t)vbase[g];
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

// Rank of every non-isolated vertex of its graph, degree-descending (ties in
// any order: each CO segment is sorted afterwards): r = #{deg > d} + the
// vertex's position among those of degree d, from LDS counters per tile plus
// one global reservation per (tile, degree). sv[svbase[g] + r] = union id.
__global__ __launch_bounds__(256) void k_co_rank(const VTile *tiles, int64_t ntiles,
                                                 const int32_t *deg, const int64_t *hbase,
                                                 const int64_t *Ebase, const unsigned *dmax_g,
                                                 const int64_t *E_all, int32_t *cursor_all,
                                                 const int64_t *n_g, const int64_t *svbase,
                                                 int32_t *sv_all) {
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
      sv_all[svbase[g] + r] = (int32_t)v;
    }
  }
}

// Number of mu tiles of each rank tile (its first rank has the top degree).
__global__ void k_co_tiles(const RTile *rt, int64_t nrt, const int32_t *sv_all,
                           const int64_t *svbase, const int32_t *deg, int32_t *tiles_of) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < nrt;
       t += (int64_t)gridDim.x * blockDim.x)
    tiles_of[t] = (deg[sv_all[svbase[rt[t].g] + rt[t].r0]] + kFillMu - 1) / kFillMu;
}

// One workgroup per (rank tile, mu tile): kFillRanks consecutive ranks x
// kFillMu consecutive mu, read row-contiguously from NO_SIM into LDS and
// written segment-contiguously into the unsorted core order.
__global__ __launch_bounds__(256) void k_co_fill(const RTile *rt, int64_t nrt,
                                                 const int64_t *tile_first, const int32_t *sv_all,
                                                 const int64_t *svbase, const int64_t *nz_g,
                                                 const int32_t *deg, const int64_t *off,
                                                 const double *no_sim, const int64_t *coabs_all,
                                                 const int64_t *coabs_base, const int64_t *vbase,
                                                 double *co_key, int32_t *co_id) {
  __shared__ double tile[kFillMu][kFillRanks + 1];
  __shared__ int32_t vs[kFillRanks], vd[kFillRanks];
  __shared__ int64_t vo[kFillRanks];
  __shared__ int64_t s_t, s_k;
  const int64_t total = tile_first[nrt];
  for (int64_t b = blockIdx.x; b < total; b += gridDim.x) {
    __syncthreads();
    if (threadIdx.x == 0) {
      int64_t lo = 0, hi = nrt;  // last rank tile with tile_first <= b
      while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        if (tile_first[mid] <= b) lo = mid;
        else hi = mid;
      }
      s_t = lo;
      s_k = b - tile_first[lo];
    }
    __syncthreads();
    const RTile r = rt[s_t];
    const int64_t r0 = r.r0;
    const int32_t j0 = (int32_t)(s_k * kFillMu);
    const int64_t *coabs = coabs_all + coabs_base[r.g];
    const int32_t vb = (int32_t)vbase[r.g];
    if (threadIdx.x < kFillRanks) {
      const int64_t rr = r0 + threadIdx.x;
      int32_t v = 0, d = 0;
      int64_t o = 0;
      if (rr < nz_g[r.g]) {
        v = sv_all[svbase[r.g] + rr];
        d = deg[v];
        o = off[v];
      }
      vs[threadIdx.x] = v - vb;
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
        const int64_t pos = coabs[j0 + j + 2] + r0 + i;
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

template <class T>
scan_status to_device(DevArena &tmp, T **dst, const std::vector<T> &src, hipStream_t s) {
  SCAN_TRY(tmp.alloc(dst, (int64_t)src.size()));
  if (!src.empty())
    SCAN_HIP_TRY(hipMemcpyAsync(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, s));
  return SCAN_OK;
}

}  // namespace

scan_status build_index_batch(const scan_csr *gs, int32_t G, int32_t kind, uint32_t flags,
                              hipStream_t s, const IntersectConfig &cfg, scan_index **outs) {
  if (G < 0 || (G > 0 && (!gs || !outs))) return fail(SCAN_EINVAL, "bad batch arguments");
  for (int32_t g = 0; g < G; ++g) {
    outs[g] = nullptr;
    SCAN_TRY(check_csr(&gs[g]));
  }
  if (kind != SCAN_SIM_COSINE && kind != SCAN_SIM_JACCARD) return fail(SCAN_EINVAL, "unknown similarity kind %d", kind);
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
  int64_t *d_item_base;
  SCAN_TRY(to_device(tmp, &d_gd, hd, s));
  SCAN_TRY(to_device(tmp, &d_item_base, item_base, s));
  SCAN_HIP_TRY(hipMemsetAsync(d_dmax, 0, (size_t)G * 4, s));
  SCAN_HIP_TRY(hipMemsetAsync(off_u, 0, 8, s));
  {
    const int64_t total = item_base[G];
    // graphs without vertices contribute only their (zero) end offset
    std::vector<GraphDesc> fix = hd;
    bool any_empty = false;
    for (int32_t g = 0; g < G; ++g)
      if (gs[g].n == 0) any_empty = true;
    int64_t *zero_off = nullptr;
    if (any_empty) {
      SCAN_TRY(tmp.alloc(&zero_off, 1));
      SCAN_HIP_TRY(hipMemsetAsync(zero_off, 0, 8, s));
      for (int32_t g = 0; g < G; ++g)
        if (gs[g].n == 0) {
          fix[g].off = zero_off;
          fix[g].off_bits = 64;
        }
      SCAN_HIP_TRY(hipMemcpyAsync(d_gd, fix.data(), fix.size() * sizeof(GraphDesc), hipMemcpyHostToDevice, s));
      SCAN_HIP_TRY(hipStreamSynchronize(s));
    }
    if (total > 0)
      k_union_prepare<<<grid_for(total, 256), 256, 0, s>>>(d_gd, d_item_base, G, total, copy_adj ? 1 : 0,
                                                          off_u, deg, adj_u, d_dmax);
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
  std::vector<unsigned> hdmax(G);
  SCAN_HIP_TRY(hipMemcpyAsync(hdmax.data(), d_dmax, (size_t)G * 4, hipMemcpyDeviceToHost, s));
  SCAN_HIP_TRY(hipStreamSynchronize(s));
  SCAN_HIP_TRY(hipGetLastError());
  mark(1);

  int32_t *no_ids, *co_ids, *counts = nullptr;
  double *no_sim, *co_thr, *sims;
  SCAN_TRY(arena_alloc(*arena, &no_ids, NNZ));
  SCAN_TRY(arena_alloc(*arena, &no_sim, NNZ));
  SCAN_TRY(arena_alloc(*arena, &co_ids, NNZ));
  SCAN_TRY(arena_alloc(*arena, &co_thr, NNZ));
  if (flags & SCAN_KEEP_SIMS) SCAN_TRY(arena_alloc(*arena, &sims, NNZ));
  else SCAN_TRY(tmp.alloc(&sims, NNZ));
  if (flags & SCAN_KEEP_COUNTS) SCAN_TRY(arena_alloc(*arena, &counts, NNZ));

  // Per-graph core-order bookkeeping (host), filled below.
  std::vector<int64_t> hbase(G + 1, 0), Ebase(G + 1, 0), cobase(G + 1, 0), ng(G), nz(G, 0), svbase(G + 1, 0);
  for (int32_t g = 0; g < G; ++g) {
    hbase[g + 1] = hbase[g] + hdmax[g] + 1;
    Ebase[g + 1] = Ebase[g] + hdmax[g] + 2;
    cobase[g + 1] = cobase[g] + hdmax[g] + 3;
    ng[g] = gs[g].n;
  }
  std::vector<int64_t> corel(cobase[G], 0);  // per-graph co_off, relative

  if (NNZ > 0) {
    // a2-a4: ownership plan, intersection and similarity over the union.
    IntersectStats ist;
    if (prof) {
      ist.ev_start = prof->ev[2];
      ist.ev_end = prof->ev[3];
    }
    SCAN_TRY(intersect_all(cfg, N, NNZ, off_u, deg, adj_u, kind, sims, counts, device, s, &ist));
    if (prof) {
      prof->owners = ist.owners_small;
      prof->intersect_launches = (ist.owners_small > 0) + (ist.chunks_big > 0);
    }

    // a5: neighbour order, then ids made local to each graph.
    SCAN_TRY(segmented_sort(off_u, N, NNZ, sims, adj_u, no_sim, no_ids, s));
    int64_t *d_vbase, *d_ebase;
    SCAN_TRY(to_device(tmp, &d_vbase, vbase, s));
    SCAN_TRY(to_device(tmp, &d_ebase, ebase, s));
    if (G > 1) k_localize_ids<<<grid_for(NNZ, 256), 256, 0, s>>>(no_ids, d_ebase, d_vbase, G, NNZ);
    mark(4);

    // a6: core order. Degree histograms per graph -> sizes (host).
    std::vector<VTile> vt;
    for (int32_t g = 0; g < G; ++g)
      for (int64_t v0 = vbase[g]; v0 < vbase[g + 1]; v0 += kRankTile)
        vt.push_back(VTile{g, 0, v0, std::min(vbase[g + 1], v0 + kRankTile)});
    VTile *d_vt;
    int64_t *d_hbase;
    int32_t *d_hist, *d_cursor;
    SCAN_TRY(to_device(tmp, &d_vt, vt, s));
    SCAN_TRY(to_device(tmp, &d_hbase, hbase, s));
    SCAN_TRY(tmp.alloc(&d_hist, hbase[G]));
    SCAN_TRY(tmp.alloc(&d_cursor, hbase[G]));
    SCAN_HIP_TRY(hipMemsetAsync(d_hist, 0, (size_t)hbase[G] * 4, s));
    SCAN_HIP_TRY(hipMemsetAsync(d_cursor, 0, (size_t)hbase[G] * 4, s));
    if (!vt.empty())
      k_graph_hist<<<grid_for((int64_t)vt.size(), 1, 8192), 256, 0, s>>>(d_vt, (int64_t)vt.size(), deg, d_hbase, d_dmax, d_hist);
    std::vector<int32_t> hist(hbase[G]);
    SCAN_HIP_TRY(hipMemcpyAsync(hist.data(), d_hist, hist.size() * 4, hipMemcpyDeviceToHost, s));
    SCAN_HIP_TRY(hipStreamSynchronize(s));
    std::vector<int64_t> E(Ebase[G]), coabs(cobase[G]), seg;
    std::vector<RTile> rt;
    seg.reserve(hbase[G] + 1);
    for (int32_t g = 0; g < G; ++g) {
      const int64_t dm = hdmax[g], n = gs[g].n;
      int64_t *Eg = &E[Ebase[g]];
      int64_t *cr = &corel[cobase[g]];
      Eg[0] = 0;
      for (int64_t d = 0; d <= dm; ++d) Eg[d + 1] = Eg[d] + hist[hbase[g] + d];
      cr[0] = cr[1] = cr[2] = 0;
      for (int64_t mu = 2; mu <= dm + 1; ++mu) cr[mu + 1] = cr[mu] + (n - Eg[mu - 1]);
      for (int64_t mu = 0; mu <= dm + 2; ++mu) coabs[cobase[g] + mu] = ebase[g] + cr[mu];
      for (int64_t mu = 2; mu <= dm + 1; ++mu) seg.push_back(ebase[g] + cr[mu]);
      nz[g] = dm > 0 ? n - hist[hbase[g]] : 0;
      svbase[g + 1] = svbase[g] + nz[g];
      for (int64_t r0 = 0; r0 < nz[g]; r0 += kFillRanks) rt.push_back(RTile{g, (int32_t)r0});
    }
    seg.push_back(NNZ);
    int64_t *d_E, *d_Ebase, *d_coabs, *d_cobase, *d_seg, *d_ng, *d_nz, *d_svbase, *d_tile_first, *scan_ws;
    RTile *d_rt;
    int32_t *d_sv, *d_tiles_of;
    double *co_key;
    int32_t *co_id;
    SCAN_TRY(to_device(tmp, &d_E, E, s));
    SCAN_TRY(to_device(tmp, &d_Ebase, Ebase, s));
    SCAN_TRY(to_device(tmp, &d_coabs, coabs, s));
    SCAN_TRY(to_device(tmp, &d_cobase, cobase, s));
    SCAN_TRY(to_device(tmp, &d_seg, seg, s));
    SCAN_TRY(to_device(tmp, &d_ng, ng, s));
    SCAN_TRY(to_device(tmp, &d_nz, nz, s));
    SCAN_TRY(to_device(tmp, &d_svbase, svbase, s));
    SCAN_TRY(to_device(tmp, &d_rt, rt, s));
    const int64_t nrt = (int64_t)rt.size();
    SCAN_TRY(tmp.alloc(&d_sv, std::max<int64_t>(svbase[G], 1)));
    SCAN_TRY(tmp.alloc(&d_tiles_of, std::max<int64_t>(nrt, 1)));
    SCAN_TRY(tmp.alloc(&d_tile_first, nrt + 1));
    SCAN_TRY(tmp.alloc(&scan_ws, scan_workspace_elems(std::max<int64_t>(nrt, 1))));
    SCAN_TRY(tmp.alloc(&co_key, NNZ));
    SCAN_TRY(tmp.alloc(&co_id, NNZ));
    k_co_rank<<<grid_for((int64_t)vt.size(), 1, 8192), 256, 0, s>>>(d_vt, (int64_t)vt.size(), deg, d_hbase, d_Ebase, d_dmax,
                                                                   d_E, d_cursor, d_ng, d_svbase, d_sv);
    if (nrt > 0) {
      k_co_tiles<<<grid_for(nrt, 256), 256, 0, s>>>(d_rt, nrt, d_sv, d_svbase, deg, d_tiles_of);
      SCAN_TRY(exclusive_scan(d_tiles_of, d_tile_first, nrt, scan_ws, s));
      k_co_fill<<<grid_for(NNZ / 512 + 1, 1, 1 << 16), 256, 0, s>>>(d_rt, nrt, d_tile_first, d_sv, d_svbase, d_nz, deg,
                                                                    off_u, no_sim, d_coabs, d_cobase, d_vbase,
                                                                    co_key, co_id);
    }
    SCAN_TRY(segmented_sort(d_seg, (int64_t)seg.size() - 1, NNZ, co_key, co_id, co_thr, co_ids, s));
    SCAN_HIP_TRY(hipGetLastError());
    mark(5);
    SCAN_HIP_TRY(hipStreamSynchronize(s));  // host-side tables above feed async copies
  } else {
    for (int k = 2; k < 6; ++k) mark(k);
  }

  // Per-graph offsets (local) and core-order offsets, then the index views.
  int64_t *off_local = off_u, *d_corel;
  std::vector<int64_t> obase(G + 1, 0);
  for (int32_t g = 0; g < G; ++g) obase[g + 1] = obase[g] + gs[g].n + 1;
  if (G > 1) {
    int64_t *d_obase, *d_vb, *d_eb;
    SCAN_TRY(arena_alloc(*arena, &off_local, obase[G]));
    SCAN_TRY(to_device(tmp, &d_obase, obase, s));
    SCAN_TRY(to_device(tmp, &d_vb, vbase, s));
    SCAN_TRY(to_device(tmp, &d_eb, ebase, s));
    k_local_offsets<<<grid_for(obase[G], 256), 256, 0, s>>>(off_u, d_obase, d_vb, d_eb, G, obase[G], off_local);
  }
  SCAN_TRY(arena_alloc(*arena, &d_corel, cobase[G]));
  SCAN_HIP_TRY(hipMemcpyAsync(d_corel, corel.data(), corel.size() * 8, hipMemcpyHostToDevice, s));
  SCAN_HIP_TRY(hipGetLastError());
  SCAN_HIP_TRY(hipStreamSynchronize(s));

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
