// Index object and internal entry points shared by the library's host code.
#pragma once

#include <functional>
#include <memory>
#include <mutex>
#include <vector>

#include "common.h"

namespace scan {

// Tunable parameters of the intersection kernels (chosen per graph by the
// autotuner or the defaults).
struct IntersectConfig {
  int32_t small_max = 256;  // owners of degree <= small_max: one wavefront each
  int32_t spc = 512;        // row slots per chunk of a larger owner
  int32_t wbits = 20;       // LDS bitmap window of 2^wbits ids (clamped to LDS)
  bool search_windows = false;  // several windows: search row ranges instead of tabling them
  int32_t skip_deg = 0x7fffffff;  // edges whose endpoints both exceed this degree are left unwritten
                                  // (approximate builds overwrite them)
};

struct IntersectStats {
  int32_t wbits = 0;
  int32_t launches = 0;
  // Optional pinned host int32[4]: receives (light vertices, bitmap chunks,
  // -, heavy vertices) asynchronously, in stream order.
  int32_t *host_counts = nullptr;
  // around the small-owner launches and around the large-owner launch (on
  // the streams that run them; the two may overlap)
  hipEvent_t ev_plan_end = nullptr;  // after the ownership plan
  hipEvent_t ev_small_begin = nullptr, ev_small_end = nullptr;
  hipEvent_t ev_big_begin = nullptr, ev_big_end = nullptr;
};

// a2: the ownership plan, enqueued on s (the work lists live in `arena`,
// which must outlive intersect_all), with a copy of its counts to pinned host
// memory; intersect_all waits for them on the host. Launched early, the plan
// is read back by a wait the caller makes anyway.
struct IntersectPlan {
  int64_t n = 0, nnz = 0;
  int32_t *small_list = nullptr, *heavy_list = nullptr;
  void *big_list = nullptr, *counts = nullptr;  // device chunk list and counts
  void *host = nullptr;                         // pinned copy of the counts
  hipEvent_t ready = nullptr;
  // helper streams already ordered after the plan (set by the caller), used
  // for the two small-owner kernels; null: intersect_all orders its own
  hipStream_t helper[2] = {nullptr, nullptr};
  int32_t wbits = 0;       // the large-owner kernel's id window width
  int32_t *wt = nullptr;   // window table (ids over several windows), or null
  IntersectPlan() = default;
  IntersectPlan(const IntersectPlan &) = delete;
  IntersectPlan &operator=(const IntersectPlan &) = delete;
  ~IntersectPlan();
};
scan_status intersect_plan(const IntersectConfig &cfg, int64_t n, int64_t nnz, const int64_t *off,
                           const int32_t *deg, const int32_t *adj, int device, DevArena &arena, hipStream_t s,
                           IntersectPlan &plan);

// a2-a4: ownership plan, then intersection + similarity for every edge,
// written into both CSR slots of sims (and counts if non-null).
// after_launch (may be empty) runs on the host once every intersection
// kernel is enqueued, so that the host enqueues other work (on streams it has
// ordered itself) while the device intersects. plan (may be null: then it
// plans on s itself) is one made by intersect_plan on s with the same cfg,
// n, nnz and deg.
scan_status intersect_all(const IntersectConfig &cfg, int64_t n, int64_t nnz, const int64_t *off,
                          const int32_t *deg, const int32_t *adj, int kind, double *sims,
                          int32_t *counts, int device, hipStream_t s, IntersectStats *stats,
                          const std::function<scan_status()> &after_launch = {},
                          const IntersectPlan *plan = nullptr);

// Approximate similarities (lsh.hip): k samples, and the random draws on
// the device (gauss n x k for SimHash, perm for MinHash).
struct LshSpec {
  int32_t samples = 0;
  const double *gauss = nullptr;
  const uint32_t *perm = nullptr;
};

// Weighted cosine of every edge into both CSR slots of sims (weighted.hip);
// events (may be null) before the square sums, before the products, after.
// The square sums are timed as the "small" part, the owner products as the
// "big" part (stats may be null).
scan_status weighted_similarity_all(int64_t n, int64_t nnz, const int64_t *off, const int32_t *deg,
                                    const int32_t *adj, const double *w, double *sims, DevArena &tmp,
                                    hipStream_t s, const IntersectStats *stats, int32_t skip_deg = 0x7fffffff);
// Overwrites sims of the edges between two high-degree vertices with their
// SimHash (cosine kinds) or k-partition MinHash (Jaccard) estimates; w may
// be null (unweighted). spec's pointers are device pointers.
scan_status lsh_overwrite(const LshSpec &spec, int64_t n, int64_t nnz, const int64_t *off, const int32_t *adj,
                          const double *w, int kind, double *sims, DevArena &tmp, hipStream_t s);
// SCAN_EGRAPH unless every weight is finite (waits for the stream).
scan_status check_weights(const double *w, int64_t nnz, DevArena &tmp, hipStream_t s);

// Per-query device workspace (one slot of a batch).
struct QuerySlot {
  int32_t *parent = nullptr;  // int32[n] union-find parents (read for cores only)
  uint8_t *flag = nullptr;    // uint8[n] state: 2 core, 1 candidate border; all zero between queries
  size_t bytes = 0;
};

// Device-side descriptor of one query of a batch (query.hip).
struct QueryDesc {
  int32_t mu;
  int32_t pad;
  double eps;
  int64_t base;  // co_off[mu] (0 if mu > dmax + 1)
  int64_t K;     // number of cores
  int32_t *parent;
  uint8_t *flag;
  int32_t *memb;  // nullptr: unused batch entry
  uint8_t *is_core;
};

}  // namespace scan

namespace scan {

struct DevAlloc {
  void *p;
  size_t bytes;
};

// Device buffers shared by the indexes of one batched build (each index is a
// view into them); freed when the last index referring to it is freed.
struct SharedArena {
  hipStream_t stream = nullptr;
  std::vector<DevAlloc> allocs;
  int64_t bytes = 0;
  // Pinned staging of the build's host tables, returned to the pool once
  // `done` (recorded at the end of the build) has completed.
  std::vector<PinnedBlock> pinned;
  hipEvent_t done = nullptr;
  ~SharedArena();
};

// SCAN_PROFILE events of a build (shared by the indexes of a batch): start,
// prepare, plan, intersect, neighbour order, core order, then the begin and
// end of the small-owner launches (6, 7) and of the large-owner launch (8,
// 9), which may run concurrently on two streams.
struct BuildProfileEvents {
  hipEvent_t ev[10] = {};
  int32_t window_bits = 0;
  int32_t intersect_launches = 0;
  // (light owners, big chunks, -, heavy owners), written by the host when it
  // reads the plan's counts back
  int32_t plan_counts[4] = {0, 0, 0, 0};
  ~BuildProfileEvents();
};

}  // namespace scan

struct scan_index {
  int64_t n = 0, nnz = 0, dmax = 0;
  int32_t kind = 0;
  uint32_t flags = 0;
  hipStream_t stream = nullptr;
  int device = 0;
  int64_t *off = nullptr;      // int64[n+1]
  int32_t *no_ids = nullptr;   // int32[nnz]
  double *no_sim = nullptr;    // double[nnz]
  int64_t *co_off = nullptr;   // int64[dmax+3]
  int32_t *co_ids = nullptr;   // int32[nnz]
  double *co_thr = nullptr;    // double[nnz]
  double *sims = nullptr;      // double[nnz] (SCAN_KEEP_SIMS)
  int32_t *counts = nullptr;   // int32[nnz]  (SCAN_KEEP_COUNTS)
  std::shared_ptr<scan::SharedArena> arena;        // owns the arrays above
  std::shared_ptr<scan::BuildProfileEvents> prof;  // SCAN_PROFILE only
  int64_t bytes = 0;                               // device bytes of this index's arrays
  // Query workspace pool: a slot may be reused once its last use completed
  // (event) or when the new use is on the same stream.
  struct PooledSlot {
    scan::QuerySlot slot;
    hipEvent_t done = nullptr;
    hipStream_t last_stream = nullptr;
    bool busy = false;
  };
  std::mutex pool_mu;
  std::vector<PooledSlot *> pool;
};

namespace scan {

void index_release(scan_index *ix);

scan_status build_index(const scan_csr *g, int32_t kind, uint32_t flags, hipStream_t stream,
                        const IntersectConfig &cfg, scan_index **out);
// weights: per-slot edge weights (kind SCAN_SIM_WEIGHTED_COSINE, one graph
// only), on the same side (host or device) as the graph. lsh (one graph only):
// approximate the edges between high-degree vertices; its draws are on the
// graph's side too.
scan_status build_index_batch(const scan_csr *gs, int32_t count, int32_t kind, uint32_t flags,
                              hipStream_t stream, const IntersectConfig &cfg, scan_index **outs,
                              const double *weights = nullptr, const LshSpec *lsh = nullptr);

// Runs `count` queries. mu/eps host arrays; memberships[i] / is_core[i] are
// device pointers (is_core may hold nulls). Slots are workspaces, one per
// query.
scan_status run_queries(const scan_index *ix, int32_t count, const int32_t *mu, const double *eps,
                        int32_t *const *memberships, uint8_t *const *is_core,
                        const QuerySlot *slots, hipStream_t s);

scan_status alloc_query_slot(const scan_index *ix, QuerySlot *slot, hipStream_t s);

// Enqueues the four query kernels for `count` device descriptors.
void launch_query_kernels(const scan_index *ix, QueryDesc *d, int32_t count, hipStream_t s);
// Modularity terms (quality.hip): terms[0] += s_in, terms[1] += sd2 for one
// clustering; dsum (int64[n]) must be zero on entry and is zero on return.
void zero64(int64_t *p, int64_t count, hipStream_t s);
void launch_modularity_terms(const scan_index *ix, const int32_t *memb, int64_t *dsum, int64_t *terms,
                             hipStream_t s);
double modularity_value(int64_t s_in, int64_t sd2, int64_t nnz);

// Hub / outlier roles of the unclustered vertices of one query's memberships.
void launch_roles(const scan_index *ix, const int32_t *memb, uint8_t *roles, hipStream_t s);
// One query whose workspace is the library's file-scope scratch array (no
// allocation); memberships / is_core are device pointers.
scan_status query_noalloc(const scan_index *ix, int32_t mu, double eps, int32_t *memberships, uint8_t *is_core,
                          hipStream_t s);
QueryDesc make_query_desc(int32_t mu, double eps, const QuerySlot &slot, int32_t *memb,
                          uint8_t *is_core);
void free_query_slot(QuerySlot *slot, hipStream_t s);

IntersectConfig default_config();

scan_status similarity_values(int32_t kind, int64_t count, const int64_t *c, const int64_t *a_u,
                              const int64_t *a_v, double *out);

}  // namespace scan
