/*
 * scan.h — C ABI of an exact index-based SCAN library for AMD MI355X (gfx950).
 *
 * Method: Tseng, Dhulipala and Shun, "Parallel Index-Based Structural Graph
 * Clustering and Its Approximation" (SIGMOD 2021):
 *   - structural similarity over closed neighbourhoods (Section 3.1),
 *     cosine or Jaccard (Section 2.1.1), computed per edge as in Algorithm 1;
 *   - the GS*-style index: neighbour order NO and core order CO (Section 3.2,
 *     Algorithm 2);
 *   - (mu, eps) clustering queries over the index (Section 4.2, Algorithms
 *     3-5), with the deterministic border rule of Section 7.3.4.
 *
 * Conventions shared by every entry point
 *   - Vertex ids are 0-based int32. A graph is simple and undirected, stored as
 *     CSR with both directions of every edge, each row strictly ascending, no
 *     self-loops (Section 2.2). nnz = 2|E|.
 *   - Similarities are IEEE binary64, computed exactly as
 *       cosine : c / sqrt((double)a_u * (double)a_v)
 *       Jaccard: (double)c / (double)(a_u + a_v - c)
 *     with c = |N[u] ∩ N[v]| and a_v = |N[v]| = deg(v) + 1.
 *   - Both orders sort by similarity descending, ties by vertex id ascending.
 *   - Query results: memberships[v] is the smallest core id of v's cluster, or
 *     -1 if v is unclustered. A border vertex joins the cluster of its most
 *     similar eps-similar core neighbour, ties to the lower id.
 *   - Errors: every call returns a scan_status; on failure scan_last_error()
 *     returns a message for the calling thread. No C++ exception crosses the
 *     ABI. Argument errors are detected before any device work is enqueued.
 *   - Streams: `stream` is a hipStream_t (NULL = the default stream). Device
 *     work is enqueued on it asynchronously unless a function says otherwise;
 *     the builds (scan_build_index*) wait on the host only for small
 *     read-backs that size their grids, see there.
 *   - Ownership: the caller owns the CSR and every output buffer; the library
 *     keeps no caller pointer after a call returns, but device work a call has
 *     enqueued may read the caller's device inputs until `stream` passes it. The library owns each
 *     scan_index and scan_server and their device memory until the matching
 *     free/destroy call.
 */
#ifndef SCAN_MI355X_H
#define SCAN_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SCAN_OK = 0,
  SCAN_EINVAL = -1,  /* bad argument: null pointer, negative size, odd nnz,
                        unknown kind, mu < 2, NaN eps, short buffer        */
  SCAN_EGRAPH = -2,  /* (with SCAN_VALIDATE) not a simple undirected CSR   */
  SCAN_ENOMEM = -3,  /* device allocation failed                           */
  SCAN_EDEVICE = -4, /* HIP runtime error                                  */
  SCAN_EBUSY = -5    /* server admission refused: no slot or memory        */
} scan_status;

/* SCAN_SIM_WEIGHTED_COSINE (Section 3.1's weighted form) is built only by
 * scan_build_index_weighted, which takes the edge weights. */
typedef enum { SCAN_SIM_COSINE = 0, SCAN_SIM_JACCARD = 1, SCAN_SIM_WEIGHTED_COSINE = 2 } scan_sim_kind;

/* Build flags. */
enum {
  SCAN_VALIDATE = 1u,    /* check the CSR on the device; SCAN_EGRAPH if bad
                            (synchronises the stream)                        */
  SCAN_KEEP_SIMS = 2u,   /* keep per-CSR-slot similarities (export SIMS)      */
  SCAN_KEEP_COUNTS = 4u, /* keep per-CSR-slot counts c (export COUNTS)        */
  SCAN_PROFILE = 8u      /* record per-phase device times with hipEvents      */
};

/* Per-phase device times of a build made with SCAN_PROFILE, in milliseconds,
 * from hipEvents recorded on the build stream between phases:
 *   prepare     degrees, offsets, max degree (and validation if asked),
 *               the per-row window table (when ids span several bitmap
 *               windows), the edge-ownership plan (chunk lists per table
 *               class) and the read-back of the max degree and plan counts
 *   plan        from that read-back to the first intersection launch (the
 *               device is idle here)
 *   intersect   all intersection + similarity launches, split into
 *               intersect_small (owners of degree <= small_max, one
 *               wavefront each) and intersect_big (bitmap-window owners)
 *   no_sort     neighbour-order segmented sort
 *   core_order  core-order sizes, placement and segmented sort
 * total spans all of them (host synchronisation gaps included). */
typedef struct {
  double total_ms;
  double prepare_ms;
  double plan_ms;
  double intersect_ms;
  double no_sort_ms;
  double core_order_ms;
  double intersect_small_ms;
  double intersect_big_ms;
  int32_t intersect_launches;
  int32_t small_owners;  /* vertices of degree 1..small_max (LDS hash path) */
  int32_t big_chunks;    /* row chunks of larger vertices (bitmap path)    */
  int32_t window_bits;   /* bitmap window used (2^window_bits ids)         */
} scan_build_profile;

/* A graph in CSR form. offsets has n+1 entries of offset_bits (32 or 64)
 * bits; adj has nnz int32 entries. on_device = 1: both are device pointers
 * (read by the build's device work, not retained); 0: host pointers (copied
 * to the device before the build call returns). */
typedef struct {
  int64_t n;
  int64_t nnz;
  int32_t offset_bits;
  int32_t on_device;
  const void *offsets;
  const int32_t *adj;
} scan_csr;

typedef struct scan_index scan_index; /* opaque, device resident, immutable */

typedef struct {
  int64_t n;
  int64_t nnz;
  int64_t dmax;          /* maximum degree; CO has segments mu = 2..dmax+1  */
  int32_t kind;          /* scan_sim_kind                                   */
  int32_t flags;         /* build flags kept (SCAN_KEEP_*)                  */
  int64_t device_bytes;  /* device memory held by the index                 */
} scan_index_info;

/* Index arrays, all device resident, for scan_index_export / _device_ptr.
 *   OFFSETS  int64[n+1]     CSR offsets, shared by NO and the slot arrays
 *   NO_IDS   int32[nnz]     row v of NO = neighbours of v, sim desc / id asc
 *   NO_SIM   double[nnz]    their similarities
 *   CO_OFF   int64[dmax+3]  CO[mu] = co entries [CO_OFF[mu], CO_OFF[mu+1])
 *   CO_IDS   int32[nnz]     vertices with deg >= mu-1, thr desc / id asc
 *   CO_THR   double[nnz]    core thresholds NO_SIM[off[v] + mu - 2]
 *   SIMS     double[nnz]    per CSR slot, same order as adj (SCAN_KEEP_SIMS)
 *   COUNTS   int32[nnz]     c per CSR slot (SCAN_KEEP_COUNTS)               */
typedef enum {
  SCAN_ARR_OFFSETS = 0,
  SCAN_ARR_NO_IDS = 1,
  SCAN_ARR_NO_SIM = 2,
  SCAN_ARR_CO_OFF = 3,
  SCAN_ARR_CO_IDS = 4,
  SCAN_ARR_CO_THR = 5,
  SCAN_ARR_SIMS = 6,
  SCAN_ARR_COUNTS = 7
} scan_array;

/* Device memory hooks. alloc returns a device pointer of at least `bytes`
 * usable on `stream`, or NULL; release frees it (stream-ordered). Passing
 * NULL for both restores hipMalloc/hipFree. Process-wide; set it before
 * building. */
typedef void *(*scan_alloc_fn)(size_t bytes, void *stream, void *ctx);
typedef void (*scan_release_fn)(void *ptr, size_t bytes, void *stream, void *ctx);
scan_status scan_set_allocator(scan_alloc_fn alloc, scan_release_fn release, void *ctx);

/* Builds the index of Section 3.2 (Algorithms 1 and 2) for graph g: degrees,
 * per-edge intersection + similarity, the neighbour-order segmented sort and
 * the core-order sort, run on `stream`.
 * Asynchronous: the call returns once every kernel of the build is enqueued;
 * *out may be used on `stream` at once (that work is ordered after the
 * build) and on another stream once it waits for `stream`. Inside the call
 * the host waits only for small read-backs that size the grids: the maximum
 * degree together with the owner work counts (one round trip after the
 * degree pass, which also waits for work queued on `stream` before the
 * build), and the size classes of each segmented sort (read back early into
 * pinned memory, normally ready by the time they are needed); with
 * SCAN_VALIDATE also for the validation result. Builds on different streams
 * overlap on the device. A host-resident CSR may be freed once the call
 * returns; a device-resident one is read until `stream` passes the build, so
 * free it in stream order on `stream` (or with hipFree) and do not write it
 * from another stream before then.
 * Errors: SCAN_EINVAL (null g/out/pointers with n > 0, n < 0, nnz < 0, odd
 * nnz, offset_bits not 32/64, unknown kind or flag, n or nnz too large for
 * int32 ids / the chosen offsets), SCAN_EGRAPH (SCAN_VALIDATE only),
 * SCAN_ENOMEM, SCAN_EDEVICE. On error *out is NULL. */
scan_status scan_build_index(const scan_csr *g, scan_sim_kind kind, uint32_t flags, void *stream,
                             scan_index **out);

/* Builds `count` independent indexes (one per graph) with the graphs' work
 * merged into shared launches: one degree pass, one persistent intersection
 * launch over all graphs' edges, one neighbour-order sort and one core-order
 * sort. outs[i] equals what scan_build_index(&gs[i], ...) returns. All graphs
 * must be device resident (on_device = 1) or all host resident. Errors as for
 * scan_build_index; on error no index is returned. */
scan_status scan_build_index_batch(const scan_csr *gs, int32_t count, scan_sim_kind kind,
                                   uint32_t flags, void *stream, scan_index **outs);

/* Builds the index of graph g under the weighted cosine similarity of
 * Section 3.1 (the measure Algorithm 1 is written for):
 *   sigma(u, v) = D / sqrt(S_u * S_v),  D = sum over x in N[u] ∩ N[v] of
 *   w(u, x) w(v, x),  S_v = sum over x in N[v] of w(v, x)^2,
 * over closed neighbourhoods with w(x, x) = 1. weights[k] (nnz doubles,
 * parallel to g->adj, host or device like the graph) is w(u, adj[k]) for the
 * row u holding slot k; the two directions of an edge may differ. Every sum
 * adds its terms one by one in ascending vertex id, so the result is one
 * fixed FP64 value per edge; with all weights 1 the index equals the
 * SCAN_SIM_COSINE one bit for bit. Neighbour order, core order and queries are
 * as for the other kinds; the index has no intersection counts. The weights
 * follow the CSR's rules (host: may be freed once the call returns; device:
 * read until `stream` passes the build).
 * Errors: as scan_build_index, plus SCAN_EINVAL for a null weights pointer
 * with nnz > 0 or SCAN_KEEP_COUNTS, and SCAN_EGRAPH (SCAN_VALIDATE only) for a
 * weight that is not finite. */
scan_status scan_build_index_weighted(const scan_csr *g, const double *weights, uint32_t flags,
                                      void *stream, scan_index **out);

/* Approximate index (Section 5; the degree heuristic of Section 6.3): the
 * edges between two high-degree vertices (degree > samples for the cosine
 * kinds, > 3 * samples / 2 for Jaccard) get LSH estimates, every other edge
 * its exact similarity; the orders and queries are built on those values.
 *   SCAN_SIM_COSINE / SCAN_SIM_WEIGHTED_COSINE: SimHash. Bit i of v's sketch
 *     is 1 iff sum over x in N[v] (ascending x) of w(v, x) * gauss[x * k + i]
 *     is >= 0 (w(v, v) = 1; all weights 1 for SCAN_SIM_COSINE); the estimate
 *     is cos(pi * h / k) for h differing bits of the two sketches.
 *   SCAN_SIM_JACCARD: k-partition MinHash with one permutation: bin(x) =
 *     floor(perm[x] * k / n), entry b of v's sketch the least perm[x] over x
 *     in N[v] in bin b; the estimate is matching non-empty entries / (k -
 *     entries empty in both).
 * The random draws are caller inputs (host or device, like the graph):
 * gauss holds n * samples standard normal values, perm a permutation of
 * 0..n-1 (values >= n are rejected). */
typedef struct {
  int32_t samples;          /* k: a multiple of 64 in [64, 4096]              */
  int32_t reserved;         /* 0                                              */
  const double *gauss;      /* SimHash draws, row-major [x * samples + i]     */
  const uint32_t *perm;     /* MinHash permutation                            */
  const double *weights;    /* SCAN_SIM_WEIGHTED_COSINE: edge weights as for
                               scan_build_index_weighted; otherwise NULL     */
} scan_lsh;

/* Builds the approximate index of graph g. kind: SCAN_SIM_COSINE or
 * SCAN_SIM_WEIGHTED_COSINE (SimHash, needs gauss) or SCAN_SIM_JACCARD
 * (MinHash, needs perm). Inputs follow the CSR's rules of scan_build_index;
 * this build also waits for the device after its LSH pass (it reads back
 * the permutation check or keeps a host table until then). Errors: as scan_build_index, plus SCAN_EINVAL for a
 * null lsh, samples out of range, a missing draw array, weights with another
 * kind or none with SCAN_SIM_WEIGHTED_COSINE, SCAN_KEEP_COUNTS, or a
 * permutation value >= n. */
scan_status scan_build_index_lsh(const scan_csr *g, scan_sim_kind kind, const scan_lsh *lsh, uint32_t flags,
                                 void *stream, scan_index **out);

/* Shape parameters of the intersection kernels (Algorithm 1's per-edge
 * intersections). Every setting gives the same index bit for bit; they only
 * change speed. A zero field takes its default.
 *   small_max  owners of degree <= small_max use one wavefront each, with
 *              their row in LDS (1..4096; default 256)
 *   spc        row slots per work chunk of a larger owner (1..1024; default
 *              512)
 *   wbits      LDS bitmap window of 2^wbits vertex ids for larger owners
 *              (10..24; default 20); lowered to what LDS holds and to the id
 *              space; when the ids span several windows each chunk sweeps the
 *              windows that hold its owner's neighbours
 *   flags      0, or SCAN_TUNE_SEARCH_WINDOWS: with several windows, locate
 *              each lower neighbour's ids per window by search inside the
 *              chunk instead of reading them from a per-row window table
 *              ((windows + 1) * n * 4 bytes, built once per build; the search
 *              is used anyway where the table would exceed 4 GiB) */
#define SCAN_TUNE_SEARCH_WINDOWS 1
typedef struct {
  int32_t small_max;
  int32_t spc;
  int32_t wbits;
  int32_t flags;
} scan_tune;

/* scan_build_index_batch with explicit intersection shapes (tune may be
 * NULL: defaults). count = 1 builds a single graph. Errors as for
 * scan_build_index_batch; SCAN_EINVAL for a field out of range. */
scan_status scan_build_index_ex(const scan_csr *gs, int32_t count, scan_sim_kind kind,
                                uint32_t flags, const scan_tune *tune, void *stream,
                                scan_index **outs);

/* Autotuner: times the phases of builds of gs (count graphs, merged as in
 * scan_build_index_batch) up to the end of the intersection (prepare, which
 * holds the ownership plan and any window table, plan and intersect) over a
 * coordinate sweep of scan_tune (small_max, then spc, then wbits; each
 * candidate run `reps` times, the minimum kept) and writes the fastest
 * setting to *best and that time to *best_ms (may be NULL). Synchronous;
 * builds and frees temporary indexes on `stream`. reps in 1..16. */
scan_status scan_autotune(const scan_csr *gs, int32_t count, scan_sim_kind kind, int32_t reps,
                          void *stream, scan_tune *best, float *best_ms);

/* Clustering query (mu, eps), Algorithms 3-5 of Section 4.2 with the border
 * rule of Section 7.3.4. memberships: DEVICE pointer to int32[n]. Runs on the
 * stream the index was built on; asynchronous.
 * Errors: SCAN_EINVAL for a null pointer, mu < 2 or NaN eps. mu > dmax+1 is
 * not an error: no vertex is a core and every entry is -1. */
scan_status scan_query(const scan_index *ix, int32_t mu, double eps, int32_t *memberships);

/* As scan_query, on `stream`, optionally also writing is_core (uint8[n],
 * nullable). out_on_device = 0: memberships/is_core are host pointers and the
 * call returns after they are written (synchronous). Concurrent calls on
 * different streams are safe: each takes its own workspace. */
scan_status scan_query_ex(const scan_index *ix, int32_t mu, double eps, int32_t *memberships,
                          uint8_t *is_core, int32_t out_on_device, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the query of
 * scan_query_ex with device outputs, whose workspace (union-find parents,
 * state bytes and the query descriptor, 5 * n + 256 bytes) lives in a
 * file-scope device array of the library (40 MiB + 256 bytes, held on each
 * device the library runs on until the process ends) instead of allocated
 * memory. It calls no allocator and never waits for the device.
 * memberships: DEVICE int32[n]; is_core: DEVICE uint8[n] or NULL. Work is
 * enqueued on `stream` (NULL = the default stream) and the call returns at
 * once. Every call on one device shares that array: calls that overlap in
 * time on one device (other streams, other threads) race and their results
 * are undefined; calls ordered on one stream are safe. Each call clears the
 * state bytes it uses with a kernel (no memset node), so a result does not
 * depend on earlier calls.
 * Errors: SCAN_EINVAL for a null index or memberships, mu < 2, NaN eps, or an
 * index of more than 2^23 vertices; SCAN_EDEVICE if the array's address
 * cannot be taken or a launch fails. */
scan_status scan_query_noalloc(const scan_index *ix, int32_t mu, double eps, int32_t *memberships,
                               uint8_t *is_core, void *stream);

/* `count` queries (mu[i], eps[i]) answered together in shared launches:
 * memberships is int32[count * n], query i writing [i*n, (i+1)*n). mu and eps
 * are HOST arrays. out_on_device as in scan_query_ex. Each result is identical
 * to the single-query result. Errors: SCAN_EINVAL if any (mu, eps) is
 * invalid (nothing is enqueued then). */
scan_status scan_query_batch(const scan_index *ix, int32_t count, const int32_t *mu,
                             const double *eps, int32_t *memberships, int32_t out_on_device,
                             void *stream);

/* Hubs and outliers among the unclustered vertices (Section 4.3, with the
 * definitions of Section 2): roles[v] = SCAN_ROLE_CLUSTERED if
 * memberships[v] >= 0; otherwise SCAN_ROLE_HUB if v's neighbours belong to at
 * least two distinct clusters, else SCAN_ROLE_OUTLIER (neighbours in one
 * cluster or in none, isolated vertices included). memberships: DEVICE
 * int32[n], a query result on this index (labels are compared, so any
 * labelling with -1 for "unclustered" works); roles: DEVICE uint8[n], written.
 * Runs on `stream` (NULL: the index's stream), asynchronous, O(m) work.
 * Errors: SCAN_EINVAL for a null pointer. */
#define SCAN_ROLE_CLUSTERED 0
#define SCAN_ROLE_HUB 1
#define SCAN_ROLE_OUTLIER 2
scan_status scan_query_roles(const scan_index *ix, const int32_t *memberships, uint8_t *roles,
                             void *stream);

/* Modularity (Section 7.2, Newman's definition) of one clustering, every
 * unclustered vertex in a cluster of its own as in Section 7.3.4:
 *   q = 1/(2m) * sum over ordered pairs (u, v) of (A_uv - d_u d_v / 2m) delta_uv
 *     = (s_in - sd2 / 2m) / 2m, 2m = nnz,
 * with s_in (ordered neighbour pairs inside a cluster) and sd2 (sum over
 * clusters of the squared degree sum) accumulated exactly as integers on
 * the device; the last step is those two FP64 divisions. memberships: DEVICE
 * int32[n], labels -1 or in [0, n) (any other value: SCAN_EINVAL). Runs on
 * `stream` (NULL: the index's stream) and returns when *q (host) is set. */
scan_status scan_query_modularity(const scan_index *ix, const int32_t *memberships, double *q,
                                  void *stream);

/* The parameter selection of Section 7.3.4: the modularity (as above) of
 * the clustering of each (mu[i], eps[i]), i < count (host arrays), run as
 * batched queries of up to `batch` (1..256) on `stream`; q[i] (host) is
 * written. Synchronous. Device memory: batch * n * 4 + n * 8 + count * 24
 * bytes. Errors: SCAN_EINVAL for a null pointer, a bad batch, or an
 * invalid (mu, eps) (nothing is run then). */
scan_status scan_sweep_modularity(const scan_index *ix, int32_t count, const int32_t *mu,
                                  const double *eps, int32_t batch, double *q, void *stream);

scan_status scan_index_get_info(const scan_index *ix, scan_index_info *out);

/* Copies one index array to host memory (synchronous). dst_bytes must be at
 * least the array's size. SCAN_EINVAL for an array that was not kept. */
scan_status scan_index_export(const scan_index *ix, scan_array what, void *host_dst,
                              int64_t dst_bytes);

/* Device pointer and byte size of one index array (valid until the index is
 * freed; read only). */
scan_status scan_index_device_ptr(const scan_index *ix, scan_array what, const void **ptr,
                                  int64_t *bytes);

/* Phase times of a build made with SCAN_PROFILE (waits for the build to
 * finish). SCAN_EINVAL if the index was built without SCAN_PROFILE. */
scan_status scan_index_build_profile(const scan_index *ix, scan_build_profile *out);

/* Frees the index after the work enqueued on its stream completes.
 * NULL is a no-op. */
void scan_index_free(scan_index *ix);

/* ---- Serving: continuous batching of (mu, eps) queries ----------------
 * A server keeps one index resident and answers GS*-Query requests (Section
 * 4.2) submitted from any host thread. Its device memory is split into
 * max_slots / max_batch batch buffers of max_batch query slots each (fewer if
 * memory_budget holds fewer slots: each takes about 9*n bytes). A launcher
 * thread starts a device batch of up to max_batch queued requests whenever a
 * buffer is free; requests that arrive meanwhile queue and join the next
 * batch, so several batches run at once on their own streams. A completer
 * thread copies each finished result to the caller's host array. Every
 * result is identical to scan_query's for the same (mu, eps).
 * The index must outlive the server and stay unmodified; create waits for
 * the index's stream. */
typedef struct {
  int32_t max_slots;        /* query slots over all batch buffers (>= 1)      */
  int32_t max_batch;        /* queries per device batch (1..1024)             */
  int64_t memory_budget;    /* device bytes for query workspaces + outputs    */
  int32_t use_graph;        /* 1: replay a captured HIP graph per batch       */
} scan_server_opts;

typedef struct scan_server scan_server;

/* Errors: SCAN_EINVAL (bad opts), SCAN_ENOMEM (budget below one slot or an
 * allocation failed), SCAN_EDEVICE (stream, event or graph set-up failed). */
scan_status scan_server_create(const scan_index *ix, const scan_server_opts *opts,
                               scan_server **out);
/* Queues (mu, eps); the memberships (int32[n], as scan_query's) are written
 * to host `dst`, which must stay valid until the ticket completes. Pinned
 * host memory (hipHostMalloc) is written by the device directly; pageable
 * memory goes through the server's pinned staging and one host copy.
 * SCAN_EBUSY when the request queue (4 * slots, at least 64) is full: nothing
 * is queued and the caller retries later. SCAN_EINVAL for mu < 2 or NaN eps.
 * *ticket (> 0) identifies the request. */
scan_status scan_server_submit(scan_server *s, int32_t mu, double eps, int32_t *dst,
                               uint64_t *ticket);
/* As scan_server_submit; dst_on_device = 1: dst is device memory (int32[n]
 * on the index's device), written by the query kernels directly, with no
 * host copy; the result is visible to any stream once the ticket completes.
 * latency_ms (host, may be NULL) receives the time from this call until the
 * result was in dst. */
scan_status scan_server_submit_ex(scan_server *s, int32_t mu, double eps, int32_t *dst,
                                  int32_t dst_on_device, double *latency_ms, uint64_t *ticket);
/* *done = 1 once the result for ticket is in dst. A ticket that reported
 * done is forgotten (later polls also report done). */
scan_status scan_server_poll(scan_server *s, uint64_t ticket, int32_t *done);
/* Blocks until the ticket completes; returns SCAN_EDEVICE if a device batch
 * failed since the server started. */
scan_status scan_server_wait(scan_server *s, uint64_t ticket);
/* Drains outstanding requests (their results are still delivered), joins the
 * server threads, then frees everything. NULL is a no-op. */
void scan_server_destroy(scan_server *s);

/* Diagnostic: evaluates the device similarity function the build uses on
 * `count` triples (c[i], a_u[i], a_v[i]) given in HOST arrays and writes
 * out[i] (host). Synchronous, on the default stream. For checking the device
 * FP64 rounding (sqrt, division) against a host computation.
 * Errors: SCAN_EINVAL (count < 0, null pointer with count > 0, unknown kind),
 * SCAN_ENOMEM, SCAN_EDEVICE. */
scan_status scan_similarity_values(scan_sim_kind kind, int64_t count, const int64_t *c,
                                   const int64_t *a_u, const int64_t *a_v, double *out);

/* Diagnostic: the segmented sort the neighbour and core orders use, on HOST
 * arrays. Segment i is [seg_off[i], seg_off[i+1]) (seg_off[0] = 0, non-
 * decreasing); each is sorted by key descending, ties by id ascending (the
 * order of Algorithm 2's rows and segments), into keys_out / ids_out.
 * Keys must be finite doubles other than -0 (negative keys order below
 * positive ones), ids in [0, INT32_MAX). Synchronous,
 * on the default stream. Errors: SCAN_EINVAL, SCAN_ENOMEM, SCAN_EDEVICE. */
scan_status scan_segmented_sort(const int64_t *seg_off, int64_t nseg, const double *keys,
                                const int32_t *ids, double *keys_out, int32_t *ids_out);

/* Thread-local message describing the last failure on this thread. */
const char *scan_last_error(void);

/* Library version string. */
const char *scan_version(void);

#ifdef __cplusplus
}
#endif
#endif /* SCAN_MI355X_H */
