// C ABI of the library: argument checking, errors, device memory hooks, the
// index object's accessors and the query entry points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <initializer_list>
#include <vector>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>

#include "index.h"

namespace scan {

static thread_local char g_err[512] = "";

void set_error(const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

scan_status fail(scan_status st, const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return st;
}

static std::mutex g_alloc_mu;
static scan_alloc_fn g_alloc = nullptr;
static scan_release_fn g_release = nullptr;
static void *g_alloc_ctx = nullptr;

void *dev_alloc(size_t bytes, hipStream_t stream) {
  scan_alloc_fn a;
  void *ctx;
  {
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    a = g_alloc;
    ctx = g_alloc_ctx;
  }
  if (a) return a(bytes, (void *)stream, ctx);
  void *p = nullptr;
  if (hipMallocAsync(&p, bytes, stream) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return p;
}

void dev_free(void *p, size_t bytes, hipStream_t stream) {
  if (!p) return;
  scan_release_fn r;
  void *ctx;
  {
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    r = g_release;
    ctx = g_alloc_ctx;
  }
  if (r) {
    r(p, bytes, (void *)stream, ctx);
    return;
  }
  (void)hipFreeAsync(p, stream);
}

static std::mutex g_pinned_mu;
static std::vector<PinnedBlock> g_pinned_free;

PinnedBlock pinned_take(size_t bytes) {
  size_t cap = kPinnedBlock;
  while (cap < bytes) cap <<= 1;
  {
    std::lock_guard<std::mutex> lk(g_pinned_mu);
    for (size_t i = 0; i < g_pinned_free.size(); ++i)
      if (g_pinned_free[i].cap == cap) {
        const PinnedBlock b = g_pinned_free[i];
        g_pinned_free[i] = g_pinned_free.back();
        g_pinned_free.pop_back();
        return b;
      }
  }
  PinnedBlock b;
  if (hipHostMalloc(&b.p, cap, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    return PinnedBlock{};
  }
  b.cap = cap;
  return b;
}

void pinned_give(const PinnedBlock &b) {
  if (!b.p) return;
  std::lock_guard<std::mutex> lk(g_pinned_mu);
  g_pinned_free.push_back(b);
}

void *pinned_get() { return pinned_take(kPinnedBlock).p; }

void pinned_put(void *p) { pinned_give(PinnedBlock{p, kPinnedBlock}); }

static std::mutex g_helper_mu;
static std::vector<hipStream_t> g_helper;  // kHelpers per device

hipStream_t helper_stream(int k) {
  int dev = 0;
  (void)hipGetDevice(&dev);
  std::lock_guard<std::mutex> lk(g_helper_mu);
  const size_t at = (size_t)dev * kHelpers + (size_t)k;
  if (g_helper.size() <= at) g_helper.resize((size_t)(dev + 1) * kHelpers, nullptr);
  if (!g_helper[at] && hipStreamCreateWithFlags(&g_helper[at], hipStreamNonBlocking) != hipSuccess) {
    (void)hipGetLastError();
    g_helper[at] = nullptr;
  }
  return g_helper[at];
}

scan_status stream_wait(hipStream_t waiter, hipStream_t signaller) {
  if (waiter == signaller) return SCAN_OK;
  hipEvent_t e;
  SCAN_HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  hipError_t r = hipEventRecord(e, signaller);
  if (r == hipSuccess) r = hipStreamWaitEvent(waiter, e, 0);
  (void)hipEventDestroy(e);
  if (r != hipSuccess) return fail(SCAN_EDEVICE, "stream ordering failed: %s", hipGetErrorString(r));
  return SCAN_OK;
}

}  // namespace scan

using namespace scan;

static const int64_t kArrayElem[] = {8, 4, 8, 8, 4, 8, 8, 4};

static scan_status array_of(const scan_index *ix, scan_array what, const void **p, int64_t *bytes) {
  switch (what) {
    case SCAN_ARR_OFFSETS: *p = ix->off; *bytes = (ix->n + 1) * 8; break;
    case SCAN_ARR_NO_IDS: *p = ix->no_ids; *bytes = ix->nnz * 4; break;
    case SCAN_ARR_NO_SIM: *p = ix->no_sim; *bytes = ix->nnz * 8; break;
    case SCAN_ARR_CO_OFF: *p = ix->co_off; *bytes = (ix->dmax + 3) * 8; break;
    case SCAN_ARR_CO_IDS: *p = ix->co_ids; *bytes = ix->nnz * 4; break;
    case SCAN_ARR_CO_THR: *p = ix->co_thr; *bytes = ix->nnz * 8; break;
    case SCAN_ARR_SIMS:
      if (!ix->sims) return fail(SCAN_EINVAL, "similarities were not kept (build with SCAN_KEEP_SIMS)");
      *p = ix->sims; *bytes = ix->nnz * 8; break;
    case SCAN_ARR_COUNTS:
      if (!ix->counts) return fail(SCAN_EINVAL, "counts were not kept (build with SCAN_KEEP_COUNTS)");
      *p = ix->counts; *bytes = ix->nnz * 4; break;
    default:
      return fail(SCAN_EINVAL, "unknown array %d", (int)what);
  }
  (void)kArrayElem;
  return SCAN_OK;
}

static scan_status check_query(const scan_index *ix, int32_t mu, double eps) {
  if (!ix) return fail(SCAN_EINVAL, "null index");
  if (mu < 2) return fail(SCAN_EINVAL, "mu must be >= 2 (got %d)", mu);
  if (std::isnan(eps)) return fail(SCAN_EINVAL, "eps is NaN");
  return SCAN_OK;
}

// Takes `count` query slots for use on stream s: a pooled slot is reusable if
// it is not busy and either its last use was on s (stream order) or its
// completion event has fired.
static scan_status acquire_slots(scan_index *ix, int count, hipStream_t s,
                                 std::vector<scan_index::PooledSlot *> &got) {
  std::lock_guard<std::mutex> lk(ix->pool_mu);
  for (auto *p : ix->pool) {
    if ((int)got.size() == count) break;
    if (p->busy) continue;
    bool ok = p->last_stream == s || !p->done || hipEventQuery(p->done) == hipSuccess;
    if (ok) {
      p->busy = true;
      got.push_back(p);
    }
  }
  while ((int)got.size() < count) {
    auto *p = new scan_index::PooledSlot();
    scan_status st = alloc_query_slot(ix, &p->slot, s);
    if (st != SCAN_OK) {
      delete p;
      for (auto *q : got) q->busy = false;
      got.clear();
      return st;
    }
    if (hipEventCreateWithFlags(&p->done, hipEventDisableTiming) != hipSuccess) p->done = nullptr;
    p->busy = true;
    ix->pool.push_back(p);
    got.push_back(p);
  }
  return SCAN_OK;
}

static void release_slots(scan_index *ix, std::vector<scan_index::PooledSlot *> &got, hipStream_t s) {
  std::lock_guard<std::mutex> lk(ix->pool_mu);
  for (auto *p : got) {
    if (p->done) (void)hipEventRecord(p->done, s);
    p->last_stream = s;
    p->busy = false;
  }
  got.clear();
}

static scan_status query_impl(const scan_index *cix, int32_t count, const int32_t *mu,
                              const double *eps, int32_t *memberships, uint8_t *is_core,
                              int32_t out_on_device, hipStream_t s) {
  scan_index *ix = const_cast<scan_index *>(cix);
  const int64_t n = ix->n;
  std::vector<scan_index::PooledSlot *> got;
  SCAN_TRY(acquire_slots(ix, count, s, got));
  std::vector<QuerySlot> slots(count);
  for (int i = 0; i < count; ++i) slots[i] = got[i]->slot;
  std::vector<int32_t *> mptr(count);
  std::vector<uint8_t *> cptr(count, nullptr);
  DevArena tmp(s);
  int32_t *dm = memberships;
  uint8_t *dc = is_core;
  scan_status st = SCAN_OK;
  if (!out_on_device) {
    st = tmp.alloc(&dm, (int64_t)count * n);
    if (st == SCAN_OK && is_core) st = tmp.alloc(&dc, (int64_t)count * n);
  }
  if (st == SCAN_OK) {
    for (int i = 0; i < count; ++i) {
      mptr[i] = dm + (int64_t)i * n;
      if (dc) cptr[i] = dc + (int64_t)i * n;
    }
    st = run_queries(ix, count, mu, eps, mptr.data(), dc ? cptr.data() : nullptr, slots.data(), s);
  }
  if (st == SCAN_OK && !out_on_device && n > 0) {
    hipError_t e = hipMemcpyAsync(memberships, dm, (size_t)count * n * 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess && is_core)
      e = hipMemcpyAsync(is_core, dc, (size_t)count * n, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) st = fail(SCAN_EDEVICE, "result copy: %s", hipGetErrorString(e));
  }
  release_slots(ix, got, s);
  return st;
}

// Zero fields take the defaults; ranges are checked by the build.
static scan_status tune_to_config(const scan_tune *t, IntersectConfig *c) {
  *c = default_config();
  if (!t) return SCAN_OK;
  if (t->flags & ~SCAN_TUNE_SEARCH_WINDOWS) return fail(SCAN_EINVAL, "unknown scan_tune.flags %d", t->flags);
  c->search_windows = (t->flags & SCAN_TUNE_SEARCH_WINDOWS) != 0;
  if (t->small_max) c->small_max = t->small_max;
  if (t->spc) c->spc = t->spc;
  if (t->wbits) c->wbits = t->wbits;
  return SCAN_OK;
}

extern "C" {

scan_status scan_set_allocator(scan_alloc_fn alloc, scan_release_fn release, void *ctx) {
  if ((alloc == nullptr) != (release == nullptr))
    return fail(SCAN_EINVAL, "alloc and release must both be set or both be NULL");
  std::lock_guard<std::mutex> lk(g_alloc_mu);
  g_alloc = alloc;
  g_release = release;
  g_alloc_ctx = ctx;
  return SCAN_OK;
}

scan_status scan_build_index(const scan_csr *g, scan_sim_kind kind, uint32_t flags, void *stream,
                             scan_index **out) {
  if (!out) return fail(SCAN_EINVAL, "null output pointer");
  *out = nullptr;
  return build_index(g, (int32_t)kind, flags, (hipStream_t)stream, default_config(), out);
}

scan_status scan_build_index_weighted(const scan_csr *g, const double *weights, uint32_t flags,
                                      void *stream, scan_index **out) {
  if (!out) return fail(SCAN_EINVAL, "null output pointer");
  *out = nullptr;
  if (!g) return fail(SCAN_EINVAL, "null graph");
  if (!weights && g->nnz > 0) return fail(SCAN_EINVAL, "null weights");
  return build_index_batch(g, 1, SCAN_SIM_WEIGHTED_COSINE, flags, (hipStream_t)stream, default_config(), out,
                           weights);
}

scan_status scan_build_index_lsh(const scan_csr *g, scan_sim_kind kind, const scan_lsh *lsh, uint32_t flags,
                                 void *stream, scan_index **out) {
  if (!out) return fail(SCAN_EINVAL, "null output pointer");
  *out = nullptr;
  if (!g || !lsh) return fail(SCAN_EINVAL, "null graph or LSH description");
  if (lsh->reserved) return fail(SCAN_EINVAL, "scan_lsh.reserved must be 0");
  const bool weighted = kind == SCAN_SIM_WEIGHTED_COSINE;
  if (weighted != (lsh->weights != nullptr) && g->nnz > 0)
    return fail(SCAN_EINVAL, "edge weights go with SCAN_SIM_WEIGHTED_COSINE and only with it");
  LshSpec spec;
  spec.samples = lsh->samples;
  spec.gauss = lsh->gauss;
  spec.perm = lsh->perm;
  return build_index_batch(g, 1, (int32_t)kind, flags, (hipStream_t)stream, default_config(), out,
                           weighted ? lsh->weights : nullptr, &spec);
}

scan_status scan_build_index_batch(const scan_csr *gs, int32_t count, scan_sim_kind kind,
                                   uint32_t flags, void *stream, scan_index **outs) {
  return build_index_batch(gs, count, (int32_t)kind, flags, (hipStream_t)stream, default_config(),
                           outs);
}

scan_status scan_build_index_ex(const scan_csr *gs, int32_t count, scan_sim_kind kind, uint32_t flags,
                                const scan_tune *tune, void *stream, scan_index **outs) {
  IntersectConfig cfg;
  SCAN_TRY(tune_to_config(tune, &cfg));
  return build_index_batch(gs, count, (int32_t)kind, flags, (hipStream_t)stream, cfg, outs);
}

scan_status scan_autotune(const scan_csr *gs, int32_t count, scan_sim_kind kind, int32_t reps,
                          void *stream, scan_tune *best, float *best_ms) {
  if (!best || count < 1 || !gs) return fail(SCAN_EINVAL, "null argument or empty batch");
  if (reps < 1 || reps > 16) return fail(SCAN_EINVAL, "reps must be in 1..16");
  const hipStream_t s = (hipStream_t)stream;
  std::vector<scan_index *> outs(count, nullptr);
  // Time of one build with cfg up to the end of the intersection (minimum
  // over reps).
  auto time_cfg = [&](const IntersectConfig &cfg, float *ms) -> scan_status {
    float bt = INFINITY;
    for (int32_t r = 0; r < reps; ++r) {
      SCAN_TRY(build_index_batch(gs, count, (int32_t)kind, SCAN_PROFILE, s, cfg, outs.data()));
      scan_build_profile prof;
      const scan_status st = scan_index_build_profile(outs[0], &prof);
      for (auto *&o : outs) {
        scan_index_free(o);
        o = nullptr;
      }
      SCAN_TRY(st);
      bt = std::min(bt, (float)(prof.prepare_ms + prof.plan_ms + prof.intersect_ms));
    }
    *ms = bt;
    return SCAN_OK;
  };
  IntersectConfig cur = default_config();
  float cur_ms;
  SCAN_TRY(time_cfg(cur, &cur_ms));
  auto sweep = [&](int32_t IntersectConfig::*field, std::initializer_list<int32_t> values) -> scan_status {
    const IntersectConfig base = cur;
    for (int32_t v : values) {
      if (base.*field == v) continue;
      IntersectConfig c = base;
      c.*field = v;
      float ms;
      SCAN_TRY(time_cfg(c, &ms));
      if (ms < 0.98f * cur_ms) {  // a clear gain only: keeps the choice stable under noise
        cur = c;
        cur_ms = ms;
      }
    }
    return SCAN_OK;
  };
  SCAN_TRY(sweep(&IntersectConfig::small_max, {32, 64, 128, 256, 512, 1024}));
  SCAN_TRY(sweep(&IntersectConfig::spc, {128, 256, 512, 768, 1024}));
  SCAN_TRY(sweep(&IntersectConfig::wbits, {17, 18, 19, 20}));
  *best = scan_tune{cur.small_max, cur.spc, cur.wbits, 0};
  if (best_ms) *best_ms = cur_ms;
  return SCAN_OK;
}

scan_status scan_query(const scan_index *ix, int32_t mu, double eps, int32_t *memberships) {
  SCAN_TRY(check_query(ix, mu, eps));
  if (!memberships && ix->n > 0) return fail(SCAN_EINVAL, "null memberships");
  return query_impl(ix, 1, &mu, &eps, memberships, nullptr, 1, ix->stream);
}

scan_status scan_query_ex(const scan_index *ix, int32_t mu, double eps, int32_t *memberships,
                          uint8_t *is_core, int32_t out_on_device, void *stream) {
  SCAN_TRY(check_query(ix, mu, eps));
  if (!memberships && ix->n > 0) return fail(SCAN_EINVAL, "null memberships");
  return query_impl(ix, 1, &mu, &eps, memberships, is_core, out_on_device, (hipStream_t)stream);
}

scan_status scan_query_noalloc(const scan_index *ix, int32_t mu, double eps, int32_t *memberships,
                               uint8_t *is_core, void *stream) {
  SCAN_TRY(check_query(ix, mu, eps));
  if (!memberships && ix->n > 0) return fail(SCAN_EINVAL, "null memberships");
  return query_noalloc(ix, mu, eps, memberships, is_core, (hipStream_t)stream);
}

scan_status scan_query_batch(const scan_index *ix, int32_t count, const int32_t *mu,
                             const double *eps, int32_t *memberships, int32_t out_on_device,
                             void *stream) {
  if (!ix) return fail(SCAN_EINVAL, "null index");
  if (count < 0) return fail(SCAN_EINVAL, "negative count");
  if (count == 0) return SCAN_OK;
  if (!mu || !eps || (!memberships && ix->n > 0)) return fail(SCAN_EINVAL, "null argument");
  for (int32_t i = 0; i < count; ++i) SCAN_TRY(check_query(ix, mu[i], eps[i]));
  return query_impl(ix, count, mu, eps, memberships, nullptr, out_on_device, (hipStream_t)stream);
}

scan_status scan_query_roles(const scan_index *ix, const int32_t *memberships, uint8_t *roles,
                             void *stream) {
  if (!ix) return fail(SCAN_EINVAL, "null index");
  if (ix->n == 0) return SCAN_OK;
  if (!memberships || !roles) return fail(SCAN_EINVAL, "null memberships or roles");
  launch_roles(ix, memberships, roles, stream ? (hipStream_t)stream : ix->stream);
  SCAN_HIP_TRY(hipGetLastError());
  return SCAN_OK;
}

scan_status scan_query_modularity(const scan_index *ix, const int32_t *memberships, double *q, void *stream) {
  if (!ix || !q) return fail(SCAN_EINVAL, "null index or q");
  if (ix->n > 0 && !memberships) return fail(SCAN_EINVAL, "null memberships");
  *q = 0.0;
  if (ix->n == 0) return SCAN_OK;
  hipStream_t s = stream ? (hipStream_t)stream : ix->stream;
  DevArena tmp(s);
  int64_t *dsum, *terms;
  SCAN_TRY(tmp.alloc(&dsum, ix->n));
  SCAN_TRY(tmp.alloc(&terms, 3));
  zero64(dsum, ix->n, s);
  zero64(terms, 3, s);
  launch_modularity_terms(ix, memberships, dsum, terms, s);
  int64_t h[3];
  SCAN_HIP_TRY(hipMemcpyAsync(h, terms, sizeof(h), hipMemcpyDeviceToHost, s));
  SCAN_HIP_TRY(hipStreamSynchronize(s));
  if (h[2]) return fail(SCAN_EINVAL, "%lld memberships outside [-1, n)", (long long)h[2]);
  *q = modularity_value(h[0], h[1], ix->nnz);
  return SCAN_OK;
}

scan_status scan_sweep_modularity(const scan_index *ix, int32_t count, const int32_t *mu, const double *eps,
                                  int32_t batch, double *q, void *stream) {
  if (!ix) return fail(SCAN_EINVAL, "null index");
  if (count < 0) return fail(SCAN_EINVAL, "negative count");
  if (count == 0) return SCAN_OK;
  if (!mu || !eps || !q) return fail(SCAN_EINVAL, "null argument");
  if (batch < 1 || batch > 256) return fail(SCAN_EINVAL, "batch %d outside 1..256", batch);
  for (int32_t i = 0; i < count; ++i) SCAN_TRY(check_query(ix, mu[i], eps[i]));
  const int64_t n = ix->n;
  if (n == 0) {
    for (int32_t i = 0; i < count; ++i) q[i] = 0.0;
    return SCAN_OK;
  }
  hipStream_t s = stream ? (hipStream_t)stream : ix->stream;
  const int32_t B = std::min(batch, count);
  DevArena tmp(s);
  int32_t *memb;
  int64_t *dsum, *terms;
  SCAN_TRY(tmp.alloc(&memb, (int64_t)B * n));
  SCAN_TRY(tmp.alloc(&dsum, n));
  SCAN_TRY(tmp.alloc(&terms, (int64_t)3 * count));
  zero64(dsum, n, s);
  zero64(terms, (int64_t)3 * count, s);
  for (int32_t i = 0; i < count; i += B) {
    const int32_t c = std::min(B, count - i);
    SCAN_TRY(query_impl(ix, c, mu + i, eps + i, memb, nullptr, 1, s));
    for (int32_t j = 0; j < c; ++j) launch_modularity_terms(ix, memb + (int64_t)j * n, dsum, terms + 3 * (int64_t)(i + j), s);
    SCAN_HIP_TRY(hipGetLastError());
  }
  std::vector<int64_t> h((size_t)3 * count);
  SCAN_HIP_TRY(hipMemcpyAsync(h.data(), terms, h.size() * sizeof(int64_t), hipMemcpyDeviceToHost, s));
  SCAN_HIP_TRY(hipStreamSynchronize(s));
  for (int32_t i = 0; i < count; ++i) q[i] = modularity_value(h[3 * i], h[3 * i + 1], ix->nnz);
  return SCAN_OK;
}

scan_status scan_index_get_info(const scan_index *ix, scan_index_info *out) {
  if (!ix || !out) return fail(SCAN_EINVAL, "null argument");
  out->n = ix->n;
  out->nnz = ix->nnz;
  out->dmax = ix->dmax;
  out->kind = ix->kind;
  out->flags = (int32_t)ix->flags;
  out->device_bytes = ix->bytes;
  return SCAN_OK;
}

scan_status scan_index_device_ptr(const scan_index *ix, scan_array what, const void **ptr,
                                  int64_t *bytes) {
  if (!ix || !ptr || !bytes) return fail(SCAN_EINVAL, "null argument");
  return array_of(ix, what, ptr, bytes);
}

scan_status scan_index_export(const scan_index *ix, scan_array what, void *host_dst,
                              int64_t dst_bytes) {
  if (!ix) return fail(SCAN_EINVAL, "null index");
  const void *p;
  int64_t bytes;
  SCAN_TRY(array_of(ix, what, &p, &bytes));
  if (bytes > 0 && !host_dst) return fail(SCAN_EINVAL, "null destination");
  if (dst_bytes < bytes) return fail(SCAN_EINVAL, "destination holds %lld bytes, need %lld", (long long)dst_bytes, (long long)bytes);
  if (bytes == 0) return SCAN_OK;
  SCAN_HIP_TRY(hipMemcpyAsync(host_dst, p, (size_t)bytes, hipMemcpyDeviceToHost, ix->stream));
  SCAN_HIP_TRY(hipStreamSynchronize(ix->stream));
  return SCAN_OK;
}

scan_status scan_index_build_profile(const scan_index *ix, scan_build_profile *out) {
  if (!ix || !out) return fail(SCAN_EINVAL, "null argument");
  if (!ix->prof || !ix->prof->ev[0]) return fail(SCAN_EINVAL, "index was built without SCAN_PROFILE");
  const auto &ev = ix->prof->ev;
  SCAN_HIP_TRY(hipEventSynchronize(ev[5]));
  float t[6] = {0, 0, 0, 0, 0, 0};
  for (int k = 1; k < 6; ++k) SCAN_HIP_TRY(hipEventElapsedTime(&t[k], ev[k - 1], ev[k]));
  float total = 0, small = 0, big = 0;
  SCAN_HIP_TRY(hipEventElapsedTime(&total, ev[0], ev[5]));
  SCAN_HIP_TRY(hipEventElapsedTime(&small, ev[6], ev[7]));
  SCAN_HIP_TRY(hipEventElapsedTime(&big, ev[8], ev[9]));
  out->total_ms = total;
  out->prepare_ms = t[1];
  out->plan_ms = t[2];
  out->intersect_ms = t[3];
  out->no_sort_ms = t[4];
  out->core_order_ms = t[5];
  out->intersect_small_ms = small;
  out->intersect_big_ms = big;
  const int32_t *pc = ix->prof->plan_counts;  // (light, chunks, -, heavy), complete at ev[5]
  out->small_owners = pc[0] + pc[3];
  out->big_chunks = pc[1];
  out->intersect_launches = ix->prof->intersect_launches;
  out->window_bits = ix->prof->window_bits;
  return SCAN_OK;
}

void scan_index_free(scan_index *ix) {
  if (!ix) return;
  {
    std::lock_guard<std::mutex> lk(ix->pool_mu);
    for (auto *p : ix->pool) {
      if (p->done) {
        (void)hipEventSynchronize(p->done);
        (void)hipEventDestroy(p->done);
      }
      free_query_slot(&p->slot, ix->stream);
      delete p;
    }
    ix->pool.clear();
  }
  index_release(ix);
  delete ix;
}

const char *scan_last_error(void) { return g_err; }

scan_status scan_similarity_values(scan_sim_kind kind, int64_t count, const int64_t *c,
                                   const int64_t *a_u, const int64_t *a_v, double *out) {
  if (count < 0) return fail(SCAN_EINVAL, "negative count");
  if (kind != SCAN_SIM_COSINE && kind != SCAN_SIM_JACCARD) return fail(SCAN_EINVAL, "unknown kind");
  if (count == 0) return SCAN_OK;
  if (!c || !a_u || !a_v || !out) return fail(SCAN_EINVAL, "null argument");
  return similarity_values((int32_t)kind, count, c, a_u, a_v, out);
}

scan_status scan_segmented_sort(const int64_t *seg_off, int64_t nseg, const double *keys,
                                const int32_t *ids, double *keys_out, int32_t *ids_out) {
  if (nseg < 0 || (nseg > 0 && !seg_off)) return fail(SCAN_EINVAL, "bad segment offsets");
  if (nseg == 0) return SCAN_OK;
  if (seg_off[0] != 0) return fail(SCAN_EINVAL, "seg_off[0] must be 0");
  for (int64_t i = 0; i < nseg; ++i)
    if (seg_off[i + 1] < seg_off[i]) return fail(SCAN_EINVAL, "segment offsets decrease at %lld", (long long)i);
  const int64_t total = seg_off[nseg];
  if (total > 0 && (!keys || !ids || !keys_out || !ids_out)) return fail(SCAN_EINVAL, "null argument");
  for (int64_t i = 0; i < total; ++i) {
    if (!std::isfinite(keys[i]) || (keys[i] == 0.0 && std::signbit(keys[i])))
      return fail(SCAN_EINVAL, "keys must be finite and not -0");
    if (ids[i] < 0 || ids[i] == INT32_MAX) return fail(SCAN_EINVAL, "ids must be in [0, INT32_MAX)");
  }
  return segmented_sort_values(seg_off, nseg, keys, ids, keys_out, ids_out);
}

const char *scan_version(void) { return "scan-mi355x 0.1 (gfx950)"; }

}  // extern "C"
