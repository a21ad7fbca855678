// Query server (placeholder: answers each request synchronously on submit).
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>
#include <unordered_map>

#include "index.h"

using namespace scan;

struct scan_server {
  const scan_index *ix;
  scan_server_opts opts;
  hipStream_t stream;
  std::mutex mu;
  uint64_t next = 1;
};

extern "C" {

scan_status scan_server_create(const scan_index *ix, const scan_server_opts *opts, scan_server **out) {
  if (!ix || !opts || !out) return fail(SCAN_EINVAL, "null argument");
  if (opts->max_slots < 1 || opts->max_batch < 1) return fail(SCAN_EINVAL, "bad server options");
  scan_server *s = new scan_server();
  s->ix = ix;
  s->opts = *opts;
  s->stream = nullptr;
  if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess) {
    delete s;
    return fail(SCAN_EDEVICE, "stream creation failed");
  }
  *out = s;
  return SCAN_OK;
}

scan_status scan_server_submit(scan_server *s, int32_t mu, double eps, int32_t *dst, uint64_t *ticket) {
  if (!s || !ticket || (!dst && s->ix->n > 0)) return fail(SCAN_EINVAL, "null argument");
  if (mu < 2 || std::isnan(eps)) return fail(SCAN_EINVAL, "invalid (mu, eps)");
  std::lock_guard<std::mutex> lk(s->mu);
  SCAN_TRY(scan_query_ex(s->ix, mu, eps, dst, nullptr, 0, s->stream));
  *ticket = s->next++;
  return SCAN_OK;
}

scan_status scan_server_poll(scan_server *s, uint64_t ticket, int32_t *done) {
  if (!s || !done) return fail(SCAN_EINVAL, "null argument");
  (void)ticket;
  *done = 1;
  return SCAN_OK;
}

scan_status scan_server_wait(scan_server *s, uint64_t ticket) {
  if (!s) return fail(SCAN_EINVAL, "null argument");
  (void)ticket;
  return SCAN_OK;
}

void scan_server_destroy(scan_server *s) {
  if (!s) return;
  (void)hipStreamSynchronize(s->stream);
  (void)hipStreamDestroy(s->stream);
  delete s;
}

}  // extern "C"
