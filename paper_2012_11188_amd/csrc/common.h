// Shared device/host definitions for the SCAN library (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <vector>
#include <stdint.h>

#include <string>

#include "../../include/scan.h"

namespace scan {

constexpr int kWave = 64;

// ---------------------------------------------------------------------------
// Similarity (Section 3.1 over closed neighbourhoods; Section 2.1.1 measures).
// c = |N[u] ∩ N[v]|, a_u = deg(u) + 1, a_v = deg(v) + 1. One IEEE sqrt and one
// IEEE division (cosine) or one division (Jaccard); the build compiles without
// fast-math and without FP contraction so the bits equal a host computation.
__device__ __forceinline__ double similarity(int kind, int64_t c, int64_t a_u, int64_t a_v) {
  if (kind == SCAN_SIM_COSINE) return (double)c / sqrt((double)a_u * (double)a_v);
  return (double)c / (double)(a_u + a_v - c);
}

// Order key for "similarity descending". The IEEE bits of a double, with the
// sign bit flipped for non-negative values and every bit flipped for negative
// ones, order like the values (the usual radix-sort transform); the complement
// orders the other way. Exact similarities lie in (0, 1]; SimHash estimates
// cos(pi h / k) are negative for h > k / 2, so negatives must order too.
// Sorting (key, id) ascending gives similarity descending, ties by id
// ascending.
__device__ __forceinline__ uint64_t desc_key(double s) {
  const uint64_t b = (uint64_t)__double_as_longlong(s);
  return (b >> 63) ? b : ~(b ^ 0x8000000000000000ull);
}
__device__ __forceinline__ double key_to_sim(uint64_t k) {
  return __longlong_as_double((long long)((k >> 63) ? k : ~k ^ 0x8000000000000000ull));
}
__device__ __forceinline__ bool key_less(uint64_t ka, int32_t ia, uint64_t kb, int32_t ib) {
  return ka < kb || (ka == kb && ia < ib);
}

constexpr uint64_t kPadKey = ~0ull;
constexpr int32_t kPadId = 0x7fffffff;

// ---------------------------------------------------------------------------
// Host side helpers.

void set_error(const char *fmt, ...);
scan_status fail(scan_status st, const char *fmt, ...);

// Device memory through the allocator hooks (hipMalloc by default).
void *dev_alloc(size_t bytes, hipStream_t stream);
void dev_free(void *p, size_t bytes, hipStream_t stream);

#define SCAN_HIP_TRY(expr)                                                         \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess)                                                          \
      return ::scan::fail(SCAN_EDEVICE, "%s failed: %s (%s:%d)", #expr,          \
                          hipGetErrorString(e_), __FILE__, __LINE__);              \
  } while (0)

#define SCAN_TRY(expr)               \
  do {                               \
    scan_status s_ = (expr);         \
    if (s_ != SCAN_OK) return s_;    \
  } while (0)

// A scoped group of device allocations released together (stream ordered).
// Scoped device temporaries, released (stream-ordered) when the arena goes
// out of scope. Small requests are carved from chunks of kChunk bytes, so a
// build makes a handful of allocator calls rather than one per buffer (each
// call may cross into the caller's allocator hook); large requests get their
// own allocation. Offsets are 256-byte aligned.
class DevArena {
 public:
  static constexpr size_t kChunk = (size_t)32 << 20;
  static constexpr size_t kAlign = 256;
  explicit DevArena(hipStream_t s) : stream_(s) {}
  ~DevArena() { release(); }
  DevArena(const DevArena &) = delete;
  DevArena &operator=(const DevArena &) = delete;
  template <class T>
  scan_status alloc(T **p, int64_t count) {
    const size_t bytes = ((size_t)(count > 0 ? count : 1) * sizeof(T) + kAlign - 1) & ~(kAlign - 1);
    if (bytes >= kChunk / 4) {  // large: its own allocation
      void *q = dev_alloc(bytes, stream_);
      if (!q) return fail(SCAN_ENOMEM, "device allocation of %zu bytes failed", bytes);
      items_.push_back({q, bytes});
      *p = (T *)q;
      return SCAN_OK;
    }
    if (used_ + bytes > cap_) {  // new chunk
      void *q = dev_alloc(kChunk, stream_);
      if (!q) return fail(SCAN_ENOMEM, "device allocation of %zu bytes failed", kChunk);
      items_.push_back({q, kChunk});
      cur_ = (unsigned char *)q;
      used_ = 0;
      cap_ = kChunk;
    }
    *p = (T *)(cur_ + used_);
    used_ += bytes;
    return SCAN_OK;
  }
  void release() {
    for (auto &it : items_) dev_free(it.p, it.bytes, stream_);
    items_.clear();
    cur_ = nullptr;
    used_ = cap_ = 0;
  }

 private:
  struct Item {
    void *p;
    size_t bytes;
  };
  hipStream_t stream_;
  std::vector<Item> items_;
  unsigned char *cur_ = nullptr;
  size_t used_ = 0, cap_ = 0;
};

// Helper streams of the current device (k < kHelpers; default priority,
// non-blocking), created once per device, for work that may overlap the
// caller's stream inside one library call: the call forks them from its own
// stream and joins them back before returning or freeing anything the
// helper work reads. Null if a stream cannot be created.
constexpr int kHelpers = 3;
hipStream_t helper_stream(int k = 0);
// `waiter` waits for everything enqueued on `signaller` so far.
scan_status stream_wait(hipStream_t waiter, hipStream_t signaller);

// Joins `helper` into `main` when it goes out of scope (also on early
// returns), so that stream-ordered frees on `main` come after helper work.
struct JoinOnExit {
  hipStream_t main, helper;
  ~JoinOnExit() {
    if (helper && helper != main) (void)stream_wait(main, helper);
  }
};

// Grid size for grid-stride kernels.
inline unsigned grid_for(int64_t work, int block, int64_t cap = 1 << 16) {
  int64_t g = (work + block - 1) / block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

// Exclusive prefix sum of int32 counts into int64 offsets: out[0..n], out[n]
// = total. `ws` must hold scan_workspace_elems(n) int64 values.
int64_t scan_workspace_elems(int64_t n);
scan_status exclusive_scan(const int32_t *in, int64_t *out, int64_t n, int64_t *ws,
                           hipStream_t s);
scan_status exclusive_scan64(const int64_t *in, int64_t *out, int64_t n, int64_t *ws,
                             hipStream_t s);

// Pinned host memory, pooled across calls: staging for host tables sent to
// the device and for values read back while other work runs. A block holds
// at least the bytes asked for (a power of two, at least kPinnedBlock); p is
// null if pinned memory cannot be had. A block goes back to the pool only
// once every copy that uses it has completed.
constexpr size_t kPinnedBlock = 4096;
struct PinnedBlock {
  void *p = nullptr;
  size_t cap = 0;
};
PinnedBlock pinned_take(size_t bytes);
void pinned_give(const PinnedBlock &b);
// One kPinnedBlock block (null on failure) and its return.
void *pinned_get();
void pinned_put(void *p);

// A segmented sort in two steps. sort_classify enqueues, on stream s, the
// classification of the segments [seg_off[i], seg_off[i+1]) by length (the
// class lists live in `arena`, which must outlive sort_run) and a copy of the
// class sizes to pinned host memory. sort_run then waits on the host for
// those sizes (they size the grids; classified early, they are there before
// they are needed) and enqueues on s the sort of every segment by key
// descending, id ascending (ids distinct within a segment), reading
// key_in/id_in and writing key_out/id_out (no aliasing). s and the stream of
// sort_classify may differ.
struct SortClasses {
  int64_t nseg = 0;
  int32_t *lists = nullptr;
  int32_t *big_tiles_of = nullptr;
  void *stats = nullptr;       // device class sizes
  void *host = nullptr;        // pinned copy
  hipEvent_t ready = nullptr;  // recorded after the copy
  hipStream_t stream = nullptr;
  SortClasses() = default;
  SortClasses(const SortClasses &) = delete;
  SortClasses &operator=(const SortClasses &) = delete;
  ~SortClasses();
};
scan_status sort_classify(const int64_t *seg_off, int64_t nseg, DevArena &arena, hipStream_t s,
                          SortClasses &c);
scan_status sort_run(const SortClasses &c, const int64_t *seg_off, int64_t total, const double *key_in,
                     const int32_t *id_in, double *key_out, int32_t *id_out, hipStream_t s);
// Both steps on s.
scan_status segmented_sort(const int64_t *seg_off, int64_t nseg, int64_t total,
                           const double *key_in, const int32_t *id_in, double *key_out,
                           int32_t *id_out, hipStream_t s);
// The same on host arrays, synchronous (diagnostic entry point).
scan_status segmented_sort_values(const int64_t *seg_off, int64_t nseg, const double *keys,
                                  const int32_t *ids, double *keys_out, int32_t *ids_out);

}  // namespace scan
