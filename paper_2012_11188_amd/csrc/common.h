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

// Sorts every segment [seg_off[i], seg_off[i+1]) of (key, id) by key
// descending, id ascending (ids must be distinct within a segment). Reads
// key_in/id_in, writes key_out/id_out (may not alias). Waits once for the
// segment class sizes (they size the grids).
scan_status segmented_sort(const int64_t *seg_off, int64_t nseg, int64_t total,
                           const double *key_in, const int32_t *id_in, double *key_out,
                           int32_t *id_out, hipStream_t s);
// The same on host arrays, synchronous (diagnostic entry point).
scan_status segmented_sort_values(const int64_t *seg_off, int64_t nseg, const double *keys,
                                  const int32_t *ids, double *keys_out, int32_t *ids_out);

}  // namespace scan
