// Host-side utilities shared by the C ABI's translation units (driver.hip,
// serve.hip): error messages, device queries, the stream-ordered workspace pool.
#pragma once
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/kmeans.h"
#include "km_internal.h"

namespace km {

inline thread_local std::string g_err;

inline km_status fail(km_status st, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
inline km_status fail(km_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

#define HIP_TRY(call)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess) {                                                             \
      rc = fail(KM_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_));             \
      goto done;                                                                        \
    }                                                                                   \
  } while (0)

inline double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

inline int device_cus() {
  static std::mutex mu;
  static std::vector<int> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  std::lock_guard<std::mutex> lk(mu);
  if ((int)cache.size() <= dev) cache.resize(dev + 1, 0);
  if (!cache[dev]) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        v <= 0)
      v = 256;
    cache[dev] = v;
  }
  return cache[dev];
}

inline size_t device_lds_limit() {
  static std::mutex mu;
  static std::vector<size_t> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 65536;
  std::lock_guard<std::mutex> lk(mu);
  if ((int)cache.size() <= dev) cache.resize(dev + 1, 0);
  if (!cache[dev]) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess ||
        v <= 0)
      v = 65536;
    cache[dev] = (size_t)v;
  }
  // leave room for the kernels' static LDS
  return cache[dev] > 2048 ? cache[dev] - 2048 : cache[dev];
}

inline int64_t subset_size(int64_t n, int32_t k, double f) {
  int64_t m = (int64_t)std::floor(f * (double)n + 0.5);
  return std::min<int64_t>(n, std::max<int64_t>(k, m));
}

// Sub-allocations of one device block, 256-byte aligned.
struct Carver {
  size_t off = 0;
  template <typename T>
  size_t take(size_t count) {
    size_t o = off;
    off += (count * sizeof(T) + 255) / 256 * 256;
    return o;
  }
};

template <typename T>
inline T* at(void* base, size_t off) {
  return reinterpret_cast<T*>(static_cast<unsigned char*>(base) + off);
}

inline bool valid_common(int64_t n, int32_t d, int32_t k) {
  if (n < 1) return !fail(KM_EINVAL, "n must be >= 1 (got %lld)", (long long)n);
  if (d < 1) return !fail(KM_EINVAL, "d must be >= 1 (got %d)", d);
  if (k < 1) return !fail(KM_EINVAL, "k must be >= 1 (got %d)", k);
  if (n > INT64_MAX / d) return !fail(KM_EINVAL, "n*d overflows int64");
  if ((int64_t)k * (d + 1) > (1LL << 31)) return !fail(KM_EINVAL, "k*(d+1) too large");
  return true;
}

// Per-device stream-ordered pool that keeps freed blocks for reuse, so the
// workspace of repeated calls costs no new device mapping.
inline std::mutex g_pool_mu;
inline std::vector<hipMemPool_t> g_pools;

inline hipMemPool_t device_pool() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  std::lock_guard<std::mutex> lk(g_pool_mu);
  if ((int)g_pools.size() <= dev) g_pools.resize(dev + 1, nullptr);
  if (!g_pools[dev]) {
    hipMemPoolProps props;
    memset(&props, 0, sizeof props);
    props.allocType = hipMemAllocationTypePinned;
    props.location.type = hipMemLocationTypeDevice;
    props.location.id = dev;
    hipMemPool_t pool = nullptr;
    if (hipMemPoolCreate(&pool, &props) != hipSuccess) return nullptr;
    uint64_t thr = UINT64_MAX;
    (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
    g_pools[dev] = pool;
  }
  return g_pools[dev];
}

// Device memory for one call: the caller's workspace or a stream-ordered allocation.
struct DevMem {
  void* ptr = nullptr;
  bool owned = false;
  hipStream_t s = nullptr;
  km_status get(size_t bytes, void* ws, size_t ws_bytes, hipStream_t st) {
    s = st;
    if (ws) {
      if (ws_bytes < bytes)
        return fail(KM_ENOMEM, "workspace of %zu bytes is smaller than the %zu needed", ws_bytes,
                    bytes);
      ptr = ws;
      return KM_OK;
    }
    hipMemPool_t pool = device_pool();
    hipError_t e = pool ? hipMallocFromPoolAsync(&ptr, std::max<size_t>(bytes, 256), pool, st)
                        : hipMallocAsync(&ptr, std::max<size_t>(bytes, 256), st);
    if (e != hipSuccess) {
      ptr = nullptr;
      return fail(KM_ENOMEM, "device allocation of %zu bytes failed: %s", bytes,
                  hipGetErrorString(e));
    }
    owned = true;
    return KM_OK;
  }
  // Frees (stream-ordered) what get() allocated.
  void release() {
    if (owned && ptr) (void)hipFreeAsync(ptr, s);
    ptr = nullptr;
    owned = false;
  }
  ~DevMem() { release(); }
};

// The two-stage fit behind kmeans_fit_ex (driver.hip).  noalloc: the device
// memory is opt->workspace and the call creates no pinned buffer or event.
km_status fit_impl(const void* X, int64_t n, int32_t d, int32_t k, double subset_frac,
                   uint64_t seed, const km_options* opt, float* centers_out, int32_t* labels_out,
                   km_info* info, bool noalloc);

}  // namespace km
