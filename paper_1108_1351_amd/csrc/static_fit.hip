// kmeans_fit_static: the two-stage fit of kmeans_fit_ex with its scratch in a
// fixed device array instead of allocated memory, for callers that cannot
// allocate (see include/kmeans.h).
#include "host_common.h"

using namespace km;

// The scratch: one fixed device array that the library holds on every GPU it
// runs on until the process ends.  In host code `scratch` names a host-side
// stand-in, not device memory; each GPU's copy has its own device address,
// which static_scratch looks up, and only that address is handed to kernels
// and copies.
static __device__ __align__(256) unsigned char scratch[KM_STATIC_SCRATCH_BYTES];

namespace {

// Device address of this GPU's copy of `scratch`, looked up once per device
// (with that device current: the calling thread's).
km_status static_scratch(void** out) {
  static std::mutex mu;
  static std::vector<void*> ptrs;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(KM_EDEVICE, "hipGetDevice failed: %s", hipGetErrorString(e));
  std::lock_guard<std::mutex> lk(mu);
  if ((int)ptrs.size() <= dev) ptrs.resize(dev + 1, nullptr);
  if (!ptrs[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(KM_EDEVICE, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
    ptrs[dev] = p;
  }
  *out = ptrs[dev];
  return KM_OK;
}

}  // namespace

extern "C" {

km_status kmeans_fit_static(const void* X, int64_t n, int32_t d, int32_t k,
                            double subset_frac, uint64_t seed, const km_options* opt,
                            float* centers_out, int32_t* labels_out, km_info* info) {
  g_err.clear();
  if (!opt) return fail(KM_EINVAL, "opt must not be NULL");
  if (opt->workspace)
    return fail(KM_EINVAL, "kmeans_fit_static takes its scratch from the library; "
                           "opt->workspace must be NULL");
  // the size query validates the arguments (its message stays on failure)
  const size_t need = kmeans_workspace_bytes(n, d, k, subset_frac, opt);
  if (need == 0) return KM_EINVAL;
  if (need > (size_t)KM_STATIC_SCRATCH_BYTES)
    return fail(KM_ENOMEM, "the problem needs %zu bytes of scratch; kmeans_fit_static holds %zu",
                need, (size_t)KM_STATIC_SCRATCH_BYTES);
  void* ws = nullptr;
  const km_status rc = static_scratch(&ws);
  if (rc != KM_OK) return rc;
  km_options o = *opt;
  o.workspace = ws;
  o.workspace_bytes = (size_t)KM_STATIC_SCRATCH_BYTES;
  return fit_impl(X, n, d, k, subset_frac, seed, &o, centers_out, labels_out, info, true);
}

}  // extern "C"
