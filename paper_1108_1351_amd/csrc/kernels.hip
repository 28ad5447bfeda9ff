// HIP kernels (gfx950) of the two-stage k-means library.
//
// Method: Salman et al., "Fast k-means algorithm clustering" (arXiv
// 1108.1351), section 2 (Algorithm).  Per Lloyd pass each point takes the
// center with the smallest squared distance (the Algorithm's "modified
// distance"), J of eq. (3) sums those distances, and each center moves to the
// average of its points.  The fast stage runs these passes on a random subset
// drawn here by a radix selection over SplitMix64 keys.
//
// Numerics.  Distances are ranked through the expansion
//   ||x - c||^2 = ||x||^2 + (||c||^2 - 2 x.c)
// evaluated in FP32 (the ||x||^2 term is common to all centers and dropped).
// A rigorous bound on the FP32 error decides whether the best center is
// certain; for the rare point where it is not, the wavefront recomputes the
// point's distances to all centers in FP64 in the direct form sum (x - c)^2,
// the exact formula of the definition.  Cluster sums are accumulated as exact
// 64-bit integer sums of rint(x * 2^F) (F chosen from max |x|), so they do not
// depend on the order of accumulation; J is summed in FP64 in a fixed order.
#include <float.h>
#include <limits.h>
#include <math.h>

#include <algorithm>
#include <type_traits>

#include "km_internal.h"

namespace km {

// ----------------------------------------------------------------------------
// SplitMix64 (Steele, Lea and Flood, OOPSLA 2014): output number i+1 of a
// generator seeded with `seed`.  This is the key of point i.
__device__ __forceinline__ uint64_t split_key(uint64_t seed, int64_t i) {
  uint64_t z = seed + (uint64_t)(i + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

template <typename T> __device__ __forceinline__ float widen(T v);
template <> __device__ __forceinline__ float widen<float>(float v) { return v; }
template <> __device__ __forceinline__ float widen<uint16_t>(uint16_t v) {
  return __uint_as_float((uint32_t)v << 16);
}

__device__ __forceinline__ int64_t shfl_i64(int64_t v, int src) {
  int lo = __shfl((int)(uint32_t)(v & 0xffffffffll), src);
  int hi = __shfl((int)(uint32_t)((uint64_t)v >> 32), src);
  return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint64_t)(uint32_t)lo);
}

__device__ __forceinline__ bool gated(const int32_t* gate) { return gate && *gate; }

// Loads that bypass this CU's cache (other blocks of the kernel wrote them).
__device__ __forceinline__ double ld_agent(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ long long ld_agent(const long long* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int32_t ld_agent(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Round to the nearest BF16 (ties to even); inputs are finite.
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}


// ============================================================================
// Sampling: the r smallest keys among `count` candidates (indices 0..count-1,
// or the indices listed in idx_arr), by 12-bit digits from the top.
// ============================================================================
__global__ void k_sel_init(SelState* st, int64_t r, int64_t count) {
  st->prefix = 0;
  st->bits = 0;
  st->need = r;
  st->bin_count = count;
  st->done = r >= count ? 1 : 0;
}

__global__ __launch_bounds__(256) void k_sel_hist(const int64_t* __restrict__ idx_arr,
                                                  int64_t count, uint64_t seed,
                                                  const SelState* __restrict__ st,
                                                  unsigned long long* __restrict__ hist) {
  if (st->done) return;
  __shared__ uint32_t h[kSelBins];
  const int bits = st->bits;
  const uint64_t prefix = st->prefix;
  const int next = min(kSelDigitBits, 64 - bits);
  const int shift = 64 - bits - next;
  const uint64_t mask = (1ull << next) - 1ull;
  for (int b = threadIdx.x; b < kSelBins; b += blockDim.x) h[b] = 0;
  __syncthreads();
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count; e += stride) {
    int64_t i = idx_arr ? idx_arr[e] : e;
    uint64_t key = split_key(seed, i);
    if (bits > 0 && (key >> (64 - bits)) != prefix) continue;
    atomicAdd(&h[(key >> shift) & mask], 1u);
  }
  __syncthreads();
  for (int b = threadIdx.x; b < kSelBins; b += blockDim.x)
    if (h[b]) atomicAdd(&hist[b], (unsigned long long)h[b]);
}

// One block of 256 threads: choose the bin holding the need-th smallest key.
__global__ __launch_bounds__(256) void k_sel_pick(SelState* __restrict__ st,
                                                  unsigned long long* __restrict__ hist) {
  if (st->done) return;
  constexpr int per = kSelBins / 256;
  __shared__ unsigned long long part[256];
  const int tid = threadIdx.x;
  unsigned long long loc = 0;
  for (int q = 0; q < per; ++q) loc += hist[tid * per + q];
  part[tid] = loc;
  __syncthreads();
  if (tid == 0) {
    const unsigned long long need = (unsigned long long)st->need;
    unsigned long long below = 0;
    int t = 0;
    while (t < 255 && below + part[t] < need) below += part[t++];
    int b = t * per;
    while (b < t * per + per - 1 && below + hist[b] < need) below += hist[b++];
    const int next = min(kSelDigitBits, 64 - st->bits);
    const unsigned long long cnt = hist[b];
    st->prefix = (st->bits == 0 ? 0ull : (st->prefix << next)) | (uint64_t)b;
    st->bits += next;
    st->need = (int64_t)(need - below);
    st->bin_count = (int64_t)cnt;
    st->done = (need - below == cnt || st->bits >= 64) ? 1 : 0;
  }
  __syncthreads();
  for (int q = 0; q < per; ++q) hist[tid * per + q] = 0ull;
}

__device__ __forceinline__ bool sel_take(uint64_t key, const SelState& st) {
  return st.bits == 0 ? true : ((key >> (64 - st.bits)) <= st.prefix);
}

__global__ __launch_bounds__(256) void k_sel_count(const int64_t* __restrict__ idx_arr,
                                                   int64_t count, uint64_t seed,
                                                   const SelState* __restrict__ st_,
                                                   int64_t* __restrict__ blk) {
  const SelState st = *st_;
  const int64_t base = (int64_t)blockIdx.x * kSelChunk;
  const int64_t end = min(base + kSelChunk, count);
  int c = 0;
  for (int64_t e = base + threadIdx.x; e < end; e += blockDim.x) {
    int64_t i = idx_arr ? idx_arr[e] : e;
    c += sel_take(split_key(seed, i), st) ? 1 : 0;
  }
  __shared__ int red[256];
  red[threadIdx.x] = c;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) blk[blockIdx.x] = red[0];
}

// Exclusive scan of a[0..nb) in place; a[nb] receives the total.  One block of 256.
__global__ __launch_bounds__(256) void k_scan_excl(int64_t* __restrict__ a, int64_t nb) {
  __shared__ int64_t part[256];
  const int tid = threadIdx.x;
  const int64_t per = (nb + 255) / 256;
  const int64_t b0 = min(nb, tid * per), b1 = min(nb, b0 + per);
  int64_t s = 0;
  for (int64_t b = b0; b < b1; ++b) s += a[b];
  part[tid] = s;
  __syncthreads();
  if (tid == 0) {
    int64_t run = 0;
    for (int t = 0; t < 256; ++t) {
      int64_t v = part[t];
      part[t] = run;
      run += v;
    }
    a[nb] = run;
  }
  __syncthreads();
  int64_t run = part[tid];
  for (int64_t b = b0; b < b1; ++b) {
    int64_t v = a[b];
    a[b] = run;
    run += v;
  }
}

// Ordered compaction: selected indices of each chunk, in index order.  256 threads.
__global__ __launch_bounds__(256) void k_sel_write(const int64_t* __restrict__ idx_arr,
                                                   int64_t count, uint64_t seed,
                                                   const SelState* __restrict__ st_,
                                                   const int64_t* __restrict__ blk, int64_t r,
                                                   int64_t* __restrict__ out) {
  const SelState st = *st_;
  const int64_t base = (int64_t)blockIdx.x * kSelChunk;
  const int64_t end = min(base + kSelChunk, count);
  int64_t off = blk[blockIdx.x];
  __shared__ int wtot[4];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int64_t e0 = base; e0 < end; e0 += 256) {
    const int64_t e = e0 + threadIdx.x;
    int64_t i = 0;
    bool take = false;
    if (e < end) {
      i = idx_arr ? idx_arr[e] : e;
      take = sel_take(split_key(seed, i), st);
    }
    const unsigned long long bal = __ballot(take);
    const int before = __popcll(bal & ((1ull << lane) - 1ull));
    if (lane == 0) wtot[wid] = __popcll(bal);
    __syncthreads();
    int woff = 0;
    for (int w = 0; w < wid; ++w) woff += wtot[w];
    const int tot = wtot[0] + wtot[1] + wtot[2] + wtot[3];
    const int64_t pos = off + woff + before;
    if (take && pos < r) out[pos] = i;
    off += tot;
    __syncthreads();
  }
}

// out[rank of key] = sel[e]: the selected indices ordered by key (keys are distinct).
__global__ __launch_bounds__(256) void k_rank(const int64_t* __restrict__ sel, int32_t k,
                                              uint64_t seed, int64_t* __restrict__ out) {
  __shared__ uint64_t kk[256];
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t mine = e < k ? split_key(seed, sel[e]) : 0ull;
  int rank = 0;
  for (int c0 = 0; c0 < k; c0 += 256) {
    __syncthreads();
    if (c0 + (int)threadIdx.x < k) kk[threadIdx.x] = split_key(seed, sel[c0 + threadIdx.x]);
    __syncthreads();
    const int lim = min(256, k - c0);
    if (e < k)
      for (int q = 0; q < lim; ++q) rank += kk[q] < mine ? 1 : 0;
  }
  if (e < k && rank < k) out[rank] = sel[e];
}

hipError_t sel_run(const int64_t* idx_arr, int64_t count, uint64_t seed, int64_t r,
                   SelState* st, unsigned long long* hist, int64_t* blk, int64_t* out,
                   hipStream_t s) {
  hipLaunchKernelGGL(k_sel_init, dim3(1), dim3(1), 0, s, st, r, count);
  const int64_t hb = std::min<int64_t>((count + 255) / 256, 4096);
  for (int level = 0; level < 6; ++level) {
    hipLaunchKernelGGL(k_sel_hist, dim3((unsigned)hb), dim3(256), 0, s, idx_arr, count, seed,
                       (const SelState*)st, hist);
    hipLaunchKernelGGL(k_sel_pick, dim3(1), dim3(256), 0, s, st, hist);
  }
  const int64_t nb = (count + kSelChunk - 1) / kSelChunk;
  hipLaunchKernelGGL(k_sel_count, dim3((unsigned)nb), dim3(256), 0, s, idx_arr, count, seed,
                     (const SelState*)st, blk);
  hipLaunchKernelGGL(k_scan_excl, dim3(1), dim3(256), 0, s, blk, nb);
  hipLaunchKernelGGL(k_sel_write, dim3((unsigned)nb), dim3(256), 0, s, idx_arr, count, seed,
                     (const SelState*)st, (const int64_t*)blk, r, out);
  return hipGetLastError();
}

hipError_t rank_by_key(const int64_t* sel, int32_t k, uint64_t seed, int64_t* out,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_rank, dim3((unsigned)((k + 255) / 256)), dim3(256), 0, s, sel, k, seed,
                     out);
  return hipGetLastError();
}

// ============================================================================
// Gathers, max |x|, center preparation, stage set-up
// ============================================================================
__device__ __forceinline__ int64_t clamp_row(int64_t i, int64_t nrows) {
  return i < 0 ? 0 : (i >= nrows ? nrows - 1 : i);
}

template <typename T>
__global__ __launch_bounds__(256) void k_gather(const T* __restrict__ X, int64_t nrows,
                                                int32_t d, const int64_t* __restrict__ idx,
                                                int64_t m, T* __restrict__ out) {
  const int64_t total = m * d, stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
    const int64_t r = e / d, t = e - r * d;
    out[e] = X[clamp_row(idx[r], nrows) * d + t];
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_centers_from_rows(const T* __restrict__ X,
                                                           int64_t nrows, int32_t d,
                                                           const int64_t* __restrict__ idx,
                                                           int32_t k, double* __restrict__ c64) {
  const int64_t total = (int64_t)k * d, stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
    const int64_t j = e / d, t = e - j * d;
    c64[e] = (double)widen<T>(X[clamp_row(idx[j], nrows) * d + t]);
  }
}

hipError_t gather_rows(const void* X, int64_t nrows, int dtype, int32_t d, const int64_t* idx,
                       int64_t m, void* out, hipStream_t s) {
  const int64_t total = m * d;
  const unsigned g = (unsigned)std::min<int64_t>((total + 255) / 256, 8192);
  if (dtype == 0)
    hipLaunchKernelGGL(k_gather<float>, dim3(g), dim3(256), 0, s, (const float*)X, nrows, d,
                       idx, m, (float*)out);
  else
    hipLaunchKernelGGL(k_gather<uint16_t>, dim3(g), dim3(256), 0, s, (const uint16_t*)X, nrows,
                       d, idx, m, (uint16_t*)out);
  return hipGetLastError();
}

hipError_t centers_from_rows(const void* X, int64_t nrows, int dtype, int32_t d,
                             const int64_t* idx, int32_t k, double* c64, hipStream_t s) {
  const int64_t total = (int64_t)k * d;
  const unsigned g = (unsigned)std::min<int64_t>((total + 255) / 256, 4096);
  if (dtype == 0)
    hipLaunchKernelGGL(k_centers_from_rows<float>, dim3(g), dim3(256), 0, s, (const float*)X,
                       nrows, d, idx, k, c64);
  else
    hipLaunchKernelGGL(k_centers_from_rows<uint16_t>, dim3(g), dim3(256), 0, s,
                       (const uint16_t*)X, nrows, d, idx, k, c64);
  return hipGetLastError();
}

__global__ void k_stage_reset(PassState* st) {
  st->maxabs_bits = 0u;
  st->xn2max_bits = 0u;
  st->qcount = 0u;
  st->ticket = 0u;
  st->dcn_bits = 0u;
  st->done = 0;
  st->reseed_j = -1;
}

// Rounding error of one BF16 entry of the screen's center copy: the stored
// value minus -2c, exactly (both fit in FP64).
__device__ __forceinline__ double bf16_err(uint16_t b, double c) {
  return (double)__uint_as_float((uint32_t)b << 16) + 2.0 * c;
}

// -2c as a sum of two BF16 values hi + lo (hi = -2c rounded, lo = the rest
// rounded); returns the error hi + lo + 2c.
__device__ __forceinline__ double bf16_split(double c, uint16_t& hi, uint16_t& lo) {
  hi = f32_to_bf16((float)(-2.0 * c));
  const double h = (double)__uint_as_float((uint32_t)hi << 16);
  lo = f32_to_bf16((float)(-2.0 * c - h));
  return h + (double)__uint_as_float((uint32_t)lo << 16) + 2.0 * c;
}

// Publishes a block's squared rounding-error norm into the running maximum
// (non-negative floats order as their bits); rounded up so that the stored
// bound is not below the exact norm.
__device__ __forceinline__ void dcn_max(PassState* st, double e2) {
  const float e = (float)(sqrt(e2) * (1.0 + 0x1p-40)) * (1.0f + 0x1p-22f);
  atomicMax(&st->dcn_bits, __float_as_uint(e));
}

// The last block of a kernel that rewrote the copy: the maximum becomes the
// bound the screen reads, and the accumulator starts over.
__device__ __forceinline__ void dcn_publish(PassState* st) {
  st->dcn = __uint_as_float(__hip_atomic_load(&st->dcn_bits, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT));
  st->dcn_bits = 0u;
}

hipError_t stage_reset(PassState* st, hipStream_t s) {
  hipLaunchKernelGGL(k_stage_reset, dim3(1), dim3(1), 0, s, st);
  return hipGetLastError();
}

// E consecutive elements of a row widened to FP32: one 16-byte load when E
// elements fill 16 bytes (the caller guarantees the alignment), else E loads.
template <typename T, int E>
__device__ __forceinline__ void load_vec(const T* __restrict__ p, bool ok, float (&v)[E]) {
  if constexpr (E * sizeof(T) == 16) {
    uint4 w = make_uint4(0u, 0u, 0u, 0u);
    if (ok) w = *reinterpret_cast<const uint4*>(p);
    const uint32_t w4[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if constexpr (sizeof(T) == 4) {
        v[u] = __uint_as_float(w4[u]);
      } else {
        v[2 * u] = __uint_as_float(w4[u] << 16);
        v[2 * u + 1] = __uint_as_float(w4[u] & 0xffff0000u);
      }
    }
  } else {
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = ok ? widen<T>(p[e]) : 0.f;
  }
}

// Elements per lane of the row-group kernels: 16 bytes when every row starts
// on a 16-byte boundary, else one.
int row_vec(int dtype, int32_t d, const void* X) {
  const int E = dtype == 0 ? 4 : 8;
  const size_t s = dtype == 0 ? 4 : 2;
  const bool aligned = ((size_t)d * s) % 16 == 0 && (reinterpret_cast<uintptr_t>(X) & 15u) == 0;
  return aligned ? E : 1;
}

// log2 of the lanes that cover one row: E*G >= d, G a power of two <= 64.
int row_glog(int32_t d, int E) {
  const int64_t need = ((int64_t)d + E - 1) / E;
  int g = 0;
  while ((1 << g) < need && g < 6) ++g;
  return g;
}

// Per stage: max |x| over all elements (NaN/Inf show as bits >= 0x7f800000) and,
// with norms, max ||x||^2 over the rows.  A group of G = 2^glog lanes covers a
// row, each lane E consecutive elements per column step, so a wave reads whole
// rows with 16-byte loads.
template <typename T, int E>
__global__ __launch_bounds__(256) void k_row_stats(const T* __restrict__ X, int64_t rows, int d,
                                                   int glog, int norms,
                                                   PassState* __restrict__ st) {
  const int G = 1 << glog;
  const int lane = threadIdx.x & 63, gi = lane >> glog, gl = lane & (G - 1);
  const int64_t wave = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int64_t step = (int64_t)gridDim.x * 4 * (64 >> glog);
  uint32_t mx = 0u;
  float xn2 = 0.f;
  for (int64_t base = wave * (64 >> glog); base < rows; base += step) {
    const int64_t r = base + gi;
    const bool valid = r < rows;
    const T* xr = X + (valid ? r : 0) * d;
    float s2 = 0.f;
    for (int c0 = gl * E; c0 < d; c0 += G * E) {
      float v[E];
      load_vec<T, E>(xr + c0, valid, v);
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const bool in = E == 1 || c0 + e < d;
        const float f = in ? v[e] : 0.f;
        mx = max(mx, __float_as_uint(f) & 0x7fffffffu);
        s2 = __builtin_fmaf(f, f, s2);
      }
    }
    if (norms) {
      for (int o = G >> 1; o > 0; o >>= 1) s2 += __shfl_xor(s2, o);
      xn2 = fmaxf(xn2, s2);
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    mx = max(mx, (uint32_t)__shfl_xor((int)mx, o));
    xn2 = fmaxf(xn2, __shfl_xor(xn2, o));
  }
  __shared__ uint32_t w[4];
  __shared__ float wn[4];
  if (lane == 0) {
    w[threadIdx.x >> 6] = mx;
    wn[threadIdx.x >> 6] = xn2;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    atomicMax(&st->maxabs_bits, max(max(w[0], w[1]), max(w[2], w[3])));
    if (norms)
      atomicMax(&st->xn2max_bits,
                __float_as_uint(fmaxf(fmaxf(wn[0], wn[1]), fmaxf(wn[2], wn[3]))));
  }
}

hipError_t row_stats(const void* X, int dtype, int64_t rows, int32_t d, bool norms,
                     PassState* st, hipStream_t s) {
  const int E = row_vec(dtype, d, X), glog = row_glog(d, E);
  const int64_t waves = (rows + (64 >> glog) - 1) / (64 >> glog);
  const unsigned g = (unsigned)std::max<int64_t>(1, std::min<int64_t>((waves + 3) / 4, 8192));
  auto go = [&](auto kern, auto* x) {
    hipLaunchKernelGGL(kern, dim3(g), dim3(256), 0, s, x, rows, d, glog, norms ? 1 : 0, st);
  };
  if (dtype == 0) {
    if (E == 4) go(k_row_stats<float, 4>, (const float*)X);
    else go(k_row_stats<float, 1>, (const float*)X);
  } else {
    if (E == 8) go(k_row_stats<uint16_t, 8>, (const uint16_t*)X);
    else go(k_row_stats<uint16_t, 1>, (const uint16_t*)X);
  }
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_zero_i64(long long* __restrict__ p, int64_t count) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count; e += stride)
    p[e] = 0;
}

hipError_t zero_i64(long long* p, int64_t count, hipStream_t s) {
  const unsigned g = (unsigned)std::max<int64_t>(1, std::min<int64_t>((count + 255) / 256, 4096));
  hipLaunchKernelGGL(k_zero_i64, dim3(g), dim3(256), 0, s, p, count);
  return hipGetLastError();
}

// FP32 working copy of the centers, ||c||^2 (FP32) and ||c|| (FP64).  One wave per center.
__global__ __launch_bounds__(64) void k_prep_centers(const double* __restrict__ c64, int32_t k,
                                                     int32_t d, float* __restrict__ cw,
                                                     float* __restrict__ cn,
                                                     double* __restrict__ cnorm) {
  const int j = blockIdx.x, lane = threadIdx.x;
  double acc = 0.0;
  for (int t = lane; t < d; t += 64) {
    const double c = c64[(int64_t)j * d + t];
    cw[(int64_t)j * d + t] = (float)c;
    acc += c * c;
  }
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
  if (lane == 0) {
    cn[j] = (float)acc;
    cnorm[j] = sqrt(acc);
  }
}

hipError_t prep_centers(const double* c64, int32_t k, int32_t d, float* cw, float* cn,
                        double* cnorm, hipStream_t s) {
  hipLaunchKernelGGL(k_prep_centers, dim3(k), dim3(64), 0, s, c64, k, d, cw, cn, cnorm);
  return hipGetLastError();
}

// ceil(log2(v)) for v >= 1
__device__ __forceinline__ int ceil_log2(int64_t v) {
  int b = 0;
  while (b < 63 && (1ll << b) < v) ++b;
  return b;
}

__global__ __launch_bounds__(256) void k_stage_begin(PassState* __restrict__ st,
                                                     int32_t max_iter, double tol, int64_t rows,
                                                     const double* __restrict__ cnorm,
                                                     int32_t k, int32_t d_, int64_t pg,
                                                     int reseed) {
  __shared__ double red[256];
  double m = 0.0;
  for (int j = threadIdx.x; j < k; j += 256) m = fmax(m, cnorm[j]);
  red[threadIdx.x] = m;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const uint32_t bits = st->maxabs_bits;
    int F = 0;
    st->nonfinite = bits >= 0x7f800000u ? 1 : 0;
    if (bits != 0u && bits < 0x7f800000u) {
      // |q| = |rint(x 2^F)| < 2^30, and rows * 2^30 stays below 2^63
      const int e = ilogbf(__uint_as_float(bits));
      F = 29 - e - max(0, ceil_log2(rows) - 33);
      F = min(100, max(-100, F));
    }
    st->F = F;
    st->scale = ldexpf(1.0f, F);
    // the FP32 sum of squares of a row is within d * 2^-24 of ||x||^2, so xm
    // bounds every row's squared norm
    const float xm = __uint_as_float(st->xn2max_bits) * (1.0f + (float)(d_ + 2) * 0x1p-23f);
    const float cm = (float)(red[0] * (1.0 + 0x1p-20)) * (1.0f + 0x1p-20f);
    // The sorted update rounds each lane's part of a point's squared distance to
    // a multiple of 2^-FJ.  Centers of later passes are averages of rows (or kept),
    // so ||x - c|| <= 2 max(sqrt(xm), cmax) for the whole stage: a part stays
    // below 2^80 units and all rows' parts below 2^96.
    int FJ = 0;
    if (pg > 0 && !st->nonfinite) {
      const float r = 2.0f * fmaxf(sqrtf(xm), cm) * (1.0f + 0x1p-20f);
      const float bound = fmaxf(r * r, 0x1p-100f);
      FJ = min(80, 96 - ceil_log2(rows)) - ilogbf(bound) - 1;
      FJ = min(600, max(-600, FJ));
    }
    st->FJ = FJ;
    // BF16 screen offset: every score ||c||^2 + B - 2 x.c stays positive, also
    // after the screen's rounding (at most 2^-7 ||x|| ||c|| from BF16 operands
    // and (d+8) 2^-24 of the magnitudes from FP32 accumulation).  Every center
    // of the stage is a starting center, an average of rows or (re-seeding) a
    // row, so ||c|| <= max(cm, sqrt(xm)) bounds them all.
    {
      const float sx = sqrtf(xm);
      const float cb = fmaxf(cm, sx * (1.0f + 0x1p-20f));
      st->B = xm + 0.04f * sx * cb + (float)(d_ + 16) * 0x1p-22f * (xm + cb * cb + 2.f * sx * cb);
    }
    st->qcount = 0u;
    st->cmax = cm;
    st->ticket = 0u;
    st->max_iter = max_iter;
    st->tol = tol;
    st->iter = 0;
    st->done = st->nonfinite ? 1 : 0;
    st->converged = 0;
    st->empty = 0;
    st->J = 0.0;
    st->shift = 0.0;
    st->uncertain = 0;
    st->pairs = 0;
    st->rows = rows;
    st->reseed = reseed;
    st->reseed_j = -1;
  }
}

hipError_t stage_begin(PassState* st, int32_t max_iter, double tol, int64_t rows,
                       const double* cnorm, int32_t k, int32_t d, int64_t pg, hipStream_t s,
                       int reseed) {
  hipLaunchKernelGGL(k_stage_begin, dim3(1), dim3(256), 0, s, st, max_iter, tol, rows, cnorm, k,
                     d, pg, reseed);
  return hipGetLastError();
}

// ============================================================================
// Assignment
// ============================================================================

// Row of X into registers, zero-padded to DMAX.
template <typename T, int DMAX>
__device__ __forceinline__ void load_row(const T* __restrict__ row, int d, bool valid,
                                         float (&x)[DMAX]) {
  if (!valid) {
#pragma unroll
    for (int t = 0; t < DMAX; ++t) x[t] = 0.f;
    return;
  }
  const bool al16 = (reinterpret_cast<uintptr_t>(row) & 15u) == 0;
  if constexpr (sizeof(T) == 4 && DMAX % 4 == 0) {
    if (d == DMAX && al16) {
#pragma unroll
      for (int t = 0; t < DMAX; t += 4) {
        const float4 v = *reinterpret_cast<const float4*>(row + t);
        x[t] = v.x; x[t + 1] = v.y; x[t + 2] = v.z; x[t + 3] = v.w;
      }
      return;
    }
  }
  if constexpr (sizeof(T) == 2 && DMAX % 8 == 0) {
    if (d == DMAX && al16) {
#pragma unroll
      for (int t = 0; t < DMAX; t += 8) {
        const uint4 v = *reinterpret_cast<const uint4*>(row + t);
        const uint32_t w4[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          x[t + 2 * q] = __uint_as_float(w4[q] << 16);
          x[t + 2 * q + 1] = __uint_as_float(w4[q] & 0xffff0000u);
        }
      }
      return;
    }
  }
#pragma unroll
  for (int t = 0; t < DMAX; ++t) x[t] = t < d ? widen<T>(row[t]) : 0.f;
}

// Scores ||c_j||^2 - 2 x.c_j for centers [0, jc) of an LDS tile; keeps the best
// two values and the best index (lowest index on equal values).
template <int DMAX, int P>
__device__ __forceinline__ void score_tile(const float* __restrict__ w,
                                           const float* __restrict__ cnl, int jc, int j0,
                                           const float (&x)[P][DMAX], float (&best)[P],
                                           float (&sec)[P], int (&bi)[P]) {
  for (int jj = 0; jj < jc; ++jj) {
    const float* wj = w + jj * DMAX;
    float s[P];
    const float c0 = cnl[jj];
#pragma unroll
    for (int p = 0; p < P; ++p) s[p] = c0;
    if constexpr (DMAX % 4 == 0) {
#pragma unroll
      for (int t = 0; t < DMAX; t += 4) {
        const float4 wv = *reinterpret_cast<const float4*>(wj + t);
#pragma unroll
        for (int p = 0; p < P; ++p) {
          s[p] = __builtin_fmaf(x[p][t], wv.x, s[p]);
          s[p] = __builtin_fmaf(x[p][t + 1], wv.y, s[p]);
          s[p] = __builtin_fmaf(x[p][t + 2], wv.z, s[p]);
          s[p] = __builtin_fmaf(x[p][t + 3], wv.w, s[p]);
        }
      }
    } else {
#pragma unroll
      for (int t = 0; t < DMAX; ++t) {
        const float wv = wj[t];
#pragma unroll
        for (int p = 0; p < P; ++p) s[p] = __builtin_fmaf(x[p][t], wv, s[p]);
      }
    }
    const int j = j0 + jj;
#pragma unroll
    for (int p = 0; p < P; ++p) {
      const float nb = fminf(best[p], s[p]);
      sec[p] = __builtin_amdgcn_fmed3f(best[p], s[p], sec[p]);
      bi[p] = s[p] < best[p] ? j : bi[p];
      best[p] = nb;
    }
  }
}

// Squared distance in FP64, direct form, plain multiply and add in index order.
template <typename T>
__device__ __forceinline__ double dist64_row(const T* __restrict__ xr,
                                             const double* __restrict__ c, int d) {
  double D = 0.0;
  int t = 0;
  // eight loads in flight, then the adds in the same order
  for (; t + 8 <= d; t += 8) {
    double cv[8], xv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      cv[u] = c[t + u];
      xv[u] = (double)widen<T>(xr[t + u]);
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const double diff = xv[u] - cv[u];
      D = D + diff * diff;
    }
  }
  for (; t < d; ++t) {
    const double diff = (double)widen<T>(xr[t]) - c[t];
    D = D + diff * diff;
  }
  return D;
}

// Every lane of the wave must call this.  Lanes with `unc` set get the index
// of the nearest center under FP64 distances (lowest index on equal values).
template <typename T>
__device__ __forceinline__ int64_t wave_fp64_fallback(bool unc, int64_t i,
                                                      const T* __restrict__ X, int d, int k,
                                                      const double* __restrict__ c64,
                                                      int& label) {
  const int lane = threadIdx.x & 63;
  unsigned long long m = __ballot(unc);
  const int64_t cnt = __popcll(m);
  while (m) {
    const int src = __ffsll((long long)m) - 1;
    m &= m - 1ull;
    const int64_t ii = shfl_i64(i, src);
    const T* xr = X + ii * d;
    double bD = INFINITY;
    int bj = INT_MAX;
    for (int j = lane; j < k; j += 64) {
      const double D = dist64_row<T>(xr, c64 + (int64_t)j * d, d);
      if (D < bD) { bD = D; bj = j; }
    }
    for (int o = 32; o > 0; o >>= 1) {
      const double oD = __shfl_xor(bD, o);
      const int oj = __shfl_xor(bj, o);
      if (oD < bD || (oD == bD && oj < bj)) { bD = oD; bj = oj; }
    }
    if (lane == src) label = bj < k ? bj : 0;  // NaN distances never yield an index
  }
  return cnt;
}

// Assignment of one tile of P*256 points against all centers (staged in LDS by
// tiles of ktile centers when `tiled`), then certification and FP64 fallback.
// When `S`/`N` are given, cluster sums are added into LDS.
template <typename T, int DMAX, int P, bool TILED>
__device__ __forceinline__ void assign_tile(
    const T* __restrict__ X, int64_t n, int d, int k, int64_t base, const float* __restrict__ cw,
    const float* __restrict__ cn, const double* __restrict__ c64, float* __restrict__ w,
    float* __restrict__ cnl, int ktile, float cmax, float scale,
    unsigned long long* __restrict__ S, int32_t* __restrict__ labels, bool wantJ, double& Jacc,
    int64_t& ucnt) {
  float x[P][DMAX];
  int64_t ip[P];
  bool valid[P];
#pragma unroll
  for (int p = 0; p < P; ++p) {
    ip[p] = base + p * 256 + threadIdx.x;
    valid[p] = ip[p] < n;
    load_row<T, DMAX>(X + (valid[p] ? ip[p] : 0) * d, d, valid[p], x[p]);
  }
  float best[P], sec[P];
  int bi[P];
#pragma unroll
  for (int p = 0; p < P; ++p) { best[p] = INFINITY; sec[p] = INFINITY; bi[p] = 0; }
  if constexpr (TILED) {
    for (int j0 = 0; j0 < k; j0 += ktile) {
      const int jc = min(ktile, k - j0);
      __syncthreads();
      for (int e = threadIdx.x; e < jc * DMAX; e += 256) {
        const int jj = e / DMAX, t = e - jj * DMAX;
        w[e] = t < d ? -2.f * cw[(int64_t)(j0 + jj) * d + t] : 0.f;
      }
      for (int jj = threadIdx.x; jj < jc; jj += 256) cnl[jj] = cn[j0 + jj];
      __syncthreads();
      score_tile<DMAX, P>(w, cnl, jc, j0, x, best, sec, bi);
    }
  } else {
    score_tile<DMAX, P>(w, cnl, k, 0, x, best, sec, bi);
  }
  // FP32 error bound of a score: (d+2) u (||c||^2 + 2 ||x|| ||c||), u = 2^-24
  const float Kd = (float)(d + 2) * 0x1p-24f * 1.001f;
#pragma unroll
  for (int p = 0; p < P; ++p) {
    float xn2 = 0.f;
#pragma unroll
    for (int t = 0; t < DMAX; ++t) xn2 = __builtin_fmaf(x[p][t], x[p][t], xn2);
    const float xn = sqrtf(xn2) * 1.0001f;
    const float E = Kd * __builtin_fmaf(2.f * xn, cmax, cmax * cmax);
    const bool unc = valid[p] && k > 1 && !((sec[p] - best[p]) > 2.f * E);
    ucnt += wave_fp64_fallback<T>(unc, ip[p], X, d, k, c64, bi[p]);
  }
#pragma unroll
  for (int p = 0; p < P; ++p) {
    if (!valid[p]) continue;
    const int l = bi[p];
    if (wantJ) {
      const double* cl = c64 + (int64_t)l * d;
      double D = 0.0;
#pragma unroll
      for (int t = 0; t < DMAX; ++t) {
        // a clamped load and a zero term past d: no branch per element, so the
        // loads of the row are in flight together
        const double cv = cl[t < d ? t : 0];
        const double diff = t < d ? (double)x[p][t] - cv : 0.0;
        D = D + diff * diff;
      }
      Jacc += D;
    }
    if (labels) labels[ip[p]] = l;
    if (S) {
#pragma unroll
      for (int t = 0; t < DMAX; ++t) {
        if (t < d) {
          const long long q = (long long)__float2int_rn(x[p][t] * scale);
          atomicAdd(&S[(int64_t)l * (d + 1) + t], (unsigned long long)q);
        }
      }
      atomicAdd(&S[(int64_t)l * (d + 1) + d], 1ull);
    }
  }
}

// Adds a block's LDS cluster sums S [k][d+1] (counts in the last column; the
// padded row also spreads rows over LDS banks) into slot row blockIdx.x %
// kSlots with 64-bit integer atomics, whose result does not depend on their
// order.
__device__ __forceinline__ void flush_sums(const unsigned long long* __restrict__ S, int k,
                                           int d, long long* __restrict__ slots) {
  unsigned long long* row = reinterpret_cast<unsigned long long*>(
      slots + (int64_t)(blockIdx.x % kSlots) * k * (d + 1));
  for (int e = threadIdx.x; e < k * (d + 1); e += blockDim.x) {
    const unsigned long long v = S[e];
    if (v) atomicAdd(&row[e], v);
  }
}

// Fixed-order block sum of J (FP64) and of the FP64-check counts (full checks
// and pair decisions; both wave-uniform), in wave order.  Up to 16 waves.
__device__ __forceinline__ void block_sum_J(double Jacc, int64_t ucnt, int64_t pcnt,
                                            double* Jpart, long long* upart,
                                            int64_t idx = -1) {
  if (idx < 0) idx = blockIdx.x;
  __shared__ double wJ[16];
  __shared__ long long wU[16], wP[16];
  const int nw = (int)(blockDim.x >> 6);  // up to 16 waves (1024 threads)
  for (int o = 32; o > 0; o >>= 1) Jacc += __shfl_xor(Jacc, o);
  if ((threadIdx.x & 63) == 0) {
    wJ[threadIdx.x >> 6] = Jacc;
    wU[threadIdx.x >> 6] = ucnt;
    wP[threadIdx.x >> 6] = pcnt;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double J = 0.0;
    long long U = 0, P = 0;
    for (int w = 0; w < nw; ++w) {
      J += wJ[w];
      U += wU[w];
      P += wP[w];
    }
    Jpart[idx] = J;
    upart[2 * idx] = U;
    upart[2 * idx + 1] = P;
  }
  __syncthreads();  // wJ/wU/wP may be reused by a following call
}

// Fused pass for small k*d: assignment, J and LDS-private cluster sums; each
// block writes its sums to row blockIdx.x of `part` ([rows][k][d+1], counts last).
template <typename T, int DMAX, int P>
__global__ __launch_bounds__(256) void k_fused(
    const T* __restrict__ X, int64_t n, int d, int k, const float* __restrict__ cw,
    const float* __restrict__ cn, const double* __restrict__ c64, const PassState* __restrict__ st,
    const int32_t* __restrict__ gate, int update, long long* __restrict__ slots,
    double* __restrict__ Jpart, long long* __restrict__ upart, int32_t* __restrict__ labels) {
  if (gated(gate)) return;
  extern __shared__ __align__(16) unsigned char smem[];
  float* w = reinterpret_cast<float*>(smem);
  float* cnl = w + (size_t)k * DMAX;
  unsigned long long* S =
      reinterpret_cast<unsigned long long*>(smem + (((size_t)k * DMAX + k) * 4 + 15) / 16 * 16);
  for (int e = threadIdx.x; e < k * DMAX; e += 256) {
    const int j = e / DMAX, t = e - j * DMAX;
    w[e] = t < d ? -2.f * cw[(int64_t)j * d + t] : 0.f;
  }
  for (int j = threadIdx.x; j < k; j += 256) cnl[j] = cn[j];
  if (update)
    for (int e = threadIdx.x; e < k * (d + 1); e += 256) S[e] = 0ull;
  __syncthreads();
  const float scale = st->scale, cmax = st->cmax;
  double Jacc = 0.0;
  int64_t ucnt = 0, pcnt = 0;
  const int64_t tile = 256 * P;
  for (int64_t base = (int64_t)blockIdx.x * tile; base < n; base += (int64_t)gridDim.x * tile)
    assign_tile<T, DMAX, P, false>(X, n, d, k, base, cw, cn, c64, w, cnl, k, cmax, scale,
                                   update ? S : nullptr, labels, true, Jacc, ucnt);
  __syncthreads();
  if (update) flush_sums(S, k, d, slots);
  block_sum_J(Jacc, ucnt, pcnt, Jpart, upart);
}

// Assignment only, centers streamed through LDS by tiles; writes labels.
template <typename T, int DMAX, int P>
__global__ __launch_bounds__(256) void k_assign_tiled(
    const T* __restrict__ X, int64_t n, int d, int k, int ktile, const float* __restrict__ cw,
    const float* __restrict__ cn, const double* __restrict__ c64, const PassState* __restrict__ st,
    const int32_t* __restrict__ gate, double* __restrict__ Jpart, long long* __restrict__ upart,
    int32_t* __restrict__ labels, int wantJ) {
  if (gated(gate)) return;
  extern __shared__ __align__(16) unsigned char smem[];
  float* w = reinterpret_cast<float*>(smem);
  float* cnl = w + (size_t)ktile * DMAX;
  const float cmax = st->cmax;
  double Jacc = 0.0;
  int64_t ucnt = 0, pcnt = 0;
  const int64_t tile = 256 * P;
  for (int64_t base = (int64_t)blockIdx.x * tile; base < n; base += (int64_t)gridDim.x * tile)
    assign_tile<T, DMAX, P, true>(X, n, d, k, base, cw, cn, c64, w, cnl, ktile, cmax, 1.f,
                                  nullptr, labels, wantJ != 0, Jacc, ucnt);
  block_sum_J(Jacc, ucnt, pcnt, Jpart, upart);
}

// Rows with d above the largest register tile: one point per thread, the row
// read from memory (L1/L2) for every center.
template <typename T>
__global__ __launch_bounds__(256) void k_assign_generic(
    const T* __restrict__ X, int64_t n, int d, int k, const float* __restrict__ cw,
    const float* __restrict__ cn, const double* __restrict__ c64, const PassState* __restrict__ st,
    const int32_t* __restrict__ gate, double* __restrict__ Jpart, long long* __restrict__ upart,
    int32_t* __restrict__ labels, int wantJ) {
  if (gated(gate)) return;
  const float cmax = st->cmax;
  const float Kd = (float)(d + 2) * 0x1p-24f * 1.001f;
  double Jacc = 0.0;
  int64_t ucnt = 0, pcnt = 0;
  for (int64_t base = (int64_t)blockIdx.x * 256; base < n; base += (int64_t)gridDim.x * 256) {
    const int64_t i = base + threadIdx.x;
    const bool valid = i < n;
    const T* xr = X + (valid ? i : 0) * d;
    float best = INFINITY, sec = INFINITY, xn2 = 0.f;
    int bi = 0;
    if (valid) {
      for (int t = 0; t < d; ++t) {
        const float v = widen<T>(xr[t]);
        xn2 = __builtin_fmaf(v, v, xn2);
      }
      for (int j = 0; j < k; ++j) {
        const float* cj = cw + (int64_t)j * d;
        float s = cn[j];
        for (int t = 0; t < d; ++t) s = __builtin_fmaf(widen<T>(xr[t]), -2.f * cj[t], s);
        const float nb = fminf(best, s);
        sec = __builtin_amdgcn_fmed3f(best, s, sec);
        bi = s < best ? j : bi;
        best = nb;
      }
    }
    const float xn = sqrtf(xn2) * 1.0001f;
    const float E = Kd * __builtin_fmaf(2.f * xn, cmax, cmax * cmax);
    const bool unc = valid && k > 1 && !((sec - best) > 2.f * E);
    ucnt += wave_fp64_fallback<T>(unc, i, X, d, k, c64, bi);
    if (valid) labels[i] = bi;
    if (valid && wantJ) {
      const double* cl = c64 + (int64_t)bi * d;
      double D = 0.0;
      for (int t = 0; t < d; ++t) {
        const double diff = (double)widen<T>(xr[t]) - cl[t];
        D = D + diff * diff;
      }
      Jacc += D;
    }
  }
  block_sum_J(Jacc, ucnt, pcnt, Jpart, upart);
}

// ============================================================================
// Cluster sums by label order, for k*d too large for LDS-private sums: a
// counting sort of the point indices by label (chunk histograms, an exclusive
// scan over (label, chunk), a scatter), then groups of lanes walk runs of
// equal labels, adding whole rows in registers with the run's center at hand.
// The sums are exact integers, so the scatter's order does not matter.
// ============================================================================

// Histogram of the labels of chunk b into cnt[j * G + b] (label-major, so an
// exclusive scan gives each chunk's first position within label j's run).
__global__ __launch_bounds__(256) void k_lab_count(const int32_t* __restrict__ labels, int64_t n,
                                                   int k, int64_t chunk, int64_t G,
                                                   long long* __restrict__ cnt,
                                                   const int32_t* __restrict__ gate) {
  if (gated(gate)) return;
  extern __shared__ uint32_t h[];
  const int64_t b = blockIdx.x, i0 = b * chunk, i1 = min(n, i0 + chunk);
  const bool lds = k <= kHistLds;
  if (lds) {
    for (int j = threadIdx.x; j < k; j += 256) h[j] = 0u;
    __syncthreads();
  }
  // labels four at a time per thread, so the loads overlap
  for (int64_t i0t = i0 + threadIdx.x; i0t < i1; i0t += 1024) {
    int jv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t i = i0t + 256 * u;
      jv[u] = i < i1 ? labels[i] : -1;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int j = jv[u];
      if ((unsigned)j >= (unsigned)k) continue;
      if (lds) atomicAdd(&h[j], 1u);
      else atomicAdd(reinterpret_cast<unsigned long long*>(&cnt[(int64_t)j * G + b]), 1ull);
    }
  }
  if (lds) {
    __syncthreads();
    for (int j = threadIdx.x; j < k; j += 256) cnt[(int64_t)j * G + b] = h[j];
  }
}

// Exclusive scan of tiles of 2048 entries in place; tile totals to tot[].
__global__ __launch_bounds__(256) void k_scan_tiles(long long* __restrict__ a, int64_t count,
                                                    long long* __restrict__ tot,
                                                    const int32_t* __restrict__ gate) {
  if (gated(gate)) return;
  __shared__ long long part[256];
  const int64_t t0 = (int64_t)blockIdx.x * 2048 + threadIdx.x * 8;
  long long v[8], run = 0;
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    v[u] = t0 + u < count ? a[t0 + u] : 0;
    run += v[u];
  }
  part[threadIdx.x] = run;
  __syncthreads();
  for (int o = 1; o < 256; o <<= 1) {  // inclusive Hillis-Steele scan of the thread sums
    const long long add = threadIdx.x >= o ? part[threadIdx.x - o] : 0;
    __syncthreads();
    part[threadIdx.x] += add;
    __syncthreads();
  }
  long long e = part[threadIdx.x] - run;
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    if (t0 + u < count) a[t0 + u] = e;
    e += v[u];
  }
  if (threadIdx.x == 255) tot[blockIdx.x] = part[255];
}

__global__ __launch_bounds__(256) void k_scan_add(long long* __restrict__ a, int64_t count,
                                                  const long long* __restrict__ tot,
                                                  const int32_t* __restrict__ gate) {
  if (gated(gate)) return;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < count) a[i] += tot[i >> 11];
}

// First position of every label's run: start[j] = off[j * G], start[k] = n.
__global__ __launch_bounds__(256) void k_run_starts(const long long* __restrict__ off, int k,
                                                    int64_t G, int64_t n,
                                                    long long* __restrict__ start,
                                                    const int32_t* __restrict__ gate) {
  if (gated(gate)) return;
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j < k) start[j] = off[(int64_t)j * G];
  if (j == k) start[k] = n;
}

// Point indices of chunk b to their places in label order.
__global__ __launch_bounds__(256) void k_lab_scatter(const int32_t* __restrict__ labels,
                                                     int64_t n, int k, int64_t chunk, int64_t G,
                                                     long long* __restrict__ off,
                                                     uint32_t* __restrict__ perm,
                                                     const int32_t* __restrict__ gate) {
  if (gated(gate)) return;
  extern __shared__ uint32_t h[];
  const int64_t b = blockIdx.x, i0 = b * chunk, i1 = min(n, i0 + chunk);
  const bool lds = k <= kHistLds;
  if (lds) {
    for (int j = threadIdx.x; j < k; j += 256) h[j] = (uint32_t)off[(int64_t)j * G + b];
    __syncthreads();
  }
  for (int64_t i = i0 + threadIdx.x; i < i1; i += 256) {
    const int j = labels[i];
    if ((unsigned)j >= (unsigned)k) continue;
    const uint64_t pos =
        lds ? (uint64_t)atomicAdd(&h[j], 1u)
            : atomicAdd(reinterpret_cast<unsigned long long*>(&off[(int64_t)j * G + b]), 1ull);
    perm[pos] = (uint32_t)i;
  }
}

// As k_lab_scatter, for k <= kScatterLdsK: each range of S points of chunk b
// is first sorted by label in LDS (histogram, exclusive scan, placement), then
// written out in that order, so the indices of one label go to consecutive
// words of perm (runs of about S/k) instead of one scattered word per point.
// LDS: base, lcnt, lst (k words each) and the sorted range (S words); S <= 2^14
// and k <= 2^18 so a sorted entry packs (label << 14) | offset.
__global__ __launch_bounds__(256) void k_lab_scatter_lds(const int32_t* __restrict__ labels,
                                                         int64_t n, int k, int64_t chunk,
                                                         int64_t G, int S,
                                                         const long long* __restrict__ off,
                                                         uint32_t* __restrict__ perm,
                                                         const int32_t* __restrict__ gate) {
  if (gated(gate)) return;
  extern __shared__ uint32_t sm[];
  uint32_t* base = sm;          // next position of label j in perm for this chunk
  uint32_t* lcnt = sm + k;      // the range's count of label j
  uint32_t* lst = sm + 2 * k;   // its first place in the sorted range (after
                                // placement: one past its last)
  uint32_t* lsrt = sm + 3 * k;  // the range in label order
  __shared__ uint32_t wtot[4];
  const int64_t b = blockIdx.x, i0 = b * chunk, i1 = min(n, i0 + chunk);
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int kc = (k + 255) / 256;  // scan entries per thread
  for (int j = t; j < k; j += 256) base[j] = (uint32_t)off[(int64_t)j * G + b];
  for (int64_t s0 = i0; s0 < i1; s0 += S) {
    const int m = (int)min((int64_t)S, i1 - s0);
    for (int j = t; j < k; j += 256) lcnt[j] = 0u;
    __syncthreads();
    // labels four at a time per thread, so the loads overlap
    for (int e0 = t; e0 < m; e0 += 1024) {
      int jv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int e = e0 + 256 * u;
        jv[u] = e < m ? labels[s0 + e] : -1;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if ((unsigned)jv[u] < (unsigned)k) atomicAdd(&lcnt[jv[u]], 1u);
    }
    __syncthreads();
    // exclusive scan of lcnt into lst; thread t takes entries [t*kc, t*kc + kc)
    uint32_t own = 0;
    for (int q = 0; q < kc; ++q) {
      const int j = t * kc + q;
      if (j < k) own += lcnt[j];
    }
    uint32_t inc = own;
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t v = __shfl_up(inc, o);
      if (lane >= o) inc += v;
    }
    if (lane == 63) wtot[wave] = inc;
    __syncthreads();
    uint32_t pre = inc - own;
    for (int w = 0; w < wave; ++w) pre += wtot[w];
    for (int q = 0; q < kc; ++q) {
      const int j = t * kc + q;
      if (j < k) {
        lst[j] = pre;
        pre += lcnt[j];
      }
    }
    __syncthreads();
    for (int e0 = t; e0 < m; e0 += 1024) {
      int jv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int e = e0 + 256 * u;
        jv[u] = e < m ? labels[s0 + e] : -1;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if ((unsigned)jv[u] < (unsigned)k) {
          const uint32_t pos = atomicAdd(&lst[jv[u]], 1u);
          lsrt[pos] = ((uint32_t)jv[u] << 14) | (uint32_t)(e0 + 256 * u);
        }
    }
    __syncthreads();
    const uint32_t tot = (wtot[0] + wtot[1]) + (wtot[2] + wtot[3]);
    for (uint32_t q = t; q < tot; q += 256) {
      const uint32_t w = lsrt[q];
      const int j = (int)(w >> 14);
      const uint32_t first = lst[j] - lcnt[j];
      perm[(uint64_t)base[j] + (q - first)] = (uint32_t)(s0 + (int64_t)(w & 0x3fffu));
    }
    __syncthreads();
    for (int j = t; j < k; j += 256) base[j] += lcnt[j];
    __syncthreads();
  }
}

// The E center coordinates of a lane (FP64).
template <int E>
__device__ __forceinline__ void load_center(const double* __restrict__ c64, int j, int d, int col,
                                            bool act, double (&c)[E]) {
#pragma unroll
  for (int e = 0; e < E; ++e) c[e] = act ? c64[(int64_t)j * d + col + e] : 0.0;
}

// A group of G = 2^glog lanes walks positions [p0, p0 + pg) of the label order
// (pg <= 2^13); lane gl owns the E dims at col = blockIdx.y*G*E + gl*E.  Per run
// of equal labels it adds rint(x * 2^F) in FP64 registers (exact integers below
// 2^43) and flushes them to slot row (group mod kSlots) with 64-bit atomics when
// the run ends.  J: each lane's part of a point's squared distance to the run's
// center, rounded to a multiple of 2^-FJ (below 2^80 units), is added as two
// 40-bit limbs (exact in FP64 over 2^13 points); the group's limbs are summed
// once at the end into jslots.  Every sum is an exact integer, so neither the
// order of the label sort nor that of the atomics changes a bit of the result.
template <typename T, int E>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5))) void k_run_sums(
    const T* __restrict__ X, int64_t n, int d, int k, int glog, int64_t pg,
    const uint32_t* __restrict__ perm, const long long* __restrict__ start,
    const double* __restrict__ c64, const PassState* __restrict__ st,
    const int32_t* __restrict__ gate, long long* __restrict__ slots,
    long long* __restrict__ jslots) {
  if (gated(gate)) return;
  const int G = 1 << glog;
  const int lane = threadIdx.x & 63, gi = lane >> glog, gl = lane & (G - 1);
  const int64_t group = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * (64 >> glog) + gi;
  // groups past the end walk nothing but still take part in the final reduction
  const int64_t p0 = min(n, group * pg), p1 = min(n, p0 + pg);
  const int col = (int)blockIdx.y * G * E + gl * E;
  const bool act = col < d;  // E > 1 divides d
  const float scale = st->scale;
  const double sj = ldexp(1.0, st->FJ);
  // the label of position p0: the largest j with start[j] <= p0 (start[k] = n > p0)
  int lo = 0, hi = k;
  while (p0 < n && hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (start[mid] <= p0) lo = mid;
    else hi = mid;
  }
  int j = lo;
  int64_t run_end = p0 < n ? start[j + 1] : n;
  double c[E], acc[E];
  load_center<E>(c64, j, d, col, act && p0 < n, c);
#pragma unroll
  for (int e = 0; e < E; ++e) acc[e] = 0.0;
  double j0 = 0.0, j1 = 0.0;  // J limbs: units of 2^-FJ and of 2^(40-FJ)
  long long cnt = 0;
  const int slot = (int)(group & (kSlots - 1));
  long long* srow = slots + (int64_t)slot * k * (d + 1);
  auto flush = [&]() {
    if (cnt == 0) return;
    long long* row = srow + (int64_t)j * (d + 1);
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const long long v = (long long)acc[e];
      if (act && v) atomicAdd(reinterpret_cast<unsigned long long*>(&row[col + e]),
                              (unsigned long long)v);
      acc[e] = 0.0;
    }
    if (blockIdx.y == 0 && gl == 0)
      atomicAdd(reinterpret_cast<unsigned long long*>(&row[d]), (unsigned long long)cnt);
    cnt = 0;
  };
  // Rows in flight per group.  Whole 16-byte pieces stay packed until added,
  // and only two are in flight, which fits the kernel in five waves per SIMD:
  // the gathered rows are served faster by more resident groups than by
  // deeper batches per group (8 rows at three waves per SIMD, or 16 at two,
  // measured slower; the 8-element form spills a few registers at five waves
  // and is still the fastest).
  constexpr bool PK = E * sizeof(T) == 16;
  constexpr int R = PK ? 2 : 8;
  // the label order's row indices of the next R positions, loaded one batch
  // ahead so that the row loads do not wait for them
  uint32_t pidx[R];
#pragma unroll
  for (int r = 0; r < R; ++r) pidx[r] = p0 + r < p1 ? perm[p0 + r] : 0u;
  for (int64_t p = p0; p < p1; p += R) {
    uint4 xw[PK ? R : 1];
    float xf[PK ? 1 : R][E];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const bool in = p + r < p1;
      const T* src = X + (int64_t)pidx[r] * d + col;
      if constexpr (PK) {
        xw[r] = make_uint4(0u, 0u, 0u, 0u);
        if (in && act) xw[r] = *reinterpret_cast<const uint4*>(src);
      } else {
        load_vec<T, E>(src, in && act, xf[r]);
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) pidx[r] = p + R + r < p1 ? perm[p + R + r] : 0u;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int64_t pr = p + r;
      if (pr < p1) {
        if (pr >= run_end) {
          flush();
          do {
            ++j;
            run_end = start[j + 1];
          } while (pr >= run_end);
          load_center<E>(c64, j, d, col, act, c);
        }
        float x[E];
        if constexpr (PK) {
          const uint32_t w4[4] = {xw[r].x, xw[r].y, xw[r].z, xw[r].w};
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            if constexpr (sizeof(T) == 4) {
              x[u] = __uint_as_float(w4[u]);
            } else {
              x[2 * u] = __uint_as_float(w4[u] << 16);
              x[2 * u + 1] = __uint_as_float(w4[u] & 0xffff0000u);
            }
          }
        } else {
#pragma unroll
          for (int e = 0; e < E; ++e) x[e] = xf[r][e];
        }
        double part = 0.0;
#pragma unroll
        for (int e = 0; e < E; ++e) {
          acc[e] += (double)rintf(x[e] * scale);
          const double df = (double)x[e] - c[e];
          part = part + df * df;
        }
        const double q = rint(part * sj);
        const double h = floor(q * 0x1p-40);
        j1 += h;
        j0 += __builtin_fma(-h, 0x1p40, q);
        ++cnt;
      }
    }
  }
  flush();
  long long l0 = (long long)j0, l1 = (long long)j1;
  for (int o = G >> 1; o > 0; o >>= 1) {
    l0 += __shfl_xor(l0, o);
    l1 += __shfl_xor(l1, o);
  }
  if (gl == 0 && (l0 | l1)) {
    l1 += l0 >> 40;
    l0 &= (1ll << 40) - 1;
    atomicAdd(reinterpret_cast<unsigned long long*>(&jslots[2 * slot]), (unsigned long long)l0);
    atomicAdd(reinterpret_cast<unsigned long long*>(&jslots[2 * slot + 1]), (unsigned long long)l1);
  }
}

// ============================================================================
// Fused pass on MFMA: x.c^T as 32x32x2 FP32 tiles
// ============================================================================
typedef float v16f __attribute__((ext_vector_type(16)));

__device__ __forceinline__ int med3_i32(int a, int b, int c) {
  return max(min(a, b), min(max(a, b), c));
}

__device__ __forceinline__ float bf16_lo(uint32_t w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bf16_hi(uint32_t w) { return __uint_as_float(w & 0xffff0000u); }

// The value x of the lane in the other half of the wave (lane ^ 32): one
// permlane32 swap, no LDS traffic.  h is the lane's half (lane >> 5).
__device__ __forceinline__ int other_half(int x, int h) {
  const auto r = __builtin_amdgcn_permlane32_swap(x, x, false, false);
  return h ? (int)r[0] : (int)r[1];
}

// v + (v of the lane in the other half): the sum over the two lane halves.
__device__ __forceinline__ double sum_halves(double v, int h) {
  const long long b = __double_as_longlong(v);
  const int lo = other_half((int)(uint32_t)b, h);
  const int hi = other_half((int)(uint32_t)((uint64_t)b >> 32), h);
  return v + __longlong_as_double((long long)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
}
__device__ __forceinline__ float sum_halves(float v, int h) {
  return v + __int_as_float(other_half(__float_as_int(v), h));
}

// Dims [hH, hH + H) of row `row` (H = KD/2) into registers.  FULL (d == KD):
// one aligned vector load per half row (the launcher checks the alignment of
// X); otherwise element loads with bounds (zero past d).
template <typename T, int KD, bool FULL>
__device__ __forceinline__ void load_half_row(const T* __restrict__ X, int64_t row, int d, int h,
                                              float (&xo)[KD / 2]) {
  constexpr int H = KD / 2;
  if constexpr (FULL) {
    const T* p = X + row * KD + h * H;
    if constexpr (sizeof(T) == 4) {
      if constexpr (H == 1) {
        xo[0] = p[0];
      } else if constexpr (H == 2) {
        const float2 v = *reinterpret_cast<const float2*>(p);
        xo[0] = v.x; xo[1] = v.y;
      } else {
#pragma unroll
        for (int q = 0; q < H; q += 4) {
          const float4 v = *reinterpret_cast<const float4*>(p + q);
          xo[q] = v.x; xo[q + 1] = v.y; xo[q + 2] = v.z; xo[q + 3] = v.w;
        }
      }
    } else {
      if constexpr (H == 1) {
        xo[0] = widen<T>(p[0]);
      } else if constexpr (H == 2) {
        const uint32_t w = *reinterpret_cast<const uint32_t*>(p);
        xo[0] = bf16_lo(w); xo[1] = bf16_hi(w);
      } else if constexpr (H == 4) {
        const uint2 w = *reinterpret_cast<const uint2*>(p);
        xo[0] = bf16_lo(w.x); xo[1] = bf16_hi(w.x); xo[2] = bf16_lo(w.y); xo[3] = bf16_hi(w.y);
      } else {
#pragma unroll
        for (int q = 0; q < H; q += 8) {
          const uint4 w = *reinterpret_cast<const uint4*>(p + q);
          const uint32_t w4[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            xo[q + 2 * u] = bf16_lo(w4[u]);
            xo[q + 2 * u + 1] = bf16_hi(w4[u]);
          }
        }
      }
    }
  } else {
    const T* p = X + row * d;
#pragma unroll
    for (int q = 0; q < H; ++q) {
      const int t = h * H + q;
      xo[q] = t < d ? widen<T>(p[t]) : 0.f;
    }
  }
}

// Whether the whole-row kernels may load half rows of X as aligned vectors.
template <typename T>
inline bool full_rows_ok(int kd, int d, const void* X) {
  const size_t vb = (size_t)(kd / 2) * sizeof(T), al = vb < 16 ? vb : 16;
  return kd == d && (reinterpret_cast<uintptr_t>(X) % al) == 0;
}

// Dims [h*H, h*H + H) of a row into registers; zero beyond d and for invalid rows.
template <typename T, int H>
__device__ __forceinline__ void load_half(const T* __restrict__ row, int d, int h, bool valid,
                                          float (&x)[H]) {
  const int t0 = h * H;
#pragma unroll
  for (int q = 0; q < H; ++q) x[q] = 0.f;
  if (!valid) return;
  const T* p = row + t0;
  const bool full = t0 + H <= d;
  const uintptr_t ad = reinterpret_cast<uintptr_t>(p);
  if constexpr (sizeof(T) == 4 && H % 4 == 0) {
    if (full && (ad & 15u) == 0) {
#pragma unroll
      for (int q = 0; q < H; q += 4) {
        const float4 v = *reinterpret_cast<const float4*>(p + q);
        x[q] = v.x; x[q + 1] = v.y; x[q + 2] = v.z; x[q + 3] = v.w;
      }
      return;
    }
  }
  if constexpr (sizeof(T) == 4 && H == 2) {
    if (full && (ad & 7u) == 0) {
      const float2 v = *reinterpret_cast<const float2*>(p);
      x[0] = v.x; x[1] = v.y;
      return;
    }
  }
  if constexpr (sizeof(T) == 2 && H % 8 == 0) {
    if (full && (ad & 15u) == 0) {
#pragma unroll
      for (int q = 0; q < H; q += 8) {
        const uint4 v = *reinterpret_cast<const uint4*>(p + q);
        const uint32_t w4[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          x[q + 2 * u] = __uint_as_float(w4[u] << 16);
          x[q + 2 * u + 1] = __uint_as_float(w4[u] & 0xffff0000u);
        }
      }
      return;
    }
  }
#pragma unroll
  for (int q = 0; q < H; ++q)
    if (t0 + q < d) x[q] = widen<T>(p[q]);
}

// FP64 check of the uncertain points of a 32-point MFMA tile.  Every lane of
// the wave calls this; point p's row sits in registers x of lanes p (dims
// [0, H)) and p + 32 (dims [H, 2H)), the FP64 centers in LDS (row stride d+1,
// or `stride`).
// Each lane takes centers lane, lane + 64, ...; the wave then reduces (D, j)
// to the smallest D, lowest j on ties.  The squared distance is the plain
// direct form summed over t = 0..d-1.
template <int H>
__device__ __forceinline__ int64_t mfma_fp64_check(bool unc, const float (&x)[H], int d, int k,
                                                   const double* __restrict__ cs, int& label,
                                                   int stride = -1) {
  if (stride < 0) stride = d + 1;
  const int lane = threadIdx.x & 63;
  unsigned long long m = __ballot(unc);
  const int64_t cnt = __popcll(m);
  while (m) {
    const int src = __ffsll((long long)m) - 1;
    m &= m - 1ull;
    float xv[2 * H];
#pragma unroll
    for (int q = 0; q < H; ++q) {
      xv[q] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x[q]), src));
      xv[H + q] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x[q]), src + 32));
    }
    double bD = INFINITY;
    int bj = INT_MAX;
    for (int j = lane; j < k; j += 64) {
      const double* cj = cs + (int64_t)j * stride;
      double D = 0.0;
#pragma unroll
      for (int t = 0; t < 2 * H; ++t) {
        const double cv = cj[t < d ? t : 0];
        const double diff = t < d ? (double)xv[t] - cv : 0.0;
        D = D + diff * diff;
      }
      if (D < bD) { bD = D; bj = j; }
    }
    for (int o = 32; o > 0; o >>= 1) {
      const double oD = __shfl_xor(bD, o);
      const int oj = __shfl_xor(bj, o);
      if (oD < bD || (oD == bD && oj < bj)) { bD = oD; bj = oj; }
    }
    if (lane == src) label = bj < k ? bj : 0;
  }
  return cnt;
}

// Fused pass for d <= 32 and k <= 128.  A wave takes 32 points at a time; for
// each tile of 32 centers one chain of 32x32x2 MFMAs gives every lane 16
// squared distances ||x||^2 + ||c||^2 - 2 x.c of its point (lane and lane^32
// hold the two halves of the 32 centers; the last K=2 step adds ||x||^2 and
// ||c||^2).  The best three are kept as integer keys (distance bits with the
// center index in the low bits, so one min/med3 ranks value and index
// together); a rigorous error bound certifies the best center, decides close
// pairs in FP64, or sends the point to the FP64 check.  Cluster sums go to LDS,
// then to the slots.  J in FP64, each lane half adding its dims' part.
// FULL: d == KD (whole half rows, no padded dims).
template <typename T, int KD, int NT, bool FULL>
__global__ __launch_bounds__(256) void k_fused_mfma(
    const T* __restrict__ X, int64_t n, int d, int k, const float* __restrict__ cw,
    const float* __restrict__ cn, const double* __restrict__ c64, const PassState* __restrict__ st,
    const int32_t* __restrict__ gate, int update, long long* __restrict__ slots,
    double* __restrict__ Jpart, long long* __restrict__ upart, int32_t* __restrict__ labels) {
  if (gated(gate)) return;
  constexpr int H = KD / 2;
  constexpr int BL = NT == 1 ? 4 : (NT == 2 ? 5 : 6);  // bits of a lane-local index (16*NT values)
  constexpr int BG = BL + 1;                            // bits of a center index (32*NT centers)
  constexpr int LM = (1 << BL) - 1, GM = (1 << BG) - 1;
  extern __shared__ __align__(16) unsigned char smem[];
  // [k][CSS] FP64 centers, zero past d (rows padded to an odd number of 16-byte
  // units, so that the lanes' reads of their own centers spread over the banks)
  constexpr int CSS = KD + 2;
  double* cs = reinterpret_cast<double*>(smem);
  unsigned long long* S = reinterpret_cast<unsigned long long*>(cs + (size_t)k * CSS);  // [k][d+1]
  const int lane = threadIdx.x & 63, h = lane >> 5, pc = lane & 31, wave = threadIdx.x >> 6;
  for (int e = threadIdx.x; e < k * KD; e += 256) {
    const int j = e / KD, t = e - j * KD;
    cs[j * CSS + t] = t < d ? c64[(int64_t)j * d + t] : 0.0;
  }
  if (update)
    for (int e = threadIdx.x; e < k * (d + 1); e += 256) S[e] = 0ull;
  const float cmax = st->cmax, scale = st->scale;
  // A operand of step q for center tile t: -2 c[32t + pc][h*H + q]; the extra
  // step pairs (1, ||c||^2) of the center with (||x||^2, 1) of the point.
  float a[NT][H], an[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int j = 32 * t + pc;
#pragma unroll
    for (int q = 0; q < H; ++q) {
      const int dim = h * H + q;
      a[t][q] = (j < k && dim < d) ? -2.f * cw[(int64_t)j * d + dim] : 0.f;
    }
    an[t] = h == 0 ? 1.f : (j < k ? cn[j] : 1e30f);
  }
  __syncthreads();
  // error bound of a distance: (KD + H + 6) u (||x|| + ||c||)^2; keys drop BG bits
  const float KE = (float)(KD + H + 6) * 0x1p-24f * 1.01f;
  const float delta = (float)(1 << BG) * 0x1p-23f * 1.01f;
  double Jacc = 0.0;
  int64_t ucnt = 0, pcnt = 0;
  const int64_t ntile = (n + 31) >> 5;
  const int64_t tstride = (int64_t)gridDim.x * 4;
  int64_t tile = (int64_t)blockIdx.x * 4 + wave;
  float xnext[H];
  // rows past n read the last row (their results are not used)
  load_half_row<T, KD, FULL>(X, min((tile << 5) + pc, n - 1), d, h, xnext);
  for (; tile < ntile; tile += tstride) {
    const int64_t i = (tile << 5) + pc;
    const bool valid = i < n;
    float x[H];
#pragma unroll
    for (int q = 0; q < H; ++q) x[q] = xnext[q];
    // rows of this wave's next tile, loaded while this one computes
    load_half_row<T, KD, FULL>(X, min(((tile + tstride) << 5) + pc, n - 1), d, h, xnext);
    float xs = 0.f;
#pragma unroll
    for (int q = 0; q < H; ++q) xs = __builtin_fmaf(x[q], x[q], xs);
    const float xn2 = sum_halves(xs, h);
    const float bx = h == 0 ? xn2 : 1.f;
    int m1 = INT_MAX, m2 = INT_MAX, m3 = INT_MAX;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      v16f acc;
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[r] = 0.f;
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(an[t], bx, acc, 0, 0, 0);
#pragma unroll
      for (int q = 0; q < H; ++q) acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a[t][q], x[q], acc, 0, 0, 0);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        // the value part drops BG bits already here: the later switch from the
        // lane-local index l to the center index j (monotone in l within a lane
        // half) then cannot reorder keys whose value parts are equal
        const int kv = (__float_as_int(acc[r]) & ~GM) | (16 * t + r);
        m3 = med3_i32(m2, kv, m3);
        m2 = med3_i32(m1, kv, m2);
        m1 = min(m1, kv);
      }
    }
    // lane-local index -> center index, then merge the two halves of the centers
    auto glob = [&](int key) {
      const int l = key & LM;
      return (key & ~GM) | (32 * (l >> 4) + 8 * ((l & 15) >> 2) + 4 * h + (l & 3));
    };
    int g1 = glob(m1), g2 = glob(m2), g3 = glob(m3);
    {
      const int ov[3] = {other_half(g1, h), other_half(g2, h), other_half(g3, h)};
#pragma unroll
      for (int u = 0; u < 3; ++u) {
        g3 = med3_i32(g2, ov[u], g3);
        g2 = med3_i32(g1, ov[u], g2);
        g1 = min(g1, ov[u]);
      }
    }
    int bi = g1 & GM;
    const int b2 = g2 & GM;
    const float v1 = __int_as_float(g1 & ~GM), v2 = __int_as_float(g2 & ~GM),
                v3 = __int_as_float(g3 & ~GM);
    // the hardware square root is within an ulp; the 1e-4 factor covers it
    const float xn = __builtin_amdgcn_sqrtf(xn2) * 1.0001f + cmax;
    const float E2 = 2.f * (KE * xn * xn + 1e-30f);
    // certain: the best beats every other center; pair: the best is one of the best two
    const bool certain = k == 1 || (bi < k && (v2 - v1) > E2 + delta * (fabsf(v2) + fabsf(v1)));
    const bool pair = valid && !certain && bi < k && b2 < k &&
                      (k == 2 || (v3 - v1) > E2 + delta * (fabsf(v3) + fabsf(v1)));
    const bool full = valid && !certain && !pair;
    if (bi >= k) bi = 0;
    auto dist64 = [&](int j) {  // FP64 direct form over this lane's dims (zero past d)
      const double* cj = cs + j * CSS + h * H;
      double p = 0.0;
#pragma unroll
      for (int q = 0; q < H; ++q) {
        const double e = (double)x[q] - cj[q];
        p = __builtin_fma(e, e, p);
      }
      return p;
    };
    double p1 = dist64(bi);
    if (__ballot(pair)) {
      // the second candidate's FP64 distance decides the pair (lowest index on ties)
      const double p2 = dist64(pair ? b2 : 0);
      const double D1 = sum_halves(p1, h), D2 = sum_halves(p2, h);
      if (pair && (D2 < D1 || (D2 == D1 && b2 < bi))) {
        bi = b2;
        p1 = p2;
      }
      pcnt += __popcll(__ballot(pair && h == 0));
    }
    if (__ballot(full)) {
      ucnt += mfma_fp64_check<H>(full && h == 0, x, d, k, cs, bi, CSS);
      const int bfull = __shfl(bi, pc);
      if (full) {
        bi = bfull < k ? bfull : 0;
        p1 = dist64(bi);
      }
    }
    if (valid) {
      // each lane half adds its dims' part of the point's distance to J
      Jacc += p1;
      if (h == 0 && labels) labels[i] = bi;
      if (update) {
        unsigned long long* Sr = S + (int64_t)bi * (d + 1);
#pragma unroll
        for (int q = 0; q < H; ++q) {
          const int dim = h * H + q;
          if (FULL || dim < d) {
            const int qv = __float2int_rn(x[q] * scale);
            atomicAdd(&Sr[dim], (unsigned long long)(long long)qv);
          }
        }
        if (h == 0) atomicAdd(&Sr[d], 1ull);
      }
    }
  }
  __syncthreads();
  if (update) flush_sums(S, k, d, slots);
  block_sum_J(Jacc, ucnt, pcnt, Jpart, upart);
}

// ============================================================================
// BF16 screen: x.c^T as 32x32x16 BF16 MFMA tiles, for d in (32, 256] or BF16 data
// ============================================================================
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));

// Dims [t0, t0+8) of a row as BF16 (zero beyond d and for invalid rows).  BF16
// data is taken as is; FP32 data is rounded to the nearest BF16.
template <typename T>
__device__ __forceinline__ v8bf load8_bf16(const T* __restrict__ row, int t0, int d, bool valid) {
  u16x8 b = {0, 0, 0, 0, 0, 0, 0, 0};
  if (valid) {
    const T* p = row + t0;
    const bool full = t0 + 8 <= d;
    if constexpr (sizeof(T) == 2) {
      if (full && (reinterpret_cast<uintptr_t>(p) & 15u) == 0) {
        return __builtin_bit_cast(v8bf, *reinterpret_cast<const uint4*>(p));
      }
#pragma unroll
      for (int e = 0; e < 8; ++e)
        if (t0 + e < d) b[e] = p[e];
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e)
        if (t0 + e < d) b[e] = f32_to_bf16(p[e]);
    }
  }
  return __builtin_bit_cast(v8bf, b);
}

// As load8_bf16, also adding the squared rounding errors of FP32 data to r2
// (BF16 data is taken exactly).
template <typename T>
__device__ __forceinline__ v8bf load8_bf16(const T* __restrict__ row, int t0, int d, bool valid,
                                           float& r2) {
  if constexpr (sizeof(T) == 2) {
    return load8_bf16<T>(row, t0, d, valid);
  } else {
    u16x8 b = {0, 0, 0, 0, 0, 0, 0, 0};
    if (valid) {
      const T* p = row + t0;
#pragma unroll
      for (int e = 0; e < 8; ++e)
        if (t0 + e < d) {
          b[e] = f32_to_bf16(p[e]);
          const float r = p[e] - __uint_as_float((uint32_t)b[e] << 16);  // exact
          r2 = __builtin_fmaf(r, r, r2);
        }
    }
    return __builtin_bit_cast(v8bf, b);
  }
}


// Among candidate centers cand[0..nc) (wave-uniform loop bound ncmax), the
// nearest to the lane's point: FP32 direct-form distances first, certified by
// their error bound; FP64 when the FP32 gap is inside it.  The point's row
// comes from X (both lane halves compute half the dims; lane h holds dims
// [h*KH, (h+1)*KH) of each 16-dim step).  Ties go to the lowest index.
template <typename T, int KS>
__device__ __forceinline__ int rerank(const T* __restrict__ xr, int d, int h, bool active,
                                      const int* cand, int nc, int ncmax,
                                      const float* __restrict__ cw,
                                      const double* __restrict__ c64, float cmax,
                                      int64_t& fp64_count) {
  float best = INFINITY, sec = INFINITY;
  int bj = INT_MAX;
  for (int q = 0; q < ncmax; ++q) {
    const int j = (active && q < nc) ? cand[q] : 0;
    const float* cj = cw + (int64_t)j * d;
    float part = 0.f;
    for (int s = 0; s < KS; ++s)
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int t = 16 * s + 8 * h + e;
        const int tc = t < d ? t : 0;
        const float cv = cj[tc], xv = widen<T>(xr[tc]);
        const float diff = t < d ? xv - cv : 0.f;
        part = __builtin_fmaf(diff, diff, part);
      }
    const float D = part + __shfl_xor(part, 32);
    if (active && q < nc) {
      if (D < best || (D == best && j < bj)) {
        sec = best;
        best = D;
        bj = j;
      } else if (D < sec) {
        sec = D;
      }
    }
  }
  // FP32 direct form: (KS*8 + 4) u D from the arithmetic, 2 sqrt(D) u ||c|| from
  // the rounded center
  const float u = 0x1p-24f * 1.01f;
  auto err = [&](float D) { return (float)(KS * 8 + 4) * u * D + 2.f * sqrtf(D) * u * cmax + 1e-30f; };
  const bool sure = nc <= 1 || (sec - best) > err(best) + err(sec);
  const bool need = active && !sure;
  if (__ballot(need)) {
    double b64 = INFINITY;
    int b64j = INT_MAX;
    for (int q = 0; q < ncmax; ++q) {
      const int j = (need && q < nc) ? cand[q] : 0;
      const double* cj = c64 + (int64_t)j * d;
      double part = 0.0;
      for (int s = 0; s < KS; ++s)
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int t = 16 * s + 8 * h + e;
          const int tc = t < d ? t : 0;
          const double cv = cj[tc], xv = (double)widen<T>(xr[tc]);
          const double diff = t < d ? xv - cv : 0.0;
          part = __builtin_fma(diff, diff, part);
        }
      const double D = part + __shfl_xor(part, 32);
      if (need && q < nc && (D < b64 || (D == b64 && j < b64j))) {
        b64 = D;
        b64j = j;
      }
    }
    if (need) bj = b64j;
    fp64_count += __popcll(__ballot(need && h == 0));
  }
  return bj;
}

// As rerank, for 16-byte aligned rows with d a multiple of 8: the point's row
// and the candidate rows are read with 16-byte loads.
template <typename T, int KS>
__device__ __forceinline__ int rerank_vec(const T* __restrict__ xr, int d,
                                          int h, bool active, const int* cand, int nc, int ncmax,
                                          const float* __restrict__ cw,
                                          const double* __restrict__ c64, float cmax,
                                          int64_t& fp64_count) {
  // BF16 data: the lane's dims 16 s + 8 h + e, read once for all candidates
  uint4 xw[KS];
  if constexpr (sizeof(T) == 2) {
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      const int t0 = 16 * s + 8 * h;
      xw[s] = t0 < d ? *reinterpret_cast<const uint4*>(xr + t0) : make_uint4(0u, 0u, 0u, 0u);
    }
  }
  // the lane's values: dims 16 s + 8 h + e
  auto xval = [&](int s, float (&v)[8]) {
    if constexpr (sizeof(T) == 2) {
      const uint4 w = xw[s];
      const uint32_t w4[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        v[2 * u] = bf16_lo(w4[u]);
        v[2 * u + 1] = bf16_hi(w4[u]);
      }
    } else {
      const int t0 = 16 * s + 8 * h;
      if (t0 < d) {
        const float4 a = *reinterpret_cast<const float4*>(xr + t0);
        const float4 b = *reinterpret_cast<const float4*>(xr + t0 + 4);
        v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
        v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = 0.f;
      }
    }
  };
  float best = INFINITY, sec = INFINITY;
  int bj = INT_MAX;
  for (int q = 0; q < ncmax; ++q) {
    const int j = (active && q < nc) ? cand[q] : 0;
    const float* cj = cw + (int64_t)j * d;
    float part = 0.f;
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      const int t0 = 16 * s + 8 * h;
      if (t0 < d) {
        float v[8];
        xval(s, v);
        const float4 a = *reinterpret_cast<const float4*>(cj + t0);
        const float4 b = *reinterpret_cast<const float4*>(cj + t0 + 4);
        const float c[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const float diff = v[e] - c[e];
          part = __builtin_fmaf(diff, diff, part);
        }
      }
    }
    const float D = part + __shfl_xor(part, 32);
    if (active && q < nc) {
      if (D < best || (D == best && j < bj)) {
        sec = best;
        best = D;
        bj = j;
      } else if (D < sec) {
        sec = D;
      }
    }
  }
  const float u = 0x1p-24f * 1.01f;
  auto err = [&](float D) { return (float)(KS * 8 + 4) * u * D + 2.f * sqrtf(D) * u * cmax + 1e-30f; };
  const bool sure = nc <= 1 || (sec - best) > err(best) + err(sec);
  const bool need = active && !sure;
  if (__ballot(need)) {
    double b64 = INFINITY;
    int b64j = INT_MAX;
    for (int q = 0; q < ncmax; ++q) {
      const int j = (need && q < nc) ? cand[q] : 0;
      const double* cj = c64 + (int64_t)j * d;
      double part = 0.0;
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        const int t0 = 16 * s + 8 * h;
        if (t0 < d) {
          float v[8];
          xval(s, v);
#pragma unroll
          for (int e2 = 0; e2 < 4; ++e2) {
            const double2 c = *reinterpret_cast<const double2*>(cj + t0 + 2 * e2);
            const double d0 = (double)v[2 * e2] - c.x, d1 = (double)v[2 * e2 + 1] - c.y;
            part = __builtin_fma(d0, d0, part);
            part = __builtin_fma(d1, d1, part);
          }
        }
      }
      const double D = part + __shfl_xor(part, 32);
      if (need && q < nc && (D < b64 || (D == b64 && j < b64j))) {
        b64 = D;
        b64j = j;
      }
    }
    if (need) bj = b64j;
    fp64_count += __popcll(__ballot(need && h == 0));
  }
  return bj;
}

// Dims [t0, t0 + 8) of a row widened to FP64 (zero beyond d).  vec: the row
// start is 16-byte aligned and d is a multiple of 8, so whole 16-byte loads
// cover the eight dims.
template <typename T>
__device__ __forceinline__ void load8_f64(const T* __restrict__ row, int t0, int d, bool vec,
                                          double (&v)[8]) {
  if (vec && t0 + 8 <= d) {
    if constexpr (sizeof(T) == 2) {
      const uint4 w = *reinterpret_cast<const uint4*>(row + t0);
      const uint32_t w4[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        v[2 * u] = (double)bf16_lo(w4[u]);
        v[2 * u + 1] = (double)bf16_hi(w4[u]);
      }
    } else {
      const float4 a = *reinterpret_cast<const float4*>(row + t0);
      const float4 b = *reinterpret_cast<const float4*>(row + t0 + 4);
      v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
      v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
    }
  } else {
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = t0 + e < d ? (double)widen<T>(row[t0 + e]) : 0.0;
  }
}

// Sum over the 64 lanes of a wave (xor butterfly).
__device__ __forceinline__ int64_t wave_sum_i64(int64_t v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// A copy of v the compiler must keep in a VGPR: with the key mask in an SGPR,
// a key is then one v_and_or_b32 (one scalar operand per VALU instruction).
__device__ __forceinline__ int opaque_vgpr(int v) {
  int r;
  asm("v_mov_b32 %0, %1" : "=v"(r) : "v"(v));
  return r;
}

// Marks v as used here (no instruction): keeps the code that computes it from
// being sunk past this point by the optimizer.
__device__ __forceinline__ void pin_here(int& v) { asm volatile("" : "+v"(v)); }

// Fused pass for d <= 16 and k <= 128 on the BF16 matrix cores (the BF16
// screen asked for at small d).  A wave takes 32 points at a time; lane half h
// holds dims [hH, hH + H) of its point (H = KD/2) as K elements 8h .. 8h + H - 1
// of the MFMA operands (the others are zero).  For each tile of 32 centers one
// 32x32x16 BF16 MFMA gives every lane 16 screened scores ||c||^2 + B + x^.c'hi
// of its point (c'hi the BF16 copy of -2c, x^ the point as BF16; lane and
// lane^32 hold the two halves of the tile's centers; the C input is
// ||c||^2 + B).  Each lane keeps its best three as integer keys; the two halves'
// keys give the best three of all.  The screen's error band (the exact
// rounding-error norms of the center copy and of the point, and the FP32
// accumulation) certifies the best center; when only the second best is within
// the band, FP64 distances decide between the two; otherwise the FP64 check
// over all centers decides.  J in FP64 (each lane half adds its dims' part) and
// the exact cluster sums as in the FP32 fused pass.  FULL: d == KD.
template <typename T, int KD, int NT, bool FULL>
__global__ __launch_bounds__(256, NT > 3 ? 2 : 3) void k_fused_screen(
    const T* __restrict__ X, int64_t n, int d, int k, const float* __restrict__ cnB, const double* __restrict__ c64,
    const PassState* __restrict__ st, const int32_t* __restrict__ gate, int update,
    long long* __restrict__ slots, double* __restrict__ Jpart, long long* __restrict__ upart,
    int32_t* __restrict__ labels) {
  if (gated(gate)) return;
  constexpr int H = KD / 2;                             // dims per lane half
  static_assert(KD >= 2 && KD <= 16, "one 16-element K step holds both halves");
  constexpr int BL = NT == 1 ? 4 : (NT == 2 ? 5 : 6);  // bits of a lane-local index (16*NT values)
  constexpr int BG = BL + 1;                            // bits of a center index (32*NT centers)
  constexpr int LM = (1 << BL) - 1, GM = (1 << BG) - 1;
  extern __shared__ __align__(16) unsigned char smem[];
  // [k][CSS] FP64 centers, zero past d (rows padded to an odd number of 16-byte
  // units, so that the lanes' reads of their own centers spread over the banks)
  constexpr int CSS = KD + 2;
  double* cs = reinterpret_cast<double*>(smem);
  unsigned long long* S = reinterpret_cast<unsigned long long*>(cs + (size_t)k * CSS);  // [k][d+1]
  const int lane = threadIdx.x & 63, h = lane >> 5, pc = lane & 31, wave = threadIdx.x >> 6;
  for (int e = threadIdx.x; e < k * KD; e += 256) {
    const int j = e / KD, t = e - j * KD;
    cs[j * CSS + t] = t < d ? c64[(int64_t)j * d + t] : 0.0;
  }
  if (update)
    for (int e = threadIdx.x; e < k * (d + 1); e += 256) S[e] = 0ull;
  __syncthreads();
  // A operand (center rows 32t + pc, dims hH .. hH + H - 1 of the BF16 copy of
  // -2c, rounded as the pass state's error norm assumes) and the C input (rows
  // 8(r/4) + 4h + r%4 of the tile) of every center tile
  v8bf a[NT];
  v16f bias[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int j = 32 * t + pc;
    u16x8 v = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int q = 0; q < H; ++q)
      v[q] = f32_to_bf16((float)(j < k ? -2.0 * cs[j * CSS + h * H + q] : 0.0));
    a[t] = __builtin_bit_cast(v8bf, v);
#pragma unroll
    for (int r = 0; r < 16; ++r) bias[t][r] = cnB[32 * t + 8 * (r >> 2) + 4 * h + (r & 3)];
  }
  const float B = st->B, cmax = st->cmax, dcn = st->dcn * 1.01f, scale = st->scale;
  const float ea = (float)(16 + 8) * 0x1p-23f * 1.01f;
  const float delta = (float)(1 << BG) * 0x1p-23f * 1.01f;
  auto load_x = [&](int64_t row, float (&xo)[H]) { load_half_row<T, KD, FULL>(X, row, d, h, xo); };
  double Jacc = 0.0;
  int64_t ucnt = 0, pcnt = 0;
  const int64_t ntile = (n + 31) >> 5;
  const int64_t tstride = (int64_t)gridDim.x * 4;
  int64_t tile = (int64_t)blockIdx.x * 4 + wave;
  float xnext[H];
  // rows past n read the last row (their results are not used)
  load_x(min((tile << 5) + pc, n - 1), xnext);
  for (; tile < ntile; tile += tstride) {
    const int64_t i = (tile << 5) + pc;
    const bool valid = i < n;
    float x[H];
#pragma unroll
    for (int q = 0; q < H; ++q) x[q] = xnext[q];
    // rows of this wave's next tile, loaded while this one computes
    load_x(min(((tile + tstride) << 5) + pc, n - 1), xnext);
    // the point as the B operand (BF16 data is exact; FP32 data rounds to
    // nearest even, two values per instruction)
    typedef float f32x2 __attribute__((ext_vector_type(2)));
    typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
    constexpr int HP = (H + 1) / 2;  // packed pairs
    uint32_t xw[4] = {0u, 0u, 0u, 0u};
    float s2 = 0.f, r2 = 0.f;
#pragma unroll
    for (int q = 0; q < HP; ++q) {
      const f32x2 pr = {x[2 * q], 2 * q + 1 < H ? x[2 * q + 1] : 0.f};
      xw[q] = __builtin_bit_cast(uint32_t, __builtin_convertvector(pr, bf16x2));
      const float lo = bf16_lo(xw[q]), hi = bf16_hi(xw[q]);
      s2 = __builtin_fmaf(lo, lo, s2);
      s2 = __builtin_fmaf(hi, hi, s2);
      if constexpr (sizeof(T) == 4) {
        const float r0 = x[2 * q] - lo;  // exact
        r2 = __builtin_fmaf(r0, r0, r2);
        if (2 * q + 1 < H) {
          const float r1 = x[2 * q + 1] - hi;
          r2 = __builtin_fmaf(r1, r1, r2);
        }
      }
    }
    // norms for the band (the hardware square root is within an ulp; the 1%
    // factor covers it)
    const float xn = __builtin_amdgcn_sqrtf(sum_halves(s2, h)) * 1.01f;
    float xr = 0.f;
    if constexpr (sizeof(T) == 4) xr = __builtin_amdgcn_sqrtf(sum_halves(r2, h)) * 1.01f;
    const v8bf xv = __builtin_bit_cast(v8bf, xw);
    int m1 = INT_MAX, m2 = INT_MAX, m3 = INT_MAX;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const v16f acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[t], xv, bias[t], 0, 0, 0);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        // the value part drops BG bits already here, so that the switch to the
        // center index below cannot reorder keys whose value parts differ
        const int kv = (__float_as_int(acc[r]) & ~GM) | (16 * t + r);
        m3 = med3_i32(m2, kv, m3);
        m2 = med3_i32(m1, kv, m2);
        m1 = min(m1, kv);
      }
    }
    auto glob = [&](int key) {
      const int l = key & LM;
      return (key & ~GM) | (32 * (l >> 4) + 8 * ((l & 15) >> 2) + 4 * h + (l & 3));
    };
    int g1 = glob(m1), g2 = glob(m2), g3 = glob(m3);
    {
      const int ov[3] = {other_half(g1, h), other_half(g2, h), other_half(g3, h)};
#pragma unroll
      for (int u = 0; u < 3; ++u) {
        g3 = med3_i32(g2, ov[u], g3);
        g2 = med3_i32(g1, ov[u], g2);
        g1 = min(g1, ov[u]);
      }
    }
    int bi = g1 & GM;
    const int b2 = g2 & GM;
    const float v1 = __int_as_float(g1 & ~GM), v2 = __int_as_float(g2 & ~GM),
                v3 = __int_as_float(g3 & ~GM);
    // two screened scores differ from their exact values by at most E2 together
    // (x.c' - x^.c'hi = x^.(c' - c'hi) + (x - x^).c', and the FP32 accumulation)
    const float E2 = 2.f * xn * dcn + 4.f * xr * cmax +
                     2.f * ea * (cmax * cmax + B + 2.f * xn * cmax);
    auto apart = [&](float lo, float hi) {
      return (hi - lo) > E2 + delta * (fabsf(hi) + fabsf(lo));
    };
    // certain: the best beats every other center; pair: the best is one of the best two
    const bool certain = k == 1 || (bi < k && apart(v1, v2));
    const bool pair = valid && !certain && bi < k && b2 < k && (k == 2 || apart(v1, v3));
    const bool full = valid && !certain && !pair;
    if (bi >= k) bi = 0;
    auto dist64 = [&](int j) {  // FP64 direct form over this lane's dims (zero past d)
      const double* cj = cs + j * CSS + h * H;
      double p = 0.0;
#pragma unroll
      for (int q = 0; q < H; ++q) {
        const double e = (double)x[q] - cj[q];
        p = __builtin_fma(e, e, p);
      }
      return p;
    };
    double p1 = dist64(bi);
    if (__ballot(pair)) {
      // the second candidate's FP64 distance decides (lowest index on ties)
      const double p2 = dist64(pair ? b2 : 0);
      const double D1p = sum_halves(p1, h), D2p = sum_halves(p2, h);
      if (pair && (D2p < D1p || (D2p == D1p && b2 < bi))) {
        bi = b2;
        p1 = p2;
      }
      pcnt += __popcll(__ballot(pair && h == 0));
    }
    if (__ballot(full)) {
      ucnt += mfma_fp64_check<H>(full && h == 0, x, d, k, cs, bi, CSS);
      const int bfull = __shfl(bi, pc);
      if (full) {
        bi = bfull < k ? bfull : 0;
        p1 = dist64(bi);
      }
    }
    if (valid) {
      // each lane half adds its dims' part of the point's distance to J
      Jacc += p1;
      if (h == 0 && labels) labels[i] = bi;
      if (update) {
        unsigned long long* Sr = S + (int64_t)bi * (d + 1);
#pragma unroll
        for (int q = 0; q < H; ++q) {
          const int dim = h * H + q;
          if (FULL || dim < d) {
            const int qv = __float2int_rn(x[q] * scale);
            atomicAdd(&Sr[dim], (unsigned long long)(long long)qv);
          }
        }
        if (h == 0) atomicAdd(&Sr[d], 1ull);
      }
    }
  }
  __syncthreads();
  if (update) flush_sums(S, k, d, slots);
  block_sum_J(Jacc, ucnt, pcnt, Jpart, upart);
}

// Whole rows of X into registers: KD values of row `row` (zero past d).
// FULL (d == KD): aligned vector loads (the launcher checks the alignment).
template <typename T, int KD, bool FULL>
__device__ __forceinline__ void load_row_full(const T* __restrict__ X, int64_t row, int d,
                                              float (&xo)[KD]) {
  if constexpr (FULL) {
    const T* p = X + row * KD;
    if constexpr (sizeof(T) == 4) {
#pragma unroll
      for (int q = 0; q < KD; q += 4) {
        const float4 v = *reinterpret_cast<const float4*>(p + q);
        xo[q] = v.x; xo[q + 1] = v.y; xo[q + 2] = v.z; xo[q + 3] = v.w;
      }
    } else if constexpr (KD == 4) {
      const uint2 w = *reinterpret_cast<const uint2*>(p);
      xo[0] = bf16_lo(w.x); xo[1] = bf16_hi(w.x); xo[2] = bf16_lo(w.y); xo[3] = bf16_hi(w.y);
    } else {
#pragma unroll
      for (int q = 0; q < KD; q += 8) {
        const uint4 w = *reinterpret_cast<const uint4*>(p + q);
        const uint32_t w4[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          xo[q + 2 * u] = bf16_lo(w4[u]);
          xo[q + 2 * u + 1] = bf16_hi(w4[u]);
        }
      }
    }
  } else {
    const T* p = X + row * d;
#pragma unroll
    for (int q = 0; q < KD; ++q) xo[q] = q < d ? widen<T>(p[q]) : 0.f;
  }
}

// Whether the paired-tile kernel may load whole rows of X as aligned vectors.
template <typename T>
inline bool full_row_ok(int kd, int d, const void* X) {
  const size_t rb = (size_t)kd * sizeof(T), al = rb < 16 ? rb : 16;
  return kd == d && (reinterpret_cast<uintptr_t>(X) % al) == 0;
}

// FP64 check of the uncertain points of a wave whose lanes hold whole rows
// (KD values, zero past d): for each such lane in turn the wave scores all
// centers (lane j takes centers j, j + 64, ...; FP64 centers in LDS with row
// stride CSS), then reduces to the smallest distance, lowest index on ties.
template <int KD, int CSS>
__device__ __forceinline__ int64_t row_fp64_check(bool unc, const float (&x)[KD], int k,
                                                  const double* __restrict__ cs, int& label) {
  const int lane = threadIdx.x & 63;
  unsigned long long m = __ballot(unc);
  const int64_t cnt = __popcll(m);
  while (m) {
    const int src = __ffsll((long long)m) - 1;
    m &= m - 1ull;
    double xv[KD];
#pragma unroll
    for (int t = 0; t < KD; ++t)
      xv[t] = (double)__int_as_float(__builtin_amdgcn_readlane(__float_as_int(x[t]), src));
    double bD = INFINITY;
    int bj = INT_MAX;
    for (int j = lane; j < k; j += 64) {
      const double* cj = cs + (int64_t)j * CSS;
      double D = 0.0;
#pragma unroll
      for (int t = 0; t < KD; ++t) {
        const double e = xv[t] - cj[t];
        D = D + e * e;
      }
      if (D < bD) { bD = D; bj = j; }
    }
    for (int o = 32; o > 0; o >>= 1) {
      const double oD = __shfl_xor(bD, o);
      const int oj = __shfl_xor(bj, o);
      if (oD < bD || (oD == bD && oj < bj)) { bD = oD; bj = oj; }
    }
    if (lane == src) label = bj < k ? bj : 0;
  }
  return cnt;
}

// The fused pass of auto precision for d <= 16 and k <= 128: a split BF16
// screen on pairs of point tiles.  Scores ||c||^2 + B + x.c' (c' = -2c) come from
// 32x32x16 BF16 MFMAs with FP32 accumulation (C input ||c||^2 + B) over three
// products per dim, c'hi x^ + c'lo x^ + c'hi xlo, where c'hi and x^ are the BF16
// roundings, c'lo = BF16(c' - c'hi) and xlo = BF16(x - x^) carry the next 8 bits
// (BF16 data: x^ = x, two products).  In lane half h the K elements list the
// terms one after the other, each over the half's H dims.
// A wave takes 64 consecutive points; lane l loads the whole row of point l and
// rounds it.  One permlane32 swap per packed word gives each lane half its
// operand halves of both 32-point tiles (tile A: points 0..31, tile B: 32..63).
// Each lane ranks its 16 NT scores of both tiles (best three as integer keys:
// score bits with the center index in the low bits); one swap per key
// then hands lane l the other half's keys of its own point (lane half 0
// finishes tile A, half 1 tile B), so the merge, the error band, the FP64
// decisions, J and the cluster sums run once per point, on whole rows.  The
// band certifies the best center; when only the second best is within it, FP64
// distances decide between the two; otherwise the FP64 check over all centers
// decides.  FULL: d == KD.
template <typename T, int KD, int NT, bool FULL>
__global__ __launch_bounds__(256, (KD == 16 && FULL) ? 4 : 3) void k_fused_pair(
    const T* __restrict__ X, int64_t n, int d, int k, const float* __restrict__ cnB,
    const double* __restrict__ c64, const PassState* __restrict__ st,
    const int32_t* __restrict__ gate, int update, long long* __restrict__ slots,
    double* __restrict__ Jpart, long long* __restrict__ upart, int32_t* __restrict__ labels) {
  if (gated(gate)) return;
  constexpr int H = KD / 2;                              // dims per lane half
  static_assert(KD >= 4 && KD <= 16, "whole packed words per lane half");
  constexpr int HW = H / 2;                              // packed words per half row
  constexpr int NS = sizeof(T) == 4 ? 3 : 2;             // products per dim
  constexpr int NM = (NS * H + 7) / 8;                   // MFMAs per center tile
  constexpr int NE = NM * 8;                             // K elements per lane half
  constexpr int BG = NT == 1 ? 5 : (NT == 2 ? 6 : 7);   // bits of a center index (32 NT)
  constexpr int GM = (1 << BG) - 1;
  extern __shared__ __align__(16) unsigned char smem[];
  // [k][CSS] FP64 centers, zero past d: a row stride of KD + 2 doubles (an odd
  // number of 16-byte units) spreads the rows that the lanes of a wave read for
  // their own centers over the LDS banks
  constexpr int CSS = KD + 2;
  double* cs = reinterpret_cast<double*>(smem);
  unsigned long long* S = reinterpret_cast<unsigned long long*>(cs + (size_t)k * CSS);  // [k][d+1]
  // then, 16-byte aligned: the A operands [NT][NM][64 lanes] and the C input
  // [32 NT] (both read from LDS where the MFMAs need them, which keeps the
  // registers for two tiles of points)
  const size_t tail = ((size_t)k * CSS * 8 + (size_t)k * (d + 1) * 8 + 15) & ~(size_t)15;
  v8bf* aop = reinterpret_cast<v8bf*>(smem + tail);
  float* cbias = reinterpret_cast<float*>(smem + tail + (size_t)NT * NM * 64 * 16);
  const int lane = threadIdx.x & 63, h = lane >> 5;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  for (int e = threadIdx.x; e < k * KD; e += 256) {
    const int j = e / KD, t = e - j * KD;
    cs[j * CSS + t] = t < d ? c64[(int64_t)j * d + t] : 0.0;
  }
  if (update)
    for (int e = threadIdx.x; e < k * (d + 1); e += 256) S[e] = 0ull;
  for (int e = threadIdx.x; e < 32 * NT; e += 256) cbias[e] = cnB[e];
  __syncthreads();
  // A operand of lane ln, center tile t, dims hH .. hH + H - 1 (h = ln / 32); K
  // elements c'hi, c'lo and, for FP32 data, c'hi again, each over the half's H
  // dims.  Row i = ln % 32 of the tile holds center 32t + 16 ((i / 4) % 2) +
  // 4 (i / 8) + i % 4: output register r of lane half h (row 8 (r / 4) + 4h +
  // r % 4) is then center 32t + 16h + r, so a key's low bits are its center.
  for (int e = threadIdx.x; e < NT * 64; e += 256) {
    const int t = e >> 6, ln = e & 63, hh = ln >> 5, i = ln & 31;
    const int j = 32 * t + 16 * ((i >> 2) & 1) + 4 * (i >> 3) + (i & 3);
    uint16_t e16[NE];
#pragma unroll
    for (int u = 0; u < NE; ++u) e16[u] = 0;
#pragma unroll
    for (int q = 0; q < H; ++q) {
      const double cp = j < k ? -2.0 * cs[j * CSS + hh * H + q] : 0.0;
      const uint16_t hi = f32_to_bf16((float)cp);
      e16[q] = hi;
      e16[H + q] = f32_to_bf16((float)(cp - (double)__uint_as_float((uint32_t)hi << 16)));
      if constexpr (NS == 3) e16[2 * H + q] = hi;
    }
#pragma unroll
    for (int m = 0; m < NM; ++m) {
      u16x8 v;
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = e16[8 * m + u];
      aop[(t * NM + m) * 64 + ln] = __builtin_bit_cast(v8bf, v);
    }
  }
  __syncthreads();
  // The band of two scores, E2 = c0 + c1 xn + c2 xr (xn >= ||x^||, xr >= ||x - x^||):
  // the dropped part x^.e + xlo.(c' - c'hi) + r.c' (||e|| <= 2^-8 ||c' - c'hi||,
  // ||xlo|| <= (1 + 2^-8) ||x - x^||, ||r|| <= 2^-8 ||x - x^||) and the FP32
  // accumulation of the C input and the products.
  const float B = st->B, cmax = st->cmax, dcn = st->dcn * 1.01f;
  const double scale64 = (double)st->scale;
  const float ea = (float)(16 * NM + 8) * 0x1p-23f * 1.01f;
  const float cc = 2.f * cmax + 2.004f * dcn;
  const float c0 = (2.f * ea * (cmax * cmax + B) + 1e-30f) * 1.0001f;
  const float c1 = (2.f * dcn * 0x1p-8f * 1.001f + 2.f * ea * cc) * 1.0001f;
  const float c2 = (2.f * dcn * 1.004f + 0x1p-6f * cmax + 2.f * ea * 1.004f * cc) * 1.0001f;
  const float delta = (float)(1 << BG) * 0x1p-23f * 1.01f;
  double Jacc = 0.0;
  int64_t ucnt = 0, pcnt = 0;
  const int64_t npair = (n + 63) >> 6;
  const int64_t pstride = (int64_t)gridDim.x * 4;
  int64_t pp = (int64_t)blockIdx.x * 4 + wave;
  // rows of the next 64 points load while this wave works on the current ones,
  // except for whole 16-dim rows, where those registers buy a fourth wave per
  // SIMD instead (measured faster)
  constexpr bool PREF = !(KD == 16 && FULL);
  float xnext[PREF ? KD : 1];
  // rows past n read the last row (their results are not used)
  if constexpr (PREF) load_row_full<T, KD, FULL>(X, min((pp << 6) + lane, n - 1), d, xnext);
  for (; pp < npair; pp += pstride) {
    const int64_t i = (pp << 6) + lane;
    const bool valid = i < n;
    float x[KD];
    if constexpr (PREF) {
#pragma unroll
      for (int q = 0; q < KD; ++q) x[q] = xnext[q];
      load_row_full<T, KD, FULL>(X, min(((pp + pstride) << 6) + lane, n - 1), d, xnext);
    } else {
      load_row_full<T, KD, FULL>(X, min(i, n - 1), d, x);
    }
    // the row as BF16: x^ (RNE, two values per instruction) and, for FP32 data,
    // xlo = BF16(x - x^) (the difference is exact); packed word w holds dims
    // 2w, 2w + 1, so words [0, HW) are the first half row
    typedef float f32x2 __attribute__((ext_vector_type(2)));
    typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
    uint32_t xw[H], lw[H] = {};
    float s2 = 0.f, r2 = 0.f;
#pragma unroll
    for (int q = 0; q < H; ++q) {
      const f32x2 pr = {x[2 * q], x[2 * q + 1]};
      xw[q] = __builtin_bit_cast(uint32_t, __builtin_convertvector(pr, bf16x2));
      const float lo = bf16_lo(xw[q]), hi = bf16_hi(xw[q]);
      s2 = __builtin_fmaf(lo, lo, s2);
      s2 = __builtin_fmaf(hi, hi, s2);
      if constexpr (sizeof(T) == 4) {
        const f32x2 rr = {x[2 * q] - lo, x[2 * q + 1] - hi};
        r2 = __builtin_fmaf(rr.x, rr.x, r2);
        r2 = __builtin_fmaf(rr.y, rr.y, r2);
        lw[q] = __builtin_bit_cast(uint32_t, __builtin_convertvector(rr, bf16x2));
      }
    }
    // swap (first half word, second half word): afterwards word [0] is this
    // lane half's part of tile A's point pc and [1] that of tile B's point pc
    uint32_t hA[HW], hB[HW], lA[HW], lB[HW];
#pragma unroll
    for (int q = 0; q < HW; ++q) {
      const auto r = __builtin_amdgcn_permlane32_swap(xw[q], xw[HW + q], false, false);
      hA[q] = r[0];
      hB[q] = r[1];
      if constexpr (NS == 3) {
        const auto s = __builtin_amdgcn_permlane32_swap(lw[q], lw[HW + q], false, false);
        lA[q] = s[0];
        lB[q] = s[1];
      }
    }
    // B operands: the terms' words one after the other (x^, x^, then xlo for
    // FP32 data), zero padded
    auto operands = [&](const uint32_t (&hw)[HW], const uint32_t (&lo)[HW], v8bf (&ov)[NM]) {
      uint32_t words[NE / 2];
#pragma unroll
      for (int w = 0; w < NE / 2; ++w) {
        const int u = w / HW, q = w % HW;
        words[w] = u < 2 ? hw[q] : (u == 2 && NS == 3 ? lo[q] : 0u);
      }
#pragma unroll
      for (int m = 0; m < NM; ++m) {
        const uint32_t w4[4] = {words[4 * m], words[4 * m + 1], words[4 * m + 2], words[4 * m + 3]};
        ov[m] = __builtin_bit_cast(v8bf, w4);
      }
    };
    v8bf oA[NM], oB[NM];
    operands(hA, lA, oA);
    operands(hB, lB, oB);
    int a1 = INT_MAX, a2 = INT_MAX, a3 = INT_MAX, b1 = INT_MAX, b2 = INT_MAX, b3 = INT_MAX;
    auto rank = [&](const v16f& acc, int t, int& m1, int& m2, int& m3) {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        // the value part drops BG bits (the index bits and the lane half)
        const int kv = (__float_as_int(acc[r]) & ~GM) | (32 * t + r);
        m3 = med3_i32(m2, kv, m3);
        m2 = med3_i32(m1, kv, m2);
        m1 = min(m1, kv);
      }
    };
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      // the C input of this lane's centers 32t + 16h + r
      v16f bias;
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const float4 v = *reinterpret_cast<const float4*>(&cbias[32 * t + 16 * h + 4 * g]);
        bias[4 * g] = v.x; bias[4 * g + 1] = v.y; bias[4 * g + 2] = v.z; bias[4 * g + 3] = v.w;
      }
      v8bf at = aop[(t * NM) * 64 + lane];
      v16f accA = __builtin_amdgcn_mfma_f32_32x32x16_bf16(at, oA[0], bias, 0, 0, 0);
      v16f accB = __builtin_amdgcn_mfma_f32_32x32x16_bf16(at, oB[0], bias, 0, 0, 0);
#pragma unroll
      for (int m = 1; m < NM; ++m) {
        at = aop[(t * NM + m) * 64 + lane];
        accA = __builtin_amdgcn_mfma_f32_32x32x16_bf16(at, oA[m], accA, 0, 0, 0);
        accB = __builtin_amdgcn_mfma_f32_32x32x16_bf16(at, oB[m], accB, 0, 0, 0);
      }
      rank(accA, t, a1, a2, a3);
      rank(accB, t, b1, b2, b3);
    }
    // the lane half into the index bits (which then hold the center), then
    // swap: lane l gets the other half's keys of its own point and merges
    const int hb = h << 4;
    int g1, g2, g3;
    {
      const auto s1 = __builtin_amdgcn_permlane32_swap(a1 | hb, b1 | hb, false, false);
      const auto s2k = __builtin_amdgcn_permlane32_swap(a2 | hb, b2 | hb, false, false);
      const auto s3 = __builtin_amdgcn_permlane32_swap(a3 | hb, b3 | hb, false, false);
      g1 = (int)s1[0];
      g2 = (int)s2k[0];
      g3 = (int)s3[0];
      const int ov[3] = {(int)s1[1], (int)s2k[1], (int)s3[1]};
#pragma unroll
      for (int u = 0; u < 3; ++u) {
        g3 = med3_i32(g2, ov[u], g3);
        g2 = med3_i32(g1, ov[u], g2);
        g1 = min(g1, ov[u]);
      }
    }
    auto center = [&](int key) { return key & GM; };
    int bi = center(g1);
    const int bj2 = center(g2);
    const float v1 = __int_as_float(g1 & ~GM), v2 = __int_as_float(g2 & ~GM),
                v3 = __int_as_float(g3 & ~GM);
    // norms for the band (the hardware square root is within an ulp; the 1%
    // factor covers it)
    const float xn = __builtin_amdgcn_sqrtf(s2) * 1.01f;
    const float xr = sizeof(T) == 4 ? __builtin_amdgcn_sqrtf(r2) * 1.01f : 0.f;
    const float E2 = __builtin_fmaf(c2, xr, __builtin_fmaf(c1, xn, c0));
    auto apart = [&](float lo, float hi) {
      return (hi - lo) > E2 + delta * (fabsf(hi) + fabsf(lo));
    };
    // certain: the best beats every other center; pair: the best is one of the best two
    const bool certain = k == 1 || (bi < k && apart(v1, v2));
    const bool pair = valid && !certain && bi < k && bj2 < k && (k == 2 || apart(v1, v3));
    const bool full = valid && !certain && !pair;
    if (bi >= k) bi = 0;
    double x64[KD];
#pragma unroll
    for (int q = 0; q < KD; ++q) x64[q] = (double)x[q];
    auto dist64 = [&](int j) {  // FP64 direct form over the whole row (zero past d)
      const double* cj = cs + j * CSS;
      double p = 0.0;
#pragma unroll
      for (int q = 0; q < KD; ++q) {
        const double e = x64[q] - cj[q];
        p = __builtin_fma(e, e, p);
      }
      return p;
    };
    double p1 = dist64(bi);
    if (__ballot(pair)) {
      // the second candidate's FP64 distance decides (lowest index on ties)
      const double p2 = dist64(pair ? bj2 : 0);
      if (pair && (p2 < p1 || (p2 == p1 && bj2 < bi))) {
        bi = bj2;
        p1 = p2;
      }
      pcnt += __popcll(__ballot(pair));
    }
    if (__ballot(full)) {
      ucnt += row_fp64_check<KD, CSS>(full, x, k, cs, bi);
      if (full) p1 = dist64(bi);
    }
    if (valid) {
      Jacc += p1;
      if (labels) labels[i] = bi;
      if (update) {
        // q = rint(x 2^F) as the bits of 1.5 2^52 + q: one FMA (x 2^F is exact,
        // |q| < 2^30), added biased; the finalize takes N kSumBias off
        unsigned long long* Sr = S + (int64_t)bi * (d + 1);
#pragma unroll
        for (int q = 0; q < KD; ++q) {
          if (FULL || q < d) {
            const double tq = __builtin_fma(x64[q], scale64, 0x1.8p52);
            atomicAdd(&Sr[q], (unsigned long long)__double_as_longlong(tq));
          }
        }
        atomicAdd(&Sr[d], 1ull);
      }
    }
  }
  __syncthreads();
  if (update) flush_sums(S, k, d, slots);
  block_sum_J(Jacc, ucnt, pcnt, Jpart, upart);
}

// The BF16 screen of all points.  A block (4 waves) takes 4*PT tiles of 32
// points; each wave keeps its rows as the B operand of 32x32x16 BF16 MFMAs in
// registers.  Centers stream through LDS in stages of 128 rows, double-buffered:
// the next stage is copied global -> LDS directly (no registers) while the
// current one is on the matrix cores, with one barrier per stage.  A score is
// ||c||^2 + B - 2 x.c (FP32 accumulation; B >= every ||x||^2 plus the screen's
// error, so scores are positive and their bits order as integers).  Each lane
// owns 16 center rows of every tile ("slots"); per pair of slots it keeps the
// two smallest keys (score bits with the tile index and the row parity in the
// low bits): three VALU operations per score.  At the end the lane halves merge the tracked keys;
// a key not tracked is at least the second key of its slot pair, which bounds what
// was not kept.  The point is certain when the best two tracked keys are
// apart by more than the error band; re-ranked in FP32 (then FP64) when at
// most three tracked keys lie in the band and no slot pair holds two of them; and
// queued for the re-screen otherwise.
template <typename T, int KS, int PT, int NW, bool R16 = false>
__global__ __launch_bounds__(64 * NW, PT == 1 && NW == 8 && KS == 8 ? 4 : 2) void k_screen_bf16(
    const T* __restrict__ X, int64_t n, int d, int k, const uint16_t* __restrict__ cb16,
    const float* __restrict__ cnB, const float* __restrict__ cw, const double* __restrict__ c64,
    PassState* __restrict__ st, const int32_t* __restrict__ gate, int32_t* __restrict__ labels,
    uint32_t* __restrict__ queue, float* __restrict__ qthr, int4* __restrict__ rq_c,
    double* __restrict__ Jpart, long long* __restrict__ upart) {
  if (gated(gate)) return;
  constexpr int KD = KS * 16;
  constexpr int C8 = KD / 8;                  // 16-byte chunks per center row
  constexpr int SC = 128;                     // center rows per stage
  constexpr int NI = SC * KD * 2 / 1024;      // 1 KB LDS-direct loads per stage
  // two stage buffers as separate objects, each used by its own code path, so
  // that reads of one need not wait for the LDS-direct loads into the other
  __shared__ __align__(16) uint16_t cb0[SC * KD], cb1[SC * KD];
  __shared__ __align__(16) float bb0[SC], bb1[SC];
  const int lane = threadIdx.x & 63, h = lane >> 5, pc = lane & 31;
  // wave-uniform (scalar) wave index: the stage-copy loops below then run on
  // the scalar unit
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  // an even number of stages over the padded rows (padding rows score 1e30):
  // the stage loop below runs in pairs without a branch
  const int nst = ((k + 2 * SC - 1) / (2 * SC)) * 2, nct = nst * (SC / 32);
  static_assert(kScreenRows % (2 * SC) == 0, "stage pairs must tile the padded rows");
  // a key: score bits, then the tile index and the slot's row parity (TB + 1 bits)
  int TB = 0;
  while ((1 << TB) < nct) ++TB;
  const int TM = (1 << (TB + 1)) - 1;
  int BG = 5;
  while ((1 << BG) < 32 * nct) ++BG;
  const int GM = (1 << BG) - 1;
  const float B = st->B, cmax = st->cmax, dcn = st->dcn * 1.01f;
  // FP32 accumulation of a score, with any rounding of the partial sums
  const float ea = (float)(KD + 8) * 0x1p-23f * 1.01f;
  const float delta = (float)(1 << BG) * 0x1p-23f * 1.01f;
  const int64_t per_block = NW * PT * 32;
  int64_t nfull = 0, ncand = 0;
  // Stage g of the (padded, tiled) center copy into a buffer with LDS-direct
  // loads: the stage is one contiguous range, copied as is.  In LDS, chunk c of
  // row r of tile t sits at ((t * C8 + c) * 32 + r) * 16 bytes, so the 32 rows
  // a wave reads for one MFMA operand are 512 contiguous bytes (no bank conflicts).
  auto issue_stage = [&](int g, uint16_t* cdst, float* bdst) {
    static_assert(NI % NW == 0, "every wave copies the same number of 1 KB pieces");
#pragma unroll
    for (int u = 0; u < NI / NW; ++u) {
      const int i = u * NW + wave;
      __builtin_amdgcn_global_load_lds(
          static_cast<const void*>(cb16 + (int64_t)g * SC * KD + i * 512 + lane * 8),
          static_cast<void*>(cdst + i * 512), 16, 0, 0);
    }
    static_assert(SC % 64 == 0, "a stage's biases are whole 64-float loads");
    for (int i = NW - 1 - wave; i < SC / 64; i += NW)
      __builtin_amdgcn_global_load_lds(
          static_cast<const void*>(cnB + (int64_t)g * SC + 64 * i + lane),
          static_cast<void*>(bdst + 64 * i), 4, 0, 0);
  };
  // every wave's LDS-direct loads are in LDS before the barrier
  auto stage_sync = [&]() {
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
  };
  // Blocks start at different stages (the order of the stages does not change
  // the kept keys), so that they do not all read the same center rows from the
  // same L2 channels at once.
  const int rot = (int)(blockIdx.x % (unsigned)nst);
  auto next_stage = [&](int gs) { return gs + 1 < nst ? gs + 1 : 0; };
  if ((int64_t)blockIdx.x * per_block < n) issue_stage(rot, cb0, bb0);
  // The wave's rows of a batch, as the MFMAs' B operands.  BF16 data: loaded
  // at the end of the previous batch, before its merges and candidate work, so
  // that the loads' latency hides behind that work (the accumulators are free
  // by then); FP32 data is rounded as it is loaded, at the start of the batch.
  constexpr bool EARLY = sizeof(T) == 2;
  v8bf x[PT][KS];
  // R16 (chosen by the host): every row is KS*16 BF16 dims on a 16-byte
  // boundary, so each piece is one 16-byte load with no checks (a point past
  // n reads row 0; its column of the MFMAs is never used).
  auto load_rows = [&](int64_t b0) {
    if constexpr (R16) {
#pragma unroll
      for (int p = 0; p < PT; ++p) {
        const int64_t e = b0 + (int64_t)(wave * PT + p) * 32 + pc;
        const T* row = X + (e < n ? e : 0) * d + 8 * h;
#pragma unroll
        for (int s = 0; s < KS; ++s)
          x[p][s] = __builtin_bit_cast(v8bf, *reinterpret_cast<const uint4*>(row + 16 * s));
      }
      return;
    }
#pragma unroll
    for (int p = 0; p < PT; ++p) {
      const int64_t e = b0 + (int64_t)(wave * PT + p) * 32 + pc;
      const bool ok = e < n;
#pragma unroll
      for (int s = 0; s < KS; ++s)
        x[p][s] = load8_bf16<T>(X + (ok ? e : 0) * d, 16 * s + 8 * h, d, ok);
    }
  };
  if constexpr (EARLY) load_rows((int64_t)blockIdx.x * per_block);
  for (int64_t base = (int64_t)blockIdx.x * per_block; base < n;
       base += (int64_t)gridDim.x * per_block) {
    int64_t ip[PT];
    bool valid[PT];
    float xn[PT], xr[PT];
    int m1[PT][8], m2[PT][8];  // per slot pair (rows r, r ^ 1): the two smallest keys
#pragma unroll
    for (int p = 0; p < PT; ++p) {
      const int64_t e = base + (int64_t)(wave * PT + p) * 32 + pc;
      valid[p] = e < n;
      ip[p] = valid[p] ? e : 0;
      float s2 = 0.f, r2 = 0.f;
      if constexpr (EARLY) {
        // ||x^||^2 by BF16 dot products (FP32 accumulation), two dims per step
        typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
#pragma unroll
        for (int s = 0; s < KS; ++s) {
          const uint4 w = __builtin_bit_cast(uint4, x[p][s]);
          const uint32_t w4[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const bf16x2 v = __builtin_bit_cast(bf16x2, w4[u]);
            s2 = __builtin_amdgcn_fdot2_f32_bf16(v, v, s2, false);
          }
        }
      } else {
#pragma unroll
        for (int s = 0; s < KS; ++s) {
          x[p][s] = load8_bf16<T>(X + ip[p] * d, 16 * s + 8 * h, d, valid[p], r2);
          const uint4 w = __builtin_bit_cast(uint4, x[p][s]);
          const uint32_t w4[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            s2 = __builtin_fmaf(bf16_lo(w4[u]), bf16_lo(w4[u]), s2);
            s2 = __builtin_fmaf(bf16_hi(w4[u]), bf16_hi(w4[u]), s2);
          }
        }
      }
      // (the 1% covers the rounding of the FP32 sums and of the square root)
      xn[p] = sqrtf(s2 + __shfl_xor(s2, 32)) * 1.01f;
      xr[p] = sqrtf(r2 + __shfl_xor(r2, 32)) * 1.01f;
#pragma unroll
      for (int g = 0; g < 8; ++g) m1[p][g] = m2[p][g] = INT_MAX;
    }
    // Software pipeline over the 32-center tiles: while the MFMAs of tile t
    // accumulate into one set of registers, the key updates of tile t-1 read
    // the other set, and the LDS reads of later steps are in flight (a ring of
    // four A operands three steps ahead, and the next tile's bias).  accP holds
    // the pending tile (index ctP); at the start of a batch it holds scores of
    // 1e30, which never displace a real key (see the merge below).
    v16f accA[PT], accP[PT];
    int ctP = 0;
#pragma unroll
    for (int p = 0; p < PT; ++p)
#pragma unroll
      for (int r = 0; r < 16; ++r) accP[p][r] = 1e30f;
    // key update of score (p, r) of a tile: three VALU operations
    auto key1 = [&](const v16f (&acc)[PT], int p, int r, int vc0, int vc1) {
      const int kv = (__float_as_int(acc[p][r]) & ~TM) | ((r & 1) ? vc1 : vc0);
      m2[p][r >> 1] = med3_i32(m1[p][r >> 1], kv, m2[p][r >> 1]);
      m1[p][r >> 1] = min(m1[p][r >> 1], kv);
    };
    auto keys = [&](const v16f (&acc)[PT], int ct) {
      const int vc0 = opaque_vgpr(ct << 1), vc1 = opaque_vgpr((ct << 1) | 1);
#pragma unroll
      for (int p = 0; p < PT; ++p)
#pragma unroll
        for (int r = 0; r < 16; ++r) key1(acc, p, r, vc0, vc1);
    };
    constexpr int NT = SC / 32;          // tiles per stage
    constexpr int NSTEP = NT * KS;       // MFMA steps (of PT MFMAs) per stage
    constexpr int SPG = 16 / KS;         // key updates placed after each MFMA
    static_assert(16 % KS == 0, "key updates split evenly over the MFMAs");
    // the A operand of step i (tile i / KS, dims 16 (i % KS) ...) of a stage buffer
    auto lds_a = [&](const uint16_t* cbuf, int i) -> v8bf {
      const int t = i / KS, s = i % KS;
      return *reinterpret_cast<const v8bf*>(&cbuf[((t * C8 + 2 * s + h) * 32 + pc) * 8]);
    };
    auto lds_bias = [&](const float* bbuf, int t, v16f& b) {
#pragma unroll
      for (int r = 0; r < 16; ++r) b[r] = bbuf[t * 32 + 8 * (r >> 2) + 4 * h + (r & 3)];
    };
    // One tile: each MFMA into `out` is followed by its share of the key
    // updates of `in` (tile ctin) and fenced, so that the scheduler keeps the
    // interleave (the matrix cores and the VALU then work side by side).
    auto tile = [&](int t, const uint16_t* cbuf, const float* bbuf, v8bf (&ring)[4], v16f& bias,
                    v16f (&out)[PT], const v16f (&in)[PT], int ctin) {
      const int vc0 = opaque_vgpr(ctin << 1), vc1 = opaque_vgpr((ctin << 1) | 1);
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        const int i = t * KS + s;
        if (i + 3 < NSTEP) ring[(i + 3) & 3] = lds_a(cbuf, i + 3);
#pragma unroll
        for (int p = 0; p < PT; ++p) {
          out[p] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ring[i & 3], x[p][s],
                                                           s == 0 ? bias : out[p], 0, 0, 0);
          const int q0 = (s * PT + p) * SPG;
#pragma unroll
          for (int q = q0; q < q0 + SPG; ++q) {
            key1(in, q >> 4, q & 15, vc0, vc1);
            if (q & 1) {
              pin_here(m1[q >> 4][(q & 15) >> 1]);
              pin_here(m2[q >> 4][(q & 15) >> 1]);
            }
          }
          __builtin_amdgcn_sched_barrier(0);
        }
        if (s == 0 && t + 1 < NT) lds_bias(bbuf, t + 1, bias);
      }
    };
    // the four tiles of stage gs, read from one buffer; tile 3 stays pending
    auto compute_stage = [&](int gs, const uint16_t* cbuf, const float* bbuf) {
      static_assert(NT == 4, "the stage code below names four tiles");
      v8bf ring[4];
      v16f bias;
      lds_bias(bbuf, 0, bias);
      ring[0] = lds_a(cbuf, 0);
      ring[1] = lds_a(cbuf, 1);
      ring[2] = lds_a(cbuf, 2);
      const int ct0 = gs * NT;
      tile(0, cbuf, bbuf, ring, bias, accA, accP, ctP);
      tile(1, cbuf, bbuf, ring, bias, accP, accA, ct0);
      tile(2, cbuf, bbuf, ring, bias, accA, accP, ct0 + 1);
      tile(3, cbuf, bbuf, ring, bias, accP, accA, ct0 + 2);
      ctP = ct0 + 3;
    };
    stage_sync();
    // stages in pairs: buffer 0 holds stages 0, 2, ..., buffer 1 stages 1, 3, ...;
    // each stage's successor loads into the other buffer while it computes
    int gs = rot;
    for (int g = 0; g < nst; g += 2) {
      const int gs1 = next_stage(gs), gs2 = next_stage(gs1);
      issue_stage(gs1, cb1, bb1);
      compute_stage(gs, cb0, bb0);
      stage_sync();
      if (g + 2 < nst) issue_stage(gs2, cb0, bb0);
      compute_stage(gs1, cb1, bb1);
      stage_sync();
      gs = gs2;
    }
    keys(accP, ctP);
    // both buffers are free: the next batch's first stage and (BF16 data) rows
    // load during the merges below
    if (base + (int64_t)gridDim.x * per_block < n) {
      issue_stage(rot, cb0, bb0);
      if constexpr (EARLY) load_rows(base + (int64_t)gridDim.x * per_block);
    }
#pragma unroll
    for (int p = 0; p < PT; ++p) {
      // Two scores differ from their exact values (||c||^2 + B - 2 x.c) by at most
      // E2 together: x^ . (e_1 - e_2) for the centers' rounding errors e_j
      // (||e_j|| <= dcn), 2 (x^ - x) . (c_1 - c_2) for rounded FP32 data, and
      // the FP32 accumulation of both.
      const float E2 = 2.f * xn[p] * dcn + 4.f * xr[p] * cmax +
                       2.f * ea * (cmax * cmax + B + 2.f * xn[p] * cmax);
      // Tracked keys -> global keys (score bits above BG, center index below).
      // After the first tile every slot pair holds two keys (real ones, or the
      // 1e30 keys of the batch start), so none is empty.  Within a pair the
      // global keys keep the order of their score bits, which is all that the
      // merge below needs: keys whose score bits agree are within the error
      // band of each other, so the choice between them is made exactly later.
      const int hoff = 4 * h;
      auto glob = [&](int a, int c) {  // c: offset of the pair's even row
        const int u = ((a & (TM - 1)) << 4) + hoff + c;  // 32 ct + row offset
        return (a & ~GM) | u | (a & 1);
      };
      // two sorted pairs -> sorted four
      auto merge22 = [](int a0, int a1, int b0, int b1, int (&o)[4]) {
        const int x = max(a0, b0), y = min(a1, b1);
        o[0] = min(a0, b0);
        o[1] = min(x, y);
        o[2] = max(x, y);
        o[3] = max(a1, b1);
      };
      // two sorted fours -> the sorted four smallest (bitonic merge)
      auto merge44 = [](const int (&a)[4], const int (&b)[4], int (&o)[4]) {
        const int c0 = min(a[0], b[3]), c1 = min(a[1], b[2]), c2 = min(a[2], b[1]),
                  c3 = min(a[3], b[0]);
        const int d0 = min(c0, c2), d2 = max(c0, c2), d1 = min(c1, c3), d3 = max(c1, c3);
        o[0] = min(d0, d1);
        o[1] = max(d0, d1);
        o[2] = min(d2, d3);
        o[3] = max(d2, d3);
      };
      int q4[4][4], r4[2][4], g4[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        // slot pairs 2u and 2u+1: rows at offsets 8u + 4h + {0,1} and {2,3}
        merge22(glob(m1[p][2 * u], 8 * u), glob(m2[p][2 * u], 8 * u),
                glob(m1[p][2 * u + 1], 8 * u + 2), glob(m2[p][2 * u + 1], 8 * u + 2), q4[u]);
      }
      merge44(q4[0], q4[1], r4[0]);
      merge44(q4[2], q4[3], r4[1]);
      merge44(r4[0], r4[1], g4);
      // the other lane half's four
      {
        int o[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) o[u] = other_half(g4[u], h);
        int t[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) t[u] = g4[u];
        merge44(t, o, g4);
      }
      int mm2 = m2[p][0];
#pragma unroll
      for (int g = 1; g < 8; ++g) mm2 = min(mm2, m2[p][g]);
      mm2 = min(mm2, other_half(mm2, h));
      float v[4];
      int jj[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        v[u] = __int_as_float(g4[u] & ~GM);
        jj[u] = g4[u] & GM;
      }
      const float vm2 = __int_as_float(mm2 & ~GM);
      auto apart = [&](float a, float b) {
        return (b - a) > E2 + delta * (fabsf(a) + fabsf(b));
      };
      // a point is decided (best key apart from the rest), re-ranked (its
      // candidates: the tracked keys within the band of the best, at most four)
      // or queued for the re-screen (the band may hold untracked centers)
      int nc = 0, label = 0;
      bool inb[4] = {true, false, false, false};
      bool full = false, decided = false;
      if (k == 1 || (jj[0] < k && apart(v[0], v[1]))) {
        decided = true;
        label = jj[0] < k ? jj[0] : 0;
      } else if (jj[0] < k && (k <= 4 || (apart(v[0], v[3]) && apart(v[0], vm2)))) {
        nc = 1;
#pragma unroll
        for (int u = 1; u < 4; ++u) {
          inb[u] = jj[u] < k && !apart(v[0], v[u]);
          nc += inb[u] ? 1 : 0;
        }
      } else {
        full = true;
      }
      const bool q = valid[p] && full && h == 0;
      const unsigned long long bq = __ballot(q);
      if (bq) {
        unsigned base_q = 0;
        if (lane == 0) base_q = atomicAdd(&st->qcount, (unsigned)__popcll(bq));
        base_q = __shfl(base_q, 0);
        if (q) {
          const unsigned pos = base_q + __popcll(bq & ((1ull << lane) - 1ull));
          queue[pos] = (uint32_t)ip[p];  // n < 2^32 on this path
          qthr[pos] = v[0] + E2 + 4.f * delta * (fabsf(v[0]) + E2) + 1e-30f;
        }
      }
      nfull += __popcll(bq);
      if (!valid[p]) {
        decided = true;
        nc = 0;
      }
      const bool rr = !decided && !full && nc > 0;
      // a point to re-rank gets the label -1 and its candidates (k_rerank_list
      // decides among them in FP64 and writes the label)
      if (rr && h == 0)
        rq_c[ip[p]] = make_int4(jj[0], inb[1] ? jj[1] : -1, inb[2] ? jj[2] : -1,
                                inb[3] ? jj[3] : -1);
      ncand += __popcll(__ballot(rr && h == 0));
      // every valid point gets a label here: the re-rank list reads -1 as its
      // marker, so no point may keep a stale label, and the points queued for
      // the re-screen hold 0 until the re-screen writes theirs
      if (valid[p] && h == 0) labels[ip[p]] = rr ? -1 : (full ? 0 : (label < k ? label : 0));
    }
  }
  block_sum_J(0.0, nfull, ncand, Jpart, upart);
}

// The re-rank of the points the screen marked (label -1): for each, the
// nearest of its (at most four) candidates by the direct form sum (x - c)^2,
// lowest index among equal distances.  A block takes ranges of RB points: its
// threads list the marked ones in LDS, then groups of 16 lanes take one listed
// point each (eight dims per lane; the row and every candidate row requested
// before any is summed).  The distances are FP32 first, with the error bound of
// the FP32 direct form; a point whose best two are closer than that bound is
// decided in FP64.
template <typename T, int KS>
__global__ __launch_bounds__(256) void k_rerank_list(
    const T* __restrict__ X, int64_t n, int d, int k, const float* __restrict__ cw,
    const double* __restrict__ c64, const PassState* __restrict__ st,
    const int32_t* __restrict__ gate, int32_t* __restrict__ labels,
    const int4* __restrict__ rq_c, long long* __restrict__ upart) {
  if (gated(gate)) return;
  constexpr int RB = 4096;                    // points per block range
  constexpr int NS8 = (KS * 16 + 127) / 128;  // 128-dim chunks of a row
  __shared__ uint16_t list[RB];
  __shared__ int cnt;
  const int li = threadIdx.x & 15, grp = threadIdx.x >> 4;
  const bool vec = (d & 7) == 0 && (reinterpret_cast<uintptr_t>(X) & 15u) == 0;
  const bool cvec = (d & 3) == 0;
  // FP32 direct form over a lane's <= 8 NS8 terms and four pairwise adds,
  // plus 2 sqrt(D) ||c - cw|| for the rounded center
  const float u32 = 0x1p-24f * 1.01f;
  const float cmax = st->cmax;
  auto err = [&](float D) {
    return (float)(8 * NS8 + 6) * u32 * D + 2.f * sqrtf(D) * u32 * cmax + 1e-30f;
  };
  int64_t nfp64 = 0;
  for (int64_t r0 = (int64_t)blockIdx.x * RB; r0 < n; r0 += (int64_t)gridDim.x * RB) {
    if (threadIdx.x == 0) cnt = 0;
    __syncthreads();
    const int rn = (int)min<int64_t>(RB, n - r0);
    // the thread's labels are loaded four at a time before their list updates,
    // so the loads overlap instead of each waiting behind the previous atomic
#pragma unroll 1
    for (int u0 = 0; u0 < RB / 256; u0 += 4) {
      int lv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int o = (u0 + u) * 256 + (int)threadIdx.x;
        lv[u] = o < rn ? labels[r0 + o] : 0;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (lv[u] < 0) list[atomicAdd(&cnt, 1)] = (uint16_t)((u0 + u) * 256 + threadIdx.x);
    }
    __syncthreads();
    const int m = cnt;
    // the 16 lanes of a group take the same q (uniform loop within a group)
    for (int q = grp; q < m; q += 16) {
      const int64_t pt = r0 + list[q];
      const int4 cj = rq_c[pt];
      auto ok = [&](int j) { return (j >= 0 && j < k) ? j : -1; };  // defensively
      const int cand[4] = {ok(cj.x), ok(cj.y), ok(cj.z), ok(cj.w)};
      const T* xr = X + pt * d;
      float xv[NS8][8];
      float part[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int s8 = 0; s8 < NS8; ++s8) {
        const int t0 = 128 * s8 + 8 * li;
        double xd[8];
        load8_f64<T>(xr, t0, d, vec, xd);  // zero past d
#pragma unroll
        for (int e8 = 0; e8 < 8; ++e8) xv[s8][e8] = (float)xd[e8];  // exact
        float cv[4][8];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const float* cr = cw + (int64_t)(cand[u] >= 0 ? cand[u] : 0) * d + t0;
          if (cand[u] >= 0 && cvec && t0 + 8 <= d) {
            const float4 a = *reinterpret_cast<const float4*>(cr);
            const float4 b = *reinterpret_cast<const float4*>(cr + 4);
            cv[u][0] = a.x; cv[u][1] = a.y; cv[u][2] = a.z; cv[u][3] = a.w;
            cv[u][4] = b.x; cv[u][5] = b.y; cv[u][6] = b.z; cv[u][7] = b.w;
          } else {
#pragma unroll
            for (int e8 = 0; e8 < 8; ++e8)
              cv[u][e8] = (cand[u] >= 0 && t0 + e8 < d) ? cr[e8] : 0.f;
          }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int e8 = 0; e8 < 8; ++e8)
            if (t0 + e8 < d) {
              const float diff = xv[s8][e8] - cv[u][e8];
              part[u] = __builtin_fmaf(diff, diff, part[u]);
            }
      }
      float best = INFINITY, sec = INFINITY;
      int bj = INT_MAX, nc = 0;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        float v = part[u];
        v += __shfl_xor(v, 8);
        v += __shfl_xor(v, 4);
        v += __shfl_xor(v, 2);
        v += __shfl_xor(v, 1);
        const int j = cand[u];
        if (j < 0) continue;
        ++nc;
        if (v < best || (v == best && j < bj)) {
          sec = best;
          best = v;
          bj = j;
        } else if (v < sec) {
          sec = v;
        }
      }
      if (!(nc <= 1 || (sec - best) > err(best) + err(sec))) {
        // too close for FP32: FP64 over the candidates
        double bD = INFINITY;
        int bj64 = INT_MAX;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int j = cand[u];
          double p = 0.0;
          if (j >= 0) {
            const double* cr = c64 + (int64_t)j * d;
#pragma unroll
            for (int s8 = 0; s8 < NS8; ++s8) {
              const int t0 = 128 * s8 + 8 * li;
#pragma unroll
              for (int e8 = 0; e8 < 8; ++e8)
                if (t0 + e8 < d) {
                  const double diff = (double)xv[s8][e8] - cr[t0 + e8];
                  p = __builtin_fma(diff, diff, p);
                }
            }
          }
          p += __shfl_xor(p, 8);
          p += __shfl_xor(p, 4);
          p += __shfl_xor(p, 2);
          p += __shfl_xor(p, 1);
          if (j >= 0 && (p < bD || (p == bD && j < bj64))) {
            bD = p;
            bj64 = j;
          }
        }
        bj = bj64;
        if (li == 0) ++nfp64;
      }
      if (li == 0) labels[pt] = bj < k ? bj : 0;
    }
    __syncthreads();  // the list is rebuilt for the next range
  }
  // points decided in FP64 (the per-block counter of the FP64 checks of the pass)
  nfp64 = wave_sum_i64(nfp64);
  __shared__ long long wsum[4];
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = nfp64;
  __syncthreads();
  if (threadIdx.x == 0 && upart) upart[blockIdx.x] = (wsum[0] + wsum[1]) + (wsum[2] + wsum[3]);
}

// The re-screen of the points the screen queued: every center whose screened
// score is at most the point's threshold becomes a candidate (up to CMAX; more
// send the point to the FP64 check over all centers), then the candidates are
// re-ranked as in the screen.  512 threads: 8 waves x PT tiles of 32 points
// share each 32-center tile in LDS.
template <typename T, int KS, int PT>
__global__ __launch_bounds__(512) void k_rescreen_bf16(
    const T* __restrict__ X, int d, int k, const uint16_t* __restrict__ cb16,
    const float* __restrict__ cnB, const float* __restrict__ cw, const double* __restrict__ c64,
    PassState* __restrict__ st, const int32_t* __restrict__ gate, int32_t* __restrict__ labels,
    const uint32_t* __restrict__ queue, const float* __restrict__ qthr,
    double* __restrict__ Jpart, long long* __restrict__ upart) {
  if (gated(gate)) return;
  constexpr int KD = KS * 16;
  constexpr int RS = KD + 8;      // LDS row stride in BF16 elements (spreads rows over banks)
  constexpr int CMAX = 16;        // candidates kept per queued point
  __shared__ __align__(16) uint16_t ctile[32 * RS];
  __shared__ float cbias[32];
  __shared__ int cand_n[8 * PT * 32];
  __shared__ int cand_j[8 * PT * 32 * CMAX];
  const int lane = threadIdx.x & 63, h = lane >> 5, pc = lane & 31, wave = threadIdx.x >> 6;
  const int nct = (k + 31) / 32;
  const float cmax = st->cmax;
  const int64_t count = (int64_t)ld_agent(reinterpret_cast<const int32_t*>(&st->qcount));
  const int64_t per_block = 8 * PT * 32;
  const bool vec = (d & 7) == 0 && (reinterpret_cast<uintptr_t>(X) & 15u) == 0;
  int64_t nfull = 0, ncand = 0;
  for (int64_t base = (int64_t)blockIdx.x * per_block; base < count;
       base += (int64_t)gridDim.x * per_block) {
    v8bf x[PT][KS];
    int64_t ip[PT];
    bool valid[PT];
    float thr[PT];
#pragma unroll
    for (int p = 0; p < PT; ++p) {
      const int64_t e = base + (int64_t)(wave * PT + p) * 32 + pc;
      valid[p] = e < count;
      ip[p] = valid[p] ? (int64_t)queue[e] : 0;
      thr[p] = valid[p] ? qthr[e] : 0.f;
#pragma unroll
      for (int s = 0; s < KS; ++s) x[p][s] = load8_bf16<T>(X + ip[p] * d, 16 * s + 8 * h, d, valid[p]);
      if (h == 0) cand_n[(wave * PT + p) * 32 + pc] = 0;
    }
    for (int ct = 0; ct < nct; ++ct) {
      __syncthreads();
      for (int e = threadIdx.x; e < 32 * (KD / 8); e += 512) {
        const int row = e / (KD / 8), c8 = e - row * (KD / 8);
        const int j = ct * 32 + row;
        uint4 v = {0u, 0u, 0u, 0u};
        if (j < k) v = *reinterpret_cast<const uint4*>(cb16 + cb16_at(j, c8 * 8, KD));
        *reinterpret_cast<uint4*>(&ctile[row * RS + c8 * 8]) = v;
      }
      if (threadIdx.x < 32) {
        const int j = ct * 32 + threadIdx.x;
        cbias[threadIdx.x] = j < k ? cnB[j] : INFINITY;
      }
      __syncthreads();
      v16f acc[PT];
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const float cb = cbias[8 * (r >> 2) + 4 * h + (r & 3)];
#pragma unroll
        for (int p = 0; p < PT; ++p) acc[p][r] = cb;
      }
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        const v8bf a = *reinterpret_cast<const v8bf*>(&ctile[pc * RS + 16 * s + 8 * h]);
#pragma unroll
        for (int p = 0; p < PT; ++p)
          acc[p] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, x[p][s], acc[p], 0, 0, 0);
      }
#pragma unroll
      for (int p = 0; p < PT; ++p)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int j = ct * 32 + 8 * (r >> 2) + 4 * h + (r & 3);
          if (valid[p] && j < k && acc[p][r] <= thr[p]) {
            const int slot = (wave * PT + p) * 32 + pc;
            const int q = atomicAdd(&cand_n[slot], 1);
            if (q < CMAX) cand_j[slot * CMAX + q] = j;
          }
        }
    }
    __syncthreads();
#pragma unroll
    for (int p = 0; p < PT; ++p) {
      const int slot = (wave * PT + p) * 32 + pc;
      const int cn_ = cand_n[slot];
      // more candidates than the list holds (or, defensively, none): FP64 over
      // all centers
      const bool full = valid[p] && (cn_ > CMAX || cn_ == 0);
      const int nc = (valid[p] && !full) ? cn_ : 0;
      const int* cand = &cand_j[slot * CMAX];
      int label = 0;
      int ncmax = nc;
      for (int o = 32; o > 0; o >>= 1) ncmax = max(ncmax, __shfl_xor(ncmax, o));
      if (ncmax > 0) {
        const bool rr = nc > 0;
        const int lab =
            vec ? rerank_vec<T, KS>(X + ip[p] * d, d, h, rr, cand, nc, ncmax, cw, c64, cmax, ncand)
                : rerank<T, KS>(X + ip[p] * d, d, h, rr, cand, nc, ncmax, cw, c64, cmax, ncand);
        if (rr) label = lab;
      }
      int lab2 = label;
      nfull += wave_fp64_fallback<T>(full && h == 0, ip[p], X, d, k, c64, lab2);
      lab2 = __shfl(lab2, pc);
      if (full) label = lab2;
      if (valid[p] && h == 0) labels[ip[p]] = label < k ? label : 0;
    }
  }
  block_sum_J(0.0, nfull, ncand, Jpart, upart);
}

// ============================================================================
// New centers from the slot sums, stage bookkeeping
// ============================================================================
// Fixed-order sums of J (the assignment blocks' partials, or the sorted
// update's exact limbs in jslots, which are zeroed for the next pass), of the
// FP64 check counts, and (when update) the largest movement, the largest ||c|| and
// the empties; then the pass bookkeeping.
// Sum or maximum over the 64 lanes of a wave by an xor butterfly: every lane
// gets the same bits (each step adds the same two partials, in either order).
__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
__device__ __forceinline__ long long wave_sum(long long v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}

__device__ void conclude_block(PassState* __restrict__ st, const double* __restrict__ Jpart,
                               const long long* __restrict__ upart, int64_t nb,
                               long long* __restrict__ jslots, const double* __restrict__ shiftj,
                               const double* __restrict__ cnorm,
                               const int32_t* __restrict__ emptyj, int k, bool update,
                               double* __restrict__ J_hist, double* __restrict__ shift_hist,
                               bool mark_labelled = false) {
  __shared__ double wJ[4], wS[4], wN[4];
  __shared__ long long wU[4], wE[4], wP[4];
  __shared__ int wM[4];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  double J = 0.0, sh = 0.0, nm = 0.0;
  long long U = 0, E = 0, Pc = 0;
  int jm = INT_MAX;  // lowest empty cluster
  for (int64_t b = tid; b < nb; b += 256) {
    if (!jslots) J += ld_agent(&Jpart[b]);
    U += ld_agent(&upart[2 * b]);
    Pc += ld_agent(&upart[2 * b + 1]);
  }
  if (update)
    for (int j = tid; j < k; j += 256) {
      sh = fmax(sh, ld_agent(&shiftj[j]));
      nm = fmax(nm, ld_agent(&cnorm[j]));
      const int ej = ld_agent(&emptyj[j]);
      E += ej;
      if (ej) jm = min(jm, j);
    }
  for (int o = 32; o > 0; o >>= 1) jm = min(jm, __shfl_xor(jm, o));
  // fixed-order reductions: lanes of a wave, then the four waves
  J = wave_sum(J); U = wave_sum(U); Pc = wave_sum(Pc); E = wave_sum(E);
  sh = wave_max(sh); nm = wave_max(nm);
  if (lane == 0) {
    wJ[wv] = J; wU[wv] = U; wP[wv] = Pc; wE[wv] = E; wS[wv] = sh; wN[wv] = nm; wM[wv] = jm;
  }
  __syncthreads();
  if (tid == 0) {
    double Jt = (wJ[0] + wJ[1]) + (wJ[2] + wJ[3]);
    const long long Ut = (wU[0] + wU[1]) + (wU[2] + wU[3]);
    const long long Pt = (wP[0] + wP[1]) + (wP[2] + wP[3]);
    const long long Et = (wE[0] + wE[1]) + (wE[2] + wE[3]);
    const double St = fmax(fmax(wS[0], wS[1]), fmax(wS[2], wS[3]));
    const double Nt = fmax(fmax(wN[0], wN[1]), fmax(wN[2], wN[3]));
    if (jslots) {
      // the sorted update's J: exact integer limbs of 2^-FJ and 2^(40-FJ)
      long long a0 = 0, a1 = 0;
      for (int q = 0; q < kSlots; ++q) {
        a0 += ld_agent(&jslots[2 * q]);
        a1 += ld_agent(&jslots[2 * q + 1]);
        jslots[2 * q] = 0;
        jslots[2 * q + 1] = 0;
      }
      a1 += a0 >> 40;
      a0 &= (1ll << 40) - 1;
      Jt = ldexp((double)a1, 40 - st->FJ) + ldexp((double)a0, -st->FJ);
    }
    st->J = Jt;
    st->uncertain += Ut;
    st->pairs += Pt;
    st->qcount = 0u;
    if (update) {
      const int it = st->iter;
      st->shift = St;
      st->empty = (int32_t)Et;
      st->cmax = (float)(Nt * (1.0 + 0x1p-20)) * (1.0f + 0x1p-20f);
      if (J_hist) J_hist[it] = Jt;
      if (shift_hist) shift_hist[it] = St;
      st->iter = it + 1;
      st->converged = St < st->tol ? 1 : 0;
      st->done = (st->converged || it + 1 >= st->max_iter) ? 1 : 0;
      // re-seeding: the lowest empty cluster moves to the farthest point
      // (k_farthest, k_reseed), which then redo the stop test
      if (st->reseed && Et > 0) st->reseed_j = min(min(wM[0], wM[1]), min(wM[2], wM[3]));
    } else if (mark_labelled) {
      st->done = 2;  // a batched labelling pass ran; later launches skip it
    }
  }
}

// One block per center: the exact sum of its kSlots slot rows (zeroed for the
// next pass), then (update) the new center -- the average; an empty cluster
// keeps its center -- its movement and norm, and the BF16 copy of the screen.
// With jslots, J is that of the sorted update.  The last block concludes the
// pass.
__device__ void finalize_center(
    int j, long long* __restrict__ slots, long long* __restrict__ jslots, int k, int d,
    PassState* __restrict__ st, int update, double* __restrict__ c64, float* __restrict__ cw,
    float* __restrict__ cn, double* __restrict__ cnorm, double* __restrict__ shiftj,
    int32_t* __restrict__ emptyj, double* __restrict__ S_out, int64_t* __restrict__ N_out,
    uint16_t* __restrict__ cb16, float* __restrict__ cnB, int kd16,
    const double* __restrict__ Jpart, const long long* __restrict__ upart, int64_t nb,
    double* __restrict__ J_hist, double* __restrict__ shift_hist, bool mark_labelled = false,
    bool biased = false, double* __restrict__ trace_c = nullptr,
    long long* __restrict__ trace_n = nullptr, uint16_t* __restrict__ cb16lo = nullptr,
    int nslots = kSlots) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int64_t C = (int64_t)k * (d + 1);
  // this pass's index in the stage (the last block of the pass advances it
  // only after every block has read it)
  const int64_t it = st->iter;
  if (!update) trace_c = nullptr, trace_n = nullptr;
  double* tc = trace_c ? trace_c + (it * k + j) * d : nullptr;
  long long* col = slots + (int64_t)j * (d + 1);
  __shared__ long long scnt[kSlots];  // points per slot row (biased sums)
  __shared__ long long sN;
  __shared__ double wred[3][4];
  __shared__ int last;
  if (wv == 0) {
    long long v = 0;
    if (lane < kSlots) scnt[lane] = 0;
    if (lane < nslots) {
      v = col[(int64_t)lane * C + d];
      col[(int64_t)lane * C + d] = 0;
      scnt[lane] = v;
    }
    v = wave_sum(v);
    if (lane == 0) sN = v;
  }
  __syncthreads();
  const long long Nj = sN;
  const int F = st->F;
  double sh = 0.0, nn = 0.0, ee = 0.0;
  const int r = tid & 31, c = tid >> 5;  // 32 slots x 8 dims per round
  for (int t0 = 0; t0 < d; t0 += 8) {
    const int t = t0 + c;
    long long sv = 0;
    if (t < d && r < nslots) {
      sv = col[(int64_t)r * C + t];
      col[(int64_t)r * C + t] = 0;
      // biased sums: every point added kSumBias + q (mod 2^64)
      if (biased)
        sv = (long long)((unsigned long long)sv - (unsigned long long)scnt[r] * kSumBias);
    }
    // the 32 slot rows of dim t are the lanes of one half wave
    for (int o = 16; o > 0; o >>= 1) sv += __shfl_xor(sv, o);
    if (r == 0 && t < d) {
      const double sum = ldexp((double)sv, -F);
      if (update) {
        const double cold = c64[(int64_t)j * d + t];
        if (tc) tc[t] = cold;
        const double cnew = Nj > 0 ? sum / (double)Nj : cold;
        const double diff = cnew - cold;
        sh += diff * diff;
        nn += cnew * cnew;
        c64[(int64_t)j * d + t] = cnew;
        cw[(int64_t)j * d + t] = (float)cnew;
        if (cb16lo) {
          uint16_t hi, lo;
          const double e = bf16_split(cnew, hi, lo);
          cb16[cb16_at(j, t, kd16)] = hi;
          cb16lo[cb16_at(j, t, kd16)] = lo;
          ee += e * e;
        } else if (cb16) {
          const uint16_t b = f32_to_bf16((float)(-2.0 * cnew));
          cb16[cb16_at(j, t, kd16)] = b;
          const double e = bf16_err(b, cnew);
          ee += e * e;
        }
      }
      if (S_out) S_out[(int64_t)j * d + t] = sum;
    }
  }
  sh = wave_sum(sh);
  nn = wave_sum(nn);
  ee = wave_sum(ee);
  if (lane == 0) {
    wred[0][wv] = sh;
    wred[1][wv] = nn;
    wred[2][wv] = ee;
  }
  __syncthreads();
  const bool new_copy = update && cb16;  // the BF16 copy of this center was rewritten
  if (tid == 0) {
    const double rd0 = (wred[0][0] + wred[0][1]) + (wred[0][2] + wred[0][3]);
    const double rn0 = (wred[1][0] + wred[1][1]) + (wred[1][2] + wred[1][3]);
    const double re0 = (wred[2][0] + wred[2][1]) + (wred[2][2] + wred[2][3]);
    if (update) {
      shiftj[j] = sqrt(rd0);
      cn[j] = (float)rn0;
      cnorm[j] = sqrt(rn0);
      emptyj[j] = Nj == 0 ? 1 : 0;
      if (cnB) cnB[j] = (float)(rn0 + (double)st->B);
    }
    if (new_copy) dcn_max(st, re0);
    if (N_out) N_out[j] = (int64_t)Nj;
    if (trace_n) trace_n[it * k + j] = Nj;
    __threadfence();
    last = atomicAdd(&st->ticket, 1u) == (unsigned)(k - 1) ? 1 : 0;
  }
  __syncthreads();
  if (last) {
    __threadfence();
    conclude_block(st, Jpart, upart, nb, jslots, shiftj, cnorm, emptyj, k, update != 0, J_hist,
                   shift_hist, mark_labelled);
    if (tid == 0) {
      if (new_copy) dcn_publish(st);
      st->ticket = 0u;
    }
  }
  __syncthreads();  // the shared arrays may be reused by a following call
}

__global__ __launch_bounds__(256) void k_finalize(
    long long* __restrict__ slots, long long* __restrict__ jslots, int k, int d,
    PassState* __restrict__ st, const int32_t* __restrict__ gate, int update,
    double* __restrict__ c64, float* __restrict__ cw, float* __restrict__ cn,
    double* __restrict__ cnorm, double* __restrict__ shiftj, int32_t* __restrict__ emptyj,
    double* __restrict__ S_out, int64_t* __restrict__ N_out,
    uint16_t* __restrict__ cb16, float* __restrict__ cnB, int kd16,
    const double* __restrict__ Jpart, const long long* __restrict__ upart, int64_t nb,
    double* __restrict__ J_hist, double* __restrict__ shift_hist, int biased,
    double* __restrict__ trace_c, long long* __restrict__ trace_n) {
  if (gated(gate)) return;
  finalize_center(blockIdx.x, slots, jslots, k, d, st, update, c64, cw, cn, cnorm, shiftj, emptyj,
                  S_out, N_out, cb16, cnB, kd16, Jpart, upart, nb, J_hist, shift_hist, false,
                  biased != 0, trace_c, trace_n);
}

// ----------------------------------------------------------------------------
// Empty-cluster re-seeding (opt-in).  After the update of a pass that left
// clusters empty, the lowest-index empty cluster takes as its new center the
// point farthest from its nearest updated center (FP64 direct form; the lowest
// point index on equal distances).  Its movement joins the pass's largest
// movement, so the stop test is taken again.  One cluster per pass.
// ----------------------------------------------------------------------------
// (D, i) with D larger, or equal D and a lower index, wins.
__device__ __forceinline__ bool far_better(double D, long long i, double oD, long long oi) {
  return D > oD || (D == oD && i < oi);
}

// Per block: the farthest of its points from their nearest center.
template <typename T>
__global__ __launch_bounds__(256) void k_farthest(const T* __restrict__ X, int64_t n, int d,
                                                  int k, const double* __restrict__ c64,
                                                  const PassState* __restrict__ st,
                                                  double* __restrict__ fpart,
                                                  long long* __restrict__ fidx) {
  if (st->reseed_j < 0) return;
  __shared__ double wD[4];
  __shared__ long long wI[4];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  double bD = -1.0;
  long long bI = LLONG_MAX;
  for (int64_t i = (int64_t)blockIdx.x * 256 + tid; i < n; i += (int64_t)gridDim.x * 256) {
    const T* xr = X + i * d;
    double m = INFINITY;
    for (int j = 0; j < k; ++j) {
      const double* cj = c64 + (int64_t)j * d;
      double D = 0.0;
      for (int t = 0; t < d; ++t) {
        const double diff = (double)widen<T>(xr[t]) - cj[t];
        D += diff * diff;  // built without contraction: the product is rounded, then added
      }
      m = fmin(m, D);
    }
    if (far_better(m, i, bD, bI)) {
      bD = m;
      bI = i;
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    const double oD = __shfl_xor(bD, o);
    const long long oI = __shfl_xor(bI, o);
    if (far_better(oD, oI, bD, bI)) {
      bD = oD;
      bI = oI;
    }
  }
  if (lane == 0) {
    wD[wv] = bD;
    wI[wv] = bI;
  }
  __syncthreads();
  if (tid == 0) {
    for (int w = 1; w < 4; ++w)
      if (far_better(wD[w], wI[w], bD, bI)) {
        bD = wD[w];
        bI = wI[w];
      }
    fpart[blockIdx.x] = bD;
    fidx[blockIdx.x] = bI;
  }
}

// One block: the farthest point over the partials becomes the center of the
// empty cluster; its working copies, the bounds of the screens, the largest
// movement and the stop test follow.
template <typename T>
__global__ __launch_bounds__(256) void k_reseed(const T* __restrict__ X, int d, int k,
                                                double* __restrict__ c64, float* __restrict__ cw,
                                                float* __restrict__ cn,
                                                double* __restrict__ cnorm,
                                                uint16_t* __restrict__ cb16,
                                                float* __restrict__ cnB, int kd16,
                                                PassState* __restrict__ st,
                                                const double* __restrict__ fpart,
                                                const long long* __restrict__ fidx, int nb,
                                                double* __restrict__ shift_hist) {
  const int j = st->reseed_j;
  if (j < 0) return;
  __shared__ double wD[4], red[3][4];
  __shared__ long long wI[4];
  __shared__ long long far_i;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  double bD = -1.0;
  long long bI = LLONG_MAX;
  for (int b = tid; b < nb; b += 256)
    if (far_better(fpart[b], fidx[b], bD, bI)) {
      bD = fpart[b];
      bI = fidx[b];
    }
  for (int o = 32; o > 0; o >>= 1) {
    const double oD = __shfl_xor(bD, o);
    const long long oI = __shfl_xor(bI, o);
    if (far_better(oD, oI, bD, bI)) {
      bD = oD;
      bI = oI;
    }
  }
  if (lane == 0) {
    wD[wv] = bD;
    wI[wv] = bI;
  }
  __syncthreads();
  if (tid == 0) {
    for (int w = 1; w < 4; ++w)
      if (far_better(wD[w], wI[w], bD, bI)) {
        bD = wD[w];
        bI = wI[w];
      }
    far_i = bI;
  }
  __syncthreads();
  const T* xr = X + far_i * d;
  double mv = 0.0, nn = 0.0, ee = 0.0;
  for (int t = tid; t < d; t += 256) {
    const double x = (double)widen<T>(xr[t]);
    const double diff = x - c64[(int64_t)j * d + t];
    mv += diff * diff;
    nn += x * x;
    c64[(int64_t)j * d + t] = x;
    cw[(int64_t)j * d + t] = (float)x;
    if (cb16) {
      const uint16_t b = f32_to_bf16((float)(-2.0 * x));
      cb16[cb16_at(j, t, kd16)] = b;
      const double e = bf16_err(b, x);
      ee += e * e;
    }
  }
  mv = wave_sum(mv);
  nn = wave_sum(nn);
  ee = wave_sum(ee);
  if (lane == 0) {
    red[0][wv] = mv;
    red[1][wv] = nn;
    red[2][wv] = ee;
  }
  __syncthreads();
  if (tid == 0) {
    const double m2 = (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]);
    const double n2 = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
    const double e2 = (red[2][0] + red[2][1]) + (red[2][2] + red[2][3]);
    cn[j] = (float)n2;
    cnorm[j] = sqrt(n2);
    if (cnB) cnB[j] = (float)(n2 + (double)st->B);
    if (cb16)
      st->dcn = fmaxf(st->dcn, (float)(sqrt(e2) * (1.0 + 0x1p-40)) * (1.0f + 0x1p-22f));
    st->cmax = fmaxf(st->cmax, (float)(sqrt(n2) * (1.0 + 0x1p-20)) * (1.0f + 0x1p-20f));
    const double sh = fmax(st->shift, sqrt(m2));
    st->shift = sh;
    if (shift_hist) shift_hist[st->iter - 1] = sh;
    st->converged = sh < st->tol ? 1 : 0;
    st->done = (st->converged || st->iter >= st->max_iter) ? 1 : 0;
    st->reseed_j = -1;
  }
}

// J and FP64-check counts of a labelling pass of the fused paths.  One block.
__global__ __launch_bounds__(256) void k_sum_J(PassState* __restrict__ st,
                                               const double* __restrict__ Jpart,
                                               const long long* __restrict__ upart, int64_t nb) {
  conclude_block(st, Jpart, upart, nb, nullptr, nullptr, nullptr, nullptr, 0, false, nullptr,
                 nullptr);
}

// ============================================================================
// Many instances per launch
// ============================================================================
// The instance owning entry u: the last one whose first entry is <= u (every
// listed instance has at least one entry).
// which: 0 assignment units, 1 finalize entries, 2 cluster-sum units (an
// instance without sum units shares its first entry with the next one and is
// never the last such).
// The 64 lanes of a wave probe 64 evenly spaced instances at once, so a
// search takes two dependent loads for up to 4096 instances and three for
// 8192 (every lane of the wave must call it with the same u).
__device__ __forceinline__ int batch_find(const BatchInst* __restrict__ bi, int ninst, int64_t u,
                                          int which) {
  const int lane = threadIdx.x & 63;
  int lo = 0, span = ninst;  // the answer lies in [lo, lo + span); bi[lo] starts at or before u
  while (span > 1) {
    const int step = (span + 63) >> 6;
    const int idx = lo + lane * step;
    bool ok = false;
    if (lane * step < span) {
      const BatchInst& c = bi[idx];
      const int64_t s0 = which == 1 ? c.center0 : which == 2 ? c.sunit0 : c.unit0;
      ok = s0 <= u;
    }
    const unsigned long long m = __ballot(ok);
    const int L = 63 - __clzll((long long)m);
    lo += L * step;
    span = min(step, span - L * step);
  }
  return lo;
}

// One launch assigns the points of every listed instance: each work unit is a
// tile of P*256 points of one instance, centers staged through LDS by ktile,
// FP32 scores certified against their error bound (FP64 otherwise), J per
// point in FP64, and (Lloyd passes) exact cluster sums, privatised in LDS when
// they fit or added with 64-bit atomics into the instance's slot rows.
// Persistent: blocks loop over the units.
template <typename T, int DMAX, int P>
__global__ __launch_bounds__(256) void k_batch_assign(const BatchHead* __restrict__ hd,
                                                      const BatchInst* __restrict__ bi) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int ninst = hd->ninst;
  const int64_t units = hd->units;
  for (int64_t u = blockIdx.x; u < units; u += gridDim.x) {
    const BatchInst& b = bi[batch_find(bi, ninst, u, 0)];
    PassState* st = b.st;
    const int dn = ld_agent(&st->done);
    if ((b.mode == 1 && dn) || (b.mode == 2 && dn == 2)) continue;
    const int64_t tile = u - b.unit0;
    const int d = b.d, k = b.k, ktile = b.ktile;
    float* w = reinterpret_cast<float*>(smem);
    float* cnl = w + (size_t)ktile * DMAX;
    unsigned long long* S = nullptr;
    const bool lds = b.mode == 1 && b.lds_sums;
    const int slot = (int)(tile & (b.nslots - 1));
    unsigned long long* row =
        reinterpret_cast<unsigned long long*>(b.slots + (int64_t)slot * k * (d + 1));
    if (lds) {
      S = reinterpret_cast<unsigned long long*>(
          smem + (((size_t)ktile * (DMAX + 1) * 4 + 15) / 16) * 16);
      for (int e = threadIdx.x; e < k * (d + 1); e += 256) S[e] = 0ull;
      __syncthreads();
    } else if (b.mode == 1 && b.sunits == 0) {
      S = row;  // otherwise k_batch_sums adds them after the labels are written
    }
    double Jacc = 0.0;
    int64_t ucnt = 0;
    assign_tile<T, DMAX, P, true>(reinterpret_cast<const T*>(b.X), b.n, d, k,
                                  tile * (int64_t)(P * 256), b.cw, b.cn, b.c64, w, cnl, ktile,
                                  st->cmax, st->scale, S, b.labels, true, Jacc, ucnt);
    if (lds) {
      __syncthreads();
      for (int e = threadIdx.x; e < k * (d + 1); e += 256) {
        const unsigned long long v = S[e];
        if (v) atomicAdd(&row[e], v);
      }
    }
    block_sum_J(Jacc, ucnt, 0, b.Jpart, b.upart, tile);
  }
}

// The batched BF16 screen: one launch scores the points of every listed
// BF16 instance with d in (16, 16 KS] and k <= 256 on the matrix cores.  A work
// unit is a tile of 256 points of one instance; each wave takes 64 of them as
// two 32-point MFMA B operands (x.c^T as 32x32x16 BF16 MFMAs, FP32
// accumulation from the C input ||c||^2 + B), reading the instance's copy of
// -2c as two BF16 parts hi + lo (tiled as in the single-problem screen: the 32
// rows of one MFMA operand are 512 contiguous bytes) straight from memory.
// BF16 data is exact, so a score's error is that of hi + lo (about 2^-17 of
// |c|) and of the FP32 accumulation: the band stays narrow even when the
// points lie far from the origin compared with the clusters' spread.  Each lane keeps the best four keys of its half of every
// tile's centers; the halves merge into the point's best four.  The error
// band of two scores (the centers' exact rounding error norm dcn, the FP32
// accumulation) certifies the best; when two or three keys lie inside it and
// the fourth does not, FP64 distances decide among them; otherwise the wave's
// FP64 check over all centers decides.  Then J (FP64 direct form) and the
// label; k_batch_sums adds the exact cluster sums from the labels.
template <int KS>
__global__ __launch_bounds__(256, 3) void k_batch_screen(const BatchHead* __restrict__ hd,
                                                      const BatchInst* __restrict__ bi) {
  constexpr int KD = KS * 16;
  constexpr int C8 = KD / 8;     // 16-byte chunks per center row of the copy
  constexpr int BG = 8;          // index bits of a key (k <= 256)
  constexpr int GM = (1 << BG) - 1;
  // tiles of the copy (hi, lo: C8 * 32 chunks of 16 bytes each) and their
  // biases, double-buffered
  constexpr int TE = C8 * 32 * 8;  // BF16 elements of one part of a tile
  __shared__ __align__(16) uint16_t tl[2][2][TE];
  __shared__ __align__(16) float tb[2][32];
  const int lane = threadIdx.x & 63, h = lane >> 5, pc = lane & 31;
  const int wave = threadIdx.x >> 6;
  const int ninst = hd->ninst;
  const int64_t units = hd->units;
  for (int64_t u = blockIdx.x; u < units; u += gridDim.x) {
    const BatchInst& b = bi[batch_find(bi, ninst, u, 0)];
    PassState* st = b.st;
    const int dn = ld_agent(&st->done);
    if ((b.mode == 1 && dn) || (b.mode == 2 && dn == 2)) continue;
    const int64_t tile = u - b.unit0;
    const int d = b.d, k = b.k, nct = (k + 31) >> 5;
    const uint16_t* X = reinterpret_cast<const uint16_t*>(b.X);
    const uint16_t* cb = b.cb16;
    const uint16_t* cbl = b.cb16lo;
    const float* cnB = b.cnB;
    const int64_t n = b.n;
    // the wave's 64 points: tile A (points 0..31) and tile B (32..63) of its part
    const int64_t p0 = tile * 256 + (int64_t)wave * 64;
    const int64_t iA = p0 + pc, iB = p0 + 32 + pc;
    const bool vA = iA < n, vB = iB < n;
    v8bf xA[KS], xB[KS];
    const bool rows16 = d == KD && (reinterpret_cast<uintptr_t>(X) & 15u) == 0;
    if (rows16) {
      // whole rows of KD dims: one 16-byte load per piece (a point past n
      // reads row 0; its column of the MFMAs is not used)
      const uint16_t* rA = X + (vA ? iA : 0) * d + 8 * h;
      const uint16_t* rB = X + (vB ? iB : 0) * d + 8 * h;
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        xA[s] = __builtin_bit_cast(v8bf, *reinterpret_cast<const uint4*>(rA + 16 * s));
        xB[s] = __builtin_bit_cast(v8bf, *reinterpret_cast<const uint4*>(rB + 16 * s));
      }
    } else {
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        xA[s] = load8_bf16<uint16_t>(X + (vA ? iA : 0) * d, 16 * s + 8 * h, d, vA);
        xB[s] = load8_bf16<uint16_t>(X + (vB ? iB : 0) * d, 16 * s + 8 * h, d, vB);
      }
    }
    const float B = st->B, cmax = st->cmax, dcn = st->dcn * 1.01f;
    // FP32 accumulation of 2 KD products and the bias, any rounding of the
    // partial sums
    const float ea = (float)(2 * KD + 8) * 0x1p-23f * 1.01f;
    const float delta = (float)(1 << BG) * 0x1p-23f * 1.01f;
    // the four smallest keys of the lane's scores, ascending
    int ga[4] = {INT_MAX, INT_MAX, INT_MAX, INT_MAX}, gb[4] = {INT_MAX, INT_MAX, INT_MAX, INT_MAX};
    auto insert = [](int (&m)[4], int kv) {
      m[3] = med3_i32(m[2], kv, m[3]);
      m[2] = med3_i32(m[1], kv, m[2]);
      m[1] = med3_i32(m[0], kv, m[1]);
      m[0] = min(m[0], kv);
    };
    auto rank = [&](const v16f& acc, int t, int (&m)[4]) {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int j = 32 * t + 8 * (r >> 2) + 4 * h + (r & 3);
        insert(m, (__float_as_int(acc[r]) & ~GM) | j);
      }
    };
    // Per point: ||x||^2 (BF16 data: the MFMA sees x exactly), the error bound
    // e1 of one score, and the offset that the C input adds to ||c||^2 + B so
    // that a score is ||x - c||^2 + margin: its magnitude is that of the
    // distance, so the keys lose little to the index bits, and it stays >= 0.
    // e1: the centers' rounding (||x|| dcn), the FP32 accumulation from the C
    // input over 2 KD products (magnitudes up to ||c||^2 + ||x||^2 and
    // 2 ||x|| ||c||), and the roundings of ||c||^2 + B and of the offset.
    float e1v[2], offv[2];
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      const v8bf* x = p == 0 ? xA : xB;
      float s2 = 0.f;
      typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        const uint4 w = __builtin_bit_cast(uint4, x[s]);
        const uint32_t w4[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const bf16x2 v = __builtin_bit_cast(bf16x2, w4[q]);
          s2 = __builtin_amdgcn_fdot2_f32_bf16(v, v, s2, false);
        }
      }
      const float xn2 = s2 + __shfl_xor(s2, 32);
      const float xn = sqrtf(xn2) * 1.01f;
      const float e1 = ea * (cmax * cmax + xn2 * 1.01f + 2.f * xn * cmax) + xn * dcn +
                       3.f * 0x1p-23f * (B + cmax * cmax + xn2);
      // ||x||^2 above is an FP32 sum of KD products
      const float margin = e1 + (float)(KD + 8) * 0x1p-23f * 1.01f * xn2 + 1e-30f;
      e1v[p] = e1 * 1.001f;
      // ||c||^2 - 2 x.c = ||x - c||^2 - ||x||^2: the offset adds ||x||^2 back
      offv[p] = margin + xn2 - B;
    }
    // Tile t of the copy into LDS buffer q with LDS-direct loads (a tile's
    // part is one contiguous range of the tiled copy, 1 KB per wave
    // instruction); the four waves share it.
    auto issue_tile = [&](int t, int q) {
      static_assert(TE % 512 == 0, "a tile's part is whole 1 KB pieces");
#pragma unroll
      for (int i = wave; i < TE / 512; i += 4) {
        __builtin_amdgcn_global_load_lds(
            static_cast<const void*>(cb + (int64_t)t * TE + i * 512 + lane * 8),
            static_cast<void*>(&tl[q][0][i * 512]), 16, 0, 0);
        __builtin_amdgcn_global_load_lds(
            static_cast<const void*>(cbl + (int64_t)t * TE + i * 512 + lane * 8),
            static_cast<void*>(&tl[q][1][i * 512]), 16, 0, 0);
      }
      if (wave == 3 && lane < 32)
        __builtin_amdgcn_global_load_lds(static_cast<const void*>(cnB + 32 * t + lane),
                                         static_cast<void*>(&tb[q][0]), 4, 0, 0);
    };
    // One sweep over the center tiles (every wave of the block takes part: the
    // tiles pass through LDS): the scores of the wave's two point tiles, handed
    // to `use(acc, t, p)` tile by tile.
    auto sweep = [&](auto&& use) {
      // the buffers may still be read by an earlier sweep's last tile
      __syncthreads();
      issue_tile(0, 0);
      for (int t = 0; t < nct; ++t) {
        const int q = t & 1;
        // tile t is in LDS, and every wave is done with tile t - 1
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (t + 1 < nct) issue_tile(t + 1, q ^ 1);
        v16f accA, accB;
#pragma unroll
        for (int g = 0; g < 4; ++g) {
          const float4 v = *reinterpret_cast<const float4*>(&tb[q][8 * g + 4 * h]);
          const float cv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            accA[4 * g + e] = cv[e] + offv[0];
            accB[4 * g + e] = cv[e] + offv[1];
          }
        }
#pragma unroll
        for (int part = 0; part < 2; ++part)
#pragma unroll
          for (int s = 0; s < KS; ++s) {
            const v8bf a =
                *reinterpret_cast<const v8bf*>(&tl[q][part][((2 * s + h) * 32 + pc) * 8]);
            accA = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, xA[s], accA, 0, 0, 0);
            accB = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, xB[s], accB, 0, 0, 0);
          }
        use(accA, t, 0);
        use(accB, t, 1);
      }
    };
    sweep([&](const v16f& acc, int t, int p) { rank(acc, t, p == 0 ? ga : gb); });
    // merge the lane halves: both lanes of a point get its best four keys
    auto merge_halves = [&](int (&m)[4]) {
      int o[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) o[q] = __shfl_xor(m[q], 32);
#pragma unroll
      for (int q = 0; q < 4; ++q) insert(m, o[q]);
    };
    merge_halves(ga);
    merge_halves(gb);
    double Jacc = 0.0;
    int64_t ucnt = 0, pcnt = 0;
    // Decisions of the wave's two points per lane pair (tile A's, tile B's):
    // the band E2 of two scores, the tracked keys inside the band of the best
    // (nc: the band grows with the score, so they are a prefix), and
    //   certain: only the best inside;
    //   pair: two or three inside, all real centers, the fourth outside: FP64
    //         decides among them;
    //   full: otherwise.  A full point's candidates are every center whose
    //         score is within thr of the best (a second pass over the centers
    //         collects them, up to kBatchCands); FP64 decides among them, or
    //         over all centers when there are more.
    constexpr int kBatchCands = 16;
    __shared__ uint8_t cand[4][2][32][kBatchCands];
    __shared__ int ccnt[4][2][32];
    bool pairv[2], fullv[2];
    int ncv[2], best[2];
    float thr[2];
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      const bool valid = p == 0 ? vA : vB;
      int g[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) g[q] = p == 0 ? ga[q] : gb[q];
      const float E2 = 2.f * e1v[p];
      auto apart = [&](float lo, float hi) {
        return (hi - lo) > E2 + delta * (fabsf(hi) + fabsf(lo));
      };
      const float v1 = __int_as_float(g[0] & ~GM);
      int nc = 1;
      bool real = (g[0] & GM) < k;
#pragma unroll
      for (int q = 1; q < 4; ++q)
        if (nc == q && !apart(v1, __int_as_float(g[q] & ~GM))) {
          nc = q + 1;
          real = real && (g[q] & GM) < k;
        }
      const bool certain = k == 1 || (real && nc == 1);
      pairv[p] = valid && !certain && real && nc < 4;
      fullv[p] = valid && !certain && !pairv[p];
      ncv[p] = nc;
      best[p] = (g[0] & GM) < k ? (g[0] & GM) : 0;
      // a center whose exact distance is at most the best's scores at most
      // E2 above the smallest score; the key of that score is within delta
      thr[p] = (v1 + E2 + delta * (2.f * fabsf(v1) + E2)) * 1.0001f;
    }
    // the second sweep runs when any wave of the block has a full point
    if (__syncthreads_or(fullv[0] || fullv[1])) {
      if (h == 0) ccnt[wave][0][pc] = ccnt[wave][1][pc] = 0;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      sweep([&](const v16f& acc, int t, int p) {
        if (!fullv[p]) return;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int j = 32 * t + 8 * (r >> 2) + 4 * h + (r & 3);
          if (j < k && acc[r] <= thr[p]) {
            const int c = atomicAdd(&ccnt[wave][p][pc], 1);
            if (c < kBatchCands) cand[wave][p][pc][c] = (uint8_t)j;
          }
        }
      });
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      __builtin_amdgcn_wave_barrier();
    }
    // Candidates of pair points join the lists (a full point's list was filled
    // by the second sweep).  The listed points (one to kBatchCands candidates)
    // are then decided in FP64 by groups of 16 lanes, one point per group at a
    // time: lane l of a group holds dims 8l .. 8l+7 of the point and of each
    // candidate row, so both are read as whole rows; the 16 partial sums are
    // added in a fixed tree.  Lowest index on equal distances.
    __shared__ uint8_t lpts[4][64];
    __shared__ uint8_t blab[4][64];
    __shared__ int lcnt[4];
    bool listedv[2];
    if (__ballot(pairv[0] || pairv[1] || fullv[0] || fullv[1])) {
      if (lane == 0) lcnt[wave] = 0;
#pragma unroll
      for (int p = 0; p < 2; ++p) {
        const int* gq = p == 0 ? ga : gb;
        if (pairv[p] && h == 0) {
#pragma unroll
          for (int q = 0; q < 3; ++q)
            if (q < ncv[p]) cand[wave][p][pc][q] = (uint8_t)(gq[q] & GM);
          ccnt[wave][p][pc] = ncv[p];
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
      for (int p = 0; p < 2; ++p) {
        const int cnt = (pairv[p] || fullv[p]) ? ccnt[wave][p][pc] : 0;
        listedv[p] = (pairv[p] || fullv[p]) && cnt >= 1 && cnt <= kBatchCands;
        if (listedv[p] && h == 0) lpts[wave][atomicAdd(&lcnt[wave], 1)] = (uint8_t)(32 * p + pc);
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      const int nl = lcnt[wave];
      const int grp = lane >> 4, sub = lane & 15, t0 = 8 * sub;
      const int64_t p0w = tile * 256 + (int64_t)wave * 64;
      for (int l0 = 0; l0 < nl; l0 += 4) {
        const int li = l0 + grp;
        const bool act = li < nl;
        const int slot = act ? lpts[wave][li] : 0;
        const int pp = slot >> 5, ps = slot & 31;
        const int cnt = act ? ccnt[wave][pp][ps] : 0;
        const uint16_t* xr = X + (act ? p0w + slot : 0) * d;
        const uint4 w = rows16 ? *reinterpret_cast<const uint4*>(xr + t0)
                               : __builtin_bit_cast(uint4, load8_bf16<uint16_t>(xr, t0, d, true));
        const uint32_t w4[4] = {w.x, w.y, w.z, w.w};
        int qn = cnt;
        for (int o = 32; o > 0; o >>= 1) qn = max(qn, __shfl_xor(qn, o));
        double bd = INFINITY;
        int bj = INT_MAX;
        for (int q = 0; q < qn; ++q) {
          const bool use = act && q < cnt;
          const int j = use ? (int)cand[wave][pp][ps][q] : 0;
          const double* cj = b.c64 + (int64_t)j * d;
          double cv[8];
#pragma unroll
          for (int e = 0; e < 8; ++e) cv[e] = cj[t0 + e < d ? t0 + e : 0];
          double part = 0.0;
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            const float xv = (e & 1) ? bf16_hi(w4[e >> 1]) : bf16_lo(w4[e >> 1]);
            const double df = t0 + e < d ? (double)xv - cv[e] : 0.0;
            part = __builtin_fma(df, df, part);
          }
          part += __shfl_xor(part, 8);
          part += __shfl_xor(part, 4);
          part += __shfl_xor(part, 2);
          part += __shfl_xor(part, 1);
          if (use && (part < bd || (part == bd && j < bj))) {
            bd = part;
            bj = j;
          }
        }
        if (act && sub == 0) blab[wave][slot] = (uint8_t)(bj < k ? bj : 0);
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
      listedv[0] = listedv[1] = false;
    }
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      const int64_t i = p == 0 ? iA : iB;
      const bool valid = p == 0 ? vA : vB;
      int bi1 = best[p];
      const bool listed = listedv[p];
      if (listed) bi1 = blab[wave][32 * p + pc];
      pcnt += __popcll(__ballot(listed && h == 0));
      const bool rest = fullv[p] && !listed;
      if (__ballot(rest)) {
        int lab = bi1;
        ucnt += wave_fp64_fallback<uint16_t>(rest && h == 0, i, X, d, k, b.c64, lab);
        // the half-0 lane decided: both halves take its label
        lab = __shfl(lab, pc);
        if (rest) bi1 = lab;
      }
      if (valid && h == 0) {
        if (b.labels) b.labels[i] = bi1;
        blab[wave][32 * p + pc] = (uint8_t)bi1;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // J: the FP64 direct form of every point at its label, by groups of 16
    // lanes as above (whole rows, a fixed tree over the lanes)
    {
      const int grp = lane >> 4, sub = lane & 15, t0 = 8 * sub;
      const int64_t p0w = tile * 256 + (int64_t)wave * 64;
#pragma unroll 1
      for (int l0 = 0; l0 < 64; l0 += 4) {
        const int slot = l0 + grp;
        const bool ok = p0w + slot < n;
        const int j = ok ? (int)blab[wave][slot] : 0;
        const uint16_t* xr = X + (ok ? p0w + slot : 0) * d;
        const uint4 w = rows16 ? *reinterpret_cast<const uint4*>(xr + t0)
                               : __builtin_bit_cast(uint4, load8_bf16<uint16_t>(xr, t0, d, true));
        const uint32_t w4[4] = {w.x, w.y, w.z, w.w};
        const double* cj = b.c64 + (int64_t)j * d;
        double cv[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) cv[e] = cj[t0 + e < d ? t0 + e : 0];
        double part = 0.0;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const float xv = (e & 1) ? bf16_hi(w4[e >> 1]) : bf16_lo(w4[e >> 1]);
          const double df = t0 + e < d ? (double)xv - cv[e] : 0.0;
          part = __builtin_fma(df, df, part);
        }
        part += __shfl_xor(part, 8);
        part += __shfl_xor(part, 4);
        part += __shfl_xor(part, 2);
        part += __shfl_xor(part, 1);
        if (ok && sub == 0) Jacc += part;
      }
    }
    block_sum_J(Jacc, ucnt, pcnt, b.Jpart, b.upart, tile);
  }
}

// Exact cluster sums of the listed instances whose sums do not fit in LDS,
// from the labels the assignment launch wrote.  A work unit is a range of
// kBatchSumPts points and a range of skc centers: the block adds the rows of
// the points labelled inside its center range into an LDS table skc x (d+1)
// (64-bit integer atomics), then adds the table's non-zero entries into the
// instance's slot row.  Each point is read once, by the unit of its center
// range; integer sums do not depend on the order.  A wave takes 64 labels at a
// time and moves the selected points four at once (16 lanes a point, 8 dims a
// lane), four such groups in flight.  Persistent: blocks loop over the units.
__global__ __launch_bounds__(256) void k_batch_sums(const BatchHead* __restrict__ hd,
                                                    const BatchInst* __restrict__ bi) {
  extern __shared__ __align__(16) unsigned char smem[];
  unsigned long long* S = reinterpret_cast<unsigned long long*>(smem);
  __shared__ int order[4][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int grp = lane >> 4, sub = lane & 15;
  const int ninst = hd->ninst;
  const int64_t units = hd->units;
  for (int64_t u = blockIdx.x; u < units; u += gridDim.x) {
    const BatchInst& b = bi[batch_find(bi, ninst, u, 2)];
    PassState* st = b.st;
    if (b.mode != 1 || ld_agent(&st->done)) continue;
    const int d = b.d, k = b.k, kc = b.skc;
    const int nkr = (k + kc - 1) / kc;
    const int64_t local = u - b.sunit0;
    const int64_t pb = local / nkr;
    const int c0 = (int)(local - pb * nkr) * kc;
    const int cn = min(kc, k - c0);
    const int w = d + 1;
    for (int e = threadIdx.x; e < cn * w; e += 256) S[e] = 0ull;
    __syncthreads();
    const int64_t i0 = pb * kBatchSumPts, i1 = min(b.n, i0 + kBatchSumPts);
    const float sc = st->scale;
    const bool bf = b.dtype == 1;
    // whole 16-byte pieces of every row (8 BF16 or 2 x 4 FP32 dims)
    const bool vec = (d & 7) == 0 && (reinterpret_cast<uintptr_t>(b.X) & 15) == 0;
    const int32_t* lab = b.labels;
    for (int64_t g = i0 + (int64_t)wave * 64; g < i1; g += 256) {
      const int64_t i = g + lane;
      const int l = i < i1 ? lab[i] : -1;
      const bool sel = l >= c0 && l < c0 + cn;
      const unsigned long long m = __ballot(sel);
      const int cnt = __popcll(m);
      if (cnt == 0) continue;
      // the selected lanes in order: order[r] = lane of the r-th selected
      const int rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                 __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0));
      if (sel) order[wave][rank] = lane;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      for (int q0 = 0; q0 < cnt; q0 += 16) {
        constexpr int R = 4;
        long long qv[R][8];
        int lp[R];
        bool ok[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const int qi = q0 + 4 * r + grp;
          ok[r] = qi < cnt;
          const int src = ok[r] ? order[wave][qi] : 0;
          lp[r] = __shfl(l, src);
          const int64_t row = (g + src) * d;
          const int t0 = 8 * sub;
#pragma unroll
          for (int e = 0; e < 8; ++e) qv[r][e] = 0;
          if (ok[r] && t0 < d) {
            float xv[8];
            if (vec && bf) {
              const uint4 v = *reinterpret_cast<const uint4*>(
                  static_cast<const uint16_t*>(b.X) + row + t0);
              const uint32_t w4[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
              for (int e = 0; e < 4; ++e) {
                xv[2 * e] = bf16_lo(w4[e]);
                xv[2 * e + 1] = bf16_hi(w4[e]);
              }
            } else if (vec) {
              const float4 v0 = *reinterpret_cast<const float4*>(
                  static_cast<const float*>(b.X) + row + t0);
              const float4 v1 = *reinterpret_cast<const float4*>(
                  static_cast<const float*>(b.X) + row + t0 + 4);
              xv[0] = v0.x; xv[1] = v0.y; xv[2] = v0.z; xv[3] = v0.w;
              xv[4] = v1.x; xv[5] = v1.y; xv[6] = v1.z; xv[7] = v1.w;
            } else {
#pragma unroll
              for (int e = 0; e < 8; ++e) {
                const int t = t0 + e;
                xv[e] = t >= d ? 0.f
                        : bf ? __uint_as_float((uint32_t)static_cast<const uint16_t*>(b.X)[row + t]
                                               << 16)
                             : static_cast<const float*>(b.X)[row + t];
              }
            }
#pragma unroll
            for (int e = 0; e < 8; ++e) qv[r][e] = (long long)__float2int_rn(xv[e] * sc);
          }
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
          if (!ok[r]) continue;
          unsigned long long* Sr = S + (int64_t)(lp[r] - c0) * w;
#pragma unroll
          for (int e = 0; e < 8; ++e)
            if (8 * sub + e < d) atomicAdd(&Sr[8 * sub + e], (unsigned long long)qv[r][e]);
          if (sub == 0) atomicAdd(&Sr[d], 1ull);
        }
      }
      // order[] is rewritten by the next group of labels
      __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    unsigned long long* row = reinterpret_cast<unsigned long long*>(
        b.slots + (int64_t)(pb & (b.nslots - 1)) * k * w + (int64_t)c0 * w);
    for (int e = threadIdx.x; e < cn * w; e += 256) {
      const unsigned long long v = S[e];
      if (v) atomicAdd(&row[e], v);
    }
    __syncthreads();
  }
}

// Finalize entries of every listed instance (one per center), persistent.  The
// last entry of an instance concludes its pass (J, movement, stop test).
__global__ __launch_bounds__(256) void k_batch_finalize(const BatchHead* __restrict__ hd,
                                                        const BatchInst* __restrict__ bi) {
  const int ninst = hd->ninst;
  const int64_t centers = hd->centers;
  for (int64_t c = blockIdx.x; c < centers; c += gridDim.x) {
    const BatchInst& b = bi[batch_find(bi, ninst, c, 1)];
    const int dn = ld_agent(&b.st->done);
    if ((b.mode == 1 && dn) || (b.mode == 2 && dn == 2)) continue;
    finalize_center((int)(c - b.center0), b.slots, nullptr, b.k, b.d, b.st, b.mode == 1 ? 1 : 0,
                    b.c64, b.cw, b.cn, b.cnorm, b.shiftj, b.emptyj, nullptr, nullptr, b.cb16,
                    b.cnB, b.kd16, b.Jpart, b.upart, b.units, b.J_hist, b.shift_hist,
                    b.mode == 2, false, nullptr, nullptr, b.cb16lo, b.nslots);
  }
}

__global__ __launch_bounds__(256) void k_batch_status(const BatchHead* __restrict__ hd,
                                                      const BatchInst* __restrict__ bi,
                                                      BatchStatus* __restrict__ out) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= hd->ninst) return;
  const PassState* st = bi[i].st;
  BatchStatus r;
  r.done = st->done;
  r.iter = st->iter;
  r.converged = st->converged;
  r.empty = st->empty;
  r.nonfinite = st->nonfinite;
  r.pad = 0;
  r.J = st->J;
  r.shift = st->shift;
  r.uncertain = st->uncertain;
  out[i] = r;
}

// Uniform values in [-1, 1) from a counter-based hash (autotuning data), as
// FP32 (kind 0), BF16 bits (1) or FP64 (2).
__global__ __launch_bounds__(256) void k_fill_uniform(void* __restrict__ p, int64_t count,
                                                      uint64_t seed, int kind) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * 256) {
    uint64_t z = seed + (uint64_t)(i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    const double v = (double)(z >> 11) * 0x1p-52 - 1.0;
    if (kind == 0) static_cast<float*>(p)[i] = (float)v;
    else if (kind == 1) static_cast<uint16_t*>(p)[i] = f32_to_bf16((float)v);
    else static_cast<double*>(p)[i] = v;
  }
}

// BF16 copy of -2 c (dims padded with zeros to kd16) and ||c||^2 + B; the
// largest rounding-error norm of a row becomes st->dcn (the last block
// publishes it).
__global__ __launch_bounds__(64) void k_prep_bf16(const double* __restrict__ c64, int k, int d,
                                                  int kd16, PassState* __restrict__ st,
                                                  uint16_t* __restrict__ cb16,
                                                  float* __restrict__ cnB,
                                                  uint16_t* __restrict__ cb16lo) {
  const int j = blockIdx.x, lane = threadIdx.x;
  double acc = 0.0, e2 = 0.0;
  for (int t = lane; t < kd16; t += 64) {
    const double c = (t < d && j < k) ? c64[(int64_t)j * d + t] : 0.0;
    double e;
    if (cb16lo) {
      uint16_t hi, lo;
      e = bf16_split(c, hi, lo);
      cb16[cb16_at(j, t, kd16)] = hi;
      cb16lo[cb16_at(j, t, kd16)] = lo;
    } else {
      const uint16_t b = f32_to_bf16((float)(-2.0 * c));
      cb16[cb16_at(j, t, kd16)] = b;
      e = bf16_err(b, c);
    }
    acc += c * c;
    e2 += e * e;
  }
  for (int o = 32; o > 0; o >>= 1) {
    acc += __shfl_xor(acc, o);
    e2 += __shfl_xor(e2, o);
  }
  if (lane == 0) {
    cnB[j] = j < k ? (float)(acc + (double)st->B) : INFINITY;
    dcn_max(st, e2);
    __threadfence();
    if (atomicAdd(&st->ticket, 1u) == gridDim.x - 1) {
      __threadfence();
      dcn_publish(st);
      st->ticket = 0u;
    }
  }
}

hipError_t prep_bf16(const double* c64, int32_t k, int32_t d, int kd16, PassState* st,
                     uint16_t* cb16, float* cnB, hipStream_t s, uint16_t* cb16lo) {
  hipLaunchKernelGGL(k_prep_bf16, dim3((unsigned)bf16_rows(k)), dim3(64), 0, s, c64, k, d, kd16,
                     st, cb16, cnB, cb16lo);
  return hipGetLastError();
}

// ============================================================================
// Plans and pass launchers
// ============================================================================
static int pick_dmax(int d) {
  if (d <= 2) return 2;
  if (d <= 4) return 4;
  if (d <= 8) return 8;
  if (d <= 16) return 16;
  if (d <= 32) return 32;
  if (d <= 64) return 64;
  if (d <= 128) return 128;
  return 0;
}

static int pick_ppt(int dmax) {
  if (dmax == 0) return 1;
  if (dmax <= 8) return 4;
  if (dmax == 16) return 2;
  return 1;
}

// Calls f with the kernel instance for the plan (function pointer).
template <typename T, int KD, bool FULL, typename F>
static void visit_mfma_nt(int nt, F&& f) {
  switch (nt) {
    case 1: f(k_fused_mfma<T, KD, 1, FULL>); break;
    case 2: f(k_fused_mfma<T, KD, 2, FULL>); break;
    case 3: f(k_fused_mfma<T, KD, 3, FULL>); break;
    default: f(k_fused_mfma<T, KD, 4, FULL>); break;
  }
}

template <typename T, typename F>
static void visit_mfma(int kd, int nt, bool full, F&& f) {
  switch (kd) {
    case 2: full ? visit_mfma_nt<T, 2, true>(nt, f) : visit_mfma_nt<T, 2, false>(nt, f); break;
    case 4: full ? visit_mfma_nt<T, 4, true>(nt, f) : visit_mfma_nt<T, 4, false>(nt, f); break;
    case 8: full ? visit_mfma_nt<T, 8, true>(nt, f) : visit_mfma_nt<T, 8, false>(nt, f); break;
    case 16: full ? visit_mfma_nt<T, 16, true>(nt, f) : visit_mfma_nt<T, 16, false>(nt, f); break;
    default: full ? visit_mfma_nt<T, 32, true>(nt, f) : visit_mfma_nt<T, 32, false>(nt, f); break;
  }
}

template <typename T, int KD, bool FULL, typename F>
static void visit_fscreen_nt(int nt, F&& f) {
  switch (nt) {
    case 1: f(k_fused_screen<T, KD, 1, FULL>); break;
    case 2: f(k_fused_screen<T, KD, 2, FULL>); break;
    case 3: f(k_fused_screen<T, KD, 3, FULL>); break;
    default: f(k_fused_screen<T, KD, 4, FULL>); break;
  }
}

template <typename T, typename F>
static void visit_fscreen(int kd, int nt, bool full, F&& f) {
  switch (kd) {
    case 2: full ? visit_fscreen_nt<T, 2, true>(nt, f) : visit_fscreen_nt<T, 2, false>(nt, f); break;
    case 4: full ? visit_fscreen_nt<T, 4, true>(nt, f) : visit_fscreen_nt<T, 4, false>(nt, f); break;
    case 8: full ? visit_fscreen_nt<T, 8, true>(nt, f) : visit_fscreen_nt<T, 8, false>(nt, f); break;
    default: full ? visit_fscreen_nt<T, 16, true>(nt, f) : visit_fscreen_nt<T, 16, false>(nt, f); break;
  }
}

template <typename T, int KD, bool FULL, typename F>
static void visit_pair_nt(int nt, F&& f) {
  switch (nt) {
    case 1: f(k_fused_pair<T, KD, 1, FULL>); break;
    case 2: f(k_fused_pair<T, KD, 2, FULL>); break;
    case 3: f(k_fused_pair<T, KD, 3, FULL>); break;
    default: f(k_fused_pair<T, KD, 4, FULL>); break;
  }
}

template <typename T, typename F>
static void visit_pair(int kd, int nt, bool full, F&& f) {
  switch (kd) {
    case 4: full ? visit_pair_nt<T, 4, true>(nt, f) : visit_pair_nt<T, 4, false>(nt, f); break;
    case 8: full ? visit_pair_nt<T, 8, true>(nt, f) : visit_pair_nt<T, 8, false>(nt, f); break;
    default: full ? visit_pair_nt<T, 16, true>(nt, f) : visit_pair_nt<T, 16, false>(nt, f); break;
  }
}

template <typename T, typename F>
static void visit_fused(int dmax, F&& f) {
  switch (dmax) {
    case 2: f(k_fused<T, 2, 4>); break;
    case 4: f(k_fused<T, 4, 4>); break;
    case 8: f(k_fused<T, 8, 4>); break;
    case 16: f(k_fused<T, 16, 2>); break;
    case 32: f(k_fused<T, 32, 1>); break;
    case 64: f(k_fused<T, 64, 1>); break;
    default: f(k_fused<T, 128, 1>); break;
  }
}

template <typename T, typename F>
static void visit_tiled(int dmax, F&& f) {
  switch (dmax) {
    case 2: f(k_assign_tiled<T, 2, 4>); break;
    case 4: f(k_assign_tiled<T, 4, 4>); break;
    case 8: f(k_assign_tiled<T, 8, 4>); break;
    case 16: f(k_assign_tiled<T, 16, 2>); break;
    case 32: f(k_assign_tiled<T, 32, 1>); break;
    case 64: f(k_assign_tiled<T, 64, 1>); break;
    default: f(k_assign_tiled<T, 128, 1>); break;
  }
}

// Resident blocks of 256 threads per CU for a kernel with `lds` bytes of dynamic LDS.
template <typename K>
static int64_t resident_blocks(K kernel, size_t lds, int cus, int threads = 256) {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, threads, lds) != hipSuccess ||
      nb < 1)
    nb = 1;
  return (int64_t)nb * std::max(1, cus);
}

// Screen kernel for ks 16-dim K steps: PT point tiles per wave, NW waves a block.
template <typename T, typename F>
static void visit_screen(int ks, F&& f, bool r16 = false) {
  if constexpr (sizeof(T) == 2) {
    if (r16) {
      switch (ks) {
        case 1: f(k_screen_bf16<T, 1, 2, 4, true>); return;
        case 2: f(k_screen_bf16<T, 2, 2, 4, true>); return;
        case 4: f(k_screen_bf16<T, 4, 1, 8, true>); return;
        case 8: f(k_screen_bf16<T, 8, 2, 8, true>); return;
        default: f(k_screen_bf16<T, 16, 1, 8, true>); return;
      }
    }
  }
  switch (ks) {
    case 1: f(k_screen_bf16<T, 1, 2, 4>); break;
    case 2: f(k_screen_bf16<T, 2, 2, 4>); break;
    case 4: f(k_screen_bf16<T, 4, 1, 8>); break;
    case 8: f(k_screen_bf16<T, 8, 2, 8>); break;
    default: f(k_screen_bf16<T, 16, 1, 8>); break;
  }
}
// The screen's whole-row loads apply: BF16 rows of exactly ks*16 dims, 16-byte aligned.
static bool screen_r16(int dtype, int32_t d, int ks, const void* X) {
  return dtype == 1 && d == ks * 16 && (reinterpret_cast<uintptr_t>(X) & 15u) == 0;
}
// threads (64 NW) and points (NW PT 32) per block of the screen for each K-step count
constexpr int screen_threads(int ks) { return (ks == 4 || ks >= 8) ? 512 : 256; }
constexpr int screen_points(int ks) { return ks == 8 ? 512 : 256; }

template <typename T, typename F>
static void visit_rescreen(int ks, F&& f) {
  switch (ks) {
    case 1: f(k_rescreen_bf16<T, 1, 2>); break;
    case 2: f(k_rescreen_bf16<T, 2, 2>); break;
    case 4: f(k_rescreen_bf16<T, 4, 2>); break;
    case 8: f(k_rescreen_bf16<T, 8, 2>); break;
    default: f(k_rescreen_bf16<T, 16, 1>); break;
  }
}

template <typename T>
static int64_t plan_blocks(const PassPlan& p, int cus) {
  int64_t r = 0;
  auto f = [&](auto kern) { r = resident_blocks(kern, p.lds_assign, cus); };
  if (p.bf16)
    visit_screen<T>(
        p.ks, [&](auto kern) { r = resident_blocks(kern, 0, cus, screen_threads(p.ks)); },
        sizeof(T) == 2 && p.d == p.ks * 16);
  else if (p.fscreen && p.fsplit) visit_pair<T>(p.kd, p.nt, p.kd == p.d, f);
  else if (p.fscreen) visit_fscreen<T>(p.kd, p.nt, p.kd == p.d, f);
  else if (p.mfma) visit_mfma<T>(p.kd, p.nt, p.kd == p.d, f);
  else if (p.fused) visit_fused<T>(p.dmax, f);
  else if (p.dmax) visit_tiled<T>(p.dmax, f);
  else r = resident_blocks(k_assign_generic<T>, 0, cus);
  return r;
}

// Points per LDS-sorted range of k_lab_scatter_lds for k labels (its LDS, 3k + S
// words plus 4 static ones, within 64 KB; S a multiple of 256 in [4096, 2^14)),
// or 0 when k is too large and the plain scatter runs.
static int scatter_range(int k) {
  const int S = std::min((1 << 14) - 256, (16384 - 16 - 3 * k) / 256 * 256);
  return k >= 1 && S >= 4096 ? S : 0;
}

PassPlan plan_pass(int64_t rows, int32_t d, int32_t k, int dtype, int precision,
                   size_t lds_limit, int cus) {
  PassPlan p{};
  p.dmax = pick_dmax(d);
  p.ppt = pick_ppt(p.dmax);
  const size_t budget = std::min<size_t>(lds_limit, 65536);
  const size_t kk = (size_t)k, dd = (size_t)d;
  // BF16 screen: asked for, or automatic for BF16 data with d >= 32 (precision
  // codes follow km_precision: 0 auto, 1 FP32, 2 BF16 screen)
  const bool screen = precision == 2 || (precision == 0 && dtype == 1 && d >= 32);
  const bool small = d <= 16 && k <= 128 &&
                     kk * (size_t)(std::max(p.dmax, 2) + 2) * 8 + kk * (dd + 1) * 8 <= budget;
  // (the screen packs center indices into 27 bits)
  p.bf16 = d <= 256 && screen && !small && k < (1 << 27);
  if (p.bf16) {
    p.ks = d <= 16 ? 1 : d <= 32 ? 2 : d <= 64 ? 4 : d <= 128 ? 8 : 16;
    p.dmax = 0;
  }
  // fused MFMA passes (d <= 32, k <= 128): FP64 centers padded to the kernel's
  // dims, and the sums with counts
  // (center rows of the fused MFMA and screen passes: kd + 2 doubles)
  const size_t lds_mfma = kk * (size_t)(std::max(p.dmax, 2) + 2) * 8 + kk * (dd + 1) * 8;
  const size_t lds_fused = ((kk * (size_t)p.dmax + kk) * 4 + 15) / 16 * 16 + kk * (dd + 1) * 8;
  int64_t work = 1;  // independent units of the assignment kernel (waves' tiles)
  if (p.bf16) {
    work = (rows + screen_points(p.ks) - 1) / screen_points(p.ks);
  } else if (small && (screen || precision == 0)) {
    // small d: the fused pass scores on the BF16 matrix cores (certified).
    // Asked for the BF16 screen: one BF16 product per dim, whose band
    // (||x|| ||c|| 2^-7) sends many points of close clusters to FP64 decisions.
    // Auto precision: the split screen (c'hi x^ + c'lo x^ + c'hi xlo), whose
    // band is close to an FP32 one, at a fraction of the matrix-core time of
    // the FP32 MFMA pass, and BF16 MFMAs run beside the VALU work.
    p.fscreen = true;
    p.fsplit = !screen;
    p.fused = true;
    p.ks = 1;
    // the split screen runs on pairs of 32-point tiles, whole packed words per
    // lane half (at least 4 dims)
    p.kd = p.fsplit ? std::max(p.dmax, 4) : p.dmax;
    p.d = d;
    p.nt = (k + 31) / 32;
    p.lds_assign = kk * (size_t)(std::max(p.kd, 2) + 2) * 8 + kk * (dd + 1) * 8;
    if (p.fsplit) {
      // the paired-tile kernel: center rows of kd + 2 doubles, then its A
      // operands and C input
      const size_t nm = (size_t)((dtype == 0 ? 3 : 2) * (p.kd / 2) + 7) / 8;
      p.lds_assign = (kk * (size_t)(p.kd + 2) * 8 + kk * (dd + 1) * 8 + 15) / 16 * 16 +
                     (size_t)p.nt * nm * 64 * 16 + (size_t)p.nt * 32 * 4;
    }
    work = p.fsplit ? ((rows + 63) / 64 + 3) / 4 : ((rows + 31) / 32 + 3) / 4;
  } else if (d <= 32 && k <= 128 && lds_mfma <= budget) {
    p.mfma = true;
    p.fused = true;
    p.kd = p.dmax;
    p.d = d;
    p.nt = (k + 31) / 32;
    p.lds_assign = lds_mfma;
    work = ((rows + 31) / 32 + 3) / 4;
  }
  if (!p.mfma && !p.fscreen) {
    p.fused = !p.bf16 && p.dmax != 0 && lds_fused <= budget;
    const int64_t tile_pts = 256LL * p.ppt;
    if (!p.bf16) work = (rows + tile_pts - 1) / tile_pts;
    if (p.fused) {
      p.lds_assign = lds_fused;
      p.ktile = k;
    } else {
      if (p.dmax) {
        p.ktile = (int)std::max<int64_t>(1, std::min<int64_t>(k, 8192 / p.dmax));
        p.lds_assign = (size_t)p.ktile * p.dmax * 4 + (size_t)p.ktile * 4;
      }
      // sorted update: label counts per chunk of points, about 2^22 (label,
      // chunk) pairs at most; lane groups of pg positions, about 65536 groups
      const int64_t want = (int64_t)(((double)rows * (double)k) / (double)(1 << 22)) + 1;
      p.sort_chunk = std::max<int64_t>(4096, (want + 255) / 256 * 256);
      // chunks of at least one LDS-sorted range (longer runs of one label in
      // the scatter's writes) while that leaves 512 chunks or more
      const int64_t S = scatter_range(k);
      if (S > 0)
        p.sort_chunk = std::max(p.sort_chunk, std::min(S, rows / 512 / 256 * 256));
      p.sort_chunks = (rows + p.sort_chunk - 1) / p.sort_chunk;
      p.pg = std::min<int64_t>(1 << 13, std::max<int64_t>(64, (rows + 65535) / 65536));
      // every group walks pg positions, so the groups are sized to fill whole
      // generations of resident run-sum blocks (a last, partly filled one
      // leaves most of the GPU idle); rows of whole 16-byte pieces assumed,
      // and any pg in [64, 2^13] is correct
      const int E = dtype == 0 ? 4 : 8;
      if (((int64_t)d * (dtype == 0 ? 4 : 2)) % 16 == 0) {
        const int glog = row_glog(d, E);
        const int64_t ncb = (d + (E << glog) - 1) / (E << glog);
        const int64_t res = dtype == 0 ? resident_blocks(k_run_sums<float, 4>, 0, cus)
                                       : resident_blocks(k_run_sums<uint16_t, 8>, 0, cus);
        const int64_t gpg = std::max<int64_t>(1, res / ncb) * 4 * (64 >> glog);
        int64_t gens = std::max<int64_t>(1, (65536 + gpg / 2) / gpg);
        gens = std::max(gens, (rows + gpg * 8192 - 1) / (gpg * 8192));
        p.pg = std::min<int64_t>(1 << 13,
                                 std::max<int64_t>(64, (rows + gens * gpg - 1) / (gens * gpg)));
      }
    }
  }
  // a persistent grid: no more blocks than stay resident at once
  const int64_t res = dtype == 0 ? plan_blocks<float>(p, cus) : plan_blocks<uint16_t>(p, cus);
  p.blocks = std::max<int64_t>(1, std::min<int64_t>({work, res, (int64_t)kMaxBlocks}));
  if (p.bf16) {
    // the re-rank's blocks walk ranges of the points in a grid-stride loop:
    // all of them resident, so none waits for a second round of blocks
    auto rr = [&](auto kern) { return resident_blocks(kern, 0, cus); };
    if (dtype == 0)
      p.rr_blocks = p.ks <= 8 ? rr(k_rerank_list<float, 8>) : rr(k_rerank_list<float, 16>);
    else
      p.rr_blocks = p.ks <= 8 ? rr(k_rerank_list<uint16_t, 8>) : rr(k_rerank_list<uint16_t, 16>);
  }
  return p;
}

template <typename T>
static void dispatch_fused(const PassBufs& b, const PassPlan& p, bool update,
                           const int32_t* gate, hipStream_t s) {
  auto launch = [&](auto kern) {
    hipLaunchKernelGGL(kern, dim3((unsigned)p.blocks), dim3(256), p.lds_assign, s, (const T*)b.X,
                       b.n, b.d, b.k, b.cw, b.cn, b.c64, (const PassState*)b.st, gate,
                       update ? 1 : 0, b.slots, b.Jpart, b.upart, b.labels);
  };
  if (p.fscreen && p.fsplit) {
    visit_pair<T>(p.kd, p.nt, full_row_ok<T>(p.kd, b.d, b.X), [&](auto kern) {
      hipLaunchKernelGGL(kern, dim3((unsigned)p.blocks), dim3(256), p.lds_assign, s,
                         (const T*)b.X, b.n, b.d, b.k, (const float*)b.cnB,
                         (const double*)b.c64, (const PassState*)b.st, gate, update ? 1 : 0,
                         b.slots, b.Jpart, b.upart, b.labels);
    });
  } else if (p.fscreen) {
    visit_fscreen<T>(p.kd, p.nt, full_rows_ok<T>(p.kd, b.d, b.X), [&](auto kern) {
      hipLaunchKernelGGL(kern, dim3((unsigned)p.blocks), dim3(256), p.lds_assign, s,
                         (const T*)b.X, b.n, b.d, b.k, (const float*)b.cnB, (const double*)b.c64, (const PassState*)b.st,
                         gate, update ? 1 : 0, b.slots, b.Jpart, b.upart, b.labels);
    });
  } else if (p.mfma) {
    visit_mfma<T>(p.kd, p.nt, full_rows_ok<T>(p.kd, b.d, b.X), launch);
  } else {
    visit_fused<T>(p.dmax, launch);
  }
}

template <typename T>
static void dispatch_tiled(const PassBufs& b, const PassPlan& p, const int32_t* gate,
                           int wantJ, hipStream_t s) {
  if (p.dmax) {
    visit_tiled<T>(p.dmax, [&](auto kern) {
      hipLaunchKernelGGL(kern, dim3((unsigned)p.blocks), dim3(256), p.lds_assign, s,
                         (const T*)b.X, b.n, b.d, b.k, p.ktile, b.cw, b.cn, b.c64,
                         (const PassState*)b.st, gate, b.Jpart, b.upart, b.labels, wantJ);
    });
  } else {
    hipLaunchKernelGGL(k_assign_generic<T>, dim3((unsigned)p.blocks), dim3(256), 0, s,
                       (const T*)b.X, b.n, b.d, b.k, b.cw, b.cn, b.c64, (const PassState*)b.st,
                       gate, b.Jpart, b.upart, b.labels, wantJ);
  }
}

int row_vec(int dtype, int32_t d, const void* X);
int row_glog(int32_t d, int E);

// Counting sort of the point indices by label, then the run sums.
static void sorted_update(const PassBufs& b, const PassPlan& p, const int32_t* gate,
                          hipStream_t s) {
  const int64_t G = p.sort_chunks, cn = (int64_t)b.k * G;
  const size_t lds = b.k <= kHistLds ? (size_t)b.k * 4 : 0;
  if (!lds) (void)zero_i64(b.scnt, cn, s);
  hipLaunchKernelGGL(k_lab_count, dim3((unsigned)G), dim3(256), lds, s, (const int32_t*)b.labels,
                     b.n, b.k, p.sort_chunk, G, b.scnt, gate);
  const int64_t tiles = (cn + 2047) / 2048;
  hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)tiles), dim3(256), 0, s, b.scnt, cn, b.stot,
                     gate);
  hipLaunchKernelGGL(k_scan_excl, dim3(1), dim3(256), 0, s, reinterpret_cast<int64_t*>(b.stot),
                     tiles);
  hipLaunchKernelGGL(k_scan_add, dim3((unsigned)((cn + 255) / 256)), dim3(256), 0, s, b.scnt, cn,
                     (const long long*)b.stot, gate);
  hipLaunchKernelGGL(k_run_starts, dim3((unsigned)((b.k + 256) / 256)), dim3(256), 0, s,
                     (const long long*)b.scnt, b.k, G, b.n, b.rstart, gate);
  const int S = scatter_range(b.k);
  if (S > 0)
    hipLaunchKernelGGL(k_lab_scatter_lds, dim3((unsigned)G), dim3(256),
                       (size_t)(3 * b.k + S) * 4, s, (const int32_t*)b.labels, b.n, b.k,
                       p.sort_chunk, G, S, (const long long*)b.scnt, b.perm, gate);
  else
    hipLaunchKernelGGL(k_lab_scatter, dim3((unsigned)G), dim3(256), lds, s,
                       (const int32_t*)b.labels, b.n, b.k, p.sort_chunk, G, b.scnt, b.perm,
                       gate);
  const int E = row_vec(b.dtype, b.d, b.X), glog = row_glog(b.d, E);
  const int64_t groups = (b.n + p.pg - 1) / p.pg;
  const int64_t waves = (groups + (64 >> glog) - 1) / (64 >> glog);
  const unsigned ncb = (unsigned)((b.d + (E << glog) - 1) / (E << glog));
  const dim3 grid((unsigned)((waves + 3) / 4), ncb);
  auto go = [&](auto kern, auto* x) {
    hipLaunchKernelGGL(kern, grid, dim3(256), 0, s, x, b.n, b.d, b.k, glog, p.pg,
                       (const uint32_t*)b.perm, (const long long*)b.rstart,
                       (const double*)b.c64, (const PassState*)b.st, gate, b.slots, b.jslots);
  };
  if (b.dtype == 0) {
    if (E == 4) go(k_run_sums<float, 4>, (const float*)b.X);
    else go(k_run_sums<float, 1>, (const float*)b.X);
  } else {
    if (E == 8) go(k_run_sums<uint16_t, 8>, (const uint16_t*)b.X);
    else go(k_run_sums<uint16_t, 1>, (const uint16_t*)b.X);
  }
}

template <typename T>
static void dispatch_bf16(const PassBufs& b, const PassPlan& p, const int32_t* gate,
                          hipStream_t s) {
  visit_screen<T>(
      p.ks,
      [&](auto kern) {
        hipLaunchKernelGGL(kern, dim3((unsigned)p.blocks), dim3(screen_threads(p.ks)), 0, s,
                           (const T*)b.X, b.n, b.d, b.k, (const uint16_t*)b.cb16,
                           (const float*)b.cnB, (const float*)b.cw, (const double*)b.c64, b.st,
                           gate, b.labels, b.queue, b.qthr, b.rq_c, b.Jpart, b.upart);
      },
      screen_r16(sizeof(T) == 2 ? 1 : 0, b.d, p.ks, b.X));
}

// The screen's re-rank list, in FP64.
template <typename T>
static void dispatch_rerank(const PassBufs& b, const PassPlan& p, const int32_t* gate,
                            hipStream_t s) {
  // ranges of 4096 points, one block each (no more blocks than stay resident)
  const int64_t cap = p.rr_blocks > 0 ? std::min<int64_t>(p.rr_blocks, 2048) : 2048;
  const unsigned g = (unsigned)std::max<int64_t>(1, std::min<int64_t>((b.n + 4095) / 4096, cap));
  auto go = [&](auto kern) {
    hipLaunchKernelGGL(kern, dim3(g), dim3(256), 0, s, (const T*)b.X, b.n, b.d, b.k,
                       (const float*)b.cw, (const double*)b.c64, (const PassState*)b.st, gate,
                       b.labels, (const int4*)b.rq_c, (long long*)nullptr);
  };
  if (p.ks <= 8) go(k_rerank_list<T, 8>);
  else go(k_rerank_list<T, 16>);
}

// The points with more than four candidates, re-screened (the second half of
// the per-block counters is theirs).
template <typename T>
static void dispatch_rescreen(const PassBufs& b, const PassPlan& p, const int32_t* gate,
                              hipStream_t s) {
  visit_rescreen<T>(p.ks, [&](auto kern) {
    hipLaunchKernelGGL(kern, dim3((unsigned)p.blocks), dim3(512), 0, s, (const T*)b.X, b.d, b.k,
                       (const uint16_t*)b.cb16, (const float*)b.cnB, (const float*)b.cw,
                       (const double*)b.c64, b.st, gate, b.labels, (const uint32_t*)b.queue,
                       (const float*)b.qthr, b.Jpart + p.blocks, b.upart + 2 * p.blocks);
  });
}

hipError_t pass_assign(const PassBufs& b, const PassPlan& p, bool update, hipStream_t s) {
  const int32_t* gate = update ? &b.st->done : nullptr;
  if (p.bf16) {
    if (b.dtype == 0) dispatch_bf16<float>(b, p, gate, s);
    else dispatch_bf16<uint16_t>(b, p, gate, s);
  } else if (p.fused) {
    if (b.dtype == 0) dispatch_fused<float>(b, p, update, gate, s);
    else dispatch_fused<uint16_t>(b, p, update, gate, s);
  } else {
    // an update pass takes J from the sorted update
    if (b.dtype == 0) dispatch_tiled<float>(b, p, gate, update ? 0 : 1, s);
    else dispatch_tiled<uint16_t>(b, p, gate, update ? 0 : 1, s);
  }
  return hipGetLastError();
}

hipError_t pass_rest(const PassBufs& b, const PassPlan& p, bool update, hipStream_t s) {
  const int32_t* gate = update ? &b.st->done : nullptr;
  const int64_t nb = p.bf16 ? 2 * p.blocks : p.blocks;
  if (p.bf16) {
    if (b.dtype == 0) {
      dispatch_rerank<float>(b, p, gate, s);
      dispatch_rescreen<float>(b, p, gate, s);
    } else {
      dispatch_rerank<uint16_t>(b, p, gate, s);
      dispatch_rescreen<uint16_t>(b, p, gate, s);
    }
  }
  // The sorted update makes the sums of an update pass and, with the BF16
  // screen, J of every pass; the FP32 kernels add J themselves in a labelling
  // pass.
  const bool sorted = !p.fused && (update || p.bf16);
  if (sorted) sorted_update(b, p, gate, s);
  if (update || sorted) {
    hipLaunchKernelGGL(k_finalize, dim3((unsigned)b.k), dim3(256), 0, s, b.slots,
                       sorted ? b.jslots : nullptr, b.k, b.d, b.st, gate, update ? 1 : 0, b.c64,
                       b.cw, b.cn, b.cnorm, b.shiftj, b.emptyj, b.S_out, b.N_out,
                       copy16(p) ? b.cb16 : nullptr, copy16(p) ? b.cnB : nullptr, p.ks * 16,
                       (const double*)b.Jpart, (const long long*)b.upart, nb, b.J_hist,
                       b.shift_hist, (p.fscreen && p.fsplit) ? 1 : 0, b.trace_c, b.trace_n);
    if (update && b.fpart) {
      // re-seeding: both kernels return at once unless this pass left a cluster empty
      const unsigned g = (unsigned)std::max<int64_t>(1, std::min<int64_t>((b.n + 255) / 256,
                                                                            kFarBlocks));
      auto far = [&](auto* x) {
        using T = std::remove_const_t<std::remove_pointer_t<decltype(x)>>;
        hipLaunchKernelGGL(k_farthest<T>, dim3(g), dim3(256), 0, s, x, b.n, b.d, b.k,
                           (const double*)b.c64, (const PassState*)b.st, b.fpart, b.fidx);
        hipLaunchKernelGGL(k_reseed<T>, dim3(1), dim3(256), 0, s, x, b.d, b.k, b.c64, b.cw, b.cn,
                           b.cnorm, copy16(p) ? b.cb16 : nullptr, copy16(p) ? b.cnB : nullptr,
                           p.ks * 16, b.st, (const double*)b.fpart, (const long long*)b.fidx,
                           (int)g, b.shift_hist);
      };
      if (b.dtype == 0) far((const float*)b.X);
      else far((const uint16_t*)b.X);
    }
  } else {
    hipLaunchKernelGGL(k_sum_J, dim3(1), dim3(256), 0, s, b.st, (const double*)b.Jpart,
                       (const long long*)b.upart, nb);
  }
  return hipGetLastError();
}

// --------------------------------------------------------------- batched
int batch_dmax(int32_t d) { return pick_dmax(d); }

// Register tiles of the batched assignment: points per thread for each dmax.
template <typename T, typename F>
static bool visit_batch(int dmax, int ppt, F&& f) {
#define KM_BATCH(DM, PP)                  \
  if (dmax == DM && ppt == PP) {          \
    f(k_batch_assign<T, DM, PP>);         \
    return true;                          \
  }
  KM_BATCH(2, 2) KM_BATCH(2, 4) KM_BATCH(4, 2) KM_BATCH(4, 4) KM_BATCH(8, 2) KM_BATCH(8, 4)
  KM_BATCH(16, 1) KM_BATCH(16, 2) KM_BATCH(32, 1) KM_BATCH(64, 1) KM_BATCH(128, 1)
#undef KM_BATCH
  return false;
}

int batch_screen_ks(int dtype, int32_t d, int32_t k) {
  if (dtype != 1 || d <= 16 || d > 128 || k > 256) return 0;
  return d <= 32 ? 2 : d <= 64 ? 4 : 8;
}

template <typename F>
static bool visit_batch_screen(int ks, F&& f) {
  switch (ks) {
    case 2: f(k_batch_screen<2>); return true;
    case 4: f(k_batch_screen<4>); return true;
    case 8: f(k_batch_screen<8>); return true;
    default: return false;
  }
}

int64_t batch_resident_blocks(int dtype, int dmax, int ppt, size_t lds, int cus, int screen) {
  int64_t r = 0;
  auto f = [&](auto kern) { r = resident_blocks(kern, lds, cus); };
  if (screen) return visit_batch_screen(screen, f) ? r : 0;
  const bool ok = dtype == 0 ? visit_batch<float>(dmax, ppt, f) : visit_batch<uint16_t>(dmax, ppt, f);
  return ok ? r : 0;
}

hipError_t batch_assign(const BatchHead* hd, const BatchInst* bi, const BatchShape& sh,
                        hipStream_t s) {
  auto f = [&](auto kern) {
    hipLaunchKernelGGL(kern, dim3((unsigned)sh.blocks), dim3(256), sh.lds, s, hd, bi);
  };
  const bool ok = sh.screen ? visit_batch_screen(sh.screen, f)
                  : sh.dtype == 0 ? visit_batch<float>(sh.dmax, sh.ppt, f)
                                  : visit_batch<uint16_t>(sh.dmax, sh.ppt, f);
  if (!ok) return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t batch_sums(const BatchHead* hd, const BatchInst* bi, int blocks, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_sums, dim3((unsigned)std::max(1, blocks)), dim3(256),
                     kBatchSumLds, s, hd, bi);
  return hipGetLastError();
}

hipError_t batch_finalize(const BatchHead* hd, const BatchInst* bi, int blocks, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_finalize, dim3((unsigned)std::max(1, blocks)), dim3(256), 0, s, hd,
                     bi);
  return hipGetLastError();
}

hipError_t batch_status(const BatchHead* hd, const BatchInst* bi, BatchStatus* out,
                        hipStream_t s) {
  // up to 65536 instances per table
  hipLaunchKernelGGL(k_batch_status, dim3(256), dim3(256), 0, s, hd, bi, out);
  return hipGetLastError();
}

hipError_t fill_uniform(void* p, int kind, int64_t count, uint64_t seed, hipStream_t s) {
  const unsigned g = (unsigned)std::max<int64_t>(1, std::min<int64_t>((count + 255) / 256, 4096));
  hipLaunchKernelGGL(k_fill_uniform, dim3(g), dim3(256), 0, s, p, count, seed, kind);
  return hipGetLastError();
}

hipError_t lloyd_pass(const PassBufs& b, const PassPlan& p, bool update, hipStream_t s) {
  hipError_t e = pass_assign(b, p, update, s);
  if (e != hipSuccess) return e;
  return pass_rest(b, p, update, s);
}

hipError_t assign_only(const PassBufs& b, const PassPlan& p, hipStream_t s) {
  return lloyd_pass(b, p, false, s);
}

}  // namespace km
