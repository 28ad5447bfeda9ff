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
  st->done = 0;
}

hipError_t stage_reset(PassState* st, hipStream_t s) {
  hipLaunchKernelGGL(k_stage_reset, dim3(1), dim3(1), 0, s, st);
  return hipGetLastError();
}

template <typename T>
__global__ __launch_bounds__(256) void k_max_abs(const T* __restrict__ X, int64_t count,
                                                 PassState* __restrict__ st) {
  uint32_t mx = 0u;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count; e += stride) {
    uint32_t b = __float_as_uint(widen<T>(X[e])) & 0x7fffffffu;  // |x|; NaN/Inf >= 0x7f800000
    mx = max(mx, b);
  }
  for (int o = 32; o > 0; o >>= 1) mx = max(mx, (uint32_t)__shfl_xor((int)mx, o));
  __shared__ uint32_t w[4];
  if ((threadIdx.x & 63) == 0) w[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t v = max(max(w[0], w[1]), max(w[2], w[3]));
    atomicMax(&st->maxabs_bits, v);
  }
}

hipError_t max_abs(const void* X, int dtype, int64_t count, PassState* st, hipStream_t s) {
  const unsigned g = (unsigned)std::max<int64_t>(1, std::min<int64_t>((count + 255) / 256, 4096));
  if (dtype == 0)
    hipLaunchKernelGGL(k_max_abs<float>, dim3(g), dim3(256), 0, s, (const float*)X, count, st);
  else
    hipLaunchKernelGGL(k_max_abs<uint16_t>, dim3(g), dim3(256), 0, s, (const uint16_t*)X,
                       count, st);
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
                                                     int32_t k) {
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
    st->cmax = (float)(red[0] * (1.0 + 0x1p-20)) * (1.0f + 0x1p-20f);
    st->max_iter = max_iter;
    st->tol = tol;
    st->iter = 0;
    st->done = st->nonfinite ? 1 : 0;
    st->converged = 0;
    st->empty = 0;
    st->J = 0.0;
    st->shift = 0.0;
    st->uncertain = 0;
    st->rows = rows;
  }
}

hipError_t stage_begin(PassState* st, int32_t max_iter, double tol, int64_t rows,
                       const double* cnorm, int32_t k, hipStream_t s) {
  hipLaunchKernelGGL(k_stage_begin, dim3(1), dim3(256), 0, s, st, max_iter, tol, rows, cnorm, k);
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
  for (int t = 0; t < d; ++t) {
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
    unsigned long long* __restrict__ S, unsigned int* __restrict__ N,
    int32_t* __restrict__ labels, double& Jacc, int64_t& ucnt) {
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
    const double* cl = c64 + (int64_t)l * d;
    double D = 0.0;
#pragma unroll
    for (int t = 0; t < DMAX; ++t) {
      if (t < d) {
        const double diff = (double)x[p][t] - cl[t];
        D = D + diff * diff;
      }
    }
    Jacc += D;
    if (labels) labels[ip[p]] = l;
    if (S) {
#pragma unroll
      for (int t = 0; t < DMAX; ++t) {
        if (t < d) {
          const long long q = (long long)__float2int_rn(x[p][t] * scale);
          atomicAdd(&S[(int64_t)l * d + t], (unsigned long long)q);
        }
      }
      atomicAdd(&N[l], 1u);
    }
  }
}

// Fixed-order block sum of J (FP64) and the uncertain count.  256 threads.
__device__ __forceinline__ void block_sum_J(double Jacc, int64_t ucnt, double* Jpart,
                                            long long* upart) {
  __shared__ double wJ[4];
  __shared__ long long wU[4];
  for (int o = 32; o > 0; o >>= 1) Jacc += __shfl_xor(Jacc, o);
  // the fallback count is already wave-uniform
  if ((threadIdx.x & 63) == 0) {
    wJ[threadIdx.x >> 6] = Jacc;
    wU[threadIdx.x >> 6] = ucnt;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    Jpart[blockIdx.x] = ((wJ[0] + wJ[1]) + wJ[2]) + wJ[3];
    upart[blockIdx.x] = wU[0] + wU[1] + wU[2] + wU[3];
  }
}

// Fused pass for small k*d: assignment, J and LDS-private cluster sums; each
// block writes its sums to row blockIdx.x of `part` ([rows][k][d+1], counts last).
template <typename T, int DMAX, int P>
__global__ __launch_bounds__(256) void k_fused(
    const T* __restrict__ X, int64_t n, int d, int k, const float* __restrict__ cw,
    const float* __restrict__ cn, const double* __restrict__ c64, const PassState* __restrict__ st,
    const int32_t* __restrict__ gate, int update, long long* __restrict__ part,
    double* __restrict__ Jpart, long long* __restrict__ upart, int32_t* __restrict__ labels) {
  if (gated(gate)) return;
  extern __shared__ __align__(16) unsigned char smem[];
  float* w = reinterpret_cast<float*>(smem);
  float* cnl = w + (size_t)k * DMAX;
  unsigned long long* S =
      reinterpret_cast<unsigned long long*>(smem + (((size_t)k * DMAX + k) * 4 + 15) / 16 * 16);
  unsigned int* N = reinterpret_cast<unsigned int*>(S + (size_t)k * d);
  for (int e = threadIdx.x; e < k * DMAX; e += 256) {
    const int j = e / DMAX, t = e - j * DMAX;
    w[e] = t < d ? -2.f * cw[(int64_t)j * d + t] : 0.f;
  }
  for (int j = threadIdx.x; j < k; j += 256) cnl[j] = cn[j];
  if (update) {
    for (int e = threadIdx.x; e < k * d; e += 256) S[e] = 0ull;
    for (int j = threadIdx.x; j < k; j += 256) N[j] = 0u;
  }
  __syncthreads();
  const float scale = st->scale, cmax = st->cmax;
  double Jacc = 0.0;
  int64_t ucnt = 0;
  const int64_t tile = 256 * P;
  for (int64_t base = (int64_t)blockIdx.x * tile; base < n; base += (int64_t)gridDim.x * tile)
    assign_tile<T, DMAX, P, false>(X, n, d, k, base, cw, cn, c64, w, cnl, k, cmax, scale,
                                   update ? S : nullptr, update ? N : nullptr, labels, Jacc,
                                   ucnt);
  __syncthreads();
  if (update) {
    long long* pb = part + (int64_t)blockIdx.x * k * (d + 1);
    for (int e = threadIdx.x; e < k * d; e += 256) {
      const int j = e / d, t = e - j * d;
      pb[(int64_t)j * (d + 1) + t] = (long long)S[e];
    }
    for (int j = threadIdx.x; j < k; j += 256) pb[(int64_t)j * (d + 1) + d] = (long long)N[j];
  }
  block_sum_J(Jacc, ucnt, Jpart, upart);
}

// Assignment only, centers streamed through LDS by tiles; writes labels.
template <typename T, int DMAX, int P>
__global__ __launch_bounds__(256) void k_assign_tiled(
    const T* __restrict__ X, int64_t n, int d, int k, int ktile, const float* __restrict__ cw,
    const float* __restrict__ cn, const double* __restrict__ c64, const PassState* __restrict__ st,
    const int32_t* __restrict__ gate, double* __restrict__ Jpart, long long* __restrict__ upart,
    int32_t* __restrict__ labels) {
  if (gated(gate)) return;
  extern __shared__ __align__(16) unsigned char smem[];
  float* w = reinterpret_cast<float*>(smem);
  float* cnl = w + (size_t)ktile * DMAX;
  const float cmax = st->cmax;
  double Jacc = 0.0;
  int64_t ucnt = 0;
  const int64_t tile = 256 * P;
  for (int64_t base = (int64_t)blockIdx.x * tile; base < n; base += (int64_t)gridDim.x * tile)
    assign_tile<T, DMAX, P, true>(X, n, d, k, base, cw, cn, c64, w, cnl, ktile, cmax, 1.f,
                                  nullptr, nullptr, labels, Jacc, ucnt);
  block_sum_J(Jacc, ucnt, Jpart, upart);
}

// Rows with d above the largest register tile: one point per thread, the row
// read from memory (L1/L2) for every center.
template <typename T>
__global__ __launch_bounds__(256) void k_assign_generic(
    const T* __restrict__ X, int64_t n, int d, int k, const float* __restrict__ cw,
    const float* __restrict__ cn, const double* __restrict__ c64, const PassState* __restrict__ st,
    const int32_t* __restrict__ gate, double* __restrict__ Jpart, long long* __restrict__ upart,
    int32_t* __restrict__ labels) {
  if (gated(gate)) return;
  const float cmax = st->cmax;
  const float Kd = (float)(d + 2) * 0x1p-24f * 1.001f;
  double Jacc = 0.0;
  int64_t ucnt = 0;
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
    if (valid) {
      Jacc += dist64_row<T>(xr, c64 + (int64_t)bi * d, d);
      labels[i] = bi;
    }
  }
  block_sum_J(Jacc, ucnt, Jpart, upart);
}

// Cluster sums from labels for k*d too large for one LDS array: block (b, s, r)
// adds dims [s*slice, ...) of the points of block b whose label lies in
// center range r into LDS, then writes them to row b of `part`.
template <typename T>
__global__ __launch_bounds__(256) void k_update_split(
    const T* __restrict__ X, const int32_t* __restrict__ labels, int64_t n, int d, int k,
    int slice, int crange, const PassState* __restrict__ st, const int32_t* __restrict__ gate,
    long long* __restrict__ part) {
  if (gated(gate)) return;
  extern __shared__ __align__(16) unsigned char smem[];
  const int t0 = blockIdx.y * slice, tw = min(slice, d - t0);
  const int j0 = blockIdx.z * crange, jw = min(crange, k - j0);
  unsigned long long* S = reinterpret_cast<unsigned long long*>(smem);
  unsigned int* N = reinterpret_cast<unsigned int*>(S + (size_t)crange * slice);
  for (int e = threadIdx.x; e < jw * slice; e += 256) S[e] = 0ull;
  for (int j = threadIdx.x; j < jw; j += 256) N[j] = 0u;
  __syncthreads();
  const float scale = st->scale;
  const bool counts = blockIdx.y == 0;
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) {
    const int l = labels[i] - j0;
    if (l < 0 || l >= jw) continue;
    const T* xr = X + i * d + t0;
    for (int tt = 0; tt < tw; ++tt) {
      const long long q = (long long)__float2int_rn(widen<T>(xr[tt]) * scale);
      atomicAdd(&S[(int64_t)l * slice + tt], (unsigned long long)q);
    }
    if (counts) atomicAdd(&N[l], 1u);
  }
  __syncthreads();
  long long* pb = part + (int64_t)blockIdx.x * k * (d + 1);
  for (int e = threadIdx.x; e < jw * tw; e += 256) {
    const int jj = e / tw, tt = e - jj * tw;
    pb[(int64_t)(j0 + jj) * (d + 1) + t0 + tt] = (long long)S[(int64_t)jj * slice + tt];
  }
  if (counts)
    for (int jj = threadIdx.x; jj < jw; jj += 256)
      pb[(int64_t)(j0 + jj) * (d + 1) + d] = (long long)N[jj];
}

// ============================================================================
// Reduction of the block sums, new centers, stage bookkeeping
// ============================================================================
// part2[r][c] = sum over rows b = r, r+R, ... of part[b][c] (exact integer sums).
__global__ __launch_bounds__(256) void k_reduce_part(const long long* __restrict__ part,
                                                     int64_t rows, int64_t C, int R,
                                                     const int32_t* __restrict__ gate,
                                                     long long* __restrict__ part2) {
  if (gated(gate)) return;
  const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int r = blockIdx.y;
  if (c >= C) return;
  long long s = 0;
  for (int64_t b = r; b < rows; b += R) s += part[b * C + c];
  part2[(int64_t)r * C + c] = s;
}

// One wave per center: exact sums, new center (the average; an empty cluster
// keeps its center), its movement and norm.
__global__ __launch_bounds__(64) void k_finalize(
    const long long* __restrict__ part2, int R, int k, int d, const PassState* __restrict__ st,
    const int32_t* __restrict__ gate, double* __restrict__ c64, float* __restrict__ cw,
    float* __restrict__ cn, double* __restrict__ cnorm, double* __restrict__ shiftj,
    int32_t* __restrict__ emptyj, double* __restrict__ S_out, int64_t* __restrict__ N_out) {
  if (gated(gate)) return;
  const int j = blockIdx.x, lane = threadIdx.x;
  const int64_t C = (int64_t)k * (d + 1);
  const long long* col = part2 + (int64_t)j * (d + 1);
  long long Nj = 0;
  for (int r = 0; r < R; ++r) Nj += col[(int64_t)r * C + d];
  const int F = st->F;
  double sh = 0.0, nn = 0.0;
  for (int t = lane; t < d; t += 64) {
    long long Sj = 0;
    for (int r = 0; r < R; ++r) Sj += col[(int64_t)r * C + t];
    const double sum = ldexp((double)Sj, -F);
    const double cold = c64[(int64_t)j * d + t];
    const double cnew = Nj > 0 ? sum / (double)Nj : cold;
    const double diff = cnew - cold;
    sh += diff * diff;
    nn += cnew * cnew;
    c64[(int64_t)j * d + t] = cnew;
    cw[(int64_t)j * d + t] = (float)cnew;
    if (S_out) S_out[(int64_t)j * d + t] = sum;
  }
  for (int o = 32; o > 0; o >>= 1) {
    sh += __shfl_xor(sh, o);
    nn += __shfl_xor(nn, o);
  }
  if (lane == 0) {
    shiftj[j] = sqrt(sh);
    cn[j] = (float)nn;
    cnorm[j] = sqrt(nn);
    emptyj[j] = Nj == 0 ? 1 : 0;
    if (N_out) N_out[j] = (int64_t)Nj;
  }
}

// One block: J (fixed-order FP64 sum of the block partials), largest movement,
// empties, bound on ||c||, pass count and the stop decision.
__global__ __launch_bounds__(256) void k_conclude(
    PassState* __restrict__ st, const double* __restrict__ Jpart,
    const long long* __restrict__ upart, int64_t nb, const double* __restrict__ shiftj,
    const double* __restrict__ cnorm, const int32_t* __restrict__ emptyj, int k, int update,
    double* __restrict__ J_hist, double* __restrict__ shift_hist) {
  if (update && st->done) return;
  __shared__ double rJ[256], rS[256], rN[256];
  __shared__ long long rU[256], rE[256];
  const int tid = threadIdx.x;
  double J = 0.0;
  long long U = 0;
  for (int64_t b = tid; b < nb; b += 256) {
    J += Jpart[b];
    U += upart[b];
  }
  double sh = 0.0, nm = 0.0;
  long long E = 0;
  if (update)
    for (int j = tid; j < k; j += 256) {
      sh = fmax(sh, shiftj[j]);
      nm = fmax(nm, cnorm[j]);
      E += emptyj[j];
    }
  rJ[tid] = J; rU[tid] = U; rS[tid] = sh; rN[tid] = nm; rE[tid] = E;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (tid < o) {
      rJ[tid] += rJ[tid + o];
      rU[tid] += rU[tid + o];
      rS[tid] = fmax(rS[tid], rS[tid + o]);
      rN[tid] = fmax(rN[tid], rN[tid + o]);
      rE[tid] += rE[tid + o];
    }
    __syncthreads();
  }
  if (tid == 0) {
    st->J = rJ[0];
    st->uncertain += rU[0];
    if (update) {
      const int it = st->iter;
      st->shift = rS[0];
      st->empty = (int32_t)rE[0];
      st->cmax = (float)(rN[0] * (1.0 + 0x1p-20)) * (1.0f + 0x1p-20f);
      if (J_hist) J_hist[it] = rJ[0];
      if (shift_hist) shift_hist[it] = rS[0];
      st->iter = it + 1;
      st->converged = rS[0] < st->tol ? 1 : 0;
      st->done = (st->converged || it + 1 >= st->max_iter) ? 1 : 0;
    }
  }
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

PassPlan plan_pass(int64_t rows, int32_t d, int32_t k, size_t lds_limit) {
  PassPlan p{};
  p.dmax = pick_dmax(d);
  p.ppt = pick_ppt(p.dmax);
  const size_t budget = std::min<size_t>(lds_limit, 65536);
  const size_t kk = (size_t)k, dd = (size_t)d;
  const size_t lds_fused =
      ((kk * (size_t)p.dmax + kk) * 4 + 15) / 16 * 16 + kk * dd * 8 + kk * 4;
  p.fused = p.dmax != 0 && lds_fused <= budget;
  const int64_t tile_pts = 256LL * p.ppt;
  const int64_t tiles = std::max<int64_t>(1, (rows + tile_pts - 1) / tile_pts);
  const int64_t C = (int64_t)k * (d + 1);
  const int64_t cap_rows = std::max<int64_t>(16, (256LL << 20) / (C * 8));  // part <= 256 MB
  if (p.fused) {
    p.lds_assign = lds_fused;
    p.blocks = std::min<int64_t>(std::min<int64_t>(tiles, 2048), cap_rows);
    p.part_rows = p.blocks;
    p.ktile = k;
    return p;
  }
  if (p.dmax) {
    p.ktile = (int)std::max<int64_t>(1, std::min<int64_t>(k, 8192 / p.dmax));
    p.lds_assign = (size_t)p.ktile * p.dmax * 4 + (size_t)p.ktile * 4;
  }
  p.blocks = std::min<int64_t>(tiles, 2048);
  // split update: crange centers x slice dims of 64-bit sums + crange counts in LDS
  int crange = k, slice;
  if (kk * 12 > budget) {
    crange = (int)(budget / 12);
    slice = 1;
  } else {
    slice = (int)std::min<size_t>(dd, (budget - kk * 4) / (kk * 8));
  }
  p.crange = crange;
  p.slice = std::max(1, slice);
  p.nslices = (d + p.slice - 1) / p.slice;
  p.lds_update = (size_t)crange * p.slice * 8 + (size_t)crange * 4;
  p.ublocks = std::min<int64_t>(std::min<int64_t>((rows + 2047) / 2048, 1024), cap_rows);
  p.ublocks = std::max<int64_t>(1, p.ublocks);
  p.part_rows = p.ublocks;
  return p;
}

template <typename T, int DMAX, int P>
static void launch_fused(const PassBufs& b, const PassPlan& p, bool update, const int32_t* gate,
                         hipStream_t s) {
  hipLaunchKernelGGL((k_fused<T, DMAX, P>), dim3((unsigned)p.blocks), dim3(256), p.lds_assign, s,
                     (const T*)b.X, b.n, b.d, b.k, b.cw, b.cn, b.c64, (const PassState*)b.st,
                     gate, update ? 1 : 0, b.part, b.Jpart, b.upart, b.labels);
}

template <typename T, int DMAX, int P>
static void launch_tiled(const PassBufs& b, const PassPlan& p, const int32_t* gate,
                         hipStream_t s) {
  hipLaunchKernelGGL((k_assign_tiled<T, DMAX, P>), dim3((unsigned)p.blocks), dim3(256),
                     p.lds_assign, s, (const T*)b.X, b.n, b.d, b.k, p.ktile, b.cw, b.cn, b.c64,
                     (const PassState*)b.st, gate, b.Jpart, b.upart, b.labels);
}

template <typename T>
static void dispatch_fused(const PassBufs& b, const PassPlan& p, bool update,
                           const int32_t* gate, hipStream_t s) {
  switch (p.dmax) {
    case 2: launch_fused<T, 2, 4>(b, p, update, gate, s); break;
    case 4: launch_fused<T, 4, 4>(b, p, update, gate, s); break;
    case 8: launch_fused<T, 8, 4>(b, p, update, gate, s); break;
    case 16: launch_fused<T, 16, 2>(b, p, update, gate, s); break;
    case 32: launch_fused<T, 32, 1>(b, p, update, gate, s); break;
    case 64: launch_fused<T, 64, 1>(b, p, update, gate, s); break;
    case 128: launch_fused<T, 128, 1>(b, p, update, gate, s); break;
    default: break;
  }
}

template <typename T>
static void dispatch_tiled(const PassBufs& b, const PassPlan& p, const int32_t* gate,
                           hipStream_t s) {
  switch (p.dmax) {
    case 2: launch_tiled<T, 2, 4>(b, p, gate, s); break;
    case 4: launch_tiled<T, 4, 4>(b, p, gate, s); break;
    case 8: launch_tiled<T, 8, 4>(b, p, gate, s); break;
    case 16: launch_tiled<T, 16, 2>(b, p, gate, s); break;
    case 32: launch_tiled<T, 32, 1>(b, p, gate, s); break;
    case 64: launch_tiled<T, 64, 1>(b, p, gate, s); break;
    case 128: launch_tiled<T, 128, 1>(b, p, gate, s); break;
    default:
      hipLaunchKernelGGL(k_assign_generic<T>, dim3((unsigned)p.blocks), dim3(256), 0, s,
                         (const T*)b.X, b.n, b.d, b.k, b.cw, b.cn, b.c64,
                         (const PassState*)b.st, gate, b.Jpart, b.upart, b.labels);
      break;
  }
}

static void split_update(const PassBufs& b, const PassPlan& p, const int32_t* gate,
                         hipStream_t s) {
  const int crange = p.crange;
  const unsigned ncr = (unsigned)((b.k + crange - 1) / crange);
  dim3 grid((unsigned)p.ublocks, (unsigned)p.nslices, ncr);
  if (b.dtype == 0)
    hipLaunchKernelGGL(k_update_split<float>, grid, dim3(256), p.lds_update, s,
                       (const float*)b.X, (const int32_t*)b.labels, b.n, b.d, b.k, p.slice,
                       crange, (const PassState*)b.st, gate, b.part);
  else
    hipLaunchKernelGGL(k_update_split<uint16_t>, grid, dim3(256), p.lds_update, s,
                       (const uint16_t*)b.X, (const int32_t*)b.labels, b.n, b.d, b.k, p.slice,
                       crange, (const PassState*)b.st, gate, b.part);
}

static void reduce_finalize_conclude(const PassBufs& b, const PassPlan& p, const int32_t* gate,
                                     hipStream_t s) {
  const int64_t C = (int64_t)b.k * (b.d + 1);
  const int R = (int)std::min<int64_t>(p.part_rows, 32);
  hipLaunchKernelGGL(k_reduce_part, dim3((unsigned)((C + 255) / 256), (unsigned)R), dim3(256), 0,
                     s, (const long long*)b.part, p.part_rows, C, R, gate, b.part2);
  hipLaunchKernelGGL(k_finalize, dim3((unsigned)b.k), dim3(64), 0, s, (const long long*)b.part2,
                     R, b.k, b.d, (const PassState*)b.st, gate, b.c64, b.cw, b.cn, b.cnorm,
                     b.shiftj, b.emptyj, b.S_out, b.N_out);
  hipLaunchKernelGGL(k_conclude, dim3(1), dim3(256), 0, s, b.st, (const double*)b.Jpart,
                     (const long long*)b.upart, p.blocks, (const double*)b.shiftj,
                     (const double*)b.cnorm, (const int32_t*)b.emptyj, b.k, 1, b.J_hist,
                     b.shift_hist);
}

hipError_t pass_assign(const PassBufs& b, const PassPlan& p, bool update, hipStream_t s) {
  const int32_t* gate = update ? &b.st->done : nullptr;
  if (p.fused) {
    if (b.dtype == 0) dispatch_fused<float>(b, p, update, gate, s);
    else dispatch_fused<uint16_t>(b, p, update, gate, s);
  } else {
    if (b.dtype == 0) dispatch_tiled<float>(b, p, gate, s);
    else dispatch_tiled<uint16_t>(b, p, gate, s);
  }
  return hipGetLastError();
}

hipError_t pass_rest(const PassBufs& b, const PassPlan& p, bool update, hipStream_t s) {
  const int32_t* gate = update ? &b.st->done : nullptr;
  if (update) {
    if (!p.fused) split_update(b, p, gate, s);
    reduce_finalize_conclude(b, p, gate, s);
  } else {
    hipLaunchKernelGGL(k_conclude, dim3(1), dim3(256), 0, s, b.st, (const double*)b.Jpart,
                       (const long long*)b.upart, p.blocks, (const double*)b.shiftj,
                       (const double*)b.cnorm, (const int32_t*)b.emptyj, b.k, 0, nullptr,
                       nullptr);
  }
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
