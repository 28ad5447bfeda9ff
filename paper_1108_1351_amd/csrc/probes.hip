// Measured peaks for the roofline denominators: a streaming read of device
// memory and a loop of independent BF16 MFMAs (the instruction the BF16
// screens use), timed with HIP events on the caller's stream.
#include "host_common.h"

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// Every byte of the buffer read once with 16-byte loads (grid-stride); the xor
// of what each block read is written so that the loads cannot be dropped.
__global__ __launch_bounds__(256) void k_stream_read(const uint4* __restrict__ p, int64_t count,
                                                     uint32_t* __restrict__ sink) {
  uint32_t acc = 0;
  const int64_t stride = (int64_t)gridDim.x * 256;
  int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  for (; i + 3 * stride < count; i += 4 * stride) {
    const uint4 a = p[i], b = p[i + stride], c = p[i + 2 * stride], d = p[i + 3 * stride];
    acc ^= a.x ^ a.y ^ a.z ^ a.w ^ b.x ^ b.y ^ b.z ^ b.w ^ c.x ^ c.y ^ c.z ^ c.w ^ d.x ^ d.y ^
           d.z ^ d.w;
  }
  for (; i < count; i += stride) {
    const uint4 a = p[i];
    acc ^= a.x ^ a.y ^ a.z ^ a.w;
  }
  for (int o = 32; o > 0; o >>= 1) acc ^= __shfl_xor(acc, o);
  if ((threadIdx.x & 63) == 0) atomicXor(&sink[blockIdx.x & 1023], acc);
}

// Four independent accumulation chains of 32x32x16 BF16 MFMAs per wave.
__global__ __launch_bounds__(256) void k_mfma_loop(int iters, float* __restrict__ sink) {
  const int lane = threadIdx.x & 63;
  bf16x8 a, b;
  for (int e = 0; e < 8; ++e) {
    a[e] = (__bf16)(0.001f * (float)(lane + e));
    b[e] = (__bf16)(0.002f * (float)(lane - e));
  }
  f32x16 c0 = {}, c1 = {}, c2 = {}, c3 = {};
  for (int it = 0; it < iters; ++it) {
    c0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c0, 0, 0, 0);
    c1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c1, 0, 0, 0);
    c2 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c2, 0, 0, 0);
    c3 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c3, 0, 0, 0);
  }
  float s = 0.f;
  for (int r = 0; r < 16; ++r) s += c0[r] + c1[r] + c2[r] + c3[r];
  sink[blockIdx.x * 256 + threadIdx.x] = s;
}

}  // namespace

using namespace km;

extern "C" {

km_status km_probe_stream_read(const void* buf, size_t bytes, int32_t reps, double* gbps,
                               void* stream) {
  g_err.clear();
  if (!buf || !gbps || reps < 1 || bytes < 16 || (reinterpret_cast<uintptr_t>(buf) & 15u))
    return fail(KM_EINVAL, "need a 16-byte aligned buffer of >= 16 bytes, reps >= 1, gbps");
  km_status rc = KM_OK;
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  uint32_t* sink = nullptr;
  float ms = 0.f;
  const int64_t count = (int64_t)(bytes / 16);
  const unsigned grid = (unsigned)std::min<int64_t>((count + 255) / 256, 8 * device_cus());
  HIP_TRY(hipMallocAsync(reinterpret_cast<void**>(&sink), 4096, s));
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  hipLaunchKernelGGL(k_stream_read, dim3(grid), dim3(256), 0, s, (const uint4*)buf, count, sink);
  HIP_TRY(hipEventRecord(e0, s));
  for (int r = 0; r < reps; ++r)
    hipLaunchKernelGGL(k_stream_read, dim3(grid), dim3(256), 0, s, (const uint4*)buf, count,
                       sink);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipEventRecord(e1, s));
  HIP_TRY(hipEventSynchronize(e1));
  HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
  *gbps = (double)count * 16.0 * reps / (ms * 1e-3) / 1e9;
done:
  if (sink) (void)hipFreeAsync(sink, s);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipStreamSynchronize(s);
  return rc;
}

km_status km_probe_mfma_bf16(int32_t iters, double* tflops, void* stream) {
  g_err.clear();
  if (!tflops || iters < 1) return fail(KM_EINVAL, "need iters >= 1 and tflops");
  km_status rc = KM_OK;
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  float* sink = nullptr;
  float ms = 0.f;
  // two waves per SIMD on every CU
  const unsigned grid = (unsigned)(2 * device_cus());
  HIP_TRY(hipMallocAsync(reinterpret_cast<void**>(&sink), sizeof(float) * grid * 256, s));
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  hipLaunchKernelGGL(k_mfma_loop, dim3(grid), dim3(256), 0, s, iters, sink);
  HIP_TRY(hipEventRecord(e0, s));
  hipLaunchKernelGGL(k_mfma_loop, dim3(grid), dim3(256), 0, s, iters, sink);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipEventRecord(e1, s));
  HIP_TRY(hipEventSynchronize(e1));
  HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
  // per wave and iteration: 4 MFMAs of 2 * 32 * 32 * 16 flops
  *tflops = (double)grid * 4.0 * iters * 4.0 * 32768.0 / (ms * 1e-3) / 1e12;
done:
  if (sink) (void)hipFreeAsync(sink, s);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipStreamSynchronize(s);
  return rc;
}

}  // extern "C"
