// Measured peaks of the units the rooflines are priced against: a device
// copy (HBM), dependent-chain FMA loops (float64 and float32 vector ALU) and
// matrix-core loops (float64 16x16x4 and bf16 16x16x32 MFMA).  Each loop
// keeps enough independent chains per lane that issue, not latency, bounds
// it, and the grid fills every compute unit several times over.
#include <algorithm>

#include "device_common.h"
#include "krps_internal.h"

namespace krps {
namespace {

__global__ __launch_bounds__(256) void copy_probe_kernel(const f32x4* __restrict__ src,
                                                         f32x4* __restrict__ dst, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

constexpr int CHAINS = 8;

template <typename T>
__global__ __launch_bounds__(256) void fma_probe_kernel(T* __restrict__ out, int iters, T a) {
  T x[CHAINS];
#pragma unroll
  for (int c = 0; c < CHAINS; ++c) x[c] = (T)(threadIdx.x + c);
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int c = 0; c < CHAINS; ++c) x[c] = x[c] * a + (T)1;
  }
  T s = 0;
#pragma unroll
  for (int c = 0; c < CHAINS; ++c) s += x[c];
  // the store keeps the loop alive; a == 1 makes it overflow-free
  if (s == (T)-1) out[blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void mfma_f64_probe_kernel(double* __restrict__ out, int iters) {
  f64x4 acc[4] = {};
  const double a = 1.0 + 1e-9 * threadIdx.x, b = 1.0 - 1e-9 * threadIdx.x;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[c], 0, 0, 0);
  }
  double s = 0;
#pragma unroll
  for (int c = 0; c < 4; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
  if (s == -1.0) out[blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void mfma_bf16_probe_kernel(float* __restrict__ out, int iters) {
  f32x4 acc[4] = {};
  bf16x8 a, b;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    a[i] = (__bf16)(1.0f / (1 + i + threadIdx.x % 7));
    b[i] = (__bf16)(1.0f / (2 + i));
  }
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[c], 0, 0, 0);
  }
  float s = 0;
#pragma unroll
  for (int c = 0; c < 4; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
  if (s == -1.0f) out[blockIdx.x] = s;
}

// Milliseconds of `launch` on the stream (best of `reps` after a warm-up).
template <typename F>
hipError_t time_best(hipStream_t st, int reps, F launch, float* best) {
  hipEvent_t e0, e1;
  hipError_t e = hipEventCreate(&e0);
  if (e != hipSuccess) return e;
  e = hipEventCreate(&e1);
  if (e != hipSuccess) {
    (void)hipEventDestroy(e0);
    return e;
  }
  *best = 1e30f;
  for (int r = 0; r <= reps && e == hipSuccess; ++r) {
    e = hipEventRecord(e0, st);
    if (e == hipSuccess) launch();
    if (e == hipSuccess) e = hipGetLastError();
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e == hipSuccess && r > 0) *best = std::min(*best, ms);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return e;
}

}  // namespace

krps_status measure_peaks(int device, hipStream_t st, void* ws, size_t ws_bytes,
                          krps_peaks* out) {
  if (out == nullptr || ws == nullptr) return fail(KRPS_EINVAL, "out/workspace is NULL");
  if (ws_bytes < (size_t(1) << 26)) return fail(KRPS_EWORKSPACE, "peak probes need >= 64 MiB");
  KRPS_HIP(hipSetDevice(device));
  int cus = 0;
  KRPS_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device));
  const int blocks = std::max(cus, 1) * 16;
  float ms = 0;
  // HBM: copy half the workspace into the other half (bytes read + written)
  const int64_t n = (int64_t)(ws_bytes / 2 / sizeof(f32x4));
  const f32x4* src = (const f32x4*)ws;
  f32x4* dst = (f32x4*)ws + n;
  KRPS_HIP(launch_fill(st, KRPS_FP32, ws, n * 4));
  KRPS_HIP(time_best(st, 5, [&] {
    hipLaunchKernelGGL(copy_probe_kernel, dim3(std::max(cus, 1) * 32), dim3(256), 0, st, src, dst,
                       n);
  }, &ms));
  out->hbm_copy_gbs = 2.0 * (double)n * sizeof(f32x4) / (ms * 1e-3) / 1e9;
  const int iters = 4096;
  double* o64 = (double*)dst;
  float* o32 = (float*)dst;
  const double threads = (double)blocks * 256;
  KRPS_HIP(time_best(st, 3, [&] {
    hipLaunchKernelGGL(fma_probe_kernel<double>, dim3(blocks), dim3(256), 0, st, o64, iters, 1.0);
  }, &ms));
  out->f64_vector_tflops = 2.0 * CHAINS * iters * threads / (ms * 1e-3) / 1e12;
  KRPS_HIP(time_best(st, 3, [&] {
    hipLaunchKernelGGL(fma_probe_kernel<float>, dim3(blocks), dim3(256), 0, st, o32, iters, 1.0f);
  }, &ms));
  out->f32_vector_tflops = 2.0 * CHAINS * iters * threads / (ms * 1e-3) / 1e12;
  const int miters = 2048;
  const double waves = threads / 64;
  KRPS_HIP(time_best(st, 3, [&] {
    hipLaunchKernelGGL(mfma_f64_probe_kernel, dim3(blocks), dim3(256), 0, st, o64, miters);
  }, &ms));
  // four 16x16x4 float64 MFMAs per wave and iteration, 2 * 16 * 16 * 4 flops each
  out->f64_matrix_tflops = 2.0 * 16 * 16 * 4 * 4.0 * miters * waves / (ms * 1e-3) / 1e12;
  KRPS_HIP(time_best(st, 3, [&] {
    hipLaunchKernelGGL(mfma_bf16_probe_kernel, dim3(blocks), dim3(256), 0, st, o32, miters);
  }, &ms));
  // four 16x16x32 bf16 MFMAs per wave and iteration
  out->bf16_matrix_tflops = 2.0 * 16 * 16 * 32 * 4.0 * miters * waves / (ms * 1e-3) / 1e12;
  return KRPS_OK;
}

}  // namespace krps
