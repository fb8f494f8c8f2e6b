// Device helpers shared by the libkrps kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

namespace krps {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

template <int I, int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    static_for<I + 1, N>(f);
  }
}

// Upper-triangle tile pairs (ta <= tb < NT) enumerated row by row.
__host__ __device__ constexpr int pair_ta(int NT, int pr) {
  int ta = 0;
  while (pr >= NT - ta) {
    pr -= NT - ta;
    ++ta;
  }
  return ta;
}
__host__ __device__ constexpr int pair_tb(int NT, int pr) {
  int ta = 0;
  while (pr >= NT - ta) {
    pr -= NT - ta;
    ++ta;
  }
  return ta + pr;
}

// Packed upper-triangle offset of entry (a, b), a <= b, of an R x R matrix.
__host__ __device__ __forceinline__ int64_t packed_index(int a, int b, int R) {
  return (int64_t)a * R - ((int64_t)a * (a - 1)) / 2 + (b - a);
}

// Offset (in nodes) of the stored left children of level `lev` (>= 1) in
// a tree with L leaves and depth D; the root is node 0.
__device__ __forceinline__ int64_t level_offset(int64_t L, int D, int lev) {
  int64_t off = 1;
  for (int m = 1; m < lev; ++m) off += ((L - 1) >> (D - m + 1)) + 1;
  return off;
}

// Sum over the 64 lanes of a wave; every lane gets the result.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Inclusive prefix sum over the 64 lanes of a wave.
__device__ __forceinline__ double wave_inclusive_scan(double v, int lane) {
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    double t = __shfl_up(v, o, 64);
    if (lane >= o) v += t;
  }
  return v;
}

// Orders the LDS traffic of one wave (all lanes see the others' writes).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

}  // namespace krps
