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

// (a, b), a <= b, of packed entry p (inverse of packed_index).
__device__ __forceinline__ void unpack_index(int64_t p, int R, int& a, int& b) {
  const double q = (double)(2 * R + 1);
  int aa = (int)((q - sqrt(q * q - 8.0 * (double)p)) * 0.5);
  if (aa < 0) aa = 0;
  if (aa > R - 1) aa = R - 1;
  while (aa > 0 && packed_index(aa, aa, R) > p) --aa;
  while (aa < R - 1 && packed_index(aa + 1, aa + 1, R) <= p) ++aa;
  a = aa;
  b = aa + (int)(p - packed_index(aa, aa, R));
}

// Offset (in nodes) of the stored left children of level `lev` (>= 1) in
// a tree with L leaves and depth D; the root is node 0.
__device__ __forceinline__ int64_t level_offset(int64_t L, int D, int lev) {
  int64_t off = 1;
  for (int m = 1; m < lev; ++m) off += ((L - 1) >> (D - m + 1)) + 1;
  return off;
}

// Lane-exchange of a double through the data-parallel primitives (DPP).
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
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

// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of the
// 4 x 64-bit S-box on counter c under key (k0, k1), in place.
__device__ __forceinline__ void philox4x64_10(uint64_t c[4], uint64_t k0, uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t h0 = __umul64hi(M0, c[0]), l0 = M0 * c[0];
    const uint64_t h1 = __umul64hi(M1, c[2]), l1 = M1 * c[2];
    const uint64_t n0 = h1 ^ c[1] ^ k0, n2 = h0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = l1;
    c[2] = n2;
    c[3] = l0;
    k0 += W0;
    k1 += W1;
  }
}

// Open-interval uniform from a 64-bit word: ((x >> 11) + 0.5) 2^-53.
__device__ __forceinline__ double u01_of_word(uint64_t x) {
  return ((double)(x >> 11) + 0.5) * 0x1.0p-53;
}

// Orders the LDS traffic of one wave (all lanes see the others' writes).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

}  // namespace krps
