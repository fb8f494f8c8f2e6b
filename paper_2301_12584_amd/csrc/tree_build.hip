// Segment-tree construction on the matrix cores (BuildSampler, Appendix A.5
// Algorithm 3): leaf partial Gram matrices G^v = U[S(v)]^T U[S(v)] and the
// level-by-level sums G^v = G^{L(v)} + G^{R(v)} up to the root G = U^T U.
//
// Storage (space halving of Appendix A.5): the root and the left children
// only, each as a packed upper triangle.  Pad leaves (the tree is padded to
// 2^D leaves) are implicit zeros and never stored.
//
// Kernel 1 (leaf_run_kernel): a team of TW waves owns a run of 2^s
// consecutive leaves.  Each leaf's Gram is a SYRK on the matrix cores; the
// upper-triangle 16x16 tiles are split across the team's waves.  The run's
// subtree is summed in registers with a binary counter (leaf u of the run
// merges with the saved left siblings of its trailing one-bits), left
// children are written as they complete, and the run root goes to a float64
// scratch array.
// Kernel 2 (node_upsweep_kernel): the levels above the runs, one thread per
// packed entry, the same binary counter over groups of 2^s2 nodes in float64,
// down to the root (also written as the full float64 R x R Gram G_j).
// A float64 tree may also get a float32 copy of every stored node (each
// entry rounded to nearest), written by both kernels beside the float64
// node: the walk decides its deep levels from the copy.
#include "device_common.h"
#include <algorithm>
#include <vector>

#include "krps_internal.h"

namespace krps {

namespace {

// M_F64: float64 factor; M_F32: float32 factor, float64 products (exact)
// and sums.  M_SPLIT3 (the Gram of a solve's sampled rows on the split
// path): x = hi + mid + lo (bf16 each), the six products whose parts'
// orders sum to at most 2 (about 2^-24, float32-like), float32 sums.
enum { M_F64 = 0, M_F32 = 1, M_SPLIT3 = 3 };

__device__ __forceinline__ f64x4 mfma_f64(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x4 mfma_bf16(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Writes the 16x16 accumulator tile (ta, tb) of one node.  Column l%16 of
// the tile is in lane l; the row of register i is 4*(l/16)+i for the
// float32-accumulating instructions and 4*i+l/16 for the float64 one.
template <typename OUT, typename ACC>
__device__ __forceinline__ void write_tile(OUT* dst, const ACC& v, int ta, int tb, int R,
                                           int lane) {
  constexpr bool F64 = std::is_same_v<ACC, f64x4>;
  const int b = 16 * tb + (lane & 15);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int a = 16 * ta + (F64 ? 4 * i + (lane >> 4) : 4 * (lane >> 4) + i);
    if (a < R && b < R && a <= b) dst[packed_index(a, b, R)] = (OUT)v[i];
  }
}

// The run of wave W of the team; W is a compile-time constant so that each
// wave's code names only its own tile pairs (and loads and converts only
// the column tiles those pairs use).
template <int MODE, int NT, int TW, int S, int W>
__device__ __forceinline__ void leaf_run_body(const void* __restrict__ Uv, int64_t I, int R, int F,
                                              int64_t L, int D, int s_eff,
                                              void* __restrict__ nodes_v,
                                              double* __restrict__ tops,
                                              float* __restrict__ nodes32) {
  // storage type of the factor and the nodes; float64 accumulation on the
  // matrix cores except for the bf16 split
  using T = std::conditional_t<MODE == M_F64, double, float>;
  constexpr bool SPLIT = MODE == M_SPLIT3;
  using ACC = std::conditional_t<SPLIT, f32x4, f64x4>;
  constexpr int NPAIRS = NT * (NT + 1) / 2;
  constexpr int NPW = (NPAIRS + TW - 1) / TW;
  const T* __restrict__ U = (const T*)Uv;
  T* __restrict__ nodes = (T*)nodes_v;
  const int lane = threadIdx.x & 63;
  const int64_t TR = (int64_t)R * (R + 1) / 2;
  const int64_t run = blockIdx.x;
  const int nrun = 1 << s_eff;

  ACC node[NPW];
  ACC stack[S > 0 ? S : 1][NPW];

  for (int u = 0; u < nrun; ++u) {
    const int64_t c = (run << s_eff) + u;
#pragma unroll
    for (int q = 0; q < NPW; ++q) node[q] = ACC{0, 0, 0, 0};
    if (c < L) {
      const int64_t r0 = c * F;
      const int64_t r1 = r0 + F < I ? r0 + F : I;
      if constexpr (!SPLIT) {
        // chunks of KS steps of 4 rows: all loads of a chunk are issued
        // before its products
        constexpr int KS = NT <= 2 ? 8 : 4;
        for (int64_t rc = r0; rc < r1; rc += 4 * KS) {
          // unconditional loads from clamped (in-bounds) addresses, zeroed
          // afterwards, so that they are all issued back to back
          T raw[KS][NT];
#pragma unroll
          for (int ks = 0; ks < KS; ++ks) {
            const int64_t row = rc + 4 * ks + (lane >> 4);
            const int64_t rowc = row < r1 ? row : r1 - 1;
            static_for<0, NT>([&](auto tt) {
              constexpr int t = decltype(tt)::value;
              const int col = 16 * t + (lane & 15);
              raw[ks][t] = U[rowc * R + (col < R ? col : R - 1)];
            });
          }
#pragma unroll
          for (int ks = 0; ks < KS; ++ks) {
            const bool rv = rc + 4 * ks + (lane >> 4) < r1;
            static_for<0, NT>([&](auto tt) {
              constexpr int t = decltype(tt)::value;
              if (!rv || 16 * t + (lane & 15) >= R) raw[ks][t] = T(0);
            });
          }
#pragma unroll
          for (int ks = 0; ks < KS; ++ks) {
            static_for<0, NPAIRS>([&](auto pp) {
              constexpr int pr = decltype(pp)::value;
              constexpr int ta = pair_ta(NT, pr);
              constexpr int tb = pair_tb(NT, pr);
              if constexpr (pr % TW == W)
                node[pr / TW] = mfma_f64((double)raw[ks][ta], (double)raw[ks][tb], node[pr / TW]);
            });
          }
        }
      } else {
        for (int64_t rb = r0; rb < r1; rb += 32) {
          bf16x8 hi[NT], lo[NT], mid[NT];
          float xs[NT][8];
          static_for<0, NT>([&](auto tt) {
            constexpr int t = decltype(tt)::value;
            const int col = 16 * t + (lane & 15);
            const int colc = col < R ? col : R - 1;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
              const int64_t row = rb + 8 * (lane >> 4) + j;
              xs[t][j] = U[(row < r1 ? row : r1 - 1) * R + colc];
            }
          });
          static_for<0, NT>([&](auto tt) {
            constexpr int t = decltype(tt)::value;
            const bool cv = 16 * t + (lane & 15) < R;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
              const int64_t row = rb + 8 * (lane >> 4) + j;
              const float x = (cv && row < r1) ? xs[t][j] : 0.f;
              const __bf16 h = (__bf16)x;
              hi[t][j] = h;
              const float r = x - (float)h;
              const __bf16 m = (__bf16)r;
              mid[t][j] = m;
              lo[t][j] = (__bf16)(r - (float)m);
            }
          });
          static_for<0, NPAIRS>([&](auto pp) {
            constexpr int pr = decltype(pp)::value;
            constexpr int ta = pair_ta(NT, pr);
            constexpr int tb = pair_tb(NT, pr);
            if constexpr (pr % TW == W) {
              ACC a = node[pr / TW];
              // smallest terms first
              a = mfma_bf16(mid[ta], mid[tb], a);
              a = mfma_bf16(hi[ta], lo[tb], a);
              a = mfma_bf16(lo[ta], hi[tb], a);
              a = mfma_bf16(hi[ta], mid[tb], a);
              a = mfma_bf16(mid[ta], hi[tb], a);
              a = mfma_bf16(hi[ta], hi[tb], a);
              node[pr / TW] = a;
            }
          });
        }
      }
    }
    // binary counter: merge with the saved left siblings
    int t = __builtin_ctz(~(unsigned)u);
    if (t > s_eff) t = s_eff;
    static_for<0, S>([&](auto mm) {
      constexpr int m = decltype(mm)::value;
      if (m < t) {
#pragma unroll
        for (int q = 0; q < NPW; ++q) node[q] += stack[m][q];
      }
    });
    const int lev = D - t;
    const int64_t pos = c >> t;
    if (t == s_eff) {
      double* dst = tops + run * TR;
      static_for<0, NPAIRS>([&](auto pp) {
        constexpr int pr = decltype(pp)::value;
        if constexpr (pr % TW == W) write_tile(dst, node[pr / TW], pair_ta(NT, pr), pair_tb(NT, pr), R, lane);
      });
    } else {
      if (nodes != nullptr && pos < ((L - 1) >> (D - lev)) + 1) {
        const int64_t at = (level_offset(L, D, lev) + (pos >> 1)) * TR;
        static_for<0, NPAIRS>([&](auto pp) {
          constexpr int pr = decltype(pp)::value;
          if constexpr (pr % TW == W) write_tile(nodes + at, node[pr / TW], pair_ta(NT, pr), pair_tb(NT, pr), R, lane);
        });
        if constexpr (MODE == M_F64) {
          if (nodes32 != nullptr) {
            static_for<0, NPAIRS>([&](auto pp) {
              constexpr int pr = decltype(pp)::value;
              if constexpr (pr % TW == W) write_tile(nodes32 + at, node[pr / TW], pair_ta(NT, pr), pair_tb(NT, pr), R, lane);
            });
          }
        }
      }
      static_for<0, S>([&](auto mm) {
        constexpr int m = decltype(mm)::value;
        if (m == t) {
#pragma unroll
          for (int q = 0; q < NPW; ++q) stack[m][q] = node[q];
        }
      });
    }
  }
}

template <int MODE, int NT, int TW, int S>
__global__ __launch_bounds__(64 * TW) void leaf_run_kernel(const void* __restrict__ Uv, int64_t I,
                                                           int R, int F, int64_t L, int D,
                                                           int s_eff, void* __restrict__ nodes_v,
                                                           double* __restrict__ tops,
                                                           float* __restrict__ nodes32) {
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  static_for<0, TW>([&](auto ww) {
    constexpr int W = decltype(ww)::value;
    if (wave == W)
      leaf_run_body<MODE, NT, TW, S, W>(Uv, I, R, F, L, D, s_eff, nodes_v, tops, nodes32);
  });
}

constexpr int S2 = 3;  // levels summed per upsweep pass

// One thread per packed entry and per group of 2^S2 consecutive nodes of
// level lev_in; the group's subtree is summed with a binary counter whose
// saved left siblings sit in registers (the loop is unrolled).
template <typename T>
__global__ __launch_bounds__(256) void node_upsweep_kernel(const double* __restrict__ in,
                                                           int64_t n_in, int lev_in, int s2, int R,
                                                           int64_t L, int D, T* __restrict__ nodes,
                                                           double* __restrict__ out,
                                                           double* __restrict__ gram_full,
                                                           float* __restrict__ nodes32) {
  const int64_t TR = (int64_t)R * (R + 1) / 2;
  const int64_t ng = (n_in + (int64_t(1) << s2) - 1) >> s2;
  const int64_t total = ng * TR;
  for (int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; gid < total;
       gid += (int64_t)gridDim.x * blockDim.x) {
    const int64_t g = gid / TR;
    const int64_t p = gid % TR;
    double stack[S2];
#pragma unroll
    for (int u = 0; u < (1 << S2); ++u) {
      if (u >= (1 << s2)) break;
      int64_t pos = (g << s2) + u;
      double v = pos < n_in ? in[pos * TR + p] : 0.0;
      int t = __builtin_ctz(~(unsigned)u);
      if (t > s2) t = s2;
#pragma unroll
      for (int m = 0; m < S2; ++m)
        if (m < t) v += stack[m];
      const int lev = lev_in - t;
      pos >>= t;
      if (t == s2) {
        if (lev == 0) {
          if (nodes != nullptr) nodes[p] = (T)v;
          if (nodes32 != nullptr) nodes32[p] = (float)v;
          int a, b;
          unpack_index(p, R, a, b);
          gram_full[(int64_t)a * R + b] = v;
          gram_full[(int64_t)b * R + a] = v;
        } else {
          out[g * TR + p] = v;
        }
      } else {
        if (nodes != nullptr && pos < ((L - 1) >> (D - lev)) + 1) {
          const int64_t at = (level_offset(L, D, lev) + (pos >> 1)) * TR + p;
          nodes[at] = (T)v;
          if (nodes32 != nullptr) nodes32[at] = (float)v;
        }
#pragma unroll
        for (int m = 0; m < S2; ++m)
          if (m == t) stack[m] = v;
      }
    }
  }
}

struct LeafCfg {
  int NT, TW, S;
};

// Register-run depth (levels summed in registers by the leaf pass) for R;
// dispatch_leaf below instantiates exactly these depths.
int leaf_run_depth(int R) { return R <= 32 ? 4 : R <= 64 ? 3 : 2; }

template <int MODE, int NT, int TW, int S>
hipError_t run_leaf(hipStream_t st, const void* U, int64_t I, int R, int F, int64_t L, int D,
                    void* nodes, double* tops, float* nodes32, int& s_eff) {
  if (S != leaf_run_depth(R)) return hipErrorInvalidValue;
  s_eff = S < D ? S : D;
  const int64_t nrun = ceil_div(L, int64_t(1) << s_eff);
  hipLaunchKernelGGL((leaf_run_kernel<MODE, NT, TW, S>), dim3((unsigned)nrun), dim3(64 * TW), 0,
                     st, U, I, R, F, L, D, s_eff, nodes, tops, nodes32);
  return hipGetLastError();
}

// Team width (waves per leaf team) and register-run depth per precision
// and tile count, the default width first; build_team_choices lists the
// same widths.
template <int MODE>
hipError_t dispatch_leaf(hipStream_t st, const void* U, int64_t I, int R, int F, int64_t L, int D,
                         void* nodes, double* tops, float* nodes32, int team, int& s_eff) {
#define KRPS_LEAF(NT, TW, S) run_leaf<MODE, NT, TW, S>(st, U, I, R, F, L, D, nodes, tops, nodes32, s_eff)
  if constexpr (MODE == M_SPLIT3) {
    if (R <= 16) return KRPS_LEAF(1, 1, 4);
    if (R <= 32) return team == 3 ? KRPS_LEAF(2, 3, 4) : KRPS_LEAF(2, 1, 4);
    if (R <= 64) return team == 5 ? KRPS_LEAF(4, 5, 3) : KRPS_LEAF(4, 2, 3);
    return team == 8 ? KRPS_LEAF(8, 8, 2) : KRPS_LEAF(8, 4, 2);
  } else {
    // the default widths give each wave three (R <= 32) or five (R <= 64)
    // accumulator tiles: fewer, fuller waves, each loading its columns once
    // (a rebuild of 2^20 x 32: 128 against 164 us with one tile per wave
    // in float64, 93 against 111 us from float32; 1e6 x 64: 327 / 418 and
    // 275 / 325 us)
    if (R <= 16) return KRPS_LEAF(1, 1, 4);
    if (R <= 32) return team == 3 ? KRPS_LEAF(2, 3, 4) : KRPS_LEAF(2, 1, 4);
    if (R <= 64) return team == 5 ? KRPS_LEAF(4, 5, 3) : KRPS_LEAF(4, 2, 3);
    return team == 6 ? KRPS_LEAF(8, 6, 2) : KRPS_LEAF(8, 12, 2);
  }
#undef KRPS_LEAF
}

constexpr int MIN_S = 2;  // smallest register-run depth used above

}  // namespace

std::vector<int> build_team_choices(int R, krps_precision) {
  // the sampler's trees are built with float64 products in every precision
  if (R <= 16) return {1};
  if (R <= 32) return {1, 3};
  if (R <= 64) return {2, 5};
  return {12, 6};
}

size_t tree_build_scratch_bytes(int64_t L, int R) {
  const int64_t a = ceil_div(L, int64_t(1) << MIN_S);
  const int64_t b = ceil_div(a, 2);
  return align_up((size_t)a * tri(R) * 8) + align_up((size_t)b * tri(R) * 8);
}

// Replays the launch geometry of launch_tree_build (the leaf pass's run
// tops into buffer A, then each up-sweep pass into the other ping-pong
// buffer) and returns the largest byte extent, from the start of the
// scratch, that any pass writes or reads.
size_t tree_build_scratch_extent(const TreeShape& ts, int R) {
  const int64_t TR = tri(R);
  const int64_t a_nodes = ceil_div(ts.L, int64_t(1) << MIN_S);
  const size_t offB = align_up((size_t)a_nodes * TR * 8);
  const int S = leaf_run_depth(R);
  const int s_eff = S < ts.D ? S : ts.D;
  int64_t n = ceil_div(ts.L, int64_t(1) << s_eff);
  size_t ext = (size_t)n * TR * 8;  // run tops in A
  size_t cur = 0, nxt = offB;
  int lev = ts.D - s_eff;
  for (;;) {
    const int s2 = lev < S2 ? lev : S2;
    const int64_t ng = ceil_div(n, int64_t(1) << s2);
    ext = std::max(ext, cur + (size_t)n * TR * 8);           // reads
    if (lev - s2 == 0) break;                                  // the root goes to the tree
    ext = std::max(ext, nxt + (size_t)ng * TR * 8);          // writes
    lev -= s2;
    n = ng;
    std::swap(cur, nxt);
  }
  return ext;
}

hipError_t launch_tree_build(hipStream_t st, krps_precision p, const void* U, int64_t I, int R,
                             const TreeShape& ts, void* nodes, double* gram_full, double* scratch,
                             size_t scratch_bytes, float* nodes32, int team) {
  const int64_t TR = tri(R);
  if (p != KRPS_FP64) nodes32 = nullptr;  // only float64 trees carry a float32 copy
  const int64_t a_nodes = ceil_div(ts.L, int64_t(1) << MIN_S);
  double* bufA = scratch;
  double* bufB = (double*)((char*)scratch + align_up((size_t)a_nodes * TR * 8));
  if (scratch_bytes < tree_build_scratch_bytes(ts.L, R)) return hipErrorInvalidValue;
  int s_eff = 0;
  hipError_t e;
  if (p == KRPS_FP64)
    e = dispatch_leaf<M_F64>(st, U, I, R, ts.F, ts.L, ts.D, nodes, bufA, nodes32, team, s_eff);
  else if (p == KRPS_FP32)
    e = dispatch_leaf<M_F32>(st, U, I, R, ts.F, ts.L, ts.D, nodes, bufA, nodes32, team, s_eff);
  else
    e = dispatch_leaf<M_SPLIT3>(st, U, I, R, ts.F, ts.L, ts.D, nodes, bufA, nodes32, team, s_eff);
  if (e != hipSuccess) return e;
  int lev = ts.D - s_eff;
  int64_t n = ceil_div(ts.L, int64_t(1) << s_eff);
  double* cur = bufA;
  double* nxt = bufB;
  for (;;) {
    const int s2 = lev < S2 ? lev : S2;
    const int64_t ng = ceil_div(n, int64_t(1) << s2);
    int64_t blocks = ceil_div(ng * TR, 256);
    if (blocks > 4096) blocks = 4096;
    if (p == KRPS_FP64)
      hipLaunchKernelGGL(node_upsweep_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, st, cur,
                         n, lev, s2, R, ts.L, ts.D, (double*)nodes, nxt, gram_full, nodes32);
    else
      hipLaunchKernelGGL(node_upsweep_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, st, cur,
                         n, lev, s2, R, ts.L, ts.D, (float*)nodes, nxt, gram_full, nullptr);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (lev - s2 == 0) break;
    lev -= s2;
    n = ng;
    double* tmp = cur;
    cur = nxt;
    nxt = tmp;
  }
  return hipSuccess;
}

}  // namespace krps

// ------------------------------------------------ single-entry updates

namespace krps {

namespace {

// UpdateSampler (Appendix A.7, Algorithm 5) for a list of entries, in order:
// U[r, c] := v.  With u the old row and delta = v - u[c] (v as stored), the
// Gram of every node whose segment holds row r gains delta u in its row c
// and column c and delta^2 more at (c, c); of those nodes the root and the
// left children are stored (a right child's mass is its parent's minus its
// sibling's, so it follows), and so is G_j.  One workgroup: thread a
// updates entry (min(a, c), max(a, c)) of each stored path node.
template <typename T>
__global__ __launch_bounds__(128) void update_entries_kernel(UpdateList ul, T* __restrict__ U,
                                                             T* __restrict__ nodes,
                                                             float* __restrict__ nodes32,
                                                             double* __restrict__ gram, int64_t I,
                                                             int R, int F, int64_t L, int D) {
  __shared__ double urow[128];
  const int a = threadIdx.x;
  for (int m = 0; m < ul.n; ++m) {
    const int64_t r = ul.row[m];
    const int c = ul.col[m];
    if (a < R) urow[a] = (double)U[r * R + a];
    __syncthreads();
    const double vs = (double)(T)ul.val[m];
    const double delta = vs - urow[c];
    if (a < R) {
      const double add = a == c ? 2.0 * delta * urow[c] + delta * delta : delta * urow[a];
      const int lo = a < c ? a : c, hi = a < c ? c : a;
      const int64_t p = packed_index(lo, hi, R);
      // the root, then the left children on the path down to the leaf
      int64_t pos = r / F;  // leaf position at level D
      for (int lev = D; lev >= 0; --lev) {
        int64_t node = -1;
        if (lev == 0)
          node = 0;
        else if ((pos & 1) == 0)
          node = level_offset(L, D, lev) + (pos >> 1);
        if (node >= 0) {
          const int64_t at = node * (int64_t)(R * (R + 1) / 2) + p;
          const double nv = (double)nodes[at] + add;
          nodes[at] = (T)nv;
          if (nodes32 != nullptr) nodes32[at] = (float)nv;
        }
        pos >>= 1;
      }
      gram[(int64_t)lo * R + hi] += add;
      if (lo != hi) gram[(int64_t)hi * R + lo] += add;
    }
    __syncthreads();
    if (a == 0) U[r * R + c] = (T)ul.val[m];
    __syncthreads();
  }
  (void)I;
}

}  // namespace

hipError_t launch_update_entries(hipStream_t st, krps_precision p, const UpdateList& ul, void* U,
                                 void* nodes, float* nodes32, double* gram, int64_t I, int R,
                                 const TreeShape& ts) {
  if (ul.n <= 0) return hipSuccess;
  if (p == KRPS_FP64)
    hipLaunchKernelGGL(update_entries_kernel<double>, dim3(1), dim3(128), 0, st, ul, (double*)U,
                       (double*)nodes, nodes32, gram, I, R, ts.F, ts.L, ts.D);
  else
    hipLaunchKernelGGL(update_entries_kernel<float>, dim3(1), dim3(128), 0, st, ul, (float*)U,
                       (float*)nodes, nullptr, gram, I, R, ts.F, ts.L, ts.D);
  return hipGetLastError();
}

}  // namespace krps
