// The batched root-to-leaf descent (KRPSample, Section 3.2 Algorithm 2,
// lines 6-12; RowSample, Appendix A.5 Algorithm 4).
//
// One wavefront per sample (persistent grid-stride loop over samples).
// For each drawn mode k (increasing k != exclude):
//   stage 1: walk E_k with the history h: node mass <h h^T, P^v (*) G_k>,
//            target x1 = u01[d][k][0] * C1  -> eigen-index u
//   stage 2: h~ = h (*) V_k[:, u]; walk Z_k with node mass h~^T G^v h~,
//            target x2 = u01[d][k][1] * C2, then scan the leaf rows
//            r_i = (U_k[i] . h~)^2                            -> row t
//   update : h <- h (*) U_k[t]
// A node mass is a dot product of the stored packed upper triangle with
// the packed outer product of h (off-diagonal terms doubled), built once
// per stage and kept in registers: each level is one coalesced read of the
// node (tri(R) elements, 64 lanes) and a wavefront sum.  Branch decisions
// and the running offsets low/high are float64 in every precision.
// After the last mode h is the sampled Khatri-Rao row a_d; its probability
// q_d = a_d G^+ a_d^T / rank (Section 2.1) is the same kind of dot product
// against the packed float64 G^+.
#include "device_common.h"
#include "krps_internal.h"

namespace krps {

namespace {

constexpr int DESC_WAVES = 4;  // waves per block

// Packed outer product h h^T of the float64 vector in hb (LDS), off-diagonal
// terms doubled, lane l holding entries l + 64 m.
template <int NP>
struct Packed {
  double v[NP];
};

template <int NP>
__device__ __forceinline__ void build_packed(Packed<NP>& P, const double* hb,
                                             const uint16_t* __restrict__ tab, int TR, int lane) {
#pragma unroll
  for (int m = 0; m < NP; ++m) {
    const int p = lane + 64 * m;
    double val = 0;
    if (p < TR) {
      const uint16_t ab = tab[p];
      const int a = ab & 0xff, b = ab >> 8;
      val = hb[a] * hb[b];
      if (a != b) val += val;
    }
    P.v[m] = val;
  }
}

// Node mass <h h^T, G^v> = h^T G^v h in float64 whatever the storage type.
// R <= 64: dot product of the stored packed triangle with the packed outer
// product kept in registers (each lane reads tri(R)/64 coalesced entries).
template <typename T, int NP>
__device__ __forceinline__ double node_mass(const Packed<NP>& P, const double*,
                                            const T* __restrict__ node, int R, int TR, int lane) {
  double acc = 0;
#pragma unroll
  for (int m = 0; m < NP; ++m) {
    const int p = lane + 64 * m;
    if (p < TR) acc += P.v[m] * (double)node[p];
  }
  return wave_sum(acc);
}

// R > 64: row by row; lane l owns columns l and l + 64, the row's h_a is a
// broadcast LDS read, so no outer product has to be held in registers.
template <typename T>
__device__ __forceinline__ double node_mass(const Packed<1>&, const double* hb,
                                            const T* __restrict__ node, int R, int TR, int lane) {
  double acc0 = 0, acc1 = 0;
  int64_t start = 0;
  const int b0 = lane, b1 = lane + 64;
  for (int a = 0; a < R; ++a) {
    const double ha = hb[a];
    if (b0 >= a && b0 < R) {
      const double g = (double)node[start + (b0 - a)];
      acc0 += (b0 == a ? ha : 2.0 * ha) * g;
    }
    if (b1 >= a && b1 < R) {
      const double g = (double)node[start + (b1 - a)];
      acc1 += (b1 == a ? ha : 2.0 * ha) * g;
    }
    start += R - a;
  }
  double v = (b0 < R ? acc0 * hb[b0] : 0.0) + (b1 < R ? acc1 * hb[b1] : 0.0);
  (void)TR;
  return wave_sum(v);
}

// Inversion walk down a stored tree (root + left children): returns the
// leaf position and the offset `low` of its segment.
template <typename T, typename PK>
__device__ __forceinline__ int64_t walk(const T* __restrict__ nodes, int64_t L, int D, const PK& P,
                                        const double* hb, int R, int TR, int lane, double x,
                                        double C, double& low_out) {
  double low = 0.0, high = C;
  int64_t pos = 0;
  int64_t off = 1;
  for (int lev = 1; lev <= D; ++lev) {
    const int64_t cnt_left = ((L - 1) >> (D - lev + 1)) + 1;
    const int64_t real = ((L - 1) >> (D - lev)) + 1;
    double mL = node_mass<T>(P, hb, nodes + (off + pos) * (int64_t)TR, R, TR, lane);
    mL = mL > 0.0 ? mL : 0.0;
    const double cut = low + mL;
    const bool right_exists = 2 * pos + 1 < real;
    if (cut >= x || !right_exists || high - cut <= 0.0) {
      high = cut;
      pos = 2 * pos;
    } else {
      low = cut;
      pos = 2 * pos + 1;
    }
    off += cnt_left;
  }
  low_out = low;
  return pos;
}

// Leaf scan: first row i of [s0, s1) with low + sum_{m <= i} r_m >= x.
template <typename T>
__device__ __forceinline__ int64_t leaf_scan(const T* __restrict__ U, int R, int64_t s0, int64_t s1,
                                             const double* hb, double low, double x, int lane) {
  int64_t last_pos = -1;
  for (int64_t base = s0; base < s1; base += 64) {
    const int64_t row = base + lane;
    const bool valid = row < s1;
    double r = 0.0;
    if (valid) {
      const T* __restrict__ ur = U + row * R;
      double acc = 0;
      for (int e = 0; e < R; ++e) acc += (double)ur[e] * hb[e];
      r = acc * acc;
    }
    const double incl = wave_inclusive_scan(r, lane);
    const bool hit = valid && (low + incl >= x);
    const unsigned long long m = __ballot(hit);
    if (m != 0ull) return base + (__ffsll((long long)m) - 1);
    const unsigned long long pm = __ballot(valid && r > 0.0);
    if (pm != 0ull) last_pos = base + (63 - __clzll((long long)pm));
    low += __shfl(incl, 63, 64);
  }
  return last_pos >= 0 ? last_pos : s1 - 1;
}

// NP > 1: packed outer product in registers; NP == 1: row-broadcast masses.
template <typename T, int NP>
__global__ __launch_bounds__(64 * DESC_WAVES) void descent_kernel(DescentArgs a) {
  extern __shared__ unsigned char smem_raw[];
  const int R = a.R;
  const int TR = R * (R + 1) / 2;
  uint16_t* tab = (uint16_t*)smem_raw;
  double* hb_all = (double*)(smem_raw + ((TR * 2 + 15) / 16) * 16);
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  double* hb = hb_all + wave * 128;
  for (int p = threadIdx.x; p < TR; p += blockDim.x) {
    int aa = 0;
    while (aa < R - 1 && packed_index(aa + 1, aa + 1, R) <= p) ++aa;
    const int bb = aa + (int)(p - packed_index(aa, aa, R));
    tab[p] = (uint16_t)(aa | (bb << 8));
  }
  __syncthreads();

  const int N = a.N;
  const int64_t J = a.J;
  const double inv_rank = a.rank ? 1.0 / (double)a.rank[0] : 1.0;
  const int64_t stride = (int64_t)gridDim.x * DESC_WAVES;
  for (int64_t d = (int64_t)blockIdx.x * DESC_WAVES + wave; d < J; d += stride) {
    // history h = (*) of the rows drawn so far, float64 (lanes e, e + 64)
    double h0 = 1, h1 = 1;
    Packed<NP> P;
    for (int st = 0; st < a.nsteps; ++st) {
      const int k = a.order[st];
      const ModeDesc& md = a.mode[k];
      const double d1 = a.u01[(d * N + k) * 2 + 0];
      const double d2 = a.u01[(d * N + k) * 2 + 1];
      // ---- stage 1: eigen-component u from E_k
      if (lane < R) hb[lane] = h0;
      if (lane + 64 < R) hb[lane + 64] = h1;
      wave_lds_sync();
      if constexpr (NP > 1) build_packed(P, hb, tab, TR, lane);
      const T* __restrict__ E = (const T*)md.E;
      const double C1 = node_mass<T>(P, hb, E, R, TR, lane);
      double low;
      int u = (int)walk(E, (int64_t)R, md.DE, P, hb, R, TR, lane, d1 * C1, C1, low);
      if (u >= R) u = R - 1;
      // ---- stage 2: row t from Z_k with h~ = h (*) V[:, u]
      const T* __restrict__ V = (const T*)md.V + (int64_t)u * R;
      const double ht0 = lane < R ? h0 * (double)V[lane] : 0.0;
      const double ht1 = lane + 64 < R ? h1 * (double)V[lane + 64] : 0.0;
      wave_lds_sync();
      if (lane < R) hb[lane] = ht0;
      if (lane + 64 < R) hb[lane + 64] = ht1;
      wave_lds_sync();
      if constexpr (NP > 1) build_packed(P, hb, tab, TR, lane);
      const T* __restrict__ Z = (const T*)md.Z;
      const double C2 = node_mass<T>(P, hb, Z, R, TR, lane);
      const double x2 = d2 * C2;
      const int64_t c = walk(Z, md.L, md.D, P, hb, R, TR, lane, x2, C2, low);
      const int64_t s0 = c * md.F;
      const int64_t s1 = s0 + md.F < md.I ? s0 + md.F : md.I;
      const T* __restrict__ U = (const T*)md.U;
      int64_t t = leaf_scan(U, R, s0, s1, hb, low, x2, lane);
      if (t < 0) t = 0;
      if (t >= md.I) t = md.I - 1;
      if (lane == 0) a.idx[d * N + k] = (int32_t)t;
      if (lane < R) h0 *= (double)U[t * R + lane];
      if (lane + 64 < R) h1 *= (double)U[t * R + lane + 64];
      if (!(C1 > 0.0) || !(C2 > 0.0)) {
        if (lane == 0) atomicOr(a.status, ST_NUMERIC);
      }
      wave_lds_sync();
    }
    if (a.exclude >= 0 && lane == 0) a.idx[d * N + a.exclude] = -1;
    // ---- probability of the sampled row: q = a G^+ a^T / rank
    if (a.prob != nullptr || a.rows != nullptr || a.wout != nullptr) {
      if (lane < R) hb[lane] = h0;
      if (lane + 64 < R) hb[lane + 64] = h1;
      wave_lds_sync();
      double acc = 0.0;
      for (int p = lane; p < TR; p += 64) {
        const uint16_t ab = tab[p];
        const int ia = ab & 0xff, ib = ab >> 8;
        const double v = hb[ia] * hb[ib] * a.gplus[p];
        acc += ia == ib ? v : 2.0 * v;
      }
      const double q = wave_sum(acc) * inv_rank;
      if (lane == 0 && a.prob != nullptr) a.prob[d] = q;
      const double w = 1.0 / sqrt((double)J * q);
      if (lane == 0 && a.wout != nullptr) a.wout[d] = w;
      if (a.rows != nullptr) {
        T* rows = (T*)a.rows + d * R;
        const double sc = a.scale_rows ? w : 1.0;
        if (lane < R) rows[lane] = (T)(h0 * sc);
        if (lane + 64 < R) rows[lane + 64] = (T)(h1 * sc);
      }
      wave_lds_sync();
    }
  }
}

// q of given multi-indices: a = (*)_k U_k[idx[d][k]], q = a G^+ a^T / rank.
template <typename T>
__global__ __launch_bounds__(64 * DESC_WAVES) void row_prob_kernel(DescentArgs a) {
  const int R = a.R;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  __shared__ double hbs[DESC_WAVES][128];
  double* hb = hbs[wave];
  const double inv_rank = 1.0 / (double)a.rank[0];
  const int64_t stride = (int64_t)gridDim.x * DESC_WAVES;
  for (int64_t d = (int64_t)blockIdx.x * DESC_WAVES + wave; d < a.J; d += stride) {
    double h0 = 1, h1 = 1;
    bool in_range = true;
    for (int st = 0; st < a.nsteps; ++st) {
      const int k = a.order[st];
      const T* U = (const T*)a.mode[k].U;
      const int64_t t = a.idx[d * a.N + k];
      if (t < 0 || t >= a.mode[k].I) {
        in_range = false;
        continue;
      }
      if (lane < R) h0 *= (double)U[t * R + lane];
      if (lane + 64 < R) h1 *= (double)U[t * R + lane + 64];
    }
    if (!in_range) {
      if (lane == 0) {
        a.prob[d] = __builtin_nan("");
        atomicOr(a.status, ST_NUMERIC);
      }
      continue;
    }
    if (lane < R) hb[lane] = h0;
    if (lane + 64 < R) hb[lane + 64] = h1;
    wave_lds_sync();
    double acc = 0.0;
    for (int ia = 0; ia < R; ++ia) {
      for (int ib = ia + lane; ib < R; ib += 64) {
        const double v = hb[ia] * hb[ib] * a.gplus[packed_index(ia, ib, R)];
        acc += ia == ib ? v : 2.0 * v;
      }
    }
    const double q = wave_sum(acc) * inv_rank;
    if (lane == 0) a.prob[d] = q;
    wave_lds_sync();
  }
}

template <typename T, int NP>
hipError_t run_descent(hipStream_t st, const DescentArgs& a) {
  const int TR = a.R * (a.R + 1) / 2;
  const size_t lds = ((TR * 2 + 15) / 16) * 16 + DESC_WAVES * 128 * sizeof(double);
  int64_t blocks = (a.J + DESC_WAVES - 1) / DESC_WAVES;
  if (blocks > 256 * 8) blocks = 256 * 8;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL((descent_kernel<T, NP>), dim3((unsigned)blocks), dim3(64 * DESC_WAVES), lds, st,
                     a);
  return hipGetLastError();
}

template <typename T>
hipError_t dispatch_descent(hipStream_t st, const DescentArgs& a) {
  if (a.R <= 16) return run_descent<T, 3>(st, a);
  if (a.R <= 32) return run_descent<T, 9>(st, a);
  if (a.R <= 64) return run_descent<T, 33>(st, a);
  return run_descent<T, 1>(st, a);
}

}  // namespace

hipError_t launch_descent(hipStream_t st, krps_precision p, const DescentArgs& a) {
  if (a.J <= 0) return hipSuccess;
  if (p == KRPS_FP64) return dispatch_descent<double>(st, a);
  return dispatch_descent<float>(st, a);
}

hipError_t launch_row_prob(hipStream_t st, krps_precision p, const DescentArgs& a) {
  if (a.J <= 0) return hipSuccess;
  int64_t blocks = (a.J + DESC_WAVES - 1) / DESC_WAVES;
  if (blocks > 2048) blocks = 2048;
  if (p == KRPS_FP64)
    hipLaunchKernelGGL(row_prob_kernel<double>, dim3((unsigned)blocks), dim3(64 * DESC_WAVES), 0, st,
                       a);
  else
    hipLaunchKernelGGL(row_prob_kernel<float>, dim3((unsigned)blocks), dim3(64 * DESC_WAVES), 0, st,
                       a);
  return hipGetLastError();
}

}  // namespace krps
