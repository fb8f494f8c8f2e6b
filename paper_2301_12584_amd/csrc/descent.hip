// The batched root-to-leaf descent (the per-sample walk of KRPSample,
// Section 3.2 Algorithm 2; RowSample, Appendix A.5 Algorithm 4).
//
// A group of LPS lanes per sample, 64 / LPS samples per wavefront
// (persistent grid-stride loop over samples).
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
// node (tri(R) elements over the group's lanes) and a butterfly sum over
// the group.  Branch decisions
// and the running offsets low/high are float64 in every precision.
// After the last mode h is the sampled Khatri-Rao row a_d; its probability
// q_d = a_d G^+ a_d^T / rank (Section 2.1) is the same kind of dot product
// against the packed float64 G^+.
#include "device_common.h"
#include "krps_internal.h"

namespace krps {

namespace {

constexpr int DESC_WAVES = 4;  // waves per block
// Waves per SIMD the register allocation of a walk shape must allow: the
// walk is bound by the latency of its dependent reads, so samples in
// flight matter more than registers.  With the packed weights in LDS the
// shapes with 17 entries per lane fit three waves (<= 168 VGPRs) and those
// with 33 two (<= 256, no AGPR overflow); the LDS of a block (4 waves of
// packed weights, h and the index table) allows that many blocks per CU.
template <int NP>
constexpr int desc_min_waves() {
  return NP >= 33 ? 2 : NP >= 17 ? 3 : 1;
}

// Sum over the LPS lanes of one lane group (groups are aligned, LPS a
// power of two <= 64); every lane of the group gets the result.  Within a
// row of 16 lanes the partners come from DPP (quad swaps, half-row and row
// mirrors), across rows from the gfx950 row-swap instructions: VALU
// latency, no LDS round trip.  Every step adds the same two values in both
// partner lanes, so all lanes of the group end with the same bits and take
// the same branch.
__device__ __forceinline__ double swap16_sum(double v) {
  // permlane16_swap(x, x) returns the even rows of x in both rows of each
  // pair, and the odd rows in both rows of each pair
  const int lo = __double2loint(v), hi = __double2hiint(v);
  const auto l = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
  const auto h = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
  return __hiloint2double((int)h[0], (int)l[0]) + __hiloint2double((int)h[1], (int)l[1]);
}
__device__ __forceinline__ double swap32_sum(double v) {
  // the same for the two halves of 32 lanes
  const int lo = __double2loint(v), hi = __double2hiint(v);
  const auto l = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
  const auto h = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
  return __hiloint2double((int)h[0], (int)l[0]) + __hiloint2double((int)h[1], (int)l[1]);
}

template <int LPS>
__device__ __forceinline__ double group_sum(double v) {
  if constexpr (LPS >= 2) v += dpp_d<0xB1>(v);   // quad_perm [1,0,3,2]
  if constexpr (LPS >= 4) v += dpp_d<0x4E>(v);   // quad_perm [2,3,0,1]
  if constexpr (LPS >= 8) v += dpp_d<0x141>(v);  // row_half_mirror
  if constexpr (LPS >= 16) v += dpp_d<0x140>(v); // row_mirror
  if constexpr (LPS >= 32) v = swap16_sum(v);
  if constexpr (LPS >= 64) v = swap32_sum(v);
  return v;
}

// Lane exchange through DPP where lanes without a source lane (outside the
// row, or in a row that ROWMASK leaves out) read 0.
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_or0(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROWMASK, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROWMASK, 0xF, false);
  return __hiloint2double(hi, lo);
}

// Inclusive prefix sum over the LPS lanes of each group: shifts within a
// row of 16 lanes, then the last lane of a row added to the following
// row(s) of the group.
template <int LPS>
__device__ __forceinline__ double group_inclusive_scan(double v, int sl) {
  constexpr int W = LPS < 16 ? LPS : 16;
  if constexpr (W > 1) {
    const double t = dpp_or0<0x111, 0xF>(v);  // row_shr:1
    if (sl >= 1) v += t;
  }
  if constexpr (W > 2) {
    const double t = dpp_or0<0x112, 0xF>(v);  // row_shr:2
    if (sl >= 2) v += t;
  }
  if constexpr (W > 4) {
    const double t = dpp_or0<0x114, 0xF>(v);  // row_shr:4
    if (sl >= 4) v += t;
  }
  if constexpr (W > 8) {
    const double t = dpp_or0<0x118, 0xF>(v);  // row_shr:8
    if (sl >= 8) v += t;
  }
  if constexpr (LPS >= 32) v += dpp_or0<0x142, 0xA>(v);  // row_bcast:15 into rows 1, 3
  if constexpr (LPS >= 64) v += dpp_or0<0x143, 0xC>(v);  // row_bcast:31 into rows 2, 3
  return v;
}

// Value of lane L (a compile-time lane) in every lane.
template <int L>
__device__ __forceinline__ double lane_value(double v) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), L),
                          __builtin_amdgcn_readlane(__double2loint(v), L));
}

// Packed outer product h h^T of the group's float64 vector in hb (LDS),
// off-diagonal terms doubled, held in LDS: entry sl + LPS m at v[LPS m] of
// lane sl's pointer (the group's slot of NP LPS doubles, offset by sl), so
// that each lane reads back only what it wrote (no barrier) and a wave's
// reads of one m are consecutive doubles (no bank conflicts).
template <int LPS, int NP>
struct Packed {
  double* v;
};

// Branch-free: entries past the triangle read entry tri-1 and get weight 0.
// The LDS reads go in batches of 8 entries (a compiler barrier between
// batches) so that at most 8 entries' operands are in flight in registers.
template <int LPS, int NP>
__device__ __forceinline__ void build_packed(Packed<LPS, NP>& P, const double* hb,
                                             const uint16_t* __restrict__ tab, int TR, int sl) {
#pragma unroll
  for (int m = 0; m < NP; ++m) {
    if (m % 8 == 0) asm volatile("" ::: "memory");
    const int p = sl + LPS * m;
    const uint16_t ab = tab[p < TR ? p : TR - 1];
    const int a = ab & 0xff, b = ab >> 8;
    const double w = p < TR ? (a != b ? 2.0 : 1.0) : 0.0;
    P.v[LPS * m] = w * hb[a] * hb[b];
  }
}

// Node mass <h h^T, G^v> = h^T G^v h in float64 whatever the storage type:
// the stored packed triangle (tri(R) entries, read by the group's lanes in
// coalesced strides) dotted with the packed outer product in registers.
template <typename T, int LPS, int NP>
__device__ __forceinline__ double node_mass(const Packed<LPS, NP>& P, const double*,
                                            const T* __restrict__ node, int R, int TR, int sl,
                                            const uint16_t* __restrict__ = nullptr) {
  // all loads first, then the float64 products.  Only the npr strides
  // that reach into the triangle are read (npr is uniform); the last may
  // run up to LPS - 1 entries past the node, into the next node or the
  // zero padding that follows every node array, with packed weight 0.
  const int npr = (TR + LPS - 1) / LPS;
  T g[NP];
  if (npr >= NP) {
#pragma unroll
    for (int m = 0; m < NP; ++m) g[m] = node[sl + LPS * m];
  } else {
#pragma unroll
    for (int m = 0; m < NP; ++m) g[m] = m < npr ? node[sl + LPS * m] : T(0);
  }
  // four partial sums: the dependent chain of FMAs is a quarter as long
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int m = 0; m < NP; ++m) acc[m & 3] += P.v[LPS * m] * (double)g[m];
  return group_sum<LPS>((acc[0] + acc[1]) + (acc[2] + acc[3]));
}

// R > 64 (one sample per wavefront, NP == 0): the packed outer product is
// not held in registers; each lane forms w h_a h_b for its packed entries
// (lane + 64 m) from the (a, b) table and h in LDS, eight entries at a
// time with their loads issued together.
template <typename T>
__device__ __forceinline__ double node_mass(const Packed<64, 0>&, const double* hb,
                                            const T* __restrict__ node, int R, int TR, int lane,
                                            const uint16_t* __restrict__ tab) {
  double acc = 0;
  const int npr = (TR + 63) / 64;
  for (int m0 = 0; m0 < npr; m0 += 8) {
    T g[8];
    uint16_t ab[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int p = lane + 64 * (m0 + q);
      const int pc = p < TR ? p : TR - 1;
      g[q] = node[pc];
      ab[q] = tab[pc];
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int p = lane + 64 * (m0 + q);
      const int a = ab[q] & 0xff, b = ab[q] >> 8;
      const double w = p < TR ? (a != b ? 2.0 : 1.0) : 0.0;
      acc += w * hb[a] * hb[b] * (double)g[q];
    }
  }
  (void)R;
  return group_sum<64>(acc);
}

// The same mass from the float32 copy g32 of a float64 node g64, with
// s = sum_p |P_p g32_p|.  Rounding to nearest gives |g64 - g32| <=
// 2^-24 |g64| (plus 2^-126 where the copy lost range), so the float64 node's
// exact mass is within 2^-24 / (1 - 2^-24) s + 2^-125 sum_p |P_p| of m; the
// float64 sums on either side add a few ulps of s, which the margin below
// (6.0e-8 > 5.9605e-8) covers.
struct MassB {
  double m, s;
};

template <int LPS, int NP>
__device__ __forceinline__ MassB node_mass32(const Packed<LPS, NP>& P, const double*,
                                             const float* __restrict__ node, int TR, int sl,
                                             const uint16_t* __restrict__ = nullptr) {
  const int npr = (TR + LPS - 1) / LPS;
  float g[NP];
  if (npr >= NP) {
#pragma unroll
    for (int m = 0; m < NP; ++m) g[m] = node[sl + LPS * m];
  } else {
#pragma unroll
    for (int m = 0; m < NP; ++m) g[m] = m < npr ? node[sl + LPS * m] : 0.f;
  }
  double acc[4] = {0.0, 0.0, 0.0, 0.0}, sab[2] = {0.0, 0.0};
#pragma unroll
  for (int m = 0; m < NP; ++m) {
    const double t = P.v[LPS * m] * (double)g[m];
    acc[m & 3] += t;
    sab[m & 1] += fabs(t);
  }
  return {group_sum<LPS>((acc[0] + acc[1]) + (acc[2] + acc[3])), group_sum<LPS>(sab[0] + sab[1])};
}

__device__ __forceinline__ MassB node_mass32(const Packed<64, 0>&, const double* hb,
                                             const float* __restrict__ node, int TR, int lane,
                                             const uint16_t* __restrict__ tab) {
  double acc = 0, sab = 0;
  const int npr = (TR + 63) / 64;
  for (int m0 = 0; m0 < npr; m0 += 8) {
    float g[8];
    uint16_t ab[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int p = lane + 64 * (m0 + q);
      const int pc = p < TR ? p : TR - 1;
      g[q] = node[pc];
      ab[q] = tab[pc];
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int p = lane + 64 * (m0 + q);
      const int a = ab[q] & 0xff, b = ab[q] >> 8;
      const double w = p < TR ? (a != b ? 2.0 : 1.0) : 0.0;
      const double t = w * hb[a] * hb[b] * (double)g[q];
      acc += t;
      sab += fabs(t);
    }
  }
  return {group_sum<64>(acc), group_sum<64>(sab)};
}

constexpr double F32_COPY_REL = 6.0e-8;  // >= 2^-24 / (1 - 2^-24) + float64 sums
constexpr double F32_COPY_ABS = 0x1p-124;  // per unit of sum_p |P_p| (range loss)
constexpr double ADD_SLACK = 1e-15;       // float64 additions of the offsets, relative

// Inversion walk down a stored tree (root + left children) for each group's
// sample: returns the leaf position and the offset `low` of its segment.
// All groups of a wavefront walk the same tree, so the loop is uniform and
// only the positions differ.
template <typename T, int LPS, int NP>
__device__ __forceinline__ int64_t walk(const T* __restrict__ nodes, int64_t L, int D,
                                        const Packed<LPS, NP>& P, const double* hb, int R, int TR,
                                        int sl, double x, double C, double& low_out,
                                        const uint16_t* __restrict__ tab) {
  double low = 0.0, high = C;
  int64_t pos = 0;
  int64_t off = 1;
  for (int lev = 1; lev <= D; ++lev) {
    const int64_t cnt_left = ((L - 1) >> (D - lev + 1)) + 1;
    const int64_t real = ((L - 1) >> (D - lev)) + 1;
    double mL = node_mass<T>(P, hb, nodes + (off + pos) * (int64_t)TR, R, TR, sl, tab);
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

// The walk of `walk` over a float64 tree whose levels below `top` are
// decided from its float32 copy.  It tracks approximations lowA, highA of
// the offsets the float64 walk would hold, with |low - lowA| and
// |high - highA| <= B; a level is decided only if the float64 walk's
// comparison has the same outcome for every mass and offset within the
// bounds (left: x <= cut - E; right: x > cut + E and high - cut > 0 for
// sure), else the walk is marked undecided (`amb`) and goes on left, and
// the caller walks that sample again from the float64 tree.  Levels up to
// `top` read the float64 nodes, with the float64 walk's own arithmetic, so
// that B stays 0 there.  sP = sum_p |P_p| = (sum_a |h_a|)^2.
template <int LPS, int NP>
__device__ __forceinline__ int64_t walk_filtered(const double* __restrict__ nodes,
                                                 const float* __restrict__ nodes32, int64_t L,
                                                 int D, int top, const Packed<LPS, NP>& P,
                                                 const double* hb, int R, int TR, int sl, double x,
                                                 double C, double sP, double& low_out,
                                                 double& bound_out, bool& amb,
                                                 const uint16_t* __restrict__ tab) {
  double low = 0.0, high = C, B = 0.0;
  int64_t pos = 0;
  int64_t off = 1;
  amb = false;
  for (int lev = 1; lev <= D; ++lev) {
    const int64_t cnt_left = ((L - 1) >> (D - lev + 1)) + 1;
    const int64_t real = ((L - 1) >> (D - lev)) + 1;
    const bool right_exists = 2 * pos + 1 < real;
    const int64_t at = (off + pos) * (int64_t)TR;
    bool left;
    double cut;
    if (lev <= top) {
      double mL = node_mass<double>(P, hb, nodes + at, R, TR, sl, tab);
      mL = mL > 0.0 ? mL : 0.0;
      cut = low + mL;
      left = cut >= x || !right_exists || high - cut <= 0.0;
    } else {
      const MassB mb = node_mass32(P, hb, nodes32 + at, TR, sl, tab);
      const double mL = mb.m > 0.0 ? mb.m : 0.0;
      cut = low + mL;
      // bound on |cut64 - cut|: the offset's, the mass's (the clamp at 0 is
      // monotone, so it only shrinks it) and the two additions' rounding
      const double beta = F32_COPY_REL * mb.s + F32_COPY_ABS * sP;
      const double E = (B + beta) * (1.0 + 1e-12) + ADD_SLACK * (fabs(cut) + fabs(x));
      if (!(E <= __DBL_MAX__)) amb = true;  // non-finite copy or bound
      if (!right_exists || x <= cut - E) {
        left = true;
      } else if (x > cut + E && (high - B) - (cut + E) > ADD_SLACK * fabs(high)) {
        left = false;
      } else {
        amb = true;
        left = true;
      }
      B = E;
    }
    if (left) {
      high = cut;
      pos = 2 * pos;
    } else {
      low = cut;
      pos = 2 * pos + 1;
    }
    off += cnt_left;
  }
  low_out = low;
  bound_out = B;
  return pos;
}

// The same walk with the node masses read from a table (LDS) instead of
// formed from stored nodes: `tm[n]` is the mass of stored node n.
__device__ __forceinline__ int64_t walk_table(const double* tm, int64_t L, int D, double x,
                                              double C, double& low_out) {
  double low = 0.0, high = C;
  int64_t pos = 0;
  int64_t off = 1;
  for (int lev = 1; lev <= D; ++lev) {
    const int64_t cnt_left = ((L - 1) >> (D - lev + 1)) + 1;
    const int64_t real = ((L - 1) >> (D - lev)) + 1;
    double mL = tm[off + pos];
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

// walk_table over a table in global memory for one lane group, K levels
// per memory round trip: lane m < 2^K - 1 of the group reads the mass of
// stored node (level lev + i, position pos 2^i + j), m = 2^i - 1 + j, i.e.
// every left child the next K levels can reach from the current node;
// the K decisions are then taken from those lanes' values (lane exchange)
// with the arithmetic of walk_table, so the outcome is the same.
// Candidates past a level's stored nodes are clamped into it and never
// chosen (the walk only goes where a right sibling exists).
template <int LPS>
__device__ __forceinline__ int64_t walk_table_group(const double* __restrict__ tm, int64_t L, int D,
                                                    double x, double C, double& low_out, int sl) {
  constexpr int K = LPS >= 64 ? 6 : LPS >= 32 ? 5 : LPS >= 16 ? 4 : LPS >= 8 ? 3 : 2;
  const int li = 31 - __clz(sl + 1);  // this lane's level within a round
  const int lj = sl + 1 - (1 << li);  // and position within that level
  double low = 0.0, high = C;
  int64_t pos = 0;
  int64_t off = 1;
  for (int lev = 1; lev <= D; lev += K) {
    const int nk = K < D - lev + 1 ? K : D - lev + 1;
    double v = 0.0;
    if (li < nk) {
      int64_t o = off;
      for (int i = 0; i < li; ++i) o += ((L - 1) >> (D - (lev + i) + 1)) + 1;
      const int64_t cnt = ((L - 1) >> (D - (lev + li) + 1)) + 1;
      int64_t q = (pos << li) + lj;
      if (q > cnt - 1) q = cnt - 1;
      v = tm[o + q];
    }
    int jb = 0;
    for (int i = 0; i < nk; ++i) {
      const int l = lev + i;
      const int64_t cnt_left = ((L - 1) >> (D - l + 1)) + 1;
      const int64_t real = ((L - 1) >> (D - l)) + 1;
      double mL = __shfl(v, (1 << i) - 1 + jb, LPS);
      mL = mL > 0.0 ? mL : 0.0;
      const double cut = low + mL;
      const bool right_exists = 2 * pos + 1 < real;
      if (cut >= x || !right_exists || high - cut <= 0.0) {
        high = cut;
        pos = 2 * pos;
        jb = 2 * jb;
      } else {
        low = cut;
        pos = 2 * pos + 1;
        jb = 2 * jb + 1;
      }
      off += cnt_left;
    }
  }
  low_out = low;
  return pos;
}

// Dot product of the factor row `ur` (R contiguous values) with hb.  The
// loads of each chunk of up to 32 values are issued together.
template <int RMAX, typename T>
__device__ __forceinline__ double row_dot(const T* __restrict__ ur, const double* hb, int R) {
  constexpr int CH = RMAX < 32 ? RMAX : (sizeof(T) == 8 ? 16 : 32);
  double acc = 0;
  if constexpr (std::is_same_v<T, float>) {
    if ((R & 3) == 0) {
      for (int c0 = 0; c0 < R; c0 += CH) {
        const float4* __restrict__ u4 = (const float4*)(ur + c0);
        float4 v[CH / 4];
#pragma unroll
        for (int q = 0; q < CH / 4; ++q)
          if (c0 + 4 * q < R) v[q] = u4[q];
#pragma unroll
        for (int q = 0; q < CH / 4; ++q)
          if (c0 + 4 * q < R) {
            const double* hh = hb + c0 + 4 * q;
            acc += (double)v[q].x * hh[0] + (double)v[q].y * hh[1] + (double)v[q].z * hh[2] +
                   (double)v[q].w * hh[3];
          }
      }
      return acc;
    }
  } else {
    if ((R & 1) == 0) {
      for (int c0 = 0; c0 < R; c0 += CH) {
        const double2* __restrict__ u2 = (const double2*)(ur + c0);
        double2 v[CH / 2];
#pragma unroll
        for (int q = 0; q < CH / 2; ++q)
          if (c0 + 2 * q < R) v[q] = u2[q];
#pragma unroll
        for (int q = 0; q < CH / 2; ++q)
          if (c0 + 2 * q < R) acc += v[q].x * hb[c0 + 2 * q] + v[q].y * hb[c0 + 2 * q + 1];
      }
      return acc;
    }
  }
  for (int e = 0; e < R; ++e) acc += (double)ur[e] * hb[e];
  return acc;
}

// Leaf scan of each group's leaf [s0, s1): first row i with
// low + sum_{m <= i} r_m >= x, r_m = (U[m] . h~)^2; one row per lane of the
// group, LPS rows at a time.  `nchunk` (uniform) bounds the chunks.
template <int LPS, int RMAX, typename T>
__device__ __forceinline__ int64_t leaf_scan(const T* __restrict__ U, int R, int64_t s0, int64_t s1,
                                             int nchunk, const double* hb, double low, double x,
                                             int sl, int sub) {
  const unsigned long long gmask = LPS == 64 ? ~0ull : ((1ull << LPS) - 1ull);
  int64_t found = -1, last_pos = -1;
  for (int ch = 0; ch < nchunk; ++ch) {
    // h~ is re-read from LDS in every chunk rather than held in registers
    // across the scan (RMAX doubles per lane would cost occupancy)
    asm volatile("" ::: "memory");
    const int64_t base = s0 + (int64_t)ch * LPS;
    const int64_t row = base + sl;
    const bool valid = row < s1;
    // rows past the leaf re-read its last row and count 0
    const double acc = row_dot<RMAX>(U + (valid ? row : s1 - 1) * R, hb, R);
    const double r = valid ? acc * acc : 0.0;
    const double incl = group_inclusive_scan<LPS>(r, sl);
    const bool hit = valid && found < 0 && (low + incl >= x);
    const unsigned long long m = (__ballot(hit) >> (sub * LPS)) & gmask;
    if (found < 0 && m != 0ull) found = base + (__ffsll((long long)m) - 1);
    const unsigned long long pm = (__ballot(valid && r > 0.0) >> (sub * LPS)) & gmask;
    if (pm != 0ull) last_pos = base + (63 - __clzll((long long)pm));
    if constexpr (LPS == 64) {
      low += lane_value<63>(incl);
    } else if constexpr (LPS == 32) {
      const double t0 = lane_value<31>(incl), t1 = lane_value<63>(incl);
      low += sub ? t1 : t0;
    } else {
      low += __shfl(incl, LPS - 1, LPS);
    }
  }
  if (found >= 0) return found;
  return last_pos >= 0 ? last_pos : s1 - 1;
}

// `leaf_scan` with the offset known only as lowA, |low - lowA| <= B (from
// walk_filtered): row i is a sure hit if lowA + incl_i - E >= x, a sure
// miss if lowA + incl_i + E < x; the scan's answer is decided if a sure hit
// comes before every unsure row, or if every row is a sure miss (then the
// float64 scan's fallback rule, which does not read the offset, applies).
// Otherwise `amb` is set.
template <int LPS, int RMAX, typename T>
__device__ __forceinline__ int64_t leaf_scan_filtered(const T* __restrict__ U, int R, int64_t s0,
                                                      int64_t s1, int nchunk, const double* hb,
                                                      double low, double B, double x, int sl,
                                                      int sub, bool& amb) {
  const unsigned long long gmask = LPS == 64 ? ~0ull : ((1ull << LPS) - 1ull);
  int64_t found = -1, last_pos = -1;
  bool undecided = false;
  for (int ch = 0; ch < nchunk; ++ch) {
    asm volatile("" ::: "memory");
    const int64_t base = s0 + (int64_t)ch * LPS;
    const int64_t row = base + sl;
    const bool valid = row < s1;
    const double acc = row_dot<RMAX>(U + (valid ? row : s1 - 1) * R, hb, R);
    const double r = valid ? acc * acc : 0.0;
    const double incl = group_inclusive_scan<LPS>(r, sl);
    const double v = low + incl;
    const double E = B * (1.0 + 1e-12) + ADD_SLACK * (fabs(v) + fabs(x));
    const bool sure = valid && v - E >= x;
    const bool unsure = valid && !sure && v + E >= x;
    const unsigned long long ms = (__ballot(sure) >> (sub * LPS)) & gmask;
    const unsigned long long mu = (__ballot(unsure) >> (sub * LPS)) & gmask;
    if (found < 0 && !undecided) {
      // the first row that may hit decides: a sure hit, or an unsure row
      const unsigned long long any = ms | mu;
      if (any != 0ull) {
        const int f = __ffsll((long long)any) - 1;
        if ((ms >> f) & 1ull)
          found = base + f;
        else
          undecided = true;
      }
    }
    const unsigned long long pm = (__ballot(valid && r > 0.0) >> (sub * LPS)) & gmask;
    if (pm != 0ull) last_pos = base + (63 - __clzll((long long)pm));
    double tot;
    if constexpr (LPS == 64) {
      tot = lane_value<63>(incl);
    } else if constexpr (LPS == 32) {
      const double t0 = lane_value<31>(incl), t1 = lane_value<63>(incl);
      tot = sub ? t1 : t0;
    } else {
      tot = __shfl(incl, LPS - 1, LPS);
    }
    low += tot;
    B = B * (1.0 + 1e-12) + ADD_SLACK * fabs(low);
  }
  amb = undecided;
  if (found >= 0) return found;
  return last_pos >= 0 ? last_pos : s1 - 1;
}

// The walk of the samples base + (lane group) of one wavefront: 64 / LPS
// samples at once, LPS lanes per sample.  `tab` maps packed entry p to its
// (a, b) pair (LDS or global); `hb` is this group's RMAX doubles of LDS.
// NP == 0 selects the masses formed entry by entry from h in LDS (R > 64,
// LPS == 64).
template <typename T, int LPS, int NP, int RMAX>
__device__ __forceinline__ void descend(const DescentArgs& a, int64_t base,
                                        const uint16_t* __restrict__ tab, double* hb, int lane,
                                        double* pslot) {
  constexpr int HE = (RMAX + LPS - 1) / LPS;  // history entries per lane
  const int R = a.R;
  const int TR = R * (R + 1) / 2;
  const int sub = lane / LPS;
  const int sl = lane % LPS;
  const int N = a.N;
  const int64_t J = a.J;
  const double inv_rank = a.rank ? 1.0 / (double)a.rank[0] : 1.0;
  const int64_t d = base + sub;
  const bool active = d < J;
  // history h = (*) of the rows drawn so far, float64; entry e = sl + LPS i
  double h[HE];
#pragma unroll
  for (int i = 0; i < HE; ++i) h[i] = 1.0;
  Packed<LPS, NP> P{pslot + sl};
  // false once a walk's total mass came out <= 0 (finite): rounding of the
  // stored values has swallowed the sample's mass, so its draw is not
  // governed by the method's probabilities and it gets weight 0
  bool mass_ok = true;
  for (int st = 0; st < a.nsteps; ++st) {
    const int k = a.order[st];
    const ModeDesc& md = a.mode[k];
    double d1 = 0.5, d2 = 0.5;
    if (a.u01 != nullptr) {
      if (active) {
        d1 = a.u01[(d * N + k) * 2 + 0];
        d2 = a.u01[(d * N + k) * 2 + 1];
      }
    } else {
      // in-kernel uniforms: Philox4x64-10 of (ctr_base + d, k, c2, 0) under
      // (seed, 0), c2 = ctr2 (+ the device word ctr2_dev when given: the
      // sweep's offset, set outside a captured sweep); word 0 drives stage 1,
      // word 1 stage 2
      const uint64_t c2 = a.ctr2 + (a.ctr2_dev != nullptr ? *a.ctr2_dev : 0ull);
      uint64_t c[4] = {a.ctr_base + (uint64_t)d, (uint64_t)k, c2, 0};
      philox4x64_10(c, a.seed, 0);
      if (active) {
        d1 = u01_of_word(c[0]);
        d2 = u01_of_word(c[1]);
      }
    }
    // ---- stage 1: eigen-component u from E_k
    double C1, low;
    int u;
    if (st == 0 && md.em != nullptr) {
      // first drawn mode: h = 1, so E_k's node masses are the same for
      // every sample; the group walks a copy of them in its LDS slot
      // (ne <= 2^DE <= RMAX stored nodes)
      for (int n = sl; n < md.ne; n += LPS) hb[n] = md.em[n];
      wave_lds_sync();
      C1 = hb[0];
      u = (int)walk_table(hb, (int64_t)R, md.DE, d1 * C1, C1, low);
    } else {
#pragma unroll
      for (int i = 0; i < HE; ++i)
        if (sl + LPS * i < R) hb[sl + LPS * i] = h[i];
      wave_lds_sync();
      if constexpr (NP > 0) build_packed(P, hb, tab, TR, sl);
      const T* __restrict__ E = (const T*)md.E;
      C1 = node_mass<T>(P, hb, E, R, TR, sl, tab);
      u = (int)walk(E, (int64_t)R, md.DE, P, hb, R, TR, sl, d1 * C1, C1, low, tab);
    }
    if (u >= R) u = R - 1;
    // ---- stage 2: row t from Z_k with h~ = h (*) V[:, u]
    const T* __restrict__ V = (const T*)md.V + (int64_t)u * R;
    double ht[HE];
#pragma unroll
    for (int i = 0; i < HE; ++i) {
      const int e = sl + LPS * i;
      ht[i] = e < R ? h[i] * (double)V[e] : 0.0;
    }
    wave_lds_sync();
#pragma unroll
    for (int i = 0; i < HE; ++i)
      if (sl + LPS * i < R) hb[sl + LPS * i] = ht[i];
    wave_lds_sync();
    if constexpr (NP > 0)
      if (!(st == 0 && md.zt != nullptr)) build_packed(P, hb, tab, TR, sl);
    const T* __restrict__ Z = (const T*)md.Z;
    const T* __restrict__ U = (const T*)md.U;
    const int nchunk = (md.F + LPS - 1) / LPS;
    double C2, x2;
    int64_t t;
    if (st == 0 && md.zt != nullptr) {
      // first drawn mode: the node masses for h~ = V[:, u] were tabulated
      // by the preparation; the walk reads one float64 per level
      const double* __restrict__ zt = md.zt + (int64_t)u * md.zn;
      C2 = zt[0];
      x2 = d2 * C2;
      const int64_t c = walk_table_group<LPS>(zt, md.L, md.D, x2, C2, low, sl);
      const int64_t s0 = c * md.F;
      t = leaf_scan<LPS, RMAX>(U, R, s0, s0 + md.F < md.I ? s0 + md.F : md.I, nchunk, hb, low, x2,
                               sl, sub);
    } else {
      C2 = node_mass<T>(P, hb, Z, R, TR, sl, tab);
      x2 = d2 * C2;
      bool plain = true;
      if constexpr (std::is_same_v<T, double>) {
        if (md.z32 != nullptr) {
          // deep levels from the float32 copy; undecided samples (rare:
          // a target within the copy's error of a cut) walk again below
          double sh = 0.0;
#pragma unroll
          for (int i = 0; i < HE; ++i)
            if (sl + LPS * i < R) sh += fabs(ht[i]);
          sh = group_sum<LPS>(sh);
          const double sP = 2.0 * sh * sh;
          double B;
          bool amb_w, amb_l;
          const int64_t c = walk_filtered(Z, md.z32, md.L, md.D, md.ztop, P, hb, R, TR, sl, x2,
                                          C2, sP, low, B, amb_w, tab);
          const int64_t s0 = c * md.F;
          t = leaf_scan_filtered<LPS, RMAX>(U, R, s0, s0 + md.F < md.I ? s0 + md.F : md.I, nchunk,
                                            hb, low, B, x2, sl, sub, amb_l);
          const bool amb = active && (amb_w || amb_l);
          plain = false;
          if (__ballot(amb) != 0ull) {
            const int64_t c2 = walk(Z, md.L, md.D, P, hb, R, TR, sl, x2, C2, low, tab);
            const int64_t s2 = c2 * md.F;
            const int64_t t2 = leaf_scan<LPS, RMAX>(
                U, R, s2, s2 + md.F < md.I ? s2 + md.F : md.I, nchunk, hb, low, x2, sl, sub);
            if (amb) t = t2;
            if (amb && sl == 0) atomicAdd(a.status + 2, 1);
          }
        }
      }
      if (plain) {
        const int64_t c = walk(Z, md.L, md.D, P, hb, R, TR, sl, x2, C2, low, tab);
        const int64_t s0 = c * md.F;
        t = leaf_scan<LPS, RMAX>(U, R, s0, s0 + md.F < md.I ? s0 + md.F : md.I, nchunk, hb, low,
                                 x2, sl, sub);
      }
    }
    if (t < 0) t = 0;
    if (t >= md.I) t = md.I - 1;
    if (sl == 0 && active) a.idx[d * N + k] = (int32_t)t;
#pragma unroll
    for (int i = 0; i < HE; ++i) {
      const int e = sl + LPS * i;
      if (e < R) h[i] *= (double)U[t * R + e];
    }
    if (active && (!(C1 > 0.0) || !(C2 > 0.0))) {
      if (!(fabs(C1) <= __DBL_MAX__) || !(fabs(C2) <= __DBL_MAX__)) {
        if (sl == 0) atomicOr(a.status, ST_NUMERIC);
      } else {
        // C1 (stage 1) or C2 (stage 2) is a p.s.d. form of stored values,
        // > 0 in exact arithmetic; at <= 0 the stored values' rounding
        // exceeds the mass (float32 eigen-tree entries of a G_{>k} with
        // condition number near 2^24 / R)
        if (sl == 0 && mass_ok) atomicAdd(a.status + 1, 1);
        mass_ok = false;
      }
    }
    wave_lds_sync();
  }
  if (a.exclude >= 0 && sl == 0 && active) a.idx[d * N + a.exclude] = -1;
  // ---- probability of the sampled row: q = a G^+ a^T / rank
  if (a.prob != nullptr || a.rows != nullptr || a.rows64 != nullptr || a.wout != nullptr) {
#pragma unroll
    for (int i = 0; i < HE; ++i)
      if (sl + LPS * i < R) hb[sl + LPS * i] = h[i];
    wave_lds_sync();
    if constexpr (NP > 0) build_packed(P, hb, tab, TR, sl);
    const double q = node_mass<double>(P, hb, a.gplus, R, TR, sl, tab) * inv_rank;
    if (active) {
      if (sl == 0 && a.prob != nullptr) a.prob[d] = q;
      // q > 0 in exact arithmetic; where rounding leaves it at or below zero
      // (a row almost in the null space of G^+), or a walk mass was <= 0
      // (above), the sample gets weight 0 and adds nothing to the sketched
      // system, rather than an infinite, NaN or misweighted row.  Such
      // samples are counted once in the second status word; a non-finite q
      // sets the numeric-error flag.
      const bool qok = mass_ok && q > 0.0 && q <= __DBL_MAX__;
      const double w = qok ? 1.0 / sqrt((double)J * q) : 0.0;
      if (sl == 0 && mass_ok && !qok) {
        if (q <= 0.0)
          atomicAdd(a.status + 1, 1);
        else
          atomicOr(a.status, ST_NUMERIC);
      }
      if (sl == 0 && a.wout != nullptr) a.wout[d] = w;
      const double sc = a.scale_rows ? w : 1.0;
      if (a.rows != nullptr) {
        T* rows = (T*)a.rows + d * R;
#pragma unroll
        for (int i = 0; i < HE; ++i) {
          const int e = sl + LPS * i;
          if (e < R) rows[e] = (T)(h[i] * sc);
        }
      }
      if (a.rows64 != nullptr) {
        double* rows = a.rows64 + d * R;
#pragma unroll
        for (int i = 0; i < HE; ++i) {
          const int e = sl + LPS * i;
          if (e < R) rows[e] = h[i] * sc;
        }
      }
    }
    wave_lds_sync();
  }
}

// (a, b) of every packed entry p of an R x R upper triangle.
__device__ __forceinline__ void fill_tab(uint16_t* tab, int R, int t0, int nt) {
  const int TR = R * (R + 1) / 2;
  for (int p = t0; p < TR; p += nt) {
    int aa = 0;
    while (aa < R - 1 && packed_index(aa + 1, aa + 1, R) <= p) ++aa;
    const int bb = aa + (int)(p - packed_index(aa, aa, R));
    tab[p] = (uint16_t)(aa | (bb << 8));
  }
}

// One problem: persistent grid-stride loop of the wavefronts over groups
// of 64 / LPS samples.
template <typename T, int LPS, int NP, int RMAX>
__global__ __launch_bounds__(64 * DESC_WAVES, desc_min_waves<NP>()) void descent_kernel(
    DescentArgs a) {
  constexpr int G = 64 / LPS;
  extern __shared__ unsigned char smem_raw[];
  const int R = a.R;
  const int TR = R * (R + 1) / 2;
  uint16_t* tab = (uint16_t*)smem_raw;
  double* hb_all = (double*)(smem_raw + ((TR * 2 + 15) / 16) * 16);
  double* p_all = hb_all + DESC_WAVES * 128;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  double* hb = hb_all + wave * 128 + (lane / LPS) * RMAX;
  double* pslot = p_all + (wave * 64 + (lane / LPS) * LPS) * NP;
  fill_tab(tab, R, threadIdx.x, blockDim.x);
  __syncthreads();
  const int64_t stride = (int64_t)gridDim.x * DESC_WAVES * G;
  for (int64_t base = ((int64_t)blockIdx.x * DESC_WAVES + wave) * G; base < a.J; base += stride)
    descend<T, LPS, NP, RMAX>(a, base, tab, hb, lane, pslot);
}

// Shape classes of the batched walk (lanes per sample, packed entries per
// lane, largest R): the default shape of R <= 8, 16, 32, 64, 128, then the
// other lanes-per-sample choices of R <= 8, 16, 32 (krps_sampler_set_lps).
template <int CLS> struct Cls;
template <> struct Cls<0> { static constexpr int LPS = 4, NP = 9, RMAX = 8; };
template <> struct Cls<1> { static constexpr int LPS = 8, NP = 17, RMAX = 16; };
template <> struct Cls<2> { static constexpr int LPS = 32, NP = 17, RMAX = 32; };
template <> struct Cls<3> { static constexpr int LPS = 64, NP = 33, RMAX = 64; };
template <> struct Cls<4> { static constexpr int LPS = 64, NP = 0, RMAX = 128; };
template <> struct Cls<5> { static constexpr int LPS = 8, NP = 5, RMAX = 8; };
template <> struct Cls<6> { static constexpr int LPS = 16, NP = 9, RMAX = 16; };
template <> struct Cls<7> { static constexpr int LPS = 16, NP = 33, RMAX = 32; };
template <> struct Cls<8> { static constexpr int LPS = 64, NP = 9, RMAX = 32; };

// Many problems of one shape class in one persistent launch (Appendix
// A.10 batching): every wavefront takes the next task -- (problem, group
// of 64 / LPS samples) -- from a device counter until all tasks are taken;
// problems are ordered by decreasing cost on the host, so the largest
// start first.  One kernel per class keeps each class's register budget
// (and so its occupancy) instead of the largest class's.
template <typename T, int CLS>
__global__ __launch_bounds__(64 * DESC_WAVES, desc_min_waves<Cls<CLS>::NP>()) void descent_batched_kernel(
    const BatchProblem* __restrict__ probs, int P, int64_t ntask,
    unsigned long long* __restrict__ counter) {
  using C = Cls<CLS>;
  __shared__ double hb_all[DESC_WAVES * 128];
  __shared__ double p_all[DESC_WAVES * 64 * (C::NP > 0 ? C::NP : 1)];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  double* hb = hb_all + wave * 128 + (lane / C::LPS) * C::RMAX;
  double* pslot = p_all + (wave * 64 + (lane / C::LPS) * C::LPS) * C::NP;
  // task numbers are wave-uniform (scalar registers), so the problem's
  // descriptor is read with scalar loads; the next task is claimed before
  // the current one is walked, which hides the counter's latency
  unsigned int claim = 0;
  if (lane == 0) claim = (unsigned int)atomicAdd(counter, 1ull);
  unsigned int next = __builtin_amdgcn_readfirstlane(claim);
  for (;;) {
    const long long t = (long long)next;
    if (t >= ntask) break;
    claim = 0;
    if (lane == 0) claim = (unsigned int)atomicAdd(counter, 1ull);
    int lo = 0, hi = P;  // last problem with task0 <= t
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (probs[mid].task0 <= t) lo = mid; else hi = mid;
    }
    const BatchProblem& b = probs[lo];
    const int64_t base = (t - b.task0) * (int64_t)(64 / C::LPS);
    descend<T, C::LPS, C::NP, C::RMAX>(b.a, base, b.tab, hb, lane, pslot);
    next = __builtin_amdgcn_readfirstlane(claim);
  }
}

// Packed-index table of each problem's R (one block per problem).
__global__ void batch_tab_kernel(const BatchProblem* __restrict__ probs) {
  const BatchProblem& b = probs[blockIdx.x];
  fill_tab((uint16_t*)b.tab, b.a.R, threadIdx.x, blockDim.x);
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

template <typename T, int LPS, int NP, int RMAX>
hipError_t run_descent(hipStream_t st, const DescentArgs& a) {
  constexpr int G = 64 / LPS;
  const int TR = a.R * (a.R + 1) / 2;
  const size_t lds = ((TR * 2 + 15) / 16) * 16 + DESC_WAVES * 128 * sizeof(double) +
                     (size_t)DESC_WAVES * 64 * NP * sizeof(double);
  int64_t blocks = (a.J + DESC_WAVES * G - 1) / (DESC_WAVES * G);
  if (blocks > 256 * 8) blocks = 256 * 8;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL((descent_kernel<T, LPS, NP, RMAX>), dim3((unsigned)blocks),
                     dim3(64 * DESC_WAVES), lds, st, a);
  return hipGetLastError();
}

// Lanes per sample (LPS) and packed entries per lane (NP = ceil(tri/LPS));
// `lps` (0 = default) selects among the compiled variants.
template <typename T>
hipError_t dispatch_descent(hipStream_t st, const DescentArgs& a, int lps) {
  if (a.R <= 8) return lps == 8 ? run_descent<T, 8, 5, 8>(st, a) : run_descent<T, 4, 9, 8>(st, a);
  if (a.R <= 16)
    return lps == 16 ? run_descent<T, 16, 9, 16>(st, a) : run_descent<T, 8, 17, 16>(st, a);
  if (a.R <= 32) {
    if (lps == 64) return run_descent<T, 64, 9, 32>(st, a);
    if (lps == 16) return run_descent<T, 16, 33, 32>(st, a);
    return run_descent<T, 32, 17, 32>(st, a);
  }
  if (a.R <= 64) return run_descent<T, 64, 33, 64>(st, a);
  return run_descent<T, 64, 0, 128>(st, a);
}

}  // namespace

hipError_t launch_descent(hipStream_t st, krps_precision p, const DescentArgs& a) {
  if (a.J <= 0) return hipSuccess;
  if (p == KRPS_FP64) return dispatch_descent<double>(st, a, a.lps);
  return dispatch_descent<float>(st, a, a.lps);
}

int batch_class(int R, int lps) {
  if (R <= 8) return lps == 8 ? 5 : 0;
  if (R <= 16) return lps == 16 ? 6 : 1;
  if (R <= 32) return lps == 16 ? 7 : lps == 64 ? 8 : 2;
  return R <= 64 ? 3 : 4;
}
int batch_group(int cls) {
  static const int lps[NBATCH_CLASSES] = {4, 8, 32, 64, 64, 8, 16, 16, 64};
  return 64 / lps[cls];
}

template <typename T, int CLS>
void launch_cls(hipStream_t st, int64_t blocks, const BatchProblem* probs, int P, int64_t ntask,
                unsigned long long* counter) {
  hipLaunchKernelGGL((descent_batched_kernel<T, CLS>), dim3((unsigned)blocks),
                     dim3(64 * DESC_WAVES), 0, st, probs, P, ntask, counter);
}

template <typename T>
void launch_batched_t(hipStream_t st, int cls, int64_t blocks, const BatchProblem* probs, int P,
                      int64_t ntask, unsigned long long* counter) {
  switch (cls) {
    case 0: launch_cls<T, 0>(st, blocks, probs, P, ntask, counter); break;
    case 1: launch_cls<T, 1>(st, blocks, probs, P, ntask, counter); break;
    case 2: launch_cls<T, 2>(st, blocks, probs, P, ntask, counter); break;
    case 3: launch_cls<T, 3>(st, blocks, probs, P, ntask, counter); break;
    case 4: launch_cls<T, 4>(st, blocks, probs, P, ntask, counter); break;
    case 5: launch_cls<T, 5>(st, blocks, probs, P, ntask, counter); break;
    case 6: launch_cls<T, 6>(st, blocks, probs, P, ntask, counter); break;
    case 7: launch_cls<T, 7>(st, blocks, probs, P, ntask, counter); break;
    default: launch_cls<T, 8>(st, blocks, probs, P, ntask, counter); break;
  }
}

hipError_t launch_descent_batched(hipStream_t st, bool f64, int cls, const BatchProblem* probs,
                                  int P, int64_t ntask, unsigned long long* counter) {
  hipLaunchKernelGGL(batch_tab_kernel, dim3((unsigned)P), dim3(256), 0, st, probs);
  if (ntask <= 0) return hipGetLastError();
  int64_t blocks = (ntask + DESC_WAVES - 1) / DESC_WAVES;
  if (blocks > 256 * 8) blocks = 256 * 8;
  if (f64)
    launch_batched_t<double>(st, cls, blocks, probs, P, ntask, counter);
  else
    launch_batched_t<float>(st, cls, blocks, probs, P, ntask, counter);
  return hipGetLastError();
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
