// Per-draw preparation in float64 (KRPSample, Section 3.2 Algorithm 2,
// lines 1-5): G = (*)_{k != j} G_k, its pseudo-inverse and rank, every
// G_{>k} = G^+ (*) prod_{m > k, m != j} G_m, their eigendecompositions
// G_{>k} = V_k Lambda_k V_k^T, and the eigen-trees E_k =
// BuildSampler(sqrt(Lambda_k) V_k^T, F = 1, G_k).
//
// Symmetric eigendecomposition: one-sided (Hestenes) Jacobi on one
// workgroup with the R x R matrix resident in LDS (R <= 128: at most
// 128 KiB of the 160 KiB).  Column pairs are rotated in parallel in the
// round-robin (circle) order, one team of lanes per pair.  For a symmetric
// p.s.d. matrix the converged columns are lambda_i v_i, so the eigenvalues
// are their norms and the eigenvectors their directions; no separate V is
// accumulated, which is what lets R = 128 fit in LDS.
#include <cfloat>

#include "device_common.h"
#include "krps_internal.h"

namespace krps {

namespace {

constexpr int PREP_THREADS = 1024;

struct GList {
  const double* G[KRPS_MAX_MODES];
  int order[KRPS_MAX_MODES];
};

__device__ __forceinline__ double team_sum(double v, int team) {
  for (int o = team >> 1; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// One-sided Jacobi on the columns of A (column c at A + c*R), all threads
// of the block.  `flag` is an int in LDS.
__device__ void jacobi_columns(double* A, int R, int* flag) {
  const int tid = threadIdx.x;
  const int n = R + (R & 1);
  const int npairs = n / 2;
  int team = blockDim.x / npairs;
  if (team > 64) team = 64;
  int t2 = 1;
  while (t2 * 2 <= team) t2 *= 2;
  team = t2;
  const int s = tid / team;
  const int li = tid % team;
  const double tol = (double)R * DBL_EPSILON;
  for (int sweep = 0; sweep < 40; ++sweep) {
    __syncthreads();
    if (tid == 0) *flag = 0;
    __syncthreads();
    for (int step = 0; step < n - 1; ++step) {
      if (s < npairs) {
        const int i0 = s, i1 = n - 1 - s;
        const int p = (i0 == 0) ? 0 : 1 + ((i0 - 1 + step) % (n - 1));
        const int q = 1 + ((i1 - 1 + step) % (n - 1));
        if (p < R && q < R) {
          double al = 0, be = 0, ga = 0;
          for (int r = li; r < R; r += team) {
            const double x = A[p * R + r], y = A[q * R + r];
            al += x * x;
            be += y * y;
            ga += x * y;
          }
          al = team_sum(al, team);
          be = team_sum(be, team);
          ga = team_sum(ga, team);
          if (al > 0 && be > 0 && fabs(ga) > tol * sqrt(al * be)) {
            const double zeta = (be - al) / (2.0 * ga);
            double t;
            if (fabs(zeta) > 1e150)
              t = 0.5 / zeta;
            else
              t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
            const double c = 1.0 / sqrt(1.0 + t * t);
            const double sn = c * t;
            for (int r = li; r < R; r += team) {
              const double x = A[p * R + r], y = A[q * R + r];
              A[p * R + r] = c * x - sn * y;
              A[q * R + r] = sn * x + c * y;
            }
            if (li == 0) *flag = 1;
          }
        }
      }
      __syncthreads();
    }
    if (*flag == 0) break;
  }
  __syncthreads();
}

// Column norms into lam[], columns normalised in place (zero columns stay).
__device__ void norms_and_normalise(double* A, int R, double* lam) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int c = wave; c < R; c += nw) {
    double ss = 0;
    for (int r = lane; r < R; r += 64) ss += A[c * R + r] * A[c * R + r];
    ss = wave_sum(ss);
    if (lane == 0) lam[c] = sqrt(ss);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < R * R; i += blockDim.x) {
    const double l = lam[i / R];
    A[i] = l > 0 ? A[i] / l : 0.0;
  }
  __syncthreads();
}

// G = (*) of the listed Grams -> G^+ (full and packed), rank, and G_{>k}
// for the drawn modes order[0..nsteps-1] (nsteps may be 0).
__global__ __launch_bounds__(PREP_THREADS) void prep_gplus_kernel(
    GList gl, int nmat, int R, int nsteps,
    double* __restrict__ gplus_full, double* __restrict__ gplus_packed, int32_t* __restrict__ rank,
    double* __restrict__ ggt, int32_t* __restrict__ status) {
  extern __shared__ double smem[];
  double* A = smem;                 // R*R
  double* lam = A + R * R;          // R
  double* red = lam + R;            // 2
  int* flag = (int*)(red + 2);
  const int tid = threadIdx.x;
  for (int i = tid; i < R * R; i += blockDim.x) {
    double v = 1.0;
    for (int m = 0; m < nmat; ++m) v *= gl.G[m][i];
    A[i] = v;
  }
  __syncthreads();
  jacobi_columns(A, R, flag);
  norms_and_normalise(A, R, lam);
  if (tid == 0) {
    double lmax = 0;
    for (int c = 0; c < R; ++c) lmax = fmax(lmax, lam[c]);
    const double tau = (double)R * DBL_EPSILON * lmax;
    int rk = 0;
    for (int c = 0; c < R; ++c) rk += lam[c] > tau;
    red[0] = tau;
    rank[0] = rk;
    if (status != nullptr && (lmax == 0.0 || !(lmax < INFINITY)))
      atomicOr(status, lmax == 0.0 ? ST_ZERO : ST_NUMERIC);
  }
  __syncthreads();
  const double tau = red[0];
  for (int i = tid; i < R * R; i += blockDim.x) {
    const int a = i / R, b = i % R;
    double v = 0;
    for (int c = 0; c < R; ++c)
      if (lam[c] > tau) v += A[c * R + a] * A[c * R + b] / lam[c];
    gplus_full[i] = v;
    if (gplus_packed != nullptr && a <= b) gplus_packed[packed_index(a, b, R)] = v;
    // G_{>k}: later drawn modes' Grams multiplied in
    for (int st = 0; st < nsteps; ++st) {
      double w = v;
      for (int s2 = st + 1; s2 < nsteps; ++s2) w *= gl.G[s2][i];
      ggt[(int64_t)gl.order[st] * R * R + i] = w;
    }
  }
}

// One block per drawn mode: eigendecomposition of G_{>k} (ascending), the
// eigenvectors in the factor type and the eigen-tree E_k.
template <typename T>
__global__ __launch_bounds__(PREP_THREADS) void prep_eig_kernel(
    GList gk, int R, const double* __restrict__ ggt,
    double* __restrict__ lam_out, T* __restrict__ vecs, T* __restrict__ etree, int64_t enodes) {
  extern __shared__ double smem[];
  double* A = smem;
  double* lam = A + R * R;
  int* perm = (int*)(lam + R);
  int* flag = perm + R;
  const int st = blockIdx.x;
  const int k = gk.order[st];
  const double* __restrict__ Gk = gk.G[st];
  const int tid = threadIdx.x;
  for (int i = tid; i < R * R; i += blockDim.x) A[i] = ggt[(int64_t)k * R * R + i];
  __syncthreads();
  jacobi_columns(A, R, flag);
  norms_and_normalise(A, R, lam);
  // ascending order, ties by column index
  for (int c = tid; c < R; c += blockDim.x) {
    int rk = 0;
    const double lc = lam[c];
    for (int c2 = 0; c2 < R; ++c2) rk += (lam[c2] < lc) || (lam[c2] == lc && c2 < c);
    perm[rk] = c;
  }
  __syncthreads();
  for (int i = tid; i < R * R; i += blockDim.x) {
    const int u = i / R, e = i % R;
    vecs[(int64_t)k * R * R + i] = (T)A[perm[u] * R + e];
    if (e == 0) lam_out[(int64_t)k * R + u] = lam[perm[u]];
  }
  // eigen-tree over the R rows sqrt(lam_u) v_u^T with Y = G_k: node masses
  // <h h^T, P^v, G_k> with P^v = sum_{u in S(v)} lam_u v_u v_u^T; the
  // stored node is P^v (*) G_k (packed upper triangle).
  const int64_t TR = (int64_t)R * (R + 1) / 2;
  const int DE = R > 1 ? 32 - __builtin_clz((unsigned)(R - 1)) : 0;
  const int64_t Lp = int64_t(1) << DE;
  T* __restrict__ E = etree + (int64_t)k * enodes * TR;
  for (int64_t p = tid; p < TR; p += blockDim.x) {
    // (a, b) of packed entry p
    int a = 0;
    while (a < R - 1 && packed_index(a + 1, a + 1, R) <= p) ++a;
    const int b = a + (int)(p - packed_index(a, a, R));
    const double g = Gk[a * R + b];
    double stack[8];
    for (int64_t u = 0; u < Lp; ++u) {
      double v = 0;
      if (u < R) {
        const int c = perm[u];
        v = lam[c] * A[c * R + a] * A[c * R + b] * g;
      }
      int t = __builtin_ctzll(~(unsigned long long)u);
      if (t > DE) t = DE;
      for (int m = 0; m < t; ++m) v += stack[m];
      const int lev = DE - t;
      const int64_t pos = u >> t;
      if (lev == 0) {
        E[p] = (T)v;
      } else {
        if (pos < ((int64_t)(R - 1) >> (DE - lev)) + 1)
          E[(level_offset(R, DE, lev) + (pos >> 1)) * TR + p] = (T)v;
        stack[t] = v;
      }
    }
  }
}

hipError_t set_lds(const void* fn, size_t bytes) {
  return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

}  // namespace

size_t prep_lds_bytes(int R) { return (size_t)R * R * 8 + (size_t)R * 8 + 64 + (size_t)R * 4 + 64; }

hipError_t launch_prep_gplus2(hipStream_t st, int R, int nmat, const double* const* mats,
                              int nsteps, const int* order, double* gplus_full,
                              double* gplus_packed, int32_t* rank, double* ggt, int32_t* status) {
  GList gl{};
  for (int m = 0; m < nmat; ++m) gl.G[m] = mats[m];
  for (int m = 0; m < nsteps; ++m) gl.order[m] = order[m];
  const size_t lds = prep_lds_bytes(R);
  hipError_t e = set_lds((const void*)prep_gplus_kernel, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(prep_gplus_kernel, dim3(1), dim3(PREP_THREADS), lds, st, gl, nmat, R, nsteps,
                     gplus_full, gplus_packed, rank, ggt, status);
  return hipGetLastError();
}

hipError_t launch_prep_eig2(hipStream_t st, krps_precision p, int R, int nsteps,
                            const double* const* Gsteps, const int* order, const double* ggt,
                            double* lam, void* vecs, void* etree, int64_t enodes) {
  GList gl{};
  for (int m = 0; m < nsteps; ++m) {
    gl.G[m] = Gsteps[m];
    gl.order[m] = order[m];
  }
  const size_t lds = prep_lds_bytes(R);
  hipError_t e;
  if (p == KRPS_FP64) {
    e = set_lds((const void*)prep_eig_kernel<double>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(prep_eig_kernel<double>, dim3(nsteps), dim3(PREP_THREADS), lds, st, gl,
                       R, ggt, lam, (double*)vecs, (double*)etree, enodes);
  } else {
    e = set_lds((const void*)prep_eig_kernel<float>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(prep_eig_kernel<float>, dim3(nsteps), dim3(PREP_THREADS), lds, st, gl,
                       R, ggt, lam, (float*)vecs, (float*)etree, enodes);
  }
  return hipGetLastError();
}

hipError_t launch_pinv(hipStream_t st, int R, const double* M, double* Mp_full, int32_t* rank) {
  const double* mats[1] = {M};
  return launch_prep_gplus2(st, R, 1, mats, 0, nullptr, Mp_full, nullptr, rank, nullptr, nullptr);
}

}  // namespace krps
