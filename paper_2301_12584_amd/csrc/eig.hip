// Per-draw preparation in float64 (the set-up part of KRPSample, Section
// 3.2 Algorithm 2, before the per-sample loop): G = (*)_{k != j} G_k, its pseudo-inverse and rank, every
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

constexpr int PREP_THREADS = 1024;  // upper bound; launches use prep_threads(R)
constexpr int jacobi_team(int R);

// Block size of the one-workgroup eigensolver: a full 1024-thread block,
// so that the phases around the Jacobi sweeps (Cholesky, inverse,
// eigen-tree), whose loops run over all threads, use every SIMD; one team
// per column pair works in the sweeps and wavefronts without a pair only
// keep its barriers.
int prep_threads(int R) {
  const int npairs = (R + (R & 1)) / 2;
  int t = npairs * jacobi_team(R);
  if (t < 1024) t = 1024;
  if (t > PREP_THREADS) t = PREP_THREADS;
  return (t + 63) / 64 * 64;
}

// Sum over an aligned team of TEAM (1, 2, 4, 8 or 16) lanes: quad swaps,
// then half-row and row mirrors.
template <int TEAM>
__device__ __forceinline__ double team_sum(double v) {
  if constexpr (TEAM >= 2) v += dpp_d<0xB1>(v);   // quad_perm [1,0,3,2]
  if constexpr (TEAM >= 4) v += dpp_d<0x4E>(v);   // quad_perm [2,3,0,1]
  if constexpr (TEAM >= 8) v += dpp_d<0x141>(v);  // row_half_mirror
  if constexpr (TEAM >= 16) v += dpp_d<0x140>(v); // row_mirror
  return v;
}

// Team of lanes per column pair for a given R (RPL rows per lane at most).
constexpr int jacobi_team(int R) { return R <= 32 ? 4 : 16; }

// One-sided Jacobi on the columns of A (column c at A + c*RS, RS = R + 1 so
// that the columns of a step fall in different LDS banks).  Each step
// rotates the R/2 disjoint column pairs of the round-robin (circle)
// schedule in parallel, one team of TEAM lanes per pair; a lane keeps its
// <= RPL rows of both columns in registers between the dot products and
// the rotation.  `flag` is an int in LDS.  Returns the number of sweeps.
// One rotation of columns p and q (team lane li holds rows li + TEAM i):
// their dot products over the team, then the rotation that makes them
// orthogonal, unless they already are within tol.  Sets *flag on a
// rotation.
template <int TEAM, int RPL>
__device__ __forceinline__ void jacobi_rotate(double* A, int R, int RS, int p, int q, bool act,
                                              int li, double tol, int* flag) {
  double x[RPL], y[RPL];
  double al = 0, be = 0, ga = 0;
#pragma unroll
  for (int i = 0; i < RPL; ++i) {
    const int r = li + TEAM * i;
    const bool ok = act && r < R;
    x[i] = ok ? A[p * RS + r] : 0.0;
    y[i] = ok ? A[q * RS + r] : 0.0;
    al += x[i] * x[i];
    be += y[i] * y[i];
    ga += x[i] * y[i];
  }
  al = team_sum<TEAM>(al);
  be = team_sum<TEAM>(be);
  ga = team_sum<TEAM>(ga);
  if (act && al > 0 && be > 0 && ga * ga > (tol * tol) * (al * be)) {
    // tangent of the rotation angle, the root of t^2 + 2 zeta t - 1 = 0
    // of smaller magnitude (zeta = (be - al) / (2 ga))
    const double dd = be - al, g2 = 2.0 * ga;
    const double rr = sqrt(dd * dd + g2 * g2);
    const double t = g2 / (dd + (dd >= 0 ? rr : -rr));
    const double c = rsqrt(1.0 + t * t);
    const double sn = c * t;
#pragma unroll
    for (int i = 0; i < RPL; ++i) {
      const int r = li + TEAM * i;
      if (r < R) {
        A[p * RS + r] = c * x[i] - sn * y[i];
        A[q * RS + r] = sn * x[i] + c * y[i];
      }
    }
    if (li == 0) *flag = 1;
  }
}

template <int TEAM, int RPL>
__device__ int jacobi_columns_t(double* A, int R, int* flag) {
  const int RS = R + 1;
  const int tid = threadIdx.x;
  const int n = R + (R & 1);
  const int npairs = n / 2;
  const int s = tid / TEAM;
  const int li = tid % TEAM;
  // a pair counts as orthogonal below tol * |a_p| |a_q|; rounding keeps the
  // computed cosine of ill-separated columns near eps * kappa, so a tighter
  // tol would only spin until the sweep cap
  const double tol = 1e-13;
  int sweep = 0;
  if (npairs * TEAM <= 64) {
    // every pair in wavefront 0: it runs the sweeps with wavefront-level
    // LDS ordering between the steps, the other wavefronts wait once
    if (tid < 64) {
      for (; sweep < 24; ++sweep) {
        if (tid == 0) *flag = 0;
        wave_lds_sync();
        int cp = s == 0 ? 0 : (s - 1) % (n - 1);
        int cq = (n - 2 - s) % (n - 1);
        for (int step = 0; step < n - 1; ++step) {
          int p = 0, q = 0;
          bool act = s < npairs;
          if (act) {
            p = (s == 0) ? 0 : 1 + cp;
            q = 1 + cq;
            act = p < R && q < R;
          }
          cp = cp + 1 == n - 1 ? 0 : cp + 1;
          cq = cq + 1 == n - 1 ? 0 : cq + 1;
          jacobi_rotate<TEAM, RPL>(A, R, RS, p, q, act, li, tol, flag);
          wave_lds_sync();
        }
        if (*flag == 0) break;
      }
    }
    __syncthreads();
    return sweep + 1;
  }
  for (; sweep < 24; ++sweep) {
    __syncthreads();
    if (tid == 0) *flag = 0;
    __syncthreads();
    // circle schedule: position 0 is fixed, the others rotate by one per
    // step; pair s holds positions s and n-1-s
    int cp = s == 0 ? 0 : (s - 1) % (n - 1);
    int cq = (n - 2 - s) % (n - 1);
    // wavefronts that hold no pair only keep the barriers
    const bool wave_busy = (tid & ~63) / TEAM < npairs;
    for (int step = 0; step < n - 1; ++step) {
      if (!wave_busy) {
        __syncthreads();
        continue;
      }
      int p = 0, q = 0;
      bool act = s < npairs;
      if (act) {
        p = (s == 0) ? 0 : 1 + cp;
        q = 1 + cq;
        act = p < R && q < R;
      }
      cp = cp + 1 == n - 1 ? 0 : cp + 1;
      cq = cq + 1 == n - 1 ? 0 : cq + 1;
      jacobi_rotate<TEAM, RPL>(A, R, RS, p, q, act, li, tol, flag);
      __syncthreads();
    }
    if (*flag == 0) break;
  }
  __syncthreads();
  return sweep + 1;
}
__device__ int jacobi_columns(double* A, int R, int* flag) {
  // rows per lane: just enough for the largest R of each branch
  if (R <= 32) return jacobi_columns_t<jacobi_team(32), 32 / jacobi_team(32)>(A, R, flag);
  if (R <= 64) return jacobi_columns_t<jacobi_team(64), 64 / jacobi_team(64)>(A, R, flag);
  return jacobi_columns_t<jacobi_team(128), 128 / jacobi_team(128)>(A, R, flag);
}

// Column norms into lam[], columns normalised in place (zero columns stay).
__device__ void norms_and_normalise(double* A, int R, double* lam) {
  const int RS = R + 1;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int c = wave; c < R; c += nw) {
    double ss = 0;
    for (int r = lane; r < R; r += 64) ss += A[c * RS + r] * A[c * RS + r];
    ss = wave_sum(ss);
    if (lane == 0) lam[c] = sqrt(ss);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < R * R; i += blockDim.x) {
    const int c = i / R, r = i % R;
    const double l = lam[c];
    A[c * RS + r] = l > 0 ? A[c * RS + r] / l : 0.0;
  }
  __syncthreads();
}

// In place in the lower triangle of A (column c at A + c*RS, G in full on
// entry): the Cholesky factor L of G = L L^T, then L^{-1} in place of L
// (right-looking factorisation, right-to-left triangular inverse).  One
// wavefront (lane l holds rows l, l + 64): the R dependent column steps of
// each phase are ordered by wave-level LDS waits, not workgroup barriers
// (two barriers per column across the workgroup cost ~0.25 ms at R = 64).
// False if a pivot is not positive (every lane reads the same pivot, so
// all return together).  `tmp` holds R doubles of LDS.  Call from the
// threads of one wavefront only.
__device__ bool cholesky_inverse_lower_wave(double* A, int R, double* tmp) {
  const int RS = R + 1, lane = threadIdx.x & 63;
  for (int j = 0; j < R; ++j) {
    const double d = A[j * RS + j];  // the same value in every lane
    if (!(d > 0.0) || !(d < INFINITY)) return false;
    const double ljj = sqrt(d), inv = 1.0 / ljj;
    for (int i = j + 1 + lane; i < R; i += 64) A[j * RS + i] *= inv;
    wave_lds_sync();
    // trailing lower triangle (i, k), j < k <= i: each lane its rows, eight
    // entries at a time with every load issued before the stores
    for (int i = j + 1 + lane; i < R; i += 64) {
      const double li = A[j * RS + i];
      for (int k0 = j + 1; k0 <= i; k0 += 8) {
        double a[8], l[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const int k = k0 + q <= i ? k0 + q : i;
          a[q] = A[k * RS + i];
          l[q] = A[j * RS + k];
        }
#pragma unroll
        for (int q = 0; q < 8; ++q)
          if (k0 + q <= i) A[(k0 + q) * RS + i] = a[q] - li * l[q];
      }
    }
    if (lane == 0) A[j * RS + j] = ljj;
    wave_lds_sync();
  }
  for (int j = R - 1; j >= 0; --j) {
    for (int i = j + 1 + lane; i < R; i += 64) tmp[i] = A[j * RS + i];
    wave_lds_sync();
    const double xjj = 1.0 / A[j * RS + j];
    // column j of L^{-1} below the diagonal from the columns right of it
    for (int i = j + 1 + lane; i < R; i += 64) {
      double acc[2] = {0.0, 0.0};
      for (int k0 = j + 1; k0 <= i; k0 += 8) {
        double a[8], t[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const int k = k0 + q <= i ? k0 + q : i;
          a[q] = A[k * RS + i];
          t[q] = k0 + q <= i ? tmp[k] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) acc[q & 1] += a[q] * t[q];
      }
      A[j * RS + i] = -xjj * (acc[0] + acc[1]);
    }
    wave_lds_sync();
    if (lane == 0) A[j * RS + j] = xjj;
    wave_lds_sync();
  }
  return true;
}

// (G^{-1})_{ab} = sum_{i >= max(a, b)} X_{ia} X_{ib} from X = L^{-1} (lower
// triangle of A).
__device__ __forceinline__ double inverse_entry(const double* A, int R, int a, int b) {
  const int RS = R + 1;
  double v = 0;
  for (int i = a > b ? a : b; i < R; ++i) v += A[a * RS + i] * A[b * RS + i];
  return v;
}

// Entry (a, b) of G^{-1} once stored in the upper triangle of A (column b,
// row a < b) with the diagonal in lam.
__device__ __forceinline__ double stored_inverse(const double* A, const double* lam, int RS, int a,
                                                 int b) {
  return a == b ? lam[a] : a < b ? A[b * RS + a] : A[a * RS + b];
}

// A (column c at A + c*RS) = (*) of the nmat listed Grams; then a barrier.
__device__ void load_hadamard(const GList& gl, int nmat, int R, double* A) {
  const int RS = R + 1;
  for (int i = threadIdx.x; i < R * R; i += blockDim.x) {
    double v = 1.0;
    for (int m = 0; m < nmat; ++m) v *= gl.G[m][i];
    A[(i / R) * RS + i % R] = v;
  }
  __syncthreads();
}

// G^+ entry v at flat index i = a R + b -> full, packed (a <= b) and the
// G_{>k} products.
__device__ __forceinline__ void store_gplus(const GList& gl, int R, int nsteps, int i, double v,
                                            double* __restrict__ gplus_full,
                                            double* __restrict__ gplus_packed,
                                            double* __restrict__ ggt) {
  const int a = i / R, b = i % R;
  gplus_full[i] = v;
  if (gplus_packed != nullptr && a <= b) gplus_packed[packed_index(a, b, R)] = v;
  for (int st = 0; st < nsteps; ++st) {
    double w = v;
    for (int s2 = st + 1; s2 < nsteps; ++s2) w *= gl.G[s2][i];
    ggt[(int64_t)gl.order[st] * R * R + i] = w;
  }
}

// G = (*) of the listed Grams -> G^+ (full and packed), rank, and G_{>k}
// for the drawn modes order[0..nsteps-1] (nsteps may be 0).  One block.
//
// G^+ is the eigendecomposition pseudo-inverse (eigenvalues at most
// R eps lambda_max dropped).  When G is far from that threshold it equals
// G^{-1}, which the Cholesky factorisation gives in a few hundred light
// steps instead of the Jacobi sweeps: it is used when every pivot is
// positive and ||G||_inf ||G^{-1}||_inf R eps < 1e-4, which implies
// lambda_min >= 1 / ||G^{-1}||_inf > 1e4 R eps ||G||_inf >= 1e4 R eps
// lambda_max, so that the eigen route would keep all R eigenvalues (rank R,
// Jacobi sweep count reported as 0).  Otherwise the Jacobi route runs.
__device__ void prep_gplus_body(const GList& gl, int nmat, int R, int nsteps,
                                double* __restrict__ gplus_full, double* __restrict__ gplus_packed,
                                int32_t* __restrict__ rank, double* __restrict__ ggt,
                                int32_t* __restrict__ status, double* smem) {
  double* A = smem;                 // R*RS
  double* lam = A + R * (R + 1);    // R
  double* red = lam + R;            // 2
  int* flag = (int*)(red + 2);
  double* wmax = red + 8;           // PREP_THREADS / 64 (the space past the eigen route's perm)
  const int RS = R + 1;
  const int tid = threadIdx.x;
  if (gplus_packed != nullptr)
    for (int i = tid; i < NODE_SLACK; i += blockDim.x)
      gplus_packed[(int64_t)R * (R + 1) / 2 + i] = 0.0;
  load_hadamard(gl, nmat, R, A);
  // ---- Cholesky route
  for (int a = tid; a < R; a += blockDim.x) {
    double rs = 0;
    for (int b = 0; b < R; ++b) rs += fabs(A[b * RS + a]);
    lam[a] = rs;
  }
  __syncthreads();
  if (tid == 0) {
    double g = 0;
    for (int a = 0; a < R; ++a) g = fmax(g, lam[a]);
    red[0] = g;                     // ||G||_inf
  }
  __syncthreads();
  if (tid < 64) {
    const bool okw = cholesky_inverse_lower_wave(A, R, lam);
    if (tid == 0) *flag = okw ? 1 : 0;
  }
  __syncthreads();
  bool ok = *flag == 1;
  if (ok) {
    // G^{-1} = X^T X (X = L^{-1} in the lower triangle): every entry a <= b
    // formed once, by all threads, into registers, then stored in the upper
    // triangle of A (column b, row a < b; G's copy there is no longer
    // needed) with the diagonal in lam; ||G^{-1}||_inf from its rows, one
    // wavefront per row
    constexpr int MAXE = (128 * 129 / 2 + PREP_THREADS - 1) / PREP_THREADS;
    const int ne = R * (R + 1) / 2;
    double v[MAXE];
#pragma unroll
    for (int q = 0; q < MAXE; ++q) {
      const int p = tid + q * (int)blockDim.x;
      v[q] = 0.0;
      if (p < ne) {
        int a, b;
        unpack_index(p, R, a, b);
        v[q] = inverse_entry(A, R, a, b);
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < MAXE; ++q) {
      const int p = tid + q * (int)blockDim.x;
      if (p < ne) {
        int a, b;
        unpack_index(p, R, a, b);
        if (a == b)
          lam[a] = v[q];
        else
          A[b * RS + a] = v[q];
      }
    }
    __syncthreads();
    const int lane = tid & 63, wave = tid >> 6, nwave = (int)blockDim.x >> 6;
    double hmax = 0.0;
    for (int a = wave; a < R; a += nwave) {
      double rs = 0.0;
      for (int b = lane; b < R; b += 64) rs += fabs(stored_inverse(A, lam, RS, a, b));
      hmax = fmax(hmax, wave_sum(rs));
    }
    if (lane == 0) wmax[wave] = hmax;
    __syncthreads();
    if (tid == 0) {
      double h = 0;
      for (int w = 0; w < nwave; ++w) h = fmax(h, wmax[w]);
      const double cert = red[0] * h * (double)R * DBL_EPSILON;
      *flag = (cert < 1e-4) ? 1 : 0;
    }
    __syncthreads();
    ok = *flag == 1;
    if (ok) {
      if (tid == 0) {
        rank[0] = R;
        rank[1] = 0;
      }
      for (int i = tid; i < R * R; i += blockDim.x)
        store_gplus(gl, R, nsteps, i, stored_inverse(A, lam, RS, i / R, i % R), gplus_full,
                    gplus_packed, ggt);
      return;
    }
  }
  // ---- eigen route (one-sided Jacobi)
  __syncthreads();
  load_hadamard(gl, nmat, R, A);
  const int sweeps = jacobi_columns(A, R, flag);
  if (tid == 0) rank[1] = sweeps;
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
  for (int c = tid; c < R; c += blockDim.x) lam[c] = lam[c] > tau ? 1.0 / lam[c] : 0.0;
  __syncthreads();
  for (int i = tid; i < R * R; i += blockDim.x) {
    const int a = i / R, b = i % R;
    double v = 0;
    for (int c = 0; c < R; ++c) v += A[c * RS + a] * A[c * RS + b] * lam[c];
    store_gplus(gl, R, nsteps, i, v, gplus_full, gplus_packed, ggt);
  }
}

__global__ __launch_bounds__(PREP_THREADS) void prep_gplus_kernel(
    GList gl, int nmat, int R, int nsteps,
    double* __restrict__ gplus_full, double* __restrict__ gplus_packed, int32_t* __restrict__ rank,
    double* __restrict__ ggt, int32_t* __restrict__ status) {
  extern __shared__ double smem[];
  prep_gplus_body(gl, nmat, R, nsteps, gplus_full, gplus_packed, rank, ggt, status, smem);
}

// One block per job of a batch.
__global__ __launch_bounds__(PREP_THREADS) void prep_gplus_batched_kernel(
    const PrepJob* __restrict__ jobs) {
  extern __shared__ double smem[];
  const PrepJob& j = jobs[blockIdx.x];
  prep_gplus_body(j.gl, j.nmat, j.R, j.nsteps, j.gplus_full, j.gplus_packed, j.rank, j.ggt,
                  j.status, smem);
}

// Drawn mode `st` of gk: eigendecomposition of G_{>k} (ascending), the
// eigenvectors in the factor type and the eigen-tree E_k.  One block.
template <typename T>
__device__ void prep_eig_body(const GList& gk, int st, int R, const double* __restrict__ ggt,
                              double* __restrict__ lam_out, T* __restrict__ vecs,
                              T* __restrict__ etree, int64_t estride,
                              int32_t* __restrict__ sweep_out, double* __restrict__ emass,
                              int64_t enodes, double* smem, double* __restrict__ warm = nullptr,
                              int32_t* __restrict__ warm_ok = nullptr) {
  const int RS = R + 1;
  double* A = smem;
  double* lam = A + R * RS;
  int* perm = (int*)(lam + R);
  int* flag = perm + R;
  const int k = gk.order[st];
  const double* __restrict__ Gk = gk.G[st];
  const int tid = threadIdx.x;
  for (int i = tid; i < R * R; i += blockDim.x) A[(i / R) * RS + i % R] = ggt[(int64_t)k * R * R + i];
  __syncthreads();
  // Warm start (a caller's earlier eigenvectors V of this mode, rows
  // v_c^T): one-sided Jacobi on A V instead of A.  Its converged columns
  // A V Q are orthogonal with V Q orthogonal, so they are lambda_c v'_c
  // for the eigenpairs of A as from a cold start (any orthogonal start
  // works); near the last solve's eigenvectors few sweeps remain.
  double* Vw = warm != nullptr ? warm + (int64_t)k * R * R : nullptr;
  const bool use_warm = Vw != nullptr && warm_ok[k] != 0;
  if (use_warm) {
    constexpr int MAXO = 128 * 128 / PREP_THREADS;  // outputs per thread
    double out[MAXO];
#pragma unroll
    for (int o = 0; o < MAXO; ++o) {
      const int i = tid + o * (int)blockDim.x;
      double acc = 0.0;
      if (i < R * R) {
        const int c = i / R, r = i % R;  // (A V)[r][c] = sum_m A[r][m] V[m][c]
        for (int m = 0; m < R; ++m) acc += A[m * RS + r] * Vw[(int64_t)c * R + m];
      }
      out[o] = acc;
    }
    __syncthreads();
#pragma unroll
    for (int o = 0; o < MAXO; ++o) {
      const int i = tid + o * (int)blockDim.x;
      if (i < R * R) A[(i / R) * RS + i % R] = out[o];
    }
    __syncthreads();
  }
  const int sweeps = jacobi_columns(A, R, flag);
  if (tid == 0 && sweep_out != nullptr) sweep_out[2 + st] = sweeps;
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
    vecs[(int64_t)k * R * R + i] = (T)A[perm[u] * RS + e];
    if (Vw != nullptr) Vw[i] = A[perm[u] * RS + e];
    if (e == 0) lam_out[(int64_t)k * R + u] = lam[perm[u]];
  }
  if (Vw != nullptr && tid == 0) warm_ok[k] = 1;
  // eigen-tree over the R rows sqrt(lam_u) v_u^T with Y = G_k: node masses
  // <h h^T, P^v, G_k> with P^v = sum_{u in S(v)} lam_u v_u v_u^T; the
  // stored node is P^v (*) G_k (packed upper triangle).
  const int64_t TR = (int64_t)R * (R + 1) / 2;
  const int DE = R > 1 ? 32 - __builtin_clz((unsigned)(R - 1)) : 0;
  const int64_t Lp = int64_t(1) << DE;
  T* __restrict__ E = etree + (int64_t)k * estride;
  for (int64_t i = tid; i < NODE_SLACK; i += blockDim.x) E[estride - NODE_SLACK + i] = T(0);
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
        v = lam[c] * A[c * RS + a] * A[c * RS + b] * g;
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
  // The first drawn mode walks E_k with h = 1, where every stored node's
  // mass <w, E^v> (w = 1 on the diagonal, 2 off it) is the same for all
  // samples: one wavefront per node sums it from the stored values.
  if (st == 0 && emass != nullptr) {
    __syncthreads();
    const int lane = tid & 63;
    const int nw = blockDim.x >> 6;
    for (int64_t v = tid >> 6; v < enodes; v += nw) {
      double acc = 0.0;
      // twice every packed entry, less the diagonal once
      for (int64_t p = lane; p < TR; p += 64) acc += 2.0 * (double)E[v * TR + p];
      for (int a = lane; a < R; a += 64) acc -= (double)E[v * TR + packed_index(a, a, R)];
      acc = wave_sum(acc);
      if (lane == 0) emass[(int64_t)k * enodes + v] = acc;
    }
  }
}

template <typename T>
__global__ __launch_bounds__(PREP_THREADS) void prep_eig_kernel(
    GList gk, int R, const double* __restrict__ ggt,
    double* __restrict__ lam_out, T* __restrict__ vecs, T* __restrict__ etree, int64_t estride,
    int32_t* __restrict__ sweep_out, double* __restrict__ emass, int64_t enodes,
    double* __restrict__ warm, int32_t* __restrict__ warm_ok) {
  extern __shared__ double smem[];
  prep_eig_body<T>(gk, blockIdx.x, R, ggt, lam_out, vecs, etree, estride, sweep_out, emass,
                   enodes, smem, warm, warm_ok);
}

template <typename T>
__global__ __launch_bounds__(PREP_THREADS) void prep_eig_batched_kernel(
    const EigJob* __restrict__ jobs) {
  extern __shared__ double smem[];
  const EigJob& j = jobs[blockIdx.x];
  prep_eig_body<T>(j.gl, j.st, j.R, j.ggt, j.lam, (T*)j.vecs, (T*)j.etree, j.estride,
                   j.sweep_out, j.emass, j.enodes, smem);
}

hipError_t set_lds(const void* fn, size_t bytes) {
  return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

}  // namespace

size_t prep_lds_bytes(int R) {
  // A, lam, then 64 bytes (red, flag), the eigen route's perm and flag or
  // the Cholesky route's per-wave maxima, and slack
  return (size_t)R * (R + 1) * 8 + (size_t)R * 8 + 64 + (size_t)R * 4 + 64 +
         (size_t)PREP_THREADS / 64 * 8;
}

hipError_t launch_prep_gplus2(hipStream_t st, int R, int nmat, const double* const* mats,
                              int nsteps, const int* order, double* gplus_full,
                              double* gplus_packed, int32_t* rank, double* ggt, int32_t* status) {
  GList gl{};
  for (int m = 0; m < nmat; ++m) gl.G[m] = mats[m];
  for (int m = 0; m < nsteps; ++m) gl.order[m] = order[m];
  const size_t lds = prep_lds_bytes(R);
  hipError_t e = set_lds((const void*)prep_gplus_kernel, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(prep_gplus_kernel, dim3(1), dim3(prep_threads(R)), lds, st, gl, nmat, R, nsteps,
                     gplus_full, gplus_packed, rank, ggt, status);
  return hipGetLastError();
}

hipError_t launch_prep_eig2(hipStream_t st, krps_precision p, int R, int nsteps,
                            const double* const* Gsteps, const int* order, const double* ggt,
                            double* lam, void* vecs, void* etree, int64_t estride,
                            int32_t* sweep_out, double* emass, int64_t enodes, double* warm,
                            int32_t* warm_ok) {
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
    hipLaunchKernelGGL(prep_eig_kernel<double>, dim3(nsteps), dim3(prep_threads(R)), lds, st, gl,
                       R, ggt, lam, (double*)vecs, (double*)etree, estride, sweep_out,
                       emass, enodes, warm, warm_ok);
  } else {
    e = set_lds((const void*)prep_eig_kernel<float>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(prep_eig_kernel<float>, dim3(nsteps), dim3(prep_threads(R)), lds, st, gl,
                       R, ggt, lam, (float*)vecs, (float*)etree, estride, sweep_out,
                       emass, enodes, warm, warm_ok);
  }
  return hipGetLastError();
}

int prep_block_threads(int R) { return prep_threads(R); }

hipError_t launch_prep_batched(hipStream_t st, const PrepJob* jobs, int njobs, int Rmax) {
  if (njobs <= 0) return hipSuccess;
  const size_t lds = prep_lds_bytes(Rmax);
  hipError_t e = set_lds((const void*)prep_gplus_batched_kernel, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(prep_gplus_batched_kernel, dim3((unsigned)njobs), dim3(prep_threads(Rmax)),
                     lds, st, jobs);
  return hipGetLastError();
}

hipError_t launch_eig_batched(hipStream_t st, bool f64, const EigJob* jobs, int njobs, int Rmax) {
  if (njobs <= 0) return hipSuccess;
  const size_t lds = prep_lds_bytes(Rmax);
  hipError_t e;
  if (f64) {
    e = set_lds((const void*)prep_eig_batched_kernel<double>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(prep_eig_batched_kernel<double>, dim3((unsigned)njobs),
                       dim3(prep_threads(Rmax)), lds, st, jobs);
  } else {
    e = set_lds((const void*)prep_eig_batched_kernel<float>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(prep_eig_batched_kernel<float>, dim3((unsigned)njobs),
                       dim3(prep_threads(Rmax)), lds, st, jobs);
  }
  return hipGetLastError();
}

// ---------------------------------------------- first-mode factor-tree masses
//
// For the first drawn mode the history is h = 1, so stage 2 weights every
// node of Z_k with h~ = V[:, u]: its mass V[:, u]^T G^v V[:, u] depends only
// on the component u drawn in stage 1.  The table tab[u][n] of every stored
// node n and every u is a contraction of the packed weights
// P[u][p] = w_p V[a_p][u] V[b_p][u] (w = 2 off the diagonal) with the stored
// packed nodes: tab = P Z^T over the tri(R) packed entries, float64 over the
// stored values.  A block computes RMAX u's x NB nodes, K in chunks of KC
// packed entries staged through LDS; a thread holds 4 u's x NB/32 nodes.

// P[p][u] = w_p V[a_p][u] V[b_p][u] (columns u >= R are 0), RMAX columns.
template <typename T, int RMAX>
__device__ __forceinline__ void zweights_body(const T* __restrict__ V, int R,
                                              double* __restrict__ P, int64_t i0,
                                              int64_t stride) {
  const int TR = R * (R + 1) / 2;
  for (int64_t i = i0; i < (int64_t)TR * RMAX; i += stride) {
    const int p = (int)(i / RMAX), u = (int)(i % RMAX);
    double v = 0.0;
    if (u < R) {
      int a, b;
      unpack_index(p, R, a, b);
      v = (a == b ? 1.0 : 2.0) * (double)V[(int64_t)u * R + a] * (double)V[(int64_t)u * R + b];
    }
    P[i] = v;
  }
}

template <typename T, int RMAX>
__global__ __launch_bounds__(256) void zweights_kernel(const T* __restrict__ V, int R,
                                                       double* __restrict__ P) {
  zweights_body<T, RMAX>(V, R, P, (int64_t)blockIdx.x * blockDim.x + threadIdx.x,
                         (int64_t)gridDim.x * blockDim.x);
}

// One job per blockIdx.y.
template <typename T, int RMAX>
__global__ __launch_bounds__(256) void zweights_batched_kernel(const ZtabJob* __restrict__ jobs) {
  const ZtabJob& j = jobs[blockIdx.y];
  zweights_body<T, RMAX>((const T*)j.V, j.R, j.weights,
                         (int64_t)blockIdx.x * blockDim.x + threadIdx.x,
                         (int64_t)gridDim.x * blockDim.x);
  if (j.tab2 != nullptr)
    zweights_body<T, RMAX>((const T*)j.V2, j.R, j.weights2,
                           (int64_t)blockIdx.x * blockDim.x + threadIdx.x,
                           (int64_t)gridDim.x * blockDim.x);
}

// The contraction on the float64 matrix cores: a wavefront owns 16 nodes
// and every u (RMAX / 16 accumulator tiles of v_mfma_f64_16x16x4f64); per
// step of 4 packed entries lane l supplies A = P[p0 + l/16][16 t + l%16]
// and B = G^(n0 + l%16)[p0 + l/16], and holds the result rows 4 i + l/16 of
// column l%16.  Loads of KS steps are issued before their products.
// NS weight sets P[0..NS) contracted with the same nodes (the tables of
// two problems whose first drawn mode has the same tree share its reads).
template <typename T, int RMAX, int NS>
__device__ __forceinline__ void ztab_unit(const T* __restrict__ Z, int64_t nn, int R,
                                          const double* const* P, double* const* tab,
                                          int64_t n0, int lane) {
  constexpr int NTU = RMAX / 16;  // u tiles
  constexpr int KS = NS == 1 ? 8 : 4;  // steps of 4 entries whose loads go together
  const int TR = R * (R + 1) / 2;
  const int r16 = lane & 15, k4 = lane >> 4;
  {
    f64x4 acc[NS][NTU];
#pragma unroll
    for (int w = 0; w < NS; ++w)
#pragma unroll
      for (int t = 0; t < NTU; ++t) acc[w][t] = f64x4{0, 0, 0, 0};
    const int64_t n = n0 + r16;
    const T* __restrict__ zrow = Z + (n < nn ? n : nn - 1) * (int64_t)TR;
    for (int p0 = 0; p0 < TR; p0 += 4 * KS) {
      double bv[KS], av[NS][KS][NTU];
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        const int p = p0 + 4 * ks + k4;
        const int pc = p < TR ? p : TR - 1;
        bv[ks] = (double)zrow[pc];
#pragma unroll
        for (int w = 0; w < NS; ++w)
#pragma unroll
          for (int t = 0; t < NTU; ++t) av[w][ks][t] = P[w][(int64_t)pc * RMAX + 16 * t + r16];
      }
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        const bool ok = p0 + 4 * ks + k4 < TR && n < nn;
        const double b = ok ? bv[ks] : 0.0;
#pragma unroll
        for (int w = 0; w < NS; ++w)
#pragma unroll
          for (int t = 0; t < NTU; ++t)
            acc[w][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[w][ks][t], b, acc[w][t], 0, 0, 0);
      }
    }
#pragma unroll
    for (int w = 0; w < NS; ++w)
#pragma unroll
      for (int t = 0; t < NTU; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int u = 16 * t + 4 * i + k4;
          if (u < R && n < nn) tab[w][(int64_t)u * nn + n] = acc[w][t][i];
        }
  }
}

template <typename T, int RMAX>
__global__ __launch_bounds__(256) void ztab_kernel(const T* __restrict__ Z, int64_t nn, int R,
                                                   const double* __restrict__ P,
                                                   double* __restrict__ tab) {
  const int64_t nwave = (int64_t)gridDim.x * (blockDim.x >> 6);
  for (int64_t n0 = ((int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) * 16; n0 < nn;
       n0 += nwave * 16) {
    const double* Ps[1] = {P};
    double* tabs[1] = {tab};
    ztab_unit<T, RMAX, 1>(Z, nn, R, Ps, tabs, n0, threadIdx.x & 63);
  }
}

// Several problems' tables in one launch: wavefront w takes units w,
// w + waves, ... of the batch (a unit is 16 nodes of one job; the job is
// found by a wave-uniform binary search over the jobs' first units).
template <typename T, int RMAX>
__global__ __launch_bounds__(256) void ztab_batched_kernel(const ZtabJob* __restrict__ jobs,
                                                           int njobs, int64_t units) {
  const int64_t nwave = (int64_t)gridDim.x * (blockDim.x >> 6);
  for (int64_t un = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); un < units;
       un += nwave) {
    int lo = 0, hi = njobs;  // last job with unit0 <= un
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (jobs[mid].unit0 <= un) lo = mid; else hi = mid;
    }
    const ZtabJob& j = jobs[lo];
    if constexpr (RMAX <= 32) {
      if (j.tab2 != nullptr) {
        const double* Ps[2] = {j.weights, j.weights2};
        double* tabs[2] = {j.tab, j.tab2};
        ztab_unit<T, RMAX, 2>((const T*)j.Z, j.nn, j.R, Ps, tabs, (un - j.unit0) * 16,
                              threadIdx.x & 63);
        continue;
      }
    }
    const double* Ps[1] = {j.weights};
    double* tabs[1] = {j.tab};
    ztab_unit<T, RMAX, 1>((const T*)j.Z, j.nn, j.R, Ps, tabs, (un - j.unit0) * 16,
                          threadIdx.x & 63);
  }
}

template <typename T, int RMAX>
void run_ztab_r(hipStream_t st, const T* Z, int64_t nn, int R, const T* V, double* P,
                double* tab) {
  const int TR = R * (R + 1) / 2;
  int64_t wb = ((int64_t)TR * RMAX + 255) / 256;
  if (wb > 2048) wb = 2048;
  hipLaunchKernelGGL((zweights_kernel<T, RMAX>), dim3((unsigned)wb), dim3(256), 0, st, V, R, P);
  // four wavefronts of 16 nodes per block
  int64_t blocks = (nn + 63) / 64;
  if (blocks > 8192) blocks = 8192;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL((ztab_kernel<T, RMAX>), dim3((unsigned)blocks), dim3(256), 0, st, Z, nn, R, P,
                     tab);
}

template <typename T>
hipError_t run_ztab(hipStream_t st, const T* Z, int64_t nn, int R, const T* V, double* P,
                    double* tab) {
  if (R <= 32)
    run_ztab_r<T, 32>(st, Z, nn, R, V, P, tab);
  else if (R <= 64)
    run_ztab_r<T, 64>(st, Z, nn, R, V, P, tab);
  else
    run_ztab_r<T, 128>(st, Z, nn, R, V, P, tab);
  return hipGetLastError();
}

size_t ztab_weights_bytes(int R) {
  const int rmax = R <= 32 ? 32 : R <= 64 ? 64 : 128;
  return (size_t)R * (R + 1) / 2 * rmax * 8;
}

hipError_t launch_ztab(hipStream_t st, krps_precision p, const void* Z, int64_t nn, int R,
                       const void* V, double* weights, double* tab) {
  if (p == KRPS_FP64)
    return run_ztab<double>(st, (const double*)Z, nn, R, (const double*)V, weights, tab);
  return run_ztab<float>(st, (const float*)Z, nn, R, (const float*)V, weights, tab);
}

int ztab_rclass(int R) { return R <= 32 ? 0 : R <= 64 ? 1 : 2; }

namespace {

template <typename T, int RMAX>
void run_ztab_batched(hipStream_t st, const ZtabJob* jobs, int njobs, int64_t units) {
  // weights: the largest job's tri(R) x RMAX entries per row of blocks
  const int TR = RMAX * (RMAX + 1) / 2;
  int64_t wb = ((int64_t)TR * RMAX + 255) / 256;
  if (wb > 256) wb = 256;
  hipLaunchKernelGGL((zweights_batched_kernel<T, RMAX>), dim3((unsigned)wb, (unsigned)njobs),
                     dim3(256), 0, st, jobs);
  int64_t blocks = (units + 3) / 4;
  if (blocks > 8192) blocks = 8192;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL((ztab_batched_kernel<T, RMAX>), dim3((unsigned)blocks), dim3(256), 0, st,
                     jobs, njobs, units);
}

template <typename T>
void run_ztab_batched_t(hipStream_t st, int rclass, const ZtabJob* jobs, int njobs,
                        int64_t units) {
  if (rclass == 0)
    run_ztab_batched<T, 32>(st, jobs, njobs, units);
  else if (rclass == 1)
    run_ztab_batched<T, 64>(st, jobs, njobs, units);
  else
    run_ztab_batched<T, 128>(st, jobs, njobs, units);
}

}  // namespace

hipError_t launch_ztab_batched(hipStream_t st, bool f64, int rclass, const ZtabJob* jobs,
                               int njobs, int64_t units) {
  if (njobs <= 0 || units <= 0) return hipSuccess;
  if (njobs > 65535) return hipErrorInvalidValue;
  if (f64)
    run_ztab_batched_t<double>(st, rclass, jobs, njobs, units);
  else
    run_ztab_batched_t<float>(st, rclass, jobs, njobs, units);
  return hipGetLastError();
}

hipError_t launch_pinv(hipStream_t st, int R, const double* M, double* Mp_full, int32_t* rank,
                       int32_t* status) {
  const double* mats[1] = {M};
  return launch_prep_gplus2(st, R, 1, mats, 0, nullptr, Mp_full, nullptr, rank, nullptr, status);
}

}  // namespace krps
