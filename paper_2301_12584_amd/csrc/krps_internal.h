// Internal declarations shared by the libkrps translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/krps.h"

namespace krps {

// ---------------------------------------------------------------- errors
void set_error(const std::string& msg);
krps_status fail(krps_status st, const std::string& msg);
krps_status hip_fail(hipError_t e, const char* what);

#define KRPS_HIP(call)                                   \
  do {                                                   \
    hipError_t e_ = (call);                              \
    if (e_ != hipSuccess) return ::krps::hip_fail(e_, #call); \
  } while (0)

// ---------------------------------------------------------------- layout
inline int64_t tri(int R) { return (int64_t)R * (R + 1) / 2; }
inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline int ceil_log2(int64_t x) {
  int d = 0;
  while ((int64_t(1) << d) < x) ++d;
  return d;
}
inline size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }

// Segment tree T_{I,F}: L leaves padded to 2^D; nodes stored: the root,
// then for each level l = 1..D the left children of the real nodes.
// real(l) = ceil(L / 2^(D-l)); stored left children at level l:
// ceil(L / 2^(D-l+1)).
struct TreeShape {
  int64_t I = 0, L = 0;
  int F = 0, D = 0;
  int64_t n_nodes = 0;
  void init(int64_t I_, int F_) {
    I = I_;
    F = F_;
    L = ceil_div(I, F);
    D = L > 1 ? ceil_log2(L) : 0;
    n_nodes = 1;
    for (int l = 1; l <= D; ++l) n_nodes += ((L - 1) >> (D - l + 1)) + 1;
  }
};

// Per-mode descriptor read by the descent kernel.
struct ModeDesc {
  const void* U;      // factor, row-major I x R
  const void* Z;      // factor tree nodes
  const void* E;      // eigen tree nodes (per draw)
  const void* V;      // eigenvectors, [u][R] (per draw)
  const double* em;   // masses of E's stored nodes at h = 1 (per draw; written
                      // for the first drawn mode only) or null
  const double* zt;   // [R][zn] masses of Z's stored nodes for h~ = V[:, u]
                      // (per draw; first drawn mode only) or null
  int64_t zn;         // stored nodes of Z (the table's row length)
  const float* z32;   // float32 copy of a float64 Z (same layout), or null
  int32_t ztop;       // with z32: levels 1..ztop are decided from Z itself
  int64_t I, L;
  int32_t F, D;
  int32_t DE, ne;     // eigen-tree depth and stored nodes
};

struct DescentArgs {
  ModeDesc mode[KRPS_MAX_MODES];
  int N, R, exclude, nsteps;      // nsteps: number of drawn modes
  int order[KRPS_MAX_MODES];      // drawn modes in increasing order
  int64_t J;
  const double* u01;              // [J][N][2], or null: generated from seed / ctr_base
  uint64_t seed, ctr_base;        // in-kernel uniforms (Philox4x64-10)
  uint64_t ctr2;                  // third counter word of the in-kernel uniforms
  const uint64_t* ctr2_dev;       // device word added to ctr2, or null
  int32_t* idx;                   // [J][N]
  double* prob;                   // [J] or null
  void* rows;                     // [J][R] or null (factor type)
  double* rows64;                 // [J][R] float64 rows or null
  const double* gplus;            // packed upper G^+ (tri) float64
  const int32_t* rank;            // device rank of G
  double* wout;                   // [J] sampling weights 1/sqrt(J q) or null
  int scale_rows;                 // rows <- a_d / sqrt(J q_d)
  int lps;                        // lanes per sample of the walk (0 = default)
  int32_t* status;                // device status word
};

// Zero elements that follow every array of stored tree nodes (factor
// trees, eigen-trees, packed G^+): the walk reads each node in strides of
// its lane group without clamping, so it may read up to 63 elements past
// the node's end; they are finite and carry weight 0.
constexpr int64_t NODE_SLACK = 64;

// Grams multiplied into a preparation, and the drawn modes in order.
struct GList {
  const double* G[KRPS_MAX_MODES];
  int order[KRPS_MAX_MODES];
};

// One G^+ preparation of a batch (one block each).
struct PrepJob {
  GList gl;
  int nmat, R, nsteps, pad;
  double* gplus_full;
  double* gplus_packed;
  int32_t* rank;
  double* ggt;
  int32_t* status;
};

// One eigen-tree preparation (drawn mode st of a problem) of a batch.
struct EigJob {
  GList gl;
  int st, R;
  const double* ggt;
  double* lam;
  void* vecs;
  void* etree;
  int64_t estride;  // elements from one mode's eigen-tree to the next
  int32_t* sweep_out;
  double* emass;    // [N][enodes]: the first drawn mode's E masses at h = 1
  int64_t enodes;
};

// One problem of a batched draw: its walk arguments, its packed-index
// table (device, tri(R) uint16; unused for R > 64), its shape class and
// samples per task, and its first task in the batch's task numbering.
struct BatchProblem {
  DescentArgs a;
  const uint16_t* tab;
  int cls, G;
  int64_t task0;
};

// Fiber lookup / SpMM arguments for one solve of mode j.
struct FiberArgs {
  int N, j, lead, R;
  int64_t nnz, J;             // stored (merged) entries; samples
  const int32_t* cols;        // [N][nnz] columns of mode j's sorted entries
  const double* vals;         // [nnz] merged values
  const int64_t* off;         // [dims[lead] + 1] offsets over the leading other mode
  const int32_t* sample_idx;  // [J][N]
  const double* w;            // [J] 1/sqrt(J q_d)
  int64_t* lo;                // [J] fiber entry range
  int64_t* hi;                // [J]
  int64_t* cnt;               // [J] work items per sample (0 unless first of its fiber)
  int64_t* start;             // [J + 1] exclusive prefix of cnt
  double* coef;               // [J] (sum of w^2 over the fiber's samples) / w_d
  int32_t* slot;              // [J] hash slot of the sample's fiber (-1: empty fiber)
  unsigned long long* hkey;   // [H] fiber keys (first entry), all-ones = empty
  double* hW;                 // [H] summed w^2
  int32_t* hrep;              // [H] smallest sample index of the fiber
  int64_t H;                  // power of two >= 2 J
  int hbits;                  // log2 H
  int64_t* rflag;             // [J] 1 if the sample expands its fiber
  int64_t* rpos;              // [J + 1] exclusive prefix of rflag (rpos[J] = count)
  int32_t* rep;               // [J] expanding samples in sample order
  int64_t* rstart;            // [J + 1] first work item of each of them, then the total
  int64_t* bsum;              // [ceil(J / 1024) + 1] scan tile totals
  const int16_t* hot_slot;    // [dims[j]] slot of a hot row of mode j, -1 otherwise
  const int32_t* hot_rows;    // [nhot] the hot rows
  int nhot;
  int64_t* expanded;          // out: entries the SpMM expands, or null
  // deterministic mode (else null): hW holds the int64 high words of the
  // fixed-point sums of w^2, hWlo the low words; wscale = {2^S, 2^-S}
  long long* hWlo;            // [H]
  double* wscale;             // [2]
};

// Rows of a mode with the most stored entries (kept per workgroup in LDS by
// the SpMM).
constexpr int HOT_ROWS = KRPS_HOT_ROWS;
// LDS a workgroup of the SpMM-like kernels gives to hot-row accumulators
// (8 bytes per entry): the hot rows it accumulates are the first
// hot_rows_used() of the mode's list (slots in decreasing entry count).
constexpr size_t HOT_LDS_BYTES = size_t(128) << 10;
inline int hot_rows_used(int nhot, int R) {
  const int cap = (int)(HOT_LDS_BYTES / ((size_t)R * 8));
  return nhot < cap ? nhot : cap;
}

// Exact MTTKRP of mode j over a tensor's stored entries (mode j's copy).
struct MttkrpArgs {
  int N, j, R;
  int64_t nnz;
  const int32_t* cols;        // [N][nnz] mode j's sorted, merged entries
  const double* vals;         // [nnz]
  const void* U[KRPS_MAX_MODES];
  const int16_t* hot_slot;    // [dims[j]] slot of a hot row of mode j, -1 otherwise
  const int32_t* hot_rows;    // [nhot]
  int nhot;
};

struct FitArgs {
  int N, R;
  int64_t nnz;
  const int32_t* cols;  // [N][nnz] stored entries (any mode's order)
  const double* vals;
  const void* U[KRPS_MAX_MODES];
  const double* G[KRPS_MAX_MODES];
  const double* sigma;
};

// Status words of a sampler (int32 [3], cleared at creation): word 0 holds
// flag bits set by kernels, word 1 counts sampled rows whose computed
// probability, or a total mass of whose walk, was not positive (rounding;
// they were given weight 0), word 2
// counts walks whose float32-copy decisions were not certain and that were
// walked again from the float64 tree.
enum : int32_t { ST_ZERO = 1, ST_NUMERIC = 2 };

// ------------------------------------------------------------- launchers
// tree_build.hip
size_t tree_build_scratch_bytes(int64_t L, int R);
// Largest extent of the scratch that a build of this shape touches.
size_t tree_build_scratch_extent(const TreeShape& ts, int R);
// p: KRPS_FP64 (float64 U), KRPS_FP32 (float32 U, float64 products and
// sums, float32 nodes), KRPS_BF16X2 (float32 U, three-part bf16 split
// products summed in float32; used for the Gram of a solve's sampled rows).
hipError_t launch_tree_build(hipStream_t st, krps_precision p, const void* U, int64_t I, int R,
                             const TreeShape& ts, void* nodes, double* gram_full,
                             double* scratch, size_t scratch_bytes, float* nodes32 = nullptr,
                             int team = 0);
// Waves per team of the sampler trees' leaf pass available for R (the
// default first; 0 also selects the default).
std::vector<int> build_team_choices(int R, krps_precision p);

// Up to UPDATE_CHUNK single-entry updates (row, column, new value), passed
// by value to one launch.
constexpr int UPDATE_CHUNK = 32;
struct UpdateList {
  int64_t row[UPDATE_CHUNK];
  int32_t col[UPDATE_CHUNK];
  double val[UPDATE_CHUNK];
  int n;
};
// Algorithm 5 for the entries of ul, in order (the factor, its stored
// nodes, the float32 copy if any, and G_j).
hipError_t launch_update_entries(hipStream_t st, krps_precision p, const UpdateList& ul, void* U,
                                 void* nodes, float* nodes32, double* gram, int64_t I, int R,
                                 const TreeShape& ts);

// eig.hip
size_t prep_lds_bytes(int R);
// G = (*) mats[0..nmat-1] -> G^+ (full, and packed if non-null), rank;
// for nsteps > 0 also G_{>k} for the drawn modes order[0..nsteps-1] (host array)
// (mats must then be those modes' Grams in the same order).
hipError_t launch_prep_gplus2(hipStream_t st, int R, int nmat, const double* const* mats,
                              int nsteps, const int* order, double* gplus_full,
                              double* gplus_packed, int32_t* rank, double* ggt, int32_t* status);
hipError_t launch_prep_eig2(hipStream_t st, krps_precision p, int R, int nsteps,
                            const double* const* Gsteps, const int* order, const double* ggt,
                            double* lam, void* vecs, void* etree, int64_t estride,
                            int32_t* sweep_out, double* emass, int64_t enodes,
                            double* warm = nullptr, int32_t* warm_ok = nullptr);
// Table of the first drawn mode's factor-tree node masses for h~ = V[:, u]:
// tab[u * nn + n] = V[:,u]^T G^n V[:,u] for the nn stored nodes of Z (V as
// stored, [u][R]).  Float64 from the stored values.
// weights: scratch of ztab_weights_bytes(R) for the packed weights of every u.
size_t ztab_weights_bytes(int R);
hipError_t launch_ztab(hipStream_t st, krps_precision p, const void* Z, int64_t nn, int R,
                       const void* V, double* weights, double* tab);
// The same tables for several problems: one job per problem, all of one
// storage type and R class (R <= 32, <= 64, <= 128); unit0 = the job's
// first unit of 16 nodes in the batch's numbering, units = the total.  At
// R <= 32 a job may carry a second problem over the same tree (V2,
// weights2, tab2; else null), whose table is formed from the same reads.
struct ZtabJob {
  const void* Z;
  const void* V;
  double* weights;
  double* tab;
  const void* V2;
  double* weights2;
  double* tab2;
  int64_t nn, unit0;
  int R, pad;
};
int ztab_rclass(int R);
hipError_t launch_ztab_batched(hipStream_t st, bool f64, int rclass, const ZtabJob* jobs,
                               int njobs, int64_t units);
// rank points at two int32: the rank and the Jacobi sweep count.  A zero or
// non-finite M sets ST_ZERO / ST_NUMERIC in *status (if not null): the
// pseudo-inverse of such an M is returned as 0.
hipError_t launch_pinv(hipStream_t st, int R, const double* M, double* Mp_full, int32_t* rank,
                       int32_t* status = nullptr);

// lstsq.hip
size_t sort_temp_bytes(int64_t nnz);
// Sorted, merged copy of the tensor for mode j.  *nu < 0 on entry: the
// count of distinct coordinates is read back (one stream synchronisation)
// and stored in *nu; otherwise *nu is used as that count.
hipError_t build_fiber_index(hipStream_t st, int N, const int64_t* dims, int64_t nnz,
                             const int32_t* idx, const float* val, int j, int32_t* cols,
                             double* vals, int64_t* off, uint32_t* k0, uint32_t* k1, uint32_t* p0,
                             uint32_t* p1, void* temp, size_t temp_bytes, int64_t* nu);
hipError_t launch_norm2(hipStream_t st, const double* vals, int64_t n, double* out);
size_t norm2_bytes();  // out of launch_norm2: ||T||^2, then block partials
// U_j = mat(T, j) S (range finder), accumulated in float64 Y (I x R) and
// stored to U in the factor type.
hipError_t launch_range_finder(hipStream_t st, krps_precision p, const int32_t* cols,
                               const double* vals, int64_t nu, int N, int j, int R, uint64_t seed,
                               int64_t I, double* Y, void* U);
size_t hot_temp_bytes(int64_t dim);
hipError_t build_hot_rows(hipStream_t st, const int32_t* col, int64_t n, int64_t dim, int nhot,
                          uint32_t* c0, uint32_t* c1, uint32_t* i0, uint32_t* i1, void* temp,
                          size_t temp_bytes, int32_t* rows, int16_t* slot);
hipError_t launch_lookup(hipStream_t st, const FiberArgs& a);
// The SpMM in fixed point (int64 atomics, order-independent), then the
// listed rows of Y converted to float64 in place; p = KRPS_BF16X2 reads
// float32 rows, otherwise float64.  det: spmm_det_bytes() of scratch (its
// last two words are the fiber merge's scale, FiberArgs::wscale).
hipError_t launch_spmm_det(hipStream_t st, krps_precision p, const FiberArgs& a, const void* rows,
                           void* Y, const int32_t* list, const int64_t* count, double* det);
size_t spmm_det_bytes();
hipError_t launch_spmm(hipStream_t st, krps_precision p, const FiberArgs& a, const void* rows,
                       void* Y);
// Rows of Y that the sampled fibers reach: cleared marks over I rows, then
// mark, count per tile, scan, compacted increasing list, *count, and those
// rows of Y set to zero (the rest of Y is left as it was).
size_t row_bsum_bytes(int64_t I);
hipError_t launch_rows(hipStream_t st, const FiberArgs& a, int64_t I, int32_t* mark, int64_t* bsum,
                       int32_t* list, int64_t* count, void* Y, bool y32);
size_t solve_partial_bytes(int R);
// Generic sketched least squares (scaled rows, Z = (SA)^T S B, X = M^+ Z).
size_t lstsq_partial_bytes(int R, int64_t n);
hipError_t launch_ls_scale(hipStream_t st, krps_precision p, const void* rows, const void* sb,
                           const double* prob, int64_t J, int R, int64_t n, double* SA,
                           double* SBw);
hipError_t launch_ls_solve(hipStream_t st, const double* SA, const double* SBw, int64_t J, int R,
                           int64_t n, const double* Mp, double* partial, double* Z, double* X);
hipError_t launch_fill(hipStream_t st, krps_precision p, void* ptr, int64_t n);
hipError_t launch_fill_f64(hipStream_t st, double* ptr, int64_t n);
// *ptr = v (one thread)
hipError_t launch_set_u64(hipStream_t st, uint64_t* ptr, uint64_t v);
hipError_t launch_solve_gemm(hipStream_t st, krps_precision p, const void* Y, const double* Mp,
                             void* U, int64_t I, const int32_t* list, const int64_t* count, int R,
                             double* partial, double* sigma);
hipError_t launch_colnorm(hipStream_t st, krps_precision p, const void* U, int64_t I, int R,
                          double* partial, double* sigma);
hipError_t launch_normalize(hipStream_t st, krps_precision p, void* U, int64_t I, int R,
                            const double* sigma);
// Rows of Y that mode j's entries reach (marked, listed increasing, zeroed),
// then Y[i_j(e)] += x_e (*)_{k != j} U_k[i_k(e)] over every stored entry.
hipError_t launch_mttkrp(hipStream_t st, krps_precision p, const MttkrpArgs& a, int64_t I,
                         int32_t* mark, int64_t* bsum, int32_t* list, int64_t* count, double* Y);
size_t fit_partial_bytes();
hipError_t launch_fit(hipStream_t st, krps_precision p, const FitArgs& a, double* partial,
                      double* out);

// probes.hip: copy, FMA and MFMA loops timed on the stream (ws >= 64 MiB)
krps_status measure_peaks(int device, hipStream_t st, void* ws, size_t ws_bytes,
                          krps_peaks* out);

// descent.hip
hipError_t launch_descent(hipStream_t st, krps_precision p, const DescentArgs& a);
// Batched preparation and walk (jobs and problems in device memory).
int prep_block_threads(int R);
hipError_t launch_prep_batched(hipStream_t st, const PrepJob* jobs, int njobs, int Rmax);
hipError_t launch_eig_batched(hipStream_t st, bool f64, const EigJob* jobs, int njobs, int Rmax);
// Shape class of the batched walk for R and a lanes-per-sample choice
// (0 = default), and the samples one wavefront serves in that class.
constexpr int NBATCH_CLASSES = 9;
int batch_class(int R, int lps);
int batch_group(int cls);
hipError_t launch_descent_batched(hipStream_t st, bool f64, int cls, const BatchProblem* probs,
                                  int P, int64_t ntask, unsigned long long* counter);
hipError_t launch_row_prob(hipStream_t st, krps_precision p, const DescentArgs& a);

}  // namespace krps
