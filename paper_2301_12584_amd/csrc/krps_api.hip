// libkrps C ABI: argument validation, workspace planning and stream-ordered
// launches of the sampler kernels.  Host code only; every computation runs
// in the kernels of tree_build.hip, eig.hip and descent.hip.
#include <algorithm>
#include <cstdio>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "krps_internal.h"

namespace krps {

static thread_local std::string g_err;

void set_error(const std::string& msg) { g_err = msg; }
krps_status fail(krps_status st, const std::string& msg) {
  g_err = msg;
  return st;
}
krps_status hip_fail(hipError_t e, const char* what) {
  g_err = std::string(what) + ": " + hipGetErrorName(e) + " (" + hipGetErrorString(e) + ")";
  return KRPS_EDEVICE;
}

}  // namespace krps

using namespace krps;

struct krps_ctx_s {
  int device;
  hipStream_t stream;
  hipStream_t capture = nullptr;  // own stream for graph capture when `stream` is null
  // a second stream (default priority) and the fork / join events that let
  // a solve's M^+ run beside its fiber lookup and SpMM (created at first use)
  hipStream_t aux = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
  // pinned host staging of batched-draw descriptors (slot 0: preparation
  // jobs, slot 1: walk problems); `staged` marks the copy out of a slot
  // that must finish before the slot is rewritten
  void* pinned[2] = {nullptr, nullptr};
  size_t pinned_bytes[2] = {0, 0};
  hipEvent_t staged[2] = {nullptr, nullptr};
  bool staged_pending[2] = {false, false};
};

struct GraphKey {
  const void* t = nullptr;
  const void* uniforms = nullptr;
  const void* sigma = nullptr;
  const void* ws = nullptr;
  int64_t J = -1;
  int lps = -1, filter = -2, team = -1, det = -1;
  uint64_t seed = 0, ctr_base = 0;
  bool operator==(const GraphKey& o) const {
    return t == o.t && uniforms == o.uniforms && sigma == o.sigma && ws == o.ws && J == o.J &&
           lps == o.lps && filter == o.filter && team == o.team && det == o.det &&
           seed == o.seed &&
           ctr_base == o.ctr_base;
  }
};

struct krps_sampler_s {
  krps_ctx ctx;
  int N, R, F;
  krps_precision prec;
  int elem;                       // bytes per stored element
  std::vector<int64_t> I;
  std::vector<void*> U;
  std::vector<TreeShape> shape;
  std::vector<void*> nodes;
  std::vector<float*> nodes32;         // float32 copies of float64 trees (else null)
  int filter_top = -1;                 // levels read from the float64 tree (-1: default)
  std::vector<double*> gram;
  double* scratch;
  size_t scratch_bytes;
  int32_t* status;
  double* warm;                   // [N + 1][N][R][R] eigenvectors of the last solves
  int32_t* warm_ok;               // [N + 1][N] 1 where warm holds them
  // per-draw workspace layout
  krps_draw_layout lay;
  const void* prepared_ws = nullptr;  // ws of the last preparation
  int prepared_exclude = -2;
  int lps = 0;                         // descent lanes per sample (0 = default)
  int team = 0;                        // waves per leaf team of the tree build (0 = default)
  int det = 0;                         // solves: fixed-point (order-independent) SpMM
  // captured ALS sweep and what its kernels' arguments were made from
  hipGraphExec_t sweep_exec = nullptr;
  GraphKey gkey;
  size_t draw_bytes;
  int64_t enodes;
  int64_t estride;  // elements per mode of the eigen-tree region (nodes + zero padding)
  int DE;
  size_t emass_off;  // per-draw float64 [N][enodes]: E masses at h = 1 (internal)
  size_t ztab_off;   // per-draw float64 [R][znmax]: first-mode Z masses per u, or 0
  size_t zw_off;     // per-draw float64: the table's packed weights per u
  int64_t znmax;     // largest stored-node count of the factor trees (0: no table)
};

struct krps_tensor_s {
  krps_ctx ctx;
  int N;
  int64_t nnz;                 // entries given
  int64_t nu = -1;             // stored entries (distinct coordinates)
  std::vector<int64_t> dims;
  std::vector<int32_t*> cols;  // per mode: [N][nu]
  std::vector<double*> vals;   // per mode: [nu], duplicates summed
  std::vector<int64_t*> off;   // per mode: [dims[lead] + 1]
  std::vector<int> lead;
  std::vector<int16_t*> hot_slot;  // per mode: [dims[j]]
  std::vector<int32_t*> hot_rows;  // per mode: [nhot]
  int nhot = 0;
  double norm2 = 0;
};

namespace {

bool valid_prec(krps_precision p) { return p == KRPS_FP64 || p == KRPS_FP32 || p == KRPS_BF16X2; }
int elem_bytes(krps_precision p) { return p == KRPS_FP64 ? 8 : 4; }

// Walk shapes compiled for each R (lanes per sample; 0 = the default).
bool lps_supported(int R, int lps) {
  if (lps == 0) return true;
  if (R <= 8) return lps == 4 || lps == 8;
  if (R <= 16) return lps == 8 || lps == 16;
  if (R <= 32) return lps == 16 || lps == 32 || lps == 64;
  return lps == 64;
}
// Lanes per sample of a sampler's walks: its set value, else the default
// of its R and storage type.  At 16 < R <= 32 a float32-stored walk
// defaults to 16 lanes (four samples per wavefront in two wavefronts per
// SIMD: 99 against 93 M samples/s at 2^20 x 32 with 32 lanes), a float64
// one to 32 (the 16-lane float64 shape spills).
int default_lps(int R, krps_precision p) {
  if (R <= 8) return 4;
  if (R <= 16) return 8;
  if (R <= 32) return p == KRPS_FP64 ? 32 : 16;
  return 64;
}

std::vector<int> lps_choices(int R) {
  if (R <= 8) return {4, 8};
  if (R <= 16) return {8, 16};
  if (R <= 32) return {16, 32, 64};
  return {64};
}

krps_status check_dims(int N, const int64_t* I, int R) {
  if (N < 1 || N > KRPS_MAX_MODES) return fail(KRPS_EINVAL, "N must be in [1, KRPS_MAX_MODES]");
  if (R < 1 || R > KRPS_MAX_R) return fail(KRPS_EINVAL, "R must be in [1, 128]");
  if (I == nullptr) return fail(KRPS_EINVAL, "I is NULL");
  for (int j = 0; j < N; ++j)
    if (I[j] < 1 || I[j] > INT32_MAX) return fail(KRPS_EINVAL, "each I_j must be in [1, 2^31)");
  return KRPS_OK;
}

struct SamplerPlan {
  std::vector<TreeShape> shape;
  std::vector<size_t> node_off, node32_off, gram_off;
  size_t scratch_off = 0, scratch_bytes = 0, status_off = 0, warm_off = 0, warm_ok_off = 0;
  size_t total = 0;
};

SamplerPlan plan_sampler(int N, const int64_t* I, int R, int F, krps_precision p) {
  SamplerPlan pl;
  const int64_t TR = tri(R);
  size_t off = 0;
  size_t scratch = 0;
  for (int j = 0; j < N; ++j) {
    TreeShape ts;
    ts.init(I[j], F);
    pl.shape.push_back(ts);
    pl.node_off.push_back(off);
    off += align_up((size_t)(ts.n_nodes * TR + NODE_SLACK) * elem_bytes(p));
    // float64 trees: a float32 copy of the nodes for the walk's deep levels
    pl.node32_off.push_back(p == KRPS_FP64 ? off : 0);
    if (p == KRPS_FP64) off += align_up((size_t)(ts.n_nodes * TR + NODE_SLACK) * 4);
    pl.gram_off.push_back(off);
    off += align_up((size_t)R * R * 8);
    const size_t sb = tree_build_scratch_bytes(ts.L, R);
    if (sb > scratch) scratch = sb;
  }
  pl.scratch_off = off;
  pl.scratch_bytes = scratch;
  off += align_up(scratch);
  pl.status_off = off;
  off += 256;
  // warm starts of the solves' eigendecompositions: per exclusion (-1 .. N-1)
  // and drawn mode, the last eigenvectors (float64 R x R) and a flag
  pl.warm_ok_off = off;
  off += align_up((size_t)(N + 1) * N * 4);
  pl.warm_off = off;
  off += align_up((size_t)(N + 1) * N * R * R * 8);
  pl.total = off;
  return pl;
}

// Largest table of first-mode factor-tree masses a draw workspace holds
// (R x stored nodes float64); larger samplers walk the first mode's tree.
constexpr size_t ZTAB_MAX_BYTES = size_t(64) << 20;

void plan_draw(krps_sampler s) {
  const int R = s->R, N = s->N;
  const int64_t TR = tri(R);
  s->DE = R > 1 ? ceil_log2(R) : 0;
  TreeShape es;
  es.init(R, 1);
  s->enodes = es.n_nodes;
  s->estride = s->enodes * TR + NODE_SLACK;
  size_t off = 0;
  krps_draw_layout& l = s->lay;
  l.gplus = off;
  off += align_up((size_t)R * R * 8);
  const size_t gpacked = off;
  off += align_up((size_t)(TR + NODE_SLACK) * 8);
  l.rank = off;
  off += 256;
  l.ggt = off;
  off += align_up((size_t)N * R * R * 8);
  l.lam = off;
  off += align_up((size_t)N * R * 8);
  l.vecs = off;
  off += align_up((size_t)N * R * R * s->elem);
  l.etree = off;
  off += align_up((size_t)N * s->estride * s->elem);
  s->emass_off = off;
  off += align_up((size_t)N * s->enodes * 8);
  // the first drawn mode's factor-tree masses for every eigen-component u,
  // when the table is at most ZTAB_MAX_BYTES
  int64_t znmax = 0;
  for (int k = 0; k < N; ++k) znmax = std::max<int64_t>(znmax, s->shape[k].n_nodes);
  s->znmax = (size_t)R * znmax * 8 <= ZTAB_MAX_BYTES ? znmax : 0;
  s->ztab_off = off;
  off += align_up((size_t)R * s->znmax * 8);
  s->zw_off = off;
  off += s->znmax > 0 ? align_up(ztab_weights_bytes(R)) : 0;
  l.n_enodes = s->enodes;
  l.etree_stride = s->estride;
  s->draw_bytes = off;
  (void)gpacked;
}

size_t gpacked_off(krps_sampler s) { return s->lay.gplus + align_up((size_t)s->R * s->R * 8); }

// The split path's trees are the float32 path's: float64 products of the
// float32 factor (exact) summed in float64, nodes stored in float32, and
// G_j in float64.  bf16 split products in the trees would put ~2^-16
// relative error into G_j, which reaches G^+ and the leverage scores
// multiplied by the condition number of G, and, with the lo lo^T products
// dropped, would make the root Gram indefinite at a condition number above
// ~2^16, so that a drawn component's stage-2 mass could be <= 0.
krps_status build_tree(krps_sampler s, int j) {
  const krps_precision tp = s->prec == KRPS_BF16X2 ? KRPS_FP32 : s->prec;
  hipError_t e = launch_tree_build(s->ctx->stream, tp, s->U[j], s->I[j], s->R, s->shape[j],
                                   s->nodes[j], s->gram[j], s->scratch, s->scratch_bytes,
                                   s->nodes32[j], s->team);
  if (e != hipSuccess) return hip_fail(e, "tree build launch");
  return KRPS_OK;
}

void fill_descent_args(krps_sampler s, int exclude, void* ws, DescentArgs& a);

// Levels of factor k's tree that the walk decides from the float64 nodes
// before it turns to their float32 copy (>= D: the copy is not used).  The
// default keeps the top D - 10 levels, which the caches hold anyway, and
// filters the ten deepest, where the bytes are; each filtered level adds
// its float32 error to the running offset, so that deeper filtering makes
// undecided (re-walked) samples more frequent.
int walk_filter_top(krps_sampler s, int k) {
  const int D = s->shape[k].D;
  if (s->nodes32[k] == nullptr) return D;
  if (s->filter_top >= 0) return std::min(s->filter_top, D);
  return std::max(D - 10, 0);
}

// Enqueues the set-up part of Algorithm 2 (before its per-sample loop) for exclusion `exclude` into ws and
// fills the descent arguments.
krps_status prepare_draw(krps_sampler s, int exclude, void* ws, DescentArgs& a,
                         bool warm = false) {
  char* w = (char*)ws;
  const int R = s->R;
  int order[KRPS_MAX_MODES];
  const double* mats[KRPS_MAX_MODES];
  int nsteps = 0;
  for (int k = 0; k < s->N; ++k)
    if (k != exclude) {
      order[nsteps] = k;
      mats[nsteps] = s->gram[k];
      ++nsteps;
    }
  double* gplus_full = (double*)(w + s->lay.gplus);
  double* gplus_packed = (double*)(w + gpacked_off(s));
  int32_t* rank = (int32_t*)(w + s->lay.rank);
  double* ggt = (double*)(w + s->lay.ggt);
  double* lam = (double*)(w + s->lay.lam);
  void* vecs = w + s->lay.vecs;
  void* etree = w + s->lay.etree;
  hipStream_t st = s->ctx->stream;
  hipError_t e = launch_prep_gplus2(st, R, nsteps, mats, nsteps, order, gplus_full, gplus_packed,
                                    rank, ggt, s->status);
  if (e != hipSuccess) return hip_fail(e, "prep G+ launch");
  // the sketched solves of CP-ALS start each eigendecomposition from the
  // last solve's eigenvectors of the same exclusion and mode; plain draws
  // start cold, so that a repeated draw repeats bit for bit
  double* wv = warm ? s->warm + (size_t)(exclude + 1) * s->N * R * R : nullptr;
  int32_t* wok = warm ? s->warm_ok + (size_t)(exclude + 1) * s->N : nullptr;
  e = launch_prep_eig2(st, s->prec, R, nsteps, mats, order, ggt, lam, vecs, etree, s->estride,
                       rank, (double*)(w + s->emass_off), s->enodes, wv, wok);
  if (e != hipSuccess) return hip_fail(e, "prep eig launch");
  if (s->znmax > 0 && nsteps > 0) {
    const int k0 = order[0];
    e = launch_ztab(st, s->prec, s->nodes[k0], s->shape[k0].n_nodes, R,
                    (char*)vecs + (size_t)k0 * R * R * s->elem, (double*)(w + s->zw_off),
                    (double*)(w + s->ztab_off));
    if (e != hipSuccess) return hip_fail(e, "first-mode table launch");
  }
  fill_descent_args(s, exclude, ws, a);
  return KRPS_OK;
}

// Descent arguments for a preparation of `exclude` held in ws.
void fill_descent_args(krps_sampler s, int exclude, void* ws, DescentArgs& a) {
  char* w = (char*)ws;
  const int R = s->R;
  int order[KRPS_MAX_MODES];
  int nsteps = 0;
  for (int k = 0; k < s->N; ++k)
    if (k != exclude) order[nsteps++] = k;
  double* gplus_packed = (double*)(w + gpacked_off(s));
  int32_t* rank = (int32_t*)(w + s->lay.rank);
  memset(&a, 0, sizeof(a));
  a.N = s->N;
  a.R = R;
  a.exclude = exclude;
  a.nsteps = nsteps;
  const int64_t TR = tri(R);
  for (int i = 0; i < nsteps; ++i) a.order[i] = order[i];
  for (int k = 0; k < s->N; ++k) {
    ModeDesc& m = a.mode[k];
    m.U = s->U[k];
    m.Z = s->nodes[k];
    m.E = w + s->lay.etree + (size_t)k * s->estride * s->elem;
    m.V = w + s->lay.vecs + (size_t)k * R * R * s->elem;
    m.em = (const double*)(w + s->emass_off) + (size_t)k * s->enodes;
    m.zt = s->znmax > 0 ? (const double*)(w + s->ztab_off) : nullptr;
    m.zn = s->shape[k].n_nodes;
    const int top = walk_filter_top(s, k);
    m.z32 = top < s->shape[k].D ? s->nodes32[k] : nullptr;
    m.ztop = top;
    m.I = s->I[k];
    m.L = s->shape[k].L;
    m.F = s->shape[k].F;
    m.D = s->shape[k].D;
    m.DE = s->DE;
    m.ne = (int32_t)s->enodes;
  }
  a.gplus = gplus_packed;
  a.rank = rank;
  a.status = s->status;
  a.lps = s->lps ? s->lps : default_lps(R, s->prec);
}

// ------------------------------------------------------------ tensor plan

struct TensorPlan {
  std::vector<size_t> cols_off, vals_off, off_off, hslot_off, hrows_off;
  std::vector<int> lead;
  size_t hc0 = 0, hc1 = 0, hi0 = 0, hi1 = 0;
  int nhot = 0;
  size_t k0 = 0, k1 = 0, p0 = 0, p1 = 0, temp = 0, temp_bytes = 0, acc = 0, total = 0;
};

TensorPlan plan_tensor(int N, const int64_t* dims, int64_t nnz) {
  TensorPlan pl;
  size_t off = 0;
  for (int j = 0; j < N; ++j) {
    const int lead = N == 1 ? 0 : (j == 0 ? 1 : 0);
    pl.lead.push_back(lead);
    pl.cols_off.push_back(off);
    off += align_up((size_t)N * nnz * 4);
    pl.vals_off.push_back(off);
    off += align_up((size_t)nnz * 8);
    pl.off_off.push_back(off);
    off += align_up((size_t)(dims[lead] + 1) * 8);
  }
  pl.k0 = off;
  off += align_up((size_t)nnz * 4);
  pl.k1 = off;
  off += align_up((size_t)nnz * 4);
  pl.p0 = off;
  off += align_up((size_t)nnz * 4);
  pl.p1 = off;
  off += align_up((size_t)nnz * 4);
  // hot rows: per mode a 16-bit slot per row and the rows; temporaries sized
  // for the largest mode
  int64_t dmax = 1;
  for (int j = 0; j < N; ++j) {
    dmax = dims[j] > dmax ? dims[j] : dmax;
    pl.hslot_off.push_back(off);
    off += align_up((size_t)dims[j] * 2);
    pl.hrows_off.push_back(off);
    off += align_up((size_t)HOT_ROWS * 4);
  }
  pl.nhot = HOT_ROWS;
  pl.hc0 = off;
  off += align_up((size_t)dmax * 4);
  pl.hc1 = off;
  off += align_up((size_t)dmax * 4);
  pl.hi0 = off;
  off += align_up((size_t)dmax * 4);
  pl.hi1 = off;
  off += align_up((size_t)dmax * 4);
  pl.temp_bytes = sort_temp_bytes(nnz);
  {
    const size_t hb = hot_temp_bytes(dmax);
    if (hb > pl.temp_bytes) pl.temp_bytes = hb;
  }
  pl.temp = off;
  off += align_up(pl.temp_bytes);
  pl.acc = off;
  off += align_up(norm2_bytes());
  pl.total = off;
  return pl;
}

// ------------------------------------------------------------- solve plan

// The head of a solve workspace: scratch of the calls that do not depend on
// J (the fit, the normalisation of a factor), below every piece of
// krps_solve_layout, so that those calls leave the last solve's pieces intact.
struct SolveHead {
  size_t fitp, fitout, npart, nsig, ctrw, total;
};

SolveHead plan_head(const krps_sampler_s* s) {
  SolveHead h;
  const int R = s->R;
  size_t off = 0;
  h.fitp = off;
  off += align_up(fit_partial_bytes());
  h.fitout = off;
  off += 256;
  h.npart = off;
  off += align_up(solve_partial_bytes(R));
  h.nsig = off;
  off += align_up((size_t)R * 8);
  h.ctrw = off;
  off += 256;
  h.total = off;
  return h;
}

struct SolvePlan {
  krps_solve_layout lay;
  SolveHead head;
  size_t lo, hi, cnt, start, rank, partial, gscratch, gscratch_bytes;
  size_t coef, slot, hkey, hW, hWlo, hrep, rflag, rpos, rep, rstart, bsum, ymark, ybsum, det;
  int64_t H;
  int hbits;
  size_t total;
  int64_t Imax;
};

SolvePlan plan_solve(const krps_sampler_s* s, int64_t J) {
  SolvePlan pl;
  const int R = s->R, N = s->N;
  int64_t Imax = 0;
  for (int j = 0; j < N; ++j) Imax = s->I[j] > Imax ? s->I[j] : Imax;
  pl.Imax = Imax;
  pl.head = plan_head(s);
  size_t off = pl.head.total;
  krps_solve_layout& l = pl.lay;
  l.draw = off;
  off += align_up(s->draw_bytes);
  l.idx = off;
  off += align_up((size_t)J * N * 4);
  l.prob = off;
  off += align_up((size_t)J * 8);
  l.w = off;
  off += align_up((size_t)J * 8);
  l.rows = off;
  off += align_up((size_t)J * R * 8);
  pl.lo = off;
  off += align_up((size_t)J * 8);
  pl.hi = off;
  off += align_up((size_t)J * 8);
  pl.cnt = off;
  off += align_up((size_t)J * 8);
  pl.start = off;
  off += align_up((size_t)(J + 1) * 8);
  // fiber merge: per-sample coefficient and slot, hash table of H >= 2J slots
  pl.hbits = 6;
  while ((int64_t(1) << pl.hbits) < 2 * J) ++pl.hbits;
  pl.H = int64_t(1) << pl.hbits;
  pl.coef = off;
  off += align_up((size_t)J * 8);
  pl.slot = off;
  off += align_up((size_t)J * 4);
  pl.hkey = off;
  off += align_up((size_t)pl.H * 8);
  pl.hW = off;
  off += align_up((size_t)pl.H * 8);
  pl.hWlo = off;
  off += align_up((size_t)pl.H * 8);
  pl.hrep = off;
  off += align_up((size_t)pl.H * 4);
  pl.rflag = off;
  off += align_up((size_t)J * 8);
  pl.rpos = off;
  off += align_up((size_t)(J + 1) * 8);
  pl.rep = off;
  off += align_up((size_t)J * 4);
  pl.rstart = off;
  off += align_up((size_t)(J + 1) * 8);
  pl.bsum = off;
  off += align_up((size_t)((J + 1023) / 1024 + 2) * 8);
  l.M = off;
  off += align_up((size_t)R * R * 8);
  l.Mp = off;
  off += align_up((size_t)R * R * 8);
  pl.rank = off;
  off += 256;
  l.Y = off;
  off += align_up((size_t)Imax * R * 8);
  l.yrows = off;
  off += align_up((size_t)Imax * 4);
  l.nyrows = off;
  off += 128;
  l.expanded = off;
  off += 128;
  pl.ymark = off;
  off += align_up((size_t)Imax * 4);
  pl.ybsum = off;
  off += align_up(row_bsum_bytes(Imax));
  pl.partial = off;
  off += align_up(solve_partial_bytes(R));
  pl.det = off;
  off += align_up(spmm_det_bytes());
  TreeShape tm;
  tm.init(J > 0 ? J : 1, R);
  pl.gscratch = off;
  pl.gscratch_bytes = tree_build_scratch_bytes(tm.L, R);
  off += align_up(pl.gscratch_bytes);
  pl.total = off;
  return pl;
}

krps_status check_pair(krps_sampler s, krps_tensor t) {
  if (s == nullptr || t == nullptr) return fail(KRPS_EINVAL, "sampler/tensor is NULL");
  if (s->N != t->N) return fail(KRPS_EINVAL, "sampler and tensor have different N");
  for (int k = 0; k < s->N; ++k)
    if (s->I[k] != t->dims[k]) return fail(KRPS_EINVAL, "factor heights differ from tensor dims");
  return KRPS_OK;
}

// Where the walk of a solve takes its uniforms: the device array u01
// ([J][N][2]), or, when u01 is null, Philox4x64-10 of counter
// (ctr_base + d, k, ctr2 + *ctr2_dev, 0) under key (seed, 0).
struct UniformSrc {
  const double* u01 = nullptr;
  uint64_t seed = 0, ctr_base = 0, ctr2 = 0;
  const uint64_t* ctr2_dev = nullptr;
};

// Enqueues one sketched solve of mode j.
krps_status enqueue_solve(krps_sampler s, krps_tensor t, int j, int64_t J, const UniformSrc& us,
                          double* sigma, char* w, const SolvePlan& pl) {
  const int R = s->R, N = s->N;
  hipStream_t st = s->ctx->stream;
  const krps_solve_layout& l = pl.lay;
  DescentArgs a;
  krps_status rs = prepare_draw(s, j, w + l.draw, a, true);
  if (rs != KRPS_OK) return rs;
  // rows of S A = w_d a_d: float64 for the float64 and float32 paths (the
  // Gram M and Y are then formed in float64), float32 for the bf16 split
  const bool split = s->prec == KRPS_BF16X2;
  a.J = J;
  a.u01 = us.u01;
  a.seed = us.seed;
  a.ctr_base = us.ctr_base;
  a.ctr2 = us.ctr2;
  a.ctr2_dev = us.ctr2_dev;
  a.idx = (int32_t*)(w + l.idx);
  a.prob = (double*)(w + l.prob);
  if (split)
    a.rows = w + l.rows;
  else
    a.rows64 = (double*)(w + l.rows);
  a.wout = (double*)(w + l.w);
  a.scale_rows = 1;
  hipError_t e = launch_descent(st, s->prec, a);
  if (e != hipSuccess) return hip_fail(e, "descent launch");
  // M = (S A)^T (S A): the Gram of the scaled sampled rows, by the tree
  // builder without stored nodes
  TreeShape tm;
  tm.init(J, R);
  e = launch_tree_build(st, split ? KRPS_BF16X2 : KRPS_FP64, w + l.rows, J, R, tm, nullptr,
                        (double*)(w + l.M), (double*)(w + pl.gscratch), pl.gscratch_bytes);
  if (e != hipSuccess) return hip_fail(e, "Gram of sampled rows");
  // M^+ depends only on M: it runs on the context's second stream beside
  // the fiber lookup and the SpMM, and the GEMM waits for it (a captured
  // sweep records this fork and join as graph edges).  A non-finite M (a
  // non-finite sampled row) would give M^+ = 0 and a zero factor: it is
  // flagged in the sampler's status.
  krps_ctx cx = s->ctx;
  if (cx->aux == nullptr) {
    KRPS_HIP(hipStreamCreateWithFlags(&cx->aux, hipStreamNonBlocking));
    KRPS_HIP(hipEventCreateWithFlags(&cx->fork, hipEventDisableTiming));
    KRPS_HIP(hipEventCreateWithFlags(&cx->join, hipEventDisableTiming));
  }
  KRPS_HIP(hipEventRecord(cx->fork, st));
  KRPS_HIP(hipStreamWaitEvent(cx->aux, cx->fork, 0));
  e = launch_pinv(cx->aux, R, (double*)(w + l.M), (double*)(w + l.Mp), (int32_t*)(w + pl.rank),
                  s->status);
  if (e != hipSuccess) return hip_fail(e, "pseudo-inverse");
  KRPS_HIP(hipEventRecord(cx->join, cx->aux));
  FiberArgs fa{};
  fa.N = N;
  fa.j = j;
  fa.lead = t->lead[j];
  fa.R = R;
  fa.nnz = t->nu;
  fa.J = J;
  fa.cols = t->cols[j];
  fa.vals = t->vals[j];
  fa.off = t->off[j];
  fa.sample_idx = (const int32_t*)(w + l.idx);
  fa.w = (const double*)(w + l.w);
  fa.lo = (int64_t*)(w + pl.lo);
  fa.hi = (int64_t*)(w + pl.hi);
  fa.cnt = (int64_t*)(w + pl.cnt);
  fa.start = (int64_t*)(w + pl.start);
  fa.coef = (double*)(w + pl.coef);
  fa.slot = (int32_t*)(w + pl.slot);
  fa.hkey = (unsigned long long*)(w + pl.hkey);
  fa.hW = (double*)(w + pl.hW);
  fa.hrep = (int32_t*)(w + pl.hrep);
  fa.H = pl.H;
  fa.hbits = pl.hbits;
  fa.rflag = (int64_t*)(w + pl.rflag);
  fa.rpos = (int64_t*)(w + pl.rpos);
  fa.rep = (int32_t*)(w + pl.rep);
  fa.rstart = (int64_t*)(w + pl.rstart);
  fa.bsum = (int64_t*)(w + pl.bsum);
  fa.hot_slot = t->hot_slot[j];
  fa.hot_rows = t->hot_rows[j];
  fa.nhot = (int)std::min<int64_t>(t->nhot, t->dims[j]);
  fa.expanded = (int64_t*)(w + l.expanded);
  fa.hWlo = s->det ? (long long*)(w + pl.hWlo) : nullptr;
  fa.wscale = s->det ? (double*)(w + pl.det + spmm_det_bytes() - 16) : nullptr;
  e = launch_lookup(st, fa);
  if (e != hipSuccess) return hip_fail(e, "fiber lookup");
  // only the rows of Y that the entries reach are cleared, summed into and
  // multiplied by M^+
  int32_t* yrows = (int32_t*)(w + l.yrows);
  int64_t* nyrows = (int64_t*)(w + l.nyrows);
  // the deterministic mode sums Y in fixed point and converts it to float64
  // (also on the split path, whose Y is otherwise float32)
  const bool ydouble = !split || s->det;
  e = launch_rows(st, fa, s->I[j], (int32_t*)(w + pl.ymark), (int64_t*)(w + pl.ybsum), yrows,
                  nyrows, w + l.Y, !ydouble);
  if (e != hipSuccess) return hip_fail(e, "rows of Y");
  if (s->det)
    e = launch_spmm_det(st, split ? KRPS_BF16X2 : KRPS_FP64, fa, w + l.rows, w + l.Y, yrows, nyrows,
                        (double*)(w + pl.det));
  else
    e = launch_spmm(st, split ? KRPS_BF16X2 : KRPS_FP64, fa, w + l.rows, w + l.Y);
  if (e != hipSuccess) return hip_fail(e, "SpMM");
  KRPS_HIP(hipStreamWaitEvent(st, cx->join, 0));
  // the split path's factor is float32, like the float32 path's
  const krps_precision gp = split && s->det ? KRPS_FP32 : s->prec;
  e = launch_solve_gemm(st, gp, w + l.Y, (const double*)(w + l.Mp), s->U[j], s->I[j], yrows,
                        nyrows, R, (double*)(w + pl.partial), sigma);
  if (e != hipSuccess) return hip_fail(e, "solve GEMM");
  return build_tree(s, j);
}

// Validation and enqueue of one solve (krps_sketched_solve[_seeded]).
krps_status solve_entry(krps_sampler s, krps_tensor t, int j, int64_t J, const UniformSrc& us,
                        double* sigma, void* ws, size_t ws_bytes) {
  krps_status st = check_pair(s, t);
  if (st != KRPS_OK) return st;
  if (s->N < 2) return fail(KRPS_EINVAL, "a solve needs N >= 2");
  if (j < 0 || j >= s->N) return fail(KRPS_EINVAL, "j out of range");
  if (J < 1) return fail(KRPS_EINVAL, "J must be >= 1");
  if (sigma == nullptr || ws == nullptr) return fail(KRPS_EINVAL, "sigma/workspace is NULL");
  SolvePlan pl = plan_solve(s, J);
  if (ws_bytes < pl.total) return fail(KRPS_EWORKSPACE, "solve workspace too small");
  KRPS_HIP(hipSetDevice(s->ctx->device));
  st = enqueue_solve(s, t, j, J, us, sigma, (char*)ws, pl);
  s->prepared_ws = nullptr;
  return st;
}

// One sweep, from a uniform buffer [N][J][N][2] (uniforms != null) or from
// in-kernel Philox with counter word 2 = sweep * N + j.  The seeded form
// reads sweep * N from a word of the workspace head, written by a one-thread
// kernel enqueued before the sweep (outside any captured graph), so one
// captured graph serves every sweep.
krps_status sweep_entry(krps_sampler s, krps_tensor t, int64_t J, const double* uniforms,
                        uint64_t seed, uint64_t ctr_base, uint64_t sweep, double* sigma, void* ws,
                        size_t ws_bytes, int use_graph) {
  krps_status st = check_pair(s, t);
  if (st != KRPS_OK) return st;
  if (s->N < 2) return fail(KRPS_EINVAL, "a sweep needs N >= 2");
  if (J < 1) return fail(KRPS_EINVAL, "J must be >= 1");
  if (sigma == nullptr || ws == nullptr) return fail(KRPS_EINVAL, "sigma/workspace is NULL");
  SolvePlan pl = plan_solve(s, J);
  if (ws_bytes < pl.total) return fail(KRPS_EWORKSPACE, "solve workspace too small");
  KRPS_HIP(hipSetDevice(s->ctx->device));
  hipStream_t stream = s->ctx->stream;
  const bool seeded = uniforms == nullptr;
  uint64_t* ctrw = (uint64_t*)((char*)ws + pl.head.ctrw);
  if (seeded) {
    hipError_t e = launch_set_u64(stream, ctrw, sweep * (uint64_t)s->N);
    if (e != hipSuccess) return hip_fail(e, "sweep counter");
  }
  const size_t ublock = (size_t)J * s->N * 2;
  auto enqueue_all = [&]() -> krps_status {
    for (int j = 0; j < s->N; ++j) {
      UniformSrc us;
      if (seeded) {
        us.seed = seed;
        us.ctr_base = ctr_base;
        us.ctr2 = (uint64_t)j;
        us.ctr2_dev = ctrw;
      } else {
        us.u01 = uniforms + j * ublock;
      }
      krps_status r = enqueue_solve(s, t, j, J, us, sigma, (char*)ws, pl);
      if (r != KRPS_OK) return r;
    }
    return KRPS_OK;
  };
  if (!use_graph) {
    st = enqueue_all();
    s->prepared_ws = nullptr;
    return st;
  }
  // the captured graph is keyed by everything its kernels' arguments hold
  const GraphKey key{t,         uniforms,          sigma, ws, J, s->lps, s->filter_top,
                     s->team,   s->det,            seeded ? seed : 0, seeded ? ctr_base : 0};
  if (s->sweep_exec == nullptr || !(s->gkey == key)) {
    if (s->sweep_exec != nullptr) {
      (void)hipGraphExecDestroy(s->sweep_exec);
      s->sweep_exec = nullptr;
    }
    // the null stream cannot be captured: capture on the context's own
    // stream, replay on the caller's
    hipStream_t cap = stream;
    if (cap == nullptr) {
      if (s->ctx->capture == nullptr)
        KRPS_HIP(hipStreamCreateWithFlags(&s->ctx->capture, hipStreamNonBlocking));
      cap = s->ctx->capture;
    }
    KRPS_HIP(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
    s->ctx->stream = cap;
    st = enqueue_all();
    s->ctx->stream = stream;
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(cap, &g);
    if (st != KRPS_OK) {
      if (g) (void)hipGraphDestroy(g);
      return st;
    }
    if (e != hipSuccess) return hip_fail(e, "end capture");
    e = hipGraphInstantiate(&s->sweep_exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return hip_fail(e, "graph instantiate");
    s->gkey = key;
  }
  KRPS_HIP(hipGraphLaunch(s->sweep_exec, stream));
  s->prepared_ws = nullptr;
  return KRPS_OK;
}

}  // namespace

extern "C" {

const char* krps_last_error(void) { return g_err.c_str(); }
const char* krps_version(void) { return "libkrps 0.1 (gfx950)"; }

krps_status krps_ctx_create(int device, void* hip_stream, krps_ctx* out) {
  if (out == nullptr) return fail(KRPS_EINVAL, "out is NULL");
  int n = 0;
  KRPS_HIP(hipGetDeviceCount(&n));
  if (device < 0 || device >= n) return fail(KRPS_EINVAL, "device out of range");
  KRPS_HIP(hipSetDevice(device));
  krps_ctx c = new (std::nothrow) krps_ctx_s;
  if (c == nullptr) return fail(KRPS_EINVAL, "out of host memory");
  c->device = device;
  c->stream = (hipStream_t)hip_stream;
  *out = c;
  return KRPS_OK;
}

krps_status krps_ctx_destroy(krps_ctx ctx) {
  for (int i = 0; ctx != nullptr && i < 2; ++i) {
    if (ctx->staged[i] != nullptr) {
      (void)hipEventSynchronize(ctx->staged[i]);
      (void)hipEventDestroy(ctx->staged[i]);
    }
    if (ctx->pinned[i] != nullptr) (void)hipHostFree(ctx->pinned[i]);
  }
  if (ctx != nullptr && ctx->capture != nullptr) (void)hipStreamDestroy(ctx->capture);
  if (ctx != nullptr && ctx->aux != nullptr) {
    (void)hipStreamSynchronize(ctx->aux);
    (void)hipStreamDestroy(ctx->aux);
  }
  if (ctx != nullptr && ctx->fork != nullptr) (void)hipEventDestroy(ctx->fork);
  if (ctx != nullptr && ctx->join != nullptr) (void)hipEventDestroy(ctx->join);
  delete ctx;
  return KRPS_OK;
}

krps_status krps_measure_peaks(krps_ctx ctx, void* ws, size_t ws_bytes, krps_peaks* out) {
  if (ctx == nullptr) return fail(KRPS_EINVAL, "ctx is NULL");
  return measure_peaks(ctx->device, ctx->stream, ws, ws_bytes, out);
}

krps_status krps_ctx_sync(krps_ctx ctx) {
  if (ctx == nullptr) return fail(KRPS_EINVAL, "ctx is NULL");
  KRPS_HIP(hipStreamSynchronize(ctx->stream));
  return KRPS_OK;
}

krps_status krps_sampler_workspace_bytes(int N, const int64_t* I, int R, int F, krps_precision p,
                                         size_t* bytes) {
  krps_status st = check_dims(N, I, R);
  if (st != KRPS_OK) return st;
  if (!valid_prec(p)) return fail(KRPS_EINVAL, "unknown precision");
  if (F < 0) return fail(KRPS_EINVAL, "F must be >= 0");
  if (bytes == nullptr) return fail(KRPS_EINVAL, "bytes is NULL");
  *bytes = plan_sampler(N, I, R, F == 0 ? R : F, p).total;
  return KRPS_OK;
}

krps_status krps_sampler_create(krps_ctx ctx, int N, const int64_t* I, int R, int F,
                                void* const* U, krps_precision p, void* ws, size_t ws_bytes,
                                krps_sampler* out) {
  if (ctx == nullptr || out == nullptr) return fail(KRPS_EINVAL, "ctx/out is NULL");
  krps_status st = check_dims(N, I, R);
  if (st != KRPS_OK) return st;
  if (!valid_prec(p)) return fail(KRPS_EINVAL, "unknown precision");
  if (F < 0) return fail(KRPS_EINVAL, "F must be >= 0");
  if (U == nullptr) return fail(KRPS_EINVAL, "U is NULL");
  for (int j = 0; j < N; ++j)
    if (U[j] == nullptr) return fail(KRPS_EINVAL, "U[j] is NULL");
  if (ws == nullptr) return fail(KRPS_EINVAL, "workspace is NULL");
  const int Fe = F == 0 ? R : F;
  SamplerPlan pl = plan_sampler(N, I, R, Fe, p);
  if (ws_bytes < pl.total) return fail(KRPS_EWORKSPACE, "sampler workspace too small");
  krps_sampler s = new (std::nothrow) krps_sampler_s;
  if (s == nullptr) return fail(KRPS_EINVAL, "out of host memory");
  s->ctx = ctx;
  s->N = N;
  s->R = R;
  s->F = Fe;
  s->prec = p;
  s->elem = elem_bytes(p);
  char* w = (char*)ws;
  for (int j = 0; j < N; ++j) {
    s->I.push_back(I[j]);
    s->U.push_back(U[j]);
    s->shape.push_back(pl.shape[j]);
    s->nodes.push_back(w + pl.node_off[j]);
    s->nodes32.push_back(p == KRPS_FP64 ? (float*)(w + pl.node32_off[j]) : nullptr);
    s->gram.push_back((double*)(w + pl.gram_off[j]));
  }
  s->scratch = (double*)(w + pl.scratch_off);
  s->scratch_bytes = pl.scratch_bytes;
  s->status = (int32_t*)(w + pl.status_off);
  s->warm = (double*)(w + pl.warm_off);
  s->warm_ok = (int32_t*)(w + pl.warm_ok_off);
  plan_draw(s);
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) {
    delete s;
    return hip_fail(e, "hipSetDevice");
  }
  e = hipMemsetAsync(s->status, 0, 12, ctx->stream);
  if (e == hipSuccess)
    e = hipMemsetAsync(s->warm_ok, 0, (size_t)(N + 1) * N * 4, ctx->stream);
  for (int j = 0; j < N && e == hipSuccess; ++j) {
    e = launch_fill(ctx->stream, p, (char*)s->nodes[j] + (size_t)pl.shape[j].n_nodes * tri(R) * s->elem,
                    NODE_SLACK);
    if (e == hipSuccess && s->nodes32[j] != nullptr)
      e = launch_fill(ctx->stream, KRPS_FP32, s->nodes32[j] + pl.shape[j].n_nodes * tri(R),
                      NODE_SLACK);
  }
  if (e != hipSuccess) {
    delete s;
    return hip_fail(e, "status and padding clear");
  }
  for (int j = 0; j < N; ++j) {
    st = build_tree(s, j);
    if (st != KRPS_OK) {
      delete s;
      return st;
    }
  }
  *out = s;
  return KRPS_OK;
}

krps_status krps_sampler_update_entries(krps_sampler s, int j, int64_t M, const int64_t* rows,
                                        const int32_t* cols, const double* values) {
  if (s == nullptr) return fail(KRPS_EINVAL, "sampler is NULL");
  if (j < 0 || j >= s->N) return fail(KRPS_EINVAL, "j out of range");
  if (M < 0) return fail(KRPS_EINVAL, "M < 0");
  if (M > 0 && (rows == nullptr || cols == nullptr || values == nullptr))
    return fail(KRPS_EINVAL, "rows/cols/values is NULL");
  for (int64_t m = 0; m < M; ++m) {
    if (rows[m] < 0 || rows[m] >= s->I[j]) return fail(KRPS_EINVAL, "row out of range");
    if (cols[m] < 0 || cols[m] >= s->R) return fail(KRPS_EINVAL, "column out of range");
    if (!std::isfinite(values[m])) return fail(KRPS_EINVAL, "value is not finite");
  }
  KRPS_HIP(hipSetDevice(s->ctx->device));
  for (int64_t m0 = 0; m0 < M; m0 += UPDATE_CHUNK) {
    UpdateList ul;
    ul.n = (int)std::min<int64_t>(UPDATE_CHUNK, M - m0);
    for (int q = 0; q < ul.n; ++q) {
      ul.row[q] = rows[m0 + q];
      ul.col[q] = cols[m0 + q];
      ul.val[q] = values[m0 + q];
    }
    hipError_t e = launch_update_entries(s->ctx->stream, s->prec, ul, s->U[j], s->nodes[j],
                                         s->nodes32[j], s->gram[j], s->I[j], s->R, s->shape[j]);
    if (e != hipSuccess) return hip_fail(e, "entry update launch");
  }
  // a preparation made before the update no longer describes the trees
  s->prepared_ws = nullptr;
  return KRPS_OK;
}

krps_status krps_sampler_refresh(krps_sampler s, int j) {
  if (s == nullptr) return fail(KRPS_EINVAL, "sampler is NULL");
  if (j < 0 || j >= s->N) return fail(KRPS_EINVAL, "j out of range");
  return build_tree(s, j);
}

krps_status krps_sampler_destroy(krps_sampler s) {
  if (s != nullptr && s->sweep_exec != nullptr) (void)hipGraphExecDestroy(s->sweep_exec);
  delete s;
  return KRPS_OK;
}

krps_status krps_sampler_check(krps_sampler s, int64_t* zero_weight, int64_t* rewalked) {
  if (s == nullptr) return fail(KRPS_EINVAL, "sampler is NULL");
  KRPS_HIP(hipSetDevice(s->ctx->device));
  int32_t words[3] = {0, 0, 0};
  KRPS_HIP(hipMemcpyAsync(words, s->status, 12, hipMemcpyDeviceToHost, s->ctx->stream));
  KRPS_HIP(hipStreamSynchronize(s->ctx->stream));
  KRPS_HIP(hipMemsetAsync(s->status, 0, 12, s->ctx->stream));
  if (zero_weight != nullptr) *zero_weight = words[1];
  if (rewalked != nullptr) *rewalked = words[2];
  if (words[0] & ST_ZERO) return fail(KRPS_EZERO, "the Khatri-Rao product is zero");
  if (words[0] & ST_NUMERIC)
    return fail(KRPS_ENUMERIC, "a non-finite value or a non-positive mass was met (a draw's "
                               "masses, or a solve's sampled Gram)");
  return KRPS_OK;
}

krps_status krps_sampler_set_filter(krps_sampler s, int top) {
  if (s == nullptr) return fail(KRPS_EINVAL, "sampler is NULL");
  if (top < -1) return fail(KRPS_EINVAL, "top must be >= -1");
  s->filter_top = top;
  return KRPS_OK;
}

krps_status krps_sampler_set_deterministic(krps_sampler s, int on) {
  if (s == nullptr) return fail(KRPS_EINVAL, "sampler is NULL");
  s->det = on ? 1 : 0;
  return KRPS_OK;
}

krps_status krps_sampler_set_build(krps_sampler s, int team) {
  if (s == nullptr) return fail(KRPS_EINVAL, "sampler is NULL");
  const std::vector<int> ch = build_team_choices(s->R, s->prec);
  if (team != 0 && std::find(ch.begin(), ch.end(), team) == ch.end())
    return fail(KRPS_EINVAL, "team width not available for R and precision");
  s->team = team;
  return KRPS_OK;
}

krps_status krps_sampler_set_lps(krps_sampler s, int lps) {
  if (s == nullptr) return fail(KRPS_EINVAL, "sampler is NULL");
  if (!lps_supported(s->R, lps)) return fail(KRPS_EINVAL, "lanes per sample not available for R");
  s->lps = lps;
  return KRPS_OK;
}

krps_status krps_sample_workspace_bytes(krps_sampler s, size_t* bytes) {
  if (s == nullptr || bytes == nullptr) return fail(KRPS_EINVAL, "sampler/bytes is NULL");
  *bytes = s->draw_bytes;
  return KRPS_OK;
}

static krps_status check_draw_args(krps_sampler s, int exclude, void* ws, size_t ws_bytes) {
  if (s == nullptr) return fail(KRPS_EINVAL, "sampler is NULL");
  if (exclude < -1 || exclude >= s->N) return fail(KRPS_EINVAL, "exclude out of range");
  if (exclude >= 0 && s->N == 1) return fail(KRPS_EINVAL, "cannot exclude the only factor");
  if (ws == nullptr) return fail(KRPS_EINVAL, "workspace is NULL");
  if (ws_bytes < s->draw_bytes) return fail(KRPS_EWORKSPACE, "draw workspace too small");
  return KRPS_OK;
}

krps_status krps_sample_prepare(krps_sampler s, int exclude, void* ws, size_t ws_bytes) {
  krps_status st = check_draw_args(s, exclude, ws, ws_bytes);
  if (st != KRPS_OK) return st;
  DescentArgs a;
  st = prepare_draw(s, exclude, ws, a);
  if (st != KRPS_OK) return st;
  s->prepared_ws = ws;
  s->prepared_exclude = exclude;
  return KRPS_OK;
}

krps_status krps_sample_draw(krps_sampler s, int exclude, int64_t J, const double* uniforms,
                             int32_t* idx, double* prob, void* rows, void* ws, size_t ws_bytes) {
  krps_status st = check_draw_args(s, exclude, ws, ws_bytes);
  if (st != KRPS_OK) return st;
  if (J < 0) return fail(KRPS_EINVAL, "J < 0");
  if (J > 0 && (uniforms == nullptr || idx == nullptr))
    return fail(KRPS_EINVAL, "uniforms/idx is NULL");
  if (s->prepared_ws != ws || s->prepared_exclude != exclude)
    return fail(KRPS_EINVAL, "krps_sample_draw without a matching krps_sample_prepare");
  DescentArgs a;
  fill_descent_args(s, exclude, ws, a);
  a.J = J;
  a.u01 = uniforms;
  a.idx = idx;
  a.prob = prob;
  a.rows = rows;
  hipError_t e = launch_descent(s->ctx->stream, s->prec, a);
  if (e != hipSuccess) return hip_fail(e, "descent launch");
  return KRPS_OK;
}

krps_status krps_sample_seeded(krps_sampler s, int exclude, int64_t J, uint64_t seed,
                               uint64_t ctr_base, int32_t* idx, double* prob, void* rows,
                               void* ws, size_t ws_bytes) {
  krps_status st = krps_sample_prepare(s, exclude, ws, ws_bytes);
  if (st != KRPS_OK) return st;
  if (J < 0) return fail(KRPS_EINVAL, "J < 0");
  if (J > 0 && idx == nullptr) return fail(KRPS_EINVAL, "idx is NULL");
  DescentArgs a;
  fill_descent_args(s, exclude, ws, a);
  a.J = J;
  a.u01 = nullptr;
  a.seed = seed;
  a.ctr_base = ctr_base;
  a.idx = idx;
  a.prob = prob;
  a.rows = rows;
  hipError_t e = launch_descent(s->ctx->stream, s->prec, a);
  if (e != hipSuccess) return hip_fail(e, "descent launch");
  return KRPS_OK;
}

krps_status krps_sample(krps_sampler s, int exclude, int64_t J, const double* uniforms,
                        int32_t* idx, double* prob, void* rows, void* ws, size_t ws_bytes,
                        int check) {
  krps_status st = krps_sample_prepare(s, exclude, ws, ws_bytes);
  if (st != KRPS_OK) return st;
  st = krps_sample_draw(s, exclude, J, uniforms, idx, prob, rows, ws, ws_bytes);
  if (st != KRPS_OK) return st;
  if (check) {
    int32_t flag = 0;
    KRPS_HIP(hipMemcpyAsync(&flag, s->status, 4, hipMemcpyDeviceToHost, s->ctx->stream));
    KRPS_HIP(hipStreamSynchronize(s->ctx->stream));
    if (flag & ST_ZERO) return fail(KRPS_EZERO, "the Khatri-Rao product is zero");
    if (flag & ST_NUMERIC) return fail(KRPS_ENUMERIC, "non-finite or non-positive mass met");
  }
  return KRPS_OK;
}

}  // extern "C"

// ------------------------------------------------ allocation-free draws

// Per-draw scratch of krps_sample_static: one array per GPU the library
// runs on, held until the process ends.  In host code the name is only a
// stand-in; the device address of each GPU's copy is looked up once per
// device (with that device current) and used everywhere instead.
static __device__ __align__(256) unsigned char scratch[KRPS_STATIC_SCRATCH_BYTES];

namespace {

std::mutex g_scratch_mu;
void* g_scratch_ptr[256] = {nullptr};

// Device address of this GPU's scratch array (looked up on first use).
krps_status static_scratch(int device, void** out) {
  if (device < 0 || device >= 256) return fail(KRPS_EINVAL, "device out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device] == nullptr) {
    void* ptr = nullptr;
    KRPS_HIP(hipSetDevice(device));
    KRPS_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (ptr == nullptr) return fail(KRPS_EDEVICE, "scratch array has no device address");
    g_scratch_ptr[device] = ptr;
  }
  *out = g_scratch_ptr[device];
  return KRPS_OK;
}

}  // namespace

extern "C" {

krps_status krps_sample_static(krps_sampler s, int exclude, int64_t J, const double* uniforms,
                               int32_t* idx, double* prob, void* rows) {
  if (s == nullptr) return fail(KRPS_EINVAL, "sampler is NULL");
  if (s->draw_bytes > (size_t)KRPS_STATIC_SCRATCH_BYTES)
    return fail(KRPS_EWORKSPACE, "per-draw scratch of this sampler (" +
                                     std::to_string(s->draw_bytes) + " bytes) exceeds the " +
                                     std::to_string(KRPS_STATIC_SCRATCH_BYTES) +
                                     "-byte static scratch");
  void* ws = nullptr;
  krps_status st = static_scratch(s->ctx->device, &ws);
  if (st != KRPS_OK) return st;
  st = krps_sample_prepare(s, exclude, ws, s->draw_bytes);
  if (st != KRPS_OK) return st;
  return krps_sample_draw(s, exclude, J, uniforms, idx, prob, rows, ws, s->draw_bytes);
}

}  // extern "C"

namespace {

// Workspace of a batched draw: per problem its draw scratch and packed-
// index table, then the job and problem descriptors and two task counters.
struct BatchPlan {
  std::vector<size_t> draw_off, tab_off;
  size_t desc = 0, prep = 0, eig = 0, ztab = 0, probs = 0, counters = 0, total = 0;
  int n_eig = 0;
};

int drawn_modes(krps_sampler s, int exclude) { return exclude >= 0 ? s->N - 1 : s->N; }

BatchPlan plan_batch(int P, const krps_sampler* s, const int* exclude) {
  BatchPlan pl;
  size_t off = 0;
  for (int p = 0; p < P; ++p) {
    pl.draw_off.push_back(off);
    off += align_up(s[p]->draw_bytes);
    pl.tab_off.push_back(off);
    off += align_up((size_t)tri(s[p]->R) * 2);
    pl.n_eig += drawn_modes(s[p], exclude[p]);
  }
  pl.desc = off;
  pl.prep = off;
  off += align_up((size_t)P * sizeof(PrepJob));
  pl.eig = off;
  off += align_up((size_t)pl.n_eig * sizeof(EigJob));
  pl.ztab = off;
  off += align_up((size_t)P * sizeof(ZtabJob));
  pl.probs = off;
  off += align_up((size_t)P * sizeof(BatchProblem));
  pl.counters = off;
  off += 256;
  pl.total = off;
  return pl;
}

krps_status check_batch(krps_ctx ctx, int P, const krps_sampler* s, const int* exclude) {
  if (ctx == nullptr) return fail(KRPS_EINVAL, "ctx is NULL");
  if (P < 1) return fail(KRPS_EINVAL, "P must be >= 1");
  if (s == nullptr || exclude == nullptr) return fail(KRPS_EINVAL, "samplers/exclude is NULL");
  for (int p = 0; p < P; ++p) {
    if (s[p] == nullptr) return fail(KRPS_EINVAL, "a sampler is NULL");
    if (s[p]->ctx->device != ctx->device) return fail(KRPS_EINVAL, "sampler on another device");
    if (exclude[p] < -1 || exclude[p] >= s[p]->N) return fail(KRPS_EINVAL, "exclude out of range");
  }
  return KRPS_OK;
}

// Copies `bytes` of host descriptors to device memory `dst` on the context
// stream through pinned staging slot `slot` (waits for that slot's
// previous copy first).
krps_status stage_copy(krps_ctx ctx, int slot, const void* src, size_t bytes, void* dst) {
  if (bytes == 0) return KRPS_OK;
  if (ctx->staged_pending[slot]) {
    KRPS_HIP(hipEventSynchronize(ctx->staged[slot]));
    ctx->staged_pending[slot] = false;
  }
  if (ctx->pinned_bytes[slot] < bytes) {
    if (ctx->pinned[slot] != nullptr) KRPS_HIP(hipHostFree(ctx->pinned[slot]));
    ctx->pinned[slot] = nullptr;
    ctx->pinned_bytes[slot] = 0;
    KRPS_HIP(hipHostMalloc(&ctx->pinned[slot], bytes, hipHostMallocDefault));
    ctx->pinned_bytes[slot] = bytes;
  }
  if (ctx->staged[slot] == nullptr)
    KRPS_HIP(hipEventCreateWithFlags(&ctx->staged[slot], hipEventDisableTiming));
  memcpy(ctx->pinned[slot], src, bytes);
  KRPS_HIP(hipMemcpyAsync(dst, ctx->pinned[slot], bytes, hipMemcpyHostToDevice, ctx->stream));
  KRPS_HIP(hipEventRecord(ctx->staged[slot], ctx->stream));
  ctx->staged_pending[slot] = true;
  return KRPS_OK;
}

// Walk cost of one sample (float64 FMAs), for ordering the tasks.
double sample_cost(krps_sampler s, int exclude) {
  const double TR = (double)tri(s->R);
  double c = 0;
  for (int k = 0; k < s->N; ++k)
    if (k != exclude) c += TR * (s->DE + s->shape[k].D + 2) + (double)s->shape[k].F * s->R;
  return c;
}

}  // namespace

extern "C" {

krps_status krps_sample_batched_workspace_bytes(krps_ctx ctx, int P, const krps_sampler* s,
                                                const int* exclude, size_t* bytes) {
  krps_status st = check_batch(ctx, P, s, exclude);
  if (st != KRPS_OK) return st;
  if (bytes == nullptr) return fail(KRPS_EINVAL, "bytes is NULL");
  *bytes = plan_batch(P, s, exclude).total;
  return KRPS_OK;
}

krps_status krps_sample_batched_prepare(krps_ctx ctx, int P, const krps_sampler* s,
                                        const int* exclude, void* ws, size_t ws_bytes) {
  krps_status st = check_batch(ctx, P, s, exclude);
  if (st != KRPS_OK) return st;
  if (ws == nullptr) return fail(KRPS_EINVAL, "workspace is NULL");
  const BatchPlan pl = plan_batch(P, s, exclude);
  if (ws_bytes < pl.total) return fail(KRPS_EWORKSPACE, "batched workspace too small");
  char* w = (char*)ws;
  KRPS_HIP(hipSetDevice(ctx->device));
  hipStream_t stream = ctx->stream;
  // preparation jobs sorted by block size; eigen jobs by storage type, then
  // block size
  std::vector<PrepJob> prep(P);
  std::vector<EigJob> eig;
  std::vector<int> eprob;  // problem of each eigen job
  for (int p = 0; p < P; ++p) {
    krps_sampler sp = s[p];
    char* dw = w + pl.draw_off[p];
    PrepJob& pj = prep[p];
    memset(&pj, 0, sizeof(pj));
    int nsteps = 0;
    for (int k = 0; k < sp->N; ++k)
      if (k != exclude[p]) {
        pj.gl.order[nsteps] = k;
        pj.gl.G[nsteps] = sp->gram[k];
        ++nsteps;
      }
    pj.nmat = nsteps;
    pj.R = sp->R;
    pj.nsteps = nsteps;
    pj.gplus_full = (double*)(dw + sp->lay.gplus);
    pj.gplus_packed = (double*)(dw + gpacked_off(sp));
    pj.rank = (int32_t*)(dw + sp->lay.rank);
    pj.ggt = (double*)(dw + sp->lay.ggt);
    pj.status = sp->status;
    for (int t = 0; t < nsteps; ++t) {
      EigJob ej;
      memset(&ej, 0, sizeof(ej));
      ej.gl = pj.gl;
      ej.st = t;
      ej.R = sp->R;
      ej.ggt = pj.ggt;
      ej.lam = (double*)(dw + sp->lay.lam);
      ej.vecs = dw + sp->lay.vecs;
      ej.etree = dw + sp->lay.etree;
      ej.estride = sp->estride;
      ej.sweep_out = pj.rank;
      ej.emass = (double*)(dw + sp->emass_off);
      ej.enodes = sp->enodes;
      eig.push_back(ej);
      eprob.push_back(p);
    }
  }
  std::vector<int> pord(P);
  for (int p = 0; p < P; ++p) pord[p] = p;
  std::stable_sort(pord.begin(), pord.end(), [&](int x, int y) {
    return prep_block_threads(prep[x].R) > prep_block_threads(prep[y].R);
  });
  std::vector<PrepJob> prep_sorted;
  for (int p : pord) prep_sorted.push_back(prep[p]);
  std::vector<int> eord(eig.size());
  for (size_t i = 0; i < eig.size(); ++i) eord[i] = (int)i;
  auto ef64 = [&](int i) { return s[eprob[i]]->prec == KRPS_FP64; };
  std::stable_sort(eord.begin(), eord.end(), [&](int x, int y) {
    if (ef64(x) != ef64(y)) return ef64(x);
    return prep_block_threads(eig[x].R) > prep_block_threads(eig[y].R);
  });
  std::vector<EigJob> eig_sorted;
  for (int i : eord) eig_sorted.push_back(eig[i]);
  // first-mode table jobs, grouped by storage type and R class; within a
  // group the units of 16 nodes are numbered job after job
  std::vector<ZtabJob> zt;
  std::vector<int> zprob;
  for (int p = 0; p < P; ++p) {
    krps_sampler sp = s[p];
    if (sp->znmax == 0 || prep[p].nsteps == 0) continue;
    const int k0 = prep[p].gl.order[0];
    char* dw = w + pl.draw_off[p];
    ZtabJob zj;
    memset(&zj, 0, sizeof(zj));
    zj.Z = sp->nodes[k0];
    zj.V = dw + sp->lay.vecs + (size_t)k0 * sp->R * sp->R * sp->elem;
    zj.weights = (double*)(dw + sp->zw_off);
    zj.tab = (double*)(dw + sp->ztab_off);
    zj.nn = sp->shape[k0].n_nodes;
    zj.R = sp->R;
    // a second problem over a tree another job already reads (the
    // exclusions of one sampler whose first drawn mode is the same) rides
    // on that job at R <= 32
    bool paired = false;
    if (zj.R <= 32)
      for (ZtabJob& o : zt)
        if (o.Z == zj.Z && o.tab2 == nullptr) {
          o.V2 = zj.V;
          o.weights2 = zj.weights;
          o.tab2 = zj.tab;
          paired = true;
          break;
        }
    if (paired) continue;
    zt.push_back(zj);
    zprob.push_back(p);
  }
  std::vector<int> zord(zt.size());
  for (size_t i = 0; i < zt.size(); ++i) zord[i] = (int)i;
  auto zkey = [&](int i) {
    return (s[zprob[i]]->prec == KRPS_FP64 ? 0 : 3) + ztab_rclass(zt[i].R);
  };
  std::stable_sort(zord.begin(), zord.end(), [&](int x, int y) { return zkey(x) < zkey(y); });
  std::vector<ZtabJob> zt_sorted;
  std::vector<int64_t> zgroup_units;  // per job: its group's total units
  for (size_t i = 0; i < zord.size();) {
    size_t j = i;
    int64_t u = 0;
    while (j < zord.size() && zkey(zord[j]) == zkey(zord[i])) {
      ZtabJob zj = zt[zord[j]];
      zj.unit0 = u;
      u += (zj.nn + 15) / 16;
      zt_sorted.push_back(zj);
      ++j;
    }
    for (size_t q = i; q < j; ++q) zgroup_units.push_back(u);
    i = j;
  }
  // stage and copy the job descriptors
  std::vector<char> host(pl.probs - pl.prep);
  memcpy(host.data(), prep_sorted.data(), (size_t)P * sizeof(PrepJob));
  if (!eig_sorted.empty())
    memcpy(host.data() + (pl.eig - pl.prep), eig_sorted.data(),
           eig_sorted.size() * sizeof(EigJob));
  if (!zt_sorted.empty())
    memcpy(host.data() + (pl.ztab - pl.prep), zt_sorted.data(),
           zt_sorted.size() * sizeof(ZtabJob));
  st = stage_copy(ctx, 0, host.data(), host.size(), w + pl.prep);
  if (st != KRPS_OK) return st;
  // preparations, grouped by block size
  const PrepJob* dprep = (const PrepJob*)(w + pl.prep);
  for (int i = 0; i < P;) {
    const int bt = prep_block_threads(prep_sorted[i].R);
    int j = i, Rmax = 0;
    while (j < P && prep_block_threads(prep_sorted[j].R) == bt) {
      Rmax = prep_sorted[j].R > Rmax ? prep_sorted[j].R : Rmax;
      ++j;
    }
    hipError_t e = launch_prep_batched(stream, dprep + i, j - i, Rmax);
    if (e != hipSuccess) return hip_fail(e, "batched preparation");
    i = j;
  }
  const EigJob* deig = (const EigJob*)(w + pl.eig);
  const int ne = (int)eig_sorted.size();
  for (int i = 0; i < ne;) {
    const bool f64 = ef64(eord[i]);
    const int bt = prep_block_threads(eig_sorted[i].R);
    int j = i, Rmax = 0;
    while (j < ne && ef64(eord[j]) == f64 && prep_block_threads(eig_sorted[j].R) == bt) {
      Rmax = eig_sorted[j].R > Rmax ? eig_sorted[j].R : Rmax;
      ++j;
    }
    hipError_t e = launch_eig_batched(stream, f64, deig + i, j - i, Rmax);
    if (e != hipSuccess) return hip_fail(e, "batched eigen-trees");
    i = j;
  }
  // first-mode factor-tree mass tables, one launch pair per group
  const ZtabJob* dzt = (const ZtabJob*)(w + pl.ztab);
  for (size_t i = 0; i < zt_sorted.size();) {
    size_t j = i;
    while (j < zt_sorted.size() && zkey(zord[j]) == zkey(zord[i])) ++j;
    const bool f64 = s[zprob[zord[i]]]->prec == KRPS_FP64;
    hipError_t e = launch_ztab_batched(stream, f64, ztab_rclass(zt_sorted[i].R), dzt + i,
                                       (int)(j - i), zgroup_units[i]);
    if (e != hipSuccess) return hip_fail(e, "batched first-mode tables");
    i = j;
  }
  return KRPS_OK;
}

// The walks of a batched draw, from uniform buffers (uniforms != null) or
// from in-kernel Philox under per-problem seed[p] and ctr_base[p].
static krps_status batched_draw(krps_ctx ctx, int P, const krps_sampler* s, const int* exclude,
                                const int64_t* J, const double* const* uniforms,
                                const uint64_t* seed, const uint64_t* ctr_base,
                                int32_t* const* idx, double* const* prob, void* ws,
                                size_t ws_bytes) {
  krps_status st = check_batch(ctx, P, s, exclude);
  if (st != KRPS_OK) return st;
  if (J == nullptr || idx == nullptr) return fail(KRPS_EINVAL, "J/idx is NULL");
  if (uniforms == nullptr && (seed == nullptr || ctr_base == nullptr))
    return fail(KRPS_EINVAL, "neither uniforms nor seed/ctr_base given");
  for (int p = 0; p < P; ++p) {
    if (J[p] < 0) return fail(KRPS_EINVAL, "J < 0");
    if (J[p] > 0 && ((uniforms != nullptr && uniforms[p] == nullptr) || idx[p] == nullptr))
      return fail(KRPS_EINVAL, "uniforms/idx of a problem is NULL");
  }
  if (ws == nullptr) return fail(KRPS_EINVAL, "workspace is NULL");
  const BatchPlan pl = plan_batch(P, s, exclude);
  if (ws_bytes < pl.total) return fail(KRPS_EWORKSPACE, "batched workspace too small");
  char* w = (char*)ws;
  KRPS_HIP(hipSetDevice(ctx->device));
  hipStream_t stream = ctx->stream;
  // walk groups: (storage type, shape class), each one persistent launch,
  // problems in a group by falling cost
  std::vector<double> cost(P);
  for (int p = 0; p < P; ++p) cost[p] = sample_cost(s[p], exclude[p]) * (double)J[p];
  auto group_of = [&](int p) {
    return (s[p]->prec == KRPS_FP64 ? 0 : NBATCH_CLASSES) +
           batch_class(s[p]->R, s[p]->lps ? s[p]->lps : default_lps(s[p]->R, s[p]->prec));
  };
  std::vector<int> ord(P);
  for (int p = 0; p < P; ++p) ord[p] = p;
  std::sort(ord.begin(), ord.end(), [&](int x, int y) {
    const int gx = group_of(x), gy = group_of(y);
    if (gx != gy) return gx < gy;
    return cost[x] > cost[y];
  });
  std::vector<BatchProblem> probs(P);
  constexpr int NG = 2 * NBATCH_CLASSES;
  int64_t task[NG] = {0};
  int nprob[NG] = {0};
  for (int i = 0; i < P; ++i) {
    const int p = ord[i];
    krps_sampler sp = s[p];
    const int g = group_of(p);
    BatchProblem& b = probs[i];
    memset(&b, 0, sizeof(b));
    fill_descent_args(sp, exclude[p], w + pl.draw_off[p], b.a);
    b.a.J = J[p];
    if (uniforms != nullptr) {
      b.a.u01 = uniforms[p];
    } else {
      b.a.u01 = nullptr;
      b.a.seed = seed[p];
      b.a.ctr_base = ctr_base[p];
    }
    b.a.idx = idx[p];
    b.a.prob = prob != nullptr ? prob[p] : nullptr;
    b.tab = (const uint16_t*)(w + pl.tab_off[p]);
    b.cls = batch_class(sp->R, sp->lps ? sp->lps : default_lps(sp->R, sp->prec));
    b.G = batch_group(b.cls);
    b.task0 = task[g];
    task[g] += (J[p] + b.G - 1) / b.G;
    ++nprob[g];
  }
  st = stage_copy(ctx, 1, probs.data(), (size_t)P * sizeof(BatchProblem), w + pl.probs);
  if (st != KRPS_OK) return st;
  unsigned long long* counters = (unsigned long long*)(w + pl.counters);
  hipError_t e = launch_fill_f64(stream, (double*)counters, NG);
  if (e != hipSuccess) return hip_fail(e, "counter clear");
  const BatchProblem* dprobs = (const BatchProblem*)(w + pl.probs);
  int first = 0;
  for (int g = 0; g < NG; ++g) {
    if (nprob[g] > 0) {
      e = launch_descent_batched(stream, g < NBATCH_CLASSES, g % NBATCH_CLASSES, dprobs + first,
                                 nprob[g], task[g], counters + g);
      if (e != hipSuccess) return hip_fail(e, "batched walk");
    }
    first += nprob[g];
  }
  return KRPS_OK;
}

krps_status krps_sample_batched_draw(krps_ctx ctx, int P, const krps_sampler* s,
                                     const int* exclude, const int64_t* J,
                                     const double* const* uniforms, int32_t* const* idx,
                                     double* const* prob, void* ws, size_t ws_bytes) {
  if (uniforms == nullptr) return fail(KRPS_EINVAL, "uniforms is NULL");
  return batched_draw(ctx, P, s, exclude, J, uniforms, nullptr, nullptr, idx, prob, ws, ws_bytes);
}

krps_status krps_sample_batched_seeded(krps_ctx ctx, int P, const krps_sampler* s,
                                       const int* exclude, const int64_t* J,
                                       const uint64_t* seed, const uint64_t* ctr_base,
                                       int32_t* const* idx, double* const* prob, void* ws,
                                       size_t ws_bytes) {
  if (seed == nullptr || ctr_base == nullptr) return fail(KRPS_EINVAL, "seed/ctr_base is NULL");
  krps_status st = krps_sample_batched_prepare(ctx, P, s, exclude, ws, ws_bytes);
  if (st != KRPS_OK) return st;
  return batched_draw(ctx, P, s, exclude, J, nullptr, seed, ctr_base, idx, prob, ws, ws_bytes);
}

krps_status krps_sample_batched(krps_ctx ctx, int P, const krps_sampler* s, const int* exclude,
                                const int64_t* J, const double* const* uniforms,
                                int32_t* const* idx, double* const* prob, void* ws,
                                size_t ws_bytes) {
  if (J == nullptr || uniforms == nullptr || idx == nullptr)
    return fail(KRPS_EINVAL, "J/uniforms/idx is NULL");
  krps_status st = krps_sample_batched_prepare(ctx, P, s, exclude, ws, ws_bytes);
  if (st != KRPS_OK) return st;
  return krps_sample_batched_draw(ctx, P, s, exclude, J, uniforms, idx, prob, ws, ws_bytes);
}

krps_status krps_row_prob(krps_sampler s, int exclude, int64_t M, const int32_t* idx,
                          double* prob, void* ws, size_t ws_bytes) {
  if (s == nullptr) return fail(KRPS_EINVAL, "sampler is NULL");
  if (exclude < -1 || exclude >= s->N) return fail(KRPS_EINVAL, "exclude out of range");
  if (M < 0) return fail(KRPS_EINVAL, "M < 0");
  if (M > 0 && (idx == nullptr || prob == nullptr)) return fail(KRPS_EINVAL, "idx/prob is NULL");
  if (ws == nullptr) return fail(KRPS_EINVAL, "workspace is NULL");
  if (ws_bytes < s->draw_bytes) return fail(KRPS_EWORKSPACE, "draw workspace too small");
  DescentArgs a;
  krps_status st = prepare_draw(s, exclude, ws, a);
  if (st != KRPS_OK) return st;
  a.J = M;
  a.idx = const_cast<int32_t*>(idx);
  a.prob = prob;
  hipError_t e = launch_row_prob(s->ctx->stream, s->prec, a);
  if (e != hipSuccess) return hip_fail(e, "row prob launch");
  return KRPS_OK;
}

krps_status krps_sampler_tree_info(krps_sampler s, int j, krps_tree_info* out) {
  if (s == nullptr || out == nullptr) return fail(KRPS_EINVAL, "sampler/out is NULL");
  if (j < 0 || j >= s->N) return fail(KRPS_EINVAL, "j out of range");
  const TreeShape& t = s->shape[j];
  out->I = t.I;
  out->L = t.L;
  out->F = t.F;
  out->D = t.D;
  out->n_nodes = t.n_nodes;
  out->tri = tri(s->R);
  out->nodes = s->nodes[j];
  out->gram = s->gram[j];
  out->elem_bytes = s->elem;
  return KRPS_OK;
}

krps_status krps_draw_layout_query(krps_sampler s, krps_draw_layout* out) {
  if (s == nullptr || out == nullptr) return fail(KRPS_EINVAL, "sampler/out is NULL");
  *out = s->lay;
  return KRPS_OK;
}

krps_status krps_tensor_workspace_bytes(int N, const int64_t* dims, int64_t nnz, size_t* bytes) {
  krps_status st = check_dims(N, dims, 1);
  if (st != KRPS_OK) return st;
  if (nnz < 1 || nnz > (int64_t)UINT32_MAX) return fail(KRPS_EINVAL, "nnz must be in [1, 2^32)");
  if (bytes == nullptr) return fail(KRPS_EINVAL, "bytes is NULL");
  *bytes = plan_tensor(N, dims, nnz).total;
  return KRPS_OK;
}

krps_status krps_tensor_create(krps_ctx ctx, int N, const int64_t* dims, int64_t nnz,
                               const int32_t* idx, const float* val, void* ws, size_t ws_bytes,
                               krps_tensor* out) {
  if (ctx == nullptr || out == nullptr) return fail(KRPS_EINVAL, "ctx/out is NULL");
  krps_status st = check_dims(N, dims, 1);
  if (st != KRPS_OK) return st;
  if (nnz < 1 || nnz > (int64_t)UINT32_MAX) return fail(KRPS_EINVAL, "nnz must be in [1, 2^32)");
  if (idx == nullptr || val == nullptr || ws == nullptr)
    return fail(KRPS_EINVAL, "idx/val/workspace is NULL");
  TensorPlan pl = plan_tensor(N, dims, nnz);
  if (ws_bytes < pl.total) return fail(KRPS_EWORKSPACE, "tensor workspace too small");
  krps_tensor t = new (std::nothrow) krps_tensor_s;
  if (t == nullptr) return fail(KRPS_EINVAL, "out of host memory");
  t->ctx = ctx;
  t->N = N;
  t->nnz = nnz;
  char* w = (char*)ws;
  for (int j = 0; j < N; ++j) {
    t->dims.push_back(dims[j]);
    t->cols.push_back((int32_t*)(w + pl.cols_off[j]));
    t->vals.push_back((double*)(w + pl.vals_off[j]));
    t->off.push_back((int64_t*)(w + pl.off_off[j]));
    t->lead.push_back(pl.lead[j]);
  }
  hipStream_t s = ctx->stream;
  for (int j = 0; j < N; ++j) {
    hipError_t e = build_fiber_index(s, N, dims, nnz, idx, val, j, t->cols[j], t->vals[j],
                                     t->off[j], (uint32_t*)(w + pl.k0), (uint32_t*)(w + pl.k1),
                                     (uint32_t*)(w + pl.p0), (uint32_t*)(w + pl.p1), w + pl.temp,
                                     pl.temp_bytes, &t->nu);
    if (e != hipSuccess) {
      delete t;
      return hip_fail(e, "fiber index build");
    }
  }
  // hot rows of each mode: the i_j column of mode j's merged copy
  const int nhot = (int)std::min<int64_t>(pl.nhot, 1 << 20);
  t->nhot = nhot;
  for (int j = 0; j < N; ++j) {
    t->hot_slot.push_back((int16_t*)(w + pl.hslot_off[j]));
    t->hot_rows.push_back((int32_t*)(w + pl.hrows_off[j]));
    const int nh = (int)std::min<int64_t>(nhot, dims[j]);
    hipError_t e = build_hot_rows(s, t->cols[j] + (int64_t)j * t->nu, t->nu, dims[j], nh,
                                  (uint32_t*)(w + pl.hc0), (uint32_t*)(w + pl.hc1),
                                  (uint32_t*)(w + pl.hi0), (uint32_t*)(w + pl.hi1), w + pl.temp,
                                  pl.temp_bytes, t->hot_rows[j], t->hot_slot[j]);
    if (e != hipSuccess) {
      delete t;
      return hip_fail(e, "hot rows");
    }
  }
  double* acc = (double*)(w + pl.acc);
  hipError_t e = launch_norm2(s, t->vals[0], t->nu, acc);
  if (e == hipSuccess) e = hipMemcpyAsync(&t->norm2, acc, 8, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    delete t;
    return hip_fail(e, "tensor norm");
  }
  *out = t;
  return KRPS_OK;
}

krps_status krps_tensor_destroy(krps_tensor t) {
  delete t;
  return KRPS_OK;
}

krps_status krps_tensor_stored_entries(krps_tensor t, int64_t* out) {
  if (t == nullptr || out == nullptr) return fail(KRPS_EINVAL, "tensor/out is NULL");
  *out = t->nu;
  return KRPS_OK;
}

krps_status krps_tensor_hot_rows(krps_tensor t, int j, int32_t* rows, int* n) {
  if (t == nullptr || rows == nullptr || n == nullptr) return fail(KRPS_EINVAL, "NULL argument");
  if (j < 0 || j >= t->N) return fail(KRPS_EINVAL, "j out of range");
  const int nh = (int)std::min<int64_t>(t->nhot, t->dims[j]);
  KRPS_HIP(hipSetDevice(t->ctx->device));
  KRPS_HIP(hipMemcpyAsync(rows, t->hot_rows[j], (size_t)nh * 4, hipMemcpyDeviceToHost,
                          t->ctx->stream));
  KRPS_HIP(hipStreamSynchronize(t->ctx->stream));
  *n = nh;
  return KRPS_OK;
}

krps_status krps_tensor_norm2(krps_tensor t, double* out) {
  if (t == nullptr || out == nullptr) return fail(KRPS_EINVAL, "tensor/out is NULL");
  *out = t->norm2;
  return KRPS_OK;
}

krps_status krps_solve_workspace_bytes(krps_sampler s, krps_tensor t, int64_t J, size_t* bytes) {
  krps_status st = check_pair(s, t);
  if (st != KRPS_OK) return st;
  if (J < 1) return fail(KRPS_EINVAL, "J must be >= 1");
  if (bytes == nullptr) return fail(KRPS_EINVAL, "bytes is NULL");
  *bytes = plan_solve(s, J).total;
  return KRPS_OK;
}

krps_status krps_solve_layout_query(krps_sampler s, krps_tensor t, int64_t J,
                                    krps_solve_layout* out) {
  krps_status st = check_pair(s, t);
  if (st != KRPS_OK) return st;
  if (J < 1 || out == nullptr) return fail(KRPS_EINVAL, "J < 1 or out is NULL");
  *out = plan_solve(s, J).lay;
  return KRPS_OK;
}

krps_status krps_normalize_factor(krps_sampler s, int j, double* sigma, void* ws, size_t ws_bytes) {
  if (s == nullptr) return fail(KRPS_EINVAL, "sampler is NULL");
  if (j < 0 || j >= s->N) return fail(KRPS_EINVAL, "j out of range");
  const SolveHead h = plan_head(s);
  if (ws == nullptr || ws_bytes < h.total) return fail(KRPS_EWORKSPACE, "workspace too small");
  double* partial = (double*)((char*)ws + h.npart);
  double* sg = sigma != nullptr ? sigma : (double*)((char*)ws + h.nsig);
  hipStream_t st = s->ctx->stream;
  hipError_t e = launch_colnorm(st, s->prec, s->U[j], s->I[j], s->R, partial, sg);
  if (e == hipSuccess) e = launch_normalize(st, s->prec, s->U[j], s->I[j], s->R, sg);
  if (e != hipSuccess) return hip_fail(e, "normalise factor");
  return build_tree(s, j);
}

krps_status krps_sketched_solve(krps_sampler s, krps_tensor t, int j, int64_t J,
                                const double* uniforms, double* sigma, void* ws, size_t ws_bytes) {
  if (uniforms == nullptr) return fail(KRPS_EINVAL, "uniforms is NULL");
  UniformSrc us;
  us.u01 = uniforms;
  return solve_entry(s, t, j, J, us, sigma, ws, ws_bytes);
}

krps_status krps_sketched_solve_seeded(krps_sampler s, krps_tensor t, int j, int64_t J,
                                       uint64_t seed, uint64_t ctr_base, uint64_t sweep,
                                       double* sigma, void* ws, size_t ws_bytes) {
  if (s == nullptr) return fail(KRPS_EINVAL, "sampler is NULL");
  UniformSrc us;
  us.seed = seed;
  us.ctr_base = ctr_base;
  us.ctr2 = sweep * (uint64_t)s->N + (uint64_t)j;
  return solve_entry(s, t, j, J, us, sigma, ws, ws_bytes);
}

krps_status krps_als_sweep(krps_sampler s, krps_tensor t, int64_t J, const double* uniforms,
                           double* sigma, void* ws, size_t ws_bytes, int use_graph) {
  if (uniforms == nullptr) return fail(KRPS_EINVAL, "uniforms is NULL");
  return sweep_entry(s, t, J, uniforms, 0, 0, 0, sigma, ws, ws_bytes, use_graph);
}

krps_status krps_als_sweep_seeded(krps_sampler s, krps_tensor t, int64_t J, uint64_t seed,
                                  uint64_t ctr_base, uint64_t sweep, double* sigma, void* ws,
                                  size_t ws_bytes, int use_graph) {
  return sweep_entry(s, t, J, nullptr, seed, ctr_base, sweep, sigma, ws, ws_bytes, use_graph);
}

}  // extern "C"

namespace {

struct LsPlan {
  size_t SA, SBw, M, Mp, rank, partial, Z, scratch, scratch_bytes, total;
};

LsPlan plan_lstsq(int R, int64_t J, int64_t n) {
  LsPlan pl;
  size_t off = 0;
  pl.SA = off;
  off += align_up((size_t)J * R * 8);
  pl.SBw = off;
  off += align_up((size_t)J * n * 8);
  pl.M = off;
  off += align_up((size_t)R * R * 8);
  pl.Mp = off;
  off += align_up((size_t)R * R * 8);
  pl.rank = off;
  off += 256;
  pl.partial = off;
  off += align_up(lstsq_partial_bytes(R, n));
  pl.Z = off;
  off += align_up((size_t)R * n * 8);
  TreeShape tm;
  tm.init(J, R);
  pl.scratch = off;
  pl.scratch_bytes = tree_build_scratch_bytes(tm.L, R);
  off += align_up(pl.scratch_bytes);
  pl.total = off;
  return pl;
}

}  // namespace

extern "C" {

krps_status krps_lstsq_workspace_bytes(int R, int64_t J, int64_t n, size_t* bytes) {
  if (R < 1 || R > KRPS_MAX_R) return fail(KRPS_EINVAL, "R outside [1, 128]");
  if (J < 1 || n < 1) return fail(KRPS_EINVAL, "J and n must be >= 1");
  if (bytes == nullptr) return fail(KRPS_EINVAL, "bytes is NULL");
  *bytes = plan_lstsq(R, J, n).total;
  return KRPS_OK;
}

krps_status krps_sketched_lstsq(krps_ctx ctx, int R, int64_t J, const void* rows,
                                const double* prob, int64_t n, const void* SB_rows, double* X,
                                krps_precision p, void* ws, size_t ws_bytes) {
  if (ctx == nullptr) return fail(KRPS_EINVAL, "ctx is NULL");
  if (!valid_prec(p)) return fail(KRPS_EINVAL, "unknown precision");
  if (R < 1 || R > KRPS_MAX_R) return fail(KRPS_EINVAL, "R outside [1, 128]");
  if (J < 1 || n < 1) return fail(KRPS_EINVAL, "J and n must be >= 1");
  if (rows == nullptr || prob == nullptr || SB_rows == nullptr || X == nullptr || ws == nullptr)
    return fail(KRPS_EINVAL, "rows/prob/SB_rows/X/workspace is NULL");
  const LsPlan pl = plan_lstsq(R, J, n);
  if (ws_bytes < pl.total) return fail(KRPS_EWORKSPACE, "least-squares workspace too small");
  KRPS_HIP(hipSetDevice(ctx->device));
  hipStream_t st = ctx->stream;
  char* w = (char*)ws;
  double* SA = (double*)(w + pl.SA);
  double* SBw = (double*)(w + pl.SBw);
  hipError_t e = launch_ls_scale(st, p, rows, SB_rows, prob, J, R, n, SA, SBw);
  if (e != hipSuccess) return hip_fail(e, "row scaling");
  TreeShape tm;
  tm.init(J, R);
  e = launch_tree_build(st, KRPS_FP64, SA, J, R, tm, nullptr, (double*)(w + pl.M),
                        (double*)(w + pl.scratch), pl.scratch_bytes);
  if (e != hipSuccess) return hip_fail(e, "Gram of sampled rows");
  e = launch_pinv(st, R, (double*)(w + pl.M), (double*)(w + pl.Mp), (int32_t*)(w + pl.rank));
  if (e != hipSuccess) return hip_fail(e, "pseudo-inverse");
  e = launch_ls_solve(st, SA, SBw, J, R, n, (const double*)(w + pl.Mp), (double*)(w + pl.partial),
                      (double*)(w + pl.Z), X);
  if (e != hipSuccess) return hip_fail(e, "solve");
  return KRPS_OK;
}

}  // extern "C"

namespace {

struct TunePlan {
  size_t sampler, draw, idx, prob, total;
  int Fmin;
};

TunePlan plan_tune(int N, const int64_t* I, int R, krps_precision p, int64_t J) {
  TunePlan pl;
  pl.Fmin = R / 2 > 0 ? R / 2 : 1;
  size_t off = 0;
  pl.sampler = off;
  const SamplerPlan sp = plan_sampler(N, I, R, pl.Fmin, p);
  off += align_up(sp.total);
  // the smallest leaf size tried has the most nodes, so the largest
  // first-mode table
  krps_sampler_s tmp;
  tmp.N = N;
  tmp.R = R;
  tmp.elem = elem_bytes(p);
  tmp.shape = sp.shape;
  plan_draw(&tmp);
  pl.draw = off;
  off += align_up(tmp.draw_bytes);
  pl.idx = off;
  off += align_up((size_t)J * N * 4);
  pl.prob = off;
  off += align_up((size_t)J * 8);
  pl.total = off;
  return pl;
}

std::string tune_key(int N, const int64_t* I, int R, krps_precision p, int64_t J) {
  std::string k = "gfx950 p=" + std::to_string((int)p) + " R=" + std::to_string(R) +
                  " J=" + std::to_string(J) + " I=";
  for (int j = 0; j < N; ++j) k += (j ? "," : "") + std::to_string(I[j]);
  return k;
}

// One line per entry: {"key": "...", "F": f, "lps": l, "team": w, "build_ms": b,
// "draw_ms": d} (entries without "team" used the default team).  Entries
// whose shapes this library does not offer for R and p (a cache written
// by another version) are skipped.
bool tune_lookup(const char* path, const std::string& key, int R, krps_precision p,
                 krps_tune* out) {
  if (path == nullptr) return false;
  FILE* f = fopen(path, "r");
  if (f == nullptr) return false;
  char line[1024];
  bool found = false;
  const std::string pat = "\"key\": \"" + key + "\"";
  while (fgets(line, sizeof(line), f) != nullptr) {
    const char* at = strstr(line, pat.c_str());
    if (at == nullptr) continue;
    const char* q = strstr(line, "\"F\": ");
    const char* l = strstr(line, "\"lps\": ");
    const char* tw = strstr(line, "\"team\": ");
    const char* b = strstr(line, "\"build_ms\": ");
    const char* d = strstr(line, "\"draw_ms\": ");
    if (q && l && b && d) {
      const int F = atoi(q + 5), lps = atoi(l + 7), team = tw ? atoi(tw + 8) : 0;
      const std::vector<int> teams = build_team_choices(R, p);
      const bool ok = F >= 1 && lps_supported(R, lps) &&
                      (team == 0 || std::find(teams.begin(), teams.end(), team) != teams.end());
      if (!ok) continue;
      out->F = F;
      out->lps = lps;
      out->team = team;
      out->build_ms = atof(b + 12);
      out->draw_ms = atof(d + 11);
      out->from_cache = 1;
      found = true;  // the last entry for a key wins
    }
  }
  fclose(f);
  return found;
}

void tune_store(const char* path, const std::string& key, const krps_tune& t) {
  if (path == nullptr) return;
  FILE* f = fopen(path, "a");
  if (f == nullptr) return;
  fprintf(f,
          "{\"key\": \"%s\", \"F\": %d, \"lps\": %d, \"team\": %d, \"build_ms\": %.6f, "
          "\"draw_ms\": %.6f}\n",
          key.c_str(), t.F, t.lps, t.team, t.build_ms, t.draw_ms);
  fclose(f);
}

}  // namespace

extern "C" {

krps_status krps_autotune_workspace_bytes(int N, const int64_t* I, int R, krps_precision p,
                                          int64_t J, size_t* bytes) {
  krps_status st = check_dims(N, I, R);
  if (st != KRPS_OK) return st;
  if (!valid_prec(p)) return fail(KRPS_EINVAL, "unknown precision");
  if (J < 1) return fail(KRPS_EINVAL, "J must be >= 1");
  if (bytes == nullptr) return fail(KRPS_EINVAL, "bytes is NULL");
  *bytes = plan_tune(N, I, R, p, J).total;
  return KRPS_OK;
}

krps_status krps_autotune(krps_ctx ctx, int N, const int64_t* I, int R, krps_precision p,
                          void* const* U, int64_t J, const double* uniforms, void* ws,
                          size_t ws_bytes, const char* cache_path, krps_tune* out) {
  if (ctx == nullptr || out == nullptr) return fail(KRPS_EINVAL, "ctx/out is NULL");
  krps_status st = check_dims(N, I, R);
  if (st != KRPS_OK) return st;
  if (!valid_prec(p)) return fail(KRPS_EINVAL, "unknown precision");
  if (J < 1 || uniforms == nullptr || U == nullptr || ws == nullptr)
    return fail(KRPS_EINVAL, "J/uniforms/U/workspace invalid");
  const std::string key = tune_key(N, I, R, p, J);
  memset(out, 0, sizeof(*out));
  if (tune_lookup(cache_path, key, R, p, out)) return KRPS_OK;
  const TunePlan pl = plan_tune(N, I, R, p, J);
  if (ws_bytes < pl.total) return fail(KRPS_EWORKSPACE, "autotune workspace too small");
  char* w = (char*)ws;
  KRPS_HIP(hipSetDevice(ctx->device));
  hipEvent_t ev[3];
  for (int i = 0; i < 3; ++i) KRPS_HIP(hipEventCreate(&ev[i]));
  std::vector<int> Fs;
  for (int f : {pl.Fmin, R, 2 * R, 4 * R})
    if (std::find(Fs.begin(), Fs.end(), f) == Fs.end()) Fs.push_back(f);
  double best = 1e300;
  krps_status result = KRPS_OK;
  for (int F : Fs) {
    krps_sampler s = nullptr;
    result = krps_sampler_create(ctx, N, I, R, F, U, p, w + pl.sampler, pl.draw - pl.sampler, &s);
    if (result != KRPS_OK) break;
    for (int lps : lps_choices(R))
    for (int team : build_team_choices(R, p)) {
      s->lps = lps;
      s->team = team;
      float bmin = 1e30f, dmin = 1e30f;
      for (int rep = 0; rep < 4 && result == KRPS_OK; ++rep) {
        hipError_t e = hipEventRecord(ev[0], ctx->stream);
        for (int j = 0; j < N && e == hipSuccess; ++j)
          if (build_tree(s, j) != KRPS_OK) e = hipErrorUnknown;
        if (e == hipSuccess) e = hipEventRecord(ev[1], ctx->stream);
        if (e != hipSuccess) {
          result = hip_fail(e, "autotune build");
          break;
        }
        result = krps_sample(s, -1, J, uniforms, (int32_t*)(w + pl.idx), (double*)(w + pl.prob),
                             nullptr, w + pl.draw, pl.idx - pl.draw, 0);
        if (result != KRPS_OK) break;
        e = hipEventRecord(ev[2], ctx->stream);
        if (e == hipSuccess) e = hipEventSynchronize(ev[2]);
        float b = 0, d = 0;
        if (e == hipSuccess) e = hipEventElapsedTime(&b, ev[0], ev[1]);
        if (e == hipSuccess) e = hipEventElapsedTime(&d, ev[1], ev[2]);
        if (e != hipSuccess) {
          result = hip_fail(e, "autotune timing");
          break;
        }
        if (rep > 0) {  // the first repetition warms up
          bmin = b < bmin ? b : bmin;
          dmin = d < dmin ? d : dmin;
        }
      }
      if (result != KRPS_OK) break;
      if (bmin + dmin < best) {
        best = bmin + dmin;
        out->F = F;
        out->lps = lps;
        out->team = team;
        out->build_ms = bmin;
        out->draw_ms = dmin;
      }
    }
    krps_sampler_destroy(s);
    if (result != KRPS_OK) break;
  }
  for (int i = 0; i < 3; ++i) (void)hipEventDestroy(ev[i]);
  if (result != KRPS_OK) return result;
  out->from_cache = 0;
  tune_store(cache_path, key, *out);
  return KRPS_OK;
}

krps_status krps_init_range_finder(krps_sampler s, krps_tensor t, int j, uint64_t seed,
                                   double* sigma, void* ws, size_t ws_bytes) {
  krps_status st = check_pair(s, t);
  if (st != KRPS_OK) return st;
  if (j < 0 || j >= s->N) return fail(KRPS_EINVAL, "j out of range");
  if (s->N > 5) return fail(KRPS_EUNSUPPORTED, "range finder supports at most 5 modes");
  if (ws == nullptr) return fail(KRPS_EINVAL, "workspace is NULL");
  SolvePlan pl = plan_solve(s, 1);
  if (ws_bytes < pl.total) return fail(KRPS_EWORKSPACE, "workspace too small");
  char* w = (char*)ws;
  hipError_t e = launch_range_finder(s->ctx->stream, s->prec, t->cols[j], t->vals[j], t->nu, s->N,
                                     j, s->R, seed, s->I[j], (double*)(w + pl.lay.Y), s->U[j]);
  if (e != hipSuccess) return hip_fail(e, "range finder");
  return krps_normalize_factor(s, j, sigma, ws, ws_bytes);
}

krps_status krps_exact_solve(krps_sampler s, krps_tensor t, int j, double* sigma, void* ws,
                             size_t ws_bytes) {
  krps_status st = check_pair(s, t);
  if (st != KRPS_OK) return st;
  if (s->N < 2) return fail(KRPS_EINVAL, "a solve needs N >= 2");
  if (j < 0 || j >= s->N) return fail(KRPS_EINVAL, "j out of range");
  if (sigma == nullptr || ws == nullptr) return fail(KRPS_EINVAL, "sigma/workspace is NULL");
  const SolvePlan pl = plan_solve(s, 1);
  if (ws_bytes < pl.total) return fail(KRPS_EWORKSPACE, "solve workspace too small");
  KRPS_HIP(hipSetDevice(s->ctx->device));
  const int R = s->R, N = s->N;
  char* w = (char*)ws;
  hipStream_t stream = s->ctx->stream;
  const krps_solve_layout& l = pl.lay;
  const SolveHead& h = pl.head;
  // M = (*)_{k != j} G_k in float64 and M^+
  const double* mats[KRPS_MAX_MODES];
  int nm = 0;
  for (int k = 0; k < N; ++k)
    if (k != j) mats[nm++] = s->gram[k];
  hipError_t e = launch_prep_gplus2(stream, R, nm, mats, 0, nullptr, (double*)(w + l.Mp), nullptr,
                                    (int32_t*)(w + pl.rank), nullptr, s->status);
  if (e != hipSuccess) return hip_fail(e, "pseudo-inverse of the Hadamard product of Grams");
  MttkrpArgs a;
  memset(&a, 0, sizeof(a));
  a.N = N;
  a.j = j;
  a.R = R;
  a.nnz = t->nu;
  a.cols = t->cols[j];
  a.vals = t->vals[j];
  for (int k = 0; k < N; ++k) a.U[k] = s->U[k];
  a.hot_slot = t->hot_slot[j];
  a.hot_rows = t->hot_rows[j];
  a.nhot = (int)std::min<int64_t>(t->nhot, t->dims[j]);
  int32_t* list = (int32_t*)(w + l.yrows);
  int64_t* count = (int64_t*)(w + l.nyrows);
  e = launch_mttkrp(stream, s->prec, a, s->I[j], (int32_t*)(w + pl.ymark),
                    (int64_t*)(w + pl.ybsum), list, count, (double*)(w + l.Y));
  if (e != hipSuccess) return hip_fail(e, "MTTKRP");
  e = launch_solve_gemm(stream, s->prec == KRPS_FP64 ? KRPS_FP64 : KRPS_FP32, w + l.Y,
                        (const double*)(w + l.Mp), s->U[j], s->I[j], list, count, R,
                        (double*)(w + pl.partial), sigma);
  if (e != hipSuccess) return hip_fail(e, "solve GEMM");
  return build_tree(s, j);
}

krps_status krps_fit(krps_sampler s, krps_tensor t, const double* sigma, double* fit, void* ws,
                     size_t ws_bytes) {
  krps_status st = check_pair(s, t);
  if (st != KRPS_OK) return st;
  if (sigma == nullptr || fit == nullptr || ws == nullptr)
    return fail(KRPS_EINVAL, "sigma/fit/workspace is NULL");
  const int R = s->R, N = s->N;
  // The Grams G_k are float64 in every precision (the split path's too),
  // so ||T~||^2 = sigma^T ((*) G_k) sigma carries no bf16 rounding, which
  // ||T~||^2 - 2 <T, T~> would amplify by ~1 / (1 - fit)^2.  The fit's
  // scratch lies in the head of the solve workspace, below the pieces of
  // krps_solve_layout.
  const SolveHead h = plan_head(s);
  if (ws_bytes < h.total) return fail(KRPS_EWORKSPACE, "workspace too small for the fit");
  char* w = (char*)ws;
  hipStream_t stream = s->ctx->stream;
  FitArgs fa;
  memset(&fa, 0, sizeof(fa));
  fa.N = N;
  fa.R = R;
  fa.nnz = t->nu;
  fa.cols = t->cols[0];
  fa.vals = t->vals[0];
  for (int k = 0; k < N; ++k) {
    fa.U[k] = s->U[k];
    fa.G[k] = s->gram[k];
  }
  fa.sigma = sigma;
  double* partial = (double*)(w + h.fitp);
  double* out = (double*)(w + h.fitout);
  hipError_t e = launch_fit(stream, s->prec, fa, partial, out);
  if (e != hipSuccess) return hip_fail(e, "fit");
  double res[2];
  KRPS_HIP(hipMemcpyAsync(res, out, 16, hipMemcpyDeviceToHost, s->ctx->stream));
  KRPS_HIP(hipStreamSynchronize(s->ctx->stream));
  const double r2 = t->norm2 + res[1] - 2.0 * res[0];
  *fit = 1.0 - sqrt(r2 > 0 ? r2 : 0.0) / sqrt(t->norm2);
  return KRPS_OK;
}

}  // extern "C"

// ------------------------------------------------------ workspace regions

namespace {

struct RegionList {
  krps_region* out;
  int cap, n = 0;
  void add(int ws, const char* name, size_t off, size_t bytes, size_t need) {
    if (n < cap && out != nullptr) {
      krps_region& r = out[n];
      memset(&r, 0, sizeof(r));
      r.workspace = ws;
      snprintf(r.name, sizeof(r.name), "%s", name);
      r.offset = off;
      r.bytes = bytes;
      r.need = need;
    }
    ++n;
  }
};

// Bytes from `off` to the next region's start in an ordered list of offsets.
size_t span(size_t off, size_t next) { return next - off; }

}  // namespace

extern "C" {

krps_status krps_workspace_regions(int N, const int64_t* I, int R, int F, krps_precision p,
                                   int64_t nnz, int64_t J, krps_region* out, int cap, int* count) {
  krps_status st = check_dims(N, I, R);
  if (st != KRPS_OK) return st;
  if (!valid_prec(p)) return fail(KRPS_EINVAL, "unknown precision");
  if (F < 0 || nnz < 1 || J < 1 || count == nullptr || cap < 0)
    return fail(KRPS_EINVAL, "F < 0, nnz < 1, J < 1, cap < 0 or count NULL");
  const int Fe = F == 0 ? R : F;
  const int64_t TR = tri(R);
  const size_t es = (size_t)elem_bytes(p);
  // the longest read past a node's end: a lane group of at most 64 lanes
  // reading a node in strides of its width
  const size_t overread = 63;
  RegionList rl{out, cap};
  // --- sampler workspace
  const SamplerPlan sp = plan_sampler(N, I, R, Fe, p);
  for (int j = 0; j < N; ++j) {
    char nm[32];
    snprintf(nm, sizeof(nm), "tree %d", j);
    const size_t nend = p == KRPS_FP64 ? sp.node32_off[j] : sp.gram_off[j];
    rl.add(0, nm, sp.node_off[j], span(sp.node_off[j], nend),
           (size_t)(sp.shape[j].n_nodes * TR + overread) * es);
    if (p == KRPS_FP64) {
      snprintf(nm, sizeof(nm), "tree %d float32 copy", j);
      rl.add(0, nm, sp.node32_off[j], span(sp.node32_off[j], sp.gram_off[j]),
             (size_t)(sp.shape[j].n_nodes * TR + overread) * 4);
    }
    snprintf(nm, sizeof(nm), "gram %d", j);
    const size_t gnext = j + 1 < N ? sp.node_off[j + 1] : sp.scratch_off;
    rl.add(0, nm, sp.gram_off[j], span(sp.gram_off[j], gnext), (size_t)R * R * 8);
  }
  size_t bext = 0;
  for (int j = 0; j < N; ++j) bext = std::max(bext, tree_build_scratch_extent(sp.shape[j], R));
  rl.add(0, "build scratch", sp.scratch_off, span(sp.scratch_off, sp.status_off), bext);
  rl.add(0, "status", sp.status_off, span(sp.status_off, sp.warm_ok_off), 12);
  rl.add(0, "warm-start flags", sp.warm_ok_off, span(sp.warm_ok_off, sp.warm_off),
         (size_t)(N + 1) * N * 4);
  rl.add(0, "warm-start vectors", sp.warm_off, span(sp.warm_off, sp.total),
         (size_t)(N + 1) * N * R * R * 8);
  // --- per-draw workspace (a host-side sampler with the same shape)
  krps_sampler_s tmp;
  tmp.N = N;
  tmp.R = R;
  tmp.F = Fe;
  tmp.prec = p;
  tmp.elem = (int)es;
  for (int j = 0; j < N; ++j) {
    tmp.I.push_back(I[j]);
    tmp.shape.push_back(sp.shape[j]);
  }
  plan_draw(&tmp);
  const krps_draw_layout& dl = tmp.lay;
  const size_t gpk = gpacked_off(&tmp);
  rl.add(1, "G+", dl.gplus, span(dl.gplus, gpk), (size_t)R * R * 8);
  rl.add(1, "G+ packed", gpk, span(gpk, dl.rank), (size_t)(TR + overread) * 8);
  rl.add(1, "rank, sweeps", dl.rank, span(dl.rank, dl.ggt), (size_t)(2 + N) * 4);
  rl.add(1, "G>k", dl.ggt, span(dl.ggt, dl.lam), (size_t)N * R * R * 8);
  rl.add(1, "eigenvalues", dl.lam, span(dl.lam, dl.vecs), (size_t)N * R * 8);
  rl.add(1, "eigenvectors", dl.vecs, span(dl.vecs, dl.etree), (size_t)N * R * R * es);
  rl.add(1, "eigen-trees", dl.etree, span(dl.etree, tmp.emass_off),
         (size_t)((N - 1) * tmp.estride + tmp.enodes * TR + overread) * es);
  rl.add(1, "eigen masses", tmp.emass_off, span(tmp.emass_off, tmp.ztab_off),
         (size_t)N * tmp.enodes * 8);
  rl.add(1, "first-mode table", tmp.ztab_off, span(tmp.ztab_off, tmp.zw_off),
         (size_t)R * tmp.znmax * 8);
  rl.add(1, "table weights", tmp.zw_off, span(tmp.zw_off, tmp.draw_bytes),
         tmp.znmax > 0 ? ztab_weights_bytes(R) : 0);
  // --- solve workspace
  const SolvePlan pl = plan_solve(&tmp, J);
  const SolveHead& h = pl.head;
  const krps_solve_layout& l = pl.lay;
  rl.add(2, "fit partials", h.fitp, span(h.fitp, h.fitout), fit_partial_bytes());
  rl.add(2, "fit result", h.fitout, span(h.fitout, h.npart), 16);
  rl.add(2, "norm partials", h.npart, span(h.npart, h.nsig), solve_partial_bytes(R));
  rl.add(2, "norm sigma", h.nsig, span(h.nsig, h.ctrw), (size_t)R * 8);
  rl.add(2, "sweep counter", h.ctrw, span(h.ctrw, l.draw), 8);
  rl.add(2, "draw", l.draw, span(l.draw, l.idx), tmp.draw_bytes);
  rl.add(2, "idx", l.idx, span(l.idx, l.prob), (size_t)J * N * 4);
  rl.add(2, "prob", l.prob, span(l.prob, l.w), (size_t)J * 8);
  rl.add(2, "w", l.w, span(l.w, l.rows), (size_t)J * 8);
  rl.add(2, "rows", l.rows, span(l.rows, pl.lo), (size_t)J * R * (p == KRPS_BF16X2 ? 4 : 8));
  rl.add(2, "fiber lo", pl.lo, span(pl.lo, pl.hi), (size_t)J * 8);
  rl.add(2, "fiber hi", pl.hi, span(pl.hi, pl.cnt), (size_t)J * 8);
  rl.add(2, "items", pl.cnt, span(pl.cnt, pl.start), (size_t)J * 8);
  rl.add(2, "item starts", pl.start, span(pl.start, pl.coef), (size_t)(J + 1) * 8);
  rl.add(2, "coef", pl.coef, span(pl.coef, pl.slot), (size_t)J * 8);
  rl.add(2, "slot", pl.slot, span(pl.slot, pl.hkey), (size_t)J * 4);
  rl.add(2, "hash keys", pl.hkey, span(pl.hkey, pl.hW), (size_t)pl.H * 8);
  rl.add(2, "hash weights", pl.hW, span(pl.hW, pl.hWlo), (size_t)pl.H * 8);
  rl.add(2, "hash weights, low words", pl.hWlo, span(pl.hWlo, pl.hrep), (size_t)pl.H * 8);
  rl.add(2, "hash reps", pl.hrep, span(pl.hrep, pl.rflag), (size_t)pl.H * 4);
  rl.add(2, "expand flags", pl.rflag, span(pl.rflag, pl.rpos), (size_t)J * 8);
  rl.add(2, "expand pos", pl.rpos, span(pl.rpos, pl.rep), (size_t)(J + 1) * 8);
  rl.add(2, "expanding", pl.rep, span(pl.rep, pl.rstart), (size_t)J * 4);
  rl.add(2, "expand starts", pl.rstart, span(pl.rstart, pl.bsum), (size_t)(J + 1) * 8);
  rl.add(2, "scan tiles", pl.bsum, span(pl.bsum, l.M), (size_t)((J + 1023) / 1024 + 2) * 8);
  rl.add(2, "M", l.M, span(l.M, l.Mp), (size_t)R * R * 8);
  rl.add(2, "M+", l.Mp, span(l.Mp, pl.rank), (size_t)R * R * 8);
  rl.add(2, "M rank", pl.rank, span(pl.rank, l.Y), 8);
  rl.add(2, "Y", l.Y, span(l.Y, l.yrows), (size_t)pl.Imax * R * (p == KRPS_BF16X2 ? 4 : 8));
  rl.add(2, "Y rows", l.yrows, span(l.yrows, l.nyrows), (size_t)pl.Imax * 4);
  rl.add(2, "Y row count", l.nyrows, span(l.nyrows, l.expanded), 8);
  rl.add(2, "expanded entries", l.expanded, span(l.expanded, pl.ymark), 8);
  rl.add(2, "row marks", pl.ymark, span(pl.ymark, pl.ybsum), (size_t)pl.Imax * 4);
  rl.add(2, "row scan", pl.ybsum, span(pl.ybsum, pl.partial), row_bsum_bytes(pl.Imax));
  rl.add(2, "solve partials", pl.partial, span(pl.partial, pl.det), solve_partial_bytes(R));
  rl.add(2, "fixed-point bound", pl.det, span(pl.det, pl.gscratch), spmm_det_bytes());
  TreeShape tm;
  tm.init(J, R);
  rl.add(2, "M scratch", pl.gscratch, span(pl.gscratch, pl.total),
         tree_build_scratch_extent(tm, R));
  // --- tensor workspace (dims = I)
  if (nnz <= (int64_t)UINT32_MAX) {
    const TensorPlan tp = plan_tensor(N, I, nnz);
    for (int j = 0; j < N; ++j) {
      char nm[32];
      snprintf(nm, sizeof(nm), "cols %d", j);
      rl.add(3, nm, tp.cols_off[j], span(tp.cols_off[j], tp.vals_off[j]), (size_t)N * nnz * 4);
      snprintf(nm, sizeof(nm), "vals %d", j);
      rl.add(3, nm, tp.vals_off[j], span(tp.vals_off[j], tp.off_off[j]), (size_t)nnz * 8);
      snprintf(nm, sizeof(nm), "offsets %d", j);
      const size_t onext = j + 1 < N ? tp.cols_off[j + 1] : tp.k0;
      rl.add(3, nm, tp.off_off[j], span(tp.off_off[j], onext), (size_t)(I[tp.lead[j]] + 1) * 8);
    }
    rl.add(3, "keys 0", tp.k0, span(tp.k0, tp.k1), (size_t)nnz * 4);
    rl.add(3, "keys 1", tp.k1, span(tp.k1, tp.p0), (size_t)nnz * 4);
    rl.add(3, "perm 0", tp.p0, span(tp.p0, tp.p1), (size_t)nnz * 4);
    rl.add(3, "perm 1", tp.p1, span(tp.p1, tp.hslot_off[0]), (size_t)nnz * 4);
    int64_t dmax = 1;
    for (int j = 0; j < N; ++j) {
      dmax = std::max<int64_t>(dmax, I[j]);
      char nm[32];
      snprintf(nm, sizeof(nm), "hot slots %d", j);
      rl.add(3, nm, tp.hslot_off[j], span(tp.hslot_off[j], tp.hrows_off[j]), (size_t)I[j] * 2);
      snprintf(nm, sizeof(nm), "hot rows %d", j);
      const size_t hnext = j + 1 < N ? tp.hslot_off[j + 1] : tp.hc0;
      rl.add(3, nm, tp.hrows_off[j], span(tp.hrows_off[j], hnext), (size_t)HOT_ROWS * 4);
    }
    rl.add(3, "hot counts 0", tp.hc0, span(tp.hc0, tp.hc1), (size_t)dmax * 4);
    rl.add(3, "hot counts 1", tp.hc1, span(tp.hc1, tp.hi0), (size_t)dmax * 4);
    rl.add(3, "hot index 0", tp.hi0, span(tp.hi0, tp.hi1), (size_t)dmax * 4);
    rl.add(3, "hot index 1", tp.hi1, span(tp.hi1, tp.temp), (size_t)dmax * 4);
    rl.add(3, "sort temp", tp.temp, span(tp.temp, tp.acc),
           std::max(sort_temp_bytes(nnz), hot_temp_bytes(dmax)));
    rl.add(3, "norm", tp.acc, span(tp.acc, tp.total), norm2_bytes());
  }
  // --- batched workspace: this sampler once per exclusion
  {
    std::vector<krps_sampler> ss(N, &tmp);
    std::vector<int> ex(N);
    for (int j = 0; j < N; ++j) ex[j] = N > 1 ? j : -1;
    const BatchPlan bp = plan_batch(N, ss.data(), ex.data());
    for (int q = 0; q < N; ++q) {
      char nm[32];
      snprintf(nm, sizeof(nm), "draw %d", q);
      rl.add(4, nm, bp.draw_off[q], span(bp.draw_off[q], bp.tab_off[q]), tmp.draw_bytes);
      snprintf(nm, sizeof(nm), "index table %d", q);
      const size_t tnext = q + 1 < N ? bp.draw_off[q + 1] : bp.prep;
      rl.add(4, nm, bp.tab_off[q], span(bp.tab_off[q], tnext), (size_t)TR * 2);
    }
    rl.add(4, "prep jobs", bp.prep, span(bp.prep, bp.eig), (size_t)N * sizeof(PrepJob));
    rl.add(4, "eigen jobs", bp.eig, span(bp.eig, bp.ztab), (size_t)bp.n_eig * sizeof(EigJob));
    rl.add(4, "table jobs", bp.ztab, span(bp.ztab, bp.probs), (size_t)N * sizeof(ZtabJob));
    rl.add(4, "problems", bp.probs, span(bp.probs, bp.counters),
           (size_t)N * sizeof(BatchProblem));
    rl.add(4, "task counters", bp.counters, span(bp.counters, bp.total),
           2 * NBATCH_CLASSES * 8);
  }
  // --- generic least squares with one right-hand side
  {
    const LsPlan lp = plan_lstsq(R, J, 1);
    TreeShape lm;
    lm.init(J, R);
    rl.add(5, "SA", lp.SA, span(lp.SA, lp.SBw), (size_t)J * R * 8);
    rl.add(5, "SB", lp.SBw, span(lp.SBw, lp.M), (size_t)J * 8);
    rl.add(5, "M", lp.M, span(lp.M, lp.Mp), (size_t)R * R * 8);
    rl.add(5, "M+", lp.Mp, span(lp.Mp, lp.rank), (size_t)R * R * 8);
    rl.add(5, "rank", lp.rank, span(lp.rank, lp.partial), 8);
    rl.add(5, "partials", lp.partial, span(lp.partial, lp.Z), lstsq_partial_bytes(R, 1));
    rl.add(5, "Z", lp.Z, span(lp.Z, lp.scratch), (size_t)R * 8);
    rl.add(5, "M scratch", lp.scratch, span(lp.scratch, lp.total), tree_build_scratch_extent(lm, R));
  }
  *count = rl.n;
  return KRPS_OK;
}

}  // extern "C"
