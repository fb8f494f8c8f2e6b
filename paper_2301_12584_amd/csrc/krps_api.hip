// libkrps C ABI: argument validation, workspace planning and stream-ordered
// launches of the sampler kernels.  Host code only; every computation runs
// in the kernels of tree_build.hip, eig.hip and descent.hip.
#include <cstdio>
#include <cstdlib>
#include <cstring>
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
  std::vector<double*> gram;
  double* scratch;
  size_t scratch_bytes;
  int32_t* status;
  // per-draw workspace layout
  krps_draw_layout lay;
  const void* prepared_ws = nullptr;  // ws of the last preparation
  int prepared_exclude = -2;
  int lps = 0;                         // descent lanes per sample (0 = default)
  size_t draw_bytes;
  int64_t enodes;
  int DE;
};

namespace {

bool valid_prec(krps_precision p) { return p == KRPS_FP64 || p == KRPS_FP32 || p == KRPS_BF16X2; }
int elem_bytes(krps_precision p) { return p == KRPS_FP64 ? 8 : 4; }

krps_status check_dims(int N, const int64_t* I, int R) {
  if (N < 1 || N > KRPS_MAX_MODES) return fail(KRPS_EINVAL, "N must be in [1, 8]");
  if (R < 1 || R > KRPS_MAX_R) return fail(KRPS_EINVAL, "R must be in [1, 128]");
  if (I == nullptr) return fail(KRPS_EINVAL, "I is NULL");
  for (int j = 0; j < N; ++j)
    if (I[j] < 1 || I[j] > INT32_MAX) return fail(KRPS_EINVAL, "each I_j must be in [1, 2^31)");
  return KRPS_OK;
}

struct SamplerPlan {
  std::vector<TreeShape> shape;
  std::vector<size_t> node_off, gram_off;
  size_t scratch_off = 0, scratch_bytes = 0, status_off = 0, total = 0;
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
    off += align_up((size_t)ts.n_nodes * TR * elem_bytes(p));
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
  pl.total = off;
  return pl;
}

void plan_draw(krps_sampler s) {
  const int R = s->R, N = s->N;
  const int64_t TR = tri(R);
  s->DE = R > 1 ? ceil_log2(R) : 0;
  TreeShape es;
  es.init(R, 1);
  s->enodes = es.n_nodes;
  size_t off = 0;
  krps_draw_layout& l = s->lay;
  l.gplus = off;
  off += align_up((size_t)R * R * 8);
  const size_t gpacked = off;
  off += align_up((size_t)TR * 8);
  l.rank = off;
  off += 256;
  l.ggt = off;
  off += align_up((size_t)N * R * R * 8);
  l.lam = off;
  off += align_up((size_t)N * R * 8);
  l.vecs = off;
  off += align_up((size_t)N * R * R * s->elem);
  l.etree = off;
  off += align_up((size_t)N * s->enodes * TR * s->elem);
  l.n_enodes = s->enodes;
  s->draw_bytes = off;
  (void)gpacked;
}

size_t gpacked_off(krps_sampler s) { return s->lay.gplus + align_up((size_t)s->R * s->R * 8); }

krps_status build_tree(krps_sampler s, int j) {
  hipError_t e = launch_tree_build(s->ctx->stream, s->prec, s->U[j], s->I[j], s->R, s->shape[j],
                                   s->nodes[j], s->gram[j], s->scratch, s->scratch_bytes);
  if (e != hipSuccess) return hip_fail(e, "tree build launch");
  return KRPS_OK;
}

void fill_descent_args(krps_sampler s, int exclude, void* ws, DescentArgs& a);

// Enqueues lines 1-5 of Algorithm 2 for exclusion `exclude` into ws and
// fills the descent arguments.
krps_status prepare_draw(krps_sampler s, int exclude, void* ws, DescentArgs& a) {
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
  e = launch_prep_eig2(st, s->prec, R, nsteps, mats, order, ggt, lam, vecs, etree, s->enodes,
                       rank);
  if (e != hipSuccess) return hip_fail(e, "prep eig launch");
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
    m.E = w + s->lay.etree + (size_t)k * s->enodes * TR * s->elem;
    m.V = w + s->lay.vecs + (size_t)k * R * R * s->elem;
    m.I = s->I[k];
    m.L = s->shape[k].L;
    m.F = s->shape[k].F;
    m.D = s->shape[k].D;
    m.DE = s->DE;
  }
  a.gplus = gplus_packed;
  a.rank = rank;
  a.status = s->status;
  a.lps = s->lps;
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
  delete ctx;
  return KRPS_OK;
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
    s->gram.push_back((double*)(w + pl.gram_off[j]));
  }
  s->scratch = (double*)(w + pl.scratch_off);
  s->scratch_bytes = pl.scratch_bytes;
  s->status = (int32_t*)(w + pl.status_off);
  if (const char* e = getenv("KRPS_DESCENT_LPS")) s->lps = atoi(e);
  plan_draw(s);
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) {
    delete s;
    return hip_fail(e, "hipSetDevice");
  }
  e = hipMemsetAsync(s->status, 0, 4, ctx->stream);
  if (e != hipSuccess) {
    delete s;
    return hip_fail(e, "status clear");
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

krps_status krps_sampler_refresh(krps_sampler s, int j) {
  if (s == nullptr) return fail(KRPS_EINVAL, "sampler is NULL");
  if (j < 0 || j >= s->N) return fail(KRPS_EINVAL, "j out of range");
  return build_tree(s, j);
}

krps_status krps_sampler_destroy(krps_sampler s) {
  delete s;
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

}  // extern "C"
