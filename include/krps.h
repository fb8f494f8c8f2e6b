/*
 * krps.h -- C ABI of libkrps: exact Khatri-Rao-product leverage-score
 * sampling and sketched CP-ALS on one AMD Instinct MI355X (gfx950).
 *
 * The operations follow Bharadwaj et al., "Fast Exact Leverage Score
 * Sampling from Khatri-Rao Products with Applications to Tensor
 * Decomposition" (NeurIPS 2023):
 *   - build a sampler over factors U_j in R^{I_j x R}             (Thm 1.1 part 1, Alg. 1)
 *   - refresh it after a factor changed                            (Thm 1.1 part 1)
 *   - draw J rows of U_1 (.) ... (.) U_N, optionally without one
 *     factor, with probability proportional to their leverage      (Thm 1.1 part 2, Alg. 2)
 *   - solve the sampled problem min ||S A X - S B||_F inside CP-ALS
 *     on a sparse tensor                                           (Sec. 2.1, Sec. 3.3, Alg. 6)
 *
 * General conventions
 *   - Every function returns a krps_status; KRPS_OK is 0, errors are
 *     negative.  krps_last_error() gives a thread-local message for the
 *     last failing call of the calling thread.  No C++ exception crosses
 *     this boundary and nothing aborts.
 *   - Pointers named U, uniforms, idx, prob, rows, ws, sigma, vals are
 *     DEVICE pointers; arrays of sizes/dims are HOST pointers.  Every
 *     device buffer is owned by the caller; the library keeps non-owning
 *     references where stated and never frees them.
 *   - All device memory the library needs beyond its inputs and outputs
 *     comes from caller-provided workspaces (size queries below); the
 *     library itself does not allocate device memory.  Host-side it
 *     allocates its handles, the pinned staging buffers of the batched
 *     draw (owned by the context, grown on demand, freed by
 *     krps_ctx_destroy) and the HIP graph of a captured sweep (owned by
 *     the sampler).
 *   - Uniform streams generated in the kernels (the *_seeded calls) are
 *     Philox4x64-10 (Salmon et al., SC'11) under key (seed, 0): sample d,
 *     mode k of a draw uses counter (ctr_base + d, k, c2, 0), c2 = 0 for a
 *     plain draw and c2 = sweep * N + j for the solve of mode j in ALS sweep
 *     `sweep`; output words x0, x1 give the two uniforms ((x >> 11) + 0.5)
 *     2^-53 of the first and second stage.
 *   - All work is enqueued on the context's HIP stream and is asynchronous;
 *     results are valid after the stream is synchronised.  Host-side
 *     validation happens before anything is enqueued.
 *   - Indices are 0-based int32 (I_j < 2^31).  Matrices are row-major.
 *   - Limits: 1 <= N <= KRPS_MAX_MODES, 1 <= R <= KRPS_MAX_R.
 */
#ifndef KRPS_H
#define KRPS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define KRPS_MAX_MODES 10
#define KRPS_MAX_R 128

typedef enum {
  KRPS_OK = 0,
  KRPS_EINVAL = -1,      /* bad shape, null pointer, index out of range, R outside [1,128] */
  KRPS_EWORKSPACE = -2,  /* workspace smaller than the size query returned */
  KRPS_EDEVICE = -3,     /* a HIP runtime call failed (message has the HIP error) */
  KRPS_EZERO = -4,       /* the Khatri-Rao product is the zero matrix (C = 0, Sec. 3) */
  KRPS_ENUMERIC = -5,    /* NaN/Inf met on the device */
  KRPS_EUNSUPPORTED = -6 /* valid request the library does not implement */
} krps_status;

/* Arithmetic of the sampler and of the sketched solve.  Factor storage is
 * float64 for KRPS_FP64 and float32 for the other two.  The trees' Gram
 * matrices are sums of float64 matrix-core products (exact for float32
 * factors) in every precision, the nodes stored in the factor's type and
 * G_j in float64 (G_j gives G^+, the leverage scores q_d and the
 * eigendecompositions of G_{>k}).  In every precision the walk's
 * arithmetic (node masses, the running offsets, probabilities) is float64
 * over the stored values, so KRPS_FP32 and KRPS_BF16X2 draw the same
 * samples.  The sketched solve keeps the scaled sampled rows w_d a_d and
 * Y = (S B)^T S A in float64 for KRPS_FP64 and KRPS_FP32; KRPS_BF16X2
 * keeps them in float32 and sums the sampled Gram M = (S A)^T S A from
 * three-part bf16 split matrix-core products (~2^-24 relative, float32
 * sums). */
typedef enum { KRPS_FP64 = 0, KRPS_FP32 = 1, KRPS_BF16X2 = 2 } krps_precision;

typedef struct krps_ctx_s* krps_ctx;
typedef struct krps_sampler_s* krps_sampler;
typedef struct krps_tensor_s* krps_tensor;

/* ------------------------------------------------------------------ */
/* Context                                                             */
/* ------------------------------------------------------------------ */

/* Creates a context on HIP device `device` that enqueues on `hip_stream`
 * (a hipStream_t; NULL = the device's null stream).  The stream is not
 * owned.  Does not initialise the GPU beyond selecting the device. */
krps_status krps_ctx_create(int device, void* hip_stream, krps_ctx* out);
krps_status krps_ctx_destroy(krps_ctx ctx);
/* Synchronises the context stream (device-side errors of a sampler are
 * read by krps_sampler_check). */
krps_status krps_ctx_sync(krps_ctx ctx);
/* Thread-local message of the last error (never NULL). */
const char* krps_last_error(void);
/* Library version string. */
const char* krps_version(void);

/* Measured peaks of the units the rooflines are priced against. */
typedef struct {
  double hbm_copy_gbs;        /* device copy: bytes read + written per second */
  double f64_vector_tflops;   /* float64 FMA loops */
  double f32_vector_tflops;   /* float32 FMA loops (no packed instructions) */
  double f64_matrix_tflops;   /* float64 16x16x4 MFMA loops */
  double bf16_matrix_tflops;  /* bf16 16x16x32 MFMA loops (float32 accumulate) */
} krps_peaks;

/* Runs the probe loops on the context's stream (synchronises; the copy uses
 * the device workspace ws, at least 64 MiB, half read and half written). */
krps_status krps_measure_peaks(krps_ctx ctx, void* ws, size_t ws_bytes, krps_peaks* out);

/* ------------------------------------------------------------------ */
/* Sampler: Algorithm 1 (ConstructKRPSampler) and Theorem 1.1 part 1   */
/* ------------------------------------------------------------------ */

/* Bytes of persistent workspace for a sampler over N factors of heights
 * I[0..N-1] and R columns with leaf size F (F = 0 picks R, the paper's
 * choice for the factor trees Z_j, Sec. 3.2).  The workspace holds, per
 * factor, the segment tree T_{I_j,F} of partial Gram matrices (root and
 * left children, packed upper triangles, Appendix A.5) and G_j in float64. */
krps_status krps_sampler_workspace_bytes(int N, const int64_t* I, int R, int F,
                                         krps_precision p, size_t* bytes);

/* Builds the sampler (Algorithm 1): for each j, Z_j = BuildSampler(U_j,
 * F, [1]) (Algorithm 3) and G_j = U_j^T U_j.
 *   U[j]   device pointer, row-major I[j] x R, float64 for KRPS_FP64 and
 *          float32 otherwise.  NON-OWNING: the caller keeps every U[j]
 *          alive and unmodified, or calls krps_sampler_refresh after
 *          changing it.  krps_sketched_solve writes U[j] in place.
 *   ws     device workspace of at least krps_sampler_workspace_bytes().
 * The sampler handle is host memory owned by the library until
 * krps_sampler_destroy. */
krps_status krps_sampler_create(krps_ctx ctx, int N, const int64_t* I, int R, int F,
                                void* const* U, krps_precision p, void* ws,
                                size_t ws_bytes, krps_sampler* out);

/* U[j] changed in place: rebuild Z_j and G_j (O(I_j R^2), Thm 1.1 part 1). */
krps_status krps_sampler_refresh(krps_sampler s, int j);

/* UpdateSampler (Appendix A.7, Algorithm 5; Thm 1.1 part 1's single-entry
 * update) for M entries, applied in order: U_j[rows[m], cols[m]] :=
 * values[m].  The library writes each new value into the caller's U[j]
 * (rounded to float32 for FP32 / BF16X2 factors) and adds the change to
 * every stored node on the path from the row's leaf to the root (the root
 * and the left children; a right child's mass is implied), to the float32
 * node copy of an FP64 sampler and to G_j: O(R log(I_j / F)) per entry,
 * in one workgroup.  rows, cols, values are HOST arrays of length M (they
 * are validated on the host and passed to the kernels by value, 32 per
 * launch).  Asynchronous on the context stream.  A preparation made before
 * the update is invalidated (krps_sample_draw then needs a new
 * krps_sample_prepare).  On float32 storage each update is added in
 * float32, so after many updates the nodes drift from a rebuild by float32
 * rounding; krps_sampler_refresh rebuilds exactly.
 * Errors: KRPS_EINVAL for j, a row or column out of range, a non-finite
 * value, M < 0 or NULL arrays with M > 0. */
krps_status krps_sampler_update_entries(krps_sampler s, int j, int64_t M, const int64_t* rows,
                                        const int32_t* cols, const double* values);
krps_status krps_sampler_destroy(krps_sampler s);

/* Synchronises the context stream, reads and clears the sampler's device
 * status.  Returns KRPS_EZERO if a preparation met a zero product
 * (C = 0), KRPS_ENUMERIC if a kernel met a non-finite value, since the
 * last check.  *zero_weight (may be NULL) receives the number of sampled
 * rows since the last check whose computed probability q_d, or a total
 * mass of whose walk (stage 1 or 2 of a mode, Sec. 3.2), was not
 * positive: both are > 0 in exact arithmetic (Sec. 2.1), so only the
 * rounding of stored values can do that (float32 eigen-trees at a G of
 * condition number near 2^24 / R, for example); such a row was given
 * weight 0 in its solve.  *rewalked (may be
 * NULL) receives the number of float64 walks (a sample and a drawn mode)
 * since the last check that the float32 node copies could not decide and
 * that were walked again from the float64 tree (krps_sampler_set_filter). */
krps_status krps_sampler_check(krps_sampler s, int64_t* zero_weight, int64_t* rewalked);

/* ------------------------------------------------------------------ */
/* Sampling: Algorithm 2 (KRPSample)                                   */
/* ------------------------------------------------------------------ */

/* Bytes of per-draw scratch for krps_sample / krps_row_prob: G^+, every
 * G_{>k} with its eigendecomposition, and the eigen-trees E_k (O(N R^3)). */
krps_status krps_sample_workspace_bytes(krps_sampler s, size_t* bytes);

/* Draws J samples from the Khatri-Rao product of all factors
 * (exclude = -1) or of all but factor `exclude` (Algorithm 2).
 *   uniforms  device float64 [J][N][2] in (0,1): uniforms[d][k][0] drives
 *             the eigen-component draw of mode k for sample d (Sec. 3.2,
 *             first-stage distribution), [d][k][1] its row draw
 *             (second-stage distribution).  Entries of the excluded mode
 *             are ignored.
 *   idx       device int32 [J][N] out: the sampled multi-index, -1 in the
 *             excluded column.
 *   prob      device float64 [J] out or NULL: q_d = l(a_d) / rank(A), the
 *             probability of the sampled row (Sec. 2.1).
 *   rows      device [J][R] out or NULL: the sampled Khatri-Rao rows
 *             a_d = (*)_{k != exclude} U_k[idx[d][k]] in the factor
 *             storage type.
 *   ws        per-draw scratch (krps_sample_workspace_bytes).
 * Returns KRPS_EZERO if the Khatri-Rao product is zero (detected on the
 * device; reported by this call after a stream synchronisation only when
 * `check` is nonzero, else at the next krps_ctx_sync). */
krps_status krps_sample(krps_sampler s, int exclude, int64_t J, const double* uniforms,
                        int32_t* idx, double* prob, void* rows, void* ws, size_t ws_bytes,
                        int check);

/* Size of the static per-GPU scratch of krps_sample_static (16 MiB). */
#define KRPS_STATIC_SCRATCH_BYTES (16u << 20)

/* krps_sample without a workspace argument and without any allocation, for
 * callers that cannot allocate (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  The per-draw scratch is a
 * static device array of KRPS_STATIC_SCRATCH_BYTES per GPU, held until the
 * process ends; the call fails with KRPS_EWORKSPACE when the sampler's
 * per-draw scratch (krps_sample_workspace_bytes: e.g. ~9 MB for N = 3,
 * R = 32, I = 2^20 and ~3.6 MB for N = 3, R = 64, I = 2e4 in float32
 * storage) is larger.  All
 * calls on one GPU share that array: calls that overlap on one GPU (two
 * streams, two host threads) race.  Results equal krps_sample's with the
 * same arguments (no status check). */
krps_status krps_sample_static(krps_sampler s, int exclude, int64_t J, const double* uniforms,
                               int32_t* idx, double* prob, void* rows);

/* krps_sample with uniforms generated in the walk instead of read: for
 * sample d and mode k, the words x0, x1 of Philox4x64-10 (Salmon et al.,
 * SC'11) of counter (ctr_base + d, k, 0, 0) under key (seed, 0) give
 * uniforms[d][k][0] = ((x0 >> 11) + 0.5) 2^-53 (first stage) and
 * uniforms[d][k][1] from x1 (second stage).  Disjoint ctr_base ranges give
 * independent draws.  Other arguments as for krps_sample (no status
 * check). */
krps_status krps_sample_seeded(krps_sampler s, int exclude, int64_t J, uint64_t seed,
                               uint64_t ctr_base, int32_t* idx, double* prob, void* rows,
                               void* ws, size_t ws_bytes);

/* The two halves of krps_sample, for callers that reuse one preparation or
 * time the walk alone.  krps_sample_prepare enqueues the set-up part of
 * Algorithm 2 (G^+, the G_{>k}, their eigendecompositions and the eigen-
 * trees E_k) into ws for exclusion `exclude`; krps_sample_draw enqueues the
 * per-sample walk and must be given the same ws and exclude after a
 * prepare (KRPS_EINVAL otherwise).  Arguments as for krps_sample. */
krps_status krps_sample_prepare(krps_sampler s, int exclude, void* ws, size_t ws_bytes);
krps_status krps_sample_draw(krps_sampler s, int exclude, int64_t J, const double* uniforms,
                             int32_t* idx, double* prob, void* rows, void* ws, size_t ws_bytes);

/* Bytes of workspace for krps_sample_batched over the P samplers s[] with
 * exclusions exclude[] (per problem its per-draw scratch and a table of
 * tri(R) packed indices, plus the job and problem descriptors). */
krps_status krps_sample_batched_workspace_bytes(krps_ctx ctx, int P, const krps_sampler* s,
                                                const int* exclude, size_t* bytes);

/* Algorithm 2 for P independent problems at once (Appendix A.10: many
 * samplers batched): the P preparations run as batched one-block jobs, and
 * the walks of all problems of one storage type and shape class (R <= 8,
 * 16, 32, 64, 128) run in ONE persistent launch, in which each wavefront
 * takes the next task (problem, group of samples) from a device counter;
 * problems are ordered by decreasing cost.  The problems may differ in N,
 * I_j, R and precision.
 *   s[p], exclude[p]  sampler and exclusion of problem p (host arrays;
 *                     every sampler on ctx's device)
 *   J[p]              samples of problem p (host array)
 *   uniforms[p]       device float64 [J[p]][N_p][2], as for krps_sample
 *   idx[p]            device int32 [J[p]][N_p] out (excluded column -1)
 *   prob[p]           device float64 [J[p]] out (NULL array or entry: no q)
 *   ws                workspace (krps_sample_batched_workspace_bytes)
 * The results equal P calls of krps_sample with the same arguments.  The
 * descriptors are staged through pinned host buffers owned by ctx (a call
 * waits for the previous batched call's copy out of the same buffer).  Device-side
 * status (EZERO, ENUMERIC) goes to each sampler's status word. */
krps_status krps_sample_batched(krps_ctx ctx, int P, const krps_sampler* s, const int* exclude,
                                const int64_t* J, const double* const* uniforms,
                                int32_t* const* idx, double* const* prob, void* ws,
                                size_t ws_bytes);

/* The two halves of krps_sample_batched, for callers that time or reuse
 * them: krps_sample_batched_prepare enqueues the P preparations into ws;
 * krps_sample_batched_draw enqueues the walks and must follow a prepare
 * with the same s[], exclude[] and ws (the samplers unchanged since).
 * Each half stages its descriptors through its own pinned buffer of ctx. */
krps_status krps_sample_batched_prepare(krps_ctx ctx, int P, const krps_sampler* s,
                                        const int* exclude, void* ws, size_t ws_bytes);
krps_status krps_sample_batched_draw(krps_ctx ctx, int P, const krps_sampler* s,
                                     const int* exclude, const int64_t* J,
                                     const double* const* uniforms, int32_t* const* idx,
                                     double* const* prob, void* ws, size_t ws_bytes);

/* krps_sample_batched with in-kernel uniforms: problem p's walk generates
 * them from seed[p] and ctr_base[p] (host arrays) as krps_sample_seeded
 * does (counter word 2 = 0).  Other arguments as for krps_sample_batched. */
krps_status krps_sample_batched_seeded(krps_ctx ctx, int P, const krps_sampler* s,
                                       const int* exclude, const int64_t* J,
                                       const uint64_t* seed, const uint64_t* ctr_base,
                                       int32_t* const* idx, double* const* prob, void* ws,
                                       size_t ws_bytes);

/* Probability q of M given multi-indices (idx [M][N], the excluded column
 * is ignored) under the leverage distribution of the (excluded) product. */
krps_status krps_row_prob(krps_sampler s, int exclude, int64_t M, const int32_t* idx,
                          double* prob, void* ws, size_t ws_bytes);

/* ------------------------------------------------------------------ */
/* Sparse tensor and sketched CP-ALS (Sec. 3.3, Alg. 6, Appendix A.9)  */
/* ------------------------------------------------------------------ */

/* Bytes of persistent workspace for a sparse tensor of N modes with the
 * given dims and nnz given entries: per mode j the entries sorted by the
 * other modes' indices (increasing mode order, then i_j), i.e. grouped into
 * the mode-j fibers that rows of mat(T, j)^T select, with entries of equal
 * coordinates merged into one float64 value (their sum), plus an offset
 * table over the leading other mode; per mode the 32 rows with the most
 * entries (the SpMM accumulates them per workgroup); and the sort's
 * scratch. */
krps_status krps_tensor_workspace_bytes(int N, const int64_t* dims, int64_t nnz, size_t* bytes);

/* Builds the per-mode fiber index of a COO tensor on the device.
 *   idx  device int32 [nnz][N], 0 <= idx[e][k] < dims[k] (not checked on
 *        the device; out-of-range indices give undefined results)
 *   val  device float32 [nnz]; duplicate coordinates are allowed and mean
 *        the sum of their values.
 * idx and val are read during this call only (the workspace keeps sorted,
 * merged copies).  Synchronises the stream (to read back the number of
 * distinct coordinates and ||T||_F^2 of the tensor with duplicates
 * summed).  nnz must be in [1, 2^32). */
krps_status krps_tensor_create(krps_ctx ctx, int N, const int64_t* dims, int64_t nnz,
                               const int32_t* idx, const float* val, void* ws, size_t ws_bytes,
                               krps_tensor* out);
krps_status krps_tensor_destroy(krps_tensor t);
/* ||T||_F^2 (host value; valid after krps_tensor_create returned). */
krps_status krps_tensor_norm2(krps_tensor t, double* out);
/* Number of stored entries: distinct coordinates after merging duplicates. */
krps_status krps_tensor_stored_entries(krps_tensor t, int64_t* out);
/* The rows of mode j with the most stored entries, in decreasing count:
 * min(KRPS_HOT_ROWS, dims[j]) of them (ties broken either way), written to
 * rows (host, room for KRPS_HOT_ROWS values), their number to *n.  The
 * SpMM and the exact MTTKRP accumulate the first min(n, 131072 / (8 R)) of
 * them per workgroup in LDS.  Copies from the device on the context's
 * stream and waits for it. */
#define KRPS_HOT_ROWS 512
krps_status krps_tensor_hot_rows(krps_tensor t, int j, int32_t* rows, int* n);

/* Bytes of scratch for one sketched solve / sweep / fit with J samples. */
krps_status krps_solve_workspace_bytes(krps_sampler s, krps_tensor t, int64_t J, size_t* bytes);

/* The initial normalisation of Algorithm 6 for factor j: sigma = column norms of U_j, then
 * U_j[:, i] /= sigma[i] (zero columns stay zero) and Z_j, G_j are rebuilt.
 * sigma: device float64 [R] out (may be NULL).  ws: a solve workspace (any
 * J); only its head below krps_solve_layout's pieces is written. */
krps_status krps_normalize_factor(krps_sampler s, int j, double* sigma, void* ws, size_t ws_bytes);

/* One STS-CP solve (Sec. 3.3; the factor update of Algorithm 6 with the sampled
 * solve): draw J rows of U_{!=j} by leverage (uniforms as in krps_sample),
 * form M = (SA)^T SA and Y = (SB)^T SA with S's weights 1/sqrt(J q_d)
 * (Sec. 2.1) and the sampled mode-j fibers of T (samples drawn more than
 * once select the same fiber; each distinct fiber is expanded once with
 * the summed weight w^2 of its samples), set
 * U_j = Y M^+ (float64 eigen-pseudo-inverse), sigma = its column norms,
 * renormalise U_j in place and rebuild Z_j and G_j.
 *   sigma  device float64 [R] out.
 * The sampler's U[j] buffer is overwritten. */
krps_status krps_sketched_solve(krps_sampler s, krps_tensor t, int j, int64_t J,
                                const double* uniforms, double* sigma, void* ws, size_t ws_bytes);

/* krps_sketched_solve with uniforms generated in the walk: Philox4x64-10 of
 * counter (ctr_base + d, k, sweep * N + j, 0) under key (seed, 0) for
 * sample d and mode k (general conventions above). */
krps_status krps_sketched_solve_seeded(krps_sampler s, krps_tensor t, int j, int64_t J,
                                       uint64_t seed, uint64_t ctr_base, uint64_t sweep,
                                       double* sigma, void* ws, size_t ws_bytes);

/* One ALS sweep: krps_sketched_solve for j = 0..N-1 in order (the inner
 * loop of Algorithm 6).  uniforms: device float64 [N][J][N][2], block j for solve j.
 * With use_graph != 0 the sweep is captured once into a HIP graph (keyed by
 * the argument pointers) and replayed on later calls with the same
 * arguments; a null context stream is captured on a stream of the
 * context's own and replayed on the null stream. */
krps_status krps_als_sweep(krps_sampler s, krps_tensor t, int64_t J, const double* uniforms,
                           double* sigma, void* ws, size_t ws_bytes, int use_graph);

/* krps_als_sweep with uniforms generated in the walks: solve j of sweep
 * `sweep` uses counter word 2 = sweep * N + j (as
 * krps_sketched_solve_seeded).  The sweep's offset sweep * N is written to
 * a word of the workspace by a one-thread kernel enqueued before the sweep,
 * so with use_graph != 0 one captured graph (keyed by t, sigma, ws, J, the
 * walk shape, seed and ctr_base) is replayed for every sweep. */
krps_status krps_als_sweep_seeded(krps_sampler s, krps_tensor t, int64_t J, uint64_t seed,
                                  uint64_t ctr_base, uint64_t sweep, double* sigma, void* ws,
                                  size_t ws_bytes, int use_graph);

/* The exact ALS step of mode j (Algorithm 6 with the full least-squares
 * problem, the reference the sampled solves are measured against): U_j =
 * mat(T, j) (U_N (.) ... (.) U_1 without U_j) ((*)_{k != j} G_k)^+ over
 * every stored entry of T (the sparse MTTKRP), sigma = its column norms,
 * U_j renormalised in place, Z_j and G_j rebuilt.  Float64 arithmetic in
 * every precision (the G_k are float64 in every precision); the factor is
 * stored in its type.  ws: a solve workspace (any J); the
 * pieces of krps_solve_layout are overwritten (M^+ at Mp, the MTTKRP in
 * float64 at Y for the rows listed at yrows, their count at nyrows). */
krps_status krps_exact_solve(krps_sampler s, krps_tensor t, int j, double* sigma, void* ws,
                             size_t ws_bytes);

/* fit = 1 - ||T~ - T||_F / ||T||_F for T~ = [sigma; U_1..U_N] (Sec. 4.3),
 * with ||T~||^2 = sigma^T ((*)_k G_k) sigma and <T, T~> over the stored
 * entries.  sigma: device float64 [R].  fit: host out (synchronises).
 * ws: a solve workspace (any J); only its head, below every piece of
 * krps_solve_layout, is written, so the last solve's pieces stay valid.
 * The G_k are the sampler's float64 Grams (float64 products in every
 * precision). */
krps_status krps_fit(krps_sampler s, krps_tensor t, const double* sigma, double* fit, void* ws,
                     size_t ws_bytes);

/* Bytes of workspace for krps_sketched_lstsq with R columns, J sampled
 * rows and n right-hand sides. */
krps_status krps_lstsq_workspace_bytes(int R, int64_t J, int64_t n, size_t* bytes);

/* The sampled least-squares problem min_X || S A X - S B ||_F on its own
 * (Section 2.1), from rows already drawn: S has one row per sample d with
 * weight w_d = 1/sqrt(J q_d) at the sampled row of A.  Normal equations
 * with a float64 eigen-pseudo-inverse: X = M^+ Z, M = sum_d w_d^2 a_d a_d^T,
 * Z = sum_d w_d^2 a_d b_d^T.
 *   rows     device [J][R]: a_d, the sampled rows of A (unscaled), float64
 *            for KRPS_FP64 and float32 otherwise
 *   prob     device float64 [J]: q_d of each sample (> 0)
 *   SB_rows  device [J][n]: b_d, the rows of B at the sampled indices
 *            (unscaled), same type as rows
 *   X        device float64 [R][n] out
 *   ws       workspace (krps_lstsq_workspace_bytes)
 * The arithmetic is float64 in every precision. */
krps_status krps_sketched_lstsq(krps_ctx ctx, int R, int64_t J, const void* rows,
                                const double* prob, int64_t n, const void* SB_rows, double* X,
                                krps_precision p, void* ws, size_t ws_bytes);

/* ------------------------------------------------------------------ */
/* Autotuning of the walk (leaf size F of the factor trees, lanes per   */
/* sample of the walk kernel)                                          */
/* ------------------------------------------------------------------ */

typedef struct {
  int32_t F;          /* leaf size of the factor trees (krps_sampler_create's F) */
  int32_t lps;        /* lanes per sample of the walk (krps_sampler_set_lps) */
  int32_t team;       /* waves per leaf team of the tree build (krps_sampler_set_build) */
  double build_ms;    /* measured: rebuild of all N trees */
  double draw_ms;     /* measured: prepare + draw of J samples over all modes */
  int32_t from_cache; /* 1 if read from the cache file, 0 if measured now */
} krps_tune;

/* Selects the walk shape of a sampler: lanes per sample (0 = default;
 * 4 or 8 for R <= 8, 8 or 16 for R <= 16, 16, 32 or 64 for R <= 32, 64
 * above; the defaults are 4, 8, 32 for float64 and 16 for float32
 * storage at R <= 32, and 64).  The index and probability of every draw do
 * not depend on it. */
krps_status krps_sampler_set_lps(krps_sampler s, int lps);

/* Deterministic sketched solves (on != 0) for runs that must repeat bit
 * for bit: the SpMM forming Y (Appendix A.13) rounds every term
 * coef x_e a_d[c] to a multiple of 2^-s and sums with int64 atomics, whose
 * result does not depend on their order; s is the largest exponent with
 * B 2^s <= 2^62 for B = the sum over all terms of |coef x_e| max_c |a_d[c]|
 * (a bound on every row's sum of |terms|, itself reduced in a fixed
 * order), so each term carries at most B 2^-63 of rounding and no sum
 * overflows.  Y is then float64 on every path.  Default 0: float atomics,
 * whose order varies the last bits of Y between runs.  Applies to
 * krps_sketched_solve*, krps_als_sweep*; a captured sweep is re-captured. */
krps_status krps_sampler_set_deterministic(krps_sampler s, int on);

/* Selects the tree build's team width: waves that share one leaf's
 * 16 x 16 accumulator tiles (0 = default; R <= 16: 1; R <= 32: 1 or 3;
 * R <= 64: 2 or 5; above: 6 or 12).
 * Fewer waves hold more tiles each (more registers, fewer loads shared).
 * The stored nodes do not depend on it.  KRPS_EINVAL for another value. */
krps_status krps_sampler_set_build(krps_sampler s, int team);

/* Float64 samplers keep a float32 copy of every factor-tree node (each
 * entry rounded to nearest; it is built with the tree and held in the
 * sampler workspace).  Below the top `top` levels of a tree, the walk of
 * Algorithm 4 reads the copy -- half the bytes -- and takes a branch only
 * when the float64 walk would take it for every value within the copy's
 * rounding bound (the node mass's bound, 2^-24 relative per entry, and the
 * running offset's, accumulated over the filtered levels); a sample whose
 * branch or leaf row that bound cannot decide is walked again from the
 * float64 nodes.  Every drawn index is therefore the float64 walk's.
 * top = -1 selects the default (all but the ten deepest levels read the
 * float64 nodes); top >= the tree depth turns the copy off.  No effect
 * on float32 and split samplers.  Returns KRPS_EINVAL for top < -1. */
krps_status krps_sampler_set_filter(krps_sampler s, int top);

/* Bytes of workspace for krps_autotune (a sampler with the smallest leaf
 * size tried, its draw scratch and J outputs). */
krps_status krps_autotune_workspace_bytes(int N, const int64_t* I, int R, krps_precision p,
                                          int64_t J, size_t* bytes);

/* Times a rebuild of the N trees plus a draw of J samples (no exclusion,
 * uniforms device float64 [J][N][2]) over the caller's factors U for leaf
 * sizes F in {R/2, R, 2R, 4R}, every lanes-per-sample choice of R and
 * every tree-build team width of R and p, and returns the fastest.
 * Results are keyed by (gfx950, precision, R, J, I_1..I_N) in the
 * JSON-lines file cache_path (NULL: no cache): a key present there is
 * returned without timing (the last entry whose shapes the library offers
 * for R and p; others are skipped); a new result is appended.  The leaf size
 * does not change any drawn index (ties go to the lower row, so the index
 * depends only on the row order).  Synchronises the stream. */
krps_status krps_autotune(krps_ctx ctx, int N, const int64_t* I, int R, krps_precision p,
                          void* const* U, int64_t J, const double* uniforms, void* ws,
                          size_t ws_bytes, const char* cache_path, krps_tune* out);

/* Randomized range-finder initialisation of factor j (the initialisation
 * the paper uses for its sparsest tensor, Section 4.3): U_j = mat(T, j) S
 * with an i.i.d. N(0,1) sketch S of prod_{k != j} I_k rows and R columns
 * that is generated only for fibers holding entries and never stored.
 * Row of S for the fiber with other-mode indices (i_a, i_b, i_c, i_d)
 * (increasing mode order, missing ones 0), column pair q: Philox4x64-10 of
 * counter (i_a | i_b << 32, i_c | i_d << 32, q, 0) under key (seed, j);
 * the first two output words x give uniforms ((x >> 11) + 0.5) 2^-53 and
 * the Box-Muller pair (cosine, sine) gives columns 2q and 2q + 1.  Then
 * the columns are normalised as krps_normalize_factor does (sigma out,
 * may be NULL) and Z_j is rebuilt.  U[j] is overwritten.  N <= 5
 * (KRPS_EUNSUPPORTED otherwise).  ws: a solve workspace (any J); the
 * float64 accumulation of mat(T, j) S overwrites the pieces of
 * krps_solve_layout. */
krps_status krps_init_range_finder(krps_sampler s, krps_tensor t, int j, uint64_t seed,
                                   double* sigma, void* ws, size_t ws_bytes);

/* Offsets (bytes into the solve workspace) of the last solve's pieces. */
typedef struct {
  size_t idx;      /* int32 [J][N] sampled multi-indices */
  size_t prob;     /* float64 [J] q_d */
  size_t w;        /* float64 [J] 1/sqrt(J q_d); 0 where the computed q_d is
                      not positive (rounding), so that sample adds nothing */
  size_t rows;     /* [J][R] w_d a_d (rows of S A): float64, float32 for KRPS_BF16X2 */
  size_t M;        /* float64 [R][R] (S A)^T S A */
  size_t Mp;       /* float64 [R][R] its pseudo-inverse */
  size_t Y;        /* [I_j][R] (S B)^T S A, float64 (float32 for KRPS_BF16X2,
                      whose rows of S A are float32 too): only the rows listed
                      at yrows are written by the solve; every other row of
                      (S B)^T S A is zero and its slot in Y is left as it was */
  size_t draw;     /* per-draw scratch (krps_draw_layout offsets are relative to this) */
  size_t yrows;    /* int32 [*nyrows] rows of mode j that the sampled fibers'
                      entries reach, increasing */
  size_t nyrows;   /* int64: their count */
  size_t expanded; /* int64: fiber entries the SpMM expanded (the sizes of
                      the distinct sampled fibers summed) */
} krps_solve_layout;

krps_status krps_solve_layout_query(krps_sampler s, krps_tensor t, int64_t J,
                                    krps_solve_layout* out);

/* ------------------------------------------------------------------ */
/* Introspection (tests and benchmarks)                                */
/* ------------------------------------------------------------------ */

typedef struct {
  int64_t I;          /* rows of the factor */
  int64_t L;          /* leaves, ceil(I / F) */
  int32_t F;          /* leaf size */
  int32_t D;          /* depth, ceil(log2 L) (0 for one leaf) */
  int64_t n_nodes;    /* stored nodes: root + left children */
  int64_t tri;        /* R (R + 1) / 2, elements per stored node */
  void* nodes;        /* device: n_nodes x tri (then 64 zero elements), packed upper triangle, row-major
                         (entry (a, b), a <= b, at a*R - a*(a-1)/2 + b - a);
                         node 0 is the root, then for level l = 1..D the left
                         children in position order (position 2m stored at m) */
  double* gram;       /* device: G_j = U_j^T U_j, R x R float64 */
  int elem_bytes;     /* 8 (FP64) or 4 */
} krps_tree_info;

krps_status krps_sampler_tree_info(krps_sampler s, int j, krps_tree_info* out);

/* Offsets (bytes into the per-draw workspace) of what krps_sample prepares
 * for exclusion `exclude`; valid after a krps_sample / krps_row_prob call
 * with that workspace. */
typedef struct {
  size_t gplus;       /* float64 R x R, G^+ of G = (*)_{k != exclude} G_k */
  size_t rank;        /* int32 [2 + N]: rank of G, then the Jacobi sweep count of
                         G (0 when G^+ = G^{-1} came from the certified Cholesky
                         route) and of each drawn mode's G_{>k} (diagnostics) */
  size_t ggt;         /* float64 [N][R][R]: G_{>k} */
  size_t lam;         /* float64 [N][R]: eigenvalues of G_{>k}, ascending */
  size_t vecs;        /* factor type [N][R][R]: eigenvector u of mode k at [k][u][:] */
  size_t etree;       /* factor type: E_k at etree + k * etree_stride elements, n_enodes
                         nodes of tri entries in the layout of Z, then zero padding */
  int64_t n_enodes;   /* stored nodes per E_k (F = 1, L = R) */
  int64_t etree_stride; /* elements from E_k to E_{k+1} */
} krps_draw_layout;

krps_status krps_draw_layout_query(krps_sampler s, krps_draw_layout* out);

/* One region of a workspace, as planned by the library. */
typedef struct {
  int32_t workspace;  /* 0 sampler, 1 per-draw, 2 solve, 3 tensor, 4 batched
                         (the sampler once per exclusion), 5 least squares (n = 1) */
  char name[28];
  uint64_t offset;    /* bytes from the workspace start */
  uint64_t bytes;     /* up to the next region */
  uint64_t need;      /* the largest extent a kernel writes or reads in it,
                         from the launch geometry (tree-build ping-pong
                         buffers, reads past a node's end) */
} krps_region;

/* The regions of every workspace the library plans for N factors of heights
 * I (also the tensor's dims), R columns, leaf size F (0 = R), precision p,
 * a tensor of nnz entries and solves of J samples.  Host only: touches no
 * device.  Writes min(cap, count) regions to out (may be NULL) and the
 * number of regions to *count.  For tests of the workspace planning. */
krps_status krps_workspace_regions(int N, const int64_t* I, int R, int F, krps_precision p,
                                   int64_t nnz, int64_t J, krps_region* out, int cap, int* count);

#ifdef __cplusplus
}
#endif
#endif /* KRPS_H */
