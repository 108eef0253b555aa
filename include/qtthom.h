/* qtthom.h -- C ABI of the MI355X hot path of SFFT/QTT Lippmann-Schwinger
 * homogenization (Hauck, Kabel, Gauger, arXiv 2512.07811).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Status: every call returns a qt_status; 0 is success, negative values are
 *   hard errors, QT_NOT_CONVERGED is informational.  The calling thread's last
 *   error message is available from qt_last_error().  No C++ exception crosses
 *   the boundary.
 * Memory: all tensor data is device memory owned by the caller (the Python
 *   binding uses PyTorch allocations).  A context made by qt_ctx_create owns
 *   its workspace, which it allocates at creation or on first need and
 *   reuses; a context made by qt_ctx_create_with_memory takes every device
 *   buffer it needs (workspace, GEMM split-K partials, tile-timing output,
 *   learned-rank state and logs) from one caller-owned block and never calls
 *   hipMalloc after creation: a call that does not fit returns QT_ENOMEM
 *   with the bytes it needed, and the size to pass is given by
 *   qt_ctx_fixed_bytes() plus qt_workspace_query / qt_ls_workspace_query.
 * Streams: calls are asynchronous on the context's stream unless a host
 *   output is requested (then they synchronize that stream before returning).
 * Numbers: every TT is complex double, interleaved (re, im).  Core k of a TT
 *   is stored row-major with shape (r_k, p_k, r_{k+1}) (left bond, physical
 *   index, right bond) packed with its ACTUAL ranks inside a slot sized by its
 *   rank CAPACITIES; r_0 = r_n = 1.  (The paper writes a core as
 *   (r_k x p x r_{k-1}); only the storage order differs.)
 * Ranks: actual ranks live in DEVICE memory and are updated by the kernels,
 *   so that a whole iteration needs no host synchronisation; capacities are
 *   host values fixed by the caller.
 * Batches: a qt_tt may describe B instances with identical modes and
 *   capacities; instance b's data starts at data + b*inst_stride elements and
 *   its ranks at ranks + b*(n+1).
 */
#ifndef QTTHOM_H
#define QTTHOM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t qt_status;
#define QT_OK             0
#define QT_NOT_CONVERGED  1   /* informational: iteration cap reached          */
#define QT_EINVAL        -1   /* bad argument, shape mismatch or aliasing       */
#define QT_ECAPACITY     -2   /* a result does not fit the output capacities    */
#define QT_ENOMEM        -3   /* workspace allocation failed                    */
#define QT_EHIP          -4   /* HIP runtime error                              */
#define QT_ENUMERIC      -5   /* Jacobi sweep cap reached or non-finite values  */

/* Rounding modes. */
#define QT_ROUND_SVD      0   /* QR sweep + truncated-SVD sweep (Sec. 2.2)       */
#define QT_ROUND_SKETCH   1   /* randomized range sketch + SVD truncation        */
#define QT_ROUND_LEARNED  2   /* sketch at MLP-predicted ranks, SVD fallback     */
#define QT_ROUND_POLAR    3   /* QR sweep + polar-decomposition truncation       */

/* Contraction precision of the product-aware roundings (tt_sketch_round,
 * ls_iterate / homogenize in the sketch and learned modes; QT_EINVAL
 * elsewhere).  QT_PREC_F64: every contraction in FP64.  QT_PREC_F32 (mixed):
 * the contractions that only choose the bases of the randomized range finder
 * (right sketches W_k and the sketched products Y_k) run on FP32 MFMA
 * (operands rounded to FP32, FP32 accumulation; each such element is within
 * (K + 4) 2^-24 sum_k |a_k||b_k| of its FP64 value for K terms), while the
 * projection onto those bases, the QR and SVD factorizations and the error
 * bookkeeping stay FP64.  The result is therefore still an exact orthogonal
 * projection of the product, and the reported error is its exact error (or
 * bound, with SVD truncation) as in FP64; what the FP32 bases cost is a larger
 * projection error: 7.5e-6 to 1.1e-4 relative for a full-width sketch of
 * small random trains (1e-13 in FP64), and, in the LS iteration of a 16^3
 * cell, an A_eff within 2e-4 of the FP64 path's with a residual floor near
 * 1e-2 (the paper computes in complex64 throughout, Sec. 4.1).  Use it where
 * eps is about 1e-3 or larger. */
#define QT_PREC_F64       0
#define QT_PREC_F32       1

typedef struct qt_ctx_s* qt_ctx;

/* A batch of B tensor trains with n cores (Sec. 2, eq. tt_format). */
typedef struct {
  int32_t n;                /* number of cores                                   */
  int32_t batch;            /* B >= 1                                            */
  const int32_t* modes;     /* host [n]: physical dimension p_k                  */
  const int32_t* cap;       /* host [n+1]: rank capacities, cap[0] = cap[n] = 1  */
  const int64_t* offsets;   /* host [n]: element offset of core k's slot         */
  int64_t inst_stride;      /* elements between instances (>= sum of slots)      */
  int32_t* ranks;           /* device [B][n+1]: actual ranks (ranks[0]=ranks[n]=1) */
  void* data;               /* device complex double                             */
} qt_tt;

/* A tensor-train operator (eq. tto_format) with fixed, host-known ranks.
 * Core k is (r_k, p_out, p_in, r_{k+1}) row-major, or, when diag[k] != 0, a
 * diagonal core stored as (r_k, p, r_{k+1}) meaning D(a,i,j,b) = B(a,i,b) d(i,j)
 * (the TT -> TTO lift, eq. tt_to_tto).
 * Several operator instances (one per microstructure of a batch) share the
 * ranks, modes and offsets: instance i starts at data + i*inst_stride elements
 * and field b of a batch uses instance b / inst_group.  Instances with lower
 * ranks are zero-padded to the common ranks (exact).  inst_stride = 0 means one
 * operator for every field.  Per-instance operators are read by the
 * product-aware (sketch/learned) kernels; the materializing tt_mpo_apply and
 * the plain iteration require inst_stride = 0. */
typedef struct {
  int32_t n;
  const int32_t* modes_out; /* host [n] */
  const int32_t* modes_in;  /* host [n] */
  const int32_t* ranks;     /* host [n+1] */
  const int32_t* diag;      /* host [n]  */
  const int64_t* offsets;   /* host [n]  */
  const void* data;         /* device complex double */
  int64_t inst_stride;      /* elements between operator instances (0: shared) */
  int32_t inst_group;       /* fields per operator instance (>= 1)             */
} qt_mpo;

typedef struct {
  double eps;               /* relative tolerance of eq. (rounding_condition_tt) */
  int32_t max_rank;         /* rank cap (<= output capacities); 0 = capacity     */
  int32_t mode;             /* QT_ROUND_*                                        */
  int32_t jacobi_max_sweeps;/* 0 = default (30)                                  */
  int32_t precision;        /* QT_PREC_* for sketch contractions                 */
  int32_t oversample;       /* extra sketch columns per bond (sketch modes)      */
  uint64_t seed;            /* counter-based Gaussian sketch seed                */
} qt_round_opts;

/* ---- context ------------------------------------------------------------ */

/* Create a context on `device` using the borrowed hipStream_t `stream`
 * (NULL = default stream).  Reserves `ws_bytes` of workspace now (0 = lazily);
 * the workspace grows (hipMalloc) when a call needs more. */
qt_status qt_ctx_create(int device, void* stream, size_t ws_bytes, qt_ctx* out);

/* Create a context whose device memory is all in the caller's block `mem`
 * (device memory on `device`, 256-byte aligned, `mem_bytes` long, borrowed:
 * the caller frees it after qt_ctx_destroy and must not touch it while the
 * context lives).  The head of the block, qt_ctx_fixed_bytes() long, holds the
 * status word, the event counters and the GEMM split-K partials (cleared by
 * this call, which synchronizes); the rest is the workspace arena, from whose
 * end persistent buffers (learned-rank state, rank and rounding logs) are
 * taken when first needed.  No call on this context allocates device memory:
 * one that needs more than is free returns QT_ENOMEM (its message gives the
 * bytes) before launching anything.  GEMM tile timing writes into the free
 * part of the arena and is skipped when that is too small.
 * Errors: QT_EINVAL for a null or misaligned block, QT_ENOMEM when mem_bytes
 * is below qt_ctx_fixed_bytes(), QT_EHIP when clearing the head fails. */
qt_status qt_ctx_create_with_memory(int device, void* stream, void* mem, size_t mem_bytes,
                                    qt_ctx* out);
/* Bytes of the fixed head of a caller-owned context block (a constant of the
 * library build, about 64 MiB of split-K partials). */
size_t    qt_ctx_fixed_bytes(void);

/* Workspace bytes tt_round (and tt_round_noalloc) needs for a train of x's
 * capacities and batch with these options.  Host-only, launches nothing.
 * QT_EINVAL for a malformed x. */
qt_status qt_workspace_query(const qt_tt* x, const qt_round_opts* opts, size_t* bytes);

void      qt_ctx_destroy(qt_ctx ctx);
/* Last error message of the calling thread ("" if none). */
const char* qt_last_error(void);
/* Block until every call issued on the context's stream has finished. */
qt_status qt_ctx_sync(qt_ctx ctx);

/* Device event counters since creation (or the last reset), int64 each:
 *  [0] truncated SVDs, [1] Jacobi sweeps they used, [2] sketch roundings whose
 *  error exceeded the budget, [3] learned instance-roundings that fell back to
 *  SVD rounding, [4] structured-GEMM flops, [5] structured-GEMM bytes,
 *  [6] learned (fixed predicted rank) instance-roundings attempted.
 *  Synchronizes the stream. */
qt_status qt_ctx_counters(qt_ctx ctx, int64_t* out, int32_t n, int32_t reset);

/* Live timing of kernel classes (bit mask: 1 structured GEMMs, 2 QR
 * factorizations, 4 truncated SVDs; 0 disables): the library records HIP
 * events on its stream around every launch of those classes.
 * qt_ctx_profile_read returns the summed event time and the number of timed
 * launches since the last read, then clears them.  Counters [4] and [5] of
 * qt_ctx_counters hold the algorithmic flops and bytes of the structured
 * GEMMs (8 flops per complex multiply-add; A, B, C touched once). */
qt_status qt_ctx_profile(qt_ctx ctx, int32_t classes);
qt_status qt_ctx_profile_read(qt_ctx ctx, double* total_ms, int64_t* launches);

/* Tile shape of the structured GEMM (the MFMA kernel of every contraction).
 * Each call has one of four output-tile shapes (64 or 32 rows by 64 or 32
 * columns); every shape sums each output element's terms in the same order,
 * so results are bitwise equal across shapes.  mode 0: always 64 x 64;
 * 1 (default): autotune - the first call of each signature (row and column
 * capacities in 32-wide steps up to 64 and in half octaves above, the
 * contraction length in octaves, item count to a power of two, conjugations,
 * stride pattern) that runs outside a graph capture and
 * without split-K times every shape once on its first instance, writing to a
 * context-owned scratch (allocated on demand, at most 256 MiB), and later
 * calls of that signature use the fastest; 2..5: always shape mode - 2 (bit 0:
 * 32 rows, bit 1: 32 columns).  Timing synchronizes the stream.  *entries
 * (may be null) receives the number of tuned signatures.  QT_EINVAL for a
 * mode outside 0..5. */
qt_status qt_ctx_autotune(qt_ctx ctx, int32_t mode, int32_t* entries);

/* ---- TT algebra (Sec. 2.1) --------------------------------------------- */

/* out = a (Hadamard) b: C_k(i) = A_k(i) (Kronecker) B_k(i); exact, ranks
 * r_a*r_b with a's bond index slow.  Needs out->cap[k] >= a->cap[k]*b->cap[k].
 * out must not alias a or b.  Batch sizes must match (or a->batch == 1, which
 * broadcasts a over b's instances). */
qt_status tt_hadamard(qt_ctx ctx, const qt_tt* a, const qt_tt* b, qt_tt* out);

/* out = A x: B_k(i) = sum_j D_k(i,j) (Kronecker) X_k(j) (TT x TTO contraction);
 * exact, ranks r_A*r_x with the operator bond slow. */
qt_status tt_mpo_apply(qt_ctx ctx, const qt_mpo* A, const qt_tt* x, qt_tt* out);

/* out = alpha*x + beta*y by block-diagonal cores (addition, constant
 * multiplication and subtraction of Sec. 2.1); ranks r_x + r_y. */
qt_status tt_add(qt_ctx ctx, double alpha_re, double alpha_im, const qt_tt* x,
                 double beta_re, double beta_im, const qt_tt* y, qt_tt* out);

/* ---- stability (Sec. 2.2) ----------------------------------------------- */

/* In-place rounding.  QT_ROUND_SVD: left QR orthogonalization sweep, then a
 * right-to-left truncated-SVD sweep keeping, per bond, the smallest rank whose
 * discarded singular-value tail does not exceed eps*||x||/sqrt(n-1), capped by
 * max_rank.  On return cores 1..n-1 are right-orthogonal.
 * err_out (device [B], may be NULL): sqrt(sum of squared discarded tails)/||x||.
 * norm_out (device [B], may be NULL): ||x||_F before rounding.
 * QT_ECAPACITY (nothing launched) when a bond's SVD block, min(cap[k],
 * p_k min(cap[k+1], max_rank)), exceeds 1024 columns.
 * QT_ROUND_POLAR (Sec. 2.2, compression via polar decomposition): the same
 * left QR sweep, then right to left every centre A (r_k x p_k r_{k+1}) is
 * split without an SVD: A^H = U H (polar factor by odd-polynomial
 * Newton-Schulz-type iterations on the MFMA GEMM), U' = sign(H - d~ I) by the
 * same iteration, P+ = (I + U')/2, C+ an orthonormal basis of range(P+) by
 * subspace iteration (QR), core k = (U C+)^H, H C+ carried to core k-1.  The
 * cutoff is absolute, d~ = delta / min(r_k, p_k r_{k+1}), so every singular
 * value above it is kept: ||x - x~|| <= eps ||x|| with ranks at least those
 * of QT_ROUND_SVD; singular values within about 5 % of d~ may land on
 * either side (the iteration counts resolve |sigma - d~| down to a
 * twentieth of d~).  max_rank keeps the directions of P+ that H ranks first
 * (subspace iteration with H^2, 4 steps).
 * err_out: sqrt(sum_k ||A_k - H C+ (U C+)^H||^2)/||x||, the discarded weight
 * of each centre formed explicitly.
 * opts->seed seeds the Gaussian start block of the subspace iteration. */
qt_status tt_round(qt_ctx ctx, qt_tt* x, const qt_round_opts* opts, double* err_out,
                   double* norm_out);

/* Allocation-free variant of tt_round, for callers that cannot allocate
 * device memory during the call: code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc.  Same arguments, kernels and results
 * as tt_round (bitwise equal on the same input), but the rounding's workspace
 * is a library-owned static device array of QT_NOALLOC_SCRATCH_BYTES per GPU
 * (held from library load until the process ends; its address is looked up
 * by qt_ctx_create), and the call performs no hipMalloc/hipFree, no GEMM
 * tile-shape timing (signatures not tuned yet use 64 x 64 tiles) and no
 * profiling events.
 * Limits: QT_ECAPACITY (nothing launched) when the rounding needs more than
 * QT_NOALLOC_SCRATCH_BYTES of workspace (e.g. rank 384 on 25 cores fits,
 * rank 512 does not) or an SVD block above 1024 columns.
 * Concurrency: every call on one GPU, from any context or thread, uses the
 * same array and leaves its contents behind; calls that overlap in time on
 * one GPU (different streams, or threads) race and give undefined results.
 * Calls on one stream are ordered and safe.  Nothing in the array needs to
 * start at zero. */
#define QT_NOALLOC_SCRATCH_BYTES (64ll << 20)
qt_status tt_round_noalloc(qt_ctx ctx, qt_tt* x, const qt_round_opts* opts, double* err_out,
                           double* norm_out);

/* Frobenius inner product of two trains with equal modes, per instance:
 * out[b] = sum_i conj(a_b(i)) x b_b(i), device [B][2] doubles (re, im),
 * contracted core by core through left environments (nothing materialized).
 * sqrt(Re tt_dot(x, x)) is the Frobenius norm of the rounding condition
 * (Sec. 2.2, eq. rounding_condition_tt) and of Algorithm 2's convergence test;
 * with a = the selector train of k times a component, Re tt_dot(a, e) / N^3
 * is the mean flux that gives a column of the effective tensor (Appendix A,
 * the macroscopic stress-strain relation in Voigt form).  a->batch is 1
 * (broadcast) or b->batch.  QT_EINVAL on mismatched modes or batches. */
qt_status tt_dot(qt_ctx ctx, const qt_tt* a, const qt_tt* b, double* out);

/* ---- product-aware rounding ---------------------------------------------- */

/* Rounds x = A y (TT x TTO contraction, Sec. 2.1; a Hadamard product is the
 * diagonal case) into `out` WITHOUT forming the rank-(r_A r_y) cores of x:
 * randomize-then-orthogonalize with a Gaussian train Omega (Al Daas et al.,
 * SIAM J. Sci. Comput. 2023), contracting A and y separately.
 *  omega: single train of sketch cores (its capacities are the sketch ranks
 *         l_k); NULL draws Philox4x32-10 Gaussians from opts->seed with
 *         l_k = min(natural rank, r_A r_y capacity, max_rank + oversample).
 *  opts->mode QT_ROUND_SKETCH: then a right-to-left truncated-SVD sweep with
 *         the remaining budget eps||x|| - e_s, e_s = (||x||^2 - ||x~||^2)^(1/2),
 *         split over the n-1 bonds, threshold (eps||x|| - e_s)/sqrt(n-1)
 *         (capped by max_rank; the truncation error is not orthogonal to the
 *         projection error, so the two add linearly);
 *         QT_ROUND_LEARNED: keep the sketch ranks (fixed-rank rounding).
 *  xnorm2: device [B] exact ||x||^2 (e.g. from tt_sandwich).
 *  err_out: device [B] (e_s + sqrt(sum of discarded tails^2))/||x||: the exact
 *         relative error in QT_ROUND_LEARNED mode, an upper bound of it in
 *         QT_ROUND_SKETCH mode (equal when nothing is truncated).
 *  fail_out: device [B] int, 1 when the sketch error alone exceeds eps*||x||.
 * A must be square (p_out = p_in = y's modes). out->cap >= sketch ranks.
 * QT_ECAPACITY (before the truncation sweep) in mode QT_ROUND_SKETCH when a
 * bond's SVD block of `out` exceeds 1024 columns. */
qt_status tt_sketch_round(qt_ctx ctx, const qt_mpo* A, const qt_tt* y, const qt_tt* omega,
                          const qt_round_opts* opts, const double* xnorm2, qt_tt* out,
                          double* err_out, int32_t* fail_out);

/* ---- AMEn product ---------------------------------------------------------- */

/* y ~ A x for a TTO A and a TT x built directly in the TT format, without the
 * rank-(r_A r_x) product and its compression: the alternating minimal energy
 * method of Sec. 2.1 (Dolgov and Savostyanov 2014), which Algorithm 2 applies
 * to the Green multiply.  Each of `sweeps` sweeps takes the cores of y from
 * the local projections of A x onto y's frames, left to right, enriched by the
 * residual approximation z ~ A x - y (updated in the same sweep), then rounds
 * y at eps (truncated-SVD sweep and delta rule of Sec. 2.2, cap max_rank;
 * 0 = capacity).
 *  y: in/out, the initial guess on entry (any ranks within its capacities),
 *     the result on return.  y->cap[k] must be >= min(max_rank, the natural
 *     rank bound of bond k) (QT_EINVAL otherwise).
 *  z: in/out, the residual guess (its ranks set the enrichment width, e.g. 4
 *     to 16); the updated residual approximation on return.
 *  err_out: device [B] (may be null), the last sweep's rounding error of y
 *     relative to its norm.
 * Batches: x, y, z share the batch; A is shared or per instance (inst_group).
 * A must be square on x's modes.  Both y and z are first made
 * right-orthogonal by a QR sweep from their last cores (exact: ranks become
 * min(r_k, p_k r_{k+1})), and z again after every sweep.  Workspace grows as
 * needed. */
qt_status tt_amen_mv(qt_ctx ctx, const qt_mpo* A, const qt_tt* x, qt_tt* y, qt_tt* z, double eps,
                     int32_t max_rank, int32_t sweeps, double* err_out);

/* out[b] = scale * Re <y_b, Q y_b> for an operator train Q (used with
 * Q = A^H A to get ||A y||^2 exactly without forming A y). */
qt_status tt_sandwich(qt_ctx ctx, const qt_mpo* Q, const qt_tt* y, double scale, double* out);

/* ---- Algorithm 2 ------------------------------------------------------------ */

/* Operands of one cell problem on a 2^L-per-axis grid: core 0 is the
 * component (control) core of mode d, cores 1..3L the x, y, z bits.
 * Scalar conductivity (Sec. 3.1 in its conductivity form): d = 3 (gradient
 * components).  Linear elasticity (Sec. 3.1, App. A): d = 6 (Voigt strain
 * with engineering shears), Kp the Voigt operator C - C0 (a full 6 x 6
 * component core), G the Green-Eshelby operator (6 x 6 component core), kp
 * absent (n = 0) and G2 = G^H G given. */
typedef struct {
  int32_t L;
  qt_tt kp;                 /* k' = k - k0, all-ones control core (n = 0: the    */
                            /* material acts through Kp on every path)           */
  qt_mpo Kp;                /* the material operator (k' as a diagonal operator, */
                            /* or C - C0)                                        */
  qt_mpo K2;                /* Kp^H Kp: ||Kp e||^2 = <e, K2 e>                   */
  double k0;                /* reference conductivity: ||G t||^2 = <t, G t>/k0   */
  qt_mpo S;                 /* SFFT operator (Q_L per axis, identity on core 0)  */
  qt_mpo Sinv;              /* its adjoint                                       */
  qt_mpo G;                 /* Green operator, momentum convention, diag spatial */
  qt_tt E;                  /* rank-1 mean field(s), batch = field batch         */
  const double* E_norm;     /* host [B]: |E| of each load                        */
  qt_tt SE;                 /* S applied to E (rank 1, batch = field batch);     */
                            /* read by the sketch modes, which round the last    */
                            /* step as S^dagger (S E - eps^) = E - S^dagger eps^ */
  qt_mpo G2;                /* G^H G for ||G t||^2 = <t, G2 t> (n = 0: use the   */
                            /* projector identity <t, G t>/k0 of conductivity)   */
} qt_operands;

typedef struct {
  qt_round_opts round;      /* applied after every step                          */
  double tol;               /* residual tolerance delta_tol                      */
  int32_t max_iter;
  int32_t graph;            /* ls_iterate, sketch mode: capture one iteration in */
                            /* a HIP graph and replay it (no host work between   */
                            /* iterations); ignored in the other modes, with the */
                            /* rank log or the kernel-class timing on            */
} qt_solve_opts;

/* n_iter basic-scheme iterations (Algorithm 2) on the field batch e (in/out):
 *   tau = round(k' (.) e); tau^ = round(S tau); eps^ = round(G tau^);
 *   e' = round(E - S^dagger eps^); r = ||e' - e||_F / (|E| N^{3/2}).
 * In the sketch and learned modes every rounding acts on the product
 * structure, and the last one rounds S^dagger t with t = S E - eps^ (the rank-1
 * term S E is added before the rounding, so there are four roundings).
 * residual_out: device [n_iter][B] doubles (may be NULL).
 * e->cap must hold opts->round.max_rank on every bond.
 * Capacity: every truncated SVD runs on a block of at most 1024 columns
 * (rank cap + oversampling on the bonds of the sketch modes; r_A r_x on the
 * materializing path), so max_rank + oversample <= 1024 / 2 on the 2-mode
 * bonds; larger blocks return QT_ECAPACITY before any launch.  The
 * workspace of a solve is given by qt_ls_workspace_query. */
qt_status ls_iterate(qt_ctx ctx, const qt_operands* ops, qt_tt* e, const qt_solve_opts* opts,
                     int32_t n_iter, double* residual_out);

/* Full solve: e_0 = E (per instance), iterate until every residual < tol or
 * max_iter; then A_eff[b][c] = Re <k_sel[c], e_b> / N^3 (Appendix A).
 * k_sel: d TTs (d = the field's component mode), train c holding row c of
 *   the material (k e_c for conductivity, row c of C in Voigt form for
 *   elasticity), each one train for every field or one per field
 *   (batch = e->batch); A_eff[b][c] is then the mean flux or the mean stress
 *   component c: column j of the effective tensor for the load e_j.
 * e: field batch used as the iterate (capacities as for ls_iterate).
 * A_eff: host [B][d], each field's from its iterate at the iteration where
 *   its residual first fell below tol (fields of a batch that converge early
 *   keep iterating with the others, but their A_eff is taken then, as a
 *   separate solve would take it; fields that do not converge: the last
 *   iterate); iters: host [B] (iterations to convergence);
 * residuals: host [max_iter][B] (may be NULL). */
qt_status homogenize(qt_ctx ctx, const qt_operands* ops, const qt_tt* k_sel, qt_tt* e,
                     const qt_solve_opts* opts, double* A_eff, int32_t* iters,
                     double* residuals);

/* Workspace bytes ls_iterate (k_sel NULL) or homogenize (k_sel = its three
 * selector trains) needs for this field batch, operands and options: the
 * iteration arena plus, in the sketch modes, the persistent learned-rank
 * state used by learned rounding and rank logging (it stays taken after the
 * solve, so a later call of another kind on the same caller-owned context
 * needs its own query added).  Rank or rounding logs (qt_ranklog_enable,
 * qt_learn_log_enable) need capacity * 100 + 768 (24 feature floats and a
 * label per row) and capacity * 48 + 512 (6 doubles per row) bytes more.  A
 * caller-owned context of qt_ctx_fixed_bytes() + *bytes runs that solve.
 * Host-only, launches nothing.  Errors as ls_iterate's argument checks. */
qt_status qt_ls_workspace_query(const qt_operands* ops, const qt_tt* k_sel, const qt_tt* e,
                                const qt_solve_opts* opts, size_t* bytes);


/* ---------------------------------------------------------------------------
 * Learned-rank rounding (rank predictor).  The method's fixed-rank truncation
 * (Sec. 2.2, "prescribe a fixed number of singular values") and its
 * coarse-grained rank classes r_c = c * r_0 (Sec. 5.1) are combined with a
 * small FP32 MLP that predicts each bond's rank from the previous iteration's
 * sketched spectrum, so that the product-aware rounding can skip its SVD
 * truncation sweep.  Batches: every instance's features are predicted, and
 * the sketch takes the largest prediction of the batch per bond.  The exact
 * a-posteriori error of each instance decides, on the device: above eps, or
 * above max(eps, accept * e_s) when e_s > eps, where e_s is the error estimate
 * (sqrt(e_proj^2 + tails^2)) of the last SVD-truncated rounding of the same
 * step and instance (e_s > eps only where the rank cap binds), the instance is
 * redone with the SVD-truncated sketch rounding (fallback, counted; the host
 * reads only the number of fallbacks and skips the redo when it is zero).  The
 * tolerance eps always holds; accept only scales the comparison with the SVD
 * truncation where the cap binds.  With accept <= 1 every rounding is as
 * accurate as the SVD truncation would be (to the drift of e_s between its
 * refreshes, which happen at every fallback).  ls_iterate does not capture
 * the learned path in a graph (its predicted widths are launch parameters).
 * ------------------------------------------------------------------------- */

/* Number of floats in the MLP parameter vector for n_in inputs and n_cls
 * classes (three hidden tanh layers of 64; W row-major [in][out], then bias,
 * for each of the four layers). */
int32_t qt_mlp_num_params(int32_t n_in, int32_t n_cls);

/* One full-batch training step of the MLP on the context's stream.
 * params, adam_m, adam_v: device [num_params] floats (in/out; Adam moments,
 *   zero-initialised by the caller; may be NULL when lr <= 0).
 * step: Adam step number (>= 1, for bias correction).
 * X: device [n][n_in] features; labels: device [n] classes in [0, n_cls).
 * Loss = mean over samples of cross-entropy + beta * sum_c p_c w(c, y), with
 *   w(c, y) = (c - y)/n_cls above the label and gamma below it.
 * lr <= 0: no update (gradient evaluation only).
 * loss_out: device float (may be NULL); grad_out: device [num_params] floats
 *   holding the mean gradient (may be NULL).
 * Errors: QT_EINVAL for NULL inputs or n_in > 32, n_cls outside [2, 32]. */
qt_status qt_mlp_train_step(qt_ctx ctx, float* params, float* adam_m, float* adam_v,
                            int32_t step, const float* X, const int32_t* labels, int32_t n,
                            int32_t n_in, int32_t n_cls, float lr, float beta, float gamma,
                            float* loss_out, float* grad_out);

/* MLP inference on device features X [n][n_in].  logits: device [n][n_cls]
 * (may be NULL).  ranks: device [n] (may be NULL): rank 8 (c + 1) of the
 * smallest class c whose cumulative softmax probability reaches quantile,
 * clipped to rank_cap[i] when rank_cap (device [n]) is given. */
qt_status qt_mlp_infer(qt_ctx ctx, const float* params, const float* X, int32_t n,
                       int32_t n_in, int32_t n_cls, float quantile, float* logits,
                       int32_t* ranks, const int32_t* rank_cap);

/* Rank log (training data): while enabled (capacity > 0), every SVD-truncated
 * product-aware rounding inside ls_iterate appends, per bond, the features of
 * the previous iteration's same step and the class min(ceil(r / 8), n_cls) - 1
 * of the rank r it kept.  capacity == 0 disables and frees the log. */
qt_status qt_ranklog_enable(qt_ctx ctx, int32_t capacity, int32_t n_cls);

/* Number of logged samples (*count, host) and a copy of the first
 * min(count, max_count) of them into caller-owned device buffers
 * features [max_count][24] and labels [max_count] (stream-ordered; may be
 * NULL when max_count == 0).  Errors: QT_EINVAL when the log is not enabled. */
qt_status qt_ranklog_get(qt_ctx ctx, float* features, int32_t* labels, int32_t max_count,
                         int32_t* count);

/* Installs the predictor for QT_ROUND_LEARNED (params: device, borrowed; must
 * stay valid while used).  quantile in (0, 1]: class choice (see qt_mlp_infer);
 * accept_factor in (0, 2]: a learned rounding is kept iff its relative error
 * is at most eps, or at most max(eps, accept_factor * e_s) where e_s > eps
 * (<= 0: 1).  Errors: QT_EINVAL for
 * other values, n_cls outside [2, 32] or quantile outside (0, 1]. */
qt_status qt_set_predictor(qt_ctx ctx, const float* params, int32_t n_cls, float quantile,
                           float accept_factor);

/* Forgets the previous-iteration features and reference errors (call before
 * iterating a new field from its start). */
qt_status qt_learn_reset(qt_ctx ctx);

/* Learned-rounding log (diagnostics): while enabled (capacity > 0), every
 * learned rounding appends one row per instance of QT_LEARN_LOG_COLS = 6
 * doubles: iteration count of the context, step (0 Hadamard, 1 SFFT, 2 Green,
 * 3 inverse SFFT), instance, its exact relative error, the reference e_s of
 * that step and instance (0 before the first SVD-truncated rounding), and 1 if
 * kept, 0 if it fell back.  capacity == 0 disables and frees the log.
 * qt_learn_log_get copies min(count, max_rows) rows to the HOST buffer rows
 * and returns the number logged in *count (synchronizes the stream).
 * Errors: QT_EINVAL when the log is not enabled or an argument is null. */
qt_status qt_learn_log_enable(qt_ctx ctx, int32_t capacity);
qt_status qt_learn_log_get(qt_ctx ctx, double* rows, int32_t max_rows, int32_t* count);

#ifdef __cplusplus
}
#endif
#endif /* QTTHOM_H */
