/* tt.h - C ABI of the MI355X (gfx950) solver for linear systems with
 * Kronecker product structure (Chen & Kressner, "Recursive blocked algorithms
 * for linear systems with Kronecker product structure", arXiv 1905.09539).
 *
 * Equations (paper notation; X x_mu A is the mu-mode product of Sec. 2,
 * defined by (X x_mu A)_(mu) = A X_(mu)):
 *
 *   Laplace-like form, eq. (1.4) / (2.2):
 *       X x_1 A_1 + X x_2 A_2 + ... + X x_d A_d = B
 *   Pair form (the family with two matrices per mode, Conclusions):
 *       sum_mu X x_1 C_1 ... x_mu A_mu ... x_d C_d = B
 *
 * Conventions shared by every entry point
 *   - d is the tensor order, 1 <= d <= 4 (solve_tri_tensor, its plans and
 *     solve_general_tensor also take d = 5: the two adjacent modes with the
 *     smallest product of sizes are merged, see tt_merge_modes_host); n[0..d-1]
 *     are the mode sizes (n[mu] >= 0; a zero-sized mode makes the call a
 *     no-op).
 *   - Tensors (B, X, G, dB, ...) are DEVICE pointers to float64 data in
 *     C order: the LAST mode is the fastest, element (i_1..i_d) sits at
 *     sum_mu i_mu * prod_{nu > mu} n[nu].  This is the reverse of the
 *     paper's column-major vec(); the solution is the same tensor.
 *   - Coefficients are passed as a HOST array of d DEVICE pointers, each to a
 *     row-major n[mu] x n[mu] float64 matrix.
 *   - "Upper quasi-triangular" is the real Schur form of Sec. 2 (Algorithm 1):
 *     zero below the first subdiagonal, and no two consecutive nonzero
 *     subdiagonal entries; a nonzero T[i+1][i] marks a 2x2 diagonal block.
 *   - The caller owns every buffer; the library keeps no pointer to caller
 *     memory after a call returns (plans keep only their own copies).
 *   - Work is ordered on opts->stream (NULL = the null stream).  The
 *     solve_* calls synchronise that stream once at the end to read the
 *     device status word; tt_plan_solve does not (see tt_plan_status).
 *   - Every function returns a tt_status; no exception crosses the ABI.
 *     tt_last_error() returns a thread-local description of the last failure.
 *   - Not re-entrant on one plan: calls that share a plan must be ordered.
 */
#ifndef TT_H_
#define TT_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TT_OK = 0,
    TT_EINVAL = 1,      /* bad argument, shape or coefficient structure      */
    TT_ESINGULAR = 2,   /* an eigenvalue sum vanished (uniqueness fails,
                           Sec. 2) or a non-finite value appeared            */
    TT_ENOMEM = 3,      /* device or host allocation failed                 */
    TT_EHIP = 4,        /* a HIP runtime call failed                        */
    TT_ENOTCONV = 5     /* mixed-precision refinement did not reach tol     */
} tt_status;

typedef enum {
    TT_FP64 = 0,        /* all arithmetic in float64                         */
    TT_MP_FP32 = 1,     /* updates/transforms in FP32, FP64 refinement       */
    TT_MP_BF16 = 2      /* updates/transforms as three-term BF16 MFMA
                           products (six per pair, FP32 accumulation),
                           FP64 refinement                                   */
} tt_prec;

typedef struct {
    int nmin;           /* leaf block edge per mode (the paper's n_min,
                           Algorithm 2); 0 = default (16 for d<=3, 8 for d=4) */
    int prec;           /* tt_prec                                           */
    double tol;         /* refinement stop: ||D||_F / ||X||_F <= tol, or
                           from the second correction on, contraction
                           rho = ratio_k / ratio_{k-1} < 1/2 with
                           rho * ratio_k <= tol (the next correction, about
                           the error left in X, would be below tol)        */
    int max_iter;       /* refinement iteration cap                          */
    int deterministic;  /* accepted for interface stability: every path is
                           bitwise reproducible run to run (each output is
                           written by one workgroup per launch, accumulation
                           orders are fixed, no floating-point atomics)      */
    void* stream;       /* hipStream_t                                       */
    void* workspace;    /* DEVICE memory owned by the caller, or NULL.  When
                           set, every device buffer of the call (or of the
                           plan built from these options) is carved from it
                           and the library calls no device allocator; it must
                           stay valid, and not be used by anything else,
                           until the call returns (for a plan: until
                           tt_plan_destroy).  tt_workspace_bytes gives a
                           sufficient size; a smaller one fails with
                           TT_ENOMEM and the needed size in tt_last_error. */
    size_t workspace_bytes;
    double info[4];     /* out: [0] refinement iterations, [1] last
                           ||D||_F/||X||_F, [2] plan build seconds,
                           [3] device solve milliseconds (when timed)        */
} tt_opts;

/* Upper bound of the device workspace (bytes) that one single-problem call
 * of solve_tri_tensor (Laplace-like or pair form), solve_general_tensor,
 * solve_backward, solve_gsylv_tensor or solve_gsylv_general_tensor with order
 * d, mode sizes n[0..d-1], precision prec (tt_prec) and the default leaf
 * size (opts->nmin = 0) needs, whatever the coefficients' 2x2-block pattern.
 * Host-only; 0 on invalid arguments.  Batched calls need the sum over their
 * problems. */
size_t tt_workspace_bytes(int d, const int64_t* n, int prec);

/* Fill *o with defaults (nmin 0, TT_FP64, tol 1e-13, max_iter 10, stream and
 * workspace NULL). */
int tt_opts_default(tt_opts* o);

/* Human-readable name of a status code (static storage). */
const char* tt_status_str(int status);

/* Thread-local message describing the last failure on this thread. */
const char* tt_last_error(void);

/* ---------------------------------------------------------------------------
 * solve_tri_tensor - triangular solve (Algorithm 2 of the paper, recursion on
 * the largest mode with the bump-aware split of Sec. 2.1, with Algorithm 3's
 * merging of small modes).
 *   T[mu]: upper quasi-triangular coefficients A_mu (device).
 *   C:     NULL for the Laplace-like form, else a host array of d device
 *          pointers to UPPER TRIANGULAR C_mu with nonzero diagonal (pair
 *          form).  The pair operator equals the Laplace-like operator of
 *          T'_mu = C_mu^{-1} A_mu followed by x_1 C_1 ... x_d C_d (products
 *          in different modes commute), so the pair form is solved as
 *          X = L(T')^{-1}(B x_1 C_1^{-1} ... x_d C_d^{-1}); T'_mu and C_mu^{-1}
 *          are formed on the host, the products run on the GPU.
 *   B:     right-hand side (device, read only unless X == B).
 *   X:     solution (device); X may alias B (FP64 only).
 *   opts->prec: TT_MP_FP32 or TT_MP_BF16 (Laplace-like form only) solves
 *          with FP32-MFMA (or split-BF16 MFMA) recursion updates and FP64
 *          leaves, and refines in FP64 with the residual
 *          B - sum_mu X x_mu T_mu; X must not alias B.
 * Errors: TT_EINVAL (d, n, NULL pointer, T not quasi-triangular, C not
 * triangular), TT_ESINGULAR (zero pivot or non-finite result; X content is
 * then unspecified), TT_ENOTCONV, TT_ENOMEM, TT_EHIP.
 * ------------------------------------------------------------------------- */
int solve_tri_tensor(int d, const int64_t* n, const double* const* T,
                     const double* const* C, const double* B, double* X,
                     tt_opts* opts);

/* ---------------------------------------------------------------------------
 * solve_tri_tensor_noalloc - solve_tri_tensor for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation): the same arguments, kernels and
 * result, but every device buffer of the call (plan tables, coefficient
 * copies, update accumulators, pair-form transforms, status word) lives in
 * a fixed scratch array of 64 MiB that the library holds on each GPU it
 * runs on until the process ends; no hipMalloc/hipFree or allocating
 * library routine is called, and every launch goes to opts->stream (no
 * side stream, no events).  Enough for a d = 3 problem of about 150^3
 * elements (two accumulators of 8 N bytes plus tables).
 *   Argument meaning, layout and ownership: as solve_tri_tensor.
 *   opts->prec must be TT_FP64; opts->workspace is ignored.
 *   Calls on one GPU share its scratch array: calls that overlap in time on
 *   one GPU (other host threads, or streams not ordered with each other)
 *   race and give wrong results.  The array keeps the last call's contents;
 *   the call itself clears what must start at zero (the status word).
 * Errors: as solve_tri_tensor; TT_EINVAL also when the problem needs more
 * than the scratch array holds (the message gives the size needed).
 * ------------------------------------------------------------------------- */
int solve_tri_tensor_noalloc(int d, const int64_t* n, const double* const* T,
                             const double* const* C, const double* B, double* X,
                             tt_opts* opts);

/* ---------------------------------------------------------------------------
 * solve_general_tensor - Algorithm 1 of the paper for dense coefficients:
 * real Schur decomposition A_mu = U_mu T_mu U_mu^T on the host (Hessenberg
 * reduction + Francis double-shift QR), B~ = B x_1 U_1^T ... x_d U_d^T on the
 * GPU, the triangular solve, and X = X~ x_1 U_1 ... x_d U_d on the GPU.
 *   A_host[mu]: HOST pointers to dense row-major n[mu] x n[mu] matrices.
 *   B, X: device tensors; X may alias B.
 * opts->prec selects FP64, TT_MP_FP32 or TT_MP_BF16: transforms and recursion
 * updates in FP32 MFMA (TT_MP_BF16: each FP64 operand split into three BF16
 * terms, six BF16 MFMA products per pair) with FP32 accumulation, leaf
 * solves (with their divisions by
 * eigenvalue sums) in FP64, and FP64 iterative refinement with the residual
 * B - sum_mu X x_mu A_mu of the dense A_mu (X must not alias B then).
 * opts->info[0..2] report the refinement iterations, the last ratio
 * ||D||_F/||X||_F and the host seconds (Schur + planning).
 * Errors: as solve_tri_tensor, plus TT_EINVAL if the QR iteration does not
 * converge, TT_ENOTCONV if refinement stops above opts->tol.
 * ------------------------------------------------------------------------- */
int solve_general_tensor(int d, const int64_t* n, const double* const* A_host,
                         const double* B, double* X, tt_opts* opts);

/* ---------------------------------------------------------------------------
 * solve_backward - adjoint of solve_tri_tensor (Laplace-like form) for a
 * scalar loss L with dL/dX = G:
 *   Lam solves sum_mu Lam x_mu T_mu^T = G   (lower quasi-triangular system),
 *   dB = Lam,
 *   dT[mu] = -Lam_(mu) X_(mu)^T, masked to the quasi-triangular pattern of
 *            T[mu] (upper triangle + nonzero bump subdiagonal) unless
 *            dense_grad != 0.
 *   X: the forward solution (device).  dB: device tensor (may alias G).
 *   dT: host array of d device pointers to n[mu] x n[mu] outputs, or NULL to
 *       skip the coefficient gradients; individual entries may be NULL.
 *   The adjoint system is solved by the same kernels in reversed index
 *   order; dT is a split-K FP64-MFMA product (workspace allocated inside).
 * Errors: as solve_tri_tensor.
 * ------------------------------------------------------------------------- */
int solve_backward(int d, const int64_t* n, const double* const* T,
                   const double* X, const double* G, double* dB,
                   double* const* dT, int dense_grad, tt_opts* opts);

/* ---------------------------------------------------------------------------
 * The second operator class of the paper, eq. (1.5) / (3.1) (generalized
 * Sylvester equations with Kronecker structure, Sec. 3):
 *     X x_1 A_1 + X x_1 C x_2 A_2 x_3 ... x_d A_d = B,
 * matrix I (x) .. (x) I (x) A_1 + A_d (x) .. (x) A_2 (x) C.  The solution is
 * unique iff the pencil A_1 + lambda C is regular and none of its
 * eigenvalues is an eigenvalue of -A_d (x) .. (x) A_2 (Sec. 3).  With
 * A_1 = -lambda I this is the shifted Kronecker product of eq. (1.6).
 *
 * solve_gsylv_tensor: triangular coefficients (the output of Algorithm 4's
 *   reductions): A[mu] DEVICE pointers to upper quasi-triangular n[mu] x n[mu]
 *   matrices (row-major), C a DEVICE pointer to an upper triangular n[0] x
 *   n[0] matrix with nonzero diagonal.  The equation is reduced exactly by
 *   C^{-1} along mode 1: X x_1 (C^{-1} A_1) + X x_2 A_2 .. x_d A_d =
 *   B x_1 C^{-1} (C^{-1} A_1 keeps the pattern of A_1); orders 1 and 2 are
 *   then Laplace-like, orders 3 and 4 run the recursion of Algorithm 5 as
 *   the hyperplane schedule of solve_tri_tensor with the second-class
 *   updates (up to d products, telescoped through partial products) and
 *   leaves.  d = 1 .. 4.
 * solve_gsylv_general_tensor: dense coefficients, Algorithm 4: host QZ of
 *   (A_1, C), host real Schur of A_2 .. A_d, the transforms on the GPU.
 *   A_host[mu], C_host: HOST row-major matrices.
 * B, X: device tensors as for solve_tri_tensor; X may alias B.  FP64 only
 * (opts->prec must be TT_FP64).  opts->nmin = 0 takes 8 (d = 3) / 5 (d = 4).
 * Errors: TT_EINVAL (arguments, structure, C not upper triangular or with a
 * zero diagonal entry, no QZ / QR convergence), TT_ESINGULAR (zero pivot or
 * non-finite value: the uniqueness condition fails), TT_ENOMEM, TT_EHIP.
 * ------------------------------------------------------------------------- */
int solve_gsylv_tensor(int d, const int64_t* n, const double* const* A, const double* C,
                       const double* B, double* X, tt_opts* opts);
int solve_gsylv_general_tensor(int d, const int64_t* n, const double* const* A_host,
                               const double* C_host, const double* B, double* X,
                               tt_opts* opts);

/* Batched forms: count independent problems of possibly different shapes,
 * solved together (one launch sequence for the whole batch).  d[b], n[b],
 * T[b], B[b], X[b] describe problem b exactly as in solve_tri_tensor
 * (Laplace-like form only).  dT may be NULL; dT[b] follows solve_backward. */
int solve_tri_tensor_batched(int count, const int* d, const int64_t* const* n,
                             const double* const* const* T,
                             const double* const* B, double* const* X,
                             tt_opts* opts);
int solve_backward_batched(int count, const int* d, const int64_t* const* n,
                           const double* const* const* T,
                           const double* const* X, const double* const* G,
                           double* const* dB, double* const* const* dT,
                           int dense_grad, tt_opts* opts);


/* ---------------------------------------------------------------------------
 * Plans: the split/merge schedule and the coefficient structure of
 * solve_tri_tensor, built once and executed many times (host work and the
 * only device->host copies happen in tt_plan_create).
 *   tt_plan_create reads T (and C) from the device, validates them and keeps
 *     device copies; trans != 0 plans the adjoint system with T_mu^T.
 *   tt_plan_solve  enqueues the solve of B into X on stream (no host sync,
 *     no allocation); X may alias B.
 *   tt_plan_status synchronises the stream of the last solve and returns
 *     TT_ESINGULAR if that solve met a zero pivot or a non-finite value.
 *   tt_plan_flops  returns the method's flop count (one FMA = 2 flops):
 *     2 * sum_mu (n_mu (n_mu - 1) / 2 + bumps_mu) * N / n_mu for the
 *     Laplace-like form, plus per mode product of a pipeline 2 n_mu N for
 *     a dense matrix and (n_mu + 1) N for an upper triangular one (the
 *     pair form's C_mu^{-1}, whose zero blocks the product skips).
 *   Batched and adjoint plans are FP64 only; tt_plan_create with
 *     opts->prec = TT_MP_FP32 or TT_MP_BF16 (Laplace-like form) refines
 *     in FP64.
 * ------------------------------------------------------------------------- */
typedef struct tt_plan_s* tt_plan;

int tt_plan_create(tt_plan* out, int d, const int64_t* n, const double* const* T,
                   const double* const* C, int trans, const tt_opts* opts);
/* Dense coefficients (Algorithm 1): the host Schur decompositions happen
 * here; tt_plan_solve then runs B x_mu U_mu^T, the triangular solve and
 * x_mu U_mu on the GPU (and the refinement loop when opts->prec is
 * TT_MP_FP32 or TT_MP_BF16).  A_host: HOST pointers to row-major n[mu] x n[mu]
 * matrices. */
int tt_plan_create_general(tt_plan* out, int d, const int64_t* n,
                           const double* const* A_host, const tt_opts* opts);

/* Dense pairs: plan for  sum_mu X x_1 C_1 .. x_mu A_mu .. x_d C_d = B  with
 * general dense HOST coefficients A_host[mu], C_host[mu] (row-major n_mu x
 * n_mu, C_mu nonsingular), the pencil form of Sec. 3: host QZ per mode
 * (A = Q S Z^T, C = Q T Z^T, Algorithm 4's reduction), then on the GPU
 * B~ = B x_mu (T_mu^{-1} Q_mu^T), the triangular solve with T_mu^{-1} S_mu
 * (upper quasi-triangular) and X = X~ x_mu Z_mu.  Solve with tt_plan_solve
 * (B and X device row-major tensors of the plan's shape).  FP64 only.
 * Errors: TT_EINVAL (bad arguments, non-finite entries, mixed precision
 * requested, no QZ convergence), TT_ESINGULAR (some C_mu singular to working
 * precision), TT_ENOMEM. */
int tt_plan_create_general_pair(tt_plan* out, int d, const int64_t* n, const double* const* A_host,
                                const double* const* C_host, const tt_opts* opts);

/* Plans of the second class (see solve_gsylv_tensor): triangular
 * coefficients on the device (tt_plan_create_gsylv) or dense coefficients on
 * the host (tt_plan_create_gsylv_general, Algorithm 4).  Solve with
 * tt_plan_solve / tt_plan_solve_graph. */
int tt_plan_create_gsylv(tt_plan* out, int d, const int64_t* n, const double* const* A,
                         const double* C, const tt_opts* opts);
int tt_plan_create_gsylv_general(tt_plan* out, int d, const int64_t* n, const double* const* A_host,
                                 const double* C_host, const tt_opts* opts);

/* Coefficient gradients with a reusable plan (the adjoint's second half):
 * for every problem i of a triangular plan (tt_plan_create /
 * tt_plan_create_batched, typically the adjoint plan trans = 1 whose solve
 * gave Lam), dT[i][mu] = -Lam_(mu) X_(mu)^T for mu < d_i, masked to the
 * quasi-triangular pattern of T[i][mu] unless dense_grad.  T[i][mu]: the
 * problem's device coefficients (n_mu x n_mu row-major), X[i], Lam[i]: device
 * tensors of the problem's shape, dT[i][mu]: device n_mu x n_mu outputs
 * (dT[i] NULL skips problem i).  Enqueued on stream; the split-K workspace is
 * allocated by the plan on first use (and grown when a call needs more).
 * Errors: TT_EINVAL (NULL arguments, a pair-form or dense-coefficient plan),
 * TT_ENOMEM. */
int tt_plan_coefficient_grads(tt_plan plan, const double* const* const* T, const double* const* X,
                              const double* const* Lam, double* const* const* dT, int dense_grad, void* stream);
int tt_plan_create_batched(tt_plan* out, int count, const int* d,
                           const int64_t* const* n, const double* const* const* T,
                           int trans, const tt_opts* opts);
int tt_plan_solve(tt_plan plan, const double* B, double* X, void* stream);
/* The same solve replayed from a HIP graph: the first call for a (B, X,
 * stream) triple records the launch sequence of tt_plan_solve (status reset,
 * input copy, every wave's leaf and update launches on the stream and the
 * plan's side stream, joined by events) and instantiates it; later calls
 * with the same triple launch the graph, saving the per-launch host and
 * queue overhead of ~200 launches.  A different triple re-records (the
 * previous graph is released after its stream drains).  Only for
 * single-problem FP64 plans (mixed precision synchronises with the host);
 * stream must be a created stream, not the default one.  B and X keep the
 * meaning, layout and ownership of tt_plan_solve; the plan keeps the graph
 * until it is destroyed.  Errors: TT_EINVAL (NULL plan or stream, batched or
 * mixed-precision plan), TT_EHIP (capture or instantiation failed). */
int tt_plan_solve_graph(tt_plan plan, const double* B, double* X, void* stream);
/* Plain device copy of n doubles, src -> dst (device pointers, not
 * overlapping), enqueued on stream with the library's copy kernel: one read
 * and one write of 8 n bytes, the reference against which hardware byte
 * counters are calibrated.  Errors: TT_EINVAL (n < 0, NULL pointer with
 * n > 0), TT_EHIP. */
int tt_copy_device(const double* src, double* dst, int64_t n, void* stream);
int tt_plan_solve_batched(tt_plan plan, const double* const* B, double* const* X,
                          void* stream);
int tt_plan_status(tt_plan plan);
/* Profiling pass: the same work as tt_plan_solve with HIP timing events
 * around every kernel launch, each on the stream the launch is on;
 * synchronises.  serial != 0 puts every launch on the caller's stream (no
 * overlap of leaf and update kernels: each duration is the kernel alone).
 * out[12] receives, for kernel class k (0 = leaf solves, 1 = recursion
 * updates): out[4k] summed launch milliseconds, out[4k+1] algorithmic flops,
 * out[4k+2] algorithmic HBM bytes, out[4k+3] launches; out[8] = milliseconds
 * from the first leaf launch to the end of the last update. */
int tt_plan_profile(tt_plan plan, const double* B, double* X, void* stream, int serial, double* out);
/* The same profiled solve, reported per hyperplane wave: waves[6k .. 6k+5]
 * (k < cap; the plan's wave count is tt_schedule_info's out[3] for its
 * problem) = start and end of wave k's leaf launch, start and end of the
 * update launch that runs beside it (milliseconds from the first leaf
 * launch; -1 when the launch is empty), its leaf blocks and its update
 * tiles.  waves is host memory of at least 6 cap doubles, owned by the
 * caller.  Same plan restrictions and errors as tt_plan_profile. */
int tt_plan_profile_waves(tt_plan plan, const double* B, double* X, void* stream, int serial, double* waves,
                          int64_t cap);
double tt_plan_flops(tt_plan plan);
/* out[4]: [0] refinement iterations of the last solve, [1] its last
 * ||D||_F/||X||_F, [2] plan build seconds (host), [3] host Schur seconds. */
int tt_plan_info(tt_plan plan, double* out);
int tt_plan_destroy(tt_plan plan);

/* Host-only schedule query (no GPU): plans the triangular solve of one
 * problem with HOST coefficients T_host[mu] (row-major) and leaf edge nmin,
 * and fills out[14]: flops, leaf flops, update flops, waves, leaves, update
 * tasks, update tiles, kernel launches, the largest leaf edge per internal
 * mode (4 entries), a dependency check of the schedule (0 = every update
 * reads only solved blocks and every leaf has all its contributions), and
 * the device bytes a plan of this schedule takes (tables, coefficient
 * copies and update accumulators; the part of tt_workspace_bytes that
 * depends on the coefficients' 2x2-block pattern).
 * Errors: as tt_plan_create. */
int tt_schedule_info(int d, const int64_t* n, const double* const* T_host, int nmin, double* out);
/* The same query for the schedule of either operator class: cls 0 the
 * Laplace-like equation (2.2) (as tt_schedule_info), cls 1 the second class
 * of Sec. 3, eq. (3.1), after the C^{-1} reduction, with T_host the
 * triangular A_mu (its default leaf edge and update tiles differ; out[0..2]
 * count the Laplace-like flops of the same schedule).
 * Errors: as tt_schedule_info; TT_EINVAL for another cls. */
int tt_schedule_info_class(int d, const int64_t* n, const double* const* T_host, int nmin, int cls, double* out);

/* Host-only real Schur decomposition A = U T U^T of Algorithm 1 (Householder
 * Hessenberg reduction, Francis double-shift QR, standardised 2x2 blocks:
 * equal diagonal entries, off-diagonal entries of opposite sign).  A, T, U:
 * HOST row-major n x n arrays (A is not modified).  No GPU is used.
 * Errors: TT_EINVAL (bad arguments, non-finite entries, no convergence). */
int tt_schur_host(int n, const double* A, double* T, double* U);

/* Host-only real generalized Schur (QZ) decomposition of the pencil (A, C),
 * the host step of Algorithm 4 (Sec. 3): A = Q S Z^T, C = Q T Z^T with S
 * upper quasi-triangular (2x2 diagonal blocks only for complex eigenvalue
 * pairs), T upper triangular, Q and Z orthogonal (Householder QR of C, Givens
 * Hessenberg-triangular reduction, implicit double-shift QZ iteration).
 * A, C, S, T, Q, Z: HOST row-major n x n arrays (A and C are not modified).
 * No GPU is used.  Errors: TT_EINVAL (bad arguments, non-finite entries, no
 * convergence), TT_ESINGULAR (C singular to working precision). */
int tt_qz_host(int n, const double* A, const double* C, double* S, double* T, double* Q, double* Z);

/* Host-only merge of two adjacent modes (Algorithm 3, Sec. 2.2 for real
 * quasi-triangular coefficients): with Ta (na x na, the slower mode) and Tb
 * (nb x nb) upper quasi-triangular, the two terms of the merged mode act as
 * A' = Ta (x) I_nb + I_na (x) Tb on the merged index i_a nb + i_b.  A perfect
 * shuffle of the block rows of each 2x2 block of Ta makes A' block upper
 * triangular with diagonal blocks of size at most 4; the 4x4 ones are brought
 * to real Schur form.  Outputs (HOST, row-major, (na nb)^2 each): Tm upper
 * quasi-triangular and V orthogonal with A' = V Tm V^T, and perm[r] = the
 * merged index at position r of the shuffled order (na nb entries).  Order-5
 * calls of solve_tri_tensor and solve_general_tensor merge the adjacent pair
 * of modes with the smallest product of sizes this way.  na nb <= 4096.
 * Errors: TT_EINVAL (sizes, NULL, structure), or that of the 4x4 Schur step. */
int tt_merge_modes_host(int na, const double* Ta, int nb, const double* Tb, double* Tm, double* V, int* perm);

#ifdef __cplusplus
}
#endif
#endif /* TT_H_ */
