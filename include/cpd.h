/*
 * cpd.h -- C ABI of libcpd, an MI355X (gfx950) implementation of the Tensor Fox CPD hot path:
 * truncated-MLSVD compression of a dense third-order tensor, damped Gauss-Newton (dGN) on the
 * compressed core with Jacobi-preconditioned conjugate gradients, and uncompression.
 *
 * Source of every operation: F. B. Diniz, "Tensor decompositions and algorithms, with
 * applications to tensor learning" (thesis, 2019), ch.3 and ch.4.  Each entry point below names
 * the section it implements.
 *
 * Conventions shared by every call
 *  - Array arguments marked (device) are device pointers owned by the caller; the library never
 *    allocates or frees memory.  Scratch memory comes from a caller workspace `ws` of `ws_bytes`
 *    bytes (device), sized by the matching *_workspace_bytes query.  Arguments marked (host) are
 *    host pointers.
 *  - Tensors are dense, C-ordered T[i1][i2][i3] (i3 fastest).  Matrices are row-major.  Factor
 *    matrices W^(l) are I_l x R (rank-one terms are columns).  Only third-order tensors (L = 3)
 *    are supported, as in the thesis's regularisation.
 *  - `stream` is a hipStream_t passed as void* (NULL = default stream).  All work is
 *    stream-ordered; a call returns after enqueueing unless it says it synchronises.
 *  - Return value: CPD_OK or a negative cpd_status.  On error no output is written, except that
 *    CPD_E_HIP can leave outputs partially written.  Non-convergence is not an error; it is
 *    reported as a stop reason.
 *  - All dGN arithmetic is FP64.  Input tensors may be FP64, FP32 (promoted exactly to FP64) or
 *    BF16 (Gram and projection with FP32 accumulation, see cpd_params.compute_dtype).
 */
#ifndef CPD_H
#define CPD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  CPD_OK = 0,
  CPD_E_INVALID = -1,      /* bad size, rank, dtype, null pointer or parameter */
  CPD_E_WORKSPACE = -2,    /* workspace missing or smaller than the query returned */
  CPD_E_HIP = -3,          /* a HIP runtime call failed (message in cpd_last_error) */
  CPD_E_NONFINITE = -4,    /* NaN or Inf met in the input tensor or initial factors */
  CPD_E_ZERO_TENSOR = -5,  /* ||T|| = 0: relative errors are undefined */
  CPD_E_UNSUPPORTED = -6   /* a size beyond the documented limits of a kernel */
} cpd_status;

typedef enum { CPD_F64 = 0, CPD_F32 = 1, CPD_BF16 = 2 } cpd_dtype;

/* Stopping conditions 1-7 of ch.4 "Stopping conditions", in the thesis's order, then maxiter. */
typedef enum {
  CPD_STOP_NONE = 0,
  CPD_STOP_REL_ERR = 1,      /* ||S - S_k|| / ||S|| < tol */
  CPD_STOP_STEP = 2,         /* ||x_k|| < tol (dGN step before norm balancing) */
  CPD_STOP_IMPROVEMENT = 3,  /* |err_{k-1} - err_k| < tol */
  CPD_STOP_GRAD = 4,         /* ||grad F||_inf < tol */
  CPD_STOP_AVG_ERR = 5,      /* windowed average error stopped decreasing */
  CPD_STOP_AVG_IMPR = 6,     /* windowed average improvement < 1e-3 * average error */
  CPD_STOP_DIVERGED = 7,     /* err_k > max(1, ||T||^2) / (1e-16 + tol) */
  CPD_STOP_MAXITER = 8
} cpd_stop;

typedef enum {
  CPD_INIT_RANDOM = 0,  /* N(0,1) entries (ch.4 "Initialization"); from W0 if given, else the
                           library's counter-based generator seeded by params.seed */
  CPD_INIT_MLSVD = 1,   /* R largest-|s| core entries on canonical vectors (ch.4 "Initialization") */
  CPD_INIT_GIVEN = 2    /* W0 used as is */
} cpd_init;

typedef struct {
  int32_t maxiter;          /* dGN iteration limit (thesis default 200) */
  double tol;               /* tolerance of every stopping condition (thesis default 1e-6) */
  double mlsvd_tol;         /* compression tolerance: smallest R~_l with tail energy ratio
                               < mlsvd_tol / 3 (ch.4 Alg. Compression); default 1e-6 */
  double init_damp;         /* tau; mu_0 = tau * mean|S| (ch.4 "Main parameters"); default 1 */
  double cg_tol;            /* CG stops when ||r||^2 < cg_tol; <= 0 means tol */
  int32_t cg_fixed;         /* > 0: fixed CG iteration cap; 0: random cap per iteration k drawn
                               uniformly from [1 + ceil(k^0.4), 2 + ceil(k^0.9)] (ch.4 CG) */
  const double* cg_uniforms;/* (host) maxiter uniform draws in [0,1) that select the random cap,
                               or NULL for the library's SplitMix64(seed, k) stream */
  uint64_t seed;            /* seed of the library's own random streams */
  int32_t init;             /* cpd_init */
  int32_t core_dims[3];     /* all > 0: fixed core size instead of the truncation rule */
  int32_t compute_dtype;    /* precision of the compression Grams for FP32/FP64 input:
                               CPD_F64 (default, FP64 accumulation) or CPD_BF16 (BF16 MFMA with
                               FP32 accumulation; the core is still projected from the input) */
  int32_t refine_iters;     /* > 0: after uncompression, up to this many further dGN iterations on
                               T itself (refinement in the original space, ch.4 benchmarks),
                               continuing the compressed run's damping parameter and CG-cap schedule;
                               the stopping rules apply with errors relative to ||T||.  Default 0 */
  int32_t st_mlsvd;         /* nonzero: sequentially truncated compression (ch.2 Alg. ST-MLSVD):
                               mode l's Gram, eigenvectors and truncation are taken on the tensor
                               already projected in modes 1..l-1; default 0 (the classic truncated
                               MLSVD of ch.4 Alg. Compression) */
  int32_t precond;          /* CG preconditioner: 0 (default) the diagonal M = diag(J^T J) + mu D
                               of ch.4; 1 block-Jacobi, the diagonal blocks Pi^(l) + mu diag(gamma_l)
                               of J^T J + mu D split by their Cholesky factors (the block-diagonal
                               preconditioner of ch.4 "Tensor Fox vs. other implementations").
                               Cores whose dGN runs in one workgroup's LDS only; others, the batched
                               solver and the tensor-train route return CPD_E_UNSUPPORTED */
  int32_t drawback;         /* nonzero: when an iteration's error exceeds 100 times the previous
                               one (ch.4 "Conditioning"), redo it from N(w_k) - x, the balanced
                               point drawn back by the step x, with a dogleg step inside the trust
                               radius ||x|| / 2 (Madsen-Nielsen-Tingleff).  Same support as precond */
} cpd_params;

/* Fills the thesis's defaults (maxiter 200, tol 1e-6, mlsvd_tol 1e-6, tau 1, random CG cap). */
void cpd_default_params(cpd_params* p);

/* Per-iteration record of the dGN (ch.4 "Updates" and "Stopping conditions"). */
typedef struct {
  int32_t k;             /* iteration number, 1-based */
  int32_t cg_iters;      /* CG iterations performed */
  int32_t cg_cap;        /* CG iteration cap used */
  int32_t stop;          /* cpd_stop after this iteration (0 = continue) */
  double rel_err;        /* ||S - S_k|| / ||S|| after the update */
  double step_norm;      /* ||x_k|| */
  double grad_inf;       /* ||grad F||_inf at the start point of the iteration */
  double gain;           /* gain ratio g */
  double mu;             /* damping parameter after the update rule */
  double cg_resid;       /* final ||r||^2 of CG */
  int64_t t_ns;          /* device time at the end of this iteration, in ns since the state's
                            initialisation ended (in-kernel wall-clock stamps) */
  int32_t drew_back;     /* 1 if the iteration was redone from the drawn-back point
                            (cpd_params.drawback) */
  int32_t reserved;      /* 0 */
} cpd_step_info;

typedef struct {
  int32_t iters;           /* dGN iterations performed */
  int32_t stop_reason;     /* cpd_stop */
  int32_t core_dims[3];    /* R~_l chosen by compression */
  int32_t tol_iter;        /* first iteration with rel_err < tol, or -1 */
  double rel_err_core;     /* final ||S - S_k|| / ||S|| */
  double rel_err_full;     /* ||T - sum_r lambda_r w_r^(1) o w_r^(2) o w_r^(3)|| / ||T|| */
  double t_norm;           /* ||T|| */
  int32_t refine_iters;    /* refinement iterations performed (cpd_params.refine_iters) */
  int32_t refine_stop;     /* cpd_stop of the refinement (0 if none ran) */
  int64_t time_to_tol_ns;  /* device time from the call's first kernel (T resident, compression
                              included) to the end of iteration tol_iter, from in-kernel
                              wall-clock stamps; -1 if the error never fell below tol.  Batched
                              solves count from the member's dGN start (compression excluded) */
} cpd_solve_info;

/* Last error message of the calling thread (static storage, never NULL). */
const char* cpd_last_error(void);

/* Library version string. */
const char* cpd_version(void);

/* ------------------------------------------------------------------------------------------ */
/* Compression: ch.2 Alg. MLSVD (left singular vectors via the Gram T_(l) T_(l)^T, App. B),    */
/* ch.4 Alg. Compression (P_l = min(I_l, R), truncation rule) and the core                    */
/* S = (U^(1)T, U^(2)T, U^(3)T) . T.                                                           */
/* ------------------------------------------------------------------------------------------ */

/* Workspace bytes needed by cpd_compress and cpd_solve for this problem. */
size_t cpd_workspace_bytes(const int64_t dims[3], int32_t R, const cpd_params* p);

/*
 * cpd_compress: truncated MLSVD of T.
 *   T          (device) dims[0]*dims[1]*dims[2] elements of `dtype`, C order.
 *   U_out[l]   (device) capacity dims[l]*P_l doubles, P_l = min(dims[l], R) (or core_dims[l]);
 *              receives U^(l) as a dims[l] x R~_l row-major matrix with orthonormal columns,
 *              each column signed so its largest-magnitude entry is positive.
 *   sigma_out[l] (device, nullable) capacity P_l doubles: leading mode-l singular values.
 *   S_out      (device) capacity P_1*P_2*P_3 doubles: the core, R~_1 x R~_2 x R~_3, C order.
 *   core_dims_out (host) receives R~_l.
 * Synchronises `stream` (the truncation ranks are read back).  Limits: I_l <= 4096,
 * P_l <= 64 when I_l > 64.
 */
cpd_status cpd_compress(const void* T, int32_t dtype, const int64_t dims[3], int32_t R,
                        const cpd_params* p, double* U_out[3], double* sigma_out[3], double* S_out,
                        int32_t core_dims_out[3], void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------------------------ */
/* dGN on the core: ch.4 "dGN" (residual, gradient, CG with cap, updates, damping rule,       */
/* stopping conditions) with J^T J v from ch.3 Thm Hv and D, M from ch.4 "Diagonal            */
/* regularization".                                                                            */
/* ------------------------------------------------------------------------------------------ */

/* Bytes of the device state buffer for a core of the given size. */
size_t cpd_state_bytes(const int32_t core_dims[3], int32_t R, const cpd_params* p);

/*
 * cpd_state_init: prepares a dGN state in `state` (device, cpd_state_bytes bytes): initial point
 * (p->init; W0 (device, nullable) holds three core_dims[l] x R row-major matrices packed one
 * after the other), norm balancing, mu_0 = tau * mean|S|, residual and MTTKRP at the start point.
 *   S (device) core, core_dims C order.  t_norm2: ||T||^2 for the divergence test (<= 0: ||S||^2).
 * Does not synchronise.
 */
cpd_status cpd_state_init(void* state, const double* S, const int32_t core_dims[3], int32_t R,
                          const double* W0, double t_norm2, const cpd_params* p, void* stream);

/*
 * cpd_dgn_step: one dGN iteration on the state; fills `info` (host).  Synchronises `stream`.
 * Calling it after a stop condition fired returns CPD_OK with info->stop set and changes nothing.
 */
cpd_status cpd_dgn_step(void* state, const double* S, const cpd_params* p, cpd_step_info* info,
                        void* stream);

/*
 * cpd_dgn_run: iterates until a stopping condition fires, all on the device (one persistent
 * workgroup).  `log` (host, nullable) receives up to `log_cap` per-iteration records.
 * Synchronises `stream`; returns the number of iterations in *iters and the reason in *stop.
 */
cpd_status cpd_dgn_run(void* state, const double* S, const cpd_params* p, int32_t* iters,
                       int32_t* stop, cpd_step_info* log, int32_t log_cap, void* stream);

/* Copies the current core factors (three core_dims[l] x R matrices, packed, device) out of the
 * state, or (set = 1) into it: the next iteration then starts from them as given (not balanced),
 * first recomputing the residual and the MTTKRP there; mu, the iteration count and the error
 * history continue.  Synchronises `stream`. */
cpd_status cpd_state_factors(void* state, double* W, int32_t set, void* stream);

/* ------------------------------------------------------------------------------------------ */
/* Full pipeline: ch.4 flow chart Compress -> Initialize -> dGN -> Uncompress, output with    */
/* unit columns and lambda.                                                                    */
/* ------------------------------------------------------------------------------------------ */

/*
 * cpd_solve:
 *   W0        (device, nullable) three R~_l x R initial core factors, packed (init RANDOM/GIVEN);
 *             R~_l must equal the core dims compression chooses (use cpd_compress first).
 *   W_out[l]  (device) dims[l] x R row-major, unit columns; modes 1, 2 signed so each column's
 *             largest-|.| entry is positive; terms sorted by decreasing lambda.
 *   lambda_out(device) R doubles, >= 0.
 *   info      (host) summary.  Synchronises `stream`.
 */
cpd_status cpd_solve(const void* T, int32_t dtype, const int64_t dims[3], int32_t R,
                     const cpd_params* p, const double* W0, double* W_out[3], double* lambda_out,
                     cpd_solve_info* info, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------------------------ */
/* Kernel-level entry points (the pieces of the path, exposed for parity tests and timing).   */
/* ------------------------------------------------------------------------------------------ */

/* G (device, dims[mode]^2 doubles) = T_(mode) T_(mode)^T, the unfolding Gram of App. B lemma.
 * ws: cpd_gram_workspace_bytes. */
size_t cpd_gram_workspace_bytes(const int64_t dims[3], int32_t mode);
cpd_status cpd_gram(const void* T, int32_t dtype, const int64_t dims[3], int32_t mode,
                    int32_t compute_dtype, double* G, void* ws, size_t ws_bytes, void* stream);

/* Leading P eigenpairs of a symmetric n x n matrix G (device): U (device, n x P row-major,
 * columns signed as in cpd_compress) and lam (device, P, descending).  n <= 64 uses cyclic
 * Jacobi on all of G; larger n uses subspace iteration with Rayleigh-Ritz (P <= 56). */
size_t cpd_eig_workspace_bytes(int32_t n, int32_t P);
cpd_status cpd_eig_top(const double* G, int32_t n, int32_t P, double* U, double* lam, void* ws,
                       size_t ws_bytes, void* stream);

/* M (device, dims[mode] x R, FP64) = T_(mode) (W^(L) (.) ... (.) W^(1) without W^(mode)), the
 * MTTKRP of the gradient theorem (ch.4 "Computing the gradient").  W[l] (device) dims[l] x R FP64,
 * R <= 64.  compute_dtype selects the matrix cores:
 *   CPD_F64  -- any input dtype, promoted exactly; FP64 products and sums (order-only rounding);
 *   CPD_F32  -- FP32 or BF16 input: FP32 MFMA; the inner factor (W^(3), or W^(2) for mode 3) is
 *               rounded to FP32, the outer one is applied in FP32, inner sums accumulate in FP32,
 *               the partial sums of different workgroups are added in FP64;
 *   CPD_BF16 -- BF16 input only: BF16 MFMA with FP32 accumulation; the inner factor is rounded
 *               (to nearest even) to BF16, the rest as for CPD_F32.
 * Any other pairing returns CPD_E_INVALID.  ws: cpd_mttkrp_workspace_bytes (covers every
 * compute_dtype). */
size_t cpd_mttkrp_workspace_bytes(const int64_t dims[3], int32_t R, int32_t mode);
cpd_status cpd_mttkrp(const void* T, int32_t dtype, const int64_t dims[3], const double* const W[3],
                      int32_t R, int32_t mode, int32_t compute_dtype, double* M, void* ws, size_t ws_bytes,
                      void* stream);

/* ------------------------------------------------------------------------------------------ */
/* Batched solve: many small independent CPDs (every mode <= 64), each the full path of ch.4     */
/* (Alg. Compression, dGN with CG, uncompression) exactly as cpd_solve does it, one workgroup   */
/* per member and stage in five launches with no host round trip between them.                 */
/* ------------------------------------------------------------------------------------------ */
typedef struct {
  const void* T;          /* (device) dense C-ordered dims[0] x dims[1] x dims[2] tensor */
  int64_t dims[3];        /* each 1..64 */
  int32_t R;              /* rank, 1..64 */
  const double* W0[3];    /* (device) initial core factors, P_l x R row-major with
                             P_l = min(dims[l], R) (or min(dims[l], core_dims[l]) when the
                             params fix the core); only the first R~_l rows are used when the
                             truncation rule shrinks mode l.  All three NULL: N(0,1) entries
                             from params.seed and the member index.  All or none. */
  double* W[3];           /* (device) out: dims[l] x R factors with unit columns */
  double* lambda;         /* (device) out: R weights, decreasing */
} cpd_batch_item;

/* Workspace for cpd_solve_batched / cpd_batch_plan_create with these members; 0 if invalid. */
size_t cpd_batch_workspace_bytes(const cpd_batch_item* items /* host, n */, int32_t n,
                                 const cpd_params* p);

/* Solves every member with the same params (maxiter, tol, mlsvd_tol, init_damp, cg_tol, caps:
 * one random CG-cap schedule shared by all members).  dtype: CPD_F64 or CPD_F32 for all members.
 * info (host, n entries, may be NULL) receives each member's result as cpd_solve would report
 * it; stop_reason is -1 for a member whose tensor is zero or holds NaN/Inf (its outputs are then
 * meaningless).  Synchronises the stream. */
cpd_status cpd_solve_batched(const cpd_batch_item* items, int32_t n, int32_t dtype, const cpd_params* p,
                             cpd_solve_info* info, void* ws, size_t ws_bytes, void* stream);

/* A plan fixes the members, params and workspace, picks the Gram tile variant by timing each
 * candidate on this batch, and captures the five launches in a hipGraph.  cpd_batch_plan_run
 * replays the graph on `stream`; with info != NULL it then waits and copies the results.  The
 * plan keeps pointers into `ws` and to the members' buffers: they must stay valid.  The tensors
 * may change between runs (same shapes).  Plans are host objects; destroy frees them. */
typedef struct cpd_batch_plan cpd_batch_plan;
cpd_status cpd_batch_plan_create(const cpd_batch_item* items, int32_t n, int32_t dtype, const cpd_params* p,
                                 void* ws, size_t ws_bytes, void* stream, cpd_batch_plan** out);
cpd_status cpd_batch_plan_run(cpd_batch_plan* plan, cpd_solve_info* info, void* stream);
/* Chosen Gram variant (0..3); variant_ms (host, 4 entries, may be NULL) gets each candidate's time. */
int32_t cpd_batch_plan_variant(const cpd_batch_plan* plan, float* variant_ms);
void cpd_batch_plan_destroy(cpd_batch_plan* plan);

/* Precision variant of cpd_solve for large tensors: the three compression Grams (ch.4 Alg.
 * Compression, eigenvector route of the App. B lemma) are formed from T_lo, a BF16 copy of T
 * (device, same shape, lo_dtype = CPD_BF16), on the BF16 matrix cores with FP32 accumulation
 * (FP64 across split-K chunks).  Everything else reads T (FP32 or FP64): the core projection, the
 * dGN on the core (FP64 throughout, so every CG inner product, the damping update and the final
 * iterations are FP64) and the final error.  Arguments, workspace (cpd_workspace_bytes of T's
 * shape) and results as cpd_solve. */
cpd_status cpd_solve_mixed(const void* T_lo, int32_t lo_dtype, const void* T, int32_t dtype, const int64_t dims[3],
                           int32_t R, const cpd_params* p, const double* W0, double* W_out[3], double* lambda_out,
                           cpd_solve_info* info, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------------------------ */
/* Tensors of order L >= 4: ch.4 "Tensor train and the CPD", Alg. TT-SVD (every TT-rank R) and */
/* Alg. CPD-TTD (a rank-R CPD of the second core, a Bi-CPD with the first factor fixed to the   */
/* inverse transpose of the previous third factor for each further core, outer factors from    */
/* the first and last cores).                                                                   */
/* ------------------------------------------------------------------------------------------ */

/* Workspace bytes of cpd_solve_tt; 0 if the shape is outside its limits. */
size_t cpd_tt_workspace_bytes(int32_t L, const int64_t* dims, int32_t R, const cpd_params* p);

/*
 * cpd_solve_tt: rank-R CPD of an order-L tensor (4 <= L <= 16) through the tensor train.
 *   T        (device) prod(dims) elements, C order, CPD_F64 or CPD_F32.
 *   dims     (host) L sizes, each 1..4096, with R <= min(dims[0], dims[L-1]), R * dims[l] <= 4096 and
 *            R <= 56 whenever R * dims[l] > 64 (the eigensolver's limits), and the trailing products
 *            at least R.
 *   W0       (device, nullable) start points of the third-order CPDs, packed: for the second core
 *            (R x I_2 x R, compressed to R x min(I_2, R) x R) three row-major R x R, min(I_2, R) x R,
 *            R x R matrices; then for each core l = 3..L-1 an I_l x R and an R x R matrix.  NULL:
 *            N(0,1) starts from params.seed.
 *   W_out[l] (device, host array of L pointers) I_l x R, unit columns, modes 1..L-1 signed so each
 *            column's largest-|.| entry is positive, terms by decreasing lambda; lambda_out (device) R.
 *   info     (host): iters = dGN iterations over all inner CPDs, stop_reason = the last one's,
 *            rel_err_core = the largest inner relative error, rel_err_full = ||T - T^|| / ||T||.
 * The inner CPDs use p's dGN parameters (classic compression, no refinement).  Synchronises the
 * stream (once per Bi-CPD).  CPD_E_NONFINITE if a third factor to be inverted is singular.
 */
cpd_status cpd_solve_tt(const void* T, int32_t dtype, int32_t L, const int64_t* dims, int32_t R, const cpd_params* p,
                        const double* W0, double* const* W_out, double* lambda_out, cpd_solve_info* info, void* ws,
                        size_t ws_bytes, void* stream);

/* out (device, 1 double) = ||T - sum_r w_r^(1) o w_r^(2) o w_r^(3)||^2, fused (ch.4 "Computing the
 * residual" applied to the input tensor).  ws: cpd_residual_workspace_bytes. */
size_t cpd_residual_workspace_bytes(const int64_t dims[3]);
cpd_status cpd_residual_norm2(const void* T, int32_t dtype, const int64_t dims[3],
                              const double* const W[3], int32_t R, double* out, void* ws,
                              size_t ws_bytes, void* stream);

/* cpd_residual_norm2 for callers that cannot allocate or pass a workspace (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): same arguments and result, minus
 * ws.  Its scratch (the per-block partial sums) is a static device array of 64 KiB per GPU, held
 * until the process ends; the device address is looked up once per device on the first call made
 * with that device current.  Calls that overlap on one GPU (several streams or threads) race on
 * that scratch and must be serialised by the caller.  Returns CPD_E_UNSUPPORTED if the partial
 * sums would exceed the scratch (they never do for dims <= 4096); calls no allocating routine. */
cpd_status cpd_residual_norm2_noalloc(const void* T, int32_t dtype, const int64_t dims[3],
                                      const double* const W[3], int32_t R, double* out, void* stream);

/* out[l] (device, dims[l] x R) = block l of J^T J v (ch.3 Thm Hv) for factors W[l] and direction
 * V[l] (device, dims[l] x R each).  One workgroup; dims[l] <= 4096, R <= 64. */
cpd_status cpd_jtj_v(const double* const W[3], const double* const V[3], const int32_t dims[3],
                     int32_t R, double* const out[3], void* stream);

/* ------------------------------------------------------------------------------------------ */
/* Learned initialisation (an extension; the thesis has no learned part): a multilayer          */
/* perceptron y = W3^T relu(W2^T relu(W1^T x + b1) + b2) + b3 mapping a normalised compressed     */
/* core (n_in = prod(core dims)) to initial core factors (n_out = R * sum(core dims)), trained   */
/* with the mean squared error and Adam.  All arrays FP32, device, row-major: W[l] is             */
/* dims[l] x dims[l+1] with dims = {n_in, n_h1, n_h2, n_out}; a batch is B x n_in (inputs) or    */
/* B x n_out (outputs).  The GEMMs run on the FP32 matrix cores with FP32 accumulation.          */
/* ------------------------------------------------------------------------------------------ */
typedef struct {
  int32_t n_in, n_h1, n_h2, n_out;
  float* W[3];
  float* b[3];
} cpd_mlp;

typedef struct {
  float* dW[3];   /* same shapes as the weights */
  float* db[3];
} cpd_mlp_grads;

typedef struct {
  float lr, beta1, beta2, eps;   /* Adam hyper-parameters (Kingma & Ba 2015) */
  int32_t step;                  /* updates done so far; cpd_mlp_adam_step increments it */
  float* mW[3];                  /* first and second moments, same shapes as the weights, zeroed */
  float* mb[3];                  /* by the caller before the first step */
  float* vW[3];
  float* vb[3];
} cpd_adam;

/* Workspace of cpd_mlp_forward / cpd_mlp_backward for batch size B (the hidden activations of the
 * last forward pass live in it: backward must follow a forward of the same x with the same ws). */
size_t cpd_mlp_workspace_bytes(const cpd_mlp* net, int32_t B);
cpd_status cpd_mlp_forward(const cpd_mlp* net, const float* x, float* y, int32_t B, void* ws, size_t ws_bytes,
                           void* stream);
/* Mean over n entries of (y - t)^2 into *loss (device float) and its gradient dy = 2 (y - t) / n.
 * ws: at least 8 KiB (device). */
cpd_status cpd_mlp_mse(const float* y, const float* t, int64_t n, float* dy, float* loss, void* ws, size_t ws_bytes,
                       void* stream);
/* Gradients of a loss with output gradient dy (B x n_out) into g, using the activations left in ws by
 * cpd_mlp_forward(net, x, ...). */
cpd_status cpd_mlp_backward(const cpd_mlp* net, const float* x, const float* dy, cpd_mlp_grads* g, int32_t B,
                            void* ws, size_t ws_bytes, void* stream);
/* One Adam update of every weight and bias (host struct a: step is incremented on the host). */
cpd_status cpd_mlp_adam_step(cpd_mlp* net, const cpd_mlp_grads* g, cpd_adam* a, void* stream);

/* Encoding of the learned start.  Feature of a core S: x = S / ||S|| (FP32).  Target of a CPD of
 * the core with unit columns W[l] and weights lambda: t = [w_r^(l) lambda_r^{1/3}] / ||S||^{1/3}
 * (FP32, the three core_dims[l] x R row-major blocks one after the other).  The start from a
 * network output y is W = y ||S||^{1/3}, the inverse map. */
/* Features of n_items cores stored back to back (device FP64, n entries each) into x (device
 * FP32, n_items x n) and their norms into norms (device FP64, n_items).  Does not synchronise. */
cpd_status cpd_learned_features(const double* S, int32_t n_items, int64_t n, float* x, double* norms,
                                void* stream);
/* Target of one core's CPD (W[l] device core_dims[l] x R, lambda device R, s_norm = ||S|| > 0 on
 * the host) into t (device FP32, R sum(core_dims) entries).  Does not synchronise. */
cpd_status cpd_learned_target(const double* const W[3], const double* lambda, const int32_t core_dims[3],
                              int32_t R, double s_norm, float* t, void* stream);
size_t cpd_learned_start_workspace_bytes(const cpd_mlp* net, const int32_t core_dims[3], int32_t R,
                                         int32_t judge_iters);
/*
 * cpd_learned_start: the starting point for the dGN on the core S (device FP64, core_dims C order)
 * from the network net (n_in = prod(core_dims), n_out = R sum(core_dims)), written to W_out (device,
 * the three core_dims[l] x R factors packed, as cpd_state_init's W0).
 * judge_iters = 0: the network's start.  judge_iters > 0: the dGN residual judges the network:
 * judge_iters dGN iterations (parameters p: tol, damping, CG cap from p->seed or p->cg_uniforms,
 * precond and drawback) run from the network's start and from the fallback start, W_fallback
 * (device, packed like W_out) or, when NULL, the library's N(0,1) start for p->seed (the start
 * cpd_solve draws with CPD_INIT_RANDOM; the thesis's random initialisation, ch.4
 * "Initialization"); W_out is the network's start unless its core relative error after them
 * exceeds judge_margin (>= 1) times the fallback's (a non-finite error counts as exceeding), in
 * which case it is the fallback.  chosen (host, nullable): 0 network, 1 fallback;
 * judge_err (host, nullable, 2 entries): the two errors after the judge iterations (0 when
 * judge_iters = 0).  p may be NULL (defaults).  Synchronises `stream` when judge_iters > 0; without
 * the judge the calls are only enqueued (ws must then stay valid until the stream reaches them).
 */
cpd_status cpd_learned_start(const cpd_mlp* net, const double* S, const int32_t core_dims[3], int32_t R,
                             int32_t judge_iters, double judge_margin, const cpd_params* p,
                             const double* W_fallback, double* W_out, int32_t* chosen, double* judge_err, void* ws,
                             size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------------------------ */
/* Kernel timing: when enabled, HIP events are recorded on the launch stream around the main   */
/* kernels of the path; cpd_profile_read waits for them and accumulates durations.  Intended   */
/* for single-threaded measurement runs.                                                        */
/* ------------------------------------------------------------------------------------------ */
typedef enum {
  CPD_PK_GRAM = 0,      /* Gram partial-tile kernel (per mode) */
  CPD_PK_DGN = 1,       /* persistent dGN kernel (one launch per cpd_dgn_run / cpd_solve) */
  CPD_PK_PROJECT = 2,   /* first mode product of the core projection (reads T) */
  CPD_PK_RESIDUAL = 3,  /* full-tensor fused residual kernel */
  CPD_PK_MTTKRP = 4,    /* full-tensor MTTKRP */
  CPD_PK_EIG = 5,       /* eigensolver (all kernels of one cpd_eig_top call) */
  CPD_PK_COUNT = 6
} cpd_profile_kernel;

typedef struct {
  int64_t launches;
  double total_ms;
} cpd_kernel_time;

void cpd_profile_enable(int32_t on);
/* Which kernels are timed while enabled: bit k for cpd_profile_kernel k (default: all).  Timing a
 * few kernels keeps the event recording (host API calls) out of the rest of a measured step. */
void cpd_profile_select(uint32_t mask);
void cpd_profile_reset(void);
/* Waits for the recorded events, then fills out[CPD_PK_COUNT]. */
cpd_status cpd_profile_read(cpd_kernel_time* out);

/* Measured floor of the one-workgroup reductions: one workgroup of `nthreads` (a multiple of 64,
 * <= 1024) chains `reps` block sums (wavefront shuffle, one barrier, one LDS round trip each) timed
 * with the device wall clock; *ns_out (host) receives ns per block sum.  ws: 16 device bytes.
 * Synchronises the stream. */
cpd_status cpd_profile_block_sum_ns(int32_t nthreads, int32_t reps, void* ws, size_t ws_bytes, double* ns_out,
                                    void* stream);

#ifdef __cplusplus
}
#endif

#endif /* CPD_H */
