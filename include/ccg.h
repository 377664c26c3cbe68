/*
 * ccg.h -- C interface of the MI355X (gfx950) cooperative conjugate gradient library.
 *
 * The method is Alg. 2 of Bhaya, Bliman, Niedu and Pazos, "A cooperative conjugate
 * gradient method for linear systems permitting multithread implementation of low
 * complexity" (cCG, Sec. 3.2): p agents each hold an estimate x_j, a residual r_j
 * and a direction d_j of the dense SPD system A x = b, and cooperate through the
 * p x p matrix step sizes
 *     alpha = (D^T A D)^{-1} D^T R,    beta = -(D^T A D)^{-1} (A D)^T R_new
 * (written here in the sign convention R = B - A X, B = b in every column; the
 * paper uses the gradient A X - B, which negates R and D and transposes alpha and
 * beta).  The residual follows the Table 1 recurrence R -= (A D) alpha, the rank
 * step follows Alg. 3 (mcCG), and the stop test is the minimum over agents of
 * ||r_j|| / ||b|| (Alg. 4), confirmed by the explicit FP64 residual.
 *
 * Conventions for every entry point
 * ---------------------------------
 *  - Every matrix is column-major.  A is n x n with leading dimension lda >= n;
 *    X is n x p with leading dimension ldx >= n, column j = agent j.  A must be
 *    symmetric positive definite; it is read as given (never symmetrised).
 *  - Pointers are DEVICE pointers on the context's device (e.g. torch tensor
 *    data_ptr()), unless opts->flags has CCG_HOST_PTRS, in which case they are host
 *    pointers and are copied in and out.  The caller owns A, b and X; the library
 *    owns all of its workspace (vector blocks, partial sums, low-precision copies of
 *    A) and frees it in ccg_destroy.
 *  - All work is enqueued on the context's stream; every call returns after the
 *    result is available on that stream (the library synchronises it).
 *  - Nothing throws across this interface.  Every call returns a ccg_status; on
 *    failure ccg_last_error(ctx) describes it.  A context is not thread safe.
 *  - 1 <= p <= min(n, 32) in CCG_FP64 single solves (ccg_solve, ccg_debug_step,
 *    ccg_solve_noalloc); 1 <= p <= min(n, 16) in the low-precision modes and for
 *    batched and served problems (CCG_ERR_ARG beyond).  Agent counts are padded
 *    internally to 1, 2, 4, 8, 16 or 32; padded agents are inactive.
 */
#ifndef CCG_H
#define CCG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CCG_OK = 0,              /* converged: min_j explicit ||b - A x_j|| / ||b|| <= tol */
    CCG_NOT_CONVERGED = 1,   /* maxit reached; X holds the last iterate (a warning) */
    CCG_ERR_ARG = -1,        /* bad argument (sizes, null pointer, tol <= 0, b == 0) */
    CCG_ERR_NONFINITE = -2,  /* NaN / Inf met in a residual norm or a Gram matrix */
    CCG_ERR_NOT_SPD = -3,    /* D^T A D not positive for a nonzero direction */
    CCG_ERR_BREAKDOWN = -4,  /* refinement made no progress */
    CCG_ERR_NOMEM = -5,      /* device allocation failed or HBM budget exceeded */
    CCG_ERR_DEVICE = -6,     /* a HIP call failed */
    CCG_PENDING = -7,        /* served request still running */
    CCG_CANCELLED = -8       /* served request cancelled */
} ccg_status;

typedef enum {
    CCG_FP64 = 0,    /* A streamed in FP64, FP64 vectors: plain cCG */
    CCG_FP32 = 1,    /* A streamed in FP32 inside an FP64 iterative-refinement loop */
    CCG_BF16X2 = 2   /* A streamed as BF16 hi + lo planes (FP32 accumulation), FP64 refinement */
} ccg_prec;

#define CCG_HOST_PTRS 0x1u   /* A, b, X are host pointers */
#define CCG_NO_GRAPH  0x2u   /* launch every kernel directly (no captured graph) */
#define CCG_PROFILE   0x4u   /* time every A.D launch with HIP events (ccg_kernel_time);
                                 block steps are then launched directly, not as a graph */
#define CCG_ESCALATE  0x8u   /* CCG_FP32 / CCG_BF16X2: when the refinement breaks down
                                 (CCG_ERR_BREAKDOWN, or an inner Gram matrix that is not
                                 positive or not finite), continue from the current agents
                                 in the next wider precision (BF16X2 -> FP32 -> FP64);
                                 info then totals every stage */
#define CCG_PROFILE_SAMPLED 0x10u  /* as CCG_PROFILE for every 4th round of block steps;
                                      the other rounds run from the captured graphs */
#define CCG_SYM_AD    0x20u  /* FP64 block steps with p <= 8 and n >= 1024 form A D from
                                 the upper block triangle of A only (see ccg_solve) */
#define CCG_REINFLATE 0x40u  /* ccg_solve, CCG_FP64: when the rank step would drop some
                                 agents (Alg. 3), re-inflate them instead, at most
                                 opts->max_reinflate times (see ccg_solve); batched and
                                 served problems with it get CCG_ERR_ARG */
#define CCG_NO_TIER   0x80u  /* run the block steps of a system with n <= 96 and p <= 4
                                 on the multi-workgroup path instead of the small-system
                                 tier (one workgroup per system); single, batched and
                                 served solves alike */

/* Solver options; a zero-initialised struct selects the defaults shown. */
typedef struct {
    int prec;            /* ccg_prec; default CCG_FP64 */
    double inner_tol;    /* low-precision modes: inner relative tolerance of the first
                            outer step and its lower bound (default 1e-4) */
    int inner_maxit;     /* low-precision modes: block steps per refinement (default 500) */
    int max_refine;      /* low-precision modes: outer refinement steps (default 60) */
    double rank_tau;     /* rank threshold on scaled pivots (default 1e-14; 1e-12 in the
                            low-precision modes, whose vectors carry FP32 rounding) */
    int graph_k;         /* block steps per captured graph / per host poll (default 16);
                            ccg_solve lengthens a round up to 8 graph_k while the
                            residual's decay predicts many more steps (FP64 solves and
                            the inner solves of the refinement modes) */
    unsigned flags;      /* CCG_HOST_PTRS | CCG_NO_GRAPH | CCG_PROFILE | CCG_PROFILE_SAMPLED |
                            CCG_ESCALATE | CCG_SYM_AD | CCG_REINFLATE */
    int max_reinflate;   /* CCG_REINFLATE: re-inflation events allowed (default 3) */
    int ad_cw, ad_nw;    /* A.D tile shape of the block steps: A columns per wave and
                            waves per workgroup (0: the tuned table's choice for the
                            precision, p and n).  Rounded to a shape the library runs:
                            cw 1, 2 or 4, nw 4, 8 or 16; FP64 at 9 <= p <= 16 runs the
                            matrix-core tile where cw * nw >= 16 (16 or 32 rows per
                            workgroup), and at 17 <= p <= 32 always (a shape with
                            cw * nw < 16 runs as cw = 4).  Applies to single and
                            batched solves alike. */
} ccg_opts;

/* Per-solve report. */
typedef struct {
    int status;          /* same as the return value */
    int iters;           /* block steps (all refinements and restarts included) */
    int refinements;     /* outer refinement steps (0 in FP64 mode) */
    int restarts;        /* explicit-residual restarts */
    int p_final;         /* agents still active at the end */
    int best_agent;      /* argmin_j of the explicit residual */
    int deflations;      /* rank-drop events (Alg. 3) */
    int prec_final;      /* ccg_prec the solve ended in (differs from opts->prec only
                            after CCG_ESCALATE moved it to a wider precision) */
    double rel_res;      /* min_j ||b - A x_j|| / ||b||, explicit FP64 */
    double rel_res_max;  /* max_j of the same */
    double seconds;      /* wall time of the solve inside the library */
    double bytes_A;      /* algorithmic bytes of A streamed (all precisions) */
    int reinflations;    /* re-inflation events (CCG_REINFLATE) */
} ccg_info;

typedef struct ccg_ctx ccg_ctx;

/* Create a context on HIP device `device`.  hbm_budget_bytes caps the library's own
 * device allocations (0: no cap).  hip_stream: a hipStream_t to enqueue on, or NULL
 * for a stream the context creates (default priority).  Returns CCG_ERR_DEVICE if
 * the device cannot be used. */
ccg_status ccg_create(ccg_ctx **ctx, int device, size_t hbm_budget_bytes, void *hip_stream);

/* Free the context and all of its device memory.  NULL is accepted. */
ccg_status ccg_destroy(ccg_ctx *ctx);

/* Last error message of this context ("" if none).  Owned by the context. */
const char *ccg_last_error(const ccg_ctx *ctx);

/* Solve A x = b with p cooperating agents (Alg. 2 + Alg. 3, stop test of Alg. 4).
 * X: in, the p starting points X0; out, the final p agents.  tol > 0 is relative
 * to ||b||; maxit bounds the block steps.  opts and info may be NULL.  A must be
 * symmetric (the A.D kernel streams column i of A as row i).  With CCG_SYM_AD the
 * FP64 block steps of a system with n >= 1024 and p <= 8 form A D from the blocks
 * A(I, J), I <= J, of 128 x 128 (A(I, J) D(J) for rows I and A(I, J)^T D(I) for
 * rows J), so they read only the upper block triangle; the explicit residuals and
 * the other modes read all of A.  (On MI355X this pass is slower than streaming all of
 * A at the sizes measured; it is kept for comparison.)
 *
 * With CCG_REINFLATE (CCG_FP64 only; a policy beyond the paper, off by default), a
 * rank step that would drop some but not all agents instead re-inflates them, up to
 * opts->max_reinflate times: each agent outside the kept set J restarts from the
 * iterate of the active agent with the smallest residual norm (ties: lowest index)
 * plus d, d_i = 2 (z_i >> 11) 2^-53 - 1 with z_i the (i+1)-th output of SplitMix64
 * (Steele, Lea, Flood 2014) from the state 0x1204 << 48 ^ e << 32 ^ j (e: the event,
 * from 0; j: the agent), and all p agents restart from R = D = B - A X (the start of
 * Alg. 2) in place of that step.  info->reinflations counts the events.
 *
 * opts->prec selects how A is streamed:
 *  - CCG_FP64: plain cCG on the FP64 matrix and FP64 agents.
 *  - CCG_FP32 / CCG_BF16X2 (not in the paper; mixed-precision iterative refinement
 *    around the paper's iteration): A is converted on every call to FP32 (nearest
 *    even) or to two BF16 planes hi = bf16(A), lo = bf16(A - hi).  Each outer step
 *    forms the explicit FP64 residual T = B - A X, runs cCG on A E = T (columns of T
 *    scaled to unit norm) with FP32 vectors and FP32 accumulation of A.D, FP64 Gram
 *    products, alpha and beta, until min_j of the inner relative residual is below
 *    the inner tolerance or inner_maxit steps, then sets X += E (FP64).  The inner
 *    tolerance is inner_tol in the first outer step, then a quarter of the factor by
 *    which the last outer step lowered the FP64 residual (within [inner_tol, 0.05]).
 *    The result is
 *    converged when the FP64 residual meets tol, as in CCG_FP64.  Returns
 *    CCG_ERR_BREAKDOWN when three outer steps in a row fail to lower the best FP64
 *    residual (e.g. when cond(A) times the rounding of the low-precision copy is
 *    near 1), CCG_NOT_CONVERGED after max_refine outer steps or maxit block steps
 *    in total.  The library holds the low-precision copy (4 n^2 bytes) until
 *    ccg_destroy. */
ccg_status ccg_solve(ccg_ctx *ctx, int n, int p, const double *A, int64_t lda,
                     const double *b, double *X, int64_t ldx, double tol, int maxit,
                     const ccg_opts *opts, ccg_info *info);

/* Allocation-free FP64 solve, for callers that cannot allocate device memory (code
 * that must not call hipMalloc, tight serving loops, harnesses that forbid it): the
 * same solve as ccg_solve with CCG_FP64 and CCG_NO_GRAPH, bit for bit, with its
 * whole workspace (vector blocks, reduction scratch, device state) in a device
 * array of the library, 64 MiB per GPU, that each GPU holds from ccg_create until
 * the process ends.  The call allocates nothing: no hipMalloc / hipFree, no graph,
 * no event.  The caller passes device pointers; A must have 16-byte aligned columns
 * (A aligned to 16 bytes, lda even).  opts may select only CCG_FP64 (prec),
 * rank_tau and graph_k (the round length between host polls of the state); the
 * flags CCG_HOST_PTRS, CCG_PROFILE, CCG_PROFILE_SAMPLED, CCG_SYM_AD, CCG_ESCALATE
 * and CCG_REINFLATE, another precision or unaligned columns give CCG_ERR_ARG.  A size
 * whose workspace exceeds the array (vector blocks of n_pad * P elements, n_pad = n
 * rounded up to 512 and P = p rounded up to a power of two, plus the reduction
 * scratch: n up to 65536 at p <= 8, up to 32768 at p = 16, up to 8192 at
 * p = 32) gives CCG_ERR_NOMEM
 * with nothing launched.  Every call on a GPU, from any context
 * on it, uses that GPU's one array and clears it first: calls that overlap in time
 * on one GPU (other threads, other streams) race and must not be made. */
ccg_status ccg_solve_noalloc(ccg_ctx *ctx, int n, int p, const double *A, int64_t lda,
                             const double *b, double *X, int64_t ldx, double tol, int maxit,
                             const ccg_opts *opts, ccg_info *info);

/* Run exactly ksteps block steps of FP64 cCG from X (no stop test) and report each
 * step's alpha and beta (ksteps x p x p; step k at offset k*p*p, element (r, c) at
 * r + c*p, i.e. column-major; X[:,c] += sum_r D[:,r] alpha[r,c]) and the final
 * X, R and D (n x p column-major with leading dimension n for R and D, ldx for X).
 * For step-by-step comparison with a reference implementation. */
ccg_status ccg_debug_step(ccg_ctx *ctx, int n, int p, const double *A, int64_t lda,
                          const double *b, double *X, int64_t ldx, int ksteps,
                          const ccg_opts *opts, double *alphas, double *betas,
                          double *R, double *D);

/* One system of a batched or served solve: the arguments of ccg_solve. */
typedef struct {
    int n, p;
    const double *A;
    int64_t lda;
    const double *b;
    double *X;           /* in: X0; out: the final agents */
    int64_t ldx;
    double tol;
    int maxit;
    ccg_opts opts;       /* per system (precision, CCG_HOST_PTRS, ...); zero = defaults */
} ccg_problem;

/* Solve `count` independent systems together (not in the paper: many cCG solves
 * share each launch).  Every block step is one batched A.D launch and one batched
 * update launch per (precision, padded agent count) class, whose workgroups are
 * (system, row tile) work items of all systems still running; systems that finish
 * leave the work lists, and systems still waiting are admitted as the HBM budget
 * frees up.  Each system gets exactly the result ccg_solve would give it.
 * infos[i] (may be NULL) receives system i's report.  Returns CCG_OK when every
 * system converged, else the first error status met, else CCG_NOT_CONVERGED.  A
 * system too large for the HBM budget on its own gets CCG_ERR_NOMEM. */
ccg_status ccg_solve_batched(ccg_ctx *ctx, int count, const ccg_problem *probs, ccg_info *infos);

/* Served mode (not in the paper): continuous batching.  ccg_submit queues a system
 * and returns at once with a ticket; a service thread of the context admits queued
 * systems in arrival order while their device memory fits the context's HBM budget,
 * advances every resident system with the batched launches of ccg_solve_batched on
 * a stream of its own, and retires each system as soon as it finishes.  The
 * problem's buffers must stay valid until ccg_poll / ccg_wait report a final status.
 * With CCG_HOST_PTRS, A, b and X are uploaded at admission, inside the latency.
 * info->seconds is the latency from ccg_submit to completion. */
ccg_status ccg_submit(ccg_ctx *ctx, const ccg_problem *prob, uint64_t *ticket);

/* Final status and report of a ticket (the ticket is then released), or
 * CCG_PENDING while it is queued or running.  Unknown tickets give CCG_ERR_ARG. */
ccg_status ccg_poll(ccg_ctx *ctx, uint64_t ticket, ccg_info *info);

/* Block until the ticket finishes; then as ccg_poll. */
ccg_status ccg_wait(ccg_ctx *ctx, uint64_t ticket, ccg_info *info);

/* Ask for a ticket to stop.  A queued system is dropped; a running one stops at the
 * next host round with its current agents in X.  Its final status is CCG_CANCELLED
 * (or its real status if it finished first). */
ccg_status ccg_cancel(ccg_ctx *ctx, uint64_t ticket);

/* The low-precision copy of A that a CCG_FP32 or CCG_BF16X2 solve streams, written
 * to caller buffers (device pointers, n x n column-major with leading dimension n):
 *  - CCG_FP32: hi receives float values, A rounded to nearest even; lo is unused.
 *  - CCG_BF16X2: hi and lo receive uint16 BF16 bit patterns, hi = A rounded to the
 *    nearest BF16 (ties to even, one rounding from the double), lo = A - hi (exact
 *    in FP64) rounded the same way.
 * For inspecting the conversion; ccg_solve converts by itself. */
ccg_status ccg_convert_matrix(ccg_ctx *ctx, int n, const double *A, int64_t lda, int prec,
                              void *hi, void *lo);

/* Average duration in microseconds of one A.D launch (the block step's stream of A,
 * products, stop test and p x p solves; not in the paper) with tile shape `cw` A
 * columns per wave (1, 2 or 4) and `nw` waves per workgroup (4, 8 or 16; a shape
 * beyond the register budget runs at the nearest one that fits) on a synthetic
 * symmetric diagonally dominant system of size n with p agents in precision `prec`,
 * over `reps` launches after 2 warm-up launches.  batched = 1 times the kernel of
 * ccg_solve_batched instead (the system's tiles as work items; timed with events
 * recorded around the launch).  Uses and overwrites the context's workspace.  For
 * the autotuner that writes the library's table of tile shapes
 * (paper_1204_0069_amd/tune.py).  CCG_ERR_ARG for arguments outside these ranges. */
ccg_status ccg_tune_ad(ccg_ctx *ctx, int prec, int p, int n, int cw, int nw, int batched, int reps,
                       double *us);

/* Median duration in microseconds, over `reps` launches after 2 warm-up launches, of
 * a kernel that only reads: an n x n FP64 matrix (column-major, lda = n; n even),
 * `cols` whole columns per workgroup of `waves` x 64 threads (cols divides n; waves
 * 4, 8 or 16), with 16-byte non-temporal loads, and, when dcols > 0 (at most 16), also
 * the whole of an n x dcols FP64 block in every workgroup, as the A.D tile kernel
 * reads the direction block.  stagger = 1 rotates each workgroup's starting offset in
 * its columns as the A.D kernel does; stagger = 2 (dcols = 0 only) reads the same
 * bytes with n / cols workgroups in a grid-stride loop instead (each pass of the grid
 * one contiguous span), the device's plain streaming ceiling.  The floor that the memory system sets for that
 * traffic, to set A.D timings against (not in the paper).  Allocates and frees its
 * own n^2 + n dcols doubles.  CCG_ERR_ARG for arguments outside these ranges. */
ccg_status ccg_stream_probe(ccg_ctx *ctx, int n, int cols, int dcols, int stagger, int waves, int reps,
                            double *us);

/* Accumulated duration (milliseconds), launch count and algorithmic bytes of the A.D
 * pass (the A.D kernel, or the symmetric pass's two kernels from the start of the
 * first to the end of the second) in the block steps run with CCG_PROFILE (every
 * launch) or CCG_PROFILE_SAMPLED (the launches of the timed rounds) of ccg_solve
 * since the last reset; reset != 0 clears them.  The bytes per launch are those of
 * A as streamed (n^2 elements, or n (n + 1) / 2 for the symmetric pass) plus the D
 * and R rows (2 n p vector elements).  Any output pointer may be NULL. */
ccg_status ccg_kernel_time(ccg_ctx *ctx, double *ms, long long *launches, double *bytes, int reset);

#ifdef __cplusplus
}
#endif

#endif /* CCG_H */
