/*
 * spaqr.h — C-ABI of the MI355X spaQR least-squares library (libspaqr.so).
 *
 * Method: Gnanasekaran & Darve, "Hierarchical Orthogonal Factorization:
 * Sparse Least Squares problems" (arXiv 2102.09878).  The library computes
 * an approximate factorization Q^T (A D^-1) W^-1 ~ I of a tall sparse
 * matrix A (M x N, M >= N, full column rank; Section 1, eq. (1.1)) by the
 * level-by-level algorithm of Section 2 (Algorithm 1), and uses D^-1 W^-1 as
 * a right preconditioner inside CGLS (Section 4).
 *
 * Conventions shared by every call:
 *  - Every call returns an int status: SPAQR_OK (0), a negative error code,
 *    or SPAQR_NOCONV (+1, CGLS reached max_iter; the result is still
 *    written).  No C++ exception crosses this boundary.  After an error,
 *    spaqr_last_error(h) returns a message owned by the handle (or by the
 *    library for calls that failed before a handle existed, h == NULL).
 *  - The caller owns every buffer it passes.  The library copies what it
 *    keeps; inputs may be freed as soon as a call returns.
 *  - The handle owns all device memory of the plan and of the factors.
 *  - "dev" pointers are device (GPU) pointers, e.g. torch.Tensor.data_ptr();
 *    work on them is ordered on the handle's HIP stream (opt->stream, NULL
 *    for the default stream).  Calls return after that work completed.
 *  - CSR input: int64 row_ptr (M+1), int32 col_idx sorted and unique within
 *    each row, double vals; every column must hold a nonzero.
 *  - Columns are ordered by the analysis; "slots" below are column
 *    positions 0..N-1 in which the factor W acts.
 */
#ifndef SPAQR_H
#define SPAQR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SPAQR_OK 0
#define SPAQR_NOCONV 1
#define SPAQR_EARG (-1)    /* invalid argument or malformed input           */
#define SPAQR_ESTATE (-2)  /* call order violated (e.g. cgls before factor) */
#define SPAQR_ERANK (-3)   /* a scaling block is numerically rank deficient */
#define SPAQR_EHIP (-4)    /* HIP runtime error (no GPU, launch failure)    */
#define SPAQR_ENOMEM (-5)  /* device or host allocation failed              */

#define SPAQR_FP64 0          /* fronts and factors in FP64                  */
#define SPAQR_FP32_FACTOR 1   /* fronts and factors in FP32; rank decisions,  */
                              /* apply accumulation and CGLS in FP64          */

#define SPAQR_MAX_LEVELS 32  /* tree levels the per-level statistics hold */

#define SPAQR_WINV 0   /* out = W^-1 in  (slot space)  */
#define SPAQR_WINVT 1  /* out = W^-T in  (slot space)  */

typedef struct spaqr_handle_s* spaqr_handle;

typedef struct {
  int32_t nd_depth;      /* tree levels including the leaves; 0 => ceil(log2(N/64)) (Section 4) */
  int32_t sparsify_skip; /* leaf-side levels left unsparsified; -1 => 2 (1 when depth <= 4)      */
  int32_t grid[3];       /* nx, ny, nz of the cell grid (x fastest), nz = 1 in 2D; column j is   */
                         /* cell j: geometric partitioning (Section 4.1).  grid[0] = 0: a       */
                         /* general matrix, partitioned by graph nested dissection of G(A^T A)  */
                         /* with a max-product row matching (Section 2.2).                       */
  int32_t sep_width;     /* separator thickness in cell planes; 0 => 2                           */
  int32_t precision;     /* SPAQR_FP64 or SPAQR_FP32_FACTOR                                      */
  int32_t device;        /* HIP device ordinal                                                   */
  void* stream;          /* hipStream_t, NULL => default stream                                  */
} spaqr_options;

typedef struct {
  int32_t iters;           /* CGLS iterations taken                                          */
  int32_t converged;       /* 1 if the stopping test held                                    */
  double residual;         /* ||A^T (b - A x)|| / (||A||_2 ||b||), recomputed from x at exit */
  double paper_residual;   /* ||A^T (A x - b)|| / ||A^T b|| (Section 4)                      */
  double norm_a;           /* the ||A||_2 estimate used (30 power steps on A^T A from ones) */
  double seconds;          /* wall time of the call                                          */
} spaqr_cgls_info;

typedef struct {
  int32_t levels;            /* tree depth d                                        */
  int32_t num_ops;           /* elementary ops of W                                 */
  int32_t num_ranks;         /* rank decisions made (step 1 and step 2)             */
  int32_t top_cols;          /* columns of the root cluster when it was eliminated  */
  int32_t top_rows;          /* rows of the root cluster when it was eliminated     */
  int32_t launches;          /* kernel launches of the last factorization           */
  int32_t syncs;             /* host synchronisations of the last factorization     */
  int32_t pad_;
  int64_t mem_factor;        /* stored factor entries (mem_F of Table 1)            */
  int64_t device_bytes;      /* device bytes held by the handle                     */
  double flops[5];           /* algorithmic flops per phase: eliminate, reassign,   */
  double bytes[5];           /* scale, sparsify, merge; and bytes moved per phase   */
  double phase_seconds[5];   /* wall time per phase of the last factorization       */
  double factor_seconds;     /* wall time of the last factorization                 */
  /* Per-launch timing of one kernel family, chosen by spaqr_time_kernel();
   * accumulated over every factorization and solve since that call. */
  int64_t kernel_calls;      /* launches timed                                      */
  double kernel_seconds;     /* sum of their HIP-event durations                    */
  double kernel_bytes;       /* algorithmic bytes those launches move               */
  double kernel_flops;       /* algorithmic flops of those launches                 */
  /* Per tree level m (index m, 1 <= m <= levels; index 0 unused), the
   * quantities of Section 4.2's profiling, for sparsified levels only
   * (zeros elsewhere): */
  int32_t level_interfaces[SPAQR_MAX_LEVELS]; /* interfaces scaled at level m          */
  double level_aspect[SPAQR_MAX_LEVELS];      /* median rows / columns of their        */
                                              /* diagonal blocks at scaling            */
  int64_t level_cols[SPAQR_MAX_LEVELS];       /* their columns before sparsification   */
  int64_t level_rank1[SPAQR_MAX_LEVELS];      /* sum of step-1 ranks (rows kept)       */
  int64_t level_rank2[SPAQR_MAX_LEVELS];      /* sum of step-2 ranks (columns kept)    */
  double sync_wait_seconds;  /* host time spent waiting in those synchronisations   */
  int64_t kernel_span_calls;   /* timed launches with in-kernel clock stamps          */
  double kernel_span_seconds;  /* sum of their first-start to last-end spans         */
} spaqr_stats;

/* Launch shapes of the factorization (see spaqr_autotune). */
typedef struct {
  int32_t pqr_poll;        /* pivot steps launched ahead of the last one the GPU has reported (16)    */
  int32_t pqr_reg_rows;    /* tallest row window a pivot step keeps in registers, 0..1024 (1024)      */
  int32_t tall_coop;       /* 1: tall panels in one cooperative launch; 0: two launches per column (1)*/
  int32_t from_cache;      /* spaqr_autotune: 1 if the choice was read from the cache file           */
  int32_t evaluations;     /* settings timed when it was tuned                                        */
  int32_t pad_;
  double seconds_default;  /* best factorization time with the defaults when it was tuned            */
  double seconds_best;     /* best factorization time with the chosen shapes                          */
} spaqr_tune;

typedef struct {
  int32_t kind;   /* 0 eliminate (R_ss, R_sN), 1 scale (R_pp), 2 sparsify (Q_pp reflectors) */
  int32_t n1;     /* eliminate: c_s;  scale: c_p;  sparsify: c_p                          */
  int32_t n2;     /* eliminate: c_N;  scale: 0;    sparsify: rank r (reflector count)      */
  int32_t round;  /* level-local round the op was created in                              */
  int32_t level;  /* tree level being processed when the op was created                   */
} spaqr_op_desc;

/* Analysis (host only, no GPU needed): column norms of the given values
 * (Algorithm 1 scales every column to unit 2-norm before partitioning),
 * nested dissection with interfaces and their hierarchy (Section 2.2):
 * geometric on the cell grid, or on the column graph G(A^T A) when
 * opt->grid[0] = 0; row matching (on a grid column j <-> row j, the
 * Laplacian row of cell j; otherwise the matching of largest product of
 * |a_ij|) and max-norm assignment of the other rows (Section 2.2).  The
 * device copy of the scaled matrix and the ||A||_2 estimate of the CGLS
 * stopping test are made by device kernels on first GPU use.
 * Errors: SPAQR_EARG for M < N, N < 1, a malformed CSR, an empty column, a
 * grid that does not match N or is too small for the depth (a graph too
 * small to split), a row that couples two sibling subtrees, or (no grid) an
 * explicit zero entry or no matching that covers every column.  On success
 * *out owns a new handle. */
int spaqr_analyze(const int64_t* row_ptr, const int32_t* col_idx, const double* vals, int64_t M,
                  int64_t N, const spaqr_options* opt, spaqr_handle* out);

/* Column order and row owners chosen by the analysis (host buffers):
 * col_perm[N] lists the columns cluster by cluster (finest clusters in
 * elimination order, cells ascending); row_owner[M] is the finest-cluster
 * index owning each row.  Either pointer may be NULL. */
int spaqr_get_ordering(spaqr_handle h, int32_t* col_perm, int32_t* row_owner);

/* Replace the nonzero values (same pattern) from a device buffer of nnz
 * doubles in CSR order; the analysis (ordering, row owners) is kept, the
 * column scaling (Algorithm 1) and the ||A||_2 estimate are recomputed on
 * the device.  Any factor is invalidated.  SPAQR_EARG if a column becomes
 * zero. */
int spaqr_set_values(spaqr_handle h, const double* vals_dev);

/* Numeric factorization with tolerance eps >= 0 (Algorithm 1).  Ranks of
 * the rank-revealing QRs follow |R_ii| >= eps |R_11| (Section 4).  Returns
 * SPAQR_ERANK if a scaling block has |R_ii| <= 64 u ||A_pp||_F. */
int spaqr_factorize(spaqr_handle h, double eps);

/* Same, but every rank decision takes the next entry of ranks[nranks]
 * (host buffer, in decision order: per level, step 1 over interfaces then
 * step 2 round by round).  Used to compare factors with another
 * implementation that chose these ranks.  SPAQR_EARG if the list is short
 * or not fully used. */
int spaqr_factorize_forced(spaqr_handle h, double eps, const int32_t* ranks, int32_t nranks);

/* One-shot seminormal solve x = D^-1 W^-1 W^-T D^-1 A^T b (Section 1).
 * b_dev: M doubles; x_dev: N doubles, original column order. */
int spaqr_apply(spaqr_handle h, const double* b_dev, double* x_dev);

/* Corrected seminormal equations with iterative refinement (Section 1:
 * the solution from W^T W x = A^T b, refined): x_0 = D^-1 W^-1 W^-T D^-1
 * A^T b, then x += D^-1 W^-1 W^-T D^-1 A^T (b - A x) until
 * ||A^T (b - A x)|| <= tol ||A||_2 ||b|| (checked before every
 * correction) or max_steps corrections were made.  b_dev: M doubles,
 * x_dev: N doubles (original order); info (may be NULL) gets the number of
 * corrections in iters and the final residuals (the worst problem of a
 * batch handle).  SPAQR_NOCONV when tol was not reached (x is written). */
int spaqr_csne(spaqr_handle h, const double* b_dev, double tol, int32_t max_steps, double* x_dev,
               spaqr_cgls_info* info);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * solve as spaqr_apply, bit for bit, with every intermediate in the
 * library's static device scratch array of 2^21 doubles (16 MiB, held by
 * each GPU the library runs on until the process ends) instead of handle
 * or freshly allocated memory.  The call allocates nothing; it needs
 * N + (W-sweep staging) + (W-sweep partials) doubles, each part rounded up
 * to 256 bytes, and returns SPAQR_EARG (naming the size) above the limit.
 * All calls on one GPU share the array: calls that overlap on one GPU
 * (other streams or threads) race.  SPAQR_ESTATE before a factorization.
 * b_dev: M doubles; x_dev: N doubles, original column order. */
int spaqr_apply_noalloc(spaqr_handle h, const double* b_dev, double* x_dev);

/* out = W^-1 in or W^-T in, both N doubles in slot space (Section 2.7). */
int spaqr_apply_op(spaqr_handle h, int32_t op, const double* in_dev, double* out_dev);

/* CGLS on A D^-1 W^-1 (right preconditioning, Section 4) from x0 = 0,
 * stopping when ||A^T (b - A x)|| <= tol ||A||_2 ||b||.  b_dev: M doubles,
 * x_dev: N doubles (original order).  info may be NULL.  Returns
 * SPAQR_NOCONV when max_iter was reached. */
int spaqr_cgls(spaqr_handle h, const double* b_dev, double tol, int32_t max_iter, double* x_dev,
               spaqr_cgls_info* info);

/* Batch of independent problems in one handle.  Each member is analysed
 * as by spaqr_analyze (arrays of count pointers / sizes / options); the
 * handle then holds their block-diagonal union: member g owns columns
 * [col_off[g], col_off[g+1]) and rows [row_off[g], row_off[g+1]) of the
 * batch vectors.  Tree levels are aligned from the leaves, so
 * spaqr_factorize on the handle eliminates, scales and sparsifies the
 * same-level clusters of every member in the same launches (Algorithm 1
 * run on all members at once; each member's factor equals its own).
 * Members must share precision, device, stream, sparsify_skip and
 * sep_width (SPAQR_EARG otherwise, naming the member).  spaqr_apply and
 * spaqr_apply_op act on the batch vectors; spaqr_cgls runs every member's
 * CGLS independently and reports the worst member; spaqr_adjoint needs a
 * single-problem handle. */
int spaqr_batch_analyze(int32_t count, const int64_t* const* row_ptr, const int32_t* const* col_idx,
                        const double* const* vals, const int64_t* M, const int64_t* N,
                        const spaqr_options* opts, spaqr_handle* out);

/* Member count and offsets (host buffers of count + 1, either may be NULL). */
int spaqr_batch_info(spaqr_handle h, int32_t* count, int64_t* col_off, int64_t* row_off);

/* CGLS of every member at once, each with its own recurrence scalars and
 * stopping test (Section 4); a member that has converged is frozen while
 * the others go on.  b_dev: total-M doubles, x_dev: total-N doubles (batch
 * order); infos: count entries (may be NULL).  SPAQR_NOCONV if a member
 * reached max_iter. */
int spaqr_batch_cgls(spaqr_handle h, const double* b_dev, double tol, int32_t max_iter, double* x_dev,
                     spaqr_cgls_info* infos);

/* Adjoint of the least-squares solution x = argmin ||A x - b|| for a loss
 * with gradient g = dL/dx: solves A^T A lambda = g by conjugate gradients
 * preconditioned with the factor of the current values, M^-1 =
 * D^-1 W^-1 W^-T D^-1 (A^T A ~ D W^T W D, Section 2.7), and forms
 *   grad_b[i]    = (A lambda)_i,
 *   grad_vals[e] = r_i lambda_j - (A lambda)_i x_j  (entry e at row i, col j),
 * with r = b - A x.  x_dev, g_dev: N doubles; b_dev, grad_b_dev: M doubles;
 * grad_vals_dev: nnz doubles in CSR order; lambda_dev: N doubles.  Any of
 * grad_b_dev, grad_vals_dev, lambda_dev may be NULL (grad_vals needs x and
 * b).  Stops when ||g - A^T A lambda|| <= tol ||g|| (recurrence); info gets
 * iterations, the true relative residual (residual), the recurrence one
 * (paper_residual) and seconds.  SPAQR_ESTATE before a factorization,
 * SPAQR_NOCONV at max_iter (outputs still written). */
int spaqr_adjoint(spaqr_handle h, const double* x_dev, const double* b_dev, const double* g_dev,
                  double tol, int32_t max_iter, double* grad_b_dev, double* grad_vals_dev,
                  double* lambda_dev, spaqr_cgls_info* info);

/* Statistics of the last factorization (Section 4.2 quantities, the
 * per-phase ledger, launch and synchronisation counts). */
int spaqr_factor_stats(spaqr_handle h, spaqr_stats* out);

/* Time every `every`-th launch (every >= 1) of one kernel family with HIP
 * events on the handle's stream and count the algorithmic bytes and flops
 * of the timed launches (exposed through spaqr_factor_stats); resets the
 * counters.  For "pqr_step" every launch is timed instead, in stretches of
 * `every` consecutive launches between two events (two event packets per
 * stretch), so kernel_seconds / kernel_calls is the time per launch on the
 * stream, dispatch included.  family: "pqr_step" (one pivot step of the batched
 * rank-revealing QRs: algorithmic flops and bytes of each batch, block read
 * and kept rows written once, shared over its step launches), "apply" (one
 * batch of W^-1 / W^-T ops) or "qrp_coop" (one cooperative tall Householder
 * panel of an elimination round), or NULL / "" to stop.  SPAQR_EARG for an unknown family or every < 1.
 * The first "pqr_step" launch of each stretch also stamps its first
 * work-group start and last work-group end with the GPU's constant-rate
 * clock (kernel_span_*).
 * Measurement aid: each timed launch adds two event records. */
int spaqr_time_kernel(spaqr_handle h, const char* family, int32_t every);

/* Rank decisions of the last factorization, in decision order (host
 * buffer of capacity cap); *n receives the count. */
int spaqr_get_ranks(spaqr_handle h, int32_t* ranks, int32_t cap, int32_t* n);

/* Elementary op i of W (creation order) and its data, copied to host
 * buffers sized from the descriptor:
 *   eliminate: mat = [R_ss R_sN] row-major c_s x (c_s + c_N) (upper part of
 *              R_ss only), slots1 = c_s slots, slots2 = c_N slots;
 *   scale:     mat = R_pp row-major c_p x c_p, slots1 = c_p slots;
 *   sparsify:  mat = reflectors row-major c_p x r (unit diagonal, zeros
 *              above), tau = r scalars, slots1 = c_p slots.
 * Any output pointer may be NULL. */
int spaqr_get_op(spaqr_handle h, int32_t i, spaqr_op_desc* desc, double* mat, int32_t* slots1,
                 int32_t* slots2, double* tau);

/* Project-written autotuner of the launch shapes for this handle's
 * problem (the batching form's tile choice): it times whole
 * factorizations with eps (the best of reps >= 1 runs per setting),
 * descends one knob at a time from the defaults (run-ahead window 4 / 8 /
 * 16 steps; register window 256 / 512 / 1024 rows; cooperative or
 * two-launch tall panels), keeps the fastest, and leaves the handle
 * factorized with it.  cache_path (may be NULL): a text file of
 * "signature poll rows coop t_default t_best evaluations" lines; an entry
 * whose signature (M, N, nnz, depth, skip, members, precision, eps, GPU
 * architecture) matches is used without timing, a new choice is appended.
 * The knobs change no result beyond the rounding of the panel form.
 * out (may be NULL) receives the choice.  SPAQR_EARG for reps < 1 or an
 * unwritable cache. */
int spaqr_autotune(spaqr_handle h, double eps, int32_t reps, const char* cache_path, spaqr_tune* out);

/* Set (validated: 1 <= pqr_poll <= 4096, 0 <= pqr_reg_rows <= 1024,
 * tall_coop 0 or 1; other fields ignored) or read the launch shapes;
 * they apply from the next factorization. */
int spaqr_set_tune(spaqr_handle h, const spaqr_tune* t);
int spaqr_get_tune(spaqr_handle h, spaqr_tune* out);

/* Release every resource of the handle. */
int spaqr_destroy(spaqr_handle h);

/* Message of the last error on h (or of the last handle-less failure). */
const char* spaqr_last_error(spaqr_handle h);

#ifdef __cplusplus
}
#endif
#endif /* SPAQR_H */
