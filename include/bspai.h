/*
 * bspai.h -- C interface of the MI355X BSPAI-GMRES-IR library (libbspai.so).
 *
 * Method: Khan & Carson, "Mixed Precision Iterative Refinement with Adaptive
 * Precision Sparse Approximate Inverse Preconditioning" (arXiv 2307.03914).
 * The library builds a sparse approximate inverse M of A on a prescribed
 * pattern (Algorithm 1 without pattern augmentation, run on A^T and
 * transposed as in Algorithm 4, step 1), splits M's entries by magnitude into
 * precision buckets (Algorithm 2, intervals of eq. (nint)), applies the
 * bucketed M (Algorithm 3) and solves A x = b with GMRES-based iterative
 * refinement preconditioned by it (Algorithm 4).
 *
 * Conventions
 *  - Matrices are square CSR, 0-based, int32 row pointers and column indices
 *    (column indices sorted ascending within a row, no duplicates), FP64
 *    values.  nnz fields are int64 but must fit in int32 row pointers.
 *  - Every pointer inside bspai_csr / bspai_pattern and every vector argument
 *    is DEVICE memory on the current HIP device, owned by the caller, and is
 *    only read (or, for outputs, written) during the call / the stream work
 *    it enqueues.  Host pointers are named *_host.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *  - Functions return BSPAI_OK (0) or a negative status; a message for the
 *    last failure of the calling thread is available from bspai_last_error().
 *    Nothing throws across this interface.
 */
#ifndef BSPAI_H
#define BSPAI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Storage precisions of the buckets (Table 2 of the paper plus bfloat16 and
 * OCP FP8 E4M3FN).  BSPAI_DROP is the pseudo-precision with unit roundoff 1
 * whose entries are discarded (Section 4, the choice u_q = 1). */
typedef enum {
    BSPAI_FP64 = 0,
    BSPAI_FP32 = 1,
    BSPAI_FP16 = 2,
    BSPAI_BF16 = 3,
    BSPAI_FP8_E4M3 = 4,
    BSPAI_DROP = 5
} bspai_prec;

enum {
    BSPAI_OK = 0,
    BSPAI_EINVAL = -1,   /* bad argument: sizes, unsorted or duplicate precisions, DROP not last, q > 6 */
    BSPAI_ENOMEM = -2,   /* device or host allocation failed */
    BSPAI_EHIP = -3,     /* HIP runtime error (including a solver synchronisation timeout) */
    BSPAI_EZEROROW = -4, /* a row of M would be zero: k is not in the shadow of its pattern (Section 4) */
    BSPAI_ERANK = -5,    /* a reduced least-squares problem is rank deficient */
    BSPAI_ENOCONV = -6,  /* i_max refinement steps without meeting a tolerance; x and stats are valid */
    BSPAI_ENAN = -7,     /* a NaN or infinity appeared in the residual */
    BSPAI_ESTAG = -8     /* the corrections stagnated (stop_reason 3) before tol_rr or tol_be was met;
                            x and stats are valid, x is the last iterate */
};

typedef struct {
    int32_t n;
    int64_t nnz;
    const int32_t *row_ptr; /* [n+1] */
    const int32_t *col;     /* [nnz] */
    const double *val;      /* [nnz] */
} bspai_csr;

typedef struct {
    int32_t n;
    int64_t nnz;
    const int32_t *row_ptr; /* [n+1] */
    const int32_t *col;     /* [nnz] */
} bspai_pattern;

typedef struct {
    int build_T;     /* also pack (M_b)^T, needed by bspai_apply_T and the transposed solve */
    int keep_fp64_M; /* keep the unbucketed FP64 M on the device (x_0 = M b, Algorithm 4 step 2) */
    int scale;       /* one-sided column scaling of A^T before the least squares (Section 4) */
    bspai_prec u_f;  /* precision of the SPAI least squares (Section 4's settings): BSPAI_FP64 (0,
                      * the default), BSPAI_FP32 or BSPAI_FP16; see bspai_build and
                      * bspai_build_adaptive.  Ignored by bspai_import */
} bspai_opts;

typedef struct bspai_handle bspai_handle;

/*
 * bspai_build -- SPAI of A on the pattern P, then bucketing.
 *   Row k of M solves min || e_k(I) - A^T(I, J) m ||_2 with J = P(k,:) and
 *   I the shadow { i : sum_{j in J} |a_{ji}| != 0 } (eq. (redprob) for A^T;
 *   Algorithm 1's least-squares steps with no augmentation), in FP64 by
 *   Householder QR.  Then ||M||_inf, the thresholds t_k = fl(eps_b ||M||_inf)/u_k
 *   and the buckets of eq. (nint); entries are stored in their bucket's format
 *   (fp16 and fp8 with a power-of-two per-bucket scale).
 *   A, P: device CSR (P NULL means the pattern of A).  precs[0..q-1]: host
 *   array, strictly increasing unit roundoff (fp64 < fp32 < fp16 < bf16 <
 *   fp8 < drop), DROP only last, 1 <= q <= 6.  opts may be NULL (defaults:
 *   build_T = 1, keep_fp64_M = 1, scale = 0, u_f = FP64).  On success *out
 *   owns device memory until bspai_free.  Synchronises `stream`.
 *   u_f = FP32 or FP16 (Section 4's single and half settings): each entry of
 *   the reduced matrix (scaled if `scale`) is rounded to u_f, the Householder
 *   QR and back substitution run in u_f arithmetic, and M's entries are
 *   rounded to u_f (kept as FP64 numbers for x_0 and the bucketing).  Only
 *   rows whose least squares fit one wavefront are supported there (|J| <= 64,
 *   at most 1,024 shadow candidates, a tile of at most 8,192 values): EINVAL
 *   otherwise.  An overflow of u_f (use `scale`) is ENAN.
 *   Errors: EINVAL, ENOMEM, EHIP, EZEROROW, ERANK, ENAN (no handle is returned).
 */
int bspai_build(const bspai_csr *A, const bspai_pattern *P, double eps_b, const bspai_prec *precs, int q,
                const bspai_opts *opts, bspai_handle **out, void *stream);

/*
 * bspai_import -- bucket an externally computed FP64 M (device CSR) exactly as
 * bspai_build does after its least squares (Algorithm 2 and the storage).
 *   Same precision rules, options and ownership as bspai_build; M is copied.
 */
int bspai_import(const bspai_csr *M, double eps_b, const bspai_prec *precs, int q, const bspai_opts *opts,
                 bspai_handle **out, void *stream);

/*
 * bspai_apply -- Y = M_b X (Algorithm 3 with the storage precision of each
 * bucket decoupled from the arithmetic): every stored value is decoded
 * exactly, the partial sum of each bucket is accumulated in FP32 (FP64 for
 * the fp64 bucket and for xy_prec = FP64), and the partials are added from
 * the least to the most precise bucket in FP64 before rounding to xy_prec.
 *   x, y: device arrays of n x nrhs values of type xy_prec (BSPAI_FP32 or
 *   BSPAI_FP64), row-major with leading dimension ld >= nrhs (ignored for
 *   nrhs = 1); x and y must not overlap.  Asynchronous on `stream`.
 */
int bspai_apply(const bspai_handle *M, const void *x, void *y, int nrhs, int64_t ld, bspai_prec xy_prec,
                void *stream);

/* bspai_apply_T -- Y = (M_b)^T X with the same stored values and bucket
 * assignment as bspai_apply (the handle must be built with build_T). */
int bspai_apply_T(const bspai_handle *M, const void *x, void *y, int nrhs, int64_t ld, bspai_prec xy_prec,
                  void *stream);

typedef struct {
    bspai_prec u_g; /* GMRES working precision, also the precision u_p of products with A: FP32 or FP64 */
    int ur_dd;      /* 1: residual r = b - A x in double-double (for u_r ~ u^2); 0: FP64 */
    double tau;     /* GMRES relative tolerance on the preconditioned residual */
    double tol_rr;  /* stop when ||r||_inf / ||b||_inf <= tol_rr */
    double tol_be;  /* stop when ||r||_inf / (||A||_inf ||x||_inf + ||b||_inf) <= tol_be */
    int i_max;      /* at most this many refinement corrections (<= 64) */
    int gmres_max;  /* at most this many GMRES iterations per correction; capped at min(n, 160),
                       the size whose rotated Hessenberg matrix stays on chip */
    int x0_mode;    /* 0: x_0 = M b with the FP64 M; 1: with M_b; 2: x_0 = 0; 3: x holds x_0 on entry */
    int trans;      /* 1: solve A^T x = b with (M_b)^T as a right preconditioner (adjoint solve) */
    double stag_ratio; /* stagnation: stop when ||d_i||/||x_{i+1}|| > stag_ratio times the previous ratio
                          (from the second correction on); 0 selects 0.5, a negative value never stops */
    int orth;          /* Arnoldi orthogonalisation: 0 modified Gram-Schmidt (the paper's), 1 classical
                          Gram-Schmidt twice (CGS2: two grid-wide reductions per step instead of j + 1;
                          one right-hand side per system: gmres_ir_solve / gmres_ir_solve_ab with
                          nrhs = 1, and bspai_multi_plan) */
} gmres_ir_tol;

typedef struct {
    int steps;       /* GMRES calls (corrections) made */
    int its_total;   /* total GMRES iterations */
    int stop_reason; /* 1 relres, 2 backward error, 3 stagnation, 4 i_max, 5 NaN */
    int status;      /* status code of this right-hand side: BSPAI_OK only for stop_reason 1 or 2;
                        ESTAG for 3, ENOCONV for 4, ENAN for 5 */
    int its[64];     /* GMRES iterations per correction */
    double eta[65];  /* normwise backward error before each correction and at the end */
    double relres[65];
} gmres_ir_stats;

/*
 * gmres_ir_solve -- BSPAI-GMRES-IR (Algorithm 4) on one GPU.
 *   x_0 per x0_mode; then, per step i: r_i = b - A x_i (FP64 or double-double,
 *   stored FP64), stopping tests, left-preconditioned MGS-GMRES on
 *   M_b A d = M_b r_i in u_g with A rounded to u_g (right-preconditioned
 *   A^T M_b^T for trans = 1) to relative tolerance tau, x_{i+1} = x_i + d_i in FP64.
 *   orth = 1 orthogonalises by CGS2 instead of MGS (nrhs = 1; EINVAL otherwise).
 *   Stops on tol_rr, tol_be, stagnation of ||d_i||/||x_{i+1}|| (more than
 *   stag_ratio times the previous ratio after the first correction) or i_max.
 *   A: device CSR; b, x: device FP64 arrays of n x nrhs, row-major (entry
 *   (i, c) at i * nrhs + c), 1 <= nrhs <= 64; st_host: host array of nrhs
 *   stats (or NULL).  nrhs = 1 runs as one persistent kernel; nrhs > 1 runs
 *   every column's refinement together, each pass over the vectors and each
 *   product with M_b and A serving all columns, every column stopping on its
 *   own tests (a finished column takes no further corrections).  Needs
 *   device workspace of about (gmres_max + 5) n nrhs values of u_g.
 *   M: handle from bspai_build / bspai_import (keep_fp64_M for x0_mode 0,
 *   build_T for trans).  Synchronises `stream`.  A solve's kernels keep every
 *   compute unit of its GPU in grid-wide exchanges, so solves on one GPU run
 *   one at a time: calls of the same kind (nrhs = 1, or nrhs > 1) from
 *   several threads of a process wait for each other; a solve that overlaps
 *   one of the other kind, or another process's, may end with BSPAI_EHIP
 *   (an exchange timeout) rather than wait.  Returns BSPAI_OK only when
 *   every right-hand side met tol_rr or tol_be; otherwise the worst of ENAN,
 *   ENOCONV (i_max reached) and ESTAG (stagnated first), in that order, with
 *   x and the stats still written.
 */
int gmres_ir_solve(const bspai_csr *A, const double *b, const bspai_handle *M, const gmres_ir_tol *tol,
                   double *x, int nrhs, gmres_ir_stats *st_host, void *stream);

/*
 * gmres_ir_solve_noalloc -- gmres_ir_solve for one right-hand side (nrhs = 1)
 * that allocates nothing.  For callers that cannot allocate device memory:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments (b, x: device FP64 [n]; st_host: one stats
 * struct or NULL), same kernels, results and errors as gmres_ir_solve with
 * nrhs = 1 and the same row split (bit-identical x and stats).  The solver's
 * workspace (Krylov basis, vectors, A rounded to u_g, exchange words) lives
 * in a 64 MiB array of device memory that the library holds on every GPU it
 * runs on until the process ends; EINVAL when the system needs more (about
 * 4 (gmres_max + 5) n + 8 nnz bytes in FP32 working precision: n = 65,536
 * with gmres_max 150 takes 44 MB) and for trans = 1 (the transposed solve
 * forms A^T in temporary storage).  Calls on one GPU share that array: calls
 * that overlap on one GPU (two streams, two threads) race and must not be
 * issued.  Every word that must start at zero is cleared by each call.  No
 * solver kernel timing (bspai_set_profiling is ignored).  Synchronises
 * `stream`.
 */
int gmres_ir_solve_noalloc(const bspai_csr *A, const double *b, const bspai_handle *M, const gmres_ir_tol *tol,
                           double *x, gmres_ir_stats *st_host, void *stream);

/*
 * gmres_ir_solve_ab -- gmres_ir_solve with A bucketed inside GMRES too
 * (Section 3, eqs. (nbe2) and (fe2)): every Krylov product with A (A^T for
 * trans) is the bucketed product of A_b (A_b^T), computed as bspai_apply
 * computes M_b's, instead of the product of A rounded to u_g.  The refinement
 * residual and the stopping tests keep the FP64 A.
 *   A_b: handle from bspai_import of A itself (same n, same device; build_T
 *   for trans), bucketed with its own eps and precisions; the caller keeps it
 *   alive during the call.  Other arguments, workspace and errors as
 *   gmres_ir_solve; EINVAL for a null A_b or one that does not fit A.
 */
int gmres_ir_solve_ab(const bspai_csr *A, const bspai_handle *A_b, const double *b, const bspai_handle *M,
                      const gmres_ir_tol *tol, double *x, int nrhs, gmres_ir_stats *st_host, void *stream);

/*
 * Many independent systems in one persistent launch (Algorithm 4 for each).
 *
 * bspai_multi_plan -- prepare the solve of systems A_k x_k = b_k, k < nsys,
 *   each with its own preconditioner M_k and the tolerances `tol` (as for
 *   gmres_ir_solve with nrhs = 1).  The plan copies A_k rounded to u_g (and
 *   A_k^T for trans) into device memory it owns, so A_k's values are read
 *   now; b_k and x_k are read and written at every launch and must stay
 *   allocated until bspai_multi_free.  The grid is cut into groups of
 *   blocks; each group takes the next system of its class off that class's
 *   device queue, largest first, until the queue is empty.
 *   group_blocks > 0: one class, every group of that many blocks (at least
 *   what keeps the largest system within 16 rows per thread).
 *   group_blocks = 0: size classes, each system solved by a group of the
 *   smallest power of two of blocks that keeps it within 8 rows per thread;
 *   the resident blocks are shared among the classes by estimated load
 *   (sqrt(n) times the exchange cost of the group size), a class that does
 *   not fit joining the next larger one.
 *   group_blocks = -1: autotune, i.e. plan size classes and one group size
 *   (the smallest above and its doublings up to 256), run each once, timed
 *   with HIP events, and keep the fastest (this writes every x_k; with
 *   x0_mode 3 each x_k is saved first and holds the caller's x_0 again when
 *   the call returns).
 *   max_groups (0: no limit) caps the number of groups.
 *   The launch is captured once into a HIP graph.  Synchronises `stream`.
 *   Results do not depend on which group takes a system, so replays with the
 *   same b_k give identical bits.  EINVAL when a group does not fit on the
 *   device or a system fails gmres_ir_solve's checks.
 * bspai_multi_launch -- replay the graph on `stream` (asynchronous, no
 *   allocation).  Launches of one plan must not overlap.
 * bspai_multi_poll -- 1 when the last launch has finished (reads one word of
 *   host memory that the kernel writes when its last group leaves), else 0.
 * bspai_multi_wait -- synchronise `stream`, copy the nsys stats to st_host (or
 *   skip if NULL); ENAN, ENOCONV or ESTAG (worst first, as for
 *   gmres_ir_solve) when some system met neither tolerance.
 * bspai_multi_free -- release the plan (NULL is ignored); waits for the device.
 */
typedef struct {
    bspai_csr A;                /* device CSR of system k */
    const double *b;            /* device FP64 [n] */
    double *x;                  /* device FP64 [n]: x_0 on entry for x0_mode 3, the solution on exit */
    const bspai_handle *M;      /* preconditioner of system k (same device) */
} bspai_system;

typedef struct bspai_multi bspai_multi;

int bspai_multi_plan(const bspai_system *sys, int nsys, const gmres_ir_tol *tol, int group_blocks, int max_groups,
                     bspai_multi **plan_out, void *stream);
int bspai_multi_launch(bspai_multi *plan, void *stream);
int bspai_multi_poll(const bspai_multi *plan);
int bspai_multi_wait(bspai_multi *plan, gmres_ir_stats *st_host, void *stream);
void bspai_multi_free(bspai_multi *plan);
/* bspai_multi_group_blocks -- the group size of a one-class plan (after
 * autotuning), 0 for a plan with size classes. */
int bspai_multi_group_blocks(const bspai_multi *plan);

/*
 * bspai_build_adaptive -- SPAI with Algorithm 1's augmentation loop, then
 * bucketing as bspai_build.  Run on A^T (row k of M is column k of
 * SPAI(A^T)).  Row k starts from J0(k,:) (NULL: the identity, the paper's
 * setting) and for step = 0..alpha: solves the least squares problem
 * (redprob) on the shadow of J_k by Householder QR (recomputed each round),
 * stops when the residual's 2-norm is <= eps or after the last solve, and
 * otherwise adds up to beta candidates: the rows j of A with a_jl != 0 for
 * some l in the residual's support (|s(l)| > 2^-40), not yet in J_k, scored by the residual
 * norm after adding j alone, rho_j^2 = ||s||^2 - (s . a_j)^2 / ||a_j||^2
 * (a_j the whole row j of A); rho_j is compared after rounding to fp32; the
 * candidates with rho_j at or below their mean (summed in ascending j),
 * ordered by (rho_j, j), join first.  No acceptable candidate ends the row.
 * Limits: initial entries + alpha * beta <= 64 per row; at most 4096 shadow
 * rows and 4096 distinct candidates per round (EINVAL names the row).
 * steps_host: NULL or a host array of n ints (least squares solves per row).
 * opts->u_f (FP64, FP32 or FP16; Section 4's double, single and half
 * settings) and opts->scale: every least squares solve is then that of
 * bspai_build with the same u_f and scaling (the reduced matrix rounded to
 * u_f, the QR and back substitution in u_f, M's values m_c d_c rounded to
 * u_f); the residual and the candidate scores are formed in FP64 from the
 * unscaled A and those values.  An overflow of u_f (use scale) is ENAN.
 * Errors: EZEROROW, ERANK, EINVAL, ENOMEM, EHIP, ENAN.  Synchronises `stream`.
 */
typedef struct {
    int alpha;      /* augmentation rounds: at most alpha + 1 solves per row */
    int beta;       /* at most beta entries added per round */
    double eps;     /* a row is done when its least squares residual is <= eps */
} bspai_adaptive_opts;

int bspai_build_adaptive(const bspai_csr *A, const bspai_pattern *J0, const bspai_adaptive_opts *ad, double eps_b,
                         const bspai_prec *precs, int q, const bspai_opts *opts, bspai_handle **M_out,
                         int32_t *steps_host, void *stream);

/* bspai_export_pattern -- copy M's CSR pattern to host arrays (n + 1 and nnz
 * ints; either may be NULL).  Synchronous. */
int bspai_export_pattern(const bspai_handle *M, int32_t *row_ptr_host, int32_t *col_host);

/*
 * Kernel of bspai_apply / bspai_apply_T for one right-hand side.  All of them
 * compute Algorithm 3's sum with the same per-bucket accumulation precision;
 * they differ in how entries are grouped over threads, so results can
 * differ in the last bits of the accumulation (each stays within the bound
 * of that accumulation).
 *   0 automatic: ELL/SELL copies when every bucket has one, else LDS tiles;
 *   1 the padded copies (ELL with byte or int16 column codes, else SELL-64);
 *   2 LDS tiles of contiguous rows (balanced for rows of any length);
 *   3 two rows per thread;  4 a group of lanes per row;
 *   5 entry-balanced tiles of whole rows (about 4096 entries per block, a
 *     plan built with the handle; rows of more than 64 entries are added by
 *     a whole wavefront), for rows of very different lengths with scattered
 *     columns; not available when a row has more than 4096 entries.
 * bspai_set_apply_kind -- use kernel `kind` for M_b (trans = 0) or M_b^T
 *   (trans = 1); EINVAL when the handle lacks what the kernel needs (kind 1:
 *   a copy for every bucket; padded copies are not built where padding would
 *   exceed half the entries).
 * bspai_tune_apply -- time every available kernel (20 products of an fp32
 *   vector each, HIP events on `stream`) for M_b and, with build_T, for
 *   M_b^T, and keep the fastest.  Synchronises `stream`.  Not called by
 *   bspai_build: a tuned handle's products may differ in the last bits from
 *   an untuned one's.
 */
int bspai_set_apply_kind(bspai_handle *M, int trans, int kind);
int bspai_tune_apply(bspai_handle *M, void *stream);

typedef struct {
    int32_t n;
    int32_t q;
    int64_t nnz;             /* entries of M (all buckets, dropped included) */
    bspai_prec precs[6];
    int64_t count[6];        /* entries per bucket */
    double threshold[6];     /* t_k = fl(eps_b ||M||_inf) / u_k */
    double scale[6];         /* power-of-two storage scale of each bucket */
    double norm_inf;         /* ||M||_inf of the FP64 M */
    double eps_b;
    int64_t bytes_values;    /* bytes of stored values */
    int64_t bytes_indices;   /* bytes of column indices and per-bucket row pointers */
    double storage_pct;      /* values of M_b as % of all nnz stored in u_1 (dropped: 0 B) */
    int32_t ell_width[6];    /* width W of the bucket's row-major padded copy used by bspai_apply (0: none) */
    int32_t col_bytes[6];    /* bytes per column index that bspai_apply reads for the bucket: 1 (index
                                into 256 offsets col - row), 2 (int16 offset) or 4 */
    int32_t apply_kind[2];   /* kernel bspai_apply / bspai_apply_T use (1..5, see bspai_set_apply_kind;
                                0 for apply_T without build_T) */
} bspai_bucket_stats;

/* bspai_stats -- bucket occupancy and storage of a handle (host struct). */
int bspai_stats(const bspai_handle *M, bspai_bucket_stats *out_host);

/*
 * bspai_export -- copy per-entry data back to the host in the CSR order of M:
 * bucket id (0-based) and stored value (decoded and scaled, 0 when dropped)
 * and, if kept, the FP64 M.  Any pointer may be NULL.  Synchronous.
 */
int bspai_export(const bspai_handle *M, int8_t *bucket_host, double *stored_host, double *m64_host);

/*
 * bspai_grad_vals -- gradient of a scalar loss with respect to the values of A
 * for the solution of A x = b: with lambda = A^{-T} dL/dx (a solve with
 * trans = 1), dL/da_ij = -lambda_i x_j.  Writes out[e] for every entry e of A's
 * pattern in CSR order.  lam, x: device FP64 [n]; out: device FP64 [nnz].
 * Asynchronous on `stream`.
 */
int bspai_grad_vals(const bspai_pattern *A, const double *lam, const double *x, double *out, void *stream);

/*
 * Instrumentation: with profiling on, gmres_ir_solve records HIP events on its
 * stream around its solver kernel; bspai_last_solve_kernel_ms returns the
 * elapsed time of the last such kernel in milliseconds (0 if none).
 */
void bspai_set_profiling(int on);
double bspai_last_solve_kernel_ms(void);
/* bspai_batched_mgs_profile -- with profiling on, gmres_ir_solve with several
 * right-hand sides times one launch in seven of its one-launch MGS kernel (see
 * bspai_set_batch_mode; the count runs across solves) with HIP events on its
 * stream; this returns the totals of the timed launches since the last reset:
 * milliseconds, launches and algorithmic bytes
 * ((j + 2) n c values of u_g for step j of a c-column group: v_0..v_j read,
 * v_{j+1} written), and every launch made while profiling was on, timed or
 * not.  Any pointer may be NULL; reset clears them. */
void bspai_batched_mgs_profile(int reset, double *ms_total, long long *launches, double *bytes,
                               long long *all_launches);

/*
 * bspai_set_batch_mode -- how gmres_ir_solve runs nrhs > 1 columns.
 *   1: all columns together; each MGS pass of an Arnoldi step is one kernel
 *      over the n x nrhs vectors (z read and written once per pass).
 *   2: consecutive groups of 16 bytes of u_g per row (4 columns in FP32, 2 in
 *      FP64; a trailing group of one more or fewer columns runs as in mode 1),
 *      each refined on its own; the Arnoldi step's whole MGS is one
 *      cooperative kernel that keeps the group's z in registers and reads
 *      each basis vector once (n <= 2,097,152).
 *   0 (default): mode 2 when it applies and either n nrhs values of u_g
 *      fill at least 64 MiB (there the passes are bound by bytes moved) or
 *      there are at most four groups, else mode 1.
 * Both modes compute the same arithmetic per column (the same MGS passes,
 * FP64 partial sums) and differ only in the order of the partial sums.
 * Process-wide setting; EINVAL for another value.
 */
int bspai_set_batch_mode(int mode);

/*
 * bspai_exchange_latency -- the latency floor of the persistent solver: runs
 * `iters` dependent grid-wide FP64 all-reductions by G co-resident blocks of
 * the solver's size with the solver's own exchange, and writes the average
 * time of one to *us_out (microseconds, host pointer).  Synchronises `stream`.
 * bspai_solve_blocks -- the number of blocks gmres_ir_solve uses for n rows
 *   with MGS (orth = 0, one right-hand side).
 */
int bspai_exchange_latency(int G, int iters, double *us_out, void *stream);
/* bspai_exchange_latency_placed -- the same measurement with the solver's LDS
 * footprint (one block per compute unit) and a placement: one_xcd = 0 runs G
 * blocks as the dispatcher spreads them over the XCDs; one_xcd = 1 launches
 * 8 G blocks (G <= 32), each reads its XCD from the XCC_ID hardware register,
 * and the first G on one XCD do the exchanges.  xcd_out: NULL or a host array
 * of G ints that receives the XCD of each participating block.  EHIP when no
 * XCD holds G blocks.  Synchronises `stream`. */
int bspai_exchange_latency_placed(int G, int iters, int one_xcd, double *us_out, int *xcd_out, void *stream);
int bspai_solve_blocks(int n);

/* bspai_release_workspace -- free the solvers' grow-only device workspaces
 * (the Krylov bases and vectors that gmres_ir_solve keeps between calls: one
 * for nrhs = 1, one for the column groups of nrhs > 1); the next solve
 * allocates them again.  Waits for the workspaces' devices.  For callers that
 * tear down the HIP runtime themselves: call it before the runtime goes
 * away. */
int bspai_release_workspace(void);

/* bspai_free -- release a handle (NULL is ignored).  Waits for the device. */
void bspai_free(bspai_handle *M);

/* bspai_last_error -- message of the last failure on the calling thread. */
const char *bspai_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* BSPAI_H */
