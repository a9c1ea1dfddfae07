/*
 * ddg.h -- C ABI of the MI355X DDG two-level PCG library (libddg.so).
 *
 * The library solves A u = f for a sparse symmetric positive definite A with
 * conjugate gradients preconditioned by two-level symmetric multiplicative
 * overlapping Schwarz and the Discretely-Discontinuous Galerkin coarse grid of
 * Edwards and Bridson (arXiv:1504.00907):
 *   - coarse basis (Section 4): every generating vector restricted to every
 *     non-overlapping subdomain, orthonormalised per subdomain, rank-deficient
 *     columns dropped; coarse operator A0 = R0 A R0^T;
 *   - smoother (Section 6): subdomains expanded to graph distance `overlap`
 *     in the graph of A, local problems A_i = R~_i A R~_i^T solved exactly,
 *     multiplicative update u += R~_i^T A_i^{-1} R~_i (f - A u), one pass as
 *     pre-smoother, the coarse correction, one pass in reverse as post-smoother;
 *   - Krylov (Sections 1 and 7): CG from x0 = 0.
 *
 * Conventions shared by every entry point
 *   - Return value: DDG_OK (0) or a negative ddg_status.  No C++ exception
 *     crosses the ABI.  ddg_last_error() gives a thread-local message.
 *   - "host" pointers are ordinary CPU memory, read during the call only;
 *     the library copies what it keeps and never retains caller pointers.
 *   - "device" pointers are HIP device memory on the current device (for
 *     example torch tensors); they are used on the handle's stream and must
 *     stay valid until that stream has executed the enqueued work.
 *   - All floating-point vectors are float64.  Index arrays are int32 except
 *     CSR row pointers (int64).
 *   - A handle owns all device memory it allocates; it is bound to one
 *     stream and is not thread-safe.
 */
#ifndef DDG_H
#define DDG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ddg_handle_s* ddg_handle;

typedef enum {
  DDG_OK = 0,
  DDG_ERR_INVALID_ARG = -1,    /* malformed input (shape, range, symmetry, NaN) */
  DDG_ERR_NOT_SPD = -2,        /* a local or coarse pivot <= 0 (ddg_last_error names it) */
  DDG_ERR_RANK = -3,           /* every generating vector vanishes on some subdomain */
  DDG_ERR_BREAKDOWN = -4,      /* CG: p^T q <= 0 or a non-finite scalar */
  DDG_ERR_NO_CONVERGENCE = -5, /* max_iter reached; u holds the last iterate */
  DDG_ERR_HIP = -6,            /* HIP runtime failure */
  DDG_ERR_OOM = -7,            /* device allocation failed */
  DDG_ERR_UNSUPPORTED = -8     /* size beyond a documented kernel limit */
} ddg_status;

typedef enum {
  DDG_FP64 = 0,        /* everything float64 */
  DDG_MIXED_FP32 = 1,  /* local factors stored and applied in float32, float32 accumulation */
  DDG_MIXED_BF16 = 2   /* local factors stored in bfloat16, float32 accumulation */
} ddg_precision;

/* How a preconditioner application schedules its local solves (the results are
 * the same bit for bit). */
typedef enum {
  DDG_SCHEDULE_AUTO = 0,     /* the library's choice: currently COLOURS, measured as fast or faster
                                on every workload tried */
  DDG_SCHEDULE_COLOURS = 1,  /* one launch per colour phase, each preceded by a local-residual launch */
  DDG_SCHEDULE_QUEUE = 2,    /* one launch per sweep direction: (subdomain, chain) tasks taken from a
                                device queue in sweep order, each waiting only for the earlier
                                subdomains whose sets meet its neighbourhood */
  DDG_SCHEDULE_PERSISTENT = 3 /* ddg_solve runs the whole PCG of every system of the handle in one
                                launch: workgroups take (system, step, chunk or subdomain) tasks from
                                a device ring, and the last task of a step enqueues that system's
                                next step, so the systems of a batch advance and stop independently.
                                Systems start smallest first, enough at once for about eight subdomains
                                per CU; each stopped system hands its place to the next (per-system
                                solve_ms counts from a system's start).  Same results
                                bit for bit as COLOURS with one workgroup per subdomain.  Needs exact
                                local solves, two levels, at most 32 generating vectors and an
                                explicit coarse inverse accurate without refinement (else
                                DDG_ERR_UNSUPPORTED); ddg_apply_precond keeps the colour launches. */
} ddg_schedule;

/* Direction update of CG (Sections 1 and 7 use CG; the paper does not fix the
 * formula).  Both give the same iterates when the preconditioner is a fixed
 * symmetric linear operator; Polak-Ribiere keeps consecutive directions
 * A-conjugate when it is not (an inexact inner solve, reduced precision). */
typedef enum {
  DDG_CG_FLETCHER_REEVES = 0,  /* beta = r_{k+1}^T z_{k+1} / r_k^T z_k */
  DDG_CG_POLAK_RIBIERE = 1     /* beta = z_{k+1}^T (r_{k+1} - r_k) / r_k^T z_k */
} ddg_cg_variant;

/* Storage of A for the row dots of the solve (SpMV, local residuals, coarse
 * restriction, true residual).  The results are the same bit for bit. */
typedef enum {
  DDG_MATRIX_AUTO = 0,  /* diagonals when every system's entries lie on at most 6 offset pairs +-o
                           (5-, 7- and 13-point stencils), its rows are short and its values are
                           symmetric bit for bit; else the CSR rows */
  DDG_MATRIX_CSR = 1,   /* always the CSR rows */
  DDG_MATRIX_DIA = 2    /* (reported in ddg_info only) the diagonals are in use */
} ddg_matrix_format;

/* How each subdomain problem is treated inside the Schwarz sweeps. */
typedef enum {
  DDG_LOCAL_EXACT = 0,  /* solved exactly (Section 6): stored factorisation of every A_i */
  DDG_LOCAL_SSOR = 1    /* smoothed by symmetric SOR (Section 7, the timed 3D runs): ssor_sweeps
                           forward-then-backward sweeps from zero with relaxation ssor_omega, rows
                           taken colour by colour in a greedy colouring of the graph of A_i
                           (ascending local index); FP64; no local factors are stored */
} ddg_local_solver;

/* How the coarse problem A0 y = b0 is solved in every preconditioner application. */
typedef enum {
  DDG_COARSE_INVERSE = 0,  /* exactly (Section 4): the explicit inverse of A0 formed at setup, applied
                              as a tiled FP64 GEMV (with refinement steps when A0 is ill-conditioned) */
  DDG_COARSE_IC_CG = 1     /* inexactly (Section 7, the timed 3D runs): CG on A0 from zero,
                              preconditioned by the zero-fill incomplete Cholesky factor of A0 on its
                              block pattern (every entry of the blocks of coupled subdomains), stopped
                              at ||r|| <= ic_tol ||b0|| or after ic_maxit iterations.  The
                              preconditioner then depends on its input: use DDG_CG_POLAK_RIBIERE.
                              One workgroup per system runs the whole inner solve; the triangular
                              solves go level by level over the block pattern. */
} ddg_coarse_solver;

typedef struct {
  int32_t precision;   /* ddg_precision */
  int32_t max_iter;    /* CG iteration cap (default 1000, Section 7) */
  double rtol;         /* stop at ||r_k||_2 <= rtol ||f||_2 (recurrence residual) */
  double rank_tol;     /* drop coarse column j when |R_jj| <= rank_tol |R_11| (default 1e-10) */
  int32_t tile;        /* factor tile edge 16/32/64; 0 = chosen by the autotuner */
  int32_t block_target;/* merge local levels up to this many rows; 0 = automatic */
  int32_t check_every; /* CG iterations enqueued between host convergence checks (0 = 4) */
  int32_t schedule;    /* ddg_schedule (default DDG_SCHEDULE_AUTO) */
  int32_t cg_variant;  /* ddg_cg_variant (default DDG_CG_FLETCHER_REEVES) */
  void* stream;        /* hipStream_t for all work; NULL = the null stream */
  int32_t matrix_format; /* DDG_MATRIX_AUTO (default) or DDG_MATRIX_CSR */
  int32_t local_solver;  /* ddg_local_solver (default DDG_LOCAL_EXACT) */
  double ssor_omega;     /* relaxation of DDG_LOCAL_SSOR, 0 < omega < 2 (default 1) */
  int32_t ssor_sweeps;   /* symmetric sweeps of DDG_LOCAL_SSOR, >= 1 (default 1) */
  int32_t coarse_solver; /* ddg_coarse_solver (default DDG_COARSE_INVERSE) */
  double ic_tol;         /* relative residual of the DDG_COARSE_IC_CG inner solve, >= 0 (default 1e-6) */
  int32_t ic_maxit;      /* inner iteration cap of DDG_COARSE_IC_CG, >= 1 (default 200) */
} ddg_options;

typedef struct {
  int32_t status;          /* ddg_status of the last solve */
  int32_t iters;           /* number of products A p of the last solve */
  double rel_res;          /* recurrence ||r|| / ||f|| at exit */
  double true_rel_res;     /* ||f - A u|| / ||f|| recomputed on the device at exit */
  int32_t n_coarse;        /* N_c = sum of kept coarse columns */
  int32_t n_colours;       /* colour phases per sweep */
  int32_t n_parts;
  int32_t n_blocks;        /* total dense diagonal blocks over all local factors */
  double setup_ms;         /* last ddg_setup / ddg_refactor, device numeric part */
  double solve_ms;         /* last ddg_solve, wall time on the stream */
  int64_t factor_bytes;    /* stored local factor bytes */
  int64_t coarse_bytes;    /* stored coarse inverse bytes */
  int64_t sweep_bytes;     /* algorithmic HBM bytes of one full preconditioner sweep (both passes) */
  int64_t iter_bytes;      /* algorithmic HBM bytes of one CG iteration */
  int32_t tile;            /* tile edge of the local factors (16, 32 or 64) */
  int32_t schedule;        /* ddg_schedule in effect: DDG_SCHEDULE_COLOURS or DDG_SCHEDULE_QUEUE */
  int64_t envelope_elems;  /* sum over subdomains of the envelope of the lower triangle of A_i in its
                              local order: the entries a banded (envelope) Cholesky factor would store */
  int64_t set_rows;        /* sum over subdomains of |expanded set| */
  int64_t nbhd_rows;       /* sum over subdomains of |expanded set plus the rows coupled to it by A| */
  int32_t matrix_format;   /* storage the row dots read: DDG_MATRIX_CSR or DDG_MATRIX_DIA */
  int32_t levels;          /* 1 (no coarse space), 2, or 3 (ddg_setup_three_level) */
  int32_t n_coarsest;      /* unknowns of the coarsest level (N_c with two levels) */
  int32_t coarse_refine;   /* refinement steps y += X (b0 - A0 y) of every coarse solve (0 when the
                              explicit inverse X is accurate to working precision) */
  double coarse_inverse_err; /* estimate of the spectral radius of I - X A0 (largest
                              ||(I - X A0) v|| / ||v|| over eight normalised power steps from a fixed
                              pseudo-random v), at the last setup or refactor, worst system */
  int32_t coarse_solver;   /* ddg_coarse_solver in use */
  int32_t coarse_iters;    /* DDG_COARSE_IC_CG: inner CG iterations summed over the last solve's
                              coarse solves (worst system); 0 otherwise */
  int32_t sweep_groups;    /* largest number of workgroups that shared one chain of a local solve in
                              any colour launch since setup (1: every chain ran in one workgroup) */
} ddg_info;

/* Fill *opt with defaults: FP64, max_iter 1000, rtol 1e-8, rank_tol 1e-10, automatic tiles. */
void ddg_default_options(ddg_options* opt);

/*
 * Build the two-level preconditioner (Sections 4 and 6).
 *   n, row_ptr[n+1], col_idx[nnz], val[nnz]  host; full symmetric CSR, sorted columns,
 *                                             positive diagonal (checked).
 *   k, F[n*k]        host; generating vectors, column-major (column j at F + j*n), k <= 80.
 *                    k = 0 disables the coarse grid.
 *   part[n]          host; non-overlapping subdomain id of each unknown, in [0, n_parts);
 *                    every subdomain non-empty.
 *   overlap          graph distance Delta >= 0 in the stored pattern of A (Section 6).
 *   opt              may be NULL (defaults).
 * On success *out owns the handle.  Errors: INVALID_ARG, NOT_SPD, RANK, UNSUPPORTED,
 * HIP, OOM; *out is left NULL.
 */
int ddg_setup(ddg_handle* out, int64_t n, const int64_t* row_ptr, const int32_t* col_idx,
              const double* val, int32_t k, const double* F, const int32_t* part,
              int32_t n_parts, int32_t overlap, const ddg_options* opt);

/*
 * Three-level V-cycle (Section 6, three-level paragraph): the two-level method
 * is applied again to the coarse matrix A0 = R0 A R0^T, and one application of
 * that coarse two-level preconditioner M0^{-1} replaces the coarse solve
 * A0^{-1} inside every application on the fine level:
 *   e = fine pre-sweep;  e += R0^T M0^{-1} R0 (r - A e);  fine post-sweep.
 * The coarse level's unknowns are the kept coarse columns (subdomain-major);
 * its partition puts the columns of subdomain i into coarse subdomain part0[i],
 * its generating vectors are F0 = R0 F, its graph is the block pattern of A0
 * (subdomains coupled by A), and it uses the same overlap.  The coarse level is
 * FP64 throughout and ends with the exact coarsest solve of A1 = R1 A0 R1^T.
 *   arguments as ddg_setup, plus
 *   part0[n_parts]  host; coarse subdomain of every subdomain, in [0, n_parts0),
 *                   every coarse subdomain non-empty.
 * ddg_solve, ddg_refactor (both levels refactored), ddg_apply_precond and the
 * other single-system calls accept the handle; ddg_info.levels = 3.
 * Errors: as ddg_setup (a coarse-level failure's message starts with
 * "coarse level:"); INVALID_ARG also for k = 0 or a bad part0.
 */
int ddg_setup_three_level(ddg_handle* out, int64_t n, const int64_t* row_ptr, const int32_t* col_idx,
                          const double* val, int32_t k, const double* F, const int32_t* part, int32_t n_parts,
                          int32_t overlap, const int32_t* part0, int32_t n_parts0, const ddg_options* opt);

/*
 * New matrix values with the same pattern (device pointer, nnz float64 in the
 * CSR order given to ddg_setup).  Recomputes A0 = R0 A R0^T, its inverse and
 * every local factor; the coarse basis R0 depends only on F and the partition
 * and is kept (Section 4).  Errors: NOT_SPD, HIP.
 */
int ddg_refactor(ddg_handle h, const double* val_dev);

/*
 * PCG solve (Sections 6-7): u = DDG-PCG(f) from x0 = 0.
 *   f_dev[n], u_dev[n] device; u_dev is written.  info may be NULL.
 * Returns DDG_OK, DDG_ERR_NO_CONVERGENCE (u holds the last iterate),
 * DDG_ERR_BREAKDOWN, DDG_ERR_INVALID_ARG (non-finite f) or DDG_ERR_HIP.
 */
int ddg_solve(ddg_handle h, const double* f_dev, double* u_dev, ddg_info* info);

/*
 * Batches of independent systems.  Many systems of uneven sizes share one
 * handle and advance together: every kernel launch of the solve covers all
 * systems still iterating (the local solves of a colour, for instance, run
 * every such system's subdomains of that colour in one launch), while each
 * system keeps its own CG scalars, stopping test and status (the method of
 * Sections 4-7 applied to each system separately).  Converged systems drop
 * out of the launches.  System b is described by a ddg_problem with the
 * meaning of ddg_setup's arguments (host arrays, copied during the call).
 */
typedef struct {
  int64_t n;
  const int64_t* row_ptr;   /* n+1 */
  const int32_t* col_idx;   /* row_ptr[n], local column ids */
  const double* val;
  int32_t k;                /* generating vectors (<= 80); may differ between systems */
  const double* F;          /* n x k column-major */
  const int32_t* part;      /* n, ids in [0, n_parts) */
  int32_t n_parts;
} ddg_problem;

/*
 * Set up nb systems in one handle (same options and overlap for all).  The
 * handle's vectors are the concatenation of the systems' vectors in batch
 * order (system b at rows row_off[b].., see ddg_batch_layout); ddg_solve,
 * ddg_refactor (values concatenated in the same order), ddg_spmv and
 * ddg_apply_precond act on all systems at once.  Errors as ddg_setup, with
 * the message naming the system; UNSUPPORTED beyond 2^31 - 1 total rows.
 */
int ddg_setup_batched(ddg_handle* out, int32_t nb, const ddg_problem* probs, int32_t overlap,
                      const ddg_options* opt);

/*
 * Solve every system of the batch: f_dev, u_dev are the concatenated
 * right-hand sides and solutions (device).  infos (nb entries, may be NULL)
 * receives per system: status, iters, rel_res, true_rel_res, n_coarse,
 * n_parts, and solve_ms = device time from the start of the batch solve to
 * the iteration at which that system stopped.  The return code is DDG_OK
 * when every system converged, else the first failing system's status.
 */
int ddg_solve_batched(ddg_handle h, const double* f_dev, double* u_dev, ddg_info* infos);

/* One measured candidate of ddg_tune_batched. */
typedef struct {
  int32_t tile;           /* tile edge of the local factors (16, 32, 64) */
  int32_t block_target;   /* level merge target (0 = merge only levels under 16 rows) */
  double precond_ms;      /* mean preconditioner application on the sample; -1 if the shape does not fit */
  int64_t factor_bytes;   /* local factor storage on the sample */
} ddg_tune_entry;

/*
 * Autotuner for the launch shape of the local solves (an implementation
 * choice; the method is unchanged).  Sets up a sample of the batch
 * (max_sample systems spread evenly over the size order; 0 = enough systems
 * for about 4096 subdomains, or all of them) for every
 * candidate tile edge {16, 32, 64} x level merge target {0, 64, 128}, times
 * preconditioner applications with HIP events, and writes *best = *base
 * (NULL = defaults) with the fastest tile and block_target.  report (may be
 * NULL) receives up to report_cap candidates, *n_report their count.
 * cache_path (may be NULL) is a text file of "key tile block_target ms" lines
 * keyed by the batch's shape, precision and device: a hit returns without
 * measuring (report then stays empty), a miss appends the result.
 * Uses the device and the default stream of base.  Errors: INVALID_ARG,
 * UNSUPPORTED (no candidate fits), and those of ddg_setup_batched.
 */
int ddg_tune_batched(int32_t nb, const ddg_problem* probs, int32_t overlap, const ddg_options* base,
                     int32_t max_sample, const char* cache_path, ddg_options* best, ddg_tune_entry* report,
                     int32_t report_cap, int32_t* n_report);

/* Batch layout: *nb, row_off[nb+1] (first row of each system), sub_off[nb+1]
 * (first subdomain).  Any output pointer may be NULL. */
int ddg_batch_layout(ddg_handle h, int32_t* nb, int64_t* row_off, int32_t* sub_off);

/* z = M^{-1} r, one application of the two-level preconditioner (Section 6). Device vectors. */
int ddg_apply_precond(ddg_handle h, const double* r_dev, double* z_dev);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): z = M^{-1} r
 * exactly as ddg_apply_precond computes it (same kernels, same order, same
 * bits), with the buffers those kernels fill and read back within the call
 * (local residuals, coarse restriction partials, coarse right-hand side and
 * solution, coarse GEMV partials) taken from a static device array of 32 MiB
 * that the library holds on every GPU it runs on until the process ends.  The
 * call allocates nothing: no hipMalloc, hipFree or allocating library call
 * (profiling, if enabled on the handle, is skipped for the call).
 *   r_dev[n], z_dev[n] device, caller-owned; the handle's device must be current.
 * Every call on one GPU shares that GPU's array and leaves its contents
 * behind; calls that overlap on one GPU (several streams or threads) race.
 * Errors: INVALID_ARG (null pointers, analysis-only handle, another device
 * current), UNSUPPORTED (the handle needs more than 32 MiB of such buffers:
 * 8 bytes per row of every expanded set plus the coarse buffers), HIP.
 */
int ddg_apply_precond_noalloc(ddg_handle h, const double* r_dev, double* z_dev);

/*
 * The first `stages` steps of M^{-1} r: stages 0..C-1 are the pre-sweep
 * colour phases, stage C the coarse correction, C+1..2C the post-sweep phases
 * (so stages = 2C+1 equals ddg_apply_precond).  Writes the partial
 * correction to e_dev.  For checking properties at full size.
 */
int ddg_apply_precond_stages(ddg_handle h, const double* r_dev, double* e_dev, int32_t stages);

/* y = A x on the device (the operator given to ddg_setup / ddg_refactor). */
int ddg_spmv(ddg_handle h, const double* x_dev, double* y_dev);

/* Fill *info with the handle's sizes and the statistics of the last setup/solve. */
int ddg_get_info(ddg_handle h, ddg_info* info);

/*
 * CG history of system `system` (0 for a single system) in the last solve:
 * alpha[j] = r_j^T z_j / p_j^T A p_j (j < iters), beta[j] of the direction
 * update after iteration j+1 (j < iters - 1), rel_res[j] = ||r_j|| / ||f||
 * (j <= iters; rel_res[0] = 1).  Host buffers of cap entries each (any may be
 * NULL); *count receives iters.  Errors: INVALID_ARG (bad system, no solve yet).
 */
int ddg_cg_history(ddg_handle h, int32_t system, double* alpha, double* beta, double* rel_res, int32_t cap,
                   int32_t* count);

/*
 * Reporting of Section 7 for system `system` of the last solve:
 *   frac_iters  where the linear interpolation of log ||r_j|| / ||f|| between
 *               the last iterate above rtol and the first at or below it meets
 *               log rtol (NaN when rtol was not reached);
 *   lambda_min, lambda_max  extreme eigenvalues of the Lanczos tridiagonal
 *               built from the CG coefficients (T_jj = 1/alpha_j +
 *               beta_{j-1}/alpha_{j-1}, T_{j,j+1} = sqrt(beta_j)/alpha_j), by
 *               Sturm-sequence bisection; kappa = lambda_max / lambda_min, the
 *               condition estimate of M^{-1} A;
 *   iter_bound  smallest k with 2 ((sqrt(kappa)-1)/(sqrt(kappa)+1))^k <= rtol,
 *               the CG bound the paper reports for solves stopped at the cap.
 * Computed on the host from ddg_cg_history.  Errors as ddg_cg_history.
 */
typedef struct {
  int32_t iters;
  int32_t iter_bound;
  double frac_iters;
  double lambda_min;
  double lambda_max;
  double kappa;
} ddg_cg_report;

int ddg_cg_report_get(ddg_handle h, int32_t system, ddg_cg_report* out);

/* Items for ddg_export (host buffers; `bytes` must equal the exact size). */
typedef enum {
  DDG_EXPORT_COLOURS = 0,   /* int32[n_parts]: colour of each subdomain */
  DDG_EXPORT_SET_PTR = 1,   /* int64[n_parts+1]: offsets of the expanded sets */
  DDG_EXPORT_SET_IDX = 2,   /* int32[sum |expanded set|]: global ids, in the local order of the factors */
  DDG_EXPORT_KCOUNTS = 3,   /* int32[n_parts]: kept coarse columns per subdomain */
  DDG_EXPORT_A0 = 4,        /* float64[sum_b N_c(b)^2]: A0 = R0 A R0^T, row-major, one block per system */
  DDG_EXPORT_Q = 5,         /* float64[n*k]: orthonormal coarse basis, node-major (row g: k values) */
  DDG_EXPORT_BLOCKS = 6     /* int32[n_blocks*3]: (subdomain, first local row, rows) per block */
} ddg_export_item;

/* Copy an internal structure to a host buffer.  Returns the needed byte count
 * through *bytes_needed when host_buf is NULL. */
int ddg_export(ddg_handle h, int32_t what, void* host_buf, int64_t bytes, int64_t* bytes_needed);

/*
 * Kernel timing for the roofline: when enabled, the library records HIP events
 * (on the handle's stream) around every local-solve launch and accumulates
 * their durations.  ddg_profile_read returns total milliseconds, the number
 * of launches and their algorithmic HBM bytes since the last reset.
 */
int ddg_profile_enable(ddg_handle h, int32_t on);
int ddg_profile_read(ddg_handle h, double* sweep_ms, int64_t* sweep_launches, int64_t* sweep_bytes,
                     int32_t reset);
/* Launches that ran for no system (enqueued ahead of the convergence check
 * after every system had stopped; their kernels return at once): their total
 * milliseconds and count since the last reset of ddg_profile_read.  They are
 * not part of ddg_profile_read's figures.  A launch enqueued by CG iteration t
 * is credited with the bytes of the systems still iterating after t. */
int ddg_profile_read_idle(ddg_handle h, double* idle_ms, int64_t* idle_launches);

/*
 * Host-only symbolic analysis (no device memory, no GPU calls): validates the
 * pattern and partition and builds the expanded sets (Section 6), the
 * conflict colouring and the level blocks of the local factors.  The handle
 * supports ddg_get_info (n_colours, n_parts, n_blocks, factor_bytes) and
 * ddg_export of the integer items (COLOURS, SET_PTR, SET_IDX, BLOCKS); every
 * other call on it returns DDG_ERR_INVALID_ARG.  Free it with ddg_destroy.
 */
int ddg_analyze(ddg_handle* out, int64_t n, const int64_t* row_ptr, const int32_t* col_idx,
                const int32_t* part, int32_t n_parts, int32_t overlap, const ddg_options* opt);

/* Release every device resource of the handle (NULL is ignored). */
void ddg_destroy(ddg_handle h);

/* Thread-local message describing the last error ("" when none). */
const char* ddg_last_error(void);

/* ---------------------------------------------------------------------------
 * Cell-centred variable-coefficient diffusion (the operator family of the
 * differentiation workload).  dims[3] = (nx, ny, nz), cells x-fastest;
 * the grid is 3D when nz > 1, 2D when nz = 1 < ny, else 1D, and boundary faces
 * exist only along its own axes.  Face coefficient between cells L, R is the harmonic
 * mean 2 kL kR / (kL + kR); a boundary face with a zero-Dirichlet ghost adds
 * 2 kc to the diagonal, a boundary face without one carries no flux (Neumann).
 * kappa = exp(theta).
 * ------------------------------------------------------------------------- */

/* Which boundary faces carry the zero-Dirichlet ghost. */
typedef enum {
  DDG_BC_DIRICHLET = 0,  /* every boundary face */
  DDG_BC_X0 = 1          /* only the faces on x = 0; Neumann elsewhere (Section 7, 3D Poisson problem:
                            one Dirichlet face, the rest Neumann) */
} ddg_bc;

/*
 * Write the CSR values of A(exp(theta)) into val_dev, in the sorted-column
 * CSR order of the same operator: row g holds its existing neighbours
 * g - nx*ny, g - nx, g - 1, the diagonal, g + 1, g + nx, g + nx*ny, in that
 * order (the pattern is the caller's; it is fixed by dims).  theta_dev[ncell],
 * val_dev[nnz] device, caller-owned; bc a ddg_bc value; stream may be NULL
 * (default stream).  Errors: DDG_ERR_INVALID_ARG for non-positive dims, NULL
 * pointers or an unknown bc; the launch is asynchronous and reads no other memory.
 */
int ddg_stencil_assemble(const int32_t dims[3], const double* theta_dev, int32_t bc, double* val_dev,
                         void* stream);

/*
 * Per-cell gradient dL/dtheta_c = -kappa_c * lam^T (dA/dkappa_c) u
 * (adjoint identity for L(u(theta)) with A lam = dL/du), for the operator
 * ddg_stencil_assemble builds with the same bc.
 * theta_dev, u_dev, lam_dev, grad_dev: device [ncell].  Errors as ddg_stencil_assemble.
 */
int ddg_stencil_coeff_grad(const int32_t dims[3], const double* theta_dev, const double* u_dev,
                           const double* lam_dev, int32_t bc, double* grad_dev, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* DDG_H */
