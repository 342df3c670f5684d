/*
 * pdipm — C ABI of the MI355X (gfx950) hot path of a pivoting-free
 * primal-dual interior-point method (arXiv 2508.16094).
 *
 * Problem class (Section 1, problem (1), with variable bounds):
 *     minimise   f(x) = c'x + 1/2 x'Qx + sum_i q4_i x_i^4 / 4
 *     subject to g(x) = A x - b - W (x o x) >= 0,    xl <= x <= xu
 * Derivatives evaluated on fixed sparsity patterns (Section 4):
 *     J = A - 2 W diag(x),   H = Q + diag(3 q4 o x^2) + 2 diag(W' lambda).
 * Per iteration the library forms the primal condensed KKT matrix
 * (Section 3, eq. kkt_primal)
 *     K = H + diag(Sigma_x + delta_p) + J' diag(Sigma_s) J,
 *     Sigma_s = lambda / (s + delta_d lambda),
 * factors P'KP = LL' with no pivoting (Section 2: SPD systems need none; the
 * ordering P is computed once on the host), and runs the triangular solves.
 *
 * Conventions
 *  - CSR arrays are 0-based, column indices sorted and unique per row;
 *    row pointers are int64, column indices int32.  Q is given by its lower
 *    triangle (diagonal included).
 *  - Host pointers (h_) are read during the call only; the caller keeps
 *    ownership.  Device pointers (d_) are HIP device addresses on the device
 *    current at create time.
 *  - Device memory is never allocated by the library: every handle works
 *    inside one caller-owned workspace (ipm_set_workspace) that must outlive
 *    the handle.  Work runs on the caller's stream (ipm_set_stream, default 0).
 *  - Every call returns an int status (PDIPM_* below); no exception crosses
 *    the ABI.  ipm_last_error() gives the message of the last failure.
 *  - A handle is not thread-safe; distinct handles are independent.
 */
#ifndef PDIPM_H
#define PDIPM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define PDIPM_OK 0                /* optimal / success */
#define PDIPM_MAX_ITER 1          /* iteration limit, best iterate returned */
#define PDIPM_TIME_LIMIT 2        /* wall-time limit, best iterate returned */
#define PDIPM_STALLED 3           /* line search failed, best iterate returned */
#define PDIPM_ERR_INVALID_ARG -1  /* bad input; message in ipm_last_error */
#define PDIPM_ERR_OUT_OF_MEMORY -2 /* workspace missing or too small */
#define PDIPM_ERR_NOT_PD -3       /* non-positive pivot (info->first_bad_col) */
#define PDIPM_ERR_NUMERICAL -4    /* NaN/Inf, or regularisation above 1e40 */
#define PDIPM_ERR_DEVICE -5       /* HIP runtime error; text in ipm_last_error */
#define PDIPM_ERR_NOT_ANALYZED -6 /* kkt_analyze / workspace not done yet */

#define PDIPM_FP64 0              /* factor and solve in FP64 */
#define PDIPM_FP32 1              /* FP32 factor + FP64 iterative refinement */
#define PDIPM_PRECISION_AUTO 2    /* ipm_create: FP32 or FP64 factors, chosen once */

#define PDIPM_HOST 0
#define PDIPM_DEVICE 1

#define PDIPM_KKT_PRIMAL 0        /* primal condensed K (Section 3, eq. kkt_primal) */
#define PDIPM_KKT_DUAL 1          /* dual condensed M (Section 3, eq. kkt_dual) */
#define PDIPM_KKT_AUGMENTED 2     /* augmented SQD system (Section 3, eq. augmentedKKT) */
#define PDIPM_KKT_AUTO 3          /* the condensed system with less factorisation work */

#define PDIPM_ORDER_LEVELS 0      /* nested dissection, separators = BFS levels */
#define PDIPM_ORDER_MULTILEVEL 1  /* nested dissection, separators from multilevel bisection */

typedef struct pdipm_csr {
  int64_t nrows, ncols;
  const int64_t* rowptr; /* [nrows+1]; NULL = empty matrix */
  const int32_t* colind; /* [nnz] */
  const double* val;     /* [nnz] */
} pdipm_csr;

typedef struct ipm_problem_desc {
  int64_t n, m;
  const double* c;  /* [n], required */
  const double* b;  /* [m], required when m > 0 */
  pdipm_csr A;      /* m x n, may be empty */
  pdipm_csr W;      /* m x n, may be empty.  W >= 0 keeps g concave (a
                       convex problem); negative entries make the problem
                       nonconvex, and the primal condensed form then relies
                       on inertia correction (Section 3, Regularization) */
  pdipm_csr Q;      /* n x n lower triangle, may be empty */
  const double* q4; /* [n] or NULL */
  const double* xl; /* [n] or NULL (= -inf); -INFINITY allowed */
  const double* xu; /* [n] or NULL (= +inf); +INFINITY allowed */
} ipm_problem_desc;

typedef struct ipm_options {
  double tol;            /* P, D, C tolerance, default 1e-6 */
  int32_t max_iter;      /* default 500 */
  double max_wall_time;  /* seconds, default 900 */
  double delta_p;        /* primal regularisation, default 1e-8 */
  double delta_d;        /* dual regularisation, default 1e-8 */
  int32_t precision;     /* PDIPM_FP64 or PDIPM_FP32 (workspace sized for it).
                            PDIPM_PRECISION_AUTO (ipm_create and
                            ipm_batch_create): space for both, and the create
                            call keeps FP32 factors with FP64
                            refinement when the factorisation time they save,
                            sum_j c_j^2 at 100 against 50 TFLOP/s, exceeds the
                            extra FP32 triangular solves per iteration (2 nnz(L)
                            4 bytes at 3 TB/s plus 6 us per launch each; two for
                            a single instance, 2 (min(ir_max, 3) - 1) for a
                            batch, whose refinement is fixed), else FP64
                            factors: on small or latency-bound systems FP32
                            factors save nothing and refinement costs extra.
                            From counts only, so the choice is deterministic;
                            kkt_analyze reports it. */
  int32_t ir_max;        /* refinement steps per solve, default 10 */
  double ir_tol;         /* backward-error target of refinement, 1e-14 */
  int32_t nd_leaf;       /* minimum-degree leaf size of the ordering, 64 */
  int32_t amalg_menu;    /* supernode amalgamation rule 0, 1, 2 (-1 = none) */
  int32_t print_level;   /* 0 silent, 1 per-iteration line on stderr */
  int32_t fp64_fallback; /* FP32 form: reserve FP64 factor space so that FP64
                            factors take over when FP32 refinement cannot reach
                            the accuracy an iteration needs (default 1) */
  int32_t use_graphs;    /* batched solve: 1 replays captured HIP graphs
                            (default), 0 launches the same kernels eagerly */
  int32_t graph_iters;   /* batched solve with graphs: Newton iterations held
                            by the one captured graph, replayed until every
                            instance has ended (default 20, 1 to 1000);
                            iterations the batch no longer needs cost only
                            their gated launches */
  int32_t kkt_form;      /* PDIPM_KKT_PRIMAL (default): factor the primal
                            condensed K (n x n).  PDIPM_KKT_DUAL: factor the
                            dual condensed (normal-equations) matrix
                            M = diag(1/Sigma_s) + J D J',
                            D = (H + Sigma_x + delta_p)^-1 (m x m; Section 3,
                            eq. kkt_dual), and solve K d = r as
                            d = D (r - J' M^-1 J D r), refined against K in
                            FP64.  Needs a diagonal Hessian (Q diagonal or
                            empty) and m >= 1; a non-positive pivot ends
                            ipm_solve with PDIPM_ERR_NUMERICAL (no inertia
                            correction).  The symbolic, pattern, value and
                            factor calls then describe M.
                            PDIPM_KKT_AUGMENTED: factor the augmented matrix
                            [H + diag(Sigma_x + delta_p), J'; J, -1/Sigma_s]
                            (order n + m, x first; Section 3, eq.
                            augmentedKKT), symmetric quasi-definite for convex
                            problems, as P'AP = L S L' with S = +1 on x
                            pivots and -1 on lambda pivots (Section 2: strong
                            factorisability, no pivoting), and solve K d = r
                            from A (d, w) = (r, 0), refined against K.  A
                            pivot of the wrong sign (a nonconvex H) ends
                            ipm_solve with PDIPM_ERR_NUMERICAL.  The factor
                            calls then describe A; kkt_get_factor gives L.
                            PDIPM_KKT_AUTO: when the Hessian is diagonal and
                            m >= 1, both condensed systems are analysed at
                            create and the one with fewer factorisation flops
                            sum_j (c_j^2 - 1) is kept (otherwise the primal);
                            kkt_analyze reports the choice. */
  int32_t ordering;      /* fill-reducing ordering, computed once on the host
                            (Section 2: minimum degree or nested dissection):
                            PDIPM_ORDER_LEVELS (default) takes BFS level sets
                            as separators; PDIPM_ORDER_MULTILEVEL bisects each
                            component the multilevel way (heavy-edge matching
                            down to 64 vertices, a BFS-grown bisection, greedy
                            boundary refinement on every level, parts of at
                            most 11/20 of the weight) and separates by the
                            smaller boundary side.  Both end in exact minimum
                            degree on components of at most nd_leaf vertices
                            and are deterministic. */
} ipm_options;

typedef struct kkt_symbolic_stats {
  int64_t n;             /* order of K */
  int64_t nnz_K;         /* entries of the lower triangle of K */
  int64_t nnz_L;         /* entries of L (structural, diagonal included) */
  int64_t nnz_L_stored;  /* entries of the supernodal panels (relaxed) */
  int64_t n_super;       /* supernodes */
  int64_t max_front;     /* largest front order */
  int64_t n_levels;      /* levels of the supernodal elimination tree */
  int64_t n_triples;     /* J'SJ products summed by the assembly */
  double flops;          /* sum_j (c_j^2 - 1), the factorisation's work */
  double update_bytes;   /* bytes of front update matrices (per precision) */
  int32_t kkt_form;      /* the system factored (PDIPM_KKT_*; -1 standalone) */
  int32_t precision;     /* factors a solve starts with: PDIPM_FP64 or
                            PDIPM_FP32 (the automatic choice resolved) */
} kkt_symbolic_stats;

typedef struct kkt_factor_info {
  int32_t status;
  int64_t first_bad_col; /* permuted column of the first bad pivot, or -1 */
  double ms;             /* device time of the factorisation */
  double flops;
} kkt_factor_info;

typedef struct kkt_solve_info {
  int32_t ir_steps;      /* refinement corrections applied */
  double residual;       /* backward error ||rhs - K x||_inf /
                            (max_i K_ii ||x||_inf + ||rhs||_inf) */
  int32_t fallback;      /* 0 none; 1: the FP32 factor's refinement missed the
                            target and kkt_solve refactored K in FP64 and
                            solved again (the handle keeps the FP64 factor) */
  double ms;
} kkt_solve_info;

typedef struct ipm_start {
  const double* x;       /* [n] predicted primal point */
  const double* lam;     /* [m] predicted multipliers */
  int32_t memspace;      /* PDIPM_HOST or PDIPM_DEVICE */
} ipm_start;

typedef struct ipm_result {
  int32_t status;
  int32_t iterations;
  double f, P, D, C, mu;
  double ms_total, ms_eval, ms_assemble, ms_factor, ms_solve;
  int32_t ir_steps;       /* refinement corrections over the solve */
  int32_t fp64_refactors; /* FP32 form: refactorisations in FP64 */
  int32_t inertia_corrections;
  double max_ir_residual; /* worst backward error of the KKT solves */
} ipm_result;

typedef struct ipm_profile {
  int64_t gemm32_launches; /* FP32 Schur-update and panel-solve GEMM launches */
  double gemm32_ms;        /* their summed device time (HIP events per launch) */
  double gemm32_flops;     /* their algorithmic flops (useful multiply-adds) */
  int64_t gemm64_launches; /* the same for FP64 factorisations */
  double gemm64_ms;
  double gemm64_flops;
  int64_t factorizations32, factorizations64;
  double factor_ms;        /* device time of whole factorisations */
  double factor_flops;     /* sum over factorisations of sum_j (c_j^2 - 1) */
  int64_t solves;          /* triangular solve pairs */
  double solve_bytes;      /* algorithmic bytes: 2 nnz(L) w + 4 n 8 per pair */
  double gemm32_bytes;     /* algorithmic bytes of the FP32 GEMM launches: each
                              operand block read once, C read and written once */
  double gemm64_bytes;     /* the same for FP64 */
} ipm_profile;

typedef struct ipm_handle ipm_handle;

void ipm_default_options(ipm_options* opts);
const char* ipm_status_string(int status);
const char* ipm_last_error(const ipm_handle* h); /* NULL h: last create error */

/* Create a solver for problem (1) from host CSR data (all arrays copied).
 * Builds the J and H patterns and the K pattern and runs the symbolic
 * analysis (Section 2: ordering once on the CPU).  Options NULL = defaults. */
int ipm_create(const ipm_problem_desc* prob, const ipm_options* opts, ipm_handle** out);

/* Standalone KKT handle for an explicit SPD matrix given by the lower CSR
 * pattern of K (n x n); values come later through kkt_set_values. */
int kkt_create_csr(int64_t n, const int64_t* h_rowptr, const int32_t* h_colind,
                   const ipm_options* opts, ipm_handle** out);

/* Symbolic statistics (host only; the analysis itself runs at create):
 * fill-reducing ordering, elimination tree, column counts and supernodes,
 * computed once and reused by every factorisation (Section 2: the ordering
 * is serial and amortised over the iterations).  out is a caller struct;
 * errors: INVALID_ARG for NULL arguments. */
int kkt_analyze(ipm_handle* h, kkt_symbolic_stats* out);

/* Export the symbolic analysis (host arrays sized from kkt_analyze):
 * perm[n] (perm[k] = original index at position k), etree[n] (permuted,
 * -1 root), colcount[n], sn_start[n_super+1], sn_rowptr[n_super+1],
 * sn_rows[sn_rowptr[n_super]] (permuted rows, own columns first). */
int kkt_get_symbolic(ipm_handle* h, int32_t* perm, int32_t* etree, int64_t* colcount,
                     int32_t* sn_start, int64_t* sn_rowptr, int32_t* sn_rows);

/* Lower CSR pattern of K in the original numbering (host arrays
 * rowptr[n+1], colind[nnz_K]); kkt_get_values uses this order. */
int kkt_get_pattern(ipm_handle* h, int64_t* rowptr, int32_t* colind);

/* Device workspace: query its size, hand it over (caller-owned, 256-byte
 * aligned, outlives the handle), select the stream (a hipStream_t). */
int ipm_workspace_query(ipm_handle* h, size_t* bytes);
int ipm_set_workspace(ipm_handle* h, void* d_ws, size_t bytes);
int ipm_set_stream(ipm_handle* h, void* stream);

/* Standalone: K values on the device in the order of kkt_create_csr's
 * pattern (lower triangle, FP64). */
int kkt_set_values(ipm_handle* h, const double* d_kval);

/* Assemble K for the point (x, lambda) with the given Sigma_s [m] and
 * Sigma_x [n] (device vectors, read on the handle's stream): evaluates J and
 * H on their patterns and sums H + diag(Sigma_x + delta_p) + J' diag(Sigma_s) J
 * (Section 3, eq. kkt_primal, with the bound term Sigma_x) into the
 * supernodal panels in the given precision (FP32: scaled to unit diagonal).
 * Errors: NOT_ANALYZED without a workspace, INVALID_ARG on a standalone
 * handle, NOT_PD when a diagonal entry of K is not positive. */
int kkt_assemble(ipm_handle* h, const double* d_x, const double* d_lam,
                 const double* d_sig_s, const double* d_sig_x, int precision);

/* Read back the assembled (not yet factored) K in kkt_get_pattern order. */
int kkt_get_values(ipm_handle* h, double* h_kval);

/* Numeric factorisation of the current K values (P'KP = LL', no pivoting).
 * Returns PDIPM_ERR_NOT_PD with info->first_bad_col on a pivot <= 0. */
int kkt_factor(ipm_handle* h, int precision, kkt_factor_info* info);

/* Export the factor: supernode by supernode, each panel column-major
 * (rows = its sn_rows, columns = its columns), as FP64 on the host;
 * total length nnz_L_stored. */
int kkt_get_factor(ipm_handle* h, double* h_lval);

/* Solve K x = rhs with the current factor (Section 2: L y = P'rhs, then
 * L'z = y, x = P z).  rhs and x are device FP64 vectors of length n in the
 * original numbering (may not alias); the handle's stream orders them.
 * FP64 iterative refinement against the assembled (or set) K runs up to
 * ir_max steps towards the backward error ir_tol; with an FP32 factor it
 * continues with conjugate gradients preconditioned by the factor, and when
 * that still misses the target and the handle has FP64 space, K is
 * refactored in FP64 (info->fallback = 1).  Errors: NOT_ANALYZED without a
 * valid factor, NUMERICAL on a non-finite residual. */
int kkt_solve(ipm_handle* h, const double* d_rhs, double* d_x, kkt_solve_info* info);

/* Evaluate the model at (x, lambda) on the device: f (host scalar),
 * grad f [n], g [m], J values in J's CSR order, H values in H's lower CSR
 * order (Section 4: derivative kernels on fixed patterns).  NULL outputs are
 * skipped. */
int ipm_evaluate(ipm_handle* h, const double* d_x, const double* d_lam, double* h_f,
                 double* d_grad, double* d_g, double* d_jval, double* d_hval);

/* Patterns used by ipm_evaluate: J = union of A and W (m x n), H = lower of
 * Q plus the diagonal (n x n).  Sizes through ipm_pattern_sizes. */
int ipm_pattern_sizes(ipm_handle* h, int64_t* nnz_j, int64_t* nnz_h);
int ipm_get_patterns(ipm_handle* h, int64_t* j_rowptr, int32_t* j_colind,
                     int64_t* h_rowptr, int32_t* h_colind);

/* Run the interior-point method to tolerance: the Newton iteration on the
 * barrier KKT conditions (Section 3, eq. kkt), each step from the primal
 * condensed system (Section 3, eq. kkt_primal) factored without pivoting,
 * inertia correction by delta_w I on a non-positive pivot (Section 3,
 * Regularization).  start NULL = cold start (x from the bounds,
 * s = max(g, 1), lambda = 1, z = 1); a start (host or device arrays per
 * start->memspace) is pushed into the interior first.  res (caller struct,
 * may be NULL) receives status, iterations, f, P, D, C, mu and phase times.
 * Returns the status (>= 0: best iterate kept) or an error code. */
int ipm_solve(ipm_handle* h, const ipm_start* start, ipm_result* res);

/* ipm_solve without a caller workspace, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  The handle is bound to the library's
 * own static device array of 64 MiB (one per GPU, held until the process
 * ends) and solved there; nothing is allocated.  Every call re-uploads the
 * handle's data into the array, so calls with different handles follow
 * one another safely, but calls that overlap on one GPU race, and
 * ipm_get_solution must come before the next call on that GPU.  Errors:
 * OUT_OF_MEMORY when ipm_workspace_query exceeds 64 MiB, INVALID_ARG on a
 * standalone or batch handle or when the current device is not the one
 * current at create; otherwise as ipm_solve. */
int ipm_solve_static(ipm_handle* h, const ipm_start* start, ipm_result* res);

/* Precision of the next ipm_solve on this handle: PDIPM_FP64, or
 * PDIPM_FP32 (FP32 factor, FP64 refinement).  The workspace must hold that
 * precision's factor: FP64 needs precision FP64 or fp64_fallback at create,
 * FP32 needs precision FP32 at create; otherwise INVALID_ARG. */
int ipm_set_precision(ipm_handle* h, int precision);

/* Copy the final iterate to caller buffers (memspace PDIPM_HOST/DEVICE);
 * NULL pointers are skipped. */
int ipm_get_solution(ipm_handle* h, double* x, double* s, double* lam, double* zl, double* zu,
                     int memspace);

/* Per-launch timing of the factorisation's GEMM kernel and phase totals
 * (adds two HIP events per GEMM launch while enabled).  Enabling resets the
 * counters. */
int ipm_set_profiling(ipm_handle* h, int enable);
int ipm_get_profile(ipm_handle* h, ipm_profile* out);

void ipm_destroy(ipm_handle* h);

/* ---------------------------------------------------------------------------
 * Batched solve (many independent LP/QP instances, Section 5 on throughput
 * for small instances): the instances are held as one block-diagonal
 * problem, so symbolic analysis, assembly, factorisation and the triangular
 * solves run once over all of them (each level of the elimination forest is
 * one launch across instances), while step lengths, centring and
 * termination are per instance.  The whole solve is one captured HIP graph
 * of graph_iters iterations (with use_graphs; default 20): a control kernel
 * sets device flags from the termination measures, every other kernel of
 * the graph reads its gate flag first, and the host replays the graph until
 * every instance has ended, reading the flags once per replay.  FP32 form:
 * FP32 factor and a fixed number min(ir_max, 3) of FP64 refinement steps
 * per solve; an instance whose direction misses its refinement target
 * 1e-2 tol (1 + ||grad f||) does not take it but repeats the iteration with
 * FP64 factors, which every instance uses from then on (when
 * fp64_fallback).  An instance whose direction is not finite ends with
 * PDIPM_ERR_NUMERICAL at its current iterate.  Instances must have W empty
 * and q4 NULL (LP or QP).
 * ------------------------------------------------------------------------- */
typedef struct ipm_batch ipm_batch;

typedef struct ipm_batch_info {
  int32_t iterations;      /* Newton iterations run (the slowest instance) */
  int32_t solved;          /* instances that reached status PDIPM_OK */
  int32_t graph_launches;  /* HIP graph replays (graph_iters iterations each) */
  int32_t fp64_from;       /* iteration from which FP64 factors were used (FP32
                              form), -1 never */
  int32_t factor_failures; /* factorisations that met a non-positive pivot */
  int32_t refine_misses;   /* iterations in which an instance missed its target */
  int32_t blocking;        /* blocking candidate used */
  int32_t pad;
  double ms_total;         /* wall time of ipm_batch_solve */
  double ms_capture;       /* of which graph capture and instantiation */
} ipm_batch_info;

/* Create a batch of count instances (host arrays copied; count >= 1).
 * Instance i owns columns xoff[i]..xoff[i+1]-1 and rows roff[i]..roff[i+1]-1
 * of the concatenated vectors (ipm_batch_offsets).  Errors as ipm_create,
 * message in ipm_batch_last_error(NULL). */
int ipm_batch_create(int32_t count, const ipm_problem_desc* probs, const ipm_options* opts,
                     ipm_batch** out);
int ipm_batch_analyze(ipm_batch* b, kkt_symbolic_stats* out);
/* xoff, roff: host arrays of count + 1 entries */
int ipm_batch_offsets(ipm_batch* b, int64_t* xoff, int64_t* roff);
int ipm_batch_workspace_query(ipm_batch* b, size_t* bytes);
/* Device workspace (caller-owned, 256-byte aligned, >= queried bytes) */
int ipm_batch_set_workspace(ipm_batch* b, void* d_workspace, size_t bytes);
/* Stream of the graph launches; with the null stream the batch creates a
 * private non-blocking stream (graph capture needs one). */
int ipm_batch_set_stream(ipm_batch* b, void* hip_stream);
/* Blocking candidates of the autotuner: small_h (fronts of at most this
 * height factor in one workgroup) and outer_blocks (trailing-update rank in
 * diagonal blocks); arrays of *count entries, either may be NULL. */
int ipm_batch_blockings(ipm_batch* b, int32_t* count, int32_t* small_h, int32_t* outer_blocks);
int ipm_batch_set_blocking(ipm_batch* b, int32_t index);
/* Times reps factorisations per candidate at the cold start point, keeps the
 * fastest; ms (NULL or count entries) receives each candidate's best time.
 * The choice is remembered for the rest of the process per size bucket
 * (precision, instance count, order, nnz(L) and largest front, each rounded
 * down to a power of two): a batch created later in the same bucket starts
 * with it (ipm_batch_info.blocking reports the blocking a solve used). */
int ipm_batch_autotune(ipm_batch* b, int32_t reps, int32_t* chosen, double* ms);
/* Solve every instance.  start: NULL (cold) or concatenated x (sum n_i) and
 * lambda (sum m_i), pushed into the interior per instance.  res: NULL or
 * count results (status, iterations, f, P, D, C, mu per instance). */
int ipm_batch_solve(ipm_batch* b, const ipm_start* start, ipm_result* res, ipm_batch_info* info);
/* Replace the right-hand sides b of all instances (host array, concatenated,
 * sum m_i entries): parametric problems re-solve on the same analysis. */
int ipm_batch_set_b(ipm_batch* b, const double* h_b);
/* Concatenated final iterates (memspace PDIPM_HOST/DEVICE; NULL skipped). */
int ipm_batch_get_solution(ipm_batch* b, double* x, double* s, double* lam, double* zl, double* zu,
                           int memspace);
const char* ipm_batch_last_error(const ipm_batch* b);
void ipm_batch_destroy(ipm_batch* b);

#ifdef __cplusplus
}
#endif
#endif /* PDIPM_H */
