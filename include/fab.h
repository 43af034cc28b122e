/*
 * fab.h -- C ABI of libfab: the restarted, sketched, window-truncated Krylov
 * method for the action of a matrix function, x = f(A) b, on one AMD MI355X
 * (gfx950) GPU.
 *
 * Method (Guidotti, Martinsson, Acebron, Monteiro, "Accelerating a restarted
 * Krylov method for matrix functions with randomization"):
 *   - each cycle runs the randomized Arnoldi iteration of Algorithm 1, with the
 *     sketch-space Gram-Schmidt limited to the last k basis vectors;
 *   - the sketch S is the sparse sign matrix of eq. (sparse_sign_sketch),
 *     zeta nonzeros of +-1/sqrt(zeta) per column in distinct rows;
 *   - the basis is whitened by a thin QR of S W (appendix, eq. A.1), which
 *     keeps the decomposition A V = V X + h v e_m^T Arnoldi-like
 *     (eq. rand_arnoldi);
 *   - cycles are chained as in Algorithm 2 / eq. (restart_combined), but f of
 *     the growing block matrix is evaluated through a fixed quadrature rule
 *     (the quadrature-based restart Section 4 names), so the per-cycle small
 *     work stays m x m;
 *   - the loop stops when the estimated remaining error is at most tol ||x||
 *     for every time point: the successive-difference estimate after
 *     Algorithm 2, ||y_c|| = ||x_c - x_{c-1}||, continued by the geometric tail
 *     of the increments, ||y_c|| q / (1 - q) with q their contraction ratio
 *     (see fab_info.err_est);
 *   - every sum over blocks is formed in a fixed order (per-block partials,
 *     then one reduction), so a solve gives the same bits on every run.
 *
 * Conventions
 *   - Every pointer is DEVICE memory unless its name starts with h_.
 *   - Every call returns fab_status and never aborts.  Negative values are
 *     errors (nothing usable was produced); positive values are results with a
 *     note (FAB_OK_BREAKDOWN is exact; FAB_W_* are warnings).
 *   - Work is enqueued on the context's HIP stream.  fab_solve returns after
 *     h_info is filled (it synchronises the stream once per cycle).
 *   - Ownership: the caller owns and keeps alive A's arrays, b, x and the
 *     workspace (typically torch tensors).  The library owns fab_ctx and fab_op
 *     objects, the arrays of operators made by fab_op_transpose, and an 8 KB
 *     reduction buffer per context (fab_dot).
 *   - Thread safety: one context per host thread; calls on one context are
 *     serialised by the caller.
 */
#ifndef FAB_H
#define FAB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FAB_OK = 0,
  FAB_OK_BREAKDOWN = 1,     /* invariant Krylov subspace found: result exact */
  FAB_W_NOT_CONVERGED = 2,  /* max_cycles reached; x holds the last iterate  */
  FAB_W_QUADRATURE = 3,     /* rule error > max(tol/10, 1e-11) (see below)   */
  FAB_E_INVALID = -1,       /* bad argument (sizes, nulls, parameter ranges)  */
  FAB_E_UNSUPPORTED = -2,   /* valid but not supported by this build          */
  FAB_E_HIP = -3,           /* a HIP runtime call failed                      */
  FAB_E_NONFINITE = -4,     /* NaN/Inf met in the iteration (A or b)          */
  FAB_E_DIVERGED = -5,      /* an increment exceeded 1e8 ||x|| (see fab_divergence_limit) */
  FAB_E_WORKSPACE = -6      /* work_bytes smaller than fab_workspace_size     */
} fab_status;

typedef enum { FAB_F64 = 0, FAB_F32 = 1 } fab_dtype;        /* A values and basis; x is FP64 */
/* The function f of f(A) b.  t is a per-call parameter (h_t) of the timed functions.
 *   FAB_EXP_NEG  exp(-t z)          the heat equation's solution operator (Section 5.1, 5.3)
 *   FAB_INVSQRT  z^(-1/2)           a Stieltjes function (Section 4); needs spec_lo > 0
 *   FAB_PHI1_NEG phi_1(-t z) = (1 - e^{-t z}) / (t z), the phi function of eq. conv_diff_sol3
 *   FAB_COS_SQRT cos(t sqrt z)      the membrane solution of eq. drum_sol (t absorbs the wave speed);
 *                needs the spectral interval 0 <= spec_lo < spec_hi (the rule is an ellipse
 *                around it, accurate for t sqrt(spec_hi) up to ~100 with the default 256 nodes) */
typedef enum { FAB_EXP_NEG = 0, FAB_INVSQRT = 1, FAB_PHI1_NEG = 2, FAB_COS_SQRT = 3 } fab_fun;
/* FAB_SKETCHED: the sketched cycles with the quadrature restart (fixed m x m work per cycle).
 * FAB_PLAIN_RESTART: classical restarted Arnoldi (CGS2) with the same restart, as a comparator.
 * FAB_SKETCHED_GROWING: the sketched cycles with the restart as Algorithm 2 states it, f applied
 *   to the growing block matrix of all cycles so far; exp(-t z) only, one right-hand side, and
 *   max_cycles * m <= 1024 (FAB_E_UNSUPPORTED otherwise; also when exp(-t M) e_1 would need more
 *   than 16384 Taylor steps of norm 2, i.e. t ||M||_1 > 32768). */
typedef enum { FAB_SKETCHED = 0, FAB_PLAIN_RESTART = 1, FAB_SKETCHED_GROWING = 2 } fab_method;

/* Solver parameters (Algorithm 2's arguments plus the sketch). */
typedef struct {
  int32_t m;          /* cycle length (basis size per cycle), 1 <= m <= 64            */
  int32_t k;          /* truncation window of the Gram-Schmidt, 1 <= k <= m          */
  int32_t d;          /* sketch rows, m+1 <= d <= 4096                                */
  int32_t zeta;       /* nonzeros per sketch column, 1 <= zeta <= min(32, d)          */
  uint64_t seed;      /* defines S (Philox4x32-7 counter-based spec, see fab_sketch_table) */
  double tol;         /* relative update tolerance, >= 0                              */
  int32_t max_cycles; /* >= 1                                                          */
  int32_t method;     /* fab_method; FAB_PLAIN_RESTART ignores k, d, zeta, seed        */
  int32_t n_quad;     /* 0 = default rule size (128; 256 for FAB_COS_SQRT), else 8..512, a multiple of 8 */
  double spec_lo;     /* spectral interval for FAB_INVSQRT and FAB_COS_SQRT (required there) */
  double spec_hi;
} fab_params;

typedef struct {
  int32_t status;          /* fab_status of the solve                               */
  int32_t cycles;          /* restart cycles run                                    */
  int32_t matvecs;         /* products with A                                       */
  int32_t group;           /* members per block of the fused product + sketch kernel */
  double est_rel_update;   /* max_t ||y_t|| / ||x_t|| of the last cycle (the relative *
                            * difference of two successive cycles, Alg. 2)          */
  double quad_rule_error;  /* error of the partial-fraction rule r against f over   *
                            * the spectral region, max over 256 samples and t: exp  *
                            * and phi_1: |r - f| at t z = 0 and t z geometric in    *
                            * [1e-4, 1e4]; cos(t sqrt z): |r - f| at sqrt z uniform *
                            * in [sqrt lo, sqrt hi]; z^(-1/2): |r/f - 1| at z       *
                            * geometric in [lo, hi].  The                           *
                            * restarted iteration with a fixed rule converges to     *
                            * r(A) b, so this bounds what the rule adds to the error */
  double kappa_T;          /* conditioning of the sketched basis: max over cycles of *
                            * max_i T_ii / min_i T_ii for the whitening factor T of  *
                            * S W = Q T (appendix eq. A.1), a lower bound on         *
                            * cond_2(S W); 1 for the plain method (T = I)            */
  double err_est;          /* the stopping test's estimate of the remaining relative *
                            * error after the last cycle (infinite when the          *
                            * increments did not contract): max_t of                 *
                            * (||y_t|| / ||x_t||) q / (1 - q), q the largest of the  *
                            * last three ratios ||y_t|| / ||y_t||_prev (fewer in     *
                            * cycles 2 and 3), or ||y_t|| / ||x_t|| alone where that *
                            * is at most the unit roundoff of the value type (2^-53  *
                            * FP64, 2^-24 FP32).  A time point that has passed       *
                            * (estimate <= tol) keeps that estimate and is not       *
                            * tested again; the solve stops when err_est <= tol      */
} fab_info;

typedef struct fab_ctx fab_ctx;
typedef struct fab_op fab_op;

/* Create a context bound to the current HIP device and to hip_stream (a
 * hipStream_t; NULL = the null stream).  No passage of the paper: the device,
 * stream and cached launch graphs that every call below runs on.
 * Errors: FAB_E_INVALID (ctx NULL), FAB_E_HIP. */
fab_status fab_create(fab_ctx** ctx, void* hip_stream);
fab_status fab_destroy(fab_ctx* ctx);

/* The operator A of the problem statement (Algorithm 2's first argument; the
 * sparse matrices of Section 5).
 * Wrap a CSR matrix (n x n) without copying.  rowptr[n+1], colind[nnz] are
 * int32 (ascending columns per row are not required); vals[nnz] are FP64 or FP32
 * (dtype).  BORROWS the three arrays: they must outlive the operator, and their
 * structure must not change while it exists.  Creation checks the structure on
 * the device (row pointers non-decreasing from 0 to nnz, column indices in
 * [0, n)), after the work already queued on the caller's stream, and
 * synchronises the context's stream.  When every column index lies within
 * [-32768, 32767] of the first row of its row's 256-row tile (bandwidth below
 * 32K, e.g. grid operators in natural order), creation also derives a 16-bit
 * copy of the column indices (2 bytes per nonzero, library-owned, freed by
 * fab_op_destroy) that the products read instead of colind; see
 * fab_op_index_bytes.
 * Errors: FAB_E_INVALID (n <= 0, nnz < 0, nnz >= 2^31, null pointers, a
 * malformed CSR), FAB_E_UNSUPPORTED (n >= 2^31), FAB_E_HIP. */
fab_status fab_csr_create(fab_ctx* ctx, int64_t n, int64_t nnz, const int32_t* rowptr,
                          const int32_t* colind, const void* vals, int32_t dtype, fab_op** op);
fab_status fab_op_destroy(fab_op* op);

/* A^T as a new CSR operator whose arrays the library allocates and owns (freed
 * by fab_op_destroy).  Not in the paper: the adjoint of the method for the
 * differentiation extension (gradients of <c, f(A) b>).  Rows of A^T are sorted by column index, so the result
 * is canonical.  The adjoint of the method needs it: <c, f(A) b> = <f(A^T) c,
 * b>, so d<c, f(tA) b>/db = f(tA^T) c, computed by fab_solve on A^T.  A's
 * structure is checked on the device first (row pointers non-decreasing from 0
 * to nnz, column indices in [0, n)).  Errors: FAB_E_INVALID (null arguments or
 * a malformed CSR), FAB_E_HIP (allocation or launch failure). */
fab_status fab_op_transpose(fab_ctx* ctx, const fab_op* A, fab_op** AT);

/* *h_bytes = bytes per column index the products read: 2 when the operator
 * carries the 16-bit tile offsets described at fab_csr_create (also derived
 * for fab_op_transpose results), else 4.  Errors: FAB_E_INVALID (null
 * arguments). */
fab_status fab_op_index_bytes(const fab_op* A, int32_t* h_bytes);

/* Cache policy of the stores of a single solve's step: the product's z and the
 * window update's loads and new basis vector.  Not in the paper: a property of
 * the device's 256 MB memory-side cache.  policy 0 = by size (the setting at
 * creation): non-temporal when the CSR arrays the products read (values, the
 * column indices or 16-bit offsets, the row pointers) exceed 256 MB, so that
 * they stream through that cache on every product, else the default policy;
 * 1 = the default policy; 2 = non-temporal.  The policy changes timing only,
 * never results.  *h_streaming (optional) = 1 when the stores are non-temporal.
 * Batched and ragged solves keep their own kernels' policy.  Errors:
 * FAB_E_INVALID (A null, policy outside 0..2). */
fab_status fab_op_store_policy(fab_op* A, int32_t policy, int32_t* h_streaming);

/* Copy an operator's arrays (rowptr[n+1], colind[nnz], vals[nnz] in its dtype)
 * into caller-provided device buffers (test hook for fab_op_transpose). */
fab_status fab_op_copy_arrays(fab_ctx* ctx, const fab_op* A, int32_t* rowptr, int32_t* colind, void* vals);

/* Bytes of device workspace fab_solve needs for nt time points: the basis W
 * (n x (m+1), A's dtype) and its sketch S W (d x (m+1)) of Algorithm 1, R,
 * the whitening factor T of appendix eq. A.1, the quadrature restart's weights
 * (Section 4), per-block partial sums and the solver state.
 * Errors: FAB_E_INVALID (null arguments, nt or m out of range). */
fab_status fab_workspace_size(const fab_op* A, const fab_params* p, int32_t nt, size_t* h_bytes);

/* The restarted randomized Krylov method: Algorithm 2 (RandomizedRestartedKrylov
 * with A, S given by p->d, p->zeta, p->seed, b, m, tol, k_max = max_cycles),
 * each cycle Algorithm 1 truncated to a window of k, whitened by appendix
 * eq. A.1 and restarted through a quadrature rule (Section 4).
 * x[:, i] = f_i(A) b for the nt values h_t[i] (exp(-t_i z), phi_1(-t_i z),
 * cos(t_i sqrt z)), or nt = 1 for z^(-1/2).  b[n] has A's dtype; x is n x nt FP64, column-major (ldx = n),
 * overwritten.  work is device memory of at least fab_workspace_size bytes,
 * 256-byte aligned.  h_info is filled on every return >= FAB_E_HIP.
 * One right-hand side per call: the boundary's nrhs/ldb/ldx form is the
 * separate fab_solve_batched.  Errors: FAB_E_INVALID (null pointers, sizes,
 * parameter ranges, t <= 0 or non-finite, work not 256-byte aligned),
 * FAB_E_WORKSPACE, FAB_E_UNSUPPORTED, FAB_E_HIP; FAB_E_NONFINITE and
 * FAB_E_DIVERGED come from the iteration. */
fab_status fab_solve(fab_ctx* ctx, const fab_op* A, int32_t fun, const double* h_t, int32_t nt,
                     const void* b, double* x, const fab_params* p, void* work, size_t work_bytes,
                     fab_info* h_info);

/* Batched solves (Algorithm 2 for each right-hand side; the batching extension).
 * nb right-hand sides sharing A (columns of b, b[r * ldb + i], A's dtype).
 * x[(r * nt + i) * ldx + row] = f_i(A) b_r (FP64, overwritten).  Every member runs the
 * method of fab_solve with the same parameters and its own basis, sketch (the same S), restart
 * weights and stopping test; members that have finished are skipped by every kernel while the
 * others continue.  The fused product + sketch kernel reads each CSR chunk, and generates each
 * row of S, once for a group of G members (G chosen once per operator and batch shape by timing
 * G = 1, 4, 8 and 16 on the device; a group needs its LDS bins, G d FP64, within 96 KB).
 * The whole cycle of all members is one captured graph.  h_info has nb entries; the return value
 * is the most severe member status (errors before warnings before FAB_OK_BREAKDOWN before FAB_OK).
 * 1 <= nb <= 1024; ldb, ldx >= n; FAB_PLAIN_RESTART is not batched (FAB_E_UNSUPPORTED).
 * work: fab_workspace_size_batched bytes (nb copies of the single-solve workspace). */
fab_status fab_workspace_size_batched(const fab_op* A, const fab_params* p, int32_t nt, int32_t nb,
                                      size_t* h_bytes);
fab_status fab_solve_batched(fab_ctx* ctx, const fab_op* A, int32_t fun, const double* h_t, int32_t nt,
                             int32_t nb, const void* b, int64_t ldb, double* x, int64_t ldx,
                             const fab_params* p, void* work, size_t work_bytes, fab_info* h_info);

/* Ragged batches (Algorithm 2 for each operator; the batching extension).
 * nops operators of uneven size (any mix of n, nnz and dtype), one right-hand
 * side each: x[i] (n_i x nt FP64) = f(A_i) b[i].  b and x are host arrays of nops device
 * pointers.  Every operator runs the method of fab_solve in its own part of work
 * (fab_workspace_size_ragged bytes); the operators are spread over 16 branch streams, the cycles
 * of each branch's operators are captured into one graph per branch, and the branch graphs are
 * launched together once per cycle until every operator has finished.  A context keeps the
 * graphs of its first ragged call and replays them for later calls with the same operators,
 * outputs, workspace, function, time count and parameters;
 * a call that differs runs the same cycles uncaptured, one operator after another (same results,
 * no concurrency between operators).  h_info has nops entries; the return value is the most
 * severe status.
 * 1 <= nops <= 1024; FAB_PLAIN_RESTART is not supported (FAB_E_UNSUPPORTED). */
fab_status fab_workspace_size_ragged(int32_t nops, const fab_op* const* ops, const fab_params* p, int32_t nt,
                                     size_t* h_bytes);
fab_status fab_solve_ragged(fab_ctx* ctx, int32_t nops, const fab_op* const* ops, int32_t fun,
                            const double* h_t, int32_t nt, const void* const* b, double* const* x,
                            const fab_params* p, void* work, size_t work_bytes, fab_info* h_info);

/* ---- test hooks: the same kernels as fab_solve, exposed for parity tests ---- */

/* y = A x (A's dtype for x and y): the product z = A w_j of Algorithm 1, by the
 * kernel the solve uses.  work, work_bytes: unused (may be NULL, 0).
 * Errors: FAB_E_INVALID (null arguments), FAB_E_HIP. */
fab_status fab_spmv(fab_ctx* ctx, const fab_op* A, const void* x, void* y, void* work, size_t work_bytes);

/* The sketch of eq. (sparse_sign_sketch) applied to a vector, by the kernel the
 * solve uses: Sx[d] (FP64) = S x for the sparse sign matrix defined by (n, d, zeta, seed);
 * x has dtype.  work: at least 16384 d bytes (one partial sketch per block of the
 * product kernel's grid, at most 2048 blocks; summed in a fixed order). */
fab_status fab_sketch_apply(fab_ctx* ctx, int64_t n, int32_t d, int32_t zeta, uint64_t seed,
                            int32_t dtype, const void* x, double* Sx, void* work, size_t work_bytes);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): fab_sketch_apply without
 * a workspace argument.  Sx[d] (FP64) = S x, with the same kernels, grid and
 * bits as fab_sketch_apply; the per-block partial sketches live in a static
 * device array of the library (4 MiB per GPU, held until the process ends), so
 * the call allocates nothing.  x (n, dtype) and Sx are the caller's device
 * buffers.  Limit: d <= 256 (FAB_E_UNSUPPORTED above it).  Every call on one GPU
 * shares that GPU's array: calls that overlap on one GPU (several contexts or
 * host threads on the same device) race and must be serialised by the caller.
 * Errors: FAB_E_INVALID (null pointers, n, zeta or dtype out of range),
 * FAB_E_UNSUPPORTED (d > 256), FAB_E_HIP. */
fab_status fab_sketch_apply_noalloc(fab_ctx* ctx, int64_t n, int32_t d, int32_t zeta, uint64_t seed,
                                    int32_t dtype, const void* x, double* Sx);

/* The sketch specification itself (eq. sparse_sign_sketch: zeta distinct rows
 * per column, signs +-1, scale 1/sqrt(zeta) not included): for columns
 * col0 .. col0+count-1, the rows (int32, count x zeta, row-major) and signs
 * (int8, +1/-1) of S.  Errors: FAB_E_INVALID (ranges), FAB_E_HIP. */
fab_status fab_sketch_table(fab_ctx* ctx, int64_t col0, int64_t count, int32_t d, int32_t zeta,
                            uint64_t seed, int32_t* rows, int8_t* signs);

/* One cycle of Algorithm 1 (window-truncated) with the whitening of appendix
 * eq. A.1, from start vector v (A's dtype), exposing its intermediates:
 * W n x (m+1) (A's dtype, column-major), U = S W d x (m+1), R (m+1) x m, T (m+1) x (m+1)
 * (all FP64 column-major), Rt m x m = R_m + r_{m+1,m} (T_m^{-1} t) e_m^T, the projected matrix
 * in the basis W (the whitened X of the appendix's eq. A.1 is T_m Rt T_m^{-1}), and
 * h_scal[5] = {alpha, beta, h, m_eff, whitening}: whitening = 1 when T came from the Cholesky
 * factor of the Gram matrix kept by the steps, 0 when from the Householder QR of U. */
fab_status fab_cycle_debug(fab_ctx* ctx, const fab_op* A, const void* v, const fab_params* p,
                           void* W, double* U, double* R, double* T, double* Rt, double* h_scal,
                           void* work, size_t work_bytes);

/* Test hook for the divergence status: a solve is abandoned with FAB_E_DIVERGED when a cycle's
 * relative increment max_t ||y_t|| / ||x_t|| exceeds limit (default 1e8).  A small limit forces the
 * status on any problem (the first cycle's increment is x itself, relative increment 1).  The limit
 * applies to later calls on ctx.  Errors: FAB_E_INVALID (ctx NULL, limit not > 0). */
fab_status fab_divergence_limit(fab_ctx* ctx, double limit);

/* Members per block of the batched product + sketch kernel: 1, 4, 8 or 16 (a group that does not
 * fit the grouped kernel's LDS, or an operator whose vectors reach 2^31 bytes, n times the value
 * size, falls back to 1); 0 (the default) times every candidate on the
 * first batched solve of each operator and batch shape and keeps the fastest.  Test hook: pins a
 * path.  Errors: FAB_E_INVALID (ctx NULL or another G). */
fab_status fab_batch_group(fab_ctx* ctx, int32_t G);

/* Kernel timing for benchmarks.  While enabled, every fab_solve enqueues its cycles directly on
 * the context's stream (instead of replaying the cycle graph: the same kernels with the same
 * launch configuration).  on = 1: HIP events recorded by each launch of the fused SpMV + sketch
 * kernel (the product and sketch of Algorithm 1) and of each window update (Algorithm 1's basis
 * update: the fused Gram-Schmidt + update kernel, or the update kernel alone) at the kernel's own
 * start and end (extended launches that record them), and around each cycle's m-step loop,
 * accumulating their durations.  on = 2: events around each full cycle's
 * m-step loop only (no events between its kernels, which would add their own gaps); the kernel
 * totals stay 0.  on = 0: off (graph replay again).
 * fab_timing_read returns the totals since the last read and clears them.  Counts only steps
 * that ran (steps after a breakdown are excluded).  Errors: FAB_E_INVALID (on outside 0..2),
 * FAB_E_HIP. */
fab_status fab_timing_enable(fab_ctx* ctx, int32_t on);
fab_status fab_timing_read(fab_ctx* ctx, double* h_spmv_ms, int64_t* h_spmv_launches, double* h_loop_ms,
                           int64_t* h_loop_steps, double* h_update_ms, int64_t* h_update_launches);

/* Not in the paper (the differentiation extension):
 * out[0] = <x, y> for FP64 device vectors of length n, summed in a fixed order
 * (reproducible bits).  Used for the time derivative of <c, exp(-tA) b>, which
 * is -<c, A x> with x = exp(-tA) b.  out is device memory. */
fab_status fab_dot(fab_ctx* ctx, int64_t n, const double* x, const double* y, double* out);

const char* fab_status_string(fab_status s);

/* After FAB_E_HIP: the failing HIP call and its error name, for this host thread ("" if none).
 * The string is owned by the library and valid until the next failing call on the thread. */
const char* fab_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* FAB_H */
