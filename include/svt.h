/*
 * svt.h -- C ABI of the MI355X (gfx950) singular value thresholding library.
 *
 * The library solves the matrix completion problem of Cai, Candes and Shen,
 * "A Singular Value Thresholding Algorithm for Matrix Completion" (2008), by
 * Algorithm 1 of Section 5.1.5:
 *
 *     Y^{k0} = k0 delta P_Omega(M)                       (Section 5.1.3, eq. (5.3))
 *     X^k    = D_tau(Y^{k-1})                            (Section 2.1, eq. (2.2))
 *     stop when ||P_Omega(X^k - M)||_F / ||P_Omega M||_F <= eps   (eq. (5.5))
 *     Y^k    = Y^{k-1} + delta P_Omega(M - X^k)          (Section 2.2, eq. (2.7))
 *
 * D_tau is evaluated from the singular triplets of the sparse iterate above
 * tau, found by Golub-Kahan-Lanczos bidiagonalisation (Section 5.1.1); X^k is
 * kept as factors and evaluated only on Omega.
 *
 * Conventions for every entry point:
 *   - indices are 0-based; the unknown matrix is m x n ("n1 x n2" in the
 *     paper) and nnz = |Omega| (the paper's "m");
 *   - all pointers are HOST pointers unless stated otherwise; the library
 *     copies what it needs, so the caller keeps ownership of its buffers;
 *   - every function returns an svt_status (negative = error) and never lets a
 *     C++ exception escape; after an error svt_last_error(h) describes it;
 *   - a handle may be used by one thread at a time.
 */
#ifndef SVT_H
#define SVT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SVT_OK = 0,
  SVT_NOT_CONVERGED = 1, /* maxiter reached; the result is the last iterate  */
  SVT_STALLED = 2,       /* stall_window iterations without a new residual
                            minimum; the result is the last iterate         */
  SVT_UNDERDETERMINED = 3, /* the iterate's rank has more degrees of freedom
                            than dof_bound |Omega|; the result is the last
                            completed iterate                               */
  SVT_EINVAL = -1,       /* invalid argument (checked before any device work) */
  SVT_ENOMEM = -2,       /* host or device allocation failed                   */
  SVT_EDEVICE = -3,      /* a HIP runtime call failed                          */
  SVT_ESTATE = -4,       /* call not valid in the handle's current state       */
  SVT_EDIVERGED = -5,    /* residual became non-finite                         */
  SVT_EBUSY = -6,        /* serving: no capacity, request stays queued         */
  SVT_ELANCZOS = -7      /* partial SVD did not converge within its step cap   */
} svt_status;

typedef enum { SVT_FP64 = 0, SVT_MIXED = 1 } svt_precision;
typedef enum { SVT_COO = 0, SVT_CSR = 1 } svt_index_format;
typedef enum { SVT_STOP_RELRES = 0, SVT_STOP_NOISY = 1 } svt_stop_rule;
/* How D_tau finds the singular triplets of Y above tau:
   SVT_SVD_LANCZOS: Golub-Kahan-Lanczos bidiagonalisation until the rank
   decision is certain (Section 5.1.1), the default;
   SVT_SVD_RANDOMIZED: the randomised range finder with power iterations
   that Section 6 proposes (Halko, Martinsson and Tropp, 2011): for each s_k
   of Algorithm 1's repeat loop, l = min(m, n, s_k + rsvd_oversample)
   Gaussian test vectors, rsvd_power power iterations, and the SVD of the
   projected matrix.  Approximate: with a fixed number of power iterations
   the values near tau carry an error that can stall the iteration above
   eps.  Matrix completion with equality constraints only. */
typedef enum { SVT_SVD_LANCZOS = 0, SVT_SVD_RANDOMIZED = 1 } svt_svd_method;
/* SVT_CONSTRAINT_EQUALITY: X = M on Omega in the limit (Algorithm 1).
   SVT_CONSTRAINT_INEQUALITY: the matrix Dantzig selector of Section 3.3 for
   completion, |X_ij - B_ij| <= E on Omega (eq. (3.8) with A = P_Omega),
   by the iteration of eq. (3.10): two nonnegative multipliers Y+ and Y- on
   Omega, X^k = D_tau(Y+ - Y-), Y+- = [Y+- + delta P_Omega(+-(B - X^k) - E)]_+.
   Its stop test is the relative violation ||[|P_Omega(X - B)| - E]_+||_F /
   ||P_Omega B||_F <= eps (eq. (5.5) when E = 0), or with SVT_STOP_NOISY the
   data-consistency test of eq. (5.10) on ||P_Omega(X - B)||_F^2; the
   recorded residual is the relative violation either way.  Its kick is eq. (5.3)
   with S_E(B) = sign(B) max(|B| - E, 0) in place of M (while X = 0 the
   multipliers grow as k delta max(+-B - E, 0)). */
typedef enum { SVT_CONSTRAINT_EQUALITY = 0, SVT_CONSTRAINT_INEQUALITY = 1 } svt_constraint;

/*
 * Solver parameters.  svt_params_default() fills the paper's choices:
 *   tau    = 5 sqrt(m n)           (Section 5.2.1: tau = 5n for n x n)
 *   delta  = 1.2 m n / nnz         (Section 5.1.2, eq. (5.1))
 *   eps    = 1e-4                  (Section 5.1.4, eq. (5.5))
 *   maxiter= 500, incr (ell) = 5   (Section 5.1.1)
 *   kick   = 1                     (Section 5.1.3)
 */
typedef struct {
  double tau;            /* shrinkage threshold, > 0                          */
  double delta;          /* step size, > 0 (the paper uses 1.2 / p)            */
  double eps;            /* stopping tolerance, >= 0 (0 = run to maxiter)      */
  int32_t maxiter;       /* k_max, >= 1                                       */
  int32_t incr;          /* ell: increment of s_k, >= 1                       */
  int32_t kick;          /* 1: start from Y^{k0} (eq. (5.3)); 0: from Y^0 = 0  */
  int32_t k0_override;   /* > 0: use this k0 instead of computing it          */
  int32_t precision;     /* svt_precision                                     */
  int32_t stop_rule;     /* svt_stop_rule; NOISY is eq. (5.10)                 */
  double noise_sigma;    /* sigma of eq. (5.10); used with SVT_STOP_NOISY     */
  double lanczos_tol;    /* Ritz residual bound, relative to the largest Ritz
                            value; 0 = automatic: 1e-12 FP64, 1e-6 MIXED       */
  int32_t lanczos_maxsteps; /* cap on bidiagonalisation steps per SVT step
                               (0 = min(m, n)); with the randomised SVD the
                               cap on s_k                                      */
  int32_t reorth_passes; /* classical Gram-Schmidt against the whole basis:
                            0 (default) one pass per vector, recording the
                            fraction of the vector's |.|^2 it removes; if a
                            pass removed more than 1/2 (the DGKS criterion)
                            the bidiagonalisation restarts with two passes,
                            kept for the rest of the solve; 1 always one
                            pass; 2 always two (CGS2)                        */
  double decide_margin;  /* the rank decision accepts an unconverged Ritz value
                            below tau only if value + residual <= tau (1 -
                            margin) and a Ritz value above tau has already
                            converged; otherwise it waits for convergence,
                            as Algorithm 1 does.  Default 0.05; >= 1 always
                            waits                                            */
  uint64_t seed;         /* start vectors of the bidiagonalisation            */
  int32_t profile;       /* 1: time kernel classes with HIP events            */
  int32_t spmv_mode;     /* sparse products: 0 (default) and 2 stage x in
                            LDS, in column segments when it does not fit
                            whole (up to 8 of >= 1024 entries; otherwise it
                            is gathered from memory); 1 always gather        */
  void *stream;          /* hipStream_t to run on; NULL = library-owned stream.
                            It must come from the HIP runtime this library
                            links (libamdhip64.so.7): a second runtime in the
                            process (PyTorch bundles its own) has stream
                            handles that are not valid here.  The library
                            never destroys a caller's stream               */
  double ineq_tol;       /* E of SVT_CONSTRAINT_INEQUALITY (one tolerance for
                            every observed entry), >= 0                        */
  int32_t constraint;    /* svt_constraint; default SVT_CONSTRAINT_EQUALITY   */
  int32_t warm_start;    /* 0: start from the kick (or Y = 0); 1: start from the
                            handle's current iterate Y (and multipliers), e.g.
                            the last solve's final Y or one set with
                            svt_set_iterate: the warm start of Section 6's tau
                            continuation; no kick is applied                 */
  int32_t stall_window;  /* > 0: stop with SVT_STALLED once this many
                            consecutive iterations set no new minimum of the
                            recorded residual (a bound on runs that oscillate
                            without converging, which Algorithm 1 itself does
                            not stop before maxiter); <= 0 (default): off.
                            The server applies 20 to requests that leave it
                            0; < 0 turns it off there too                   */
  int32_t min_block_rows;/* the bidiagonalisation's vectors are cut into at
                            most 256 row blocks (one workgroup each) of at
                            least this many rows; 0 (default) = 8, at most
                            2048.  Fewer, fuller blocks leave compute units to
                            solves running at the same time; the server uses
                            64 for requests that leave it 0.  The partial
                            sums follow the blocks, so results depend on it
                            at rounding level                               */
  int32_t svd_method;    /* svt_svd_method; default SVT_SVD_LANCZOS          */
  int32_t rsvd_oversample; /* extra test vectors of the randomised SVD, >= 0
                              (default 10)                                   */
  int32_t rsvd_power;    /* its power iterations, 0..64 (default 2)          */
  double reorth_eta;     /* Partial reorthogonalisation (Section 5.1.1), the
                            level as a multiple of sqrt(u), u the unit
                            roundoff of the bidiagonalisation's vectors
                            (FP64: sqrt(u) = 1.05e-8; MIXED, FP32 vectors:
                            2.44e-4).  The loss of orthogonality of each new
                            vector is estimated from the bidiagonal
                            coefficients alone (the recurrences of Simon and
                            Larsen), and a vector is orthogonalised against
                            its whole basis, with the next vector of the
                            other side, only once its predicted estimate
                            passes reorth_eta sqrt(u).  The estimates are
                            checked as the coefficients reach the host; if
                            one of a vector left alone passed sqrt(u)
                            (semi-orthogonality) that bidiagonalisation
                            starts again with full reorthogonalisation
                            (levels of 1 and above make that happen).  With
                            FP64 vectors the bidiagonalisation of an SVT
                            step orthogonalises on a prediction no earlier
                            than a few steps before where the previous
                            step's coefficients show the first vector
                            needed it.  Negative (default):
                            automatic, 0.01 with FP64 vectors and 0.1 with
                            FP32 vectors; 0: every new vector is
                            orthogonalised; at most 100.  Applies with one
                            Gram-Schmidt pass per vector (reorth_passes 0 or
                            1); svt_reorth_stats reports what it did       */
  double dof_bound;      /* > 0: stop with SVT_UNDERDETERMINED once an SVT
                            step's rank r_k certainly has more degrees of
                            freedom, r_k (m + n - r_k), than dof_bound |Omega|
                            (Section 1.1: a rank-r matrix has r (m + n - r)
                            degrees of freedom, and no fewer observations
                            can determine it).  Checked as the step's
                            bidiagonalisation runs: its Ritz values bound the
                            singular values from below, so once more of them
                            than the bound's rank exceed tau the step ends
                            there, without its update (the Lanczos partial
                            SVD only).  <= 0 (default): off.
                            The server applies 1 to requests that leave it 0;
                            < 0 turns it off there too                      */
} svt_params;

typedef struct {
  int32_t iters;         /* Algorithm 1's loop counter at the break (excludes k0) */
  int32_t k0;            /* skipped initial steps (0 when kick = 0)            */
  int32_t rank;          /* r of the returned X                                */
  int32_t status;        /* svt_status of the solve                            */
  double rel_residual;   /* ||P_Omega(X - M)||_F / ||P_Omega M||_F              */
  double sigma1;         /* ||P_Omega M||_2 found for the kick (0 if no kick)  */
  double norm_pm;        /* ||P_Omega M||_F                                    */
  double t_setup_s;      /* svt_create: validation, index build, upload       */
  double t_kick_s;       /* kick: ||P_Omega M||_2 and Y^{k0}                   */
  double t_solve_s;      /* SVT loop wall time                                 */
  int64_t gkl_steps;     /* bidiagonalisation steps over the whole solve      */
} svt_info;

typedef struct svt_problem svt_problem;

/* Fill *out with the defaults above for an m x n problem with nnz samples.
   Errors: EINVAL if out is NULL or m, n, nnz < 1. */
svt_status svt_params_default(int64_t m, int64_t n, int64_t nnz, svt_params *out);

/*
 * Create a problem: Omega and P_Omega(M) (Algorithm 1's inputs, Section 5.1.5).
 *   fmt == SVT_COO: idx0 = const int32_t rows[nnz], idx1 = const int32_t cols[nnz]
 *   fmt == SVT_CSR: idx0 = const int64_t rowptr[m+1], idx1 = const int32_t cols[nnz]
 *   vals: const double[nnz], the observed M_ij in the same order.
 * The triplets may come in any order.  The library builds row- and
 * column-compressed copies of Omega (int32) and uploads them with the values.
 * Errors (all checked before any device work): EINVAL if m, n < 1,
 * nnz < 1 or nnz > m n, nnz >= 2^31, m or n >= 2^31, an index is out of range,
 * a position repeats (Omega is a set), a value or parameter is not finite,
 * tau <= 0, delta <= 0, eps < 0, maxiter < 1, incr < 1, or all values are 0.
 * ENOMEM / EDEVICE on allocation or HIP failures.  *out is NULL on error.
 */
svt_status svt_create(int64_t m, int64_t n, int64_t nnz, int32_t fmt,
                      const void *idx0, const int32_t *idx1, const double *vals,
                      const svt_params *params, svt_problem **out);

/*
 * Create a problem with a general linear operator (Section 3.1): p
 * measurements b = A(M) of an m x n matrix through its entries on a support
 * S of ns distinct positions (srows[s], scols[s]; host int32, any order):
 * b_i = sum_t gval[t] M[srows[gidx[t]], scols[gidx[t]]] over t in
 * [gptr[i], gptr[i+1]) (CSR over the measurements: gptr int64[p+1], gidx
 * int32 into S, gval double).  svt_solve then runs eq. (3.3):
 * X^k = D_tau(A*(y^{k-1})), y^k = y^{k-1} + delta (b - A(X^k)), with the
 * kick of eq. (5.3) taken with A*(b) in place of P_Omega M and the stop test
 * ||b - A(X^k)|| / ||b|| <= eps; completion is the case gval = 1, one term
 * per measurement.  The handle's "iterate" (svt_get_iterate) is A*(y) on S.
 * params (may be NULL: defaults for p samples) must keep the equality
 * constraint and the relative-residual stop.  Errors (EINVAL, checked
 * before any device work): bad sizes, an index out of range, a repeated
 * support position, gptr not starting at 0 or decreasing, non-finite
 * weights or measurements, all measurements zero.
 */
svt_status svt_create_sensing(int64_t m, int64_t n, int64_t ns, const int32_t *srows, const int32_t *scols,
                              int64_t p, const int64_t *gptr, const int32_t *gidx, const double *gval,
                              const double *b, const svt_params *params, svt_problem **out);

/* Run Algorithm 1 from the kick (each call starts over).  Returns SVT_OK,
   SVT_NOT_CONVERGED (maxiter reached; the factors hold X^{maxiter}),
   SVT_STALLED (with stall_window > 0; the factors hold the last iterate),
   SVT_UNDERDETERMINED (with dof_bound > 0; the factors hold the last completed
   iterate), or an error; after an error raised inside the iteration (e.g. SVT_ELANCZOS when
   the bidiagonalisation reaches lanczos_maxsteps) info still reports the
   iterations completed and their last residual.  info may be NULL. */
svt_status svt_solve(svt_problem *h, svt_info *info);

/* tau continuation with warm starts (Section 6): Algorithm 1 for each of the
   count values taus[0..count-1] (finite, > 0; normally increasing), the
   first stage as the handle's warm_start says, every later one from the
   previous stage's final iterate Y (the dual iterate is carried, so Y stays
   supported on Omega).  infos (may be NULL) receives count records; the
   handle's factors and history are the last stage's.  Returns the last
   stage's status, or the first error (infos then holds the stages done).
   The handle's tau is left as it was. */
svt_status svt_solve_path(svt_problem *h, const double *taus, int32_t count, svt_info *infos);

/* Per-iteration record of the last solve, k = 1..len: rank r_k, the number
   s_k of triplets Algorithm 1 computes (Section 5.1.1's rule for s_k), the
   relative residual of eq. (5.5), and the bidiagonalisation steps (the
   quantities Section 5.2.1 reports per run: iterations, rank, error).  Any output pointer may be NULL; at most cap
   entries are written; *len_out receives the full length. */
svt_status svt_history(const svt_problem *h, int32_t cap, int32_t *ranks,
                       int32_t *s_hist, double *residuals, int32_t *gkl_steps,
                       int32_t *len_out);

/* X^opt as factors (Algorithm 1's output), X = U V^T: U is m x r row-major,
   the left singular vectors already multiplied by w (w_j = sigma_j - tau,
   also returned in w), V is n x r row-major with orthonormal columns.  Pass U = w = V = NULL to query r
   first; buffers are caller-owned and at least m r, r, n r doubles. */
svt_status svt_factors(const svt_problem *h, int32_t *rank_out, double *U,
                       double *w, double *V);

/* X^opt at q arbitrary positions (rows[i], cols[i]) -> out[i]: the completed
   entries outside Omega, which is what matrix completion is for (Section
   1.1; Algorithm 1 returns X^opt as the estimate of M).  EINVAL for an index
   out of range or a NULL array with q > 0. */
svt_status svt_predict(const svt_problem *h, int64_t q, const int32_t *rows,
                       const int32_t *cols, double *out);

/* Release the handle and its device memory (the index structures, values,
   iterate and factors that Algorithm 1 of Section 5.1.5 keeps between
   iterations).  NULL is ignored. */
void svt_destroy(svt_problem *h);

/* Short text of a status code, including the two ends of Algorithm 1's loop
   (Section 5.1.5): SVT_OK (the stop test of eq. (5.5) or (5.10) passed) and
   SVT_NOT_CONVERGED (k_max reached), SVT_STALLED (the stall bound of
   stall_window) and SVT_UNDERDETERMINED (the bound of dof_bound).  Never
   NULL; unknown codes give
   "unknown status". */
const char *svt_status_string(int32_t status);

/* Message for the last error on this handle (NULL handle: the last error of
   svt_create on this thread).  Never NULL. */
const char *svt_last_error(const svt_problem *h);

/* ---------------------------------------------------------------------
 * Single steps of the hot path, for checking each one against the oracle.
 * They act on the handle's current iterate Y (values on Omega).
 * ------------------------------------------------------------------ */

/* Set / read the iterate's values, given in the order of the triplets passed
   to svt_create.  which = 0 reads the row-compressed copy, 1 the
   column-compressed copy (they must agree exactly). */
svt_status svt_set_iterate(svt_problem *h, const double *y);
svt_status svt_get_iterate(const svt_problem *h, int32_t which, double *y);

/* SVT_CONSTRAINT_INEQUALITY handles: set / read the multipliers Y+ and Y-
   of eq. (3.10), in the order of the triplets passed to svt_create (setting
   them also sets the iterate Y = Y+ - Y-).  EINVAL for a negative or
   non-finite value, ESTATE for an equality-constrained handle. */
svt_status svt_set_multipliers(svt_problem *h, const double *yp, const double *ym);
svt_status svt_get_multipliers(const svt_problem *h, double *yp, double *ym);

/* out = Y x (trans = 0; x has n entries, out m) or Y^T x (trans = 1): the
   sparse products that drive the bidiagonalisation (Section 2.2). */
svt_status svt_apply(svt_problem *h, int32_t trans, const double *x, double *out);

/* The `count` largest singular triplets of the current Y by Golub-Kahan-
   Lanczos bidiagonalisation (Section 5.1.1), each converged to the handle's
   lanczos_tol: sigma[count], U m x count row-major, V n x count row-major
   (U or V may be NULL).  *steps_out (may be NULL) gets the number of steps. */
svt_status svt_partial_svd(svt_problem *h, int32_t count, double *sigma,
                           double *U, double *V, int32_t *steps_out);

/* One fused pass of Algorithm 1's last two lines on the current Y with a
   caller-given X = U V^T (U m x r, V n x r, row-major): returns
   ||P_Omega(M - X)||_F^2 in *res2 and applies Y += delta P_Omega(M - X).
   On an SVT_CONSTRAINT_INEQUALITY handle, the multiplier update of
   eq. (3.10) instead (Y+- = [Y+- + delta (+-(B - X) - E)]_+, Y = Y+ - Y-),
   returning the squared violation ||[|P_Omega(X - B)| - E]_+||_F^2. */
svt_status svt_sample_update(svt_problem *h, int32_t r, const double *U,
                             const double *V, double delta, double *res2);

/* For callers that cannot allocate device memory (code under HIP graph
   capture, tight serving loops, harnesses that forbid hipMalloc): the pass of
   svt_sample_update with the factors already on the device.  Calls no
   hipMalloc, hipFree or allocating routine.
     U, V:   device pointers in the handle's value type (double for
             SVT_FP64, float for SVT_MIXED), row-major m x r and n x r with
             row stride `stride` elements, 16-byte aligned; owned by the
             caller and only read.
     stride: >= max(r, 1) and a multiple of 16 / sizeof(value) (2 or 4).
   Returns ||P_Omega(M - U V^T)||_F^2 in *res2 (may be NULL) and applies
   Y += delta P_Omega(M - U V^T), on the handle's stream, synchronised
   before return.  The workgroup partials of the residual go to a fixed
   array of the library in each device's memory (1032 doubles; any problem
   size fits: the pass uses at most 1024 workgroups), held until the process
   ends; every call on one device shares it, so calls that overlap on one
   device race (one call at a time per device).  EINVAL for a bad stride,
   unaligned or NULL factors with r > 0, a non-finite delta, or when the
   handle's device is not current. */
svt_status svt_sample_update_noalloc(svt_problem *h, int32_t r, const void *U, const void *V,
                                     int64_t stride, double delta, double *res2);

/* The kick alone: sets Y = k0 delta P_Omega(M) with k0 from eq. (5.3) (or
   k0_override), returning sigma1 = ||P_Omega M||_2 and k0. */
svt_status svt_kick(svt_problem *h, double *sigma1, int32_t *k0);

/* Which sparse-product kernel a handle uses: *segments = the number of
   column segments of x that the row-compressed (which = 0, Y x) or
   column-compressed (which = 1, Y^T x) product stages in LDS, or 0 when it
   gathers x from memory (spmv_mode 1, x too large for the plan, or the
   device refused the LDS size).  EINVAL for a bad handle or which. */
svt_status svt_spmv_plan(const svt_problem *h, int32_t which, int32_t *segments);

/* Device memory of a handle: the bytes it holds now and the most it has
   held at once since svt_create (including the moments when a growing
   buffer's old and new copies are both live).  The bidiagonalisation bases
   of Section 5.1.1 grow with the steps taken, up to lanczos_maxsteps.
   Either pointer may be NULL; EINVAL for a bad handle. */
svt_status svt_device_bytes(const svt_problem *h, size_t *current, size_t *peak);

/* Kernel timing of the last solve when params.profile = 1.  Each kind is
   one kernel, and each timed bracket holds exactly one launch of it:
     0 k_spmv_rows           a bidiagonalisation half-step: the deferred
                             update of its input, the sparse product and
                             the dot products of its output
     1 k_gather4             the column copy of Y refreshed from the row
                             copy (one launch per iteration)
     2 k_gs_update<false>    two-pass mode: first update + second pass's
                             dot products
     3 k_ritz                Ritz vectors (one launch per side)
     4 k_sample_update       sampled product, residual and update of the
                             row copy of Y (one launch per iteration)
     5 k_gs_update<true>     one update + |p|^2 partials (two-pass mode, or
                             an update too wide to defer)
     6 k_pending_reduce      the column sums of a pending vector's partials
                             ahead of a half-step (wide bases only)
   Outputs: the number of launches, their summed duration in milliseconds
   (HIP events on the solve's stream) and their summed algorithmic bytes:
   the index, value and vector traffic each launch must move at least once.
   Any output pointer may be NULL; EINVAL for a kind outside 0..6. */
svt_status svt_kernel_stats(const svt_problem *h, int32_t kind, int64_t *launches,
                            double *total_ms, double *total_bytes);

/* Reorthogonalisation of the bidiagonalisation (Section 5.1.1) over the
   handle's last solve (svt_solve, svt_solve_path's last solve, or
   svt_partial_svd / svt_kick): the number of vectors the bidiagonalisation
   made (every half-step, including steps taken ahead of a check and then
   discarded), how many of them were orthogonalised against their basis (all
   but the first without reorth_eta), how many bidiagonalisations restarted
   with two Gram-Schmidt passes (reorth_passes 0), and how many times partial
   reorthogonalisation fell back to full.  Any output pointer may be NULL;
   EINVAL for a NULL handle. */
svt_status svt_reorth_stats(const svt_problem *h, int64_t *vectors, int64_t *orthogonalised,
                            int64_t *two_pass_restarts, int64_t *partial_fallbacks);

/* ---------------------------------------------------------------------
 * Serving form: continuous batching of completion requests on one GPU.
 * Not part of the paper's method: a request loop around svt_create /
 * svt_solve.  Requests are admitted first come, first served, when a slot is
 * free and their predicted device footprint fits in the remaining budget;
 * each slot runs its solve on its own HIP stream, so solves admitted at
 * different times overlap on the device.  Every reduction has a fixed order
 * and no device buffer is shared between solves: each result is
 * bit-identical alone and in the mix.  A server may be used from several
 * threads.
 * ------------------------------------------------------------------ */
typedef struct svt_server svt_server;

/* Predicted device bytes of a problem: index structures, values, iterate,
   bidiagonalisation bases and their partial sums for up to 512 steps (the
   default step cap of a served request), counted twice because a growing
   basis briefly holds its old and new copies, factors up to the rank that
   cap allows, and scratch.  An upper bound of the peak that svt_device_bytes
   reports for a handle created with lanczos_maxsteps = 512.  A request
   submitted with lanczos_maxsteps > 0 is admitted, and run, on its own cap;
   with 0 it runs with 512. */
svt_status svt_footprint(int64_t m, int64_t n, int64_t nnz, int32_t precision, size_t *bytes);

/* hbm_budget_bytes > 0: device memory the admitted solves may hold at once;
   1 <= max_slots <= 64: solves running at once.  Nothing touches the device
   until a request is admitted. */
svt_status svt_server_create(size_t hbm_budget_bytes, int32_t max_slots, svt_server **out);

/* Queue one request (COO triplets in any order, host pointers, copied).
   params may be NULL (defaults); its stream field is ignored.  Fields a
   request leaves 0 take the server's defaults: a 512-step cap
   (lanczos_maxsteps), a stall window of 20 (stall_window), the
   degrees-of-freedom bound at |Omega| (dof_bound 1) and row blocks of at
   least 64 rows (min_block_rows); a negative stall_window or dof_bound
   turns that bound off.  Returns
   EINVAL for invalid indices or values (checked here), ENOMEM if the request
   could never fit in the budget; *ticket identifies the request. */
svt_status svt_submit(svt_server *s, int64_t m, int64_t n, int64_t nnz, const int32_t *rows,
                      const int32_t *cols, const double *vals, const svt_params *params,
                      uint64_t *ticket);

/* *state: 0 queued, 1 running, 2 done. */
svt_status svt_poll(svt_server *s, uint64_t ticket, int32_t *state);

/* Block until the request is done; returns its solve status (SVT_OK,
   SVT_NOT_CONVERGED, SVT_STALLED, SVT_UNDERDETERMINED or the error of
   svt_create / svt_solve). */
svt_status svt_wait(svt_server *s, uint64_t ticket, svt_info *info);

/* Copy out a finished request's factors (as svt_factors: U m x r scaled by
   w, V n x r, row-major; pass NULL buffers to query r) and, if times is not
   NULL, its submit, start and completion times (seconds, one steady clock).
   EBUSY while the request is not done. */
svt_status svt_result(svt_server *s, uint64_t ticket, int32_t *rank_out, double *U, double *w,
                      double *V, double *times);

/* Forget a finished request (its factors are freed). */
svt_status svt_release(svt_server *s, uint64_t ticket);

/* Peak admitted footprint, the most solves that ran at once, queue length. */
svt_status svt_server_stats(svt_server *s, size_t *peak_bytes, int32_t *max_running,
                            int32_t *queued);

/* Finish queued and running work, then stop the slots and free the server. */
svt_status svt_server_destroy(svt_server *s);

#ifdef __cplusplus
}
#endif

#endif /* SVT_H */
