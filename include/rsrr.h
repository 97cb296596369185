/*
 * rsrr.h -- C ABI of the MI355X (gfx950) resolvent-sampling Rayleigh-Ritz
 * library for nonlinear eigenvalue problems T(lambda) v = 0.
 *
 * Method: J. Xiao, S. Meng, C. Zhang, C. Zheng, "Resolvent sampling based
 * Rayleigh-Ritz method for large-scale nonlinear eigenvalue problems"
 * (arXiv 1510.07522).  Algorithm 2 (RSRR) around Algorithm 1 (modified block
 * Sakurai-Sugiura for the projected problem).
 *
 * Conventions
 *  - Complex numbers are interleaved (re, im) doubles (rsrr_complex), the same
 *    bytes as C99 double complex, std::complex<double> and torch.complex128.
 *  - Matrices are column-major.  "host" pointers are ordinary CPU memory,
 *    "device" pointers are HIP device memory of the current device.
 *  - Every call returns an int status: 0 = success, < 0 = error (nothing of
 *    the output is valid; rsrr_last_error() has a message), > 0 = success
 *    with warnings (a bitwise OR of RSRR_WARN_*).
 *  - The library owns every buffer it allocates; callers own the buffers they
 *    pass.  Calls on one problem handle must not overlap (not thread-safe per
 *    handle); distinct handles may be used from distinct threads.
 *  - Work is issued on the HIP stream given at creation (NULL = the default
 *    stream).  Calls return after their results are complete.
 */
#ifndef RSRR_H
#define RSRR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct { double re, im; } rsrr_complex;

enum {
  RSRR_OK = 0,
  RSRR_EINVAL = -1,      /* invalid argument */
  RSRR_ENOMEM = -2,      /* device or host allocation failed */
  RSRR_EHIP = -3,        /* a HIP runtime call or kernel launch failed */
  RSRR_ESINGULAR = -4,   /* T(z_j) exactly singular at a sampling node */
  RSRR_EBUSY = -5,       /* request does not fit the memory budget */
  RSRR_ENOTCONV = -6,    /* an inner iteration (eigen / SVD, or the sampling's refinement
                            above order 8192) did not converge */
  RSRR_ETIMEDOUT = -7,   /* a bounded wait ended before the request finished */
  RSRR_WARN_RANK_SATURATED = 1,  /* k_S == N*L < n: the sample space may be too small (eq. eq-rank-nc) */
  RSRR_WARN_COUNT_MISMATCH = 2,  /* final count differs from the winding count (eq. eq-ncs) */
  RSRR_WARN_IR_FALLBACK = 4,     /* some nodes needed the complex128 factorisation */
  RSRR_WARN_HANKEL_FULL = 8,     /* every Hankel singular value was retained (m == K k_S): the rank
                                    condition of Alg. 1 (eq. eq-ranks) may fail; raise K or L */
  RSRR_WARN_NO_WINDING = 16      /* scalar-function callback without derivatives: no winding count */
};

/* Kinds of coefficient matrices A_k in T(z) = sum_k f_k(z) A_k (eq. eq-Z-expr). */
enum {
  RSRR_MAT_IDENTITY = 0,  /* A_k = I; data pointer ignored (may be NULL) */
  RSRR_MAT_DIAG = 1,      /* A_k = diag(d); data = n rsrr_complex */
  RSRR_MAT_REAL = 2,      /* dense real; data = n*n double, column-major */
  RSRR_MAT_DENSE = 3      /* dense complex; data = n*n rsrr_complex, column-major */
};

/* Scalar functions f_k (evaluated by the library on the host, with their
 * derivatives, at the sampling nodes, the reduced-problem nodes and the
 * eigenvalues):
 *   RSRR_F_POW : f(z) = c z^p
 *   RSRR_F_EXP : f(z) = c z^p exp(t z)
 *   RSRR_F_RAT : f(z) = c z^p / (z - t)                                       */
enum { RSRR_F_POW = 0, RSRR_F_EXP = 1, RSRR_F_RAT = 2 };
typedef struct {
  int kind;          /* RSRR_F_* */
  int p;             /* power of z, p >= 0 */
  rsrr_complex c;    /* scale */
  rsrr_complex t;    /* exponent rate (EXP) or pole (RAT); unused for POW */
} rsrr_fn;

/* Scalar functions given by the caller instead of the menu above (the
 * coefficient form allows any f_k, eq. eq-Z-expr).  The library calls
 *   f(ctx, z, m, f_out, df_out)
 * with m host nodes z[0..m-1] and expects f_k(z_q) in f_out[q*J + k] for every
 * k < J, and, when df_out is not NULL, the derivatives f_k'(z_q) in
 * df_out[q*J + k].  Calls come at the sampling nodes, the reduced-problem
 * nodes (with derivatives, for the winding count of eq. eq-ncs) and the
 * extracted eigenvalues, from the thread that runs the solve (a serving slot's
 * worker thread for rsrr_server_submit).  Return 0 on success; return 1 when
 * derivatives were asked for but are not available: the library then asks
 * again with df_out = NULL, skips the winding count (n_wind = -1) and sets
 * RSRR_WARN_NO_WINDING; any other value fails the call with RSRR_EINVAL. */
typedef int (*rsrr_scalar_fn)(void* ctx, const rsrr_complex* z, size_t m, rsrr_complex* f_out,
                              rsrr_complex* df_out);

/* Closed contour C of Alg. 2 Step 1 and Alg. 1 Step 1; interior = strictly
 * inside.  The same contour gives the sampling nodes (N of them) and the
 * moment quadrature of the reduced problem (NS nodes).
 *
 * RSRR_CONTOUR_ELLIPSE (kind 0, the zero-initialised default):
 *   phi(theta) = center + a cos(theta) + i b sin(theta) (eq. eq-contour), a the
 *   semi-axis along the real direction, b along the imaginary one (a = b = r
 *   for a circle); trapezoid angles theta_j = 2 pi (j + 1/2)/N.
 * RSRR_CONTOUR_RECT (kind 1): the rectangle center + [-a, a] x i[-b, b] (a, b
 *   the half-sides), with Gauss-Legendre nodes on each of its four sides
 *   (the paper's rectangular contours, numerical examples of Sec. 7),
 *   counter-clockwise from the lower-left corner: bottom, right, top, left.
 *   n_h nodes on each horizontal side and n_v on each vertical side for the
 *   sampling nodes, so N = 2 (n_h + n_v) (the paper's "10-5" split is n_h = 10,
 *   n_v = 5 for a wide rectangle).  n_h = n_v = 0 splits N (even, >= 4) in
 *   proportion to the side lengths: n_h = round(N/2 * a/(a+b)) clamped to
 *   [1, N/2 - 1]; the NS moment nodes are always split that way (NS even).
 * Moments and the winding count use rho = max(a, b) and the quadrature
 * weights dz_j / (2 pi i) of the contour integral (for the ellipse this is
 * eq. eq-Ap-num). */
enum { RSRR_CONTOUR_ELLIPSE = 0, RSRR_CONTOUR_RECT = 1 };
typedef struct {
  rsrr_complex center;
  double a, b;
  int kind;           /* RSRR_CONTOUR_* */
  int n_h, n_v;       /* RECT only: sampling nodes per horizontal / vertical side, or 0, 0 */
} rsrr_contour;

enum { RSRR_PREC_C128 = 0, RSRR_PREC_C64_IR = 1 };

/* How a matrix without a coefficient form (BEM) is interpolated in z for the
 * reduced problem (Sec. 6.2): RSRR_INTERP_CHEB, the Chebyshev interpolant on
 * [Re(center) - a, Re(center) + a] (eq. eq-T-interp, eq. eq-Ts-coefs), fit for
 * contours that hug that interval; RSRR_INTERP_CIRCLE, the interpolant through
 * d+1 equispaced points of the circle of radius R around the center (R =
 * max(a, b) for an ellipse, sqrt(a^2 + b^2) for a rectangle), in the basis
 * ((z - center)/R)^j, whose coefficients are the discrete Fourier transform
 * of the samples; RSRR_INTERP_AUTO (default) takes the Chebyshev interpolant
 * when b <= a/4 and the circle otherwise (a Chebyshev series evaluated at a
 * distance of order a off its interval amplifies the rounding of its high
 * coefficients like (1 + sqrt 2)^j). */
enum { RSRR_INTERP_AUTO = 0, RSRR_INTERP_CHEB = 1, RSRR_INTERP_CIRCLE = 2 };

/* How Alg. 2 Step 3 builds its subspace: from the sampling matrix S_hat
 * (eq. eq-hatS, the resolvent sampling scheme; default) or from the moment
 * matrix M_hat = S_hat D Z (eq. eq-hatMS, the moment scheme of SSRR,
 * Sec. 3.1; see rsrr_moment_matrix). */
enum { RSRR_SCHEME_SAMPLING = 0, RSRR_SCHEME_MOMENT = 1 };

typedef struct {
  int N;              /* sampling nodes on the contour (see rsrr_contour) */
  int L;              /* probing vectors (columns of U) */
  int NS;             /* quadrature nodes of the reduced problem (eq. eq-Ap-num), default 512 */
  int K;              /* Hankel blocks (eq. eq-HH), default 2 */
  double delta;       /* basis truncation: keep singular directions above delta*sigma_1, default 1e-14 */
  double tol_gap;     /* singular-value gap threshold (eq. eq-gap), default 1e3 */
  double tol_res;     /* returned pairs have ||T v||/(||T||_F ||v||) <= tol_res, default 1e-10;
                         the reduced eigenpairs get a first-order correction when a spectral
                         split of the reduced matrix drops a coupling above tol_res / 10 */
  double hankel_tol;  /* Hankel truncation sigma_j > hankel_tol*sigma_1, default 1e-13 */
  int precision;      /* RSRR_PREC_C128 or RSRR_PREC_C64_IR (default) */
  int ir_max_iter;    /* refinement sweeps before the complex128 fallback, default 5 */
  double ir_tol;      /* refinement acceptance: normwise backward error, default 1e-14 */
  int cheb_degree;    /* BEM only: interpolation degree d (eq. eq-T-interp), default 40 */
  int nb;             /* LU panel width of the sampling factorisations (1..64), default 64;
                         0: the autotuned width (rsrr_tune_lu) */
  uint64_t seed;      /* seed of the probing matrix when U is not supplied */
  int scheme;         /* RSRR_SCHEME_SAMPLING (default) or RSRR_SCHEME_MOMENT */
  int Kp;             /* moment scheme: number of moments K' (0 = N, as in the paper's comparisons) */
  double chunk_gib;   /* device memory for one batch of T_S(zeta_m) and their inverses in the
                         reduced moments (and of BEM Chebyshev samples), GiB; default 24 */
  int interp;         /* BEM only: RSRR_INTERP_*, default RSRR_INTERP_AUTO */
  int graph;          /* 1: the sampling launches (assembly and factorisation of all nodes)
                         are captured in a HIP graph kept by the handle and replayed by later
                         solves whose sizes, buffers and coefficients are the same (captured
                         again otherwise; not while kernel timers are on); default 0 */
  int nb_reduced;     /* LU panel width of the reduced-problem factorisations (1..64);
                         0 (default): 64 */
} rsrr_params;

/* Diagnostics of one solve. */
typedef struct {
  int n, N, L;
  int k_S;            /* dimension of the Rayleigh-Ritz basis (Alg. 2 Step 3) */
  int m;              /* retained Hankel singular values */
  int n_wind;         /* eigenvalue count by the winding number (eq. eq-ncs), rounded; -1 if not
                         computed (callback without derivatives) */
  int n_gap;          /* count by the singular-value gap (eq. eq-gap); -1 if no gap >= tol_gap */
  int n_eig;          /* returned eigenpairs (inside, residual <= tol_res) */
  int n_candidates;   /* extracted eigenvalues inside the contour before the residual test */
  int ir_iters;       /* refinement sweeps used (max over nodes) */
  int ir_fallback;    /* nodes solved again in complex128 */
  int status;         /* the status the solve returned */
  double wind_re, wind_im;   /* unrounded winding integral */
  double t_sample, t_basis, t_project, t_reduced, t_residual;  /* seconds per stage */
  double ws_bytes;    /* device workspace held by the handle (or server slot) after the call */
} rsrr_info;

typedef struct rsrr_problem rsrr_problem;
typedef struct rsrr_result rsrr_result;

/* Fills p with the defaults listed above (N = 32, L = 16). */
void rsrr_default_params(rsrr_params* p);

/* Coefficient-form problem T(z) = sum_{k<J} f_k(z) A_k (eq. eq-Z-expr).
 * kinds[k] is RSRR_MAT_*, A[k] a host pointer to its data (copied to the
 * device; the caller may free it on return), f[k] its scalar function.
 * 1 <= n <= 16384, 1 <= J <= 16.  stream: hipStream_t or NULL.  Orders above
 * 8192 need precision RSRR_PREC_C64_IR (complex128 factorisations, those of the
 * precision RSRR_PREC_C128 and of the refinement's fallback, go up to 8192):
 * rsrr_solve then fails with RSRR_EINVAL for RSRR_PREC_C128, and with
 * RSRR_ENOTCONV when the refinement leaves a node above ir_tol. */
int rsrr_create(rsrr_problem** out, int n, int J, const int* kinds,
                const void* const* A, const rsrr_fn* f, void* stream);

/* The same coefficient form with the scalar functions supplied by a host
 * callback (see rsrr_scalar_fn); f_ctx is passed back unchanged and must stay
 * valid for the problem's lifetime.  Arguments and errors as rsrr_create. */
int rsrr_create_fn(rsrr_problem** out, int n, int J, const int* kinds, const void* const* A,
                   rsrr_scalar_fn f, void* f_ctx, void* stream);

/* Helmholtz single-layer matrix on a point set (cf. eq. eq-nyes):
 * T_ij(z) = exp(i z r_ij)/(4 pi r_ij) for i != j, T_ii(z) = i z/(4 pi) + 1/(2h).
 * xyz: host, n*3 doubles (x, y, z per point).  Entries are generated on the fly
 * at every node; the reduced problem uses the Chebyshev interpolation of
 * eq. eq-Ts-coefs on [Re(center) - a, Re(center) + a].  2 <= n <= 16384, with the
 * limits of rsrr_create above order 8192. */
int rsrr_create_bem(rsrr_problem** out, int n, const double* xyz, double h, void* stream);

void rsrr_destroy(rsrr_problem* p);

/* Alg. 2 Steps 1-2: the sampling matrix S_hat = [T(z_0)^{-1} U ... T(z_{N-1})^{-1} U]
 * (eq. eq-hatS).  U: device, n x L complex, leading dimension ldu >= n.
 * S: device, n x (N*L) complex, leading dimension lds >= n, block j = columns
 * [j*L, (j+1)*L).  With precision RSRR_PREC_C64_IR the factorisations are
 * complex64 and fp64 iterative refinement runs until a block's normwise
 * backward error reaches the fp64 floor (4 u) or a sweep no longer halves it,
 * at most ir_max_iter sweeps; a block left above ir_tol is redone in
 * complex128.
 * info (may be NULL) receives ir_iters / ir_fallback / t_sample. */
int rsrr_sample(rsrr_problem* p, const rsrr_contour* c, const rsrr_params* prm,
                const rsrr_complex* U, int ldu, rsrr_complex* S, int lds, rsrr_info* info);

/* Moment scheme (SSRR, Sec. 3.1-3.2): from the sampling matrix S_hat of
 * rsrr_sample (device, n x N*L, leading dim lds, block i = T(z_i)^{-1} U), the
 * moment matrix M_hat = [M_0 ... M_{K'-1}] (eq. eq-hatM; device, n x K'*L,
 * leading dim ldm, block alpha = M_alpha) with
 *   M_alpha = sum_i w_i s_i^alpha T(z_i)^{-1} U   (eq. eq-malpha-qud),
 * w_i = dz_i / (2 pi i) the contour's quadrature weights at the sampling
 * nodes, s_i = (z_i - center) / max(a, b) and K' = prm->Kp (0 = N); this is
 * M_hat = S_hat D Z of eq. eq-hatMS.  S is not modified; M must not overlap
 * it.  Runs on the problem's stream and returns after it completes.
 * Errors: RSRR_EINVAL for bad arguments (lds, ldm < n, null buffers). */
int rsrr_moment_matrix(rsrr_problem* p, const rsrr_contour* c, const rsrr_params* prm,
                       const rsrr_complex* S, int lds, rsrr_complex* M, int ldm);

/* Alg. 2 Step 3: orthonormal basis Q of the columns of S_hat (device, rows x
 * cols, leading dim lds; not modified) spanning its singular directions above
 * delta * sigma_1.  Q: device, rows x min(rows, cols), leading dim ldq; the
 * first *k_S columns are the basis (Q^H Q = I to rounding). */
int rsrr_orthonormalize(int rows, int cols, const rsrr_complex* S, int lds, double delta,
                        rsrr_complex* Q, int ldq, int* k_S, void* stream);

/* Alg. 2 Step 4, projection (eq. eq-Zs-expr): B_k = Q^H A_k Q for every
 * coefficient, written to B (device) as J blocks of k_S x k_S (leading dim
 * k_S, block stride k_S*k_S).  For a BEM problem the J = d+1 blocks are the
 * coefficients P_hat_j of the interpolant prm->interp selects: Chebyshev on
 * [Re(center) - a, Re(center) + a] (eq. eq-Ts-coefs) or the circle basis
 * ((z - center)/R)^j; *J_out = d+1.  Q: device, n x k_S, leading dim ldq. */
int rsrr_project(rsrr_problem* p, const rsrr_contour* c, const rsrr_params* prm,
                 const rsrr_complex* Q, int ldq, int k_S, rsrr_complex* B, int* J_out);

/* Alg. 2 end to end: eigenvalues strictly inside the contour with residual
 * ||T(l) v||_2 / (||T(l)||_F ||v||_2) <= tol_res, their eigenvectors (unit
 * 2-norm, largest-modulus entry real positive) and residuals.  U: device n x L
 * (leading dim n) or NULL to draw a complex Gaussian U from prm->seed. */
int rsrr_solve(rsrr_problem* p, const rsrr_contour* c, const rsrr_params* prm,
               const rsrr_complex* U, rsrr_result** out);

/* Alg. 2 for `count` problems at once, of uneven orders (many independent
 * eigenproblems, Sec. 1 and 5): the sampled matrices T(z_j) of every problem
 * are factored together -- each panel step of all (problem, node) matrices
 * is one set of launches (panels, row interchanges, and the trailing updates
 * as one persistent matrix-core launch walking the tiles of all problems) --
 * then each problem's solves, refinement, basis, projection and reduced
 * problem run in turn.  The problems must be distinct, use one stream and
 * share the precision and panel width.  Results are bit-identical to
 * rsrr_solve of each problem alone with the same panel width (nb = 0 takes
 * the width tuned for the batch's largest order and total node count, which
 * a solve alone may not).  contours, prms: count entries each;
 * U: NULL, or count device pointers (n_i x L_i, leading dim n_i; an entry may
 * be NULL to draw U from prms[i].seed); out: count result pointers (free each
 * with rsrr_result_free).  Returns the bitwise OR of the problems' warnings,
 * or the first error (then no result is returned). */
int rsrr_solve_batched(int count, rsrr_problem* const* probs, const rsrr_contour* contours,
                       const rsrr_params* prms, const rsrr_complex* const* U, rsrr_result** out);

/* Upper bound of the device workspace one rsrr_solve of p with prm allocates
 * (bytes), from n, J, N, L, NS, K, nb, the precision and the scheme: the
 * admission figure of the serving loop below.  The handle's coefficients are
 * not included. */
int rsrr_workspace_bound(const rsrr_problem* p, const rsrr_contour* c, const rsrr_params* prm,
                         size_t* bytes);

/* Serving: continuous batching of rsrr_solve requests on the current device
 * (the request loop the method needs when many eigenproblems arrive over time;
 * the sampling nodes of different requests are independent, Sec. 1 and 5).
 * A server has max_slots (1..16) slots; each is one host worker thread with its
 * own non-blocking, default-priority HIP stream and device workspace, so up to
 * max_slots solves run on the device at once.  Requests are admitted in
 * submission order as soon as a slot is free and
 *   (workspace held by the other slots) + rsrr_workspace_bound(request)
 * fits hbm_budget_bytes; idle slots give their workspace back when the head of
 * the queue waits for memory.  Results are bit-identical to a solve of the same
 * request alone (every kernel is deterministic).
 *   submit: validates like rsrr_solve, copies c, prm and U_host (host, n x L
 *           column-major, or NULL to draw U from prm->seed) and returns a ticket
 *           at once; RSRR_EBUSY if the request's bound alone exceeds the budget.
 *           p must stay alive until the request has been waited for.
 *   wait:   blocks until the request has finished, or at most timeout_s
 *           seconds when timeout_s > 0 (then RSRR_ETIMEDOUT, with the slot and
 *           queue state in rsrr_last_error(); the ticket stays valid); *out
 *           receives its result (free with rsrr_result_free; NULL on error)
 *           and *latency_s (may be NULL) the time from submission to
 *           completion; returns the solve's status.  Each ticket can be
 *           waited for once.
 * Slots run without the look-ahead stream of the LU factorisations (one
 * stream per slot, no cross-stream waits).  When requests are pending and
 * nothing has been admitted or finished for RSRR_SERVER_WATCHDOG_S seconds
 * (environment, default 120, 0 = off), the slot and queue state is printed to
 * stderr.
 *   pending: requests queued and running.
 *   destroy: finishes every submitted request, frees results nobody waited
 *           for, and releases the slots. */
typedef struct rsrr_server rsrr_server;
int rsrr_server_create(rsrr_server** out, size_t hbm_budget_bytes, int max_slots);
int rsrr_server_submit(rsrr_server* srv, rsrr_problem* p, const rsrr_contour* c, const rsrr_params* prm,
                       const rsrr_complex* U_host, uint64_t* ticket);
int rsrr_server_wait(rsrr_server* srv, uint64_t ticket, double timeout_s, rsrr_result** out,
                     double* latency_s);
int rsrr_server_pending(rsrr_server* srv, int* queued, int* running);
void rsrr_server_destroy(rsrr_server* srv);

int rsrr_result_info(const rsrr_result* r, rsrr_info* info);
/* Host copies; any pointer may be NULL.  lambda: n_eig; V: n x n_eig
 * (leading dim n); resid: n_eig; resid_paper: ||T v||/||v|| (n_eig);
 * hankel_sigma: K*k_S singular values of H (descending). */
int rsrr_result_copy(const rsrr_result* r, rsrr_complex* lambda, rsrr_complex* V, double* resid,
                     double* resid_paper, double* hankel_sigma);
void rsrr_result_free(rsrr_result* r);

/* ------------------------------------------------------------------------
 * Dense building blocks of the sampling step, exposed for direct use.
 * All pointers are device pointers; matrices are column-major; batch b uses
 * A + b*sA, B + b*sB, C + b*sC (strides in elements).  Work is issued on
 * `stream` and the call returns when it is complete.
 * ---------------------------------------------------------------------- */
enum { RSRR_OP_N = 0, RSRR_OP_T = 1, RSRR_OP_C = 2 };

/* C = alpha op(A) op(B) + beta C in complex128 on the fp64 matrix cores
 * (the complex product as four real products).  op(A) is M x K, op(B) K x N. */
int rsrr_zgemm_batched(int opA, int opB, int M, int N, int K, rsrr_complex alpha,
                       const rsrr_complex* A, int lda, long long sA,
                       const rsrr_complex* B, int ldb, long long sB, rsrr_complex beta,
                       rsrr_complex* C, int ldc, long long sC, int batch, void* stream);

/* The same in complex64 (A, B, C hold interleaved float pairs; alpha/beta are
 * rounded to fp32).  gauss3m != 0 forms each complex product with three real
 * matrix-core products (Cr = P1 - P2, Ci = P3 - P1 - P2) instead of four. */
int rsrr_cgemm_batched(int opA, int opB, int M, int N, int K, rsrr_complex alpha,
                       const void* A, int lda, long long sA, const void* B, int ldb,
                       long long sB, rsrr_complex beta, void* C, int ldc, long long sC,
                       int batch, int gauss3m, void* stream);

/* Solves A_b X_b = B_b for `batch` n x n systems with the blocked LU with
 * partial pivoting of the sampling step (panel width nb in [1, 64]); A is
 * overwritten by its factors (interchanges of later panels are not applied to
 * the L columns of earlier ones), B by the solution.  complex128 when
 * precision = RSRR_PREC_C128, complex64 (interleaved floats) when
 * RSRR_PREC_C64_IR.  info_host (may be NULL): batch ints, 0 or the 1-based
 * index of the first exactly-zero pivot.  Returns RSRR_ESINGULAR if any.
 * Orders: n <= 8192 (complex128), n <= 16384 (complex64). */
int rsrr_gesv_batched(int precision, int n, int nrhs, void* A, int lda, long long sA, void* B,
                      int ldb, long long sB, int batch, int nb, int* info_host, void* stream);

/* rsrr_gesv_batched for callers that cannot allocate device memory (code
 * under stream capture, tight serving loops, hosts that forbid allocation
 * calls): the same factorisation and solve kernels, with the pivots, the
 * diagonal-block inverses and the per-matrix status in a fixed 64 MiB device
 * array of the library (one per GPU, held until the process ends) instead of
 * allocations: the call makes no device allocation (no hipMalloc, hipFree or
 * allocating library call).  Work space needed:
 * batch * (n * 4 + panels * 2 * nb^2 * element bytes) plus alignment, with
 * panels = ceil(n / nb) and 16 (complex128) or 8 (complex64) bytes per
 * element; a call that needs more than 64 MiB fails with RSRR_EINVAL and
 * touches nothing.  All calls on one GPU share the array: calls that overlap
 * in time on one GPU (other threads or streams) race and must be serialised
 * by the caller.  Arguments, results and errors as rsrr_gesv_batched, except
 * that with info_host NULL the call only enqueues its kernels on `stream`
 * and returns without copying or waiting (so it can be recorded under stream
 * capture): zero pivots are then not reported, and the results are complete
 * when the stream reaches that point. */
int rsrr_gesv_batched_noalloc(int precision, int n, int nrhs, void* A, int lda, long long sA, void* B,
                              int ldb, long long sB, int batch, int nb, int* info_host, void* stream);

/* Autotuning of the LU panel width (the sampling factorisations with blocks
 * of panels and look-ahead): rsrr_tune_lu times one factorisation of `batch`
 * synthetic matrices of order n for each candidate width (16, 32, 64) on the
 * current device, keeps the fastest in a process-wide table (precision, n,
 * batch) and returns it in *nb_best (*ms_best, may be NULL: its time).  A
 * solve with rsrr_params.nb = 0 takes the width of the table entry of its
 * precision with the nearest order (then the nearest node count), or 64 if
 * there is none.  rsrr_tune_save writes the table as JSON; rsrr_tune_load
 * reads such a file into the table and returns the number of entries read.
 * Orders as rsrr_gesv_batched. */
int rsrr_tune_lu(int precision, int n, int batch, int* nb_best, double* ms_best);
int rsrr_tune_save(const char* path);
int rsrr_tune_load(const char* path);

/* ------------------------------------------------------------------------
 * Kernel timers: when enabled, the main kernel classes (LU panel, LU trailing
 * update, solves, Gram/Cholesky, Jacobi rounds, QR sweeps, ...) are bracketed
 * by HIP events on the stream they are launched on.  Reading synchronises
 * those events.  Each class accumulates launches, total milliseconds and the
 * algorithmic flops and bytes of its launches (real flops, one complex
 * multiply-add = 8).  Launches of the main kernel functions are also
 * accumulated per function, under "sym:<name as a profiler lists it>" (for
 * example "sym:gemm_kernel<double, 0, 0, false, true>").  Process-wide; not
 * for concurrent use with solves.
 * ---------------------------------------------------------------------- */
void rsrr_timers_enable(int on);
/* Restricts the timers to the launches of one kernel function (its "sym:"
 * name without the prefix), so that a timed run pays for the events of that
 * function only; NULL or "" times every class again. */
void rsrr_timers_only(const char* sym);
void rsrr_timers_reset(void);
int rsrr_timers_count(void);
int rsrr_timers_get(int index, char* name, int name_len, long long* launches, double* total_ms,
                    double* flops, double* bytes);

/* Thread-local message of the last error (empty string if none). */
const char* rsrr_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* RSRR_H */
