/*
 * ngd.h -- C ABI of libngd: the Gramian hot path of Nystrom-preconditioned matrix-free natural
 * gradient descent for PINNs (arXiv 2505.11638), on one AMD MI355X (gfx950).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - "device" pointers are HIP device allocations owned by the caller; the library never frees or
 *   retains them beyond the call. "host" pointers are ordinary host memory.
 * - Every call enqueues its work on `stream` (a hipStream_t passed as void*, NULL = the default
 *   stream) and returns without waiting, unless its comment says it synchronises (calls that
 *   return scalars to host memory do).
 * - Working precision ("dtype") is fixed per problem handle: NGD_F64 or NGD_F32. Buffers typed
 *   "dtype" hold values of that type; buffers typed "double" are always FP64.
 * - Matrices are row-major with an explicit leading dimension (elements between consecutive rows).
 *   A set of k vectors of length P is stored as k rows: vector j starts at base + j*ld.
 * - Every call returns an ngd_status. Argument errors are detected on the host before anything is
 *   enqueued and leave all outputs untouched; ngd_last_error() then describes the problem. Nothing
 *   is thrown across the ABI. The calls are not thread-safe on one handle.
 *
 * Notation (paper -> here): parameters p -> P, collocation points q -> N, Jacobian J_theta F -> J_w
 * (rows weighted by sqrt(w_r)), damping mu -> lambda, sketch size ell, test matrix Omega.
 */
#ifndef NGD_H
#define NGD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  NGD_OK = 0,
  NGD_ERR_INVALID = 1,        /* bad argument (null pointer, size, leading dimension, dtype) */
  NGD_ERR_OOM = 2,            /* workspace allocation failed */
  NGD_ERR_NOT_PD = 3,         /* numerical failure in the FP64 sketch core */
  NGD_ERR_BREAKDOWN = 4,      /* PCG met p^T (G + lambda I) p <= 0 or a non-finite value */
  NGD_ERR_NOT_CONVERGED = 5,  /* PCG stopped at maxit above the tolerance (outputs are valid) */
  NGD_ERR_HIP = 6             /* a HIP runtime call failed */
} ngd_status;

typedef enum { NGD_F64 = 0, NGD_F32 = 1, NGD_BF16 = 2 } ngd_dtype;

/* PDE of the residual rows (Section 5.1.1 eq. energy_poisson, Section 5.1.2 eq. heat_energy,
 * Section 5.1.3 eq. navier_residual). */
typedef enum { NGD_PDE_POISSON = 0, NGD_PDE_HEAT = 1, NGD_PDE_NAVIER_STOKES = 2 } ngd_pde;

/* Kind of one collocation row. Poisson and heat problems use the first three; Navier-Stokes problems
 * the last five (an interior point gives the two momentum rows and the continuity row, a boundary
 * point one row per velocity component). */
typedef enum {
  NGD_ROW_INTERIOR = 0,
  NGD_ROW_BOUNDARY = 1,
  NGD_ROW_INITIAL = 2,
  NGD_ROW_NS_MOMENTUM_X = 3, /* -nu Laplace u_1 + u_1 d_x u_1 + u_2 d_y u_1 + d_x p - f */
  NGD_ROW_NS_MOMENTUM_Y = 4, /* -nu Laplace u_2 + u_1 d_x u_2 + u_2 d_y u_2 + d_y p - f */
  NGD_ROW_NS_CONTINUITY = 5, /* d_x u_1 + d_y u_2 */
  NGD_ROW_NS_BOUNDARY_U = 6, /* u_1 - g */
  NGD_ROW_NS_BOUNDARY_V = 7  /* u_2 - g */
} ngd_row_kind;

/*
 * One PINN least-squares problem: a tanh MLP (Section 2.3) and fixed quadrature data.
 *   widths[0] = d (input dimension), widths[1..n_layers-1] hidden widths, widths[n_layers] = 1.
 *   Poisson: all d inputs are space; interior residual = Laplace(u) + f.
 *   Heat:    inputs are (x_1..x_{d-1}, t); interior residual = u_t - Laplace_x(u) - f.
 *   Boundary and initial rows: residual = u - g. Weighted residual r_w = sqrt(w) * residual.
 * Parameter vector theta (length P): [W_1, b_1, ..., W_L+1, b_L+1], each W row-major (out x in).
 * Limits: 1 <= n_layers <= 8, 1 <= d <= 6, widths <= 256, N >= 1.
 *
 * Navier-Stokes (steady incompressible flow, Section 5.1.3, eq. navier_residual; the Gauss-Newton
 * metric of that section is J_w^T J_w): two tanh MLPs with inputs (x, y). `widths` describes the
 * velocity network (widths[0] = 2, widths[n_layers] = 2 outputs (u_1, u_2), hidden widths <= 64, at
 * least one hidden layer); the pressure network has the same input and hidden widths and one output.
 * theta = [theta_u, theta_p], P the sum of both counts. Rows use the NGD_ROW_NS_* kinds, f holds the
 * momentum rows' forcing, g the boundary rows' target, `viscosity` is nu. Such a handle supports the
 * stored-J_w path (ngd_residual_jacobian with J_w, the products, sketches, solves and line search) and
 * ngd_solution_error on the velocity; the recompute mode (ngd_jvp, ngd_vjp, operators with J == NULL)
 * and batches refuse it with NGD_ERR_INVALID.
 */
typedef struct {
  int32_t n_layers;        /* number of affine layers (hidden layers + 1) */
  const int32_t* widths;   /* host, n_layers + 1 entries; copied at create */
  int32_t pde;             /* ngd_pde */
  int32_t dtype;           /* NGD_F64 or NGD_F32: precision of theta, X, w, f, g, J_w, r_w */
  int64_t n_rows;          /* N */
  const void* X;           /* device, N x d row-major (ld = d), dtype */
  const void* w;           /* device, N, dtype: quadrature weights (> 0) */
  const void* f;           /* device, N, dtype: source on interior rows */
  const void* g;           /* device, N, dtype: target on boundary / initial rows */
  const int8_t* row_kind;  /* device, N: ngd_row_kind */
  int32_t max_ell;         /* largest sketch size that will be used with this handle, 1 .. 1024
                              (the FP64 ell x ell core kernels keep their operands in registers) */
  double viscosity;        /* nu of the Navier-Stokes rows (> 0); ignored for other PDEs */
} ngd_problem_desc;

typedef struct ngd_problem ngd_problem;  /* opaque; owns device workspace only */

/* The linear operator J_w at a fixed theta. Either J is the stored Jacobian (N x P, leading
 * dimension ldJ >= P, dtype) produced by ngd_residual_jacobian for `theta`, or J is NULL: the
 * recompute mode, where J_w is never stored whole (for N x P beyond memory; "Recompute Jacobian" of
 * Section 4.1.2). Its matvecs are formed from theta by the forward-tangent (ngd_jvp) and adjoint
 * (ngd_vjp) kernels; its sketch recomputes J_w a block of rows at a time into a scratch buffer of at
 * most 128 MB, allocated by the handle on the first recompute-mode sketch. */
typedef struct {
  const void* theta;       /* device, P, dtype (read only in the recompute mode) */
  const void* J;           /* device, N x ldJ, dtype, or NULL (recompute mode) */
  int64_t ldJ;             /* P <= ldJ <= ngd_recommended_ld when J != NULL */
} ngd_operator;

/* Create a handle: copies the descriptor (pointers are kept, data is not copied) and allocates the
 * workspace for N, P and max_ell. Returns NGD_ERR_INVALID, NGD_ERR_OOM or NGD_ERR_HIP on failure. */
ngd_status ngd_problem_create(const ngd_problem_desc* desc, ngd_problem** out);
ngd_status ngd_problem_destroy(ngd_problem* h);
/* P = sum_l (n_l n_{l-1} + n_l) (Section 2.3); -1 for a null handle. */
int64_t ngd_num_params(const ngd_problem* h);
/* Recommended leading dimension of J_w and of P-vector sets: P rounded up to 64 elements. */
int64_t ngd_recommended_ld(const ngd_problem* h);
/* Bytes of device workspace owned by the handle. */
int64_t ngd_workspace_bytes(const ngd_problem* h);
/* Thread-local description of the last non-OK status (empty string if none). */
const char* ngd_last_error(void);

/*
 * Residuals, Jacobian, gradient and loss at theta (Section 4.1.1 "Computing the full Gramian";
 * Theorem thm:matfree, eq. G_matrixfree; Alg. 1 first step).
 *   theta : device, P, dtype.
 *   r_w   : device, N, dtype, out: sqrt(w_r) * residual_r.
 *   J_w   : device, N x ldJ, dtype, out: d r_w / d theta (columns P..ldJ-1 are set to 0). ldJ >= P.
 *   grad  : device, P, double, out (nullable): J_w^T r_w = grad L.
 *   loss  : device, 1 double, out (nullable): L = 1/2 sum r_w^2.
 * J_w may be NULL (recompute mode): residuals and loss come from the forward pass alone, and grad
 * (if requested) from the adjoint kernel of ngd_vjp.
 */
ngd_status ngd_residual_jacobian(ngd_problem* h, const void* theta, void* r_w, void* J_w, int64_t ldJ,
                                 double* grad, double* loss, void* stream);

/*
 * Forward-mode product with the residual Jacobian (the parameter JVP of r_w, eq. G_matrixfree):
 * Y[j] = J_w(theta) V[j] for j < k, computed from theta without forming J_w.
 *   V : device, k x ldV, dtype (direction j at V + j*ldV; ldV >= P when k > 1).
 *   Y : device, k x ldY, dtype, out (N-vector j at Y + j*ldY; ldY >= N when k > 1).
 */
ngd_status ngd_jvp(ngd_problem* h, const void* theta, const void* V, int64_t ldV, int64_t k, void* Y,
                   int64_t ldY, void* stream);

/*
 * Adjoint product (the VJP of r_w): out = J_w(theta)^T wv, by the reverse sweep with its seeds scaled
 * by wv and the per-point parameter derivatives summed in workgroup partials (fixed-order sums).
 *   wv : device, N, dtype. out : device, P doubles.
 */
ngd_status ngd_vjp(ngd_problem* h, const void* theta, const void* wv, double* out, void* stream);

/*
 * Damped Gramian products Y[j] = (J_w^T J_w + lambda I) V[j] for j < k (eq. G_matrixfree,
 * eq. regularized_ng; "Precompute Jacobian only" strategy of Section 4.1.2). k = 1 is the
 * conjugate-gradient matvec (one pass over J_w); k > 1 is the block product of the sketch.
 *   V : device, k x ldV, dtype (vector j at V + j*ldV). Y : device, k x ldY, dtype, out.
 *   lambda >= 0. Y must not alias V or J_w.
 */
ngd_status ngd_gramian_matvec(ngd_problem* h, const ngd_operator* op, const void* V, int64_t ldV,
                              int64_t k, double lambda, void* Y, int64_t ldY, void* stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation): the conjugate-gradient product of ngd_gramian_matvec
 * (k = 1, stored J_w) without a problem handle and without any allocation,
 *   y = (J_w^T J_w + lambda I) v,
 * computed by the same one-pass kernels, so the result equals ngd_gramian_matvec's for the same
 * inputs. Its scratch (workgroup partials, FP64 copies of v and y) is a static device array of
 * NGD_NOALLOC_SCRATCH_BYTES per GPU, held until the process ends; its address is looked up once
 * per device on the first call there. Every size the one-pass matvec accepts fits
 * (ldJ * element size <= 150 KB); a size that would need more is refused with NGD_ERR_INVALID.
 * Calls that overlap on one GPU (two streams, two threads) share that scratch and race: serialise
 * them. No workspace word needs clearing between calls.
 *   dtype  : NGD_F64 or NGD_F32 (of J, v and y).
 *   J      : device, n_rows x ldJ, dtype, row-major, 16-byte aligned; ldJ >= n_params, ldJ a
 *            multiple of 16 bytes / element size.
 *   v, y   : device, n_params, dtype; y is written, must not alias v or J. lambda >= 0.
 */
#define NGD_NOALLOC_SCRATCH_BYTES (40 * 1024 * 1024)
ngd_status ngd_gramian_matvec_noalloc(int32_t dtype, const void* J, int64_t ldJ, int64_t n_rows,
                                      int64_t n_params, const void* v, double lambda, void* y,
                                      void* stream);

/*
 * Counter-based standard normal test matrix (Philox4x32-10 of Salmon et al. SC'11 with Box-Muller):
 * row j of `omega` (j < ell) is column j of the P x ell matrix Omega of eq. nystrom_approx.
 *   omega : device, ell x ld, dtype, out. ld >= P.
 */
ngd_status ngd_gaussian_omega(ngd_problem* h, uint64_t seed, uint64_t counter, int64_t ell,
                              void* omega, int64_t ld, void* stream);

typedef struct {
  double nu;        /* shift added to the ell x ell core (0 if none was needed) */
  double lam1;      /* largest Nystrom eigenvalue */
  double lam_ell;   /* smallest (ell-th) Nystrom eigenvalue */
  int32_t rank_z;   /* numerical rank of the sketch J_w Omega */
  int32_t rank;     /* number of nonzero Nystrom eigenvalues kept */
} ngd_nystrom_info;

/*
 * Randomized Nystrom approximation of the undamped Gramian G = J_w^T J_w (eq. nystrom_approx;
 * Alg. 4 first step; Alg. 6): G_nys = U diag(lam_hat) U^T.
 *   ell           : sketch size, 1 <= ell <= min(max_ell, P).
 *   omega         : device, ell x ldO, dtype (row j = column j of Omega), or NULL to generate it
 *                   on the device from (seed, counter) exactly as ngd_gaussian_omega does.
 *   sketch_dtype  : precision of the two N x P x ell products: NGD_F64 (dtype F64 only), NGD_F32
 *                   (dtype F32) or NGD_BF16 (dtype F32; BF16 inputs, FP32 accumulation). The
 *                   ell x ell core always runs in FP64.
 *   U             : device, ell x ldU, dtype, out: row i = eigenvector i (unit norm, orthogonal),
 *                   rows for dropped (zero) eigenvalues are zero. ldU >= P. Columns P..ldU-1 are not
 *                   written; the preconditioner kernels may read column P when P is odd and discard
 *                   it, so the caller keeps that padding finite (e.g. zero-initialised).
 *   lam_hat       : device, ell doubles, out: eigenvalues, descending, >= 0.
 *   info          : host, nullable. If non-NULL the call synchronises `stream`, fills it and
 *                   reports a timed-out exchange inside the FP64 core. If NULL the call does not
 *                   synchronise, and the next ngd_pcg_solve / ngd_pcg_solve_damped with this
 *                   preconditioner (same ell) reports that error instead.
 */
ngd_status ngd_nystrom_sketch(ngd_problem* h, const ngd_operator* op, int64_t ell, uint64_t seed,
                              uint64_t counter, const void* omega, int64_t ldO, int32_t sketch_dtype,
                              void* U, int64_t ldU, double* lam_hat, ngd_nystrom_info* info,
                              void* stream);

/*
 * The same Nystrom builder with a sampling test matrix (the "sampling" variant of the experiments of
 * Section 5): Omega = [e_{cols[0]}, ..., e_{cols[ell-1]}], columns of the identity, so Z = J_w Omega
 * is a gather of ell columns of J_w and the rest is as in ngd_nystrom_sketch. Repeated indices are
 * allowed (range(Omega) is what matters; the extra directions come out as dropped pairs).
 *   cols : device, ell int64 indices in [0, P) (a negative index stands for a zero column), e.g. from
 *          ngd_sample_pivots. Other arguments and the synchronisation rule as for ngd_nystrom_sketch.
 */
ngd_status ngd_nystrom_sketch_columns(ngd_problem* h, const ngd_operator* op, int64_t ell, const int64_t* cols,
                                      int32_t sketch_dtype, void* U, int64_t ldU, double* lam_hat,
                                      ngd_nystrom_info* info, void* stream);

/*
 * diag(G) = diag(J_w^T J_w), the column sums of squares of J_w (eq. gram_diagonal, with the
 * quadrature weights folded into J_w): one pass over a stored J_w, or over its rows recomputed a
 * block at a time (op->J == NULL). FP64 sums in a fixed order.
 *   diag : device, P doubles, out. Asynchronous on `stream`.
 */
ngd_status ngd_gramian_diagonal(ngd_problem* h, const ngd_operator* op, double* diag, void* stream);

/*
 * n_samples indices drawn i.i.d. from [0, P) with probability max(w_j, 0) / sum_k max(w_k, 0): the
 * pivot sampling of RPCholesky (Section 4.2.2, s ~ d) and of the sampling test matrix (Section 5).
 * Sample k of `substream` q takes the uniform u = ((x0 >> 5) 2^26 + (x1 >> 6) + 1/2) 2^-53 from the
 * first two words of Philox4x32-10 at counter (k, 2^31 + q, counter_lo, counter_hi), key (seed_lo,
 * seed_hi), and returns the first index whose running weight sum exceeds u * total.
 *   weights : device, P doubles. unique : nonzero = sort the samples and drop repeats.
 *   idx     : device, n_samples int64, out (the first *count entries are valid).
 *   count   : device, 1 int32, out: n_samples, the number of distinct indices (unique), or 0 if
 *             every weight is <= 0 (idx is then -1).
 * 0 <= n_samples <= 4096, substream < 2^31. Asynchronous on `stream`.
 */
ngd_status ngd_sample_pivots(ngd_problem* h, const double* weights, int64_t n_samples, uint64_t seed,
                             uint64_t counter, uint32_t substream, int32_t unique, int64_t* idx, int32_t* count,
                             void* stream);

/*
 * NGD with the full Gramian (Alg. 2; Section 4.1.1, "Computing the full Gramian"): the direction
 * d = (J_w^T J_w + lambda I)^{-1} g by forming G = J_w^T J_w explicitly in FP64 (the tiles on and
 * below the diagonal, O(N P^2) on the matrix cores), the Cholesky factor G + lambda I = L L^T
 * (right-looking, panels of 128 columns) and the substitutions L y = g, L^T d = y.
 *   g : device, P doubles. d : device, P doubles, out (may alias g).
 *   lambda > 0. Stored J_w, or the recompute mode (op->J == NULL: G summed over row blocks of J_w).
 * The handle allocates P x ngd_recommended_ld doubles for G on the first call and keeps them
 * (NGD_ERR_OOM if that fails). Synchronises `stream`; a non-positive pivot (G + lambda I not
 * numerically positive definite) returns NGD_ERR_NOT_PD, d then undefined.
 */
ngd_status ngd_direct_solve(ngd_problem* h, const ngd_operator* op, const double* g, double lambda, double* d,
                            void* stream);

/*
 * Block RPCholesky of G = J_w^T J_w (Section 4.2.2; the block algorithm of the appendix): G ~ F F^T
 * with F (P x r) built a block of pivots at a time. Round i (i < ceil(ell_max / block)) draws `block`
 * pivots ~ d (ngd_sample_pivots with substream i, sorted, repeats dropped), forms the residual
 * columns C = G[:, S'] - F F[S', :]^T from J_w, factors C[S', S'] = R^T R, appends C R^{-1} to F and
 * downdates d by its squared rows; it stops once the trace of the residual, sum(d), is below eps
 * (or F is full). A pivot whose residual diagonal is not safely positive (<= 1e-13 of the block's
 * largest: a direction F already holds) is dropped with its column.
 *   diag  : device, P doubles: d^(0) = diag(G) (ngd_gramian_diagonal); not modified.
 *   Ft    : device, ell_max x ldF doubles, out: row k = column k of F (rows >= rank are zero).
 *   rank  : host, out: r. trace : host, nullable, out: sum(d) at the end.
 * 1 <= block <= 64, 1 <= ell_max <= min(1024, P), ldF >= P, eps >= 0. Stored J_w, or the recompute
 * mode (op->J == NULL: every round recomputes J_w's rows a block at a time for its columns products).
 * Synchronises `stream`.
 */
ngd_status ngd_rpcholesky(ngd_problem* h, const ngd_operator* op, const double* diag, int64_t ell_max,
                          int32_t block, uint64_t seed, uint64_t counter, double eps, double* Ft, int64_t ldF,
                          int64_t* rank, double* trace, void* stream);

/*
 * The RPCholesky preconditioner P = F F^T + mu I (Section 4.2.2) in the form ngd_pcg_solve takes:
 * with the thin SVD F = U Sigma V^T (from the FP64 eigenpairs of F^T F),
 * P^{-1} = U (Sigma^2 + mu I)^{-1} U^T + mu^{-1} (I - U U^T) (eq. rpchol_svdprecond, the same P^{-1}
 * as the Woodbury form eq. rpchol_precond), which is mu^{-1} times eq. nystrom_inverse evaluated with
 * the eigenpairs of F F^T and a trailing zero pair. So U gets rank + 1 rows (the last one zero) and
 * lam_hat rank + 1 values (the last one 0); pass ell = rank + 1 to ngd_pcg_solve.
 *   Ft : device, rank x ldF doubles (from ngd_rpcholesky). U : device, (rank + 1) x ldU, dtype, out.
 *   lam_hat : device, rank + 1 doubles, out, descending.
 * rank + 1 <= max_ell. Synchronises `stream` (checks the eigensolver's exchanges).
 */
ngd_status ngd_rpchol_precond(ngd_problem* h, const double* Ft, int64_t ldF, int64_t rank, void* U, int64_t ldU,
                              double* lam_hat, void* stream);

/*
 * The RPCholesky preconditioner P = F F^T + mu I in the Woodbury-Cholesky form the paper adopts
 * (Section 4.2.2, eq. rpchol_precond): P^{-1} v = mu^{-1} (v - W W^T v) with W = F R^{-1},
 * R^T R = F^T F + mu I (FP64 Gram product and Cholesky factor of the rank x rank core, then W by one
 * triangular solve; no eigendecomposition). Written in the form ngd_pcg_solve takes: U gets the rows of
 * W^T and a trailing zero row, lam_hat = [+inf, ..., +inf, 0] (rank + 1 values), for which the apply of
 * eq. nystrom_inverse, U (Lambda + mu I)^{-1} U^T v + (lam_hat[rank] + mu)^{-1} (v - U U^T v), is
 * exactly mu^{-1} (v - W W^T v) in IEEE arithmetic. So it preconditions solves with lambda = mu only,
 * through ngd_pcg_solve (not the damped solve, whose rule reads lam_hat[0]).
 *   Ft : device, rank x ldF doubles (from ngd_rpcholesky). mu > 0. U : device, (rank + 1) x ldU, dtype,
 *   out. lam_hat : device, rank + 1 doubles, out. rank + 1 <= max_ell. The handle allocates P x max_ell
 * doubles on the first call and keeps them (NGD_ERR_OOM if that fails). Synchronises `stream` (checks
 * the factorisation's exchanges).
 */
ngd_status ngd_rpchol_precond_woodbury(ngd_problem* h, const double* Ft, int64_t ldF, int64_t rank, double mu,
                                       void* U, int64_t ldU, double* lam_hat, void* stream);

/* Nystrom preconditioner of eq. nystrom_inverse for G + mu I with mu = the solve's lambda:
 * P^{-1} v = U (Lambda + mu I)^{-1} U^T v + (lam_hat[ell-1] + mu)^{-1} (v - U U^T v). */
typedef struct {
  const void* U;           /* device, ell x ldU, dtype (as written by ngd_nystrom_sketch) */
  int64_t ldU;
  const double* lam_hat;   /* device, ell, descending */
  int64_t ell;
} ngd_precond;

typedef struct {
  int64_t iters;           /* iterations performed */
  double rel_res;          /* ||r_k|| / ||g|| of the recursively updated residual */
  int32_t converged;       /* rel_res <= rtol */
  int32_t breakdown;       /* p^T (G + lambda I) p <= 0 or non-finite */
} ngd_pcg_info;

/*
 * Solve (J_w^T J_w + lambda I) d = g by conjugate gradients, preconditioned by eq. nystrom_inverse
 * when prec != NULL, plain CG otherwise (Alg. 3: pCG(G_fun + mu Id, g, maxit, P_fun)).
 * x_0 = 0; stops when ||r_k||_2 <= rtol ||g||_2 or after maxit iterations.
 *   g : device, P doubles. d : device, P doubles, out. lambda > 0, rtol >= 0, maxit >= 0.
 *   info : host, required. The call synchronises `stream` (it polls the device-side convergence
 *          flag every few iterations). Returns NGD_ERR_NOT_CONVERGED if maxit was reached first and
 *          NGD_ERR_BREAKDOWN on breakdown; d holds the last iterate in both cases.
 */
ngd_status ngd_pcg_solve(ngd_problem* h, const ngd_operator* op, const double* g, double lambda,
                         const ngd_precond* prec, double rtol, int64_t maxit, double* d,
                         ngd_pcg_info* info, void* stream);

/*
 * ngd_pcg_solve with the damping chosen on the device by the rule of Section 4.3,
 *   lambda = max(c_lam * prec->lam_hat[0], c_loss * loss[0]^2)
 * (lam_hat[0] = lambda_hat_1 of the sketch; with c_lam = gamma eps and c_loss = 1e-4 this is the
 * paper's mu), so that the call can follow ngd_nystrom_sketch(..., info = NULL) without the host
 * reading lambda_hat_1 first: the sketch and the solve then share one host round trip.
 *   c_lam, c_loss : >= 0, not both 0. loss : device, 1 double (as written by ngd_residual_jacobian).
 *   prec          : required. lambda_used : host, nullable, out: the lambda of the solve.
 * Everything else, including the synchronisation and the errors, is as for ngd_pcg_solve.
 */
ngd_status ngd_pcg_solve_damped(ngd_problem* h, const ngd_operator* op, const double* g, double c_lam,
                                double c_loss, const double* loss, const ngd_precond* prec, double rtol,
                                int64_t maxit, double* d, ngd_pcg_info* info, double* lambda_used,
                                void* stream);

/*
 * Largest-eigenvalue estimate of J_w^T J_w by the power method (Section 4.3: 2-4 iterations):
 * v <- G v / ||G v||, returning the Rayleigh quotient v^T G v of the last normalised iterate.
 *   v0 : device, P doubles (nonzero start vector; not modified). lam1 : host, out.
 *   lam1_dev : device double, nullable, out: the same estimate, for ngd_damping. Synchronises.
 */
ngd_status ngd_power_lambda_max(ngd_problem* h, const ngd_operator* op, const double* v0, int32_t iters,
                                double* lam1, double* lam1_dev, void* stream);

/*
 * The damping rule of Section 4.3 (the experimental setup of Section 5) on the device:
 * mu = max(c_lam * lam1, c_loss * loss^2), with c_lam = gamma * eps (gamma = 10, eps the unit
 * roundoff of the working precision) and c_loss = 1e-4 in the paper's runs.
 *   lam1 : device double (lam_hat[0] of a sketch, or lam1_dev of ngd_power_lambda_max).
 *   loss : device double, nullable (then 0): the loss 1/2 ||r_w||^2 of ngd_residual_jacobian.
 *   mu   : device double, out. mu_host : host double, nullable: when given, the call synchronises
 *          and stores mu there too; otherwise it is asynchronous.
 * c_lam, c_loss finite and >= 0.
 */
ngd_status ngd_damping(ngd_problem* h, const double* lam1, const double* loss, double c_lam, double c_loss,
                       double* mu, double* mu_host, void* stream);

/*
 * Levenberg-Marquardt damping update (the heuristic by which the Navier-Stokes experiment of Section
 * 5.1.3 adapts mu; the factors are those of the trust-region radius rule of Nocedal and Wright). From
 * the step theta_new = theta - alpha d just taken, the gain ratio of the actual decrease over the
 * Gauss-Newton model's,
 *   rho = (loss0 - loss1) / (alpha g^T d - alpha^2 d^T G d / 2),   G = J_w^T J_w,
 * gives mu_next = 4 mu if rho < 1/4, mu / 2 if rho > 3/4, mu otherwise, and at least mu_floor. A step
 * not taken (alpha = 0) or a model without decrease counts as rho < 1/4 and reports rho = -1.
 *   d, grad : device, P doubles (the direction and the gradient of that step).
 *   alpha >= 0, mu > 0, mu_floor >= 0. mu_next : host, out. rho : host, nullable, out.
 * One Gramian product with d (stored J_w). Synchronises `stream`.
 */
ngd_status ngd_lm_damping(ngd_problem* h, const ngd_operator* op, const double* d, const double* grad, double alpha,
                          double loss0, double loss1, double mu, double mu_floor, double* mu_next, double* rho,
                          void* stream);

/*
 * Alg. 4's update of the sketch size (Section 4.3) from one step's eigenvalue estimates:
 * ell + dell while lam_hat[ell - 1] > 10 mu; otherwise the first 1-based index i with
 * lam_hat[i] < 10 mu plus `offset` (the text allows 1 or 2); ell if no estimate lies strictly below
 * (lam_hat[ell - 1] = 10 mu exactly); never above min(ell_max, P).
 *   lam_hat : device, ell doubles, descending (as written by ngd_nystrom_sketch).
 *   mu      : the step's damping (e.g. lambda_used of ngd_pcg_solve_damped, or mu_host of
 *             ngd_damping). next_ell : host, out. Synchronises.
 * ell >= 1, dell >= 0, offset >= 0, ell_max >= 1, mu >= 0.
 */
ngd_status ngd_next_rank(ngd_problem* h, const double* lam_hat, int64_t ell, double mu, int64_t dell,
                         int64_t offset, int64_t ell_max, int64_t* next_ell, void* stream);

/*
 * Armijo backtracking along theta - alpha d (Alg. 1, Linesearch; Section 4.4): alpha = 1, 1/2, ...
 * until L(theta - alpha d) <= loss0 - c1 alpha grad^T d, at most max_halvings halvings; alpha = 0 if
 * none is accepted. Writes theta_out = theta - alpha d (dtype; may alias theta).
 *   d, grad : device, P doubles. alpha, loss_new : host, out. Synchronises.
 */
ngd_status ngd_line_search(ngd_problem* h, const void* theta, const double* d, const double* grad,
                           double loss0, double c1, int32_t max_halvings, void* theta_out,
                           double* alpha, double* loss_new, void* stream);

/*
 * Accuracy of u_theta against a reference solution on n evaluation points, the measure by which the
 * experiments of Section 5 are compared (relative errors in L2 and H1, estimated by Monte Carlo on
 * uniform random points as in the appendix's table of discretisations). Writes four FP64 sums:
 *   sums[0] = sum_i (u(x_i) - u_ref_i)^2,          sums[1] = sum_i |grad u(x_i) - grad_u_ref_i|^2,
 *   sums[2] = sum_i u_ref_i^2,                     sums[3] = sum_i |grad_u_ref_i|^2,
 * with grad over all d inputs; then rel. L2 = sqrt(sums[0] / sums[2]) and
 * rel. H1 = sqrt((sums[0] + sums[1]) / (sums[2] + sums[3])). Evaluation only, not part of a step.
 *   theta : device, P values of the problem's dtype.  X : device, n x d row-major, problem dtype.
 *   u_ref : device, n values; grad_u_ref : device, n x d row-major (both the problem's dtype).
 *   sums  : device, 4 doubles, out (zeros for n = 0). The arithmetic is FP64 and its order is fixed.
 * Asynchronous on `stream`. NGD_ERR_INVALID for n < 0 or NULL pointers (any pointer may be NULL
 * when n = 0 except sums).
 * Navier-Stokes handles measure the velocity (the error of Section 5.1.3): X is n x 2, u_ref n x 2
 * (u_1, u_2), grad_u_ref n x 2 x 2 row-major ([k][j] = d u_k / d x_j), and the sums run over both
 * components; the network is evaluated in the problem's dtype, the sums in FP64 (per wave in point
 * order, then per workgroup, then over workgroups, all in a fixed order).
 */
ngd_status ngd_solution_error(ngd_problem* h, const void* theta, const void* X, int64_t n, const void* u_ref,
                              const void* grad_u_ref, double* sums, void* stream);

/*
 * Batches: many independent PINN problems (uneven P, N, ell; one dtype) driven together. Each batch
 * member is a full problem handle (ngd_batch_problem) usable with every single-problem entry point,
 * e.g. for its Nystrom sketch and line search; the two calls below treat all members at once.
 */
typedef struct ngd_batch ngd_batch;  /* opaque */

/* n problem descriptions (as for ngd_problem_create; all with the same dtype). */
ngd_status ngd_batch_create(const ngd_problem_desc* descs, int32_t n, ngd_batch** out);
ngd_status ngd_batch_destroy(ngd_batch* b);
int32_t ngd_batch_size(const ngd_batch* b);
/* Member i's problem handle (owned by the batch), or NULL if i is out of range. */
ngd_problem* ngd_batch_problem(ngd_batch* b, int32_t i);

/*
 * ngd_residual_jacobian for every member: persistent launches whose workgroups stride over the
 * members' point tiles, one launch per group of members whose tiles need a like amount of LDS (at
 * most three), so that narrow members are not held to the widest member's occupancy. All arrays are host arrays of n entries holding device pointers as
 * for ngd_residual_jacobian (J_w[i] with ldJ[i]; grad and loss may be NULL, or hold NULL entries).
 * Synchronises `stream` on entry (the call reuses its host-side work table).
 */
ngd_status ngd_batch_residual_jacobian(ngd_batch* b, const void* const* theta, void* const* r_w,
                                       void* const* J_w, const int64_t* ldJ, double* const* grad,
                                       double* const* loss, void* stream);

/*
 * ngd_pcg_solve for every member (Alg. 3, stored Jacobians): each PCG stage of all members is one
 * launch (matvec over all members' row blocks, update, preconditioner dot products and
 * application), and one iteration of the whole batch is captured once as a hipGraph and replayed.
 * The split of each member's rows over matvec workgroups is chosen on the first solve of a set of
 * shapes by timing candidate splits (a small autotuner).
 *   ops, g, lambda, precs, d, infos : host arrays of n entries. precs may be NULL (plain CG for
 *   all), or entries with U == NULL are plain CG. Returns NGD_ERR_NOT_CONVERGED / BREAKDOWN if any
 *   member did; infos holds each member's outcome. Synchronises `stream`.
 */
ngd_status ngd_batch_pcg_solve(ngd_batch* b, const ngd_operator* ops, const double* const* g,
                               const double* lambda, const ngd_precond* precs, double rtol, int64_t maxit,
                               double* const* d, ngd_pcg_info* infos, void* stream);

/*
 * ngd_pcg_solve_damped for every member: as ngd_batch_pcg_solve, with member i's damping from the
 * rule of Section 4.3 on the device, lambda_i = max(c_lam lam_hat_i[0], c_loss loss_i^2), from its
 * preconditioner's eigenvalues and its loss (no host round trip between the members' sketches and
 * the solve). Every member needs a preconditioner. A member's sketch taken without its summary has
 * its core's error words checked here (NGD_ERR_HIP if one timed out).
 *   loss        : host array of n device pointers (an entry may be NULL: loss 0), or NULL (all 0).
 *   lambda_used : host array of n doubles, nullable, out: each member's damping. Synchronises.
 */
ngd_status ngd_batch_pcg_solve_damped(ngd_batch* b, const ngd_operator* ops, const double* const* g,
                                      double c_lam, double c_loss, const double* const* loss,
                                      const ngd_precond* precs, double rtol, int64_t maxit, double* const* d,
                                      ngd_pcg_info* infos, double* lambda_used, void* stream);

/*
 * ngd_nystrom_sketch (Gaussian test matrix, Alg. 6 on each member's J_w) for every member, without a
 * host round trip: the members run side by side on four streams of the batch (largest ell P (N + ell)
 * first), forked from and joined back to `stream`. Member i draws Omega from (seed, counter + i 2^32),
 * so that no two members share test-matrix entries. The summaries are not returned; the core error
 * words are checked by the next batched or single solve with these preconditioners.
 *   ops, ells, U, ldU, lam_hat : host arrays of n entries (device pointers as for ngd_nystrom_sketch).
 * Asynchronous on `stream`.
 */
ngd_status ngd_batch_nystrom_sketch(ngd_batch* b, const ngd_operator* ops, const int64_t* ells, uint64_t seed,
                                    uint64_t counter, int32_t sketch_dtype, void* const* U, const int64_t* ldU,
                                    double* const* lam_hat, void* stream);

/*
 * ngd_line_search for every member (Armijo backtracking, Alg. 1's line search, Section 4.4), with the
 * acceptance test of each trial step on the device: every round evaluates the next trial steps of all
 * members still searching, side by side on the batch's streams, and brings back one decision per
 * member, so the host waits once per round (usually once) instead of once per member. Member i's
 * accepted step, new loss and theta_out are those ngd_line_search returns for it.
 *   theta, d, grad, theta_out : host arrays of n device pointers (as for ngd_line_search; theta_out[i]
 *                               may alias theta[i]). loss0 : host, n doubles (finite).
 *   alpha, loss_new : host, n doubles, out. Synchronises.
 */
ngd_status ngd_batch_line_search(ngd_batch* b, void* const* theta, double* const* d, double* const* grad,
                                 const double* loss0, double c1, int32_t max_halvings, void* const* theta_out,
                                 double* alpha, double* loss_new, void* stream);

/*
 * Measurement: the average duration of one batched matvec launch (the PCG iteration's single pass
 * over every member's J_w) on the directions of the last batched solve, from HIP events around `reps`
 * launches on `stream` (they rewrite only the solve's scratch directions). Synchronises.
 */
ngd_status ngd_batch_matvec_time(ngd_batch* b, int32_t reps, double* avg_ms, void* stream);

/*
 * Kernel timers (measurement support, not part of the method). When enabled, the library records a
 * HIP event pair on the call's stream around every launch of the timed kernels and accumulates the
 * elapsed times, so a benchmark can read the average duration of, e.g., the one-pass Gramian matvec
 * kernel while the NGD loop runs.
 */
typedef enum {
  NGD_TIMER_MATVEC_ROWS = 0,      /* one-pass J^T (J v) kernel (PCG iteration, power method, matvec) */
  NGD_TIMER_RESIDUAL_JACOBIAN = 1,/* residual + Jacobian kernel (Jacobian-writing launches only) */
  NGD_TIMER_SKETCH_Z = 2,         /* Z = J_w Omega contraction */
  NGD_TIMER_SKETCH_W = 3,         /* J_w^T Q contraction */
  NGD_TIMER_CORE = 4,             /* FP64 ell x ell core (both eigendecompositions and small products) */
  NGD_TIMER_PRECOND = 5,          /* preconditioner application inside PCG */
  NGD_TIMER_SKETCH_PREP = 6,      /* BF16 transposed copy of J_w for the second BF16 sketch product */
  NGD_NUM_TIMERS = 7
} ngd_timer_id;

/* enable != 0 turns timing on and resets all counters; enable == 0 turns it off. */
ngd_status ngd_timing_enable(ngd_problem* h, int32_t enable);
/* As ngd_timing_enable, for the timers whose bit (1u << id) is set in mask only (0: off). The
 * matvec timer stamps the kernel's own dispatch and adds no work to the stream; the others bracket
 * their kernel sequences with event records, which the device executes as extra packets. */
ngd_status ngd_timing_enable_mask(ngd_problem* h, uint32_t mask);
/* Launch count and total milliseconds of timer `id`; waits for the recorded events. */
ngd_status ngd_timing_read(ngd_problem* h, int32_t id, int64_t* launches, double* total_ms);

#ifdef __cplusplus
}
#endif

#endif /* NGD_H */
