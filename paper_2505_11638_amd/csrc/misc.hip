// Small kernels: counter-based Gaussian test matrix, precision casts, trial parameters for the
// line search, zero fill (a kernel rather than hipMemsetAsync so the work can be graph-captured).
#include <algorithm>

#include "common.h"

namespace ngd {
namespace {

// Omega^T row j (column j of the p x ell test matrix), entries 2m and 2m+1 from counter (m, j, c)
template <typename T>
__global__ void omega_kernel(uint64_t seed, uint64_t counter, int64_t P, int64_t ell, T* __restrict__ out,
                             int64_t ld) {
  const int64_t half = (P + 1) / 2;
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t j = blockIdx.y;
  if (m >= half || j >= ell) return;
  uint32_t c[4] = {(uint32_t)m, (uint32_t)j, (uint32_t)counter, (uint32_t)(counter >> 32)};
  philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
  const double x1 = u53(c[0], c[1]), x2 = u53(c[2], c[3]);
  const double rad = sqrt(-2.0 * log(x1));
  const double ang = 6.283185307179586 * x2;
  T* row = out + j * ld;
  row[2 * m] = (T)(rad * cos(ang));
  if (2 * m + 1 < P) row[2 * m + 1] = (T)(rad * sin(ang));
}

template <typename S, typename D>
__global__ void cast_kernel(const S* __restrict__ s, D* __restrict__ d, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) d[i] = (D)s[i];
}

template <typename T>
__global__ void theta_trial_kernel(const T* __restrict__ theta, const double* __restrict__ d,
                                   const double* __restrict__ alphas, double alpha0, int64_t P, T* __restrict__ out,
                                   int64_t stride) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int t = blockIdx.y;
  const double a = alphas != nullptr ? alphas[t] : alpha0;
  if (j < P) out[t * stride + j] = (T)((double)theta[j] - a * d[j]);
}

// Armijo decision on the device (Alg. 1's line search) for trials tried .. tried + nt - 1 with steps
// alphas[t] and losses[t]: the first t with loss <= loss0 - c1 alpha slope is taken, in the same
// operation order as on the host (no fused multiply-add), unless an earlier round took one.
// st: [0] found (0 / 1), [1] alpha, [2] loss, [3] index.
__global__ void armijo_kernel(const double* __restrict__ alphas, const double* __restrict__ losses,
                              const double* __restrict__ slope, double loss0, double c1, int nt, int tried,
                              double* __restrict__ st) {
  if (threadIdx.x != 0 || st[0] != 0.0) return;
  const double g = *slope;
  for (int t = 0; t < nt; ++t) {
    const double a = alphas[t], Lt = losses[t];
    if (Lt <= __dsub_rn(loss0, __dmul_rn(__dmul_rn(c1, a), g))) {
      st[0] = 1.0;
      st[1] = a;
      st[2] = Lt;
      st[3] = (double)(tried + t);
      return;
    }
  }
}

// Levenberg-Marquardt update of the damping from the step just taken (the heuristic of the Navier-Stokes
// experiment, Section 5.1.3, with the factors of the trust-region radius rule of Nocedal and Wright):
// gain ratio rho = (loss0 - loss1) / pred with the Gauss-Newton model's decrease
// pred = alpha g^T d - alpha^2 d^T G d / 2; mu * 4 if rho < 1/4, mu / 2 if rho > 3/4, else mu; never below
// floor. No step (alpha = 0) or a model without decrease (pred <= 0) counts as rho < 1/4 (rho = -1).
// out[0] = mu_next, out[1] = rho.
__global__ void lm_damping_kernel(const double* __restrict__ gd, const double* __restrict__ dgd, double alpha,
                                  double loss0, double loss1, double mu, double floor_mu, double* __restrict__ out) {
  if (threadIdx.x != 0) return;
  const double pred = __dsub_rn(__dmul_rn(alpha, *gd), __dmul_rn(__dmul_rn(0.5, __dmul_rn(alpha, alpha)), *dgd));
  const double rho = (alpha > 0.0 && pred > 0.0) ? (loss0 - loss1) / pred : -1.0;
  const double m = rho < 0.25 ? 4.0 * mu : (rho > 0.75 ? 0.5 * mu : mu);
  out[0] = fmax(m, floor_mu);
  out[1] = rho;
}

// lam[i] = +inf for i < n, lam[n] = 0: the eigenvalue slots under which the preconditioner apply of
// eq. nystrom_inverse reproduces the Woodbury form eq. rpchol_precond exactly
__global__ void woodbury_lam_kernel(double* __restrict__ lam, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i <= n; i += gridDim.x * blockDim.x)
    lam[i] = i < n ? __builtin_huge_val() : 0.0;
}

// The sketch's summary for the host, gathered so that one copy brings it back:
// out[0] = lam[0], out[1] = lam[L-1], out[2] = #{lam > 0}, out[3] = core[1] (the shift nu),
// out[4] = the modified-pivot count (an int stored at core[10]), out[5], out[6] = the error words.
__global__ __launch_bounds__(256) void sketch_info_kernel(const double* __restrict__ lam, int L,
                                                          const double* __restrict__ core,
                                                          const int* __restrict__ eig_err,
                                                          const int* __restrict__ chol_err, double* __restrict__ out) {
  __shared__ double red[4];
  double c = 0.0;
  for (int i = threadIdx.x; i < L; i += blockDim.x) c += lam[i] > 0.0 ? 1.0 : 0.0;
  c = block_sum(c, red);
  if (threadIdx.x == 0) {
    int nmod = 0;
    __builtin_memcpy(&nmod, core + 10, sizeof(int));
    out[0] = lam[0];
    out[1] = lam[L - 1];
    out[2] = c;
    out[3] = core[1];
    out[4] = (double)nmod;
    out[5] = (double)*eig_err;
    out[6] = (double)*chol_err;
  }
}

// F[k][i] = V[i][k] / sqrt(lam_i) for lam_i > 0, else 0 (rows of V are eigenvectors)
__global__ void whitening_kernel(const double* __restrict__ evals, const double* __restrict__ V, int ell,
                                 double* __restrict__ F) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;  // column of F
  const int k = blockIdx.y;                             // row of F
  if (i >= ell) return;
  const double lam = evals[i];
  F[(int64_t)k * ell + i] = lam > 0.0 ? V[(int64_t)i * ell + k] / sqrt(lam) : 0.0;
}

template <typename T>
__global__ void add_scaled_kernel(const T* __restrict__ X, int64_t ldx, double a, T* __restrict__ Y, int64_t ldy,
                                  int64_t cols) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t r = blockIdx.y;
  if (j < cols) Y[r * ldy + j] = (T)((double)Y[r * ldy + j] + a * (double)X[r * ldx + j]);
}

__global__ void zero_kernel(uint32_t* __restrict__ p, int64_t n_words) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_words) p[i] = 0u;
}

// The damping rule of Section 4.3 for n problems: mu_i = max(c_lam lam1_i, c_loss loss_i^2), with the
// inputs and the output behind per-problem device pointers (a null loss pointer counts as 0)
__global__ void damping_kernel(const double* const* __restrict__ lam1, const double* const* __restrict__ loss,
                               double c_lam, double c_loss, double* const* __restrict__ mu, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double l = loss[i] != nullptr ? *loss[i] : 0.0;
  *mu[i] = fmax(c_lam * *lam1[i], c_loss * l * l);
}

// The split of the first eigendecomposition of B^T B: pairs with lam >= tau lam_0 (and > 0) are kept
// as they are (lam_t, and their eigenvector rows in Evt); the others are zeroed in both, to be
// recomputed from B projected off the kept ones.
__global__ void split_top_kernel(const double* __restrict__ lam, const double* __restrict__ Ev, int L, double tau,
                                 double* __restrict__ lam_t, double* __restrict__ Evt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;  // column
  const int k = blockIdx.y;                             // pair
  const bool keep = lam[k] > 0.0 && lam[k] >= tau * lam[0];
  if (i == 0) lam_t[k] = keep ? lam[k] : 0.0;
  if (i < L) Evt[(int64_t)k * L + i] = keep ? Ev[(int64_t)k * L + i] : 0.0;
}

// Rows r.. of U and lam_hat from the second, projected eigendecomposition: r = the number of kept pairs
// of the first (the leading nonzeros of lam_t); destination row j >= r takes pair j - r of the second
// (eigenvalue mu, vector row U2) when mu is above the noise floor floor_rel * lam_t[0], else zeros.
// The value is capped at lam_t[r - 1] so that the order stays descending across the seam (the two
// differ there by rounding only).
template <typename T>
__global__ void merge_small_kernel(const double* __restrict__ lam_t, const double* __restrict__ mu,
                                   const T* __restrict__ U2, int64_t ld2, int L, int64_t P, double floor_rel,
                                   T* __restrict__ U, int64_t ldU, double* __restrict__ lam_hat) {
  __shared__ int r_s;
  if (threadIdx.x == 0) {
    int r = 0;
    while (r < L && lam_t[r] > 0.0) ++r;
    r_s = r;
  }
  __syncthreads();
  const int r = r_s;
  const int j = blockIdx.y;
  if (j < r) return;
  const int src = j - r;
  const double m = mu[src];
  const bool keep = r > 0 && m > 0.0 && m >= floor_rel * lam_t[0];
  if (blockIdx.x == 0 && threadIdx.x == 0) lam_hat[j] = keep ? fmin(m, lam_t[r - 1]) : 0.0;
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < P; c += (int64_t)gridDim.x * blockDim.x)
    U[(int64_t)j * ldU + c] = keep ? U2[(int64_t)src * ld2 + c] : T(0);
}

__global__ void damping1_kernel(const double* __restrict__ lam1, const double* __restrict__ loss, double c_lam,
                                double c_loss, double* __restrict__ mu) {
  const double l = loss != nullptr ? *loss : 0.0;
  *mu = fmax(c_lam * *lam1, c_loss * l * l);
}

// Alg. 4's update of the sketch size from the descending eigenvalue estimates lam[0 .. ell) and the
// damping mu: ell + dell while lam[ell - 1] > 10 mu, else the first (1-based) index with lam_i < 10 mu
// plus `offset`, else ell (lam_ell = 10 mu exactly); never above ell_max. One wave: the first index
// below the threshold is the smallest lane hit, reduced over chunks of 64.
__global__ __launch_bounds__(64) void next_rank_kernel(const double* __restrict__ lam, int64_t ell, double mu,
                                                       int64_t dell, int64_t offset,
                                                       int64_t ell_max, int64_t* __restrict__ out) {
  const double thresh = 10.0 * mu;
  int64_t next;
  if (lam[ell - 1] > thresh) {
    next = ell + dell;
  } else {
    int64_t first = ell;
    for (int64_t c = 0; c < ell && first == ell; c += 64) {
      const int64_t i = c + threadIdx.x;
      const bool hit = i < ell && lam[i] < thresh;
      const unsigned long long m = __ballot(hit);
      if (m != 0ull) first = c + (int64_t)__builtin_ctzll(m);
    }
    next = first < ell ? first + 1 + offset : ell;
  }
  if (threadIdx.x == 0) *out = next < ell_max ? next : ell_max;
}

}  // namespace

ngd_status launch_gaussian_omega(int dtype, uint64_t seed, uint64_t counter, int64_t P, int64_t ell, void* out,
                                 int64_t ld, hipStream_t s) {
  dim3 grid((unsigned)(((P + 1) / 2 + 255) / 256), (unsigned)ell);
  if (dtype == NGD_F64)
    hipLaunchKernelGGL(omega_kernel<double>, grid, dim3(256), 0, s, seed, counter, P, ell, (double*)out, ld);
  else
    hipLaunchKernelGGL(omega_kernel<float>, grid, dim3(256), 0, s, seed, counter, P, ell, (float*)out, ld);
  NGD_HIP_TRY(hipGetLastError());
  return NGD_OK;
}

ngd_status launch_cast(int st, const void* src, int dt, void* dst, int64_t n, hipStream_t s) {
  if (n <= 0) return NGD_OK;
  dim3 grid((unsigned)((n + 255) / 256));
  if (st == NGD_F64 && dt == NGD_F32)
    hipLaunchKernelGGL((cast_kernel<double, float>), grid, dim3(256), 0, s, (const double*)src, (float*)dst, n);
  else if (st == NGD_F32 && dt == NGD_F64)
    hipLaunchKernelGGL((cast_kernel<float, double>), grid, dim3(256), 0, s, (const float*)src, (double*)dst, n);
  else if (st == NGD_F64 && dt == NGD_F64)
    hipLaunchKernelGGL((cast_kernel<double, double>), grid, dim3(256), 0, s, (const double*)src, (double*)dst, n);
  else
    hipLaunchKernelGGL((cast_kernel<float, float>), grid, dim3(256), 0, s, (const float*)src, (float*)dst, n);
  NGD_HIP_TRY(hipGetLastError());
  return NGD_OK;
}

ngd_status launch_axpy_theta(int dtype, const void* theta, const double* d, const double* alphas, int n_alpha,
                             int64_t P, void* out, int64_t out_stride, hipStream_t s, double alpha0) {
  dim3 grid((unsigned)((P + 255) / 256), (unsigned)n_alpha);
  if (dtype == NGD_F64)
    hipLaunchKernelGGL(theta_trial_kernel<double>, grid, dim3(256), 0, s, (const double*)theta, d, alphas, alpha0, P,
                       (double*)out, out_stride);
  else
    hipLaunchKernelGGL(theta_trial_kernel<float>, grid, dim3(256), 0, s, (const float*)theta, d, alphas, alpha0, P,
                       (float*)out, out_stride);
  NGD_HIP_TRY(hipGetLastError());
  return NGD_OK;
}

ngd_status launch_armijo(const double* alphas, const double* losses, const double* slope, double loss0, double c1,
                         int nt, int tried, double* st, hipStream_t s) {
  hipLaunchKernelGGL(armijo_kernel, dim3(1), dim3(64), 0, s, alphas, losses, slope, loss0, c1, nt, tried, st);
  NGD_HIP_TRY(hipGetLastError());
  return NGD_OK;
}

ngd_status launch_lm_damping(const double* gd, const double* dgd, double alpha, double loss0, double loss1, double mu,
                             double floor_mu, double* out, hipStream_t s) {
  hipLaunchKernelGGL(lm_damping_kernel, dim3(1), dim3(64), 0, s, gd, dgd, alpha, loss0, loss1, mu, floor_mu, out);
  NGD_HIP_TRY(hipGetLastError());
  return NGD_OK;
}

ngd_status launch_woodbury_lam(double* lam, int n, hipStream_t s) {
  hipLaunchKernelGGL(woodbury_lam_kernel, dim3((unsigned)((n + 256) / 256)), dim3(256), 0, s, lam, n);
  NGD_HIP_TRY(hipGetLastError());
  return NGD_OK;
}

ngd_status launch_sketch_info(const double* lam, int L, const double* core, const int* eig_err, const int* chol_err,
                              double* out, hipStream_t s) {
  hipLaunchKernelGGL(sketch_info_kernel, dim3(1), dim3(256), 0, s, lam, L, core, eig_err, chol_err, out);
  NGD_HIP_TRY(hipGetLastError());
  return NGD_OK;
}

ngd_status launch_whitening(const double* evals, const double* evec_rows, int ell, double* F, hipStream_t s) {
  hipLaunchKernelGGL(whitening_kernel, dim3((unsigned)((ell + 255) / 256), (unsigned)ell), dim3(256), 0, s, evals,
                     evec_rows, ell, F);
  NGD_HIP_TRY(hipGetLastError());
  return NGD_OK;
}

ngd_status launch_add_scaled(int dtype, const void* X, int64_t ldx, double a, void* Y, int64_t ldy, int64_t rows,
                             int64_t cols, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return NGD_OK;
  dim3 grid((unsigned)((cols + 255) / 256), (unsigned)rows);
  if (dtype == NGD_F64)
    hipLaunchKernelGGL(add_scaled_kernel<double>, grid, dim3(256), 0, s, (const double*)X, ldx, a, (double*)Y, ldy, cols);
  else
    hipLaunchKernelGGL(add_scaled_kernel<float>, grid, dim3(256), 0, s, (const float*)X, ldx, a, (float*)Y, ldy, cols);
  NGD_HIP_TRY(hipGetLastError());
  return NGD_OK;
}

ngd_status launch_zero(void* p, size_t bytes, hipStream_t s) {
  const int64_t words = (int64_t)(bytes / 4);
  if (words <= 0) return NGD_OK;
  hipLaunchKernelGGL(zero_kernel, dim3((unsigned)((words + 255) / 256)), dim3(256), 0, s, (uint32_t*)p, words);
  NGD_HIP_TRY(hipGetLastError());
  return NGD_OK;
}

ngd_status launch_damping1(const double* lam1, const double* loss, double c_lam, double c_loss, double* mu,
                           hipStream_t s) {
  hipLaunchKernelGGL(damping1_kernel, dim3(1), dim3(1), 0, s, lam1, loss, c_lam, c_loss, mu);
  NGD_HIP_TRY(hipGetLastError());
  return NGD_OK;
}

ngd_status launch_damping(const double* const* lam1, const double* const* loss, double c_lam, double c_loss,
                          double* const* mu, int n, hipStream_t s) {
  if (n <= 0) return NGD_OK;
  hipLaunchKernelGGL(damping_kernel, dim3((unsigned)((n + 63) / 64)), dim3(64), 0, s, lam1, loss, c_lam, c_loss, mu, n);
  NGD_HIP_TRY(hipGetLastError());
  return NGD_OK;
}

ngd_status launch_next_rank(const double* lam, int64_t ell, double mu, int64_t dell, int64_t offset,
                            int64_t ell_max, int64_t* out, hipStream_t s) {
  hipLaunchKernelGGL(next_rank_kernel, dim3(1), dim3(64), 0, s, lam, ell, mu, dell, offset, ell_max, out);
  NGD_HIP_TRY(hipGetLastError());
  return NGD_OK;
}

ngd_status launch_split_top(const double* lam, const double* Ev, int L, double tau, double* lam_t, double* Evt,
                            hipStream_t s) {
  if (L <= 0) return NGD_OK;
  hipLaunchKernelGGL(split_top_kernel, dim3((unsigned)((L + 255) / 256), (unsigned)L), dim3(256), 0, s, lam, Ev, L, tau,
                     lam_t, Evt);
  NGD_HIP_TRY(hipGetLastError());
  return NGD_OK;
}

ngd_status launch_merge_small(int dtype, const double* lam_t, const double* mu, const void* U2, int64_t ld2, int L,
                              int64_t P, double floor_rel, void* U, int64_t ldU, double* lam_hat, hipStream_t s) {
  if (L <= 0) return NGD_OK;
  dim3 grid((unsigned)std::min<int64_t>((P + 255) / 256, 64), (unsigned)L);
  if (dtype == NGD_F64)
    hipLaunchKernelGGL(merge_small_kernel<double>, grid, dim3(256), 0, s, lam_t, mu, (const double*)U2, ld2, L, P,
                       floor_rel, (double*)U, ldU, lam_hat);
  else
    hipLaunchKernelGGL(merge_small_kernel<float>, grid, dim3(256), 0, s, lam_t, mu, (const float*)U2, ld2, L, P,
                       floor_rel, (float*)U, ldU, lam_hat);
  NGD_HIP_TRY(hipGetLastError());
  return NGD_OK;
}

}  // namespace ngd
