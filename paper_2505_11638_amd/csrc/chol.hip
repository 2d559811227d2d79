// Shifted Cholesky of the ell x ell core M + nu I = L L^T and the triangular solve Q = Z L^{-T}
// (Alg. 6: C = chol(Omega^T Y_nu), B = Y_nu / C), both blocked by panels of kNb columns:
//  * Cholesky panel j0: one workgroup factors the kNb x kNb diagonal block in LDS, then the rows
//    below are solved, L21 = A21 L11^{-T}, one row per thread, and the trailing matrix is updated
//    with one MFMA GEMM, A22 -= L21 L21^T.
//  * Triangular solve, panel j0 of Q (FP64, N x ell): Q_J -= Q_<J L_J,<J^T by one GEMM, then
//    Q_J = Q_J L_JJ^{-T} row by row.
// A pivot that is not safely positive is replaced by a floor (pivot^2 = `floor`), so the
// factorisation never fails; the directions involved are left shrunk in Q (the effect of the
// shift nu in Alg. 6). Their count is reported as a rank deficit.
#include <algorithm>

#include "common.h"

namespace ngd {
namespace {

constexpr int kNb = 32;
constexpr int kLd = kNb + 1;  // LDS row pitch of a staged block

// factor the nb x nb diagonal block at (j0, j0) of A (ld n) into Ls (LDS, lower, kNb x kLd): thread t
// owns row t % 32, and the blockDim / 32 thread groups split the columns of the trailing update
__device__ void factor_diag(const double* __restrict__ A, int n, int j0, int nb, double floor, double null_thresh,
                            double* Ls, int* nmod) {
  const int t = threadIdx.x;
  for (int e = t; e < kNb * kNb; e += blockDim.x) {
    const int r = e >> 5, c = e & 31;
    Ls[r * kLd + c] = (r < nb && c <= r) ? A[(int64_t)(j0 + r) * n + j0 + c] : 0.0;
  }
  __syncthreads();
  const int r = t & 31, half = t >> 5, halves = (int)blockDim.x >> 5;
  for (int c = 0; c < nb; ++c) {
    if (t == 0) {
      double a = Ls[c * kLd + c];
      if (!(a > null_thresh) && nmod) ++*nmod;  // direction at the level of the shift: numerically null
      if (!(a > floor)) a = floor;
      Ls[c * kLd + c] = sqrt(a);
    }
    __syncthreads();
    const double rp = 1.0 / Ls[c * kLd + c];
    if (half == 0 && r > c && r < nb) Ls[r * kLd + c] *= rp;
    __syncthreads();
    if (r > c && r < nb) {
      const double lrc = Ls[r * kLd + c];
      for (int q = c + 1 + half; q <= r; q += halves) Ls[r * kLd + q] -= lrc * Ls[q * kLd + c];
    }
    __syncthreads();
  }
}

// one row x (nb values) of X: solve x L^T = x in place; L lower in LDS (pitch kLd), rdiag its
// reciprocal diagonal
__device__ __forceinline__ void solve_row(double* __restrict__ x, const double* Ls, const double* rdiag, int nb) {
  double v[kNb];
#pragma unroll
  for (int j = 0; j < kNb; ++j) v[j] = j < nb ? x[j] : 0.0;
#pragma unroll
  for (int j = 0; j < kNb; ++j) {
    if (j < nb) {
      double s = v[j];
#pragma unroll
      for (int k = 0; k < kNb; ++k)
        if (k < j) s -= v[k] * Ls[j * kLd + k];
      v[j] = s * rdiag[j];
    }
  }
#pragma unroll
  for (int j = 0; j < kNb; ++j)
    if (j < nb) x[j] = v[j];
}

// One Cholesky panel: every workgroup factors the diagonal block of panel j0 in LDS (workgroup 0
// also stores the factor in Lblk and counts the null pivots), then solves its share of the rows
// below, L21 = A21 L11^{-T}, one row per thread. Fusing the two saves a launch and a dependency per
// panel; the factor goes to Lblk, not back into A, because the other workgroups are still reading
// A's diagonal block (copy_diag_blocks_kernel moves all factors into place at the end).
__global__ __launch_bounds__(256) void chol_panel_kernel(double* __restrict__ A, int n, int j0, int nb,
                                                         const double* __restrict__ floor_p, int* __restrict__ nmod,
                                                         double* __restrict__ Lblk) {
  __shared__ double Ls[kNb * kLd];
  __shared__ double rdiag[kNb];
  __shared__ int local_mod;
  if (threadIdx.x == 0) local_mod = 0;
  __syncthreads();
  factor_diag(A, n, j0, nb, floor_p[0], floor_p[2], Ls, &local_mod);
  if (blockIdx.x == 0) {
    double* dst = Lblk + (int64_t)(j0 / kNb) * kNb * kNb;
    for (int e = threadIdx.x; e < kNb * kNb; e += blockDim.x) {
      const int r = e >> 5, c = e & 31;
      dst[e] = (r < nb && c <= r) ? Ls[r * kLd + c] : 0.0;
    }
    if (threadIdx.x == 0) *nmod += local_mod;
  }
  if (threadIdx.x < kNb) rdiag[threadIdx.x] = threadIdx.x < nb ? 1.0 / Ls[threadIdx.x * kLd + threadIdx.x] : 0.0;
  __syncthreads();
  const int64_t below = n - j0 - nb;
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r < below) solve_row(A + (j0 + nb + r) * (int64_t)n + j0, Ls, rdiag, nb);
}

// the diagonal factors from Lblk into A's diagonal blocks (upper part of each block zeroed)
__global__ __launch_bounds__(256) void copy_diag_blocks_kernel(double* __restrict__ A, int n,
                                                               const double* __restrict__ Lblk) {
  const int j0 = blockIdx.x * kNb;
  const int nb = min(kNb, n - j0);
  const double* src = Lblk + (int64_t)blockIdx.x * kNb * kNb;
  for (int e = threadIdx.x; e < kNb * kNb; e += blockDim.x) {
    const int r = e >> 5, c = e & 31;
    if (r < nb && c < nb) A[(int64_t)(j0 + r) * n + j0 + c] = src[e];
  }
}

// rows of X (FP64, ld ldx): X[r, j0:j0+nb] <- X[r, j0:j0+nb] L_JJ^{-T}, L read from the factor
__global__ __launch_bounds__(256) void trsm_rows_kernel(const double* __restrict__ L, int n, int j0, int nb,
                                                        double* __restrict__ X, int64_t ldx, int64_t nrows) {
  __shared__ double Ls[kNb * kLd];
  __shared__ double rdiag[kNb];
  for (int e = threadIdx.x; e < kNb * kNb; e += blockDim.x) {
    const int r = e >> 5, c = e & 31;
    Ls[r * kLd + c] = (r < nb && c <= r) ? L[(int64_t)(j0 + r) * n + j0 + c] : 0.0;
  }
  __syncthreads();
  if (threadIdx.x < kNb) rdiag[threadIdx.x] = threadIdx.x < nb ? 1.0 / Ls[threadIdx.x * kLd + threadIdx.x] : 0.0;
  __syncthreads();
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r < nrows) solve_row(X + r * ldx + j0, Ls, rdiag, nb);
}

// nu = shift_rel * trace(M) added to the diagonal; floor = floor_rel * trace(M)
__global__ void shift_kernel(double* __restrict__ M, int n, double shift_rel, double floor_rel,
                             double* __restrict__ floor_out, int* __restrict__ nmod) {
  __shared__ double red[4];
  double t = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) t += M[(int64_t)i * n + i];
  t = block_sum(t, red);
  const double nu = shift_rel * t;
  for (int i = threadIdx.x; i < n; i += blockDim.x) M[(int64_t)i * n + i] += nu;
  if (threadIdx.x == 0) {
    floor_out[0] = t > 0.0 ? floor_rel * t : 1e-300;
    floor_out[1] = nu;
    floor_out[2] = 100.0 * nu;
    *nmod = 0;
  }
}

}  // namespace

// L (lower, in place of M) with L L^T = M + nu I, nu = shift_rel tr(M). `scal` holds 3 doubles
// (floor, nu, null threshold) and `nmod` the count of null pivots (both device); Lblk holds
// ceil(n / 32) 32 x 32 blocks of scratch.
ngd_status launch_shifted_cholesky(double* M, int n, double shift_rel, double floor_rel, double* scal, int* nmod,
                                   double* Lblk, hipStream_t s) {
  hipLaunchKernelGGL(shift_kernel, dim3(1), dim3(256), 0, s, M, n, shift_rel, floor_rel, scal, nmod);
  NGD_HIP_TRY(hipGetLastError());
  for (int j0 = 0; j0 < n; j0 += kNb) {
    const int nb = std::min(kNb, n - j0);
    const int below = n - j0 - nb;
    // L11 and L21 = A21 L11^{-T} in one launch
    const unsigned wgs = (unsigned)std::max(1, (below + 255) / 256);
    hipLaunchKernelGGL(chol_panel_kernel, dim3(wgs), dim3(256), 0, s, M, n, j0, nb, scal, nmod, Lblk);
    NGD_HIP_TRY(hipGetLastError());
    if (below > 0) {
      // A22 -= L21 L21^T
      const int t0 = j0 + nb;
      GemmArgs g{below, below, nb, M + (int64_t)t0 * n + j0, n, true, M + (int64_t)t0 * n + j0, n, true,
                 M + (int64_t)t0 * n + t0, n, NGD_F64, NGD_F64, NGD_F64, G_F64, -1.0, 1.0};
      ngd_status st = launch_gemm(g, s);
      if (st != NGD_OK) return st;
    }
  }
  hipLaunchKernelGGL(copy_diag_blocks_kernel, dim3((unsigned)((n + kNb - 1) / kNb)), dim3(256), 0, s, M, n, Lblk);
  NGD_HIP_TRY(hipGetLastError());
  return NGD_OK;
}

// X (nrows x n, FP64, ld ldx) <- X L^{-T} with L from launch_shifted_cholesky
ngd_status launch_trsm_right_lt(const double* L, int n, double* X, int64_t ldx, int64_t nrows, hipStream_t s) {
  for (int j0 = 0; j0 < n; j0 += kNb) {
    const int nb = std::min(kNb, n - j0);
    if (j0 > 0) {
      // X_J -= X_<J L_J,<J^T
      GemmArgs g{nrows, nb, j0, X, ldx, true, L + (int64_t)j0 * n, n, true, X + j0, ldx, NGD_F64, NGD_F64, NGD_F64,
                 G_F64, -1.0, 1.0};
      ngd_status st = launch_gemm(g, s);
      if (st != NGD_OK) return st;
    }
    hipLaunchKernelGGL(trsm_rows_kernel, dim3((unsigned)((nrows + 255) / 256)), dim3(256), 0, s, L, n, j0, nb, X, ldx,
                       nrows);
    NGD_HIP_TRY(hipGetLastError());
  }
  return NGD_OK;
}

}  // namespace ngd
