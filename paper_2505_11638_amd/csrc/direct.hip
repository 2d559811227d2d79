// NGD with the full Gramian (Alg. 2, Section 4.1.1 "Computing the full Gramian"): G = J_w^T J_w formed
// explicitly in FP64 on the matrix cores, the Cholesky factor of G + mu I, and the two triangular
// substitutions L y = g, L^T d = y.
//
// The factorisation is right-looking by panels of kNb = 128 columns:
//  1. one workgroup factors the diagonal block A_kk = L_kk L_kk^T in LDS and inverts L_kk in place
//     (the inverse is kept per panel: the panel below and both substitutions multiply by it);
//  2. the panel below, L_21 = A_21 L_kk^{-T}, is one FP64 MFMA product into a staging buffer, then
//     copied into the factor;
//  3. the trailing update A_22 -= L_21 L_21^T forms only the tiles on and below the diagonal.
// The substitutions walk the same panels: a partial product of the already solved part (spread
// over many workgroups), then the panel's kNb unknowns from the kept inverse.
#include "common.h"

namespace ngd {
namespace {

constexpr int kNb = 128;
constexpr int kPitch = kNb + 1;  // odd pitch: a column of the LDS block falls in distinct banks
constexpr int kChunk = 256;      // columns (forward) or rows (backward) per partial-product workgroup

// Factor the n x n diagonal block at (k0, k0) of A (ld), n <= kNb: L_kk over the block's lower part
// (the strict upper part zeroed), L_kk^{-1} into Linv (n x n, ld kNb). A non-positive or non-finite
// pivot records its 1-based global index in *info (first one only) and stops the block.
__global__ __launch_bounds__(1024) void potrf_block_kernel(double* __restrict__ A, int64_t ld, int64_t k0, int n,
                                                           double* __restrict__ Linv, int* __restrict__ info) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* s = reinterpret_cast<double*>(smem_raw);  // n x kPitch
  __shared__ double tmp[kNb];
  __shared__ int bad;
  const int t = threadIdx.x, nt = blockDim.x;
  if (t == 0) bad = 0;
  for (int e = t; e < n * n; e += nt) {
    const int i = e / n, j = e % n;
    s[i * kPitch + j] = j <= i ? A[(k0 + i) * ld + k0 + j] : 0.0;
  }
  __syncthreads();
  // unblocked right-looking Cholesky in LDS
  for (int j = 0; j < n; ++j) {
    if (t == 0) {
      double djj = s[j * kPitch + j];
      if (!(djj > 0.0) || !isfinite(djj)) {
        bad = 1;
        if (atomicCAS(info, 0, (int)(k0 + j + 1)) != 0) { /* an earlier pivot already failed */ }
        djj = 1.0;
      }
      s[j * kPitch + j] = sqrt(djj);
    }
    __syncthreads();
    if (bad) return;
    const double rp = 1.0 / s[j * kPitch + j];
    for (int i = j + 1 + t; i < n; i += nt) s[i * kPitch + j] *= rp;
    __syncthreads();
    const int m = n - j - 1;
    for (int e = t; e < m * m; e += nt) {
      const int i = j + 1 + e / m, c = j + 1 + e % m;
      if (c <= i) s[i * kPitch + c] -= s[i * kPitch + j] * s[c * kPitch + j];
    }
    __syncthreads();
  }
  for (int e = t; e < n * n; e += nt) {
    const int i = e / n, j = e % n;
    A[(k0 + i) * ld + k0 + j] = j <= i ? s[i * kPitch + j] : 0.0;
  }
  __syncthreads();
  // in-place inverse of the lower factor, last column first: with L = [l 0; v T] and T^{-1} already
  // in place, column j of L^{-1} below the diagonal is -(1 / l) T^{-1} v
  for (int j = n - 1; j >= 0; --j) {
    if (t == 0) s[j * kPitch + j] = 1.0 / s[j * kPitch + j];
    for (int i = j + 1 + t; i < n; i += nt) tmp[i] = s[i * kPitch + j];
    __syncthreads();
    const double ljj = s[j * kPitch + j];
    for (int i = j + 1 + t; i < n; i += nt) {
      double acc = 0.0;
      for (int m = j + 1; m <= i; ++m) acc += s[i * kPitch + m] * tmp[m];
      s[i * kPitch + j] = -ljj * acc;
    }
    __syncthreads();
  }
  for (int e = t; e < n * n; e += nt) {
    const int i = e / n, j = e % n;
    Linv[i * kNb + j] = j <= i ? s[i * kPitch + j] : 0.0;
  }
}

// A[r][r] += mu for r < n (the damping of Alg. 2's G + mu I)
__global__ void add_diag_kernel(double* __restrict__ A, int64_t ld, int64_t n, double mu) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n) A[r * ld + r] += mu;
}

// Forward substitution, partial products of panel k: part[c][i] = sum over the chunk's columns q of
// L[k0 + i][q] y[q], q < k0 (one workgroup per chunk of kChunk columns, each wave a set of rows)
__global__ __launch_bounds__(256) void fwd_partial_kernel(const double* __restrict__ L, int64_t ld, int64_t k0,
                                                          int n, const double* __restrict__ y,
                                                          double* __restrict__ part) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int64_t q0 = (int64_t)blockIdx.x * kChunk;
  double yv[kChunk / 64];
#pragma unroll
  for (int u = 0; u < kChunk / 64; ++u) {
    const int64_t q = q0 + lane + 64 * u;
    yv[u] = q < k0 ? y[q] : 0.0;
  }
  for (int i = wid; i < n; i += 4) {
    const double* row = L + (k0 + i) * ld;
    double acc = 0.0;
#pragma unroll
    for (int u = 0; u < kChunk / 64; ++u) {
      const int64_t q = q0 + lane + 64 * u;
      if (q < k0) acc += row[q] * yv[u];
    }
    acc = wave_sum_dpp(acc);
    if (lane == 0) part[(int64_t)blockIdx.x * kNb + i] = acc;
  }
}

// Backward substitution, partial products of panel k: part[c][j] = sum over the chunk's rows r of
// L[r][k0 + j] x[r], r >= k0 + n (one workgroup per chunk of kChunk rows, thread j a column)
__global__ __launch_bounds__(kNb) void bwd_partial_kernel(const double* __restrict__ L, int64_t ld, int64_t k0,
                                                          int n, int64_t P, const double* __restrict__ x,
                                                          double* __restrict__ part) {
  const int j = threadIdx.x;
  const int64_t r0 = k0 + n + (int64_t)blockIdx.x * kChunk;
  const int64_t r1 = r0 + kChunk < P ? r0 + kChunk : P;
  double acc = 0.0;
  if (j < n)
    for (int64_t r = r0; r < r1; ++r) acc += L[r * ld + k0 + j] * x[r];
  part[(int64_t)blockIdx.x * kNb + j] = acc;
}

// The panel's unknowns: r = rhs[k0 + i] - sum_c part[c][i], then out[k0 + i] = (Linv r)_i (forward)
// or (Linv^T r)_i (backward), in a fixed order of additions
__global__ __launch_bounds__(kNb) void panel_solve_kernel(const double* __restrict__ Linv, int64_t k0, int n,
                                                          const double* __restrict__ rhs,
                                                          const double* __restrict__ part, int nparts, int trans,
                                                          double* __restrict__ out) {
  __shared__ double r[kNb];
  const int i = threadIdx.x;
  if (i < n) {
    double acc = 0.0;
    for (int c = 0; c < nparts; ++c) acc += part[(int64_t)c * kNb + i];
    r[i] = rhs[k0 + i] - acc;
  }
  __syncthreads();
  if (i >= n) return;
  double v = 0.0;
  if (!trans) {
    for (int m = 0; m <= i; ++m) v += Linv[i * kNb + m] * r[m];
  } else {
    for (int m = i; m < n; ++m) v += Linv[m * kNb + i] * r[m];
  }
  out[k0 + i] = v;
}

}  // namespace

size_t direct_panel_inverse_bytes(int64_t P) { return sizeof(double) * (size_t)((P + kNb - 1) / kNb) * kNb * kNb; }
size_t direct_stage_bytes(int64_t P) { return sizeof(double) * (size_t)P * kNb; }
size_t direct_part_bytes(int64_t P) { return sizeof(double) * (size_t)((P + kChunk - 1) / kChunk + 1) * kNb; }

ngd_status launch_add_diag(double* A, int64_t ld, int64_t n, double mu, hipStream_t s) {
  if (n <= 0) return NGD_OK;
  hipLaunchKernelGGL(add_diag_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, A, ld, n, mu);
  NGD_HIP_TRY(hipGetLastError());
  return NGD_OK;
}

// Lower Cholesky factor of A (P x P, ld; lower part read) in place, the panels' inverse diagonal blocks
// into Linv. `stage` holds P x kNb doubles; `info` (device, zeroed here) receives the first failed pivot.
ngd_status launch_blocked_cholesky(double* A, int64_t ld, int64_t P, double* Linv, double* stage, int* info,
                                   hipStream_t s) {
  NGD_TRY(launch_zero(info, sizeof(int), s));
  const size_t lds = sizeof(double) * (size_t)kNb * kPitch;
  NGD_HIP_TRY(hipFuncSetAttribute((const void*)potrf_block_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)lds));
  for (int64_t k0 = 0, kb = 0; k0 < P; k0 += kNb, ++kb) {
    const int n = (int)(P - k0 < kNb ? P - k0 : kNb);
    double* Lk = Linv + kb * kNb * kNb;
    hipLaunchKernelGGL(potrf_block_kernel, dim3(1), dim3(1024), lds, s, A, ld, k0, n, Lk, info);
    NGD_HIP_TRY(hipGetLastError());
    const int64_t m = P - k0 - n;
    if (m <= 0) break;
    double* A21 = A + (k0 + n) * ld + k0;
    // L_21 = A_21 L_kk^{-T} into the staging buffer (rows m, ld kNb), then into the factor
    GemmArgs pan{m, n, n, A21, ld, true, Lk, kNb, true, stage, kNb, NGD_F64, NGD_F64, NGD_F64, G_F64, 1.0, 0.0};
    NGD_TRY(launch_gemm(pan, s));
    NGD_TRY(launch_cast_rows(NGD_F64, stage, kNb, m, n, NGD_F64, A21, ld, s));
    // A_22 -= L_21 L_21^T, the tiles on and below the diagonal only
    GemmArgs up{m, m, n, stage, kNb, true, stage, kNb, true, A + (k0 + n) * ld + (k0 + n), ld, NGD_F64, NGD_F64,
                NGD_F64, G_F64, -1.0, 1.0, nullptr, 0, 2};
    NGD_TRY(launch_gemm(up, s));
  }
  return NGD_OK;
}

// d = (L L^T)^{-1} g with the factor and panel inverses of launch_blocked_cholesky; y (P doubles) and
// part (direct_part_bytes) are scratch. d may alias g.
ngd_status launch_cholesky_solve(const double* L, int64_t ld, int64_t P, const double* Linv, const double* g,
                                 double* y, double* part, double* d, hipStream_t s) {
  const int64_t nb = (P + kNb - 1) / kNb;
  for (int64_t kb = 0; kb < nb; ++kb) {
    const int64_t k0 = kb * kNb;
    const int n = (int)(P - k0 < kNb ? P - k0 : kNb);
    const int chunks = (int)((k0 + kChunk - 1) / kChunk);
    if (chunks > 0) hipLaunchKernelGGL(fwd_partial_kernel, dim3(chunks), dim3(256), 0, s, L, ld, k0, n, y, part);
    hipLaunchKernelGGL(panel_solve_kernel, dim3(1), dim3(kNb), 0, s, Linv + kb * kNb * kNb, k0, n, g, part, chunks, 0,
                       y);
    NGD_HIP_TRY(hipGetLastError());
  }
  for (int64_t kb = nb - 1; kb >= 0; --kb) {
    const int64_t k0 = kb * kNb;
    const int n = (int)(P - k0 < kNb ? P - k0 : kNb);
    const int64_t rows = P - k0 - n;
    const int chunks = (int)((rows + kChunk - 1) / kChunk);
    if (chunks > 0)
      hipLaunchKernelGGL(bwd_partial_kernel, dim3(chunks), dim3(kNb), 0, s, L, ld, k0, n, P, d, part);
    hipLaunchKernelGGL(panel_solve_kernel, dim3(1), dim3(kNb), 0, s, Linv + kb * kNb * kNb, k0, n, y, part, chunks, 1,
                       d);
    NGD_HIP_TRY(hipGetLastError());
  }
  return NGD_OK;
}

}  // namespace ngd
