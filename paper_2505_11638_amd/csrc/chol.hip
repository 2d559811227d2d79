// Shifted Cholesky of the ell x ell core M + nu I = L L^T and the triangular solve Q = Z L^{-T}
// (Alg. 6: C = chol(Omega^T Y_nu), B = Y_nu / C):
//  * Cholesky, by panels of kNb columns: one workgroup factors the kNb x kNb diagonal block in LDS,
//    the rows below are solved, L21 = A21 L11^{-T}, one row per thread, and the trailing matrix is
//    updated with one MFMA GEMM, A22 -= L21 L21^T.
//  * Triangular solve: one launch, 16 rows of Z per workgroup (trsm_q_kernel below).
// A pivot that is not safely positive is replaced by a floor (pivot^2 = `floor`), so the
// factorisation never fails; the directions involved are left shrunk in Q (the effect of the
// shift nu in Alg. 6). Their count is reported as a rank deficit.
#include <algorithm>

#include "common.h"

namespace ngd {
namespace {

constexpr int kNb = 32;
constexpr int kLd = kNb + 1;  // LDS row pitch of a staged block

// factor the nb x nb diagonal block at (j0, j0) of A (ld n) into Ls (LDS, lower, kNb x kLd). The block
// is factored by wave 0 alone, in registers: lane l holds row l % 32, columns l / 32, l / 32 + 2, ...
// Per column c the pivot is read from its lane, the column is scaled by the lanes that hold it and
// published through LDS, and every lane applies the rank-1 update to its 16 entries; a wave needs no
// workgroup barrier for any of this.
__device__ void factor_diag(const double* __restrict__ A, int n, int j0, int nb, double floor, double null_thresh,
                            double* Ls, int* nmod) {
  __shared__ double col[kNb];
  const int t = threadIdx.x;
  if (t < 64) {
    const int r = t & 31, h = t >> 5;
    double a[kNb / 2];
#pragma unroll
    for (int i = 0; i < kNb / 2; ++i) {
      const int c = h + 2 * i;
      a[i] = (r < nb && c <= r) ? A[(int64_t)(j0 + r) * n + j0 + c] : 0.0;
    }
    int nulls = 0;
#pragma unroll
    for (int c = 0; c < kNb; ++c) {
      if (c < nb) {
        const int owner = c + 32 * (c & 1);
        double piv = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(a[c >> 1]), owner),
                                      __builtin_amdgcn_readlane(__double2loint(a[c >> 1]), owner));
        if (!(piv > null_thresh)) ++nulls;  // direction at the level of the shift: numerically null
        if (!(piv > floor)) piv = floor;
        const double d = sqrt(piv), rd = 1.0 / d;
        if (h == (c & 1)) {
          if (r == c) a[c >> 1] = d;
          else if (r > c && r < nb) a[c >> 1] *= rd;
          col[r] = (r > c && r < nb) ? a[c >> 1] : 0.0;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const double lr = col[r];
#pragma unroll
        for (int i = 0; i < kNb / 2; ++i) {
          const int q = h + 2 * i;
          if (q > c && q <= r) a[i] -= lr * col[q];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      }
    }
#pragma unroll
    for (int i = 0; i < kNb / 2; ++i) {
      const int c = h + 2 * i;
      Ls[r * kLd + c] = (r < nb && c <= r) ? a[i] : 0.0;
    }
    if (t == 0 && nmod) *nmod += nulls;
  }
  __syncthreads();
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

// ---- Q = Z L^{-T} in one launch (FP64 matrix cores) ----
// A workgroup (4 or 8 waves) owns 16 rows of Z and sweeps the ell columns in 16-column panels J:
//   S = X_<J L_J,<J^T     each wave over the column tiles it holds, as S^T = L_J,<J X_<J^T,
//   X_J = (Z_J - S) L_JJ^{-T}  by forward substitution (the wave that will hold tile J),
// with the solved tiles of X kept in registers (tile t in wave t % waves). A tile is held as
// X(row l % 16, col 16 t + 4 (l / 16) + r) in element r of lane l, which is exactly the B operand of
// v_mfma_f64_16x16x4f64 at K-step r once the contraction index of that step is taken to run over
// columns 16 t + 4 kk + r (kk = l / 16); the A operand (rows of L) is then four contiguous doubles
// per lane. Q (FP64) and / or Q^T in a compute type are written as the tiles are solved.
typedef double tq_d4 __attribute__((ext_vector_type(4)));

template <typename TZ, typename TQT, int MAXS, int kTqWaves>
__global__ __launch_bounds__(64 * kTqWaves) void trsm_q_kernel(const double* __restrict__ L, int ell,
                                                               const TZ* __restrict__ Z, int64_t N,
                                                               double* __restrict__ Q, TQT* __restrict__ Qt,
                                                               int64_t ldqt) {
  __shared__ double Sp[2][kTqWaves][256];  // partial S^T of each wave, double-buffered by panel parity
  __shared__ double Ld[2][16][17];          // L_JJ and its reciprocal diagonal
  __shared__ double Rd[2][16];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int lr = lane & 15, lq = lane >> 4;
  const int64_t row = (int64_t)blockIdx.x * 16 + lr;
  const int ntile = (ell + 15) / 16;
  tq_d4 X[MAXS];
#pragma unroll
  for (int s = 0; s < MAXS; ++s) X[s] = tq_d4{0.0, 0.0, 0.0, 0.0};
  for (int J = 0; J < ntile; ++J) {
    const int j0 = 16 * J, par = J & 1, owner = J % kTqWaves;
    const bool own = wid == owner;
    // loads first (all in flight together): the owner's L_JJ entries and Z_J, every wave's blocks
    // of the rows of L it multiplies (tiles t < J with t % kTqWaves == wid)
    double ldv[4], rdv = 0.0, zv[4];
    if (own) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int e = lane + 64 * u, ra = e >> 4, cb = e & 15;
        ldv[u] = (j0 + ra < ell && cb <= ra) ? L[(int64_t)(j0 + ra) * ell + j0 + cb] : 0.0;
      }
      if (lane < 16 && j0 + lane < ell) rdv = L[(int64_t)(j0 + lane) * ell + j0 + lane];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int c = j0 + 4 * lq + r;
        zv[r] = (row < N && c < ell) ? (double)Z[row * ell + c] : 0.0;
      }
    }
    const bool lrow = j0 + lr < ell;
    const double* Lrow = L + (int64_t)(j0 + lr) * ell + 4 * lq;
    double a[MAXS][4];
#pragma unroll
    for (int s = 0; s < MAXS; ++s) {
      const int t = wid + kTqWaves * s;
      if (t < J) {
#pragma unroll
        for (int r = 0; r < 4; ++r) a[s][r] = lrow ? Lrow[16 * t + r] : 0.0;
      }
    }
    tq_d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < MAXS; ++s) {
      const int t = wid + kTqWaves * s;
      if (t < J) {
#pragma unroll
        for (int r = 0; r < 4; ++r) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s][r], X[s][r], acc, 0, 0, 0);
      }
    }
    if (own) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int e = lane + 64 * u;
        Ld[par][e >> 4][e & 15] = ldv[u];
      }
      if (lane < 16) Rd[par][lane] = rdv != 0.0 ? 1.0 / rdv : 0.0;
    }
    // accumulator element r: S^T(lq + 4 r, lr) = S(row lr, column j0 + lq + 4 r)
#pragma unroll
    for (int r = 0; r < 4; ++r) Sp[par][wid][(lq + 4 * r) * 16 + lr] = acc[r];
    __syncthreads();
    if (own) {
      // b = Z_J - S in the tile layout: lane (lq, lr) holds row lr, columns j0 + 4 lq + r
      double b[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int c = 4 * lq + r;
        double sv = 0.0;
#pragma unroll
        for (int w = 0; w < kTqWaves; ++w) sv += Sp[par][w][c * 16 + lr];
        b[r] = zv[r] - sv;
      }
      // forward substitution over the 16 columns: x_c = b_c / L_cc, then b_c' -= x_c L_c'c
#pragma unroll
      for (int c = 0; c < 16; ++c) {
        double xc = 0.0;
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (4 * lq + r == c) xc = b[r] * Rd[par][c];
        xc = __shfl(xc, lr + 16 * (c >> 2), 64);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int cc = 4 * lq + r;
          if (cc == c) b[r] = xc;
          else if (cc > c) b[r] -= xc * Ld[par][cc][c];
        }
      }
      // keep the tile, write it out
#pragma unroll
      for (int s = 0; s < MAXS; ++s)
        if (owner + kTqWaves * s == J) X[s] = tq_d4{b[0], b[1], b[2], b[3]};
      if (row < N) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int c = j0 + 4 * lq + r;
          if (c < ell) {
            if (Q != nullptr) Q[row * ell + c] = b[r];
            if (Qt != nullptr) Qt[(int64_t)c * ldqt + row] = (TQT)(float)b[r];
          }
        }
      }
    }
  }
}

template <typename TZ, typename TQT>
ngd_status run_trsm_q(const double* L, int ell, const void* Z, int64_t N, double* Q, void* Qt, int64_t ldqt,
                      hipStream_t s) {
  const unsigned grid = (unsigned)((N + 15) / 16);
  const int ntile = (ell + 15) / 16;
  // four waves while each holds at most eight tiles (two workgroups share a CU), eight beyond
#define NGD_TQ(S, W)                                                                                          \
  hipLaunchKernelGGL((trsm_q_kernel<TZ, TQT, S, W>), dim3(grid), dim3(64 * W), 0, s, L, ell, (const TZ*)Z, N, Q, \
                     (TQT*)Qt, ldqt)
  const int s4 = (ntile + 3) / 4, s8 = (ntile + 7) / 8;
  if (s4 <= 2) NGD_TQ(2, 4);
  else if (s4 <= 4) NGD_TQ(4, 4);
  else if (s4 <= 6) NGD_TQ(6, 4);
  else if (s4 <= 8) NGD_TQ(8, 4);
  else if (s8 <= 6) NGD_TQ(6, 8);
  else if (s8 <= 8) NGD_TQ(8, 8);
  else {
    set_error("trsm: ell above 1024");
    return NGD_ERR_INVALID;
  }
#undef NGD_TQ
  NGD_HIP_TRY(hipGetLastError());
  return NGD_OK;
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
                 M + (int64_t)t0 * n + t0, n, NGD_F64, NGD_F64, NGD_F64, G_F64, -1.0, 1.0, nullptr, 0, 2};
      ngd_status st = launch_gemm(g, s);
      if (st != NGD_OK) return st;
    }
  }
  hipLaunchKernelGGL(copy_diag_blocks_kernel, dim3((unsigned)((n + kNb - 1) / kNb)), dim3(256), 0, s, M, n, Lblk);
  NGD_HIP_TRY(hipGetLastError());
  return NGD_OK;
}

// Q = Z L^{-T} for Z (N x ell, ld ell, FP32 or FP64): Q in FP64 (N x ell, ld ell) and / or Q^T
// (ell x ldqt) in `qt_type` (FP32 or BF16); either output may be NULL. ell <= 1024.
ngd_status launch_trsm_q(const double* L, int ell, int z_type, const void* Z, int64_t N, double* Q, int qt_type,
                         void* Qt, int64_t ldqt, hipStream_t s) {
  if (N <= 0 || ell <= 0) return NGD_OK;
  if (Qt == nullptr) qt_type = NGD_F32;
  if (z_type == NGD_F64 && qt_type == NGD_F32) return run_trsm_q<double, float>(L, ell, Z, N, Q, Qt, ldqt, s);
  if (z_type == NGD_F32 && qt_type == NGD_F32) return run_trsm_q<float, float>(L, ell, Z, N, Q, Qt, ldqt, s);
  if (z_type == NGD_F32 && qt_type == NGD_BF16) return run_trsm_q<float, __bf16>(L, ell, Z, N, Q, Qt, ldqt, s);
  if (z_type == NGD_F64 && qt_type == NGD_BF16) return run_trsm_q<double, __bf16>(L, ell, Z, N, Q, Qt, ldqt, s);
  set_error("trsm: unsupported types");
  return NGD_ERR_INVALID;
}

}  // namespace ngd
