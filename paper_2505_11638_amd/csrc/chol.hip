// Shifted Cholesky of the ell x ell core M + nu I = L L^T and the triangular solve Q = Z L^{-T}
// (Alg. 6: C = chol(Omega^T Y_nu), B = Y_nu / C), one launch each, both by 16-row blocks on the
// FP64 matrix cores:
//  * Cholesky: left-looking, one workgroup per row block, row blocks exchanged through flags
//    (chol_rows_kernel).
//  * Triangular solve: 16 rows of Z per workgroup (trsm_q_kernel).
// A pivot that is not safely positive is replaced by a floor (pivot^2 = `floor`), so the
// factorisation never fails; the directions involved are left shrunk in Q (the effect of the
// shift nu in Alg. 6). Their count is reported as a rank deficit.
#include <algorithm>
#include <type_traits>

#include "common.h"

namespace ngd {
namespace {

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
  // the loads of panel J: the owner's L_JJ entries and Z_J, every wave's blocks of the rows of L it
  // multiplies (tiles t < J with t % kTqWaves == wid). Panel J + 1's are issued as soon as panel J's
  // products have consumed theirs, so that their latency overlaps panel J's exchange and substitution:
  // the addresses are clamped into the matrices instead of branching around the edge entries, and the
  // raw values are masked and converted only where they are used.
  double ldv[4], rdv = 0.0, a[MAXS][4];
  TZ zr[4];
  auto load_panel = [&](int J) {
    const int j0 = 16 * J;
    if (wid == J % kTqWaves) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int e = lane + 64 * u;
        ldv[u] = L[(int64_t)min(j0 + (e >> 4), ell - 1) * ell + min(j0 + (e & 15), ell - 1)];
      }
      const int k = min(j0 + lr, ell - 1);
      rdv = L[(int64_t)k * ell + k];
      const int64_t zrow = row < N ? row : N - 1;
#pragma unroll
      for (int r = 0; r < 4; ++r) zr[r] = Z[zrow * ell + min(j0 + 4 * lq + r, ell - 1)];
    }
    const double* Lrow = L + (int64_t)min(j0 + lr, ell - 1) * ell + 4 * lq;
#pragma unroll
    for (int s = 0; s < MAXS; ++s) {
      const int t = wid + kTqWaves * s;
      if (t < J) {
#pragma unroll
        for (int r = 0; r < 4; ++r) a[s][r] = Lrow[16 * t + r];
      }
    }
  };
  load_panel(0);
  for (int J = 0; J < ntile; ++J) {
    const int j0 = 16 * J, par = J & 1, owner = J % kTqWaves;
    const bool own = wid == owner;
    // rows of L past ell (the last panel's) take no part in the products
    const bool lrow = j0 + lr < ell;
    tq_d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < MAXS; ++s) {
      const int t = wid + kTqWaves * s;
      if (t < J) {
#pragma unroll
        for (int r = 0; r < 4; ++r)
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(lrow ? a[s][r] : 0.0, X[s][r], acc, 0, 0, 0);
      }
    }
    double ldc[4], zc[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = lane + 64 * u, ra = e >> 4, cb = e & 15;
      ldc[u] = (j0 + ra < ell && cb <= ra) ? ldv[u] : 0.0;
    }
    const double rdc = (lane < 16 && j0 + lane < ell) ? rdv : 0.0;
#pragma unroll
    for (int r = 0; r < 4; ++r) zc[r] = (row < N && j0 + 4 * lq + r < ell) ? (double)zr[r] : 0.0;
    if (J + 1 < ntile) load_panel(J + 1);
    if (own) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int e = lane + 64 * u;
        Ld[par][e >> 4][e & 15] = ldc[u];
      }
      if (lane < 16) Rd[par][lane] = rdc != 0.0 ? 1.0 / rdc : 0.0;
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
        b[r] = zc[r] - sv;
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
            if (Qt != nullptr) {
              if constexpr (std::is_same<TQT, double>::value) Qt[(int64_t)c * ldqt + row] = b[r];
              else Qt[(int64_t)c * ldqt + row] = (TQT)(float)b[r];
            }
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
  else if (s8 <= 7) NGD_TQ(7, 8);
  else if (s8 <= 8) NGD_TQ(8, 8);
  else {
    set_error("trsm: ell above 1024");
    return NGD_ERR_INVALID;
  }
#undef NGD_TQ
  NGD_HIP_TRY(hipGetLastError());
  return NGD_OK;
}

// ---- Shifted Cholesky in one launch ----
// Left-looking by 16-row blocks: workgroup R owns rows 16R .. 16R+15 and forms, panel by panel,
//   L_RJ = (M_RJ - L_R,<J L_J,<J^T) L_JJ^{-T}   (J < R, as in trsm_q_kernel),
//   L_RR = chol(M_RR - L_R,<R L_R,<R^T)         (the owner wave, in registers),
// storing L over M. Row block J is read only after workgroup J has published it: the workgroup
// stores its rows with device-coherent (sc1) stores, waits for them to complete and then sets a
// flag to this call's epoch, one for L_J,<J (the products with it can start) and one, after the
// diagonal factorisation, for L_JJ; readers poll the flags (one lane per wave) and read the rows
// with device-coherent loads. All ceil(n / 16) workgroups are resident at once (checked), every wait is
// bounded, and workgroup R depends only on lower-numbered ones.
__device__ __forceinline__ void st_co(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ld_co(double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// flags: [0, 64) off-diagonal part of row block R final (A), [64, 128) diagonal block final (B)
constexpr int kCholFlagsB = 64;

__device__ __forceinline__ void wait_flag(unsigned* f, unsigned epoch, int* err) {
  long spins = 0;
  while (__hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != epoch) {
    if (++spins > (1L << 24)) {  // seconds: give up instead of hanging
      __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      break;
    }
  }
}

template <int MAXS, int W>
__global__ __launch_bounds__(64 * W) void chol_rows_kernel(double* __restrict__ M, int n,
                                                           const double* __restrict__ fl, int* __restrict__ nmod,
                                                           unsigned* __restrict__ flags, unsigned epoch,
                                                           int* __restrict__ err) {
  __shared__ double Sp[2][W][256];
  __shared__ double Ld[2][16][17];
  __shared__ double Rd[2][16];
  __shared__ double col[16];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int lr = lane & 15, lq = lane >> 4;
  const int R = blockIdx.x, r0 = 16 * R;
  const int row = r0 + lr;
  const double floor = fl[0], null_thresh = fl[2];
  tq_d4 X[MAXS];
#pragma unroll
  for (int s = 0; s < MAXS; ++s) X[s] = tq_d4{0.0, 0.0, 0.0, 0.0};
  for (int J = 0; J <= R; ++J) {
    const int j0 = 16 * J, par = J & 1, owner = J % W;
    const bool own = wid == owner, diag = J == R;
    // the owner's block of M (row lr, columns j0 + 4 lq + r), independent of the other workgroups
    double zv[4], ldv[4], rdv = 0.0;
    if (own) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int c = j0 + 4 * lq + r;
        zv[r] = (row < n && c < n && c <= row) ? M[(int64_t)row * n + c] : 0.0;
      }
    }
    // when row block J is complete already (flag B, set after flag A), one look at that flag
    // replaces both waits and every load of this step is issued together; otherwise wait for flag A
    // now (the products with L_J,<J overlap the factorisation of L_JJ) and for flag B below
    bool ready = false;
    if (!diag) {
      unsigned fb = 0;
      if (lane == 0) fb = __hip_atomic_load(flags + kCholFlagsB + J, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      ready = __builtin_amdgcn_readfirstlane(fb) == epoch;
      if (!ready && lane == 0) wait_flag(flags + J, epoch, err);  // L_J,<J is final
    }
    // this wave's share of S^T = L_J,<J L_R,<J^T over the tiles t < J held here (t % W == wid); the
    // rows of L_J come from workgroup J, or are this workgroup's own tiles when J == R
    // (all loads issued before the first product, so that their latencies overlap)
    auto load_ljj = [&] {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int e = lane + 64 * u, ra = e >> 4, cb = e & 15;
        ldv[u] = (j0 + ra < n && cb <= ra) ? ld_co(M + (int64_t)(j0 + ra) * n + j0 + cb) : 0.0;
      }
      if (lane < 16 && j0 + lane < n) rdv = ld_co(M + (int64_t)(j0 + lane) * n + j0 + lane);
    };
    if (own && !diag && ready) load_ljj();
    tq_d4 acc = {0.0, 0.0, 0.0, 0.0};
    const bool lrow = j0 + lr < n;
    double* Lrow = M + (int64_t)(j0 + lr) * n + 4 * lq;
    double a[MAXS][4];
    if (!diag) {
#pragma unroll
      for (int s = 0; s < MAXS; ++s) {
        const int t = wid + W * s;
        if (t < J && lrow) {
#pragma unroll
          for (int r = 0; r < 4; ++r) a[s][r] = ld_co(Lrow + 16 * t + r);
        }
      }
    }
#pragma unroll
    for (int s = 0; s < MAXS; ++s) {
      const int t = wid + W * s;
      if (t < J) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const double av = diag ? X[s][r] : (lrow ? a[s][r] : 0.0);
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, X[s][r], acc, 0, 0, 0);
        }
      }
    }
    if (own && !diag) {
      if (!ready) {
        if (lane == 0) wait_flag(flags + kCholFlagsB + J, epoch, err);  // L_JJ is final
        load_ljj();
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int e = lane + 64 * u;
        Ld[par][e >> 4][e & 15] = ldv[u];
      }
      if (lane < 16) Rd[par][lane] = rdv != 0.0 ? 1.0 / rdv : 0.0;
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) Sp[par][wid][(lq + 4 * r) * 16 + lr] = acc[r];
    __syncthreads();
    if (diag) {
      // every wave's stores of L_R,<R complete, then flag A: the later row blocks can form their
      // products with L_R,<R while the owner factors L_RR
      __builtin_amdgcn_s_waitcnt(0);
      __atomic_signal_fence(__ATOMIC_SEQ_CST);
      __syncthreads();
      if (threadIdx.x == 0) __hip_atomic_store(flags + R, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (!own) break;
    } else if (!own) {
      continue;
    }
    double b[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int c = 4 * lq + r;
      double sv = 0.0;
#pragma unroll
      for (int w = 0; w < W; ++w) sv += Sp[par][w][c * 16 + lr];
      b[r] = zv[r] - sv;
    }
    if (!diag) {
      // L_RJ = b L_JJ^{-T} by forward substitution over the 16 columns
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
#pragma unroll
      for (int s = 0; s < MAXS; ++s)
        if (owner + W * s == J) X[s] = tq_d4{b[0], b[1], b[2], b[3]};
      if (row < n) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int c = j0 + 4 * lq + r;
          if (c < n) st_co(M + (int64_t)row * n + c, b[r]);
        }
      }
    } else {
      // L_RR = chol(b): column by column, the pivot from its lane, the column published through LDS
      int nulls = 0;
#pragma unroll
      for (int c = 0; c < 16; ++c) {
        if (j0 + c < n) {
          const int src = c + 16 * (c >> 2);
          double piv = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(b[c & 3]), src),
                                        __builtin_amdgcn_readlane(__double2loint(b[c & 3]), src));
          if (!(piv > null_thresh)) ++nulls;  // direction at the level of the shift: numerically null
          if (!(piv > floor)) piv = floor;
          // 1 / sqrt(piv) from the hardware estimate and two Newton steps; sqrt(piv) = piv / sqrt(piv)
          double rd = __builtin_amdgcn_rsq(piv);
          rd = rd * fma(-0.5 * piv * rd, rd, 1.5);
          rd = rd * fma(-0.5 * piv * rd, rd, 1.5);
          const double d = piv * rd;
          if (lq == (c >> 2)) {
            if (lr == c) b[c & 3] = d;
            else if (lr > c) b[c & 3] *= rd;
            col[lr] = lr > c ? b[c & 3] : 0.0;
          }
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
          const double l_r = col[lr];
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int q = 4 * lq + r;
            if (q > c && q <= lr) b[r] -= l_r * col[q];
          }
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
      }
      if (row < n) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int c = j0 + 4 * lq + r;
          if (c < n) st_co(M + (int64_t)row * n + c, c <= row ? b[r] : 0.0);
        }
      }
      if (lane == 0 && nulls) atomicAdd(nmod, nulls);
      __builtin_amdgcn_s_waitcnt(0);
      __atomic_signal_fence(__ATOMIC_SEQ_CST);
      if (lane == 0) __hip_atomic_store(flags + kCholFlagsB + R, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
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

// L (lower, in place of M; the upper part of the diagonal blocks zeroed) with L L^T = M + nu I,
// nu = shift_rel tr(M). `scal` holds 3 doubles (floor, nu, null threshold) and `nmod` the count of
// null pivots (both device). `sync` is the device word block of the launch (two sets of 64 flags and
// the error word at index 128), `epoch` a value that differs from every earlier call's.
ngd_status launch_shifted_cholesky(double* M, int n, double shift_rel, double floor_rel, double* scal, int* nmod,
                                   unsigned* sync, unsigned epoch, hipStream_t s) {
  if (n <= 0) return NGD_OK;
  if (n > kMaxEll) {
    set_error("cholesky: n above 1024");
    return NGD_ERR_INVALID;
  }
  hipLaunchKernelGGL(shift_kernel, dim3(1), dim3(256), 0, s, M, n, shift_rel, floor_rel, scal, nmod);
  NGD_HIP_TRY(hipGetLastError());
  const int ntile = (n + 15) / 16;
  int* err = reinterpret_cast<int*>(sync + 2 * kCholFlagsB);
  int dev = 0, cus = 0;
  NGD_HIP_TRY(hipGetDevice(&dev));
  NGD_HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  if (ntile > cus) {
    set_error("cholesky grid cannot be co-resident");
    return NGD_ERR_HIP;
  }
#define NGD_CH(S, W)                                                                                        \
  hipLaunchKernelGGL((chol_rows_kernel<S, W>), dim3(ntile), dim3(64 * W), 0, s, M, n, (const double*)scal, nmod, \
                     sync, epoch, err)
  // eight waves beyond eight row blocks: fewer tiles per wave leaves registers for the loads
  const int s4 = (ntile + 3) / 4, s8 = (ntile + 7) / 8;
  if (s4 <= 2) NGD_CH(2, 4);
  else if (s8 <= 2) NGD_CH(2, 8);
  else if (s8 <= 4) NGD_CH(4, 8);
  else if (s8 <= 6) NGD_CH(6, 8);
  else NGD_CH(8, 8);
#undef NGD_CH
  NGD_HIP_TRY(hipGetLastError());
  return NGD_OK;
}

// Q = Z L^{-T} for Z (N x ell, ld ell, FP32 or FP64): Q in FP64 (N x ell, ld ell) and / or Q^T
// (ell x ldqt) in `qt_type` (FP32 or BF16; FP64 for FP64 Z); either output may be NULL. ell <= 1024.
ngd_status launch_trsm_q(const double* L, int ell, int z_type, const void* Z, int64_t N, double* Q, int qt_type,
                         void* Qt, int64_t ldqt, hipStream_t s) {
  if (N <= 0 || ell <= 0) return NGD_OK;
  if (Qt == nullptr) qt_type = NGD_F32;
  if (z_type == NGD_F64 && qt_type == NGD_F32) return run_trsm_q<double, float>(L, ell, Z, N, Q, Qt, ldqt, s);
  if (z_type == NGD_F32 && qt_type == NGD_F32) return run_trsm_q<float, float>(L, ell, Z, N, Q, Qt, ldqt, s);
  if (z_type == NGD_F32 && qt_type == NGD_BF16) return run_trsm_q<float, __bf16>(L, ell, Z, N, Q, Qt, ldqt, s);
  if (z_type == NGD_F64 && qt_type == NGD_BF16) return run_trsm_q<double, __bf16>(L, ell, Z, N, Q, Qt, ldqt, s);
  if (z_type == NGD_F64 && qt_type == NGD_F64) return run_trsm_q<double, double>(L, ell, Z, N, Q, Qt, ldqt, s);
  set_error("trsm: unsupported types");
  return NGD_ERR_INVALID;
}

}  // namespace ngd
