// FP64 symmetric eigendecomposition of the small ell x ell matrices of the Nystrom core.
//
// Alg. 6 needs the thin SVD of the p x ell matrix B; its right singular vectors and squared
// singular values are the eigenpairs of the ell x ell Gram matrix B^T B, computed here in FP64:
//  1. Householder tridiagonalisation Q^T A Q = T in one launch whose workgroups meet at a grid
//     barrier once per column. The trailing matrix is row-distributed over the workgroups and kept
//     in registers; each step applies the previous step's rank-2 update lazily while forming
//     p = tau A v.
//  2. Eigenvalues of T by multisection on Sturm counts (one wave per eigenvalue).
//  3. Eigenvectors of T by inverse iteration with partial-pivoting LU of T - lambda I (one wave
//     per eigenvector, the factors in its registers), modified Gram-Schmidt inside clusters of
//     (nearly) equal eigenvalues, and two Newton-Schulz steps that restore orthonormality to
//     working precision.
//  4. Back-transformation V = Q Z. Q = H_0 H_1 ... H_{n-3} is formed explicitly from the compact
//     WY blocks on the FP64 matrix cores (one workgroup per 16 columns) as soon as step 1 is done,
//     on a second stream where one is given, so that it runs beside steps 2 and 3; V is then a
//     single FP64 product.
// n <= 1024.
// Eigenpairs whose eigenvalue is below drop_rel * (Gershgorin bound of T) are returned as
// (0, zero vector).
#include <algorithm>
#include <vector>

#include "common.h"

namespace ngd {
namespace {

struct TriArgs {
  double* A0;      // input matrix (n x n, ld n), read once
  double* PV;      // 2 n: the next pivot row, double-buffered by the parity of its index
  int n;
  double* d;       // diagonal of T
  double* e;       // off-diagonal of T (n-1)
  double* V;       // Householder vectors, row k = v_k (support k+1..n-1, v_k[k+1] = 1)
  double* tau;     // Householder scalars
  double* P;       // 2 n: p = tau A v of the current step, double-buffered by step parity
  unsigned* flags; // one barrier flag per workgroup, zero at launch
  int* err;
};

// ---- register-resident tridiagonalisation (n <= kTrMaxN) ----
// The Householder recurrence with the trailing matrix in registers: 8 or 16 waves per workgroup,
// each owning two or three of the workgroup's rows, lane l holding columns l, l + 64, ... Per
// column k:
//  (A) wave 0 forms the Householder vector v_k from the pivot row (with the pending rank-2 update of
//      step k-1 applied) while every wave applies that pending update to its rows;
//  (C) each row's p_i = tau_k row_i . v_k, and the owner of row k+1 publishes that row;
//  (D) one grid barrier;
//  (E) p_k and the next pivot row are read into LDS;
//  (F) every wave forms c_k = (tau_k / 2) p_k . v_k and the new pending update w_k = p_k - c_k v_k at
//      its own columns, in registers.
// All reductions are within a wave (DPP), so a step has two workgroup barriers besides the grid
// barrier. The exchanged vectors are written and read with device-coherent (sc1) accesses, so the
// grid barrier needs no cache write-back or invalidate: each thread waits for its own stores to
// complete before the workgroup publishes its flag.
// waves per workgroup and rows per wave: 16 x 2 up to 7 columns per lane, 8 x 2 up to 13 and 8 x 3
// beyond (where more rows would not fit in registers with 16 columns per lane); these measured
// fastest among the shapes that keep the workgroup count at or below 64
constexpr int tr_waves(int qn) { return qn <= 7 ? 16 : 8; }
constexpr int tr_rows(int qn) { return qn <= 13 ? 2 : 3; }
constexpr int kTrMaxN = 1024;

__device__ __forceinline__ void st_coherent(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ld_coherent(double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Barrier number `epoch` among the G workgroups of one matrix (this one is number gme) for data
// exchanged only through st_coherent / ld_coherent. The flags of up to 64 workgroups are polled by
// wave 0 (one per lane). The wait is bounded; on timeout the error word is raised and false is
// returned to the whole workgroup.
__device__ bool grid_sync_coherent(unsigned* flags, unsigned epoch, int* err, int* timed_out, int gme, int G) {
  __builtin_amdgcn_s_waitcnt(0);
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __syncthreads();
  if (threadIdx.x < 64) {
    const unsigned target = epoch + 1u;
    if (threadIdx.x == 0) __hip_atomic_store(flags + gme, target, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    long spins = 0;
    while (true) {
      const int g = threadIdx.x;
      const bool ok = g >= G || __hip_atomic_load(flags + g, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= target;
      if (__all(ok)) break;
      if (++spins > (1L << 24)) {  // seconds: give up instead of hanging
        if (threadIdx.x == 0) {
          __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          *timed_out = 1;
        }
        break;
      }
    }
  }
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __syncthreads();
  return *timed_out == 0;
}

// entry j of a vector held as x[q] at column lane + 64 q (j wave-uniform): select the register,
// then read it from lane j % 64
__device__ __forceinline__ double read_lane(double t, int l) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(t), l),
                          __builtin_amdgcn_readlane(__double2loint(t), l));
}
#define NGD_LANE_VALUE(out, x, QN, j)                  \
  do {                                                 \
    const int q_ = (j) >> 6;                           \
    double t_ = (x)[0];                                \
    _Pragma("unroll") for (int u_ = 1; u_ < (QN); ++u_) \
      if (q_ == u_) t_ = (x)[u_];                      \
    (out) = read_lane(t_, (j) & 63);                   \
  } while (0)

// The tridiagonalisation of one matrix by workgroup g of its G workgroups.
template <int QN, int kTrRows, int kTrWaves>
__device__ __forceinline__ void tridiag_body(const TriArgs& a, const int g, const int G) {
  constexpr int kTrThreads = 64 * kTrWaves;
  constexpr int kTrCols = kTrMaxN / kTrThreads;  // per-column LDS entries per thread
  __shared__ double vbuf[2][kTrMaxN];  // v of this step and of the previous one (by parity)
  __shared__ double pbuf[kTrMaxN];     // p of the previous step
  __shared__ double pivl[kTrMaxN];     // the pivot row (before the pending update)
  __shared__ double tau_s;
  __shared__ int timed_out;
  const int n = a.n;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (threadIdx.x == 0) timed_out = 0;
  double rows[kTrRows][QN];
#pragma unroll
  for (int s = 0; s < kTrRows; ++s) {
    const int i = g + G * (wid + kTrWaves * s);
#pragma unroll
    for (int q = 0; q < QN; ++q) {
      const int c = lane + 64 * q;
      rows[s][q] = (i < n && c < n) ? a.A0[(int64_t)i * n + c] : 0.0;
    }
  }
  // the pending rank-2 update (v, w) at this lane's columns; c of the step that made it
  double vq[QN], wq[QN];
#pragma unroll
  for (int q = 0; q < QN; ++q) vq[q] = wq[q] = 0.0;
  double cprev = 0.0;
#pragma unroll
  for (int t = 0; t < kTrCols; ++t) {
    const int j = threadIdx.x + kTrThreads * t;
    pivl[j] = j < n ? a.A0[j] : 0.0;  // row 0, nothing pending
    vbuf[0][j] = 0.0;
    vbuf[1][j] = 0.0;
    pbuf[j] = 0.0;
  }
  __syncthreads();
  for (int k = 0; k + 2 < n; ++k) {
    double* vnew = vbuf[k & 1];
    const double* vold = vbuf[(k & 1) ^ 1];
    // (A) wave 0: v_k from column k of A^(k) = the pivot row with the pending update applied
    if (wid == 0) {
      const double vk = vold[k];
      double wk;
      NGD_LANE_VALUE(wk, wq, QN, k);
      double x[QN], tail = 0.0;
#pragma unroll
      for (int q = 0; q < QN; ++q) {  // unconditional LDS reads, so that they issue together
        const int c = lane + 64 * q;
        const double pl = pivl[c];
        x[q] = (c > k && c < n) ? pl - vk * wq[q] - wk * vq[q] : 0.0;
        if (c > k + 1) tail += x[q] * x[q];
      }
      tail = wave_sum_dpp(tail);
      double alpha;
      NGD_LANE_VALUE(alpha, x, QN, k + 1);
      double tau, beta, scale;
      if (tail == 0.0) {
        tau = 0.0;
        beta = alpha;
        scale = 0.0;
      } else {
        const double nrm = sqrt(alpha * alpha + tail);
        beta = alpha >= 0.0 ? -nrm : nrm;
        tau = (beta - alpha) / beta;
        scale = 1.0 / (alpha - beta);
      }
#pragma unroll
      for (int q = 0; q < QN; ++q) {
        const int c = lane + 64 * q;
        const double v = c == k + 1 ? 1.0 : (c > k + 1 ? x[q] * scale : 0.0);
        vnew[c] = v;
      }
      if (lane == 0) {
        tau_s = tau;
        if (g == 0) {
          a.d[k] = pivl[k] - 2.0 * vk * wk;
          a.e[k] = beta;
          a.tau[k] = tau;
        }
      }
    }
    // (A) every wave: the pending update of its live rows, A_ic -= v_i w_c + w_i v_c
#pragma unroll
    for (int s = 0; s < kTrRows; ++s) {
      const int i = g + G * (wid + kTrWaves * s);
      if (i <= k || i >= n) continue;
      const double vi = vold[i], wi = pbuf[i] - cprev * vi;
#pragma unroll
      for (int q = 0; q < QN; ++q) rows[s][q] -= vi * wq[q] + wi * vq[q];
    }
    __syncthreads();
    // (C) p_i = tau_k row_i . v_k; the owner of row k+1 publishes it
    const double tk = tau_s;
    double* pk = a.P + (int64_t)(k & 1) * n;
    double* nextp = a.PV + (int64_t)((k + 1) & 1) * n;
    double acc[kTrRows];
#pragma unroll
    for (int s = 0; s < kTrRows; ++s) acc[s] = 0.0;
#pragma unroll
    for (int q = 0; q < QN; ++q) {
      const double u = vnew[lane + 64 * q];
#pragma unroll
      for (int s = 0; s < kTrRows; ++s) acc[s] += rows[s][q] * u;
    }
#pragma unroll
    for (int s = 0; s < kTrRows; ++s) acc[s] = wave_sum_dpp(acc[s]);
#pragma unroll
    for (int s = 0; s < kTrRows; ++s) {
      const int i = g + G * (wid + kTrWaves * s);
      if (i <= k || i >= n) continue;
      if (lane == 0) st_coherent(pk + i, tk * acc[s]);
      if (i == k + 1) {
#pragma unroll
        for (int q = 0; q < QN; ++q) {
          const int c = lane + 64 * q;
          if (c > k && c < n) st_coherent(nextp + c, rows[s][q]);
        }
      }
    }
    // (D)
    if (!grid_sync_coherent(a.flags, (unsigned)k, a.err, &timed_out, g, G)) return;
    // (E) p_k and pivot row k+1
    double pl[kTrCols], nl[kTrCols];
#pragma unroll
    for (int t = 0; t < kTrCols; ++t) {  // unconditional (clamped) loads, so that they issue together
      const int jc = min((int)threadIdx.x + kTrThreads * t, n - 1);
      pl[t] = ld_coherent(pk + jc);
      nl[t] = ld_coherent(nextp + jc);
    }
#pragma unroll
    for (int t = 0; t < kTrCols; ++t) {
      const int j = threadIdx.x + kTrThreads * t;
      const bool live = j > k && j < n;
      pbuf[j] = live ? pl[t] : 0.0;
      pivl[j] = live ? nl[t] : 0.0;
    }
    __syncthreads();
    // (F) c_k and the new pending update at this lane's columns (every wave)
    double pv = 0.0;
#pragma unroll
    for (int q = 0; q < QN; ++q) {
      const int c = lane + 64 * q;
      pv += pbuf[c] * vnew[c];
    }
    const double ck = 0.5 * tk * wave_sum_dpp(pv);
    // v_k to V, off the path to the next barrier (only later kernels read V)
    if (g == 0 && wid == 0) {
#pragma unroll
      for (int q = 0; q < QN; ++q) {
        const int c = lane + 64 * q;
        if (c < n) a.V[(int64_t)k * n + c] = vnew[c];
      }
    }
#pragma unroll
    for (int q = 0; q < QN; ++q) {
      const int c = lane + 64 * q;
      vq[q] = vnew[c];
      wq[q] = pbuf[c] - ck * vq[q];
    }
    cprev = ck;
  }
  // the last 2 x 2 (or 1 x 1) block: pivot row n-2 and row n-1 with the pending update
  const int m = n >= 2 ? n - 2 : 0;
  if (n == 1) {
    if (g == 0 && threadIdx.x == 0) a.d[0] = pivl[0];
    return;
  }
  double vm, wm, vm1, wm1;
  NGD_LANE_VALUE(vm, vq, QN, m);
  NGD_LANE_VALUE(wm, wq, QN, m);
  NGD_LANE_VALUE(vm1, vq, QN, m + 1);
  NGD_LANE_VALUE(wm1, wq, QN, m + 1);
  if (g == 0 && threadIdx.x == 0) {
    a.d[m] = pivl[m] - 2.0 * vm * wm;
    a.e[m] = pivl[m + 1] - vm * wm1 - wm * vm1;
  }
#pragma unroll
  for (int s = 0; s < kTrRows; ++s) {
    const int i = g + G * (wid + kTrWaves * s);
    if (i != m + 1) continue;
#pragma unroll
    for (int q = 0; q < QN; ++q)
      if (lane + 64 * q == m + 1) a.d[m + 1] = rows[s][q] - 2.0 * vm1 * wm1;
  }
}

template <int QN, int kTrRows, int kTrWaves>
__global__ __launch_bounds__(64 * kTrWaves) void tridiag_reg_kernel(TriArgs a) {
  tridiag_body<QN, kTrRows, kTrWaves>(a, (int)blockIdx.x, (int)gridDim.x);
}

// Several matrices of one register shape in one launch: matrix m has workgroups first[m] ..
// first[m + 1] - 1, which meet only among themselves. The arguments travel by value.
constexpr int kTriBatchMax = 24;
struct TriBatch {
  TriArgs a[kTriBatchMax];
  int first[kTriBatchMax + 1];
  int n;
};

template <int QN, int kTrRows, int kTrWaves>
__global__ __launch_bounds__(64 * kTrWaves) void tridiag_batch_kernel(TriBatch tb) {
  int m = 0;
  while (m + 1 < tb.n && (int)blockIdx.x >= tb.first[m + 1]) ++m;
  tridiag_body<QN, kTrRows, kTrWaves>(tb.a[m], (int)blockIdx.x - tb.first[m], tb.first[m + 1] - tb.first[m]);
}

// Number of eigenvalues of T below x (Sturm sequence of the LDL^T pivots of T - x I). The pivot
// recurrence divides by the previous pivot through a reciprocal refined by one Newton step (within
// an ulp or two of the quotient: the count is then that of a T perturbed at roundoff level, which
// is all bisection needs).
__device__ int sturm_count(const double* d, const double* e2, int n, double x, double pivmin) {
  int cnt = 0;
  double q = d[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  if (q < 0) ++cnt;
  for (int i = 1; i < n; ++i) {
    double r = __builtin_amdgcn_rcp(q);
    r = fma(r, fma(-q, r, 1.0), r);
    q = (d[i] - x) - e2[i - 1] * r;
    if (fabs(q) < pivmin) q = -pivmin;
    if (q < 0) ++cnt;
  }
  return cnt;
}

// eigenvalue index i (ascending) of T by multisection on Sturm counts; also prepares e^2
// wpe (1 or 2) waves per eigenvalue, 4 / wpe eigenvalues per 256-thread workgroup: their 64 wpe lanes
// evaluate 64 wpe interior points of the current interval and the first point whose count exceeds i
// bounds eigenvalue i from above, so each round shrinks the interval (64 wpe + 1)-fold. Two waves per
// eigenvalue pay off while they still find a SIMD of their own. Every eigenvalue starts from the same
// Gershgorin interval and every round divides its width by the same factor, so the number of rounds
// is the same for all of them and is fixed up front (workgroup barriers stay uniform).
__device__ __forceinline__ void bisect_body(const double* __restrict__ d, const double* __restrict__ e, int n,
                                            int wpe, double* __restrict__ e2, double* __restrict__ lam_asc,
                                            double* __restrict__ tnorm, const int bid) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* sd = reinterpret_cast<double*>(smem_raw);
  double* se2 = sd + n;
  __shared__ double red_lo[4], red_hi[4];
  __shared__ unsigned long long mask[2][4];
  // the tridiagonal in LDS, and the Gershgorin interval by a workgroup reduction
  double glo = 1e300, ghi = -1e300;
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    const double dj = d[j];
    const double ej = j < n - 1 ? e[j] : 0.0;
    sd[j] = dj;
    if (j < n - 1) {
      se2[j] = ej * ej;
      if (bid == 0) e2[j] = ej * ej;
    }
    const double r = (j > 0 ? fabs(e[j - 1]) : 0.0) + fabs(ej);
    glo = fmin(glo, dj - r);
    ghi = fmax(ghi, dj + r);
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    glo = fmin(glo, __shfl_xor(glo, o, 64));
    ghi = fmax(ghi, __shfl_xor(ghi, o, 64));
  }
  if (lane == 0) {
    red_lo[wid] = glo;
    red_hi[wid] = ghi;
  }
  __syncthreads();
  glo = fmin(fmin(red_lo[0], red_lo[1]), fmin(red_lo[2], red_lo[3]));
  ghi = fmax(fmax(red_hi[0], red_hi[1]), fmax(red_hi[2], red_hi[3]));
  const double tn = fmax(fabs(glo), fabs(ghi));
  if (bid == 0 && threadIdx.x == 0) *tnorm = tn;
  const double pivmin = fmax(1e-300, 2.2250738585072014e-308 * fmax(1.0, tn * tn));
  double lo = glo - 1e-14 * tn - pivmin, hi = ghi + 1e-14 * tn + pivmin;
  const double tol = 4.0 * 2.220446049250313e-16 * tn + pivmin;
  // rounds until the width (hi - lo) / (64 wpe + 1)^r is at most tol (at most 16)
  const double div = 64.0 * wpe + 1.0;
  int rounds = 0;
  for (double w = hi - lo; w > tol && rounds < 16; w /= div) ++rounds;
  const int pair = wid / wpe, half = wid - pair * wpe;
  const int i = bid * (4 / wpe) + pair;
  const int ic = i < n ? i : n - 1;  // waves past the end follow a valid eigenvalue and store nothing
  for (int it = 0; it < rounds; ++it) {
    const double h = (hi - lo) / div;
    const double x = lo + h * (64 * half + lane + 1);
    const bool above = sturm_count(sd, se2, n, x, pivmin) > ic;
    const unsigned long long m = __ballot(above);
    if (lane == 0) mask[it & 1][wid] = m;
    __syncthreads();
    const unsigned long long m0 = mask[it & 1][wpe * pair];
    const unsigned long long m1 = wpe == 2 ? mask[it & 1][wpe * pair + 1] : 0ull;
    if (m0 == 0ull && m1 == 0ull) {
      lo = lo + h * (64.0 * wpe);
    } else {
      const int first = m0 != 0ull ? __ffsll((long long)m0) - 1 : 64 + __ffsll((long long)m1) - 1;
      const double nhi = lo + h * (first + 1);
      lo = first == 0 ? lo : lo + h * first;
      hi = nhi;
    }
  }
  if (i < n && half == 0 && lane == 0) lam_asc[i] = 0.5 * (lo + hi);
}

__global__ __launch_bounds__(256) void bisect_kernel(const double* __restrict__ d, const double* __restrict__ e,
                                                     int n, int wpe, double* __restrict__ e2,
                                                     double* __restrict__ lam_asc, double* __restrict__ tnorm) {
  bisect_body(d, e, n, wpe, e2, lam_asc, tnorm, (int)blockIdx.x);
}

// inverse iteration for eigenvalue i: solve (T - lam I) x = b by LU with partial pivoting
// (tridiagonal; the U factor has two superdiagonals), two sweeps. One wave per eigenvalue: the
// recurrences run on wave-uniform values, and T's diagonals and the LU factors stay in registers
// spread over the lanes (entry j in register j / 64 of lane j % 64), so a step reads its operands
// with readlane and writes its results into lane j % 64 with a select; nothing goes through
// memory. T's inputs are held shifted by one entry as well (d_{j+1}, e_{j+1}) since step j needs
// them. kInvWaves eigenvalues per workgroup; their eigenvectors leave through LDS so that each row
// of Z is written in one run. Quotients are a hardware reciprocal refined by one Newton step.
constexpr int kInvWaves = 4;
// register shapes ceil(n / 64) of the inverse iteration (n <= 1024)
#define NGD_INVIT_SHAPES(X) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16)

__device__ __forceinline__ double recip(double x) {
  double r = __builtin_amdgcn_rcp(x);
  return fma(r, fma(-x, r, 1.0), r);
}

// x[j / 64] at lane j % 64 <- v (j wave-uniform, possibly a run-time value)
__device__ __forceinline__ float read_lane_f(float t, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(t), l));
}

#define NGD_SET_ENTRY(x, QN, j, v)                                   \
  do {                                                               \
    const int qs_ = (j) >> 6, ls_ = (j) & 63;                        \
    _Pragma("unroll") for (int u_ = 0; u_ < (QN); ++u_)              \
      if (u_ == qs_) (x)[u_] = lane == ls_ ? (v) : (x)[u_];          \
  } while (0)

template <int QN>
__device__ __forceinline__ void invit_body(const double* __restrict__ d, const double* __restrict__ e, int n,
                                           const double* __restrict__ lam_asc, const double* __restrict__ tnorm,
                                           double drop_rel, double* __restrict__ Z, const int bid) {
  __shared__ double zs[64 * QN][kInvWaves];
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int i = bid * kInvWaves + w;
  double yr[QN];
#pragma unroll
  for (int q = 0; q < QN; ++q) yr[q] = 0.0;
  if (i < n && !(lam_asc[i] < drop_rel * (*tnorm))) {  // below the drop threshold: a zero vector
    const double lam = lam_asc[i];
    const double tiny = 2.220446049250313e-16 * fmax(*tnorm, 1e-300);
    const double inv_tiny = recip(tiny);
    // e_j, d_{j+1}, e_{j+1} (zero past the ends), the factors: multiplier, first superdiagonal of U,
    // 1 / pivot, interchange flag (the second superdiagonal is e_{j+1} where rows were swapped)
    double er[QN], ds[QN], es[QN], ml[QN], u1[QN], ri[QN];
    float sw[QN];
#pragma unroll
    for (int q = 0; q < QN; ++q) {
      const int j = 64 * q + lane;
      er[q] = j < n - 1 ? e[j] : 0.0;
      ds[q] = j + 1 < n ? d[j + 1] : 0.0;
      es[q] = j + 1 < n - 1 ? e[j + 1] : 0.0;
      ml[q] = u1[q] = ri[q] = 0.0;
      sw[q] = 0.f;
    }
    // factorisation of T - lam I fused with the first forward sweep (start vector: deterministic
    // pseudo-random entries in [0.5, 1.5))
    unsigned h = 2166136261u ^ ((unsigned)i * 16777619u);
    h = (h ^ 0u) * 16777619u + 0x9E3779B9u;
    double carry = 0.5 + (double)(h >> 8) * (1.0 / 16777216.0);
    double a = d[0] - lam, b = n > 1 ? e[0] : 0.0;
#pragma unroll
    for (int q = 0; q < QN; ++q) {
      const int lend = min(64, n - 1 - 64 * q);
      for (int l = 0; l < lend; ++l) {
        const int j = 64 * q + l;
        const bool me = lane == l;
        const double c = read_lane(er[q], l), dn = read_lane(ds[q], l) - lam, en = read_lane(es[q], l);
        h = (h ^ (unsigned)(j + 1)) * 16777619u + 0x9E3779B9u;
        const double nxt = 0.5 + (double)(h >> 8) * (1.0 / 16777216.0);
        // partial pivoting between rows j (a, b) and j + 1 (c, dn, en) with one reciprocal: the
        // pivot's serves the multiplier and, unless the pivot is below `tiny` (then replaced by
        // +-tiny), the stored 1/pivot
        const bool swp = !(fabs(a) >= fabs(c));
        const double piv = swp ? c : a, oth = swp ? a : c;
        const double rp = recip(piv);
        const double m = piv != 0.0 ? oth * rp : 0.0;
        u1[q] = me ? (swp ? dn : b) : u1[q];
        sw[q] = me ? (swp ? 1.f : 0.f) : sw[q];
        const double an = (swp ? b : dn) - m * (swp ? dn : b);
        b = swp ? -m * en : en;
        a = an;
        const double x0 = swp ? nxt : carry, x1 = swp ? carry : nxt;
        ml[q] = me ? m : ml[q];
        ri[q] = me ? (fabs(piv) < tiny ? (piv < 0.0 ? -inv_tiny : inv_tiny) : rp) : ri[q];
        yr[q] = me ? x0 : yr[q];
        carry = x1 - m * x0;
      }
    }
    if (fabs(a) < tiny) a = a < 0.0 ? -tiny : tiny;
    NGD_SET_ENTRY(ri, QN, n - 1, recip(a));
    NGD_SET_ENTRY(u1, QN, n - 1, 0.0);
    NGD_SET_ENTRY(sw, QN, n - 1, 0.f);
    NGD_SET_ENTRY(yr, QN, n - 1, carry);
    double scale = 1.0, ss = 0.0;
    for (int it = 0; it < 2; ++it) {
      if (it == 1) {
        // forward sweep with the stored interchanges and multipliers on the scaled previous solution
        carry = read_lane(yr[0], 0) * scale;
#pragma unroll
        for (int q = 0; q < QN; ++q) {
          const int lend = min(64, n - 1 - 64 * q);
          for (int l = 0; l < lend; ++l) {
            const int l1 = (l + 1) & 63;
            // y_{j+1}: lane j + 1 of the same register, or lane 0 of the next (the last register
            // never holds step 63, since its steps end before n - 1)
            const double ya = read_lane(yr[q], l1), yb = read_lane(yr[q + 1 < QN ? q + 1 : q], l1);
            const double nxt = (l < 63 ? ya : yb) * scale;
            const bool swp = read_lane_f(sw[q], l) != 0.f;
            const double x0 = swp ? nxt : carry, x1 = swp ? carry : nxt;
            yr[q] = lane == l ? x0 : yr[q];
            carry = x1 - read_lane(ml[q], l) * x0;
          }
        }
        NGD_SET_ENTRY(yr, QN, n - 1, carry);
      }
      // backward substitution with U, in place on y; the max-norm for scaling (and, on the last
      // sweep, the sum of squares for the final normalisation)
      double x1 = 0.0, x2 = 0.0, nrm = 0.0;
      ss = 0.0;
#pragma unroll
      for (int q = QN - 1; q >= 0; --q) {
        for (int l = min(63, n - 1 - 64 * q); l >= 0; --l) {
          const double u2 = read_lane_f(sw[q], l) != 0.f ? read_lane(es[q], l) : 0.0;
          const double x = (read_lane(yr[q], l) - read_lane(u1[q], l) * x1 - u2 * x2) * read_lane(ri[q], l);
          yr[q] = lane == l ? x : yr[q];
          x2 = x1;
          x1 = x;
          nrm = fmax(nrm, fabs(x));
          ss += x * x;
        }
      }
      scale = nrm > 0.0 ? 1.0 / nrm : 0.0;
    }
    // unit 2-norm: ss is the sum of squares of the unscaled last solution
    const double s2 = ss > 0.0 ? 1.0 / sqrt(ss) : 0.0;
#pragma unroll
    for (int q = 0; q < QN; ++q) yr[q] *= s2;
  }
#pragma unroll
  for (int q = 0; q < QN; ++q)
    if (64 * q + lane < n) zs[64 * q + lane][w] = yr[q];
  __syncthreads();
  const int i0 = bid * kInvWaves, ni = min(kInvWaves, n - i0);
  for (int t = threadIdx.x; t < n * kInvWaves; t += blockDim.x) {
    const int j = t / kInvWaves, c = t % kInvWaves;
    if (c < ni) Z[(int64_t)j * n + i0 + c] = zs[j][c];
  }
}
#undef NGD_SET_ENTRY

template <int QN>
__global__ __launch_bounds__(64 * kInvWaves) void invit_kernel(const double* __restrict__ d,
                                                               const double* __restrict__ e, int n,
                                                               const double* __restrict__ lam_asc,
                                                               const double* __restrict__ tnorm, double drop_rel,
                                                               double* __restrict__ Z) {
  invit_body<QN>(d, e, n, lam_asc, tnorm, drop_rel, Z, (int)blockIdx.x);
}

// modified Gram-Schmidt within each cluster of close eigenvalues (one workgroup per cluster start)
__device__ __forceinline__ void cluster_mgs_body(const double* __restrict__ lam_asc, int n,
                                                 const double* __restrict__ tnorm, double drop_rel,
                                                 double* __restrict__ Z, const int bid) {
  __shared__ double red[4];
  const int s0 = bid;
  const double drop = drop_rel * (*tnorm);
  const double tol = 1e-12 * (*tnorm);
  if (lam_asc[s0] < drop) return;
  if (s0 > 0 && lam_asc[s0 - 1] >= drop && lam_asc[s0] - lam_asc[s0 - 1] <= tol) return;  // not a start
  int s1 = s0 + 1;
  while (s1 < n && lam_asc[s1] - lam_asc[s1 - 1] <= tol) ++s1;
  if (s1 - s0 < 2) return;
  for (int c = s0 + 1; c < s1; ++c) {
    for (int b = s0; b < c; ++b) {
      double dot = 0.0;
      for (int j = threadIdx.x; j < n; j += blockDim.x) dot += Z[(int64_t)j * n + b] * Z[(int64_t)j * n + c];
      dot = block_sum(dot, red);
      for (int j = threadIdx.x; j < n; j += blockDim.x) Z[(int64_t)j * n + c] -= dot * Z[(int64_t)j * n + b];
      __syncthreads();
    }
    double nr = 0.0;
    for (int j = threadIdx.x; j < n; j += blockDim.x) nr += Z[(int64_t)j * n + c] * Z[(int64_t)j * n + c];
    nr = block_sum(nr, red);
    const double sc = nr > 0.0 ? 1.0 / sqrt(nr) : 0.0;
    for (int j = threadIdx.x; j < n; j += blockDim.x) Z[(int64_t)j * n + c] *= sc;
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void cluster_mgs_kernel(const double* __restrict__ lam_asc, int n,
                                                          const double* __restrict__ tnorm, double drop_rel,
                                                          double* __restrict__ Z) {
  cluster_mgs_body(lam_asc, n, tnorm, drop_rel, Z, (int)blockIdx.x);
}

// The three stages above for several matrices in one launch each: matrix m has workgroups
// first[m] .. first[m + 1] - 1 (numbered from 0 within it). The arguments travel by value.
constexpr int kMidBatchMax = 16;
struct MidItem {
  const double* d;
  const double* e;
  int n, wpe;
  double* e2;
  double* lam;
  double* tnorm;
  double drop_rel;
  double* Z;
};
struct MidBatch {
  MidItem it[kMidBatchMax];
  int first[kMidBatchMax + 1];
  int n;
};
__device__ __forceinline__ int mid_member(const MidBatch& b) {
  int m = 0;
  while (m + 1 < b.n && (int)blockIdx.x >= b.first[m + 1]) ++m;
  return m;
}
__global__ __launch_bounds__(256) void bisect_batch_kernel(MidBatch b) {
  const int m = mid_member(b);
  const MidItem& q = b.it[m];
  bisect_body(q.d, q.e, q.n, q.wpe, q.e2, q.lam, q.tnorm, (int)blockIdx.x - b.first[m]);
}
template <int QN>
__global__ __launch_bounds__(64 * kInvWaves) void invit_batch_kernel(MidBatch b) {
  const int m = mid_member(b);
  const MidItem& q = b.it[m];
  invit_body<QN>(q.d, q.e, q.n, q.lam, q.tnorm, q.drop_rel, q.Z, (int)blockIdx.x - b.first[m]);
}
__global__ __launch_bounds__(256) void cluster_mgs_batch_kernel(MidBatch b) {
  const int m = mid_member(b);
  const MidItem& q = b.it[m];
  cluster_mgs_body(q.lam, q.n, q.tnorm, q.drop_rel, q.Z, (int)blockIdx.x - b.first[m]);
}

// Back-transformation V = H_0 H_1 ... H_{n-3} Z with the reflectors taken kWy at a time in compact
// WY form: H_k0 ... H_k1 = I - Y T Y^T (Y = [v_k0 .. v_k1], T upper triangular, built as in the
// forward-accumulation recurrence T[i][i] = tau_i, T[0:i, i] = -tau_i T[0:i, 0:i] Y[:, 0:i]^T v_i).
constexpr int kWy = 16;   // reflectors per block

// T of every block of kWy reflectors (one workgroup per block), stored kWy x kWy per block. The
// Gram matrix G = Y^T Y of the block's reflectors is one 16 x 16 FP64 MFMA product over n (the four
// waves split n; with the contraction index of K-step r taken as 4 (l / 16) + r, the same four
// doubles of a lane are its A and its B operand); then T column by column, the rows of a column in
// parallel: T[i][i] = tau_i, T[0:i, i] = -tau_i T[0:i, 0:i] G[0:i, i].
typedef double wy_d4 __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void wy_t_kernel(const double* __restrict__ V, const double* __restrict__ tau, int n,
                                                   double* __restrict__ Tall) {
  const int nref = n - 2;
  const int k0 = blockIdx.x * kWy;
  const int m = min(kWy, nref - k0);
  __shared__ double Gp[4][256];
  __shared__ double Gm[kWy][kWy + 1];
  __shared__ double Ts[kWy][kWy + 1];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int lr = lane & 15, lq = lane >> 4;
  const bool rv = lr < m;
  const double* vrow = V + (int64_t)(k0 + (rv ? lr : 0)) * n;
  const int nslab = (n + 15) / 16;
  wy_d4 acc = {0.0, 0.0, 0.0, 0.0};
  for (int sl = wid; sl < nslab; sl += 4) {
    double v[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int j = 16 * sl + 4 * lq + r;
      v[r] = (rv && j < n) ? vrow[j] : 0.0;
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(v[r], v[r], acc, 0, 0, 0);
  }
  // accumulator element r: G(lq + 4 r, lr)
#pragma unroll
  for (int r = 0; r < 4; ++r) Gp[wid][(lq + 4 * r) * 16 + lr] = acc[r];
  __syncthreads();
  if (threadIdx.x < 256) {
    const int a = threadIdx.x >> 4, i = threadIdx.x & 15;
    Gm[a][i] = Gp[0][threadIdx.x] + Gp[1][threadIdx.x] + Gp[2][threadIdx.x] + Gp[3][threadIdx.x];
    Ts[a][i] = 0.0;
  }
  __syncthreads();
  for (int i = 0; i < m; ++i) {
    const double t = tau[k0 + i];
    const int a = threadIdx.x;
    if (a < i) {
      double sum = 0.0;
      for (int b = a; b < i; ++b) sum += Ts[a][b] * Gm[b][i];
      Ts[a][i] = -t * sum;
    } else if (a == i) {
      Ts[i][i] = t;
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < kWy * kWy; e += blockDim.x)
    Tall[(int64_t)blockIdx.x * kWy * kWy + e] = Ts[e / kWy][e % kWy];
}

// Forming Q on the FP64 matrix cores, for n <= kBtMaxN. A workgroup owns 16 columns of Z (the
// identity at the start, Q at the end), held in registers as 16 x 16 accumulator tiles (tile t = rows 16t .. 16t+15, tiles
// dealt round-robin to the waves). Per block of kWy reflectors, staged in LDS:
//   W = Y^T Z   (each wave over its tiles, partial sums reduced through LDS),
//   S = T W     (every wave, redundantly: four MFMAs),
//   Z -= Y S    (each wave on its tiles).
// In v_mfma_f64_16x16x4f64 lane l supplies A(l % 16, k + l / 16) and B(k + l / 16, l % 16) and
// holds C(l / 16 + 4 r, l % 16) in accumulator element r; element r of a tile is therefore exactly
// the B operand of the K-step that covers rows 4 r .. 4 r + 3 of it, so Z and S are fed to the
// next product without any data movement. Tiles wholly at or above the block's first reflector
// row are left alone (Y is zero there).
typedef double bt_d4 __attribute__((ext_vector_type(4)));
constexpr int kBtWaves = 16;
constexpr int kBtTiles = 4;  // tiles per wave
constexpr int kBtMaxN = 16 * kBtWaves * kBtTiles;
static_assert(kBtMaxN == 64 * kBtWaves, "one reflector column per thread");
// slots of the per-wave partial W in LDS: half the waves, so that the Y block (kWy x (n + 1)
// doubles) and the partials fit in 160 KB at n = 1024 with the static arrays
constexpr int kWpSlots = kBtWaves / 2;
static_assert(kBtWaves % 2 == 0, "pairwise hand-over of the partial W");

__device__ __forceinline__ bt_d4 mfma64(double a, double b, bt_d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Q = H_0 H_1 ... H_{n-3} applied to the identity, written row-major (n x n) to Qm. Each
// workgroup owns 16 columns, held in MFMA accumulators over all row tiles; the reflector blocks are
// applied from the last to the first as I - Y T Y^T (compact WY form).
__global__ __launch_bounds__(64 * kBtWaves) void form_q_mfma_kernel(const double* __restrict__ V,
                                                                    const double* __restrict__ Tall, int n,
                                                                    double* __restrict__ Qm) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int nt = (n + 15) / 16;
  const int ldy = nt * 16 + 1;  // odd pitch: the 16 reflector rows fall in distinct LDS banks
  double* Ys = reinterpret_cast<double*>(smem_raw);  // kWy x ldy
  double* Wp = Ys + (size_t)kWy * ldy;              // kWpSlots x 256 partial W
  __shared__ double Ts[kWy * kWy];
  __shared__ double Ws[256];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int lr = lane & 15, lq = lane >> 4;
  const int c0 = blockIdx.x * 16;
  const int col = c0 + lr;

  bt_d4 acc[kBtTiles];
#pragma unroll
  for (int i = 0; i < kBtTiles; ++i) {
    const int t = wid + i * kBtWaves;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 16 * t + lq + 4 * r;
      acc[i][r] = (t < nt && row < n && row == col) ? 1.0 : 0.0;
    }
  }
  const int nref = n - 2;
  const int nblk = nref > 0 ? (nref + kWy - 1) / kWy : 0;
  // a block's reflectors and T factor are fetched into registers one block ahead, so that their
  // loads are in flight while the previous block is applied
  // thread t fetches column t of the block's kWy reflectors (kBtMaxN = blockDim.x >= n)
  const int jt = threadIdx.x;
  double ypf[kWy], tpf = 0.0;
  auto prefetch = [&](int b) {
    const int k0 = b * kWy;
    const int m = min(kWy, nref - k0);
#pragma unroll
    for (int u = 0; u < kWy; ++u) ypf[u] = (u < m && jt < n) ? V[(int64_t)(k0 + u) * n + jt] : 0.0;
    if (threadIdx.x < kWy * kWy) tpf = Tall[(int64_t)b * kWy * kWy + threadIdx.x];
  };
  if (nblk > 0) prefetch(nblk - 1);
  for (int b = nblk - 1; b >= 0; --b) {
    const int k0 = b * kWy;
    __syncthreads();
    if (jt < nt * 16) {
#pragma unroll
      for (int u = 0; u < kWy; ++u) Ys[u * ldy + jt] = ypf[u];
    }
    if (threadIdx.x < kWy * kWy) Ts[threadIdx.x] = tpf;
    __syncthreads();
    if (b > 0) prefetch(b - 1);
    // W = Y^T Z over this wave's tiles (rows <= k0 of Y are zero)
    bt_d4 w = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int i = 0; i < kBtTiles; ++i) {
      const int t = wid + i * kBtWaves;
      if (t < nt && 16 * t + 15 > k0) {
#pragma unroll
        for (int r = 0; r < 4; ++r) w = mfma64(Ys[lr * ldy + 16 * t + 4 * r + lq], acc[i][r], w);
      }
    }
    // W summed over the waves in a fixed order: the upper half of the waves hands its partials to
    // the lower half (pairwise), then each entry's kWpSlots partials are added by one thread
    if (wid >= kWpSlots) {
#pragma unroll
      for (int r = 0; r < 4; ++r) Wp[(wid - kWpSlots) * 256 + (lq + 4 * r) * 16 + lr] = w[r];
    }
    __syncthreads();
    if (wid < kWpSlots) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        double* slot = Wp + wid * 256 + (lq + 4 * r) * 16 + lr;
        *slot = w[r] + *slot;
      }
    }
    __syncthreads();
    if (threadIdx.x < 256) {
      double wsum = 0.0;
      for (int q = 0; q < kWpSlots; ++q) wsum += Wp[q * 256 + threadIdx.x];
      Ws[threadIdx.x] = wsum;
    }
    __syncthreads();
    // S = T W
    bt_d4 sacc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int a = 4 * s + lq;
      sacc = mfma64(Ts[lr * kWy + a], Ws[a * 16 + lr], sacc);
    }
    // Z -= Y S
#pragma unroll
    for (int i = 0; i < kBtTiles; ++i) {
      const int t = wid + i * kBtWaves;
      if (t < nt && 16 * t + 15 > k0) {
#pragma unroll
        for (int s = 0; s < 4; ++s) acc[i] = mfma64(-Ys[(4 * s + lq) * ldy + 16 * t + lr], sacc[s], acc[i]);
      }
    }
  }
  if (col < n) {
#pragma unroll
    for (int i = 0; i < kBtTiles; ++i) {
      const int t = wid + i * kBtWaves;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * t + lq + 4 * r;
        if (t < nt && row < n) Qm[(int64_t)row * n + col] = acc[i][r];
      }
    }
  }
}

// Eigenvector rows in descending eigenvalue order from Xt = (Q Z)^T (row c = eigenvector of the c-th
// smallest eigenvalue); pairs below the drop threshold become (0, zero vector)
__global__ void eig_finalize_kernel(const double* __restrict__ Xt, const double* __restrict__ lam_asc, int n,
                                    const double* __restrict__ tnorm, double drop_rel,
                                    double* __restrict__ evals_desc, double* __restrict__ evec_rows) {
  const int row = blockIdx.x * blockDim.x + threadIdx.x;  // component
  const int col = blockIdx.y;                             // eigenvector (ascending)
  const double drop = drop_rel * (*tnorm);
  const bool keep = lam_asc[col] >= drop;
  if (row == 0) evals_desc[n - 1 - col] = keep ? lam_asc[col] : 0.0;
  if (row < n) evec_rows[(int64_t)(n - 1 - col) * n + row] = keep ? Xt[(int64_t)col * n + row] : 0.0;
}

// The n x n FP64 products of the last stage (two Newton-Schulz steps and (Q Z)^T):
// D = alpha op(A) op(B) + beta C, with op(A)(i, k) = A[k n + i] when AT (else A[i n + k]) and
// op(B)(k, j) = B[j n + k] when BT (else B[k n + j]); all row-major with ld n, C may be null when beta
// is 0. A 256-thread workgroup forms a 32 x 32 tile of D, each wave 16 x 16 of it over the whole of K
// (at these sizes a split of K and its reduction cost more in latency than they save), from L2.
// K is taken 16 at a time, in four MFMA steps whose K index for lane group q = l / 16 is 16 c + 4 q + s
// (a fixed permutation of K): an operand whose K direction is contiguous in memory then comes as four
// consecutive doubles per lane (whole cache lines per load instruction), the other as four loads of 16
// consecutive doubles per lane group. kSdChunks chunks are in flight; two accumulators in turn.
// Rows, columns and K past n are read clamped (or up to 3 doubles past a row's end, which stays within
// the workspace: it ends in a pad) and never stored or masked, so that the loop has no branch.
constexpr int kSdChunks = 4;

// (at most two waves per SIMD: the grid is small, and the registers hold the loads in flight)
template <bool AT, bool BT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 2))) void small_dgemm_kernel(const double* __restrict__ A, const double* __restrict__ B,
                                                          const double* __restrict__ C, double* __restrict__ D,
                                                          int n, double alpha, double beta) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int lr = lane & 15, lq = lane >> 4;
  const int i0 = blockIdx.y * 32 + (wid >> 1) * 16, j0 = blockIdx.x * 32 + (wid & 1) * 16;
  const int ia = min(i0 + lr, n - 1), jb = min(j0 + lr, n - 1);
  const int chunks = (n + 15) / 16;
  double av[kSdChunks][4], bv[kSdChunks][4];
  auto load = [&](int c, double (&a)[4], double (&b)[4]) {
    const int k = 16 * c + 4 * lq;
    if (AT) {
#pragma unroll
      for (int t = 0; t < 4; ++t) a[t] = A[(int64_t)min(k + t, n - 1) * n + ia];
    } else {
      const double* p = A + (int64_t)ia * n + min(k, n - 1);
#pragma unroll
      for (int t = 0; t < 4; ++t) a[t] = p[t];
    }
    if (BT) {
      const double* p = B + (int64_t)jb * n + min(k, n - 1);
#pragma unroll
      for (int t = 0; t < 4; ++t) b[t] = p[t];
    } else {
#pragma unroll
      for (int t = 0; t < 4; ++t) b[t] = B[(int64_t)min(k + t, n - 1) * n + jb];
    }
  };
#pragma unroll
  for (int u = 0; u < kSdChunks; ++u) load(u, av[u], bv[u]);
  bt_d4 acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
  for (int c0 = 0; c0 < chunks; c0 += kSdChunks) {
#pragma unroll
    for (int u = 0; u < kSdChunks; ++u) {
      const int k = 16 * (c0 + u) + 4 * lq;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const double a = k + t < n ? av[u][t] : 0.0;  // K past n adds nothing
        if (t & 1) acc1 = mfma64(a, bv[u][t], acc1);
        else acc0 = mfma64(a, bv[u][t], acc0);
      }
      load(c0 + u + kSdChunks, av[u], bv[u]);
      __builtin_amdgcn_sched_barrier(0);  // the loads stay here, a whole ring of chunks ahead of their use
    }
  }
  const int j = j0 + lr;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = i0 + lq + 4 * r;
    if (i < n && j < n) {
      const double v = alpha * (acc0[r] + acc1[r]);
      D[(int64_t)i * n + j] = beta != 0.0 ? v + beta * C[(int64_t)i * n + j] : v;
    }
  }
}

template <bool AT, bool BT>
ngd_status small_dgemm(const double* A, const double* B, const double* C, double* D, int n, double alpha,
                       double beta, hipStream_t s) {
  const unsigned t = (unsigned)((n + 31) / 32);
  hipLaunchKernelGGL((small_dgemm_kernel<AT, BT>), dim3(t, t), dim3(256), 0, s, A, B, C, D, n, alpha, beta);
  NGD_HIP_TRY(hipGetLastError());
  return NGD_OK;
}

// Workspace layout (doubles unless noted): A1, V, Z (n^2 each), wk (5 n^2), d, e, tau, e2, lam
// (n each), tnorm (8), the barrier flags (256 unsigned) and the error word (in a 1 KiB slot), the
// T factors of the reflector blocks, then Qm (n^2, the explicit product of the reflectors) and a pad
// of 8.
struct EigWs {
  double *A1, *V, *Z, *wk, *dvec, *evec, *tau, *e2, *lam, *tnorm, *Tall, *Qm;
  unsigned* flags;
  int* err;
  size_t bytes;
  EigWs(void* work, int n) {
    double* w = reinterpret_cast<double*>(work);
    const size_t nn = (size_t)n * n;
    A1 = w;
    V = A1 + nn;
    Z = V + nn;
    wk = Z + nn;
    dvec = wk + 5 * nn;
    evec = dvec + n;
    tau = evec + n;
    e2 = tau + n;
    lam = e2 + n;
    tnorm = lam + n;
    flags = reinterpret_cast<unsigned*>(tnorm + 8);
    err = reinterpret_cast<int*>(flags + 248);
    Tall = tnorm + 8 + 128;  // the 1 KiB slot of the flags and the error word
    const size_t nblk = (size_t)n + 1;  // blocks of as few as one reflector
    Qm = Tall + nblk * kWy * kWy;
    bytes = (size_t)((Qm + nn + 8) - w) * sizeof(double);  // + a pad for the small products' row reads
  }
};

// The grid barriers need every workgroup resident at once: the grids below are far smaller than
// the device's CU count, and the occupancy is checked; every barrier wait is bounded (it raises the
// error word instead of spinning forever).
ngd_status check_coresident(const void* kernel, int threads, size_t lds, int blocks) {
  int dev = 0, cus = 0, per_cu = 0;
  NGD_HIP_TRY(hipGetDevice(&dev));
  NGD_HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  NGD_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, lds));
  if ((int64_t)cus * per_cu < blocks) {
    set_error("tridiagonalisation grid cannot be co-resident");
    return NGD_ERR_HIP;
  }
  return NGD_OK;
}

template <int QN>
ngd_status launch_tridiag_reg(const TriArgs& ta, hipStream_t s) {
  // as few workgroups as hold the rows: the barrier's cost grows with the number of workgroups
  constexpr int RW = tr_rows(QN), WV = tr_waves(QN);
  const int per = WV * RW;
  const int blocks = (ta.n + per - 1) / per;
  if (blocks > 64) {  // the barrier polls one flag per lane of one wave
    set_error("tridiagonalisation: more than 64 workgroups");
    return NGD_ERR_INVALID;
  }
  NGD_TRY(check_coresident((const void*)tridiag_reg_kernel<QN, RW, WV>, 64 * WV, 0, blocks));
  hipLaunchKernelGGL((tridiag_reg_kernel<QN, RW, WV>), dim3(blocks), dim3(64 * WV), 0, s, ta);
  NGD_HIP_TRY(hipGetLastError());
  return NGD_OK;
}

ngd_status launch_tridiag(const TriArgs& ta, hipStream_t s) {
  const int n = ta.n;
  if (n <= kTrMaxN) {
    switch ((n + 63) / 64) {
      case 1: return launch_tridiag_reg<1>(ta, s);
      case 2: return launch_tridiag_reg<2>(ta, s);
      case 3: return launch_tridiag_reg<3>(ta, s);
      case 4: return launch_tridiag_reg<4>(ta, s);
      case 5: return launch_tridiag_reg<5>(ta, s);
      case 6: return launch_tridiag_reg<6>(ta, s);
      case 7: return launch_tridiag_reg<7>(ta, s);
      case 8: return launch_tridiag_reg<8>(ta, s);
      case 9: return launch_tridiag_reg<9>(ta, s);
      case 10: return launch_tridiag_reg<10>(ta, s);
      case 11: return launch_tridiag_reg<11>(ta, s);
      case 12: return launch_tridiag_reg<12>(ta, s);
      case 13: return launch_tridiag_reg<13>(ta, s);
      case 14: return launch_tridiag_reg<14>(ta, s);
      case 15: return launch_tridiag_reg<15>(ta, s);
      default: return launch_tridiag_reg<16>(ta, s);
    }
  }
  set_error("tridiagonalisation: n above 1024");
  return NGD_ERR_INVALID;
}

template <int QN>
ngd_status launch_tridiag_batch_qn(const TriArgs* items, int n, hipStream_t s) {
  constexpr int RW = tr_rows(QN), WV = tr_waves(QN);
  const int per = WV * RW;
  for (int c0 = 0; c0 < n; c0 += kTriBatchMax) {
    TriBatch tb{};
    tb.n = std::min(kTriBatchMax, n - c0);
    int total = 0;
    for (int m = 0; m < tb.n; ++m) {
      tb.a[m] = items[c0 + m];
      tb.first[m] = total;
      const int blocks = (tb.a[m].n + per - 1) / per;
      if (blocks > 64) {
        set_error("tridiagonalisation: more than 64 workgroups");
        return NGD_ERR_INVALID;
      }
      total += blocks;
    }
    tb.first[tb.n] = total;
    NGD_TRY(check_coresident((const void*)tridiag_batch_kernel<QN, RW, WV>, 64 * WV, 0, total));
    hipLaunchKernelGGL((tridiag_batch_kernel<QN, RW, WV>), dim3(total), dim3(64 * WV), 0, s, tb);
    NGD_HIP_TRY(hipGetLastError());
  }
  return NGD_OK;
}

// the matrices of each register shape (ceil(n / 64) columns per lane) in launches of their own
ngd_status launch_tridiag_batch(const TriArgs* items, int n, hipStream_t s) {
  std::vector<TriArgs> cls;
  for (int q = 1; q <= kTrMaxN / 64; ++q) {
    cls.clear();
    for (int i = 0; i < n; ++i)
      if (items[i].n >= 1 && (items[i].n + 63) / 64 == q) cls.push_back(items[i]);
    if (cls.empty()) continue;
    const int m = (int)cls.size();
    switch (q) {
      case 1: NGD_TRY(launch_tridiag_batch_qn<1>(cls.data(), m, s)); break;
      case 2: NGD_TRY(launch_tridiag_batch_qn<2>(cls.data(), m, s)); break;
      case 3: NGD_TRY(launch_tridiag_batch_qn<3>(cls.data(), m, s)); break;
      case 4: NGD_TRY(launch_tridiag_batch_qn<4>(cls.data(), m, s)); break;
      case 5: NGD_TRY(launch_tridiag_batch_qn<5>(cls.data(), m, s)); break;
      case 6: NGD_TRY(launch_tridiag_batch_qn<6>(cls.data(), m, s)); break;
      case 7: NGD_TRY(launch_tridiag_batch_qn<7>(cls.data(), m, s)); break;
      case 8: NGD_TRY(launch_tridiag_batch_qn<8>(cls.data(), m, s)); break;
      case 9: NGD_TRY(launch_tridiag_batch_qn<9>(cls.data(), m, s)); break;
      case 10: NGD_TRY(launch_tridiag_batch_qn<10>(cls.data(), m, s)); break;
      case 11: NGD_TRY(launch_tridiag_batch_qn<11>(cls.data(), m, s)); break;
      case 12: NGD_TRY(launch_tridiag_batch_qn<12>(cls.data(), m, s)); break;
      case 13: NGD_TRY(launch_tridiag_batch_qn<13>(cls.data(), m, s)); break;
      case 14: NGD_TRY(launch_tridiag_batch_qn<14>(cls.data(), m, s)); break;
      case 15: NGD_TRY(launch_tridiag_batch_qn<15>(cls.data(), m, s)); break;
      default: NGD_TRY(launch_tridiag_batch_qn<16>(cls.data(), m, s)); break;
    }
  }
  return NGD_OK;
}

// Zero the words a call must start from and fill the tridiagonalisation's arguments.
ngd_status sym_eig_prepare(double* A, int n, void* work, hipStream_t s, bool keep_err, TriArgs* ta) {
  EigWs ws(work, n);
  // the barrier flags, and the error word unless an earlier call's must survive (it lies after them)
  ngd_status st = launch_zero(ws.flags, keep_err ? sizeof(unsigned) * 248 : 1024, s);
  if (st != NGD_OK) return st;
  st = launch_zero(ws.tau, sizeof(double) * n, s);
  if (st != NGD_OK) return st;
  // exchange buffers of the tridiagonalisation (2 n each): PV in A1, P in wk (both free until it is done)
  *ta = TriArgs{A, ws.A1, n, ws.dvec, ws.evec, ws.V, ws.tau, ws.wk, ws.flags, ws.err};
  return NGD_OK;
}

}  // namespace

size_t eig_workspace_bytes(int n) { return EigWs(nullptr, n).bytes; }

ngd_status launch_sym_eig(double* A, int n, double drop_rel, double* evals_desc, double* evec_rows, void* work,
                               hipStream_t s, hipStream_t side, hipEvent_t fork, hipEvent_t join, bool keep_err) {
  if (n <= 0) return NGD_OK;
  if (n > kBtMaxN) {
    set_error("symmetric eigensolver: n above 1024");
    return NGD_ERR_INVALID;
  }
  TriArgs ta;
  NGD_TRY(sym_eig_prepare(A, n, work, s, keep_err, &ta));
  NGD_TRY(launch_tridiag(ta, s));
  return launch_sym_eig_finish(n, drop_rel, evals_desc, evec_rows, work, s, side, fork, join);
}

ngd_status launch_sym_eig_tridiag_batch(const EigJob* jobs, int n, hipStream_t s) {
  std::vector<TriArgs> items;
  for (int i = 0; i < n; ++i) {
    if (jobs[i].n <= 0) continue;
    if (jobs[i].n > kBtMaxN) {
      set_error("symmetric eigensolver: n above 1024");
      return NGD_ERR_INVALID;
    }
    TriArgs ta;
    NGD_TRY(sym_eig_prepare(jobs[i].A, jobs[i].n, jobs[i].work, s, jobs[i].keep_err, &ta));
    items.push_back(ta);
  }
  return launch_tridiag_batch(items.data(), (int)items.size(), s);
}

namespace {

// wy_t and form_q (the explicit Q) on the side stream, forked from s, or on s itself
ngd_status eig_side_q(int n, void* work, hipStream_t s, hipStream_t side, hipEvent_t fork, hipEvent_t join) {
  EigWs ws(work, n);
  // The explicit Q = H_0 ... H_{n-3} needs only the reflectors: on the side stream (when given) it
  // overlaps the eigenvalues, the eigenvectors of T and their orthogonalisation, and the
  // back-transformation becomes one product Q Z at the end.
  hipStream_t qs = side != nullptr ? side : s;
  if (side != nullptr) {
    NGD_HIP_TRY(hipEventRecord(fork, s));
    NGD_HIP_TRY(hipStreamWaitEvent(side, fork, 0));
  }
  const int nblk = n > 2 ? (n - 2 + kWy - 1) / kWy : 0;
  if (nblk > 0) hipLaunchKernelGGL(wy_t_kernel, dim3(nblk), dim3(256), 0, qs, ws.V, ws.tau, n, ws.Tall);
  const int nt = (n + 15) / 16;
  const size_t lds = sizeof(double) * ((size_t)kWy * (nt * 16 + 1) + (size_t)kWpSlots * 256);
  NGD_HIP_TRY(hipFuncSetAttribute((const void*)form_q_mfma_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)lds));
  hipLaunchKernelGGL(form_q_mfma_kernel, dim3(nt), dim3(64 * kBtWaves), lds, qs, ws.V, ws.Tall, n, ws.Qm);
  NGD_HIP_TRY(hipGetLastError());
  if (side != nullptr) NGD_HIP_TRY(hipEventRecord(join, side));
  return NGD_OK;
}

// the arguments of multisection, inverse iteration and the cluster orthogonalisation for one matrix
ngd_status eig_mid_item(int n, double drop_rel, void* work, MidItem* q) {
  EigWs ws(work, n);
  // two waves per eigenvalue while the 2n waves find a SIMD each, else one
  int dev = 0, cus = 0;
  NGD_HIP_TRY(hipGetDevice(&dev));
  NGD_HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  *q = MidItem{ws.dvec, ws.evec, n, 2 * n <= 4 * cus ? 2 : 1, ws.e2, ws.lam, ws.tnorm, drop_rel, ws.Z};
  return NGD_OK;
}

// Newton-Schulz, the product with Q (after the side stream's join) and the eigenvector rows
ngd_status eig_rest(int n, double drop_rel, double* evals_desc, double* evec_rows, void* work, hipStream_t s,
                    hipStream_t side, hipEvent_t join) {
  EigWs ws(work, n);
  double* A1 = ws.A1;
  double* Z = ws.Z;
  double* wk = ws.wk;
  double* lam = ws.lam;
  double* tnorm = ws.tnorm;
  // one Newton-Schulz step Z <- 1.5 Z - 0.5 Z (Z^T Z) removes the residual non-orthogonality of the
  // inverse-iteration vectors (quadratic convergence; dropped columns stay zero)
  double* E = A1;   // free after the tridiagonalisation
  double* Z2 = wk;  // free after inverse iteration
  for (int ns = 0; ns < 2; ++ns) {
    NGD_TRY((small_dgemm<true, false>(Z, Z, nullptr, E, n, 1.0, 0.0, s)));
    NGD_TRY((small_dgemm<false, false>(Z, E, Z, Z2, n, -0.5, 1.5, s)));
    double* t = Z;
    Z = Z2;
    Z2 = t;
  }
  // (Q Z)^T = Z^T Q^T once Q is there, then the eigenvector rows in descending order
  if (side != nullptr) NGD_HIP_TRY(hipStreamWaitEvent(s, join, 0));
  double* Xt = wk;  // free after the Newton-Schulz steps (Z is back in its own buffer)
  NGD_TRY((small_dgemm<true, true>(Z, ws.Qm, nullptr, Xt, n, 1.0, 0.0, s)));
  hipLaunchKernelGGL(eig_finalize_kernel, dim3((n + 255) / 256, n), dim3(256), 0, s, Xt, lam, n, tnorm, drop_rel,
                     evals_desc, evec_rows);
  NGD_HIP_TRY(hipGetLastError());
  return NGD_OK;
}


}  // namespace

ngd_status launch_sym_eig_finish(int n, double drop_rel, double* evals_desc, double* evec_rows, void* work,
                                 hipStream_t s, hipStream_t side, hipEvent_t fork, hipEvent_t join) {
  if (n <= 0) return NGD_OK;
  NGD_TRY(eig_side_q(n, work, s, side, fork, join));
  MidItem q;
  NGD_TRY(eig_mid_item(n, drop_rel, work, &q));
  const int per_block = 4 / q.wpe;
  hipLaunchKernelGGL(bisect_kernel, dim3((n + per_block - 1) / per_block), dim3(256), 2 * sizeof(double) * n, s, q.d,
                     q.e, n, q.wpe, q.e2, q.lam, q.tnorm);
  const dim3 inv_grid((n + kInvWaves - 1) / kInvWaves), inv_block(64 * kInvWaves);
#define NGD_INVIT(QN) \
  case QN: hipLaunchKernelGGL(invit_kernel<QN>, inv_grid, inv_block, 0, s, q.d, q.e, n, q.lam, q.tnorm, drop_rel, q.Z); break;
  switch ((n + 63) / 64) { NGD_INVIT_SHAPES(NGD_INVIT) }
#undef NGD_INVIT
  NGD_HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(cluster_mgs_kernel, dim3(n), dim3(256), 0, s, q.lam, n, q.tnorm, drop_rel, q.Z);
  NGD_HIP_TRY(hipGetLastError());
  return eig_rest(n, drop_rel, evals_desc, evec_rows, work, s, side, join);
}

ngd_status launch_sym_eig_middle_batch(const EigJob* jobs, int n, hipStream_t s) {
  std::vector<MidItem> items;
  for (int i = 0; i < n; ++i) {
    const EigJob& j = jobs[i];
    if (j.n <= 0) continue;
    NGD_TRY(eig_side_q(j.n, j.work, s, j.side, j.fork, j.join));
    MidItem q;
    NGD_TRY(eig_mid_item(j.n, j.drop_rel, j.work, &q));
    items.push_back(q);
  }
  const int m = (int)items.size();
  for (int c0 = 0; c0 < m; c0 += kMidBatchMax) {
    MidBatch b{};
    b.n = std::min(kMidBatchMax, m - c0);
    for (int k = 0; k < b.n; ++k) b.it[k] = items[c0 + k];
    auto launch = [&](auto kernel, auto blocks_of, int threads, size_t lds) {
      int total = 0;
      for (int k = 0; k < b.n; ++k) {
        b.first[k] = total;
        total += blocks_of(b.it[k]);
      }
      b.first[b.n] = total;
      hipLaunchKernelGGL(kernel, dim3(total), dim3(threads), lds, s, b);
      NGD_HIP_TRY(hipGetLastError());
      return NGD_OK;
    };
    size_t lds = 0;
    for (int k = 0; k < b.n; ++k) lds = std::max(lds, 2 * sizeof(double) * b.it[k].n);
    NGD_TRY(launch(bisect_batch_kernel, [](const MidItem& q) { return (q.n + 4 / q.wpe - 1) / (4 / q.wpe); }, 256, lds));
    int qn = 1;
    for (int k = 0; k < b.n; ++k) qn = std::max(qn, (b.it[k].n + 63) / 64);
    const auto inv_blocks = [](const MidItem& q) { return (q.n + kInvWaves - 1) / kInvWaves; };
#define NGD_INVIT(QN) \
  case QN: NGD_TRY(launch(invit_batch_kernel<QN>, inv_blocks, 64 * kInvWaves, 0)); break;
    switch (qn) { NGD_INVIT_SHAPES(NGD_INVIT) }
#undef NGD_INVIT
    NGD_TRY(launch(cluster_mgs_batch_kernel, [](const MidItem& q) { return q.n; }, 256, 0));
  }
  return NGD_OK;
}

ngd_status launch_sym_eig_rest(int n, double drop_rel, double* evals_desc, double* evec_rows, void* work,
                               hipStream_t s, hipStream_t side, hipEvent_t join) {
  if (n <= 0) return NGD_OK;
  return eig_rest(n, drop_rel, evals_desc, evec_rows, work, s, side, join);
}

const int* eig_error_flag(void* work, int n) { return EigWs(work, n).err; }

}  // namespace ngd
