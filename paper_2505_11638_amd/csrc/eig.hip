// FP64 symmetric eigendecomposition of the small ell x ell matrices of the Nystrom core.
//
// Alg. 6 needs the thin SVD of the p x ell matrix B; its right singular vectors and squared
// singular values are the eigenpairs of the ell x ell Gram matrix B^T B, computed here in FP64:
//  1. Householder tridiagonalisation Q^T A Q = T in one launch whose workgroups meet at a grid
//     barrier once per column. The trailing matrix is row-distributed over the workgroups and kept
//     in LDS; each step applies the previous step's rank-2 update lazily while forming p = tau A v.
//  2. Eigenvalues of T by multisection on Sturm counts (one wave per eigenvalue).
//  3. Eigenvectors of T by inverse iteration with partial-pivoting LU of T - lambda I (one thread
//     per eigenvector), modified Gram-Schmidt inside clusters of (nearly) equal eigenvalues, and two
//     Newton-Schulz steps that restore orthonormality to working precision.
//  4. Back-transformation V = H_0 H_1 ... H_{n-3} Z (one workgroup per group of columns).
// Eigenpairs whose eigenvalue is below drop_rel * (Gershgorin bound of T) are returned as
// (0, zero vector).
#include "common.h"

namespace ngd {
namespace {

constexpr int kTriBlocks = 64;
constexpr int kTriThreads = 256;

struct TriArgs {
  double* A0;      // input matrix (n x n, ld n), read once
  double* A1;      // two pivot-row buffers (2 n)
  int n;
  double* d;       // diagonal of T
  double* e;       // off-diagonal of T (n-1)
  double* V;       // Householder vectors, row k = v_k (support k+1..n-1, v_k[k+1] = 1)
  double* tau;     // Householder scalars
  double* p;       // 2 n: p = tau A v of the current step (double-buffered by step parity, so that
                   // a workgroup that runs ahead never overwrites values another still has to read)
  unsigned* flags; // one barrier flag per workgroup
  int* err;
};

// Grid barrier number `epoch` (0, 1, 2, ...): workgroup g publishes epoch + 1 in its own flag (no
// contended atomic) and wave 0 polls all flags. One agent-scope release fence before publishing and
// one acquire fence after the wait (each is an L2 write-back or invalidate on this GPU, so they are
// kept to the minimum). The wait is bounded: on timeout it raises `err`.
__device__ bool grid_sync(unsigned* flags, unsigned epoch, int* err) {
  __syncthreads();
  if (threadIdx.x < 64) {
    const unsigned target = epoch + 1u;
    if (threadIdx.x == 0) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      __hip_atomic_store(flags + blockIdx.x, target, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    long spins = 0;
    while (true) {
      int ok = 1;
      for (int g = threadIdx.x; g < (int)gridDim.x; g += 64)
        ok &= __hip_atomic_load(flags + g, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= target;
      if (__all(ok)) break;
      __builtin_amdgcn_s_sleep(1);
      if (++spins > (1L << 24)) {  // seconds: give up instead of hanging
        if (threadIdx.x == 0) __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
    }
    if (threadIdx.x == 0) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
  return __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0;
}

// One Householder step per column k, rows of the trailing matrix resident in LDS: workgroup g owns
// rows i = g, g + G, g + 2G, ... Each step applies the previous step's rank-2 update (v, w) to the
// owned rows in place, forms p_i = tau A_i . v, and the owner of row k+1 publishes that updated row
// (the next pivot row) to global memory. After one grid barrier every workgroup reads p and the
// pivot row together, forms w = p - (tau/2)(p . v) v and, from the pivot row, the next Householder
// vector.
__global__ __launch_bounds__(kTriThreads) void tridiag_kernel(TriArgs a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int n = a.n, G = gridDim.x, g = blockIdx.x;
  const int R = (n + G - 1) / G;  // rows per workgroup
  double* rows = reinterpret_cast<double*>(smem_raw);   // R x n
  double* vprev = rows + (size_t)R * n;
  double* wprev = vprev + n;
  double* v = wprev + n;
  double* pivl = v + n;  // the current pivot row
  __shared__ double red[8];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int r = 0; r < R; ++r) {
    const int i = g + r * G;
    for (int j = threadIdx.x; j < n; j += blockDim.x) rows[(size_t)r * n + j] = i < n ? a.A0[(int64_t)i * n + j] : 0.0;
  }
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    vprev[j] = wprev[j] = 0.0;
    pivl[j] = a.A0[j];  // step 0: row 0 of A, no pending update
  }
  __syncthreads();
  for (int k = 0; k + 2 < n; ++k) {
    // column k of A^(k) below the diagonal = pivot row k with the pending update applied
    double tail = 0.0;
    const double vk = vprev[k], wk = wprev[k];
    for (int j = k + 1 + threadIdx.x; j < n; j += blockDim.x) {
      const double x = pivl[j] - vk * wprev[j] - wk * vprev[j];
      v[j] = x;
      if (j > k + 1) tail += x * x;
    }
    const double dk = pivl[k] - 2.0 * vk * wk;
    tail = block_sum(tail, red);
    const double alpha = v[k + 1];
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
    __syncthreads();
    for (int j = k + 2 + threadIdx.x; j < n; j += blockDim.x) v[j] *= scale;
    if (threadIdx.x == 0) v[k + 1] = 1.0;
    __syncthreads();
    if (g == 0) {
      if (threadIdx.x == 0) {
        a.d[k] = dk;
        a.e[k] = beta;
        a.tau[k] = tau;
      }
      for (int j = threadIdx.x; j < n; j += blockDim.x) a.V[(int64_t)k * n + j] = j > k ? v[j] : 0.0;
    }
    // owned rows i > k: pending update in place, p_i = tau * row . v (one wave per row)
    double* next_pivot = a.A1 + (int64_t)((k + 1) & 1) * n;
    for (int r = wid; r < R; r += nw) {
      const int i = g + r * G;
      if (i <= k || i >= n) continue;
      double* row = rows + (size_t)r * n;
      const double vi = vprev[i], wi = wprev[i];
      const bool publish = (i == k + 1);
      double acc = 0.0;
      for (int j = k + 1 + lane; j < n; j += 64) {
        const double x = row[j] - vi * wprev[j] - wi * vprev[j];
        row[j] = x;
        acc += x * v[j];
        if (publish) next_pivot[j] = x;
      }
      acc = wave_sum(acc);
      if (lane == 0) a.p[(int64_t)(k & 1) * n + i] = tau * acc;
    }
    if (!grid_sync(a.flags, (unsigned)k, a.err)) return;
    // p and the next pivot row are read together; w = p - (tau/2)(p . v) v is kept by every
    // workgroup as the pending update
    double pv = 0.0;
    for (int j = k + 1 + threadIdx.x; j < n; j += blockDim.x) {
      const double pj = a.p[(int64_t)(k & 1) * n + j];
      const double nx = next_pivot[j];
      wprev[j] = pj;
      pivl[j] = nx;
      pv += pj * v[j];
    }
    pv = block_sum(pv, red);
    const double c = 0.5 * tau * pv;
    __syncthreads();
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
      if (j > k) {
        wprev[j] = wprev[j] - c * v[j];
        vprev[j] = v[j];
      } else {
        wprev[j] = 0.0;
        vprev[j] = 0.0;
      }
    }
    __syncthreads();
  }
  // last 2 x 2 (or 1 x 1) block, from the owners' rows with the pending update
  if (threadIdx.x == 0) {
    const int m = n >= 2 ? n - 2 : 0;
    for (int r = 0; r < R; ++r) {
      const int i = g + r * G;
      if (i < m || i >= n) continue;
      const double* row = rows + (size_t)r * n;
      if (i == m && n >= 2) {
        a.d[m] = row[m] - 2.0 * vprev[m] * wprev[m];
        a.e[m] = row[m + 1] - vprev[m] * wprev[m + 1] - wprev[m] * vprev[m + 1];
      } else if (i == m + 1) {
        a.d[m + 1] = row[m + 1] - 2.0 * vprev[m + 1] * wprev[m + 1];
      } else if (n == 1) {
        a.d[0] = row[0];
      }
    }
  }
}

// ---- register-resident tridiagonalisation (n <= kTrMaxN) ----
// The same Householder recurrence with the trailing matrix held in registers: 8 waves per
// workgroup, each owning up to four of the workgroup's rows, lane l holding columns l, l + 64, ...
// Only the per-column vectors go through LDS (thread t handles columns t and t + 512), so few
// workgroups (about n / 32) suffice and the grid barrier, whose latency bounds this kernel, is as
// cheap as it gets. The vectors the workgroups exchange (p and the next pivot row) are written and
// read with device-coherent (sc1) accesses, double-buffered by step parity, so the barrier needs no
// cache write-back or invalidate: each thread waits for its own stores to complete before the
// workgroup publishes its flag.
constexpr int kTrWaves = 8;
constexpr int kTrThreads = 64 * kTrWaves;
constexpr int kTrRows = 4;  // rows per wave
constexpr int kTrMaxN = 1024;
constexpr int kTrCols = kTrMaxN / kTrThreads;  // per-column vector entries per thread

__device__ __forceinline__ void st_coherent(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ld_coherent(double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Barrier number `epoch` for data exchanged only through st_coherent / ld_coherent. The flags of up
// to 64 workgroups are polled by wave 0 (one per lane). The wait is bounded; on timeout the error
// word is raised and false is returned to the whole workgroup.
__device__ bool grid_sync_coherent(unsigned* flags, unsigned epoch, int* err, int* timed_out) {
  __builtin_amdgcn_s_waitcnt(0);
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __syncthreads();
  if (threadIdx.x < 64) {
    const unsigned target = epoch + 1u;
    if (threadIdx.x == 0) __hip_atomic_store(flags + blockIdx.x, target, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    long spins = 0;
    while (true) {
      const int g = threadIdx.x;
      const bool ok = g >= (int)gridDim.x ||
                      __hip_atomic_load(flags + g, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= target;
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

template <int QN>
__global__ __launch_bounds__(kTrThreads) void tridiag_reg_kernel(TriArgs a) {
  // the three per-column vectors in one array, so that one base address serves all of them
  __shared__ double vecs[3 * kTrMaxN];
  double* vprev = vecs;
  double* wprev = vecs + kTrMaxN;
  double* vcur = vecs + 2 * kTrMaxN;
  __shared__ double red[kTrWaves];
  __shared__ int timed_out;
  const int n = a.n, G = gridDim.x, g = blockIdx.x;
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
  // per-column state of columns j_t = threadIdx.x + kTrThreads t: pivot row entry (row 0, nothing
  // pending) and the pending rank-2 update
  double piv[kTrCols], vp[kTrCols], wp[kTrCols], vj[kTrCols];
#pragma unroll
  for (int t = 0; t < kTrCols; ++t) {
    const int j = threadIdx.x + kTrThreads * t;
    piv[t] = j < n ? a.A0[j] : 0.0;
    vp[t] = wp[t] = 0.0;
    vprev[j] = 0.0;
    wprev[j] = 0.0;
  }
  __syncthreads();
  for (int k = 0; k + 2 < n; ++k) {
    // column k of A^(k) below the diagonal: the pivot row with the pending update applied
    const double vk = vprev[k], wk = wprev[k];
    double x[kTrCols], tail = 0.0;
#pragma unroll
    for (int t = 0; t < kTrCols; ++t) {
      const int j = threadIdx.x + kTrThreads * t;
      x[t] = (j > k && j < n) ? piv[t] - vk * wp[t] - wk * vp[t] : 0.0;
      vcur[j] = x[t];
      if (j > k + 1) tail += x[t] * x[t];
    }
    tail = block_sum(tail, red);
    const double alpha = vcur[k + 1];
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
    __syncthreads();  // every thread has read vcur[k + 1]
#pragma unroll
    for (int t = 0; t < kTrCols; ++t) {
      const int j = threadIdx.x + kTrThreads * t;
      vj[t] = j == k + 1 ? 1.0 : (j > k + 1 ? x[t] * scale : 0.0);
      vcur[j] = vj[t];
      if (g == 0) {
        if (j == k) a.d[k] = piv[t] - 2.0 * vk * wk;
        if (j < n) a.V[(int64_t)k * n + j] = vj[t];
      }
    }
    if (g == 0 && threadIdx.x == 0) {
      a.e[k] = beta;
      a.tau[k] = tau;
    }
    __syncthreads();
    // owned rows i > k: the pending update in place, p_i = tau * row . v. The column vectors are
    // read from LDS four columns at a time for all rows (one wait per chunk); columns c <= k and
    // c >= n need no predicate: v is zero there, and the entries they change are never read again.
    double* next_pivot = a.A1 + (int64_t)((k + 1) & 1) * n;
    double* pk = a.p + (int64_t)(k & 1) * n;
    double vi[kTrRows], wi[kTrRows], acc[kTrRows];
    bool live[kTrRows];
#pragma unroll
    for (int s = 0; s < kTrRows; ++s) {
      const int i = g + G * (wid + kTrWaves * s);
      live[s] = i > k && i < n;
      vi[s] = live[s] ? vprev[i] : 0.0;
      wi[s] = live[s] ? wprev[i] : 0.0;
      acc[s] = 0.0;
    }
#pragma unroll
    for (int q0 = 0; q0 < QN; q0 += 4) {
      double wq[4], vq[4], uq[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int c = lane + 64 * (q0 + u);
        if (q0 + u < QN) {
          wq[u] = wprev[c];
          vq[u] = vprev[c];
          uq[u] = vcur[c];
        }
      }
#pragma unroll
      for (int s = 0; s < kTrRows; ++s) {
        if (!live[s]) continue;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          if (q0 + u < QN) {
            const double y = rows[s][q0 + u] - vi[s] * wq[u] - wi[s] * vq[u];
            rows[s][q0 + u] = y;
            acc[s] += y * uq[u];
          }
        }
      }
    }
#pragma unroll
    for (int s = 0; s < kTrRows; ++s) acc[s] = wave_sum(acc[s]);
#pragma unroll
    for (int s = 0; s < kTrRows; ++s) {
      const int i = g + G * (wid + kTrWaves * s);
      if (!live[s]) continue;
      if (lane == 0) st_coherent(pk + i, tau * acc[s]);
      if (i == k + 1) {  // the next pivot row, updated
#pragma unroll
        for (int q = 0; q < QN; ++q) {
          const int c = lane + 64 * q;
          if (c > k && c < n) st_coherent(next_pivot + c, rows[s][q]);
        }
      }
    }
    if (!grid_sync_coherent(a.flags, (unsigned)k, a.err, &timed_out)) return;
    // p and the next pivot row; w = p - (tau/2)(p . v) v becomes the pending update
    double pj[kTrCols], pvs = 0.0;
#pragma unroll
    for (int t = 0; t < kTrCols; ++t) {
      const int j = threadIdx.x + kTrThreads * t;
      pj[t] = 0.0;
      if (j > k && j < n) {
        pj[t] = ld_coherent(pk + j);
        piv[t] = ld_coherent(next_pivot + j);
      }
      pvs += pj[t] * vj[t];
    }
    const double c = 0.5 * tau * block_sum(pvs, red);
#pragma unroll
    for (int t = 0; t < kTrCols; ++t) {
      const int j = threadIdx.x + kTrThreads * t;
      const bool live = j > k && j < n;
      wp[t] = live ? pj[t] - c * vj[t] : 0.0;
      vp[t] = live ? vj[t] : 0.0;
      vprev[j] = vp[t];
      wprev[j] = wp[t];
    }
    __syncthreads();
  }
  // last 2 x 2 (or 1 x 1) block: rows n-2 (the pivot) and n-1 with the pending update
  const int m = n >= 2 ? n - 2 : 0;
#pragma unroll
  for (int t = 0; t < kTrCols; ++t) {
    const int j = threadIdx.x + kTrThreads * t;
    if (g != 0) break;
    if (n == 1) {
      if (j == 0) a.d[0] = piv[t];
    } else {
      if (j == m) a.d[m] = piv[t] - 2.0 * vprev[m] * wprev[m];
      if (j == m + 1) a.e[m] = piv[t] - vprev[m] * wprev[m + 1] - wprev[m] * vprev[m + 1];
    }
  }
  if (n == 1) return;
#pragma unroll
  for (int s = 0; s < kTrRows; ++s) {
    const int i = g + G * (wid + kTrWaves * s);
    if (i != m + 1) continue;
#pragma unroll
    for (int q = 0; q < QN; ++q)
      if (lane + 64 * q == m + 1) a.d[m + 1] = rows[s][q] - 2.0 * vprev[m + 1] * wprev[m + 1];
  }
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

// eigenvalue index i (ascending) of T by bisection; also prepares e^2
__global__ void bisect_kernel(const double* __restrict__ d, const double* __restrict__ e, int n,
                              double* __restrict__ e2, double* __restrict__ lam_asc, double* __restrict__ tnorm) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* sd = reinterpret_cast<double*>(smem_raw);
  double* se2 = sd + n;
  __shared__ double lo_s, hi_s;
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    sd[j] = d[j];
    if (j < n - 1) se2[j] = e[j] * e[j];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double lo = 1e300, hi = -1e300;
    for (int j = 0; j < n; ++j) {
      double r = (j > 0 ? fabs(e[j - 1]) : 0.0) + (j < n - 1 ? fabs(e[j]) : 0.0);
      lo = fmin(lo, sd[j] - r);
      hi = fmax(hi, sd[j] + r);
    }
    lo_s = lo;
    hi_s = hi;
    if (blockIdx.x == 0) {
      *tnorm = fmax(fabs(lo), fabs(hi));
      for (int j = 0; j < n - 1; ++j) e2[j] = se2[j];
    }
  }
  __syncthreads();
  // multisection: one wave per eigenvalue; its 64 lanes evaluate 64 interior points of the current
  // interval, the first point whose Sturm count exceeds i bounds eigenvalue i from above. Each round
  // shrinks the interval 65-fold; stop at an absolute width of a few ulps of ||T||.
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (i >= n) return;
  const double tn = fmax(fabs(lo_s), fabs(hi_s));
  const double pivmin = fmax(1e-300, 2.2250738585072014e-308 * fmax(1.0, tn * tn));
  double lo = lo_s - 1e-14 * tn - pivmin, hi = hi_s + 1e-14 * tn + pivmin;
  const double tol = 4.0 * 2.220446049250313e-16 * tn + pivmin;
  for (int it = 0; it < 16 && hi - lo > tol; ++it) {
    const double h = (hi - lo) / 65.0;
    const double x = lo + h * (lane + 1);
    const bool above = sturm_count(sd, se2, n, x, pivmin) > i;
    const unsigned long long m = __ballot(above);
    if (m == 0ull) {
      lo = lo + h * 64.0;
    } else {
      const int first = __ffsll((long long)m) - 1;
      const double nhi = lo + h * (first + 1);
      lo = first == 0 ? lo : lo + h * first;
      hi = nhi;
    }
  }
  if (lane == 0) lam_asc[i] = 0.5 * (lo + hi);
}

// inverse iteration for eigenvalue i: solve (T - lam I) x = b by LU with partial pivoting
// (tridiagonal; the U factor has two superdiagonals). A workgroup of `tpw` threads handles tpw
// eigenvalues; d, e and the per-thread factor arrays live in LDS (interleaved by thread), so the
// sequential recurrences wait on LDS rather than global-memory latency.
constexpr int kInvArrays = 6;
__global__ __launch_bounds__(64) void invit_kernel(const double* __restrict__ d, const double* __restrict__ e, int n,
                                                   const double* __restrict__ lam_asc,
                                                   const double* __restrict__ tnorm, double drop_rel,
                                                   double* __restrict__ Z) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* sd = reinterpret_cast<double*>(smem_raw);
  double* se = sd + n;
  double* arr = se + n;
  const int tpw = blockDim.x;
  for (int j = threadIdx.x; j < n; j += tpw) {
    sd[j] = d[j];
    se[j] = j < n - 1 ? e[j] : 0.0;
  }
  __syncthreads();
  const int t = threadIdx.x;
  const int i = blockIdx.x * tpw + t;
  if (i >= n) return;
  const double lam = lam_asc[i];
  const double drop = drop_rel * (*tnorm);
#define W(k, j) arr[((int64_t)(k) * n + (j)) * tpw + t]
  enum { RINV = 0, U1 = 1, U2 = 2, ML = 3, Y = 4, SWP = 5 };
  if (lam < drop) {
    for (int j = 0; j < n; ++j) Z[(int64_t)j * n + i] = 0.0;
    return;
  }
  const double tiny = 2.220446049250313e-16 * fmax(*tnorm, 1e-300);
  // factorisation of T - lam I
  double a = sd[0] - lam, b = n > 1 ? se[0] : 0.0;
  for (int j = 0; j < n - 1; ++j) {
    const double c = se[j], dn = sd[j + 1] - lam, en = se[j + 1];
    double piv, m;
    if (fabs(a) >= fabs(c)) {
      piv = a;
      m = a != 0.0 ? c / a : 0.0;
      W(U1, j) = b;
      W(U2, j) = 0.0;
      W(ML, j) = m;
      a = dn - m * b;
      b = en;
      W(SWP, j) = 0.0;
    } else {
      piv = c;
      m = a / c;
      W(U1, j) = dn;
      W(U2, j) = en;
      W(ML, j) = m;
      a = b - m * dn;
      b = -m * en;
      W(SWP, j) = 1.0;
    }
    if (fabs(piv) < tiny) piv = piv < 0.0 ? -tiny : tiny;
    W(RINV, j) = 1.0 / piv;
  }
  if (fabs(a) < tiny) a = a < 0.0 ? -tiny : tiny;
  W(RINV, n - 1) = 1.0 / a;
  // start vector: deterministic pseudo-random entries in [0.5, 1.5)
  unsigned h = 2166136261u ^ ((unsigned)i * 16777619u);
  double scale = 1.0;
  for (int it = 0; it < 2; ++it) {
    // forward sweep (interchanges + multipliers) writes y; carry the running entry in a register
    double carry;
    if (it == 0) {
      h = (h ^ 0u) * 16777619u + 0x9E3779B9u;
      carry = 0.5 + (double)(h >> 8) * (1.0 / 16777216.0);
    } else {
      carry = W(Y, 0) * scale;
    }
    for (int j = 0; j < n - 1; ++j) {
      double nxt;
      if (it == 0) {
        h = (h ^ (unsigned)(j + 1)) * 16777619u + 0x9E3779B9u;
        nxt = 0.5 + (double)(h >> 8) * (1.0 / 16777216.0);
      } else {
        nxt = W(Y, j + 1) * scale;
      }
      const bool swp = W(SWP, j) != 0.0;
      const double x0 = swp ? nxt : carry, x1 = swp ? carry : nxt;
      W(Y, j) = x0;
      carry = x1 - W(ML, j) * x0;
    }
    W(Y, n - 1) = carry;
    // backward substitution with U, in place on y; track the max-norm for scaling
    double x1 = 0.0, x2 = 0.0, nrm = 0.0;
    for (int j = n - 1; j >= 0; --j) {
      const double x = (W(Y, j) - W(U1, j) * x1 - W(U2, j) * x2) * W(RINV, j);
      W(Y, j) = x;
      x2 = x1;
      x1 = x;
      nrm = fmax(nrm, fabs(x));
    }
    scale = nrm > 0.0 ? 1.0 / nrm : 0.0;
  }
  double nrm2 = 0.0;
  for (int j = 0; j < n; ++j) {
    const double v = W(Y, j) * scale;
    nrm2 += v * v;
  }
  const double s2 = nrm2 > 0.0 ? scale / sqrt(nrm2) : 0.0;
  for (int j = 0; j < n; ++j) Z[(int64_t)j * n + i] = W(Y, j) * s2;
#undef W
}

// modified Gram-Schmidt within each cluster of close eigenvalues (one workgroup per cluster start)
__global__ void cluster_mgs_kernel(const double* __restrict__ lam_asc, int n, const double* __restrict__ tnorm,
                                   double drop_rel, double* __restrict__ Z) {
  __shared__ double red[4];
  const int s0 = blockIdx.x;
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

// Back-transformation V = H_0 H_1 ... H_{n-3} Z with the reflectors taken kNb at a time in compact
// WY form: H_k0 ... H_k1 = I - Y T Y^T (Y = [v_k0 .. v_k1], T upper triangular, built as in the
// forward-accumulation recurrence T[i][i] = tau_i, T[0:i, i] = -tau_i T[0:i, 0:i] Y[:, 0:i]^T v_i).
constexpr int kWy = 16;   // reflectors per block
constexpr int kNC = 8;    // eigenvector columns per workgroup

// T of every block of wy (<= kWy) reflectors (one workgroup per block), stored kWy x kWy per block
__global__ __launch_bounds__(256) void wy_t_kernel(const double* __restrict__ V, const double* __restrict__ tau, int n,
                                                   int wy, double* __restrict__ Tall) {
  const int nref = n - 2;
  const int k0 = blockIdx.x * wy;
  const int m = min(wy, nref - k0);
  __shared__ double Gm[kWy][kWy];
  __shared__ double Ts[kWy][kWy];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  // Gm[a][i] = v_{k0+a} . v_{k0+i} for a < i (one wave per pair)
  for (int q = wid; q < kWy * kWy; q += nw) {
    const int a = q / kWy, i = q % kWy;
    double acc = 0.0;
    if (a < i && i < m) {
      const double* va = V + (int64_t)(k0 + a) * n;
      const double* vi = V + (int64_t)(k0 + i) * n;
      for (int j = k0 + i + 1 + lane; j < n; j += 64) acc += va[j] * vi[j];
      acc = wave_sum(acc);
    }
    if (lane == 0) Gm[a][i] = acc;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 0; i < kWy; ++i)
      for (int a = 0; a < kWy; ++a) Ts[a][i] = 0.0;
    for (int i = 0; i < m; ++i) {
      const double t = tau[k0 + i];
      for (int a = 0; a < i; ++a) {
        double acc = 0.0;
        for (int b = a; b < i; ++b) acc += Ts[a][b] * Gm[b][i];
        Ts[a][i] = -t * acc;
      }
      Ts[i][i] = t;
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < kWy * kWy; e += blockDim.x) Tall[(int64_t)blockIdx.x * kWy * kWy + e] = (&Ts[0][0])[e];
}

// kNC columns of Z per workgroup: for each block of wy reflectors from the last, the block's
// reflectors are staged in LDS and Z <- Z - Y (T (Y^T Z)); then the columns are written as
// eigenvector rows in descending eigenvalue order (dropped pairs as zeros)
__global__ __launch_bounds__(256) void backtransform_kernel(const double* __restrict__ Z, const double* __restrict__ V,
                                                            const double* __restrict__ Tall, int wy,
                                                            const double* __restrict__ lam_asc, int n,
                                                            const double* __restrict__ tnorm, double drop_rel,
                                                            double* __restrict__ evals_desc,
                                                            double* __restrict__ evec_rows) {
  const double drop = drop_rel * (*tnorm);
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* zc = reinterpret_cast<double*>(smem_raw);  // kNC x n
  double* Ys = zc + (size_t)kNC * n;                 // wy x n
  __shared__ double W[kWy][kNC];
  __shared__ double S[kWy][kNC];
  __shared__ double Ts[kWy * kWy];
  const int c0 = blockIdx.x * kNC;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int c = 0; c < kNC; ++c)
    for (int j = threadIdx.x; j < n; j += blockDim.x) zc[c * n + j] = (c0 + c < n) ? Z[(int64_t)j * n + c0 + c] : 0.0;
  const int nref = n - 2;
  const int nblk = nref > 0 ? (nref + wy - 1) / wy : 0;
  for (int b = nblk - 1; b >= 0; --b) {
    const int k0 = b * wy;
    const int m = min(wy, nref - k0);
    __syncthreads();
    // the block's reflectors and T factor into LDS (all loads of a thread issued before its stores)
    for (int e = threadIdx.x; e < kWy * kWy; e += blockDim.x) Ts[e] = Tall[(int64_t)b * kWy * kWy + e];
    for (int j0 = threadIdx.x; j0 < n; j0 += blockDim.x) {
      double yv[kWy];
#pragma unroll
      for (int i = 0; i < kWy; ++i) yv[i] = i < m ? V[(int64_t)(k0 + i) * n + j0] : 0.0;
#pragma unroll
      for (int i = 0; i < kWy; ++i)
        if (i < m) Ys[i * n + j0] = yv[i];
    }
    __syncthreads();
    // W = Y^T Z (one wave per (reflector, column) pair); v_k is zero at and above row k
    for (int q = wid; q < wy * kNC; q += nw) {
      const int i = q / kNC, c = q % kNC;
      double acc = 0.0;
      if (i < m) {
        for (int j = k0 + i + 1 + lane; j < n; j += 64) acc += Ys[i * n + j] * zc[c * n + j];
        acc = wave_sum(acc);
      }
      if (lane == 0) W[i][c] = acc;
    }
    __syncthreads();
    // S = T W
    if (threadIdx.x < wy * kNC) {
      const int i = threadIdx.x / kNC, c = threadIdx.x % kNC;
      double acc = 0.0;
      if (i < m)
        for (int a = i; a < m; ++a) acc += Ts[i * kWy + a] * W[a][c];
      S[i][c] = acc;
    }
    __syncthreads();
    // Z -= Y S
    for (int j = k0 + 1 + threadIdx.x; j < n; j += blockDim.x) {
      double acc[kNC];
#pragma unroll
      for (int c = 0; c < kNC; ++c) acc[c] = 0.0;
      for (int i = 0; i < m; ++i) {
        const double y = j > k0 + i ? Ys[i * n + j] : 0.0;
#pragma unroll
        for (int c = 0; c < kNC; ++c) acc[c] += y * S[i][c];
      }
#pragma unroll
      for (int c = 0; c < kNC; ++c) zc[c * n + j] -= acc[c];
    }
  }
  __syncthreads();
  for (int c = 0; c < kNC; ++c) {
    const int col = c0 + c;
    if (col >= n) break;
    const int out = n - 1 - col;  // descending order
    const double lam = lam_asc[col];
    const bool keep = lam >= drop;
    if (threadIdx.x == 0) evals_desc[out] = keep ? lam : 0.0;
    for (int j = threadIdx.x; j < n; j += blockDim.x) evec_rows[(int64_t)out * n + j] = keep ? zc[c * n + j] : 0.0;
  }
}

// The same back-transformation on the FP64 matrix cores, for n <= kBtMaxN. A workgroup owns 16
// columns of Z, held in registers as 16 x 16 accumulator tiles (tile t = rows 16t .. 16t+15, tiles
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

__device__ __forceinline__ bt_d4 mfma64(double a, double b, bt_d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__global__ __launch_bounds__(64 * kBtWaves) void backtransform_mfma_kernel(
    const double* __restrict__ Z, const double* __restrict__ V, const double* __restrict__ Tall,
    const double* __restrict__ lam_asc, int n, const double* __restrict__ tnorm, double drop_rel,
    double* __restrict__ evals_desc, double* __restrict__ evec_rows) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int nt = (n + 15) / 16;
  const int ldy = nt * 16 + 1;  // odd pitch: the 16 reflector rows fall in distinct LDS banks
  double* Ys = reinterpret_cast<double*>(smem_raw);  // kWy x ldy
  double* Wp = Ys + (size_t)kWy * ldy;              // kBtWaves x 256 partial W
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
      acc[i][r] = (t < nt && row < n && col < n) ? Z[(int64_t)row * n + col] : 0.0;
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
#pragma unroll
    for (int r = 0; r < 4; ++r) Wp[wid * 256 + (lq + 4 * r) * 16 + lr] = w[r];
    __syncthreads();
    // W summed over the waves in a fixed order, each entry by one thread
    if (threadIdx.x < 256) {
      double wsum = 0.0;
      for (int q = 0; q < kBtWaves; ++q) wsum += Wp[q * 256 + threadIdx.x];
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
  // eigenvector rows in descending eigenvalue order; dropped pairs as (0, zero vector)
  const double drop = drop_rel * (*tnorm);
  const bool keep = col < n && lam_asc[col] >= drop;
  if (wid == 0 && lq == 0 && col < n) evals_desc[n - 1 - col] = keep ? lam_asc[col] : 0.0;
  if (col < n) {
#pragma unroll
    for (int i = 0; i < kBtTiles; ++i) {
      const int t = wid + i * kBtWaves;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * t + lq + 4 * r;
        if (t < nt && row < n) evec_rows[(int64_t)(n - 1 - col) * n + row] = keep ? acc[i][r] : 0.0;
      }
    }
  }
}

// Workspace layout (doubles unless noted): A1, V, Z (n^2 each), wk (5 n^2), d, e, tau (n each),
// p (2 n), e2, lam (n each), tnorm (8), the per-workgroup barrier flags (256 unsigned) and the error word, then
// the T factors of the reflector blocks.
struct EigWs {
  double *A1, *V, *Z, *wk, *dvec, *evec, *tau, *pbuf, *e2, *lam, *tnorm, *Tall;
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
    pbuf = tau + n;
    e2 = pbuf + 2 * n;
    lam = e2 + n;
    tnorm = lam + n;
    flags = reinterpret_cast<unsigned*>(tnorm + 8);
    err = reinterpret_cast<int*>(flags + 256);
    Tall = tnorm + 8 + 130;  // 256 unsigned + err word, rounded up to doubles
    const size_t nblk = (size_t)n + 1;  // blocks of as few as one reflector
    bytes = (size_t)((Tall + nblk * kWy * kWy) - w) * sizeof(double);
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
  // as few workgroups as hold the rows (at most kTrWaves * kTrRows each): the barrier's cost grows
  // with the number of workgroups
  const int per = kTrWaves * kTrRows;
  const int blocks = (ta.n + per - 1) / per;
  NGD_TRY(check_coresident((const void*)tridiag_reg_kernel<QN>, kTrThreads, 0, blocks));
  hipLaunchKernelGGL(tridiag_reg_kernel<QN>, dim3(blocks), dim3(kTrThreads), 0, s, ta);
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
  // larger n: rows in LDS, enough workgroups that each one's rows fit next to four n-vectors
  int blocks = kTriBlocks;
  auto lds_for = [&](int G) { return sizeof(double) * ((size_t)((n + G - 1) / G) * n + 4 * (size_t)n); };
  while (lds_for(blocks) > 144 * 1024 && blocks < 256) blocks *= 2;
  const size_t lds = lds_for(blocks);
  if (lds > 144 * 1024) {
    set_error("ell too large for the LDS-resident tridiagonalisation");
    return NGD_ERR_INVALID;
  }
  NGD_HIP_TRY(hipFuncSetAttribute((const void*)tridiag_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  NGD_TRY(check_coresident((const void*)tridiag_kernel, kTriThreads, lds, blocks));
  hipLaunchKernelGGL(tridiag_kernel, dim3(blocks), dim3(kTriThreads), lds, s, ta);
  NGD_HIP_TRY(hipGetLastError());
  return NGD_OK;
}

}  // namespace

size_t eig_workspace_bytes(int n) { return EigWs(nullptr, n).bytes; }

ngd_status launch_sym_eig(double* A, int n, double drop_rel, double* evals_desc, double* evec_rows, void* work,
                               hipStream_t s) {
  if (n <= 0) return NGD_OK;
  EigWs ws(work, n);
  double* A1 = ws.A1;
  double* V = ws.V;
  double* Z = ws.Z;
  double* wk = ws.wk;
  double* dvec = ws.dvec;
  double* evec = ws.evec;
  double* tau = ws.tau;
  double* pbuf = ws.pbuf;
  double* e2 = ws.e2;
  double* lam = ws.lam;
  double* tnorm = ws.tnorm;
  unsigned* bar = ws.flags;
  int* err = ws.err;
  {
    ngd_status st = launch_zero(bar, 256 * sizeof(unsigned) + sizeof(int), s);
    if (st != NGD_OK) return st;
    st = launch_zero(tau, sizeof(double) * n, s);
    if (st != NGD_OK) return st;
  }
  TriArgs ta{A, A1, n, dvec, evec, V, tau, pbuf, bar, err};
  NGD_TRY(launch_tridiag(ta, s));
  const int tb = 256;
  hipLaunchKernelGGL(bisect_kernel, dim3((n + 3) / 4), dim3(tb), 2 * sizeof(double) * n, s, dvec, evec, n, e2,
                     lam, tnorm);
  {
    // as many eigenvalues per workgroup as fit: (2 + 6 tpw) n doubles of LDS
    int tpw = (int)((150 * 1024 / sizeof(double) - 2 * (size_t)n) / ((size_t)kInvArrays * n));
    tpw = tpw > 64 ? 64 : tpw;
    if (tpw < 1) {
      set_error("ell too large for inverse iteration in LDS");
      return NGD_ERR_INVALID;
    }
    const size_t lds = sizeof(double) * ((size_t)2 * n + (size_t)kInvArrays * n * tpw);
    NGD_HIP_TRY(hipFuncSetAttribute((const void*)invit_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL(invit_kernel, dim3((n + tpw - 1) / tpw), dim3(tpw), lds, s, dvec, evec, n, lam, tnorm,
                       drop_rel, Z);
  }
  hipLaunchKernelGGL(cluster_mgs_kernel, dim3(n), dim3(256), 0, s, lam, n, tnorm, drop_rel, Z);
  NGD_HIP_TRY(hipGetLastError());
  // one Newton-Schulz step Z <- 1.5 Z - 0.5 Z (Z^T Z) removes the residual non-orthogonality of the
  // inverse-iteration vectors (quadratic convergence; dropped columns stay zero)
  double* E = A1;   // free after the tridiagonalisation
  double* Z2 = wk;  // free after inverse iteration
  double* nswork = wk + (size_t)n * n;  // split-K partials of the n x n products (4 n^2)
  for (int ns = 0; ns < 2; ++ns) {
    GemmArgs e{n, n, n, Z, n, false, Z, n, false, E, n, NGD_F64, NGD_F64, NGD_F64, G_F64, 1.0, 0.0,
               nswork, 4 * (int64_t)n * n};
    ngd_status st = launch_gemm(e, s);
    if (st != NGD_OK) return st;
    st = launch_cast(NGD_F64, Z, NGD_F64, Z2, (int64_t)n * n, s);
    if (st != NGD_OK) return st;
    GemmArgs u{n, n, n, Z, n, true, E, n, false, Z2, n, NGD_F64, NGD_F64, NGD_F64, G_F64, -0.5, 1.5,
               nswork, 4 * (int64_t)n * n};
    st = launch_gemm(u, s);
    if (st != NGD_OK) return st;
    double* t = Z;
    Z = Z2;
    Z2 = t;
  }
  // T factors of the reflector blocks (written over the multipliers of inverse iteration, free now)
  double* Tall = ws.Tall;
  if (n <= kBtMaxN) {
    const int nblk = n > 2 ? (n - 2 + kWy - 1) / kWy : 0;
    if (nblk > 0) hipLaunchKernelGGL(wy_t_kernel, dim3(nblk), dim3(256), 0, s, V, tau, n, kWy, Tall);
    const int nt = (n + 15) / 16;
    const size_t lds = sizeof(double) * ((size_t)kWy * (nt * 16 + 1) + (size_t)kBtWaves * 256);
    NGD_HIP_TRY(hipFuncSetAttribute((const void*)backtransform_mfma_kernel,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL(backtransform_mfma_kernel, dim3(nt), dim3(64 * kBtWaves), lds, s, Z, V, Tall, lam, n, tnorm,
                       drop_rel, evals_desc, evec_rows);
    NGD_HIP_TRY(hipGetLastError());
    return NGD_OK;
  }
  // reflectors per block: as many as fit in LDS beside the kNC columns
  int wy = kWy;
  while (wy > 1 && (size_t)(kNC + wy) * n * sizeof(double) > 150 * 1024) wy >>= 1;
  const size_t bt_lds = (size_t)(kNC + wy) * n * sizeof(double);
  if (bt_lds > 150 * 1024) {
    set_error("ell too large for the back-transformation's LDS budget");
    return NGD_ERR_INVALID;
  }
  const int nblk = n > 2 ? (n - 2 + wy - 1) / wy : 0;
  if (nblk > 0) hipLaunchKernelGGL(wy_t_kernel, dim3(nblk), dim3(256), 0, s, V, tau, n, wy, Tall);
  NGD_HIP_TRY(hipFuncSetAttribute((const void*)backtransform_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)bt_lds));
  hipLaunchKernelGGL(backtransform_kernel, dim3((n + kNC - 1) / kNC), dim3(256), bt_lds, s, Z, V, Tall, wy, lam, n,
                     tnorm, drop_rel, evals_desc, evec_rows);
  NGD_HIP_TRY(hipGetLastError());
  return NGD_OK;
}

const int* eig_error_flag(void* work, int n) { return EigWs(work, n).err; }

}  // namespace ngd
