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
  double* p;       // n: p = tau A v of the current step
  unsigned* bar;   // [0] arrival count, [1] generation
  int* err;
};

// Grid barrier number `epoch` (0, 1, 2, ...) on a counter that starts at 0 for the launch: every
// workgroup adds 1 and waits for (epoch + 1) * gridDim.x arrivals. One agent-scope release fence
// before arriving and one acquire fence after the wait (each is an L2 write-back or invalidate on
// this GPU, so they are kept to the minimum). The wait is bounded: on timeout it raises `err`.
__device__ bool grid_sync(unsigned* count, unsigned epoch, int* err) {
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned target = (epoch + 1u) * gridDim.x;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __hip_atomic_fetch_add(count, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    long spins = 0;
    while (__hip_atomic_load(count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      __builtin_amdgcn_s_sleep(1);
      if (++spins > (1L << 25)) {  // a few seconds: give up instead of hanging
        __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
  return __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0;
}

// One Householder step per column k, rows of the trailing matrix resident in LDS: workgroup g owns
// rows i = g, g + G, g + 2G, ... Each step applies the previous step's rank-2 update (v, w) to the
// owned rows in place, forms p_i = tau A_i . v, and the owner of row k+1 publishes that updated row
// (the next pivot row) to global memory. After one grid barrier every workgroup reads p and the
// pivot row, forms w = p - (tau/2)(p . v) v and, from the pivot row, the next Householder vector.
__global__ __launch_bounds__(kTriThreads) void tridiag_kernel(TriArgs a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int n = a.n, G = gridDim.x, g = blockIdx.x;
  const int R = (n + G - 1) / G;  // rows per workgroup
  double* rows = reinterpret_cast<double*>(smem_raw);   // R x n
  double* vprev = rows + (size_t)R * n;
  double* wprev = vprev + n;
  double* v = wprev + n;
  __shared__ double red[8];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int r = 0; r < R; ++r) {
    const int i = g + r * G;
    for (int j = threadIdx.x; j < n; j += blockDim.x) rows[(size_t)r * n + j] = i < n ? a.A0[(int64_t)i * n + j] : 0.0;
  }
  for (int j = threadIdx.x; j < n; j += blockDim.x) vprev[j] = wprev[j] = 0.0;
  __syncthreads();
  const double* pivot = a.A0;  // step 0: row 0 of A, no pending update
  for (int k = 0; k + 2 < n; ++k) {
    // column k of A^(k) below the diagonal = pivot row k with the pending update applied
    double tail = 0.0;
    const double vk = vprev[k], wk = wprev[k];
    for (int j = k + 1 + threadIdx.x; j < n; j += blockDim.x) {
      const double x = pivot[j] - vk * wprev[j] - wk * vprev[j];
      v[j] = x;
      if (j > k + 1) tail += x * x;
    }
    const double dk = pivot[k] - 2.0 * vk * wk;
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
      if (lane == 0) a.p[i] = tau * acc;
    }
    if (!grid_sync(a.bar, (unsigned)k, a.err)) return;
    // w = p - (tau/2)(p . v) v, kept by every workgroup as the pending update
    double pv = 0.0;
    for (int j = k + 1 + threadIdx.x; j < n; j += blockDim.x) pv += a.p[j] * v[j];
    pv = block_sum(pv, red);
    const double c = 0.5 * tau * pv;
    __syncthreads();
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
      if (j > k) {
        wprev[j] = a.p[j] - c * v[j];
        vprev[j] = v[j];
      } else {
        wprev[j] = 0.0;
        vprev[j] = 0.0;
      }
    }
    __syncthreads();
    pivot = next_pivot;
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

__device__ int sturm_count(const double* d, const double* e2, int n, double x, double pivmin) {
  int cnt = 0;
  double q = d[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  if (q < 0) ++cnt;
  for (int i = 1; i < n; ++i) {
    q = d[i] - x - e2[i - 1] / q;
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
// (tridiagonal; the U factor has two superdiagonals). Per-thread arrays are interleaved by thread
// ([row][n]) so a wave's accesses are coalesced; the recurrences carry their values in registers
// and every load address is known in advance, so the loads pipeline.
__global__ __launch_bounds__(64) void invit_kernel(const double* __restrict__ d, const double* __restrict__ e, int n,
                                                   const double* __restrict__ lam_asc,
                                                   const double* __restrict__ tnorm, double drop_rel,
                                                   double* __restrict__ Z, double* __restrict__ wk) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double lam = lam_asc[i];
  const double drop = drop_rel * (*tnorm);
  const int64_t nn = (int64_t)n * n;
  double* __restrict__ rinv = wk;           // 1 / diagonal of U
  double* __restrict__ u1 = wk + nn;        // first superdiagonal
  double* __restrict__ u2 = wk + 2 * nn;    // second superdiagonal
  double* __restrict__ ml = wk + 3 * nn;    // multipliers; sign bit = row interchange
  double* __restrict__ y = wk + 4 * nn;     // right-hand side after the forward sweep
#define W(arr, j) arr[(int64_t)(j) * n + i]
  if (lam < drop) {
    for (int j = 0; j < n; ++j) W(Z, j) = 0.0;
    return;
  }
  const double tiny = 2.220446049250313e-16 * fmax(*tnorm, 1e-300);
  // factorisation of T - lam I
  double a = d[0] - lam, b = n > 1 ? e[0] : 0.0;
  for (int j = 0; j < n - 1; ++j) {
    const double c = e[j], dn = d[j + 1] - lam, en = j + 1 < n - 1 ? e[j + 1] : 0.0;
    double piv, m;
    if (fabs(a) >= fabs(c)) {
      piv = a;
      m = a != 0.0 ? c / a : 0.0;
      W(u1, j) = b;
      W(u2, j) = 0.0;
      W(ml, j) = m;          // no interchange: stored as is (flag in a separate sign convention below)
      a = dn - m * b;
      b = en;
      W(y, j) = 0.0;         // y doubles as the interchange flag during factorisation
    } else {
      piv = c;
      m = a / c;
      W(u1, j) = dn;
      W(u2, j) = en;
      W(ml, j) = m;
      a = b - m * dn;
      b = -m * en;
      W(y, j) = 1.0;
    }
    if (fabs(piv) < tiny) piv = piv < 0.0 ? -tiny : tiny;
    W(rinv, j) = 1.0 / piv;
  }
  if (fabs(a) < tiny) a = a < 0.0 ? -tiny : tiny;
  W(rinv, n - 1) = 1.0 / a;
  // interchange flags: keep them in the sign-free array `u2`'s companion by reusing Z as scratch
  for (int j = 0; j < n - 1; ++j) W(Z, j) = W(y, j);
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
      carry = W(y, 0) * scale;
    }
    for (int j = 0; j < n - 1; ++j) {
      double nxt;
      if (it == 0) {
        h = (h ^ (unsigned)(j + 1)) * 16777619u + 0x9E3779B9u;
        nxt = 0.5 + (double)(h >> 8) * (1.0 / 16777216.0);
      } else {
        nxt = W(y, j + 1) * scale;
      }
      const bool swp = W(Z, j) != 0.0;
      const double x0 = swp ? nxt : carry, x1 = swp ? carry : nxt;
      W(y, j) = x0;
      carry = x1 - W(ml, j) * x0;
    }
    W(y, n - 1) = carry;
    // backward substitution with U, in place on y; track the max-norm for scaling
    double x1 = 0.0, x2 = 0.0, nrm = 0.0;
    for (int j = n - 1; j >= 0; --j) {
      const double x = (W(y, j) - W(u1, j) * x1 - W(u2, j) * x2) * W(rinv, j);
      W(y, j) = x;
      x2 = x1;
      x1 = x;
      nrm = fmax(nrm, fabs(x));
    }
    scale = nrm > 0.0 ? 1.0 / nrm : 0.0;
  }
  double nrm2 = 0.0;
  for (int j = 0; j < n; ++j) {
    const double v = W(y, j) * scale;
    nrm2 += v * v;
  }
  const double s2 = nrm2 > 0.0 ? scale / sqrt(nrm2) : 0.0;
  for (int j = 0; j < n; ++j) W(Z, j) = W(y, j) * s2;
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

// V = H_0 ... H_{n-3} Z for NC columns per workgroup; writes eigenvector rows in descending order
constexpr int kNC = 4;
__global__ __launch_bounds__(256) void backtransform_kernel(const double* __restrict__ Z, const double* __restrict__ V,
                                                            const double* __restrict__ tau,
                                                            const double* __restrict__ lam_asc, int n,
                                                            const double* __restrict__ tnorm, double drop_rel,
                                                            double* __restrict__ evals_desc,
                                                            double* __restrict__ evec_rows) {
  const double drop = drop_rel * (*tnorm);
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* zc = reinterpret_cast<double*>(smem_raw);  // kNC x n
  __shared__ double red[kNC][4];
  const int c0 = blockIdx.x * kNC;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int c = 0; c < kNC; ++c)
    for (int j = threadIdx.x; j < n; j += blockDim.x)
      zc[c * n + j] = (c0 + c < n) ? Z[(int64_t)j * n + c0 + c] : 0.0;
  __syncthreads();
  for (int k = n - 3; k >= 0; --k) {
    const double t = tau[k];
    if (t == 0.0) continue;
    const double* vk = V + (int64_t)k * n;
    double s[kNC];
    for (int c = 0; c < kNC; ++c) s[c] = 0.0;
    for (int j = k + 1 + threadIdx.x; j < n; j += blockDim.x) {
      const double vj = vk[j];
      for (int c = 0; c < kNC; ++c) s[c] += vj * zc[c * n + j];
    }
    for (int c = 0; c < kNC; ++c) {
      double w = wave_sum(s[c]);
      if (lane == 0) red[c][wid] = w;
    }
    __syncthreads();
    for (int c = 0; c < kNC; ++c) s[c] = t * (red[c][0] + red[c][1] + red[c][2] + red[c][3]);
    for (int j = k + 1 + threadIdx.x; j < n; j += blockDim.x) {
      const double vj = vk[j];
      for (int c = 0; c < kNC; ++c) zc[c * n + j] -= s[c] * vj;
    }
    __syncthreads();
  }
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

}  // namespace

size_t eig_workspace_bytes(int n) {
  // A1, V, Z (n*n each) + invit 5*n*n + vectors + barrier words
  return sizeof(double) * ((size_t)8 * n * n + 8 * (size_t)n + 64) + 64;
}

ngd_status launch_sym_eig(double* A, int n, double drop_rel, double* evals_desc, double* evec_rows, void* work,
                               hipStream_t s) {
  if (n <= 0) return NGD_OK;
  double* w = reinterpret_cast<double*>(work);
  double* A1 = w;
  double* V = A1 + (size_t)n * n;
  double* Z = V + (size_t)n * n;
  double* wk = Z + (size_t)n * n;           // 5 n^2
  double* dvec = wk + (size_t)5 * n * n;
  double* evec = dvec + n;
  double* tau = evec + n;
  double* pbuf = tau + n;
  double* e2 = pbuf + n;
  double* lam = e2 + n;
  double* tnorm = lam + n;
  unsigned* bar = reinterpret_cast<unsigned*>(tnorm + 8);
  int* err = reinterpret_cast<int*>(bar + 4);
  {
    ngd_status st = launch_zero(bar, 4 * sizeof(unsigned) + sizeof(int) + 4, s);
    if (st != NGD_OK) return st;
    st = launch_zero(tau, sizeof(double) * n, s);
    if (st != NGD_OK) return st;
  }
  TriArgs ta{A, A1, n, dvec, evec, V, tau, pbuf, bar, err};
  // workgroups: enough that each one's rows fit in LDS next to three n-vectors
  int blocks = n < kTriBlocks ? (n < 1 ? 1 : n) : kTriBlocks;
  auto lds_for = [&](int G) { return sizeof(double) * ((size_t)((n + G - 1) / G) * n + 3 * (size_t)n); };
  while (lds_for(blocks) > 144 * 1024 && blocks < 256) blocks *= 2;
  size_t lds = lds_for(blocks);
  if (lds > 144 * 1024) {
    set_error("ell too large for the LDS-resident tridiagonalisation");
    return NGD_ERR_INVALID;
  }
  NGD_HIP_TRY(hipFuncSetAttribute((const void*)tridiag_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  // The grid barrier needs every workgroup resident at once: `blocks` (<= 64) is far below the
  // device's CU count, and the check below confirms the occupancy; the barrier's wait is bounded
  // (it sets the error flag instead of spinning forever).
  {
    int dev = 0, cus = 0, per_cu = 0;
    NGD_HIP_TRY(hipGetDevice(&dev));
    NGD_HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    NGD_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)tridiag_kernel, kTriThreads, lds));
    if ((int64_t)cus * per_cu < blocks) {
      set_error("tridiagonalisation grid cannot be co-resident");
      return NGD_ERR_HIP;
    }
  }
  hipLaunchKernelGGL(tridiag_kernel, dim3(blocks), dim3(kTriThreads), lds, s, ta);
  const int tb = 256;
  hipLaunchKernelGGL(bisect_kernel, dim3((n + 3) / 4), dim3(tb), 2 * sizeof(double) * n, s, dvec, evec, n, e2,
                     lam, tnorm);
  hipLaunchKernelGGL(invit_kernel, dim3((n + 63) / 64), dim3(64), 0, s, dvec, evec, n, lam, tnorm, drop_rel, Z, wk);
  hipLaunchKernelGGL(cluster_mgs_kernel, dim3(n), dim3(256), 0, s, lam, n, tnorm, drop_rel, Z);
  NGD_HIP_TRY(hipGetLastError());
  // one Newton-Schulz step Z <- 1.5 Z - 0.5 Z (Z^T Z) removes the residual non-orthogonality of the
  // inverse-iteration vectors (quadratic convergence; dropped columns stay zero)
  double* E = A1;   // free after the tridiagonalisation
  double* Z2 = wk;  // free after inverse iteration
  for (int ns = 0; ns < 2; ++ns) {
    GemmArgs e{n, n, n, Z, n, false, Z, n, false, E, n, NGD_F64, NGD_F64, NGD_F64, G_F64, 1.0, 0.0};
    ngd_status st = launch_gemm(e, s);
    if (st != NGD_OK) return st;
    st = launch_cast(NGD_F64, Z, NGD_F64, Z2, (int64_t)n * n, s);
    if (st != NGD_OK) return st;
    GemmArgs u{n, n, n, Z, n, true, E, n, false, Z2, n, NGD_F64, NGD_F64, NGD_F64, G_F64, -0.5, 1.5};
    st = launch_gemm(u, s);
    if (st != NGD_OK) return st;
    double* t = Z;
    Z = Z2;
    Z2 = t;
  }
  NGD_HIP_TRY(hipFuncSetAttribute((const void*)backtransform_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)(kNC * n * sizeof(double))));
  hipLaunchKernelGGL(backtransform_kernel, dim3((n + kNC - 1) / kNC), dim3(256), kNC * n * sizeof(double), s, Z, V, tau,
                     lam, n, tnorm, drop_rel, evals_desc, evec_rows);
  NGD_HIP_TRY(hipGetLastError());
  return NGD_OK;
}

const int* eig_error_flag(void* work, int n) {
  double* w = reinterpret_cast<double*>(work);
  double* tnorm = w + (size_t)8 * n * n + 6 * (size_t)n;
  unsigned* bar = reinterpret_cast<unsigned*>(tnorm + 8);
  return reinterpret_cast<const int*>(bar + 4);
}

}  // namespace ngd
