// FP64 symmetric eigendecomposition of the small ell x ell matrices of the Nystrom core.
//
// Alg. 6 needs the thin SVD of the p x ell matrix B; its right singular vectors and squared
// singular values are the eigenpairs of the ell x ell Gram matrix B^T B, computed here in FP64:
//  1. Householder tridiagonalisation Q^T A Q = T in one cooperative launch. The trailing matrix is
//     row-distributed over the workgroups; each step applies the previous step's rank-2 update
//     lazily while forming p = tau A v, so one grid barrier per column suffices.
//  2. Eigenvalues of T by bisection on Sturm counts (one thread per eigenvalue).
//  3. Eigenvectors of T by inverse iteration with partial-pivoting LU of T - lambda I (one thread
//     per eigenvector), then modified Gram-Schmidt inside clusters of close eigenvalues.
//  4. Back-transformation V = H_0 H_1 ... H_{n-3} Z (one workgroup per group of columns).
// Eigenpairs whose eigenvalue is below drop_rel * (Gershgorin bound of T) are returned as
// (0, zero vector).
#include "common.h"

namespace ngd {
namespace {

constexpr int kTriBlocks = 64;
constexpr int kTriThreads = 256;

struct TriArgs {
  double* A0;      // input matrix (n x n, ld n); used as ping buffer
  double* A1;      // pong buffer
  int n;
  double* d;       // diagonal of T
  double* e;       // off-diagonal of T (n-1)
  double* V;       // Householder vectors, row k = v_k (support k+1..n-1, v_k[k+1] = 1)
  double* tau;     // Householder scalars
  double* p;       // n: p = tau A v of the current step
  unsigned* bar;   // [0] arrival count, [1] generation
  int* err;
};

__device__ bool grid_sync(unsigned* bar, int* err) {
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned gen = __hip_atomic_load(bar + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __threadfence();
    unsigned arrived = atomicAdd(bar, 1u);
    if (arrived == gridDim.x - 1) {
      __hip_atomic_store(bar, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __threadfence();
      atomicAdd(bar + 1, 1u);
    } else {
      long spins = 0;
      while (__hip_atomic_load(bar + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gen) {
        __builtin_amdgcn_s_sleep(1);
        if (++spins > (1L << 25)) {  // a few seconds: give up instead of hanging
          atomicExch(err, 1);
          break;
        }
      }
    }
    __threadfence();
  }
  __syncthreads();
  return __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0;
}

__global__ __launch_bounds__(kTriThreads) void tridiag_kernel(TriArgs a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int n = a.n;
  double* vprev = reinterpret_cast<double*>(smem_raw);
  double* wprev = vprev + n;
  double* v = wprev + n;
  __shared__ double red[8];
  __shared__ double sh_tau;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int j = threadIdx.x; j < n; j += blockDim.x) vprev[j] = wprev[j] = 0.0;
  __syncthreads();
  double* cur = a.A0;
  double* nxt = a.A1;
  for (int k = 0; k + 2 < n; ++k) {
    // column k of A^(k) below the diagonal (pending rank-2 update applied), into v
    double tail = 0.0;
    for (int j = k + 1 + threadIdx.x; j < n; j += blockDim.x) {
      double x = cur[(int64_t)k * n + j] - vprev[k] * wprev[j] - wprev[k] * vprev[j];
      v[j] = x;
      if (j > k + 1) tail += x * x;
    }
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
    if (blockIdx.x == 0) {
      if (threadIdx.x == 0) {
        a.d[k] = cur[(int64_t)k * n + k] - 2.0 * vprev[k] * wprev[k];
        a.e[k] = beta;
        a.tau[k] = tau;
      }
      for (int j = threadIdx.x; j < n; j += blockDim.x) a.V[(int64_t)k * n + j] = j > k ? v[j] : 0.0;
    }
    // own rows: write the updated row to nxt and p_i = tau * row . v (one wave per row)
    for (int i = k + 1 + blockIdx.x * nw + wid; i < n; i += gridDim.x * nw) {
      const double vi = vprev[i], wi = wprev[i];
      const double* src = cur + (int64_t)i * n;
      double* dst = nxt + (int64_t)i * n;
      double acc = 0.0;
      for (int j = k + 1 + lane; j < n; j += 64) {
        double x = src[j] - vi * wprev[j] - wi * vprev[j];
        dst[j] = x;
        acc += x * v[j];
      }
      acc = wave_sum(acc);
      if (lane == 0) a.p[i] = tau * acc;
    }
    if (!grid_sync(a.bar, a.err)) return;
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
    double* t = cur;
    cur = nxt;
    nxt = t;
  }
  // last 2 x 2 (or 1 x 1) block with the pending update
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    const int m = n >= 2 ? n - 2 : 0;
    if (n >= 2) {
      a.d[m] = cur[(int64_t)m * n + m] - 2.0 * vprev[m] * wprev[m];
      a.e[m] = cur[(int64_t)(m + 1) * n + m] - vprev[m + 1] * wprev[m] - wprev[m + 1] * vprev[m];
      a.d[m + 1] = cur[(int64_t)(m + 1) * n + m + 1] - 2.0 * vprev[m + 1] * wprev[m + 1];
    } else {
      a.d[0] = cur[0];
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
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double tn = fmax(fabs(lo_s), fabs(hi_s));
  const double pivmin = fmax(1e-300, 2.2250738585072014e-308 * fmax(1.0, tn * tn));
  double lo = lo_s - 1e-14 * tn - pivmin, hi = hi_s + 1e-14 * tn + pivmin;
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    if (hi - lo <= 2.0 * 2.220446049250313e-16 * fmax(fabs(lo), fabs(hi)) + pivmin) break;
    if (sturm_count(sd, se2, n, mid, pivmin) > i) hi = mid;
    else lo = mid;
  }
  lam_asc[i] = 0.5 * (lo + hi);
}

// inverse iteration for eigenvalue i: solve (T - lam I) x = b by LU with partial pivoting
// (tridiagonal; the U factor has two superdiagonals). Workspace is [row][n] interleaved by thread.
__global__ void invit_kernel(const double* __restrict__ d, const double* __restrict__ e, int n,
                             const double* __restrict__ lam_asc, const double* __restrict__ tnorm, double drop_rel,
                             double* __restrict__ Z, double* __restrict__ wk) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double lam = lam_asc[i];
  const double drop = drop_rel * (*tnorm);
  double* u0 = wk;                          // diagonal of U
  double* u1 = wk + (int64_t)n * n;         // first superdiagonal
  double* u2 = wk + 2 * (int64_t)n * n;     // second superdiagonal
  double* ml = wk + 3 * (int64_t)n * n;     // multipliers
  double* piv = wk + 4 * (int64_t)n * n;    // 1 if rows j, j+1 were swapped
#define W(arr, j) arr[(int64_t)(j) * n + i]
  if (lam < drop) {
    for (int j = 0; j < n; ++j) W(Z, j) = 0.0;
    return;
  }
  const double eps = 2.220446049250313e-16;
  const double tiny = eps * fmax(*tnorm, 1e-300);
  // factorisation
  double a = d[0] - lam, b = n > 1 ? e[0] : 0.0;
  for (int j = 0; j < n - 1; ++j) {
    const double c = e[j];                  // subdiagonal entry below the pivot
    const double dn = d[j + 1] - lam;       // next diagonal
    const double en = j + 1 < n - 1 ? e[j + 1] : 0.0;
    if (fabs(a) >= fabs(c)) {
      const double m = a != 0.0 ? c / a : 0.0;
      W(u0, j) = a;
      W(u1, j) = b;
      W(u2, j) = 0.0;
      W(ml, j) = m;
      W(piv, j) = 0.0;
      a = dn - m * b;
      b = en;
    } else {
      const double m = a / c;
      W(u0, j) = c;
      W(u1, j) = dn;
      W(u2, j) = en;
      W(ml, j) = m;
      W(piv, j) = 1.0;
      a = b - m * dn;
      b = -m * en;
    }
    if (fabs(W(u0, j)) < tiny) W(u0, j) = copysign(tiny, W(u0, j) == 0.0 ? 1.0 : W(u0, j));
  }
  if (fabs(a) < tiny) a = copysign(tiny, a == 0.0 ? 1.0 : a);
  W(u0, n - 1) = a;
  W(u1, n - 1) = 0.0;
  W(u2, n - 1) = 0.0;
  // start vector: deterministic pseudo-random entries in [0.5, 1.5)
  unsigned h = 2166136261u ^ (unsigned)i * 16777619u;
  for (int j = 0; j < n; ++j) {
    h = (h ^ (unsigned)j) * 16777619u + 0x9E3779B9u;
    W(Z, j) = 0.5 + (double)(h >> 8) * (1.0 / 16777216.0);
  }
  for (int it = 0; it < 3; ++it) {
    // forward: apply the row interchanges and multipliers
    for (int j = 0; j < n - 1; ++j) {
      double x0 = W(Z, j), x1 = W(Z, j + 1);
      if (W(piv, j) != 0.0) {
        double t = x0;
        x0 = x1;
        x1 = t;
      }
      W(Z, j) = x0;
      W(Z, j + 1) = x1 - W(ml, j) * x0;
    }
    // backward substitution with U
    double nrm = 0.0;
    for (int j = n - 1; j >= 0; --j) {
      double x = W(Z, j);
      if (j + 1 < n) x -= W(u1, j) * W(Z, j + 1);
      if (j + 2 < n) x -= W(u2, j) * W(Z, j + 2);
      x /= W(u0, j);
      W(Z, j) = x;
      nrm = fmax(nrm, fabs(x));
    }
    const double s = nrm > 0.0 ? 1.0 / nrm : 0.0;
    for (int j = 0; j < n; ++j) W(Z, j) *= s;
  }
  double nrm2 = 0.0;
  for (int j = 0; j < n; ++j) nrm2 += W(Z, j) * W(Z, j);
  const double s = nrm2 > 0.0 ? 1.0 / sqrt(nrm2) : 0.0;
  for (int j = 0; j < n; ++j) W(Z, j) *= s;
#undef W
}

// modified Gram-Schmidt within each cluster of close eigenvalues (one workgroup per cluster start)
__global__ void cluster_mgs_kernel(const double* __restrict__ lam_asc, int n, const double* __restrict__ tnorm,
                                   double drop_rel, double* __restrict__ Z) {
  __shared__ double red[4];
  const int s0 = blockIdx.x;
  const double drop = drop_rel * (*tnorm);
  const double tol = 1e-8 * (*tnorm);
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
  int blocks = n < kTriBlocks ? (n < 1 ? 1 : n) : kTriBlocks;
  size_t lds = 3 * sizeof(double) * (size_t)n;
  NGD_HIP_TRY(hipFuncSetAttribute((const void*)tridiag_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  void* args[] = {&ta};
  NGD_HIP_TRY(hipLaunchCooperativeKernel((const void*)tridiag_kernel, dim3(blocks), dim3(kTriThreads), args, lds, s));
  const int tb = 256;
  hipLaunchKernelGGL(bisect_kernel, dim3((n + tb - 1) / tb), dim3(tb), 2 * sizeof(double) * n, s, dvec, evec, n, e2,
                     lam, tnorm);
  hipLaunchKernelGGL(invit_kernel, dim3((n + 63) / 64), dim3(64), 0, s, dvec, evec, n, lam, tnorm, drop_rel, Z, wk);
  hipLaunchKernelGGL(cluster_mgs_kernel, dim3(n), dim3(256), 0, s, lam, n, tnorm, drop_rel, Z);
  NGD_HIP_TRY(hipGetLastError());
  // one Newton-Schulz step Z <- 1.5 Z - 0.5 Z (Z^T Z) removes the residual non-orthogonality of the
  // inverse-iteration vectors (quadratic convergence; dropped columns stay zero)
  double* E = A1;   // free after the tridiagonalisation
  double* Z2 = wk;  // free after inverse iteration
  {
    GemmArgs e{n, n, n, Z, n, false, Z, n, false, E, n, NGD_F64, NGD_F64, NGD_F64, G_F64, 1.0, 0.0};
    ngd_status st = launch_gemm(e, s);
    if (st != NGD_OK) return st;
    st = launch_cast(NGD_F64, Z, NGD_F64, Z2, (int64_t)n * n, s);
    if (st != NGD_OK) return st;
    GemmArgs u{n, n, n, Z, n, true, E, n, false, Z2, n, NGD_F64, NGD_F64, NGD_F64, G_F64, -0.5, 1.5};
    st = launch_gemm(u, s);
    if (st != NGD_OK) return st;
  }
  Z = Z2;
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
