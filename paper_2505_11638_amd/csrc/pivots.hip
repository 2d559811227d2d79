// Diagonal of the Gramian, pivot sampling proportional to a weight vector, and column gathers: the
// pieces of the sampling test matrix of the Nystrom approximation (Omega = columns of the identity at
// indices drawn with probability proportional to diag(G); Section 5, the "sampling" variant) and of
// RPCholesky (Section 4.2.2, its block algorithm in the appendix).
#include "common.h"

namespace ngd {
namespace {

// ---- diag(G) = column sums of squares of J_w (eq. gram_diagonal with the weights folded into J_w) ----
// stage 1: work[c * P + j] = sum over rows of chunk c of J[i, j]^2 (threads along j: coalesced rows)
template <typename T>
__global__ __launch_bounds__(256) void colsq_stage1_kernel(const T* __restrict__ J, int64_t ldJ, int64_t N,
                                                           int64_t P, int64_t rows_per, double* __restrict__ work) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= P) return;
  const int64_t r0 = (int64_t)blockIdx.y * rows_per;
  const int64_t r1 = (r0 + rows_per) < N ? (r0 + rows_per) : N;
  double acc = 0.0;
  for (int64_t i = r0; i < r1; ++i) {
    const double v = (double)J[i * ldJ + j];
    acc = fma(v, v, acc);
  }
  work[(int64_t)blockIdx.y * P + j] = acc;
}

// stage 2: out[j] (+)= sum over chunks in chunk order
__global__ void colsq_stage2_kernel(const double* __restrict__ work, int nchunk, int64_t P, int accumulate,
                                    double* __restrict__ out) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= P) return;
  double acc = accumulate ? out[j] : 0.0;
  for (int c = 0; c < nchunk; ++c) acc += work[(int64_t)c * P + j];
  out[j] = acc;
}

// ---- sampling proportional to weights ----
// Sample k of substream q draws u = u53 of the first two words of Philox4x32-10 at the counter
// (k, 2^31 + q, counter_lo, counter_hi) with the key (seed_lo, seed_hi): a counter range that the
// Gaussian test matrix (second word < 2^31) never reaches.
__device__ double sample_uniform(uint64_t k, uint32_t q, uint64_t seed, uint64_t counter) {
  uint32_t c[4] = {(uint32_t)k, 0x80000000u | q, (uint32_t)counter, (uint32_t)(counter >> 32)};
  philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
  return u53(c[0], c[1]);
}

constexpr int kSampThreads = 1024;

// One workgroup. Chunk sums of max(w, 0) (thread t: entries t*chunk .. in order), their running sum
// (one thread, in order), then per sample k the inverse CDF at u_k * total: the first chunk whose
// running sum exceeds the target, then the first index inside it whose running sum exceeds it.
// unique: the picks are sorted and duplicates removed. count = number of indices written (0 when all
// weights vanish).
__global__ __launch_bounds__(kSampThreads) void sample_pivots_kernel(const double* __restrict__ w, int64_t P,
                                                                     uint64_t seed, uint64_t counter, uint32_t q,
                                                                     int64_t ns, int unique, int64_t* __restrict__ idx,
                                                                     int* __restrict__ count,
                                                                     const int64_t* __restrict__ done) {
  __shared__ double csum[kSampThreads];
  const int t = threadIdx.x;
  if (done != nullptr && *done) {  // a finished factorisation draws nothing
    for (int64_t k = t; k < ns; k += kSampThreads) idx[k] = -1;
    if (t == 0) *count = 0;
    return;
  }
  const int64_t chunk = (P + kSampThreads - 1) / kSampThreads;
  {
    const int64_t j0 = (int64_t)t * chunk, j1 = (j0 + chunk) < P ? (j0 + chunk) : P;
    double s = 0.0;
    for (int64_t j = j0; j < j1; ++j) s += fmax(w[j], 0.0);
    csum[t] = s;
  }
  __syncthreads();
  if (t == 0) {
    double a = 0.0;
    for (int i = 0; i < kSampThreads; ++i) {
      a += csum[i];
      csum[i] = a;
    }
  }
  __syncthreads();
  const double total = csum[kSampThreads - 1];
  for (int64_t k = t; k < ns; k += kSampThreads) {
    int64_t pick = -1;
    if (total > 0.0) {
      const double target = sample_uniform((uint64_t)k, q, seed, counter) * total;
      int lo = 0, hi = kSampThreads - 1;  // first chunk with csum > target (csum[last] = total > target)
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (csum[mid] > target) hi = mid;
        else lo = mid + 1;
      }
      const int64_t j0 = (int64_t)lo * chunk, j1 = (j0 + chunk) < P ? (j0 + chunk) : P;
      double a = lo > 0 ? csum[lo - 1] : 0.0;
      int64_t last_pos = -1;
      for (int64_t j = j0; j < j1; ++j) {
        const double wj = fmax(w[j], 0.0);
        if (wj > 0.0) last_pos = j;
        a += wj;
        if (a > target && wj > 0.0) {
          pick = j;
          break;
        }
      }
      if (pick < 0) pick = last_pos;  // the in-chunk running sum rounded below the target
    }
    idx[k] = pick;
  }
  __syncthreads();
  if (t == 0) {
    if (total <= 0.0) {
      *count = 0;
      return;
    }
    int64_t n = ns;
    if (unique) {
      for (int64_t i = 1; i < ns; ++i) {  // insertion sort (ns is a block size)
        const int64_t v = idx[i];
        int64_t j = i - 1;
        while (j >= 0 && idx[j] > v) {
          idx[j + 1] = idx[j];
          --j;
        }
        idx[j + 1] = v;
      }
      n = ns > 0 ? 1 : 0;
      for (int64_t i = 1; i < ns; ++i)
        if (idx[i] != idx[n - 1]) idx[n++] = idx[i];
      for (int64_t i = n; i < ns; ++i) idx[i] = -1;
    }
    *count = (int)n;
  }
}

// out[i * ld_out + c] = J[i * ldJ + cols[c]] for rows i < rows, c < ncol (zero for a negative index)
template <typename T>
__global__ void gather_cols_kernel(const T* __restrict__ J, int64_t ldJ, int64_t rows, const int64_t* __restrict__ cols,
                                   int64_t ncol, T* __restrict__ out, int64_t ld_out) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncol) return;
  const int64_t col = cols[c];
  for (int64_t i = blockIdx.y; i < rows; i += gridDim.y) out[i * ld_out + c] = col >= 0 ? J[i * ldJ + col] : T(0);
}

// ---- block RPCholesky (Section 4.2.2; the block algorithm of the appendix) ----
// Device state of one factorisation: [0] rank r so far, [1] done flag, [2] kept columns of the
// current block; sums of the downdated diagonal in `dsum`.
constexpr int kRpMaxBlock = kRpBlockMax;

// W[m * ldw + k] = F[idx[m], k] = Ft[k * ldF + idx[m]] for k < kmax (zero rows for idx < 0)
__global__ void rp_gather_f_kernel(const double* __restrict__ Ft, int64_t ldF, const int64_t* __restrict__ idx,
                                   int b, int64_t kmax, double* __restrict__ W, int64_t ldw) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int m = blockIdx.y;
  if (k >= kmax || m >= b) return;
  const int64_t s = idx[m];
  W[(int64_t)m * ldw + k] = s >= 0 ? Ft[k * ldF + s] : 0.0;
}

// One wave: the pivot block C[S', S'] (from the rows of C^T at the pivots), its Cholesky factor
// (C[S',S'] = R^T R) column by column, the lanes sharing each column's scaling and the rank-1 update
// of the trailing block (every entry is updated with the same operands in the same order as a
// sequential elimination). A pivot that is not safely positive (<= 1e-13 of the block's largest
// diagonal entry: a direction the earlier columns already hold) is dropped together with its column.
// Writes the lower factor of the kept pivots, packed, to Rt (kRpMaxBlock x kRpMaxBlock) and their
// count to st[2] (capped so that r + kept <= cap).
__global__ __launch_bounds__(64) void rp_block_chol_kernel(const double* __restrict__ Ct, int64_t ldc,
                                                           const int64_t* __restrict__ idx,
                                                           const int* __restrict__ count, int64_t* __restrict__ st,
                                                           int64_t cap, double* __restrict__ Rt,
                                                           int* __restrict__ keep_rows) {
  __shared__ double A[kRpMaxBlock][kRpMaxBlock + 1];
  __shared__ int keep[kRpMaxBlock];
  const int c = *count;
  const int t = threadIdx.x;
  for (int e = t; e < c * c; e += blockDim.x) {
    const int m = e / c, n = e - m * c;
    A[m][n] = Ct[(int64_t)m * ldc + idx[n]];
  }
  __syncthreads();
  double dmax = 0.0;
  for (int m = 0; m < c; ++m) dmax = fmax(dmax, A[m][m]);
  const int64_t r = st[0];
  const bool done = st[1] != 0;
  int kept = 0;
  for (int j = 0; j < c; ++j) {
    const double pj = A[j][j];
    const bool ok = !done && pj > 1e-13 * dmax && r + kept < cap;
    if (t == 0) keep[j] = ok ? 1 : 0;
    if (!ok) continue;  // uniform: every lane sees the same pivot
    const double rj = sqrt(pj);
    __syncthreads();
    if (t == 0) A[j][j] = rj;
    for (int m = j + 1 + t; m < c; m += blockDim.x) A[m][j] /= rj;
    __syncthreads();
    const int w = c - j - 1;
    for (int e = t; e < w * w; e += blockDim.x) {
      const int m = j + 1 + e / w, n = j + 1 + e % w;
      if (n <= m) A[m][n] -= A[m][j] * A[n][j];
    }
    __syncthreads();
    ++kept;
  }
  __syncthreads();
  if (t == 0) st[2] = kept;
  // packed lower factor of the kept pivots: Rt[a][b'] = L(kept a, kept b'), L = R^T
  if (t == 0) {
    int a = 0;
    for (int m = 0; m < c; ++m) {
      if (!keep[m]) continue;
      int bb = 0;
      for (int n = 0; n <= m; ++n) {
        if (!keep[n]) continue;
        Rt[a * kRpMaxBlock + bb] = A[m][n];
        ++bb;
      }
      keep_rows[a] = m;
      ++a;
    }
  }
}

// Per parameter p: x = L^{-1} C[p, kept] (the row p of C R^{-1}, by forward substitution with the
// packed factor), written as rows r .. r + kept - 1 of Ft; the diagonal downdated by |x|^2. Block
// partial sums of the downdated diagonal go to part[blockIdx.x].
__global__ __launch_bounds__(256) void rp_update_kernel(const double* __restrict__ Ct, int64_t ldc,
                                                        const double* __restrict__ Rt,
                                                        const int* __restrict__ keep_rows,
                                                        const int64_t* __restrict__ st, int64_t P,
                                                        double* __restrict__ Ft, int64_t ldF, double* __restrict__ d,
                                                        double* __restrict__ part) {
  __shared__ double Ls[kRpMaxBlock * kRpMaxBlock];
  __shared__ double red[16];
  const int kept = (int)st[2];
  const int64_t r = st[0];
  for (int e = threadIdx.x; e < kept * kRpMaxBlock; e += blockDim.x) Ls[e] = Rt[e];
  __syncthreads();
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double dv = 0.0;
  if (p < P) {
    double x[kRpMaxBlock];
    double dd = d[p];
    for (int a = 0; a < kept; ++a) {
      double v = Ct[(int64_t)keep_rows[a] * ldc + p];
      for (int bb = 0; bb < a; ++bb) v -= Ls[a * kRpMaxBlock + bb] * x[bb];
      x[a] = v / Ls[a * kRpMaxBlock + a];
      Ft[(r + a) * ldF + p] = x[a];
      dd -= x[a] * x[a];
    }
    d[p] = dd;
    dv = dd;
  }
  dv = block_sum(dv, red);
  if (threadIdx.x == 0) part[blockIdx.x] = dv;
}

// One thread: the rank grows by the kept columns; the factorisation is done once the trace of the
// residual (the downdated diagonal's sum, in block order) is below eps, or no room is left.
__global__ void rp_finish_kernel(const double* __restrict__ part, int nb, double eps, int64_t cap, int b,
                                 int64_t* __restrict__ st, double* __restrict__ trace_out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double tr = 0.0;
  for (int i = 0; i < nb; ++i) tr += part[i];
  st[0] += st[2];
  st[2] = 0;
  *trace_out = tr;
  if (tr < eps || st[0] + 1 > cap) st[1] = 1;
}

}  // namespace

ngd_status launch_rp_gather_f(const double* Ft, int64_t ldF, const int64_t* idx, int b, int64_t kmax, double* W,
                              int64_t ldw, hipStream_t s) {
  if (kmax <= 0 || b <= 0) return NGD_OK;
  hipLaunchKernelGGL(rp_gather_f_kernel, dim3((unsigned)((kmax + 255) / 256), (unsigned)b), dim3(256), 0, s, Ft, ldF,
                     idx, b, kmax, W, ldw);
  NGD_HIP_TRY(hipGetLastError());
  return NGD_OK;
}

ngd_status launch_rp_block(const double* Ct, int64_t ldc, const int64_t* idx, const int* count, int64_t* st,
                           int64_t cap, double* Rt, int* keep_rows, int64_t P, double* Ft, int64_t ldF, double* d,
                           double* part, double eps, int b, double* trace_out, hipStream_t s) {
  if (b > kRpMaxBlock) {
    set_error("rpcholesky: block size above 64");
    return NGD_ERR_INVALID;
  }
  hipLaunchKernelGGL(rp_block_chol_kernel, dim3(1), dim3(64), 0, s, Ct, ldc, idx, count, st, cap, Rt, keep_rows);
  NGD_HIP_TRY(hipGetLastError());
  const int nb = (int)((P + 255) / 256);
  hipLaunchKernelGGL(rp_update_kernel, dim3((unsigned)nb), dim3(256), 0, s, Ct, ldc, Rt, keep_rows, st, P, Ft, ldF, d,
                     part);
  NGD_HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(rp_finish_kernel, dim3(1), dim3(64), 0, s, part, nb, eps, cap, b, st, trace_out);
  NGD_HIP_TRY(hipGetLastError());
  return NGD_OK;
}

ngd_status launch_colsq(int dtype, const void* J, int64_t ldJ, int64_t N, int64_t P, double* work,
                        int64_t work_elems, int accumulate, double* out, hipStream_t s) {
  if (P <= 0) return NGD_OK;
  const int64_t col_blocks = (P + 255) / 256;
  int nchunk = (int)std::max<int64_t>(1, std::min<int64_t>(work_elems / P, (2048 + col_blocks - 1) / col_blocks));
  nchunk = (int)std::min<int64_t>(nchunk, std::max<int64_t>(1, N));
  const int64_t rows_per = (N + nchunk - 1) / std::max(nchunk, 1);
  if (N > 0) {
    if (dtype == NGD_F64)
      hipLaunchKernelGGL(colsq_stage1_kernel<double>, dim3((unsigned)col_blocks, (unsigned)nchunk), dim3(256), 0, s,
                         (const double*)J, ldJ, N, P, rows_per, work);
    else
      hipLaunchKernelGGL(colsq_stage1_kernel<float>, dim3((unsigned)col_blocks, (unsigned)nchunk), dim3(256), 0, s,
                         (const float*)J, ldJ, N, P, rows_per, work);
    NGD_HIP_TRY(hipGetLastError());
  }
  hipLaunchKernelGGL(colsq_stage2_kernel, dim3((unsigned)col_blocks), dim3(256), 0, s, work, N > 0 ? nchunk : 0, P,
                     accumulate, out);
  NGD_HIP_TRY(hipGetLastError());
  return NGD_OK;
}

ngd_status launch_sample_pivots(const double* w, int64_t P, uint64_t seed, uint64_t counter, uint32_t q, int64_t ns,
                                int unique, int64_t* idx, int* count, hipStream_t s, const int64_t* done) {
  hipLaunchKernelGGL(sample_pivots_kernel, dim3(1), dim3(kSampThreads), 0, s, w, P, seed, counter, q, ns, unique,
                     idx, count, done);
  NGD_HIP_TRY(hipGetLastError());
  return NGD_OK;
}

ngd_status launch_gather_cols(int dtype, const void* J, int64_t ldJ, int64_t rows, const int64_t* cols, int64_t ncol,
                              void* out, int64_t ld_out, hipStream_t s) {
  if (rows <= 0 || ncol <= 0) return NGD_OK;
  const dim3 grid((unsigned)((ncol + 127) / 128), (unsigned)std::min<int64_t>(rows, 4096));
  if (dtype == NGD_F64)
    hipLaunchKernelGGL(gather_cols_kernel<double>, grid, dim3(128), 0, s, (const double*)J, ldJ, rows, cols, ncol,
                       (double*)out, ld_out);
  else
    hipLaunchKernelGGL(gather_cols_kernel<float>, grid, dim3(128), 0, s, (const float*)J, ldJ, rows, cols, ncol,
                       (float*)out, ld_out);
  NGD_HIP_TRY(hipGetLastError());
  return NGD_OK;
}

}  // namespace ngd
