// Damped Gramian matvec y = J_w^T (J_w v) + lambda v reading the stored Jacobian once, and the
// fused kernels of the preconditioned CG iteration built on it.
//
// One pass over J ("Precompute Jacobian only", Section 4.1.2; G = J_w^T J_w by eq. G_matrixfree):
// a workgroup owns a contiguous block of rows. For each row it loads the row into registers
// (each thread holds NK 16-byte chunks), forms t = J_r . v against v staged in LDS, reduces t
// across the workgroup (wave shuffles + one LDS barrier), and accumulates t * J_r into per-thread
// registers while the next row's loads are already in flight. The per-workgroup partial sums are
// reduced in a fixed order by a second kernel (deterministic, no floating-point atomics), which
// also adds lambda v. p^T G p = sum_r t_r^2 is accumulated on the way for CG.
#include "common.h"

namespace ngd {
namespace {

typedef float vf4 __attribute__((ext_vector_type(4)));
typedef double vd2 __attribute__((ext_vector_type(2)));
template <typename T> struct Vec;
template <> struct Vec<float> { using type = vf4; static constexpr int n = 4; };
template <> struct Vec<double> { using type = vd2; static constexpr int n = 2; };

template <typename T, int NK>
struct RowRegs {
  typename Vec<T>::type c[NK];
};

typedef unsigned v4u __attribute__((ext_vector_type(4)));

// Row loads through a raw buffer resource over this workgroup's rows: the per-lane byte offset is
// one VGPR and the per-row / per-chunk offset a scalar, so holding NK chunks of the current and
// the next row costs no address registers; reads past the rows' extent return 0.
template <typename T, int K0, int K1>
__device__ __forceinline__ void load_chunks(__amdgpu_buffer_rsrc_t rsrc, int row_bytes, int64_t nchunk,
                                            typename Vec<T>::type* dst) {
  using V = typename Vec<T>::type;
  const int vo = threadIdx.x * 16;
#pragma unroll
  for (int k = K0; k < K1; ++k) {
    int64_t q = threadIdx.x + (int64_t)k * blockDim.x;
    if (q < nchunk) {
      v4u raw = __builtin_amdgcn_raw_buffer_load_b128(rsrc, vo, row_bytes + k * (int)blockDim.x * 16, 0);
      dst[k - K0] = __builtin_bit_cast(V, raw);
    } else {
      dst[k - K0] = V{};
    }
  }
}

template <typename T>
__device__ __forceinline__ T dot_vec(const typename Vec<T>::type& a, const T* v);
template <>
__device__ __forceinline__ float dot_vec<float>(const vf4& a, const float* v) {
  return a.x * v[0] + a.y * v[1] + a.z * v[2] + a.w * v[3];
}
template <>
__device__ __forceinline__ double dot_vec<double>(const vd2& a, const double* v) {
  return a.x * v[0] + a.y * v[1];
}
template <typename T>
__device__ __forceinline__ void axpy_vec(T t, const typename Vec<T>::type& a, typename Vec<T>::type& y);
template <>
__device__ __forceinline__ void axpy_vec<float>(float t, const vf4& a, vf4& y) {
  y.x += t * a.x; y.y += t * a.y; y.z += t * a.z; y.w += t * a.w;
}
template <>
__device__ __forceinline__ void axpy_vec<double>(double t, const vd2& a, vd2& y) {
  y.x += t * a.x; y.y += t * a.y;
}

// Core of the one-pass product over rows [r0, r1): acc += sum_r (J_r . vs) J_r, tsq += (J_r . vs)^2.
// vs: the vector in LDS (ld elements, zero beyond P). Every thread returns with its own chunks.
template <typename T, int NK>
__device__ __forceinline__ void rows_pass(const T* __restrict__ J, int64_t ldJ, int64_t r0, int64_t r1,
                                          const T* vs, RowRegs<T, NK>& acc, double& tsq) {
  using V = typename Vec<T>::type;
  constexpr int VN = Vec<T>::n;
  constexpr int H = (NK + 1) / 2;  // chunks of the next row prefetched before the reduction
  __shared__ double red[2][16];
  const int64_t nchunk = ldJ / VN;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int k = 0; k < NK; ++k) acc.c[k] = V{};
  if (r0 >= r1) return;
  const int row_bytes = (int)(ldJ * sizeof(T));
  const __amdgpu_buffer_rsrc_t rsrc = __builtin_amdgcn_make_buffer_rsrc(
      (void*)(J + r0 * ldJ), (short)0, (int)((r1 - r0) * row_bytes), 0x00020000);
  V cur[NK];
  load_chunks<T, 0, NK>(rsrc, 0, nchunk, cur);
  int parity = 0;
  for (int64_t r = r0; r < r1; ++r) {
    const bool more = r + 1 < r1;
    const int next_bytes = (int)(r + 1 - r0) * row_bytes;
    // first half of the next row in flight during the dot product and the reduction
    V nxt_a[H];
    if (more) load_chunks<T, 0, H>(rsrc, next_bytes, nchunk, nxt_a);
    T dot = 0;
#pragma unroll
    for (int k = 0; k < NK; ++k) {
      int64_t q = threadIdx.x + (int64_t)k * blockDim.x;
      if (q < nchunk) dot += dot_vec<T>(cur[k], vs + q * VN);
    }
    dot = wave_sum(dot);
    if (lane == 0) red[parity][wid] = (double)dot;
    __syncthreads();
    double t = 0;
    for (int i = 0; i < nw; ++i) t += red[parity][i];
    parity ^= 1;
    tsq += t * t;
    const T tt = (T)t;
#pragma unroll
    for (int k = 0; k < H; ++k) axpy_vec<T>(tt, cur[k], acc.c[k]);
    // second half of the next row, into the registers the first half just released
    V nxt_b[NK - H > 0 ? NK - H : 1];
    if (more) load_chunks<T, H, NK>(rsrc, next_bytes, nchunk, nxt_b);
#pragma unroll
    for (int k = H; k < NK; ++k) axpy_vec<T>(tt, cur[k], acc.c[k]);
#pragma unroll
    for (int k = 0; k < H; ++k) cur[k] = nxt_a[k];
#pragma unroll
    for (int k = H; k < NK; ++k) cur[k] = nxt_b[k - H];
  }
}

template <typename T, int NK>
__device__ __forceinline__ void store_partial(T* __restrict__ partial, int64_t ldJ, const RowRegs<T, NK>& acc) {
  using V = typename Vec<T>::type;
  constexpr int VN = Vec<T>::n;
  V* out = reinterpret_cast<V*>(partial + (int64_t)blockIdx.x * ldJ);
  const int64_t nchunk = ldJ / VN;
#pragma unroll
  for (int k = 0; k < NK; ++k) {
    int64_t q = threadIdx.x + (int64_t)k * blockDim.x;
    if (q < nchunk) out[q] = acc.c[k];
  }
}

__device__ __forceinline__ void row_range(int64_t N, int64_t* r0, int64_t* r1) {
  const int64_t per = N / gridDim.x, extra = N % gridDim.x, b = blockIdx.x;
  *r0 = b * per + (b < extra ? b : extra);
  *r1 = *r0 + per + (b < extra ? 1 : 0);
}

// y partials of J^T (J v) for an FP64 input vector
template <typename T, int NK>
__global__ __launch_bounds__(1024) void gram_rows_kernel(const T* __restrict__ J, int64_t ldJ, int64_t N, int64_t P,
                                                         const double* __restrict__ v, T* __restrict__ partial,
                                                         double* __restrict__ tsq_out) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* vs = reinterpret_cast<T*>(smem_raw);
  for (int64_t j = threadIdx.x; j < ldJ; j += blockDim.x) vs[j] = j < P ? (T)v[j] : T(0);
  __syncthreads();
  int64_t r0, r1;
  row_range(N, &r0, &r1);
  RowRegs<T, NK> acc;
  double tsq = 0;
  rows_pass<T, NK>(J, ldJ, r0, r1, vs, acc, tsq);
  store_partial<T, NK>(partial, ldJ, acc);
  if (threadIdx.x == 0 && tsq_out) tsq_out[blockIdx.x] = tsq;
}

// Column sums of the workgroup partials: a block covers kRedCols columns with kRedGroups threads
// per column, each summing every kRedGroups-th partial; the groups are then added in a fixed order.
constexpr int kRedCols = 32, kRedGroups = 8;

template <typename T>
__device__ __forceinline__ double sum_partials(const T* __restrict__ partial, int nwg, int64_t ld, int64_t P,
                                               double (*buf)[kRedCols], int64_t* j_out) {
  const int c = threadIdx.x % kRedCols, g = threadIdx.x / kRedCols;
  const int64_t j = (int64_t)blockIdx.x * kRedCols + c;
  double acc = 0;
  if (j < P) {
    // eight loads in flight per thread; the order of the additions is fixed
    int b = g;
    for (; b + 7 * kRedGroups < nwg; b += 8 * kRedGroups) {
      T v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = partial[(int64_t)(b + u * kRedGroups) * ld + j];
#pragma unroll
      for (int u = 0; u < 8; ++u) acc += (double)v[u];
    }
    for (; b < nwg; b += kRedGroups) acc += (double)partial[(int64_t)b * ld + j];
  }
  buf[g][c] = acc;
  __syncthreads();
  double tot = 0;
  if (g == 0)
    for (int q = 0; q < kRedGroups; ++q) tot += buf[q][c];
  *j_out = j;
  return tot;
}

template <typename T>
__global__ __launch_bounds__(256) void gram_reduce_kernel(const T* __restrict__ partial, int nwg, int64_t ld,
                                                          int64_t P, const double* __restrict__ v, double lambda,
                                                          double* __restrict__ y) {
  __shared__ double buf[kRedGroups][kRedCols];
  int64_t j;
  const double acc = sum_partials(partial, nwg, ld, P, buf, &j);
  if (threadIdx.x < kRedCols && j < P) y[j] = acc + lambda * v[j];
}

// ---------------- fused PCG iteration ----------------
// (A) search direction p = z + beta p_prev staged on the fly, then the one-pass Gramian product
template <typename T, int NK>
__global__ __launch_bounds__(1024) void pcg_rows_kernel(const T* __restrict__ J, int64_t ldJ, int64_t N, int64_t P,
                                                        const double* __restrict__ z, const double* __restrict__ p_prev,
                                                        double* __restrict__ p_cur, PcgState* __restrict__ st,
                                                        T* __restrict__ partial, double* __restrict__ tsq_out) {
  if (st->done) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* vs = reinterpret_cast<T*>(smem_raw);
  __shared__ double red[16];
  const double beta = st->beta;
  double pp = 0;
  for (int64_t j = threadIdx.x; j < ldJ; j += blockDim.x) {
    double pj = j < P ? z[j] + beta * p_prev[j] : 0.0;
    vs[j] = (T)pj;
    pp += pj * pj;
    if (blockIdx.x == 0 && j < P) p_cur[j] = pj;
  }
  pp = block_sum(pp, red);
  if (blockIdx.x == 0 && threadIdx.x == 0) st->pp = pp;
  int64_t r0, r1;
  row_range(N, &r0, &r1);
  RowRegs<T, NK> acc;
  double tsq = 0;
  rows_pass<T, NK>(J, ldJ, r0, r1, vs, acc, tsq);
  store_partial<T, NK>(partial, ldJ, acc);
  if (threadIdx.x == 0) tsq_out[blockIdx.x] = tsq;
}

// (B) q = sum partials + lambda p; alpha = rz / (p^T q); x += alpha p; r -= alpha q; convergence
template <typename T>
__global__ __launch_bounds__(256) void pcg_update_kernel(const T* __restrict__ partial, int nwg, int64_t ld, int64_t P,
                                                         const double* __restrict__ p, const double* __restrict__ tsq,
                                                         double* __restrict__ x, double* __restrict__ r,
                                                         double* __restrict__ rr_part, PcgState* __restrict__ st,
                                                         int plain_cg) {
  if (st->done) return;
  __shared__ double red[4];
  const double pGp = block_sum_array(tsq, nwg, red);
  const double pq = pGp + st->lambda * st->pp;
  const double alpha = st->rz / pq;
  const int bad = !(pq > 0.0) || !isfinite(alpha);
  double rr = 0;
  __shared__ double buf[kRedGroups][kRedCols];
  int64_t j;
  double q = sum_partials(partial, nwg, ld, P, buf, &j);
  if (!bad && threadIdx.x < kRedCols && j < P) {
    q += st->lambda * p[j];
    const double xj = x[j] + alpha * p[j];
    const double rj = r[j] - alpha * q;
    x[j] = xj;
    r[j] = rj;
    rr = rj * rj;
  }
  rr = block_sum(rr, red);
  if (threadIdx.x == 0) rr_part[blockIdx.x] = rr;
  if (!arrive_last(&st->counter)) return;
  const double tot = block_sum_array(rr_part, (int)gridDim.x, red);
  if (threadIdx.x == 0) {
    if (bad) {
      st->breakdown = 1;
      st->done = 1;
      return;
    }
    st->alpha = alpha;
    st->iters += 1;
    st->rr = tot;
    if (!isfinite(tot)) {
      st->breakdown = 1;
      st->done = 1;
    } else if (tot <= st->rtol2bb) {
      st->converged = 1;
      st->done = 1;
    } else if (st->iters >= st->maxit) {
      st->done = 1;
    }
    if (plain_cg) {
      st->beta = tot / st->rz;
      st->rz = tot;
    }
  }
}

// (C) s_i = U_i . r for every preconditioner row (one workgroup per row)
template <typename T>
__global__ __launch_bounds__(256) void precond_dots_kernel(const T* __restrict__ U, int64_t ldU, int64_t P,
                                                           const double* __restrict__ r, double* __restrict__ s,
                                                           const PcgState* __restrict__ st) {
  if (st != nullptr && st->done) return;
  __shared__ double red[4];
  const T* u = U + (int64_t)blockIdx.x * ldU;
  double acc = 0;
  for (int64_t j = threadIdx.x; j < P; j += blockDim.x) acc += (double)u[j] * r[j];
  acc = block_sum(acc, red);
  if (threadIdx.x == 0) s[blockIdx.x] = acc;
}

// (D) z = c r + sum_i (1/(lam_i + mu) - c) s_i U_i (eq. nystrom_inverse); rz = r^T z; beta
template <typename T>
__global__ __launch_bounds__(256) void precond_apply_kernel(const T* __restrict__ U, int64_t ldU, int64_t P, int ell,
                                                            const double* __restrict__ lam, double mu,
                                                            const double* __restrict__ s, const double* __restrict__ r,
                                                            double* __restrict__ z, double* __restrict__ rz_part,
                                                            PcgState* __restrict__ st) {
  if (st != nullptr && st->done) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* coef = reinterpret_cast<double*>(smem_raw);
  __shared__ double red[4];
  const double c = 1.0 / (lam[ell - 1] + mu);
  for (int i = threadIdx.x; i < ell; i += blockDim.x) coef[i] = (1.0 / (lam[i] + mu) - c) * s[i];
  __syncthreads();
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double rz = 0;
  if (j < P) {
    double acc = 0;
    for (int i = 0; i < ell; ++i) acc += coef[i] * (double)U[(int64_t)i * ldU + j];
    const double zj = c * r[j] + acc;
    z[j] = zj;
    rz = zj * r[j];
  }
  if (st == nullptr) return;
  rz = block_sum(rz, red);
  if (threadIdx.x == 0) rz_part[blockIdx.x] = rz;
  if (!arrive_last(&st->counter)) return;
  const double tot = block_sum_array(rz_part, (int)gridDim.x, red);
  if (threadIdx.x == 0) {
    if (st->iters == 0 && st->beta == 0.0) {
      st->rz = tot;                       // initial z_0 = P^{-1} r_0
    } else {
      st->beta = tot / st->rz;
      st->rz = tot;
    }
    if (!isfinite(tot) || !(tot > 0.0)) {
      st->breakdown = 1;
      st->done = 1;
    }
  }
}

// initial state: x = 0, r = g, p_prev = 0; ||g||^2 and the stopping threshold
__global__ __launch_bounds__(256) void pcg_init_kernel(const double* __restrict__ g, int64_t P, double* __restrict__ x,
                                                       double* __restrict__ r, double* __restrict__ p_prev,
                                                       double* __restrict__ part, PcgState* __restrict__ st,
                                                       double rtol, int plain_cg) {
  __shared__ double red[4];
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double gg = 0;
  if (j < P) {
    const double gj = g[j];
    x[j] = 0.0;
    r[j] = gj;
    p_prev[j] = 0.0;
    gg = gj * gj;
  }
  gg = block_sum(gg, red);
  if (threadIdx.x == 0) part[blockIdx.x] = gg;
  if (!arrive_last(&st->counter)) return;
  const double tot = block_sum_array(part, (int)gridDim.x, red);
  if (threadIdx.x == 0) {
    st->bnorm2 = tot;
    st->rr = tot;
    st->rtol2bb = rtol * rtol * tot;
    st->beta = 0.0;
    st->iters = 0;
    st->converged = 0;
    st->breakdown = 0;
    st->done = 0;
    if (plain_cg) st->rz = tot;
    if (tot == 0.0) {
      st->converged = 1;
      st->done = 1;
    } else if (st->maxit <= 0 || !isfinite(tot)) {
      st->breakdown = !isfinite(tot);
      st->done = 1;
    }
  }
}

// small FP64 vector helpers
__global__ void dot_stage_kernel(const double* __restrict__ a, const double* __restrict__ b, int64_t n,
                                 double* __restrict__ part, double* __restrict__ out, unsigned* counter) {
  __shared__ double red[4];
  double acc = 0;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x)
    acc += a[j] * b[j];
  acc = block_sum(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = acc;
  if (!arrive_last(counter)) return;
  const double tot = block_sum_array(part, (int)gridDim.x, red);
  if (threadIdx.x == 0) *out = tot;
}

__global__ void scale_by_rsqrt_kernel(const double* __restrict__ w, const double* __restrict__ ww, int64_t n,
                                      double* __restrict__ v) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n) v[j] = w[j] / sqrt(*ww);
}

}  // namespace

// ---------------- host launchers ----------------

struct RowsCfg {
  int block;
  int nk;
};

static bool rows_cfg(int dtype, int64_t ldJ, RowsCfg* c) {
  const int vn = dtype == NGD_F64 ? 2 : 4;
  const int64_t nchunk = ldJ / vn;
  const int blocks[3] = {256, 512, 1024};
  const int maxnk[3] = {8, 8, 10};
  for (int i = 0; i < 3; ++i) {
    int64_t nk = (nchunk + blocks[i] - 1) / blocks[i];
    if (nk <= maxnk[i]) {
      c->block = blocks[i];
      c->nk = (int)(nk < 1 ? 1 : nk);
      return true;
    }
  }
  return false;
}

int gram_rows_grid(int dtype, int64_t N, int64_t P) {
  (void)dtype;
  (void)P;
  int64_t g = N < 256 ? N : 256;
  return (int)(g < 1 ? 1 : g);
}

bool gram_rows_supported(int dtype, int64_t ldJ) {
  RowsCfg c;
  return rows_cfg(dtype, ldJ, &c) && (size_t)ldJ * (dtype == NGD_F64 ? 8 : 4) <= 150 * 1024;
}

#define NGD_NK_DISPATCH(NKV, CALL) \
  switch (NKV) {                   \
    case 1: CALL(1); break;        \
    case 2: CALL(2); break;        \
    case 3: CALL(3); break;        \
    case 4: CALL(4); break;        \
    case 5: CALL(5); break;        \
    case 6: CALL(6); break;        \
    case 7: CALL(7); break;        \
    case 8: CALL(8); break;        \
    case 9: CALL(9); break;        \
    default: CALL(10); break;      \
  }

template <typename T>
static ngd_status gram_rows_t(const T* J, int64_t ldJ, int64_t N, int64_t P, const double* v, T* partial,
                              double* tsq, int nwg, hipStream_t s) {
  RowsCfg c;
  if (!rows_cfg(sizeof(T) == 8 ? NGD_F64 : NGD_F32, ldJ, &c)) {
    set_error("Jacobian row too long for the one-pass matvec");
    return NGD_ERR_INVALID;
  }
  const size_t lds = (size_t)ldJ * sizeof(T);
#define NGD_CALL(NK)                                                                                    \
  do {                                                                                                  \
    auto k = gram_rows_kernel<T, NK>;                                                                   \
    NGD_HIP_TRY(hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds)); \
    hipLaunchKernelGGL(k, dim3(nwg), dim3(c.block), lds, s, J, ldJ, N, P, v, partial, tsq);            \
  } while (0)
  NGD_NK_DISPATCH(c.nk, NGD_CALL)
#undef NGD_CALL
  NGD_HIP_TRY(hipGetLastError());
  return NGD_OK;
}

ngd_status launch_gram_rows(int dtype, const void* J, int64_t ldJ, int64_t N, int64_t P, const double* v,
                            void* partial, double* tsq, int nwg, hipStream_t s) {
  if (dtype == NGD_F64)
    return gram_rows_t<double>((const double*)J, ldJ, N, P, v, (double*)partial, tsq, nwg, s);
  return gram_rows_t<float>((const float*)J, ldJ, N, P, v, (float*)partial, tsq, nwg, s);
}

ngd_status launch_gram_reduce(int dtype, const void* partial, int nwg, int64_t ld, int64_t P, const double* v,
                              double lambda, double* y, hipStream_t s) {
  dim3 grid((unsigned)((P + kRedCols - 1) / kRedCols));
  if (dtype == NGD_F64)
    hipLaunchKernelGGL(gram_reduce_kernel<double>, grid, dim3(256), 0, s, (const double*)partial, nwg, ld, P, v,
                       lambda, y);
  else
    hipLaunchKernelGGL(gram_reduce_kernel<float>, grid, dim3(256), 0, s, (const float*)partial, nwg, ld, P, v,
                       lambda, y);
  NGD_HIP_TRY(hipGetLastError());
  return NGD_OK;
}

ngd_status launch_dot(const double* a, const double* b, int64_t n, double* work, double* out, hipStream_t s) {
  // work: 64 partials followed by one unsigned counter (zero-initialised by the handle)
  int nb = (int)((n + 255) / 256);
  nb = nb < 1 ? 1 : (nb > 64 ? 64 : nb);
  hipLaunchKernelGGL(dot_stage_kernel, dim3(nb), dim3(256), 0, s, a, b, n, work, out,
                     reinterpret_cast<unsigned*>(work + 64));
  NGD_HIP_TRY(hipGetLastError());
  return NGD_OK;
}

ngd_status launch_scale_rsqrt(const double* w, const double* ww, int64_t n, double* v, hipStream_t s) {
  hipLaunchKernelGGL(scale_by_rsqrt_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, w, ww, n, v);
  NGD_HIP_TRY(hipGetLastError());
  return NGD_OK;
}

// ---------------- PCG driver pieces ----------------

struct PcgBuffers {
  double *x, *r, *z, *p[2], *s, *part, *tsq;
  void* partial;
  PcgState* st;
};

ngd_status pcg_launch_init(const double* g, int64_t P, double* x, double* r, double* p_prev, double* part,
                           PcgState* st, double rtol, int plain, hipStream_t s) {
  hipLaunchKernelGGL(pcg_init_kernel, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, s, g, P, x, r, p_prev, part,
                     st, rtol, plain);
  NGD_HIP_TRY(hipGetLastError());
  return NGD_OK;
}

template <typename T>
static ngd_status pcg_rows_t(const T* J, int64_t ldJ, int64_t N, int64_t P, const double* z, const double* p_prev,
                             double* p_cur, PcgState* st, T* partial, double* tsq, int nwg, hipStream_t s) {
  RowsCfg c;
  if (!rows_cfg(sizeof(T) == 8 ? NGD_F64 : NGD_F32, ldJ, &c)) {
    set_error("Jacobian row too long for the one-pass matvec");
    return NGD_ERR_INVALID;
  }
  const size_t lds = (size_t)ldJ * sizeof(T);
#define NGD_CALL(NK)                                                                                    \
  do {                                                                                                  \
    auto k = pcg_rows_kernel<T, NK>;                                                                    \
    NGD_HIP_TRY(hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds)); \
    hipLaunchKernelGGL(k, dim3(nwg), dim3(c.block), lds, s, J, ldJ, N, P, z, p_prev, p_cur, st, partial, tsq); \
  } while (0)
  NGD_NK_DISPATCH(c.nk, NGD_CALL)
#undef NGD_CALL
  NGD_HIP_TRY(hipGetLastError());
  return NGD_OK;
}

ngd_status pcg_launch_rows(int dtype, const void* J, int64_t ldJ, int64_t N, int64_t P, const double* z,
                           const double* p_prev, double* p_cur, PcgState* st, void* partial, double* tsq, int nwg,
                           hipStream_t s) {
  if (dtype == NGD_F64)
    return pcg_rows_t<double>((const double*)J, ldJ, N, P, z, p_prev, p_cur, st, (double*)partial, tsq, nwg, s);
  return pcg_rows_t<float>((const float*)J, ldJ, N, P, z, p_prev, p_cur, st, (float*)partial, tsq, nwg, s);
}

ngd_status pcg_launch_update(int dtype, const void* partial, int nwg, int64_t ld, int64_t P, const double* p,
                             const double* tsq, double* x, double* r, double* rr_part, PcgState* st, int plain,
                             hipStream_t s) {
  dim3 grid((unsigned)((P + kRedCols - 1) / kRedCols));
  if (dtype == NGD_F64)
    hipLaunchKernelGGL(pcg_update_kernel<double>, grid, dim3(256), 0, s, (const double*)partial, nwg, ld, P, p, tsq,
                       x, r, rr_part, st, plain);
  else
    hipLaunchKernelGGL(pcg_update_kernel<float>, grid, dim3(256), 0, s, (const float*)partial, nwg, ld, P, p, tsq, x,
                       r, rr_part, st, plain);
  NGD_HIP_TRY(hipGetLastError());
  return NGD_OK;
}

ngd_status pcg_launch_precond(int dtype, const void* U, int64_t ldU, int64_t P, int ell, const double* lam, double mu,
                              double* sbuf, const double* r, double* z, double* rz_part, PcgState* st, hipStream_t s) {
  const size_t lds = (size_t)ell * sizeof(double);
  dim3 grid((unsigned)((P + 255) / 256));
  if (dtype == NGD_F64) {
    hipLaunchKernelGGL(precond_dots_kernel<double>, dim3(ell), dim3(256), 0, s, (const double*)U, ldU, P, r, sbuf, st);
    NGD_HIP_TRY(hipFuncSetAttribute((const void*)precond_apply_kernel<double>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL(precond_apply_kernel<double>, grid, dim3(256), lds, s, (const double*)U, ldU, P, ell, lam, mu,
                       sbuf, r, z, rz_part, st);
  } else {
    hipLaunchKernelGGL(precond_dots_kernel<float>, dim3(ell), dim3(256), 0, s, (const float*)U, ldU, P, r, sbuf, st);
    NGD_HIP_TRY(hipFuncSetAttribute((const void*)precond_apply_kernel<float>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL(precond_apply_kernel<float>, grid, dim3(256), lds, s, (const float*)U, ldU, P, ell, lam, mu,
                       sbuf, r, z, rz_part, st);
  }
  NGD_HIP_TRY(hipGetLastError());
  return NGD_OK;
}

}  // namespace ngd
