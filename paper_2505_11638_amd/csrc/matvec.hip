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
// vs: the vector in LDS (ld elements, zero beyond P). Rows are taken R at a time: their R dot
// products share one workgroup reduction, and the next R rows are loaded in full while the current
// ones are reduced and accumulated, so that about 2R rows per CU are in flight against HBM.
// `stage` fills vs (and does any other per-launch set-up), followed by a workgroup barrier; for
// short rows it runs after the first rows' loads have been issued, so its own reads overlap them.
// With `wts` non-null the row coefficients are given (t_r = wts[r - r0]: wts points at row r0's, no
// dot products and no reductions): acc = sum_r t_r J_r, the one-pass form of the gradient J_w^T r_w.
template <typename T, int NK, int R, typename Stage>
__device__ __forceinline__ void rows_pass(const T* __restrict__ J, int64_t ldJ, int64_t r0, int64_t r1,
                                          const T* vs, RowRegs<T, NK>& acc, double& tsq, Stage&& stage,
                                          const T* __restrict__ wts = nullptr) {
  using V = typename Vec<T>::type;
  constexpr int VN = Vec<T>::n;
  __shared__ double red[2][R][16];
  const int64_t nchunk = ldJ / VN;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int row_bytes = (int)(ldJ * sizeof(T));
  const int nrows = r1 > r0 ? (int)(r1 - r0) : 0;
  const __amdgpu_buffer_rsrc_t rsrc = __builtin_amdgcn_make_buffer_rsrc(
      (void*)(J + r0 * ldJ), (short)0, nrows * row_bytes, 0x00020000);
  if (nrows == 0) {
    stage();
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NK; ++k) acc.c[k] = V{};
    return;
  }
  // long rows leave no registers to spare while staging: stage first there
  constexpr bool kStageFirst = NK * R >= 12;
  if constexpr (kStageFirst) {
    stage();
    __syncthreads();
  }
  V cur[R][NK], nxt[R][NK];
#pragma unroll
  for (int q = 0; q < R; ++q) {
    if (q < nrows) load_chunks<T, 0, NK>(rsrc, q * row_bytes, nchunk, cur[q]);
    else
#pragma unroll
      for (int k = 0; k < NK; ++k) cur[q][k] = V{};
  }
  if constexpr (!kStageFirst) {
    stage();
    __syncthreads();
  }
#pragma unroll
  for (int k = 0; k < NK; ++k) acc.c[k] = V{};
  int parity = 0;
  for (int base = 0; base < nrows; base += R) {
    // rows base+R .. base+2R-1 in flight during this group's dot products and reduction
#pragma unroll
    for (int q = 0; q < R; ++q) {
      if (base + R + q < nrows) load_chunks<T, 0, NK>(rsrc, (base + R + q) * row_bytes, nchunk, nxt[q]);
      else
#pragma unroll
        for (int k = 0; k < NK; ++k) nxt[q][k] = V{};
    }
    if (wts != nullptr) {  // given coefficients: accumulate and move on
#pragma unroll
      for (int q = 0; q < R; ++q) {
        const T tt = base + q < nrows ? wts[base + q] : T(0);
#pragma unroll
        for (int k = 0; k < NK; ++k) axpy_vec<T>(tt, cur[q][k], acc.c[k]);
      }
#pragma unroll
      for (int q = 0; q < R; ++q)
#pragma unroll
        for (int k = 0; k < NK; ++k) cur[q][k] = nxt[q][k];
      continue;
    }
    T dot[R];
#pragma unroll
    for (int q = 0; q < R; ++q) {
      dot[q] = 0;
#pragma unroll
      for (int k = 0; k < NK; ++k) {
        int64_t c = threadIdx.x + (int64_t)k * blockDim.x;
        if (c < nchunk) dot[q] += dot_vec<T>(cur[q][k], vs + c * VN);
      }
      dot[q] = wave_sum_dpp(dot[q]);
    }
    if (lane == 0)
#pragma unroll
      for (int q = 0; q < R; ++q) red[parity][q][wid] = (double)dot[q];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < R; ++q) {
      double t = 0;
      for (int i = 0; i < nw; ++i) t += red[parity][q][i];
      tsq += t * t;  // rows past the end are zero and add nothing
      const T tt = (T)t;
#pragma unroll
      for (int k = 0; k < NK; ++k) axpy_vec<T>(tt, cur[q][k], acc.c[k]);
    }
    parity ^= 1;
#pragma unroll
    for (int q = 0; q < R; ++q)
#pragma unroll
      for (int k = 0; k < NK; ++k) cur[q][k] = nxt[q][k];
  }
}

template <typename T, int NK>
__device__ __forceinline__ void store_partial(T* __restrict__ partial, int64_t ldJ, const RowRegs<T, NK>& acc,
                                              int bid) {
  using V = typename Vec<T>::type;
  constexpr int VN = Vec<T>::n;
  V* out = reinterpret_cast<V*>(partial + (int64_t)bid * ldJ);
  const int64_t nchunk = ldJ / VN;
#pragma unroll
  for (int k = 0; k < NK; ++k) {
    int64_t q = threadIdx.x + (int64_t)k * blockDim.x;
    if (q < nchunk) out[q] = acc.c[k];
  }
}

// rows of workgroup bid of nb: a contiguous, balanced share of [0, N)
__device__ __forceinline__ void row_range(int64_t N, int64_t* r0, int64_t* r1, int bid, int nb) {
  const int64_t per = N / nb, extra = N % nb, b = bid;
  *r0 = b * per + (b < extra ? b : extra);
  *r1 = *r0 + per + (b < extra ? 1 : 0);
}

// y partials of J^T (J v) for an FP64 input vector
template <typename T, int NK, int R, int B>
__global__ __launch_bounds__(B, (NK * R <= 10 ? 4 : 1)) void gram_rows_kernel(const T* __restrict__ J, int64_t ldJ, int64_t N, int64_t P,
                                                         const double* __restrict__ v, T* __restrict__ partial,
                                                         double* __restrict__ tsq_out) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* vs = reinterpret_cast<T*>(smem_raw);
  int64_t r0, r1;
  row_range(N, &r0, &r1, blockIdx.x, gridDim.x);
  RowRegs<T, NK> acc;
  double tsq = 0;
  rows_pass<T, NK, R>(J, ldJ, r0, r1, vs, acc, tsq, [&] {
    // short rows: several loads in flight; long rows: registers are needed for the rows
    if constexpr (NK * R < 12) {
#pragma unroll 4
      for (int64_t j = threadIdx.x; j < ldJ; j += B) vs[j] = j < P ? (T)v[j] : T(0);
    } else {
      for (int64_t j = threadIdx.x; j < ldJ; j += B) vs[j] = j < P ? (T)v[j] : T(0);
    }
  });
  store_partial<T, NK>(partial, ldJ, acc, blockIdx.x);
  if (threadIdx.x == 0 && tsq_out) tsq_out[blockIdx.x] = tsq;
}

// partials of the gradient J^T r (r in the Jacobian's dtype): rows weighted by r, no reductions
template <typename T, int NK, int R, int B>
__global__ __launch_bounds__(B) void grad_rows_kernel(const T* __restrict__ J, int64_t ldJ, int64_t N,
                                                      const T* __restrict__ r, T* __restrict__ partial,
                                                      int max_staged) {
  int64_t r0, r1;
  row_range(N, &r0, &r1, blockIdx.x, gridDim.x);
  RowRegs<T, NK> acc;
  double tsq = 0;
  // the workgroup's row coefficients in LDS when they fit (launched with that much dynamic LDS), so
  // that no global load waits inside the row loop
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* ws = reinterpret_cast<T*>(smem_raw);
  const int nr = (int)(r1 - r0);
  const bool staged = nr <= max_staged;
  if (staged)
    for (int i = threadIdx.x; i < nr; i += blockDim.x) ws[i] = r[r0 + i];
  __syncthreads();
  rows_pass<T, NK, R>(J, ldJ, r0, r1, nullptr, acc, tsq, [] {}, staged ? ws : r + r0);
  store_partial<T, NK>(partial, ldJ, acc, blockIdx.x);
}

// Column sums of the workgroup partials: a block covers kRedCols columns with kRedGroups threads
// per column, each summing every kRedGroups-th partial; the groups are then added in a fixed order.
constexpr int kRedCols = 32, kRedGroups = 8;

template <typename T>
__device__ __forceinline__ double sum_partials(const T* __restrict__ partial, int nwg, int64_t ld, int64_t P,
                                               double (*buf)[kRedCols], int64_t* j_out, int bid) {
  const int c = threadIdx.x % kRedCols, g = threadIdx.x / kRedCols;
  const int64_t j = (int64_t)bid * kRedCols + c;
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
  const double acc = sum_partials(partial, nwg, ld, P, buf, &j, blockIdx.x);
  if (threadIdx.x < kRedCols && j < P) y[j] = lambda != 0.0 ? acc + lambda * v[j] : acc;
}

// recompute-mode CG direction: p = z + beta p_prev (FP64 and a dtype copy for the JVP), pp = p.p
template <typename T>
__global__ __launch_bounds__(256) void pcg_direction_kernel(const double* __restrict__ z,
                                                            const double* __restrict__ p_prev, int64_t P,
                                                            double* __restrict__ p_cur, T* __restrict__ p_t,
                                                            double* __restrict__ part, PcgState* __restrict__ st) {
  if (st->done) return;
  __shared__ double red[4];
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double pp = 0;
  if (j < P) {
    const double pj = z[j] + st->beta * p_prev[j];
    p_cur[j] = pj;
    p_t[j] = (T)pj;
    pp = pj * pj;
  }
  pp = block_sum(pp, red);
  double tot;
  if (!publish_and_reduce(pp, part, (int)blockIdx.x, &st->counter, (unsigned)(gridDim.x), red, &tot)) return;
  if (threadIdx.x == 0) st->pp = tot;
}

// ---------------- fused PCG iteration ----------------
// (A) search direction p = z + beta p_prev staged on the fly, then the one-pass Gramian product
template <typename T, int NK, int R, int B>
__device__ __forceinline__ void pcg_rows_body(const T* __restrict__ J, int64_t ldJ, int64_t N, int64_t P,
                                              const double* __restrict__ z, const double* __restrict__ p_prev,
                                              double* __restrict__ p_cur, PcgState* __restrict__ st,
                                              T* __restrict__ partial, double* __restrict__ tsq_out, int bid, int nb) {
  if (st->done) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* vs = reinterpret_cast<T*>(smem_raw);
  __shared__ double red[16];
  int64_t r0, r1;
  row_range(N, &r0, &r1, bid, nb);
  RowRegs<T, NK> acc;
  double tsq = 0;
  rows_pass<T, NK, R>(J, ldJ, r0, r1, vs, acc, tsq, [&] {
    const double beta = st->beta;
    double pp = 0;
    auto one = [&](int64_t j) {
      double pj = j < P ? z[j] + beta * p_prev[j] : 0.0;
      vs[j] = (T)pj;
      pp += pj * pj;
      if (bid == 0 && j < P) p_cur[j] = pj;
    };
    if constexpr (NK * R < 12) {
#pragma unroll 4
      for (int64_t j = threadIdx.x; j < ldJ; j += B) one(j);
    } else {
      for (int64_t j = threadIdx.x; j < ldJ; j += B) one(j);
    }
    pp = block_sum(pp, red);
    if (bid == 0 && threadIdx.x == 0) st->pp = pp;
  });
  store_partial<T, NK>(partial, ldJ, acc, bid);
  if (threadIdx.x == 0) tsq_out[bid] = tsq;
}

template <typename T, int NK, int R, int B>
__global__ __launch_bounds__(B, (NK * R <= 10 ? 4 : 1)) void pcg_rows_kernel(const T* __restrict__ J, int64_t ldJ, int64_t N, int64_t P,
                                                     const double* __restrict__ z, const double* __restrict__ p_prev,
                                                     double* __restrict__ p_cur, PcgState* __restrict__ st,
                                                     T* __restrict__ partial, double* __restrict__ tsq_out) {
  pcg_rows_body<T, NK, R, B>(J, ldJ, N, P, z, p_prev, p_cur, st, partial, tsq_out, blockIdx.x, gridDim.x);
}

// (B) q = sum partials + lambda p; alpha = rz / (p^T q); x += alpha p; r -= alpha q; convergence
template <typename T>
__device__ __forceinline__ void pcg_update_body(const T* __restrict__ partial, int nwg, int64_t ld, int64_t P,
                                                const double* __restrict__ p, const double* __restrict__ tsq,
                                                double* __restrict__ x, double* __restrict__ r,
                                                double* __restrict__ rr_part, PcgState* __restrict__ st, int plain_cg,
                                                int bid, int nb) {
  if (st->done) return;
  __shared__ double red[4];
  const double pGp = block_sum_array(tsq, nwg, red);
  const double pq = pGp + st->lambda * st->pp;
  const double alpha = st->rz / pq;
  const int bad = !(pq > 0.0) || !isfinite(alpha);
  double rr = 0;
  __shared__ double buf[kRedGroups][kRedCols];
  int64_t j;
  double q = sum_partials(partial, nwg, ld, P, buf, &j, bid);
  if (!bad && threadIdx.x < kRedCols && j < P) {
    q += st->lambda * p[j];
    const double xj = x[j] + alpha * p[j];
    const double rj = r[j] - alpha * q;
    x[j] = xj;
    r[j] = rj;
    rr = rj * rj;
  }
  rr = block_sum(rr, red);
  double tot;
  if (!publish_and_reduce(rr, rr_part, (int)bid, &st->counter, (unsigned)(nb), red, &tot)) return;
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

template <typename T>
__global__ __launch_bounds__(256) void pcg_update_kernel(const T* __restrict__ partial, int nwg, int64_t ld, int64_t P,
                                                         const double* __restrict__ p, const double* __restrict__ tsq,
                                                         double* __restrict__ x, double* __restrict__ r,
                                                         double* __restrict__ rr_part, PcgState* __restrict__ st,
                                                         int plain_cg) {
  pcg_update_body<T>(partial, nwg, ld, P, p, tsq, x, r, rr_part, st, plain_cg, blockIdx.x, gridDim.x);
}

// (C) s_i = U_i . r for every preconditioner row (one workgroup per row)
template <typename T>
__device__ __forceinline__ void precond_dots_body(const T* __restrict__ U, int64_t ldU, int64_t P,
                                                  const double* __restrict__ r, double* __restrict__ s,
                                                  const PcgState* __restrict__ st, int bid) {
  if (st != nullptr && st->done) return;
  __shared__ double red[4];
  const T* u = U + (int64_t)bid * ldU;
  double acc = 0;
  for (int64_t j = threadIdx.x; j < P; j += blockDim.x) acc += (double)u[j] * r[j];
  acc = block_sum(acc, red);
  if (threadIdx.x == 0) s[bid] = acc;
}

// (C) for one problem: workgroup (g, c) forms the dots of preconditioner rows kDotRows g ..
// kDotRows g + kDotRows - 1 with r over column chunk c, into part[c * ell + i]; the apply kernel adds
// the chunks in a fixed order. r is read once per kDotRows rows, and the grid has rows x chunks
// workgroups instead of one per row.
constexpr int kDotRows = 4;

template <typename T>
__global__ __launch_bounds__(256) void precond_dots_chunk_kernel(const T* __restrict__ U, int64_t ldU, int64_t P,
                                                                 int ell, int64_t chunk,
                                                                 const double* __restrict__ r,
                                                                 double* __restrict__ part,
                                                                 const PcgState* __restrict__ st) {
  if (st != nullptr && st->done) return;
  __shared__ double red[kDotRows][4];
  const int i0 = blockIdx.x * kDotRows;
  const int64_t j0 = (int64_t)blockIdx.y * chunk;
  const int64_t j1 = j0 + chunk < P ? j0 + chunk : P;
  double acc[kDotRows];
#pragma unroll
  for (int q = 0; q < kDotRows; ++q) acc[q] = 0.0;
  for (int64_t j = j0 + threadIdx.x; j < j1; j += blockDim.x) {
    const double rj = r[j];
#pragma unroll
    for (int q = 0; q < kDotRows; ++q)
      if (i0 + q < ell) acc[q] += (double)U[(int64_t)(i0 + q) * ldU + j] * rj;
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < kDotRows; ++q) acc[q] = wave_sum_dpp(acc[q]);
  if (lane == 0)
#pragma unroll
    for (int q = 0; q < kDotRows; ++q) red[q][wid] = acc[q];
  __syncthreads();
  if (threadIdx.x < kDotRows && i0 + (int)threadIdx.x < ell) {
    const int q = threadIdx.x;
    part[(int64_t)blockIdx.y * ell + i0 + q] = red[q][0] + red[q][1] + red[q][2] + red[q][3];
  }
}

// (D) z = c r + sum_i (1/(lam_i + mu) - c) s_i U_i (eq. nystrom_inverse); rz = r^T z; beta
template <typename T>
__device__ __forceinline__ void precond_apply_body(const T* __restrict__ U, int64_t ldU, int64_t P, int ell,
                                                   const double* __restrict__ lam, double mu,
                                                   const double* __restrict__ s, const double* __restrict__ r,
                                                   double* __restrict__ z, double* __restrict__ rz_part,
                                                   PcgState* __restrict__ st, int bid, int nb) {
  if (st != nullptr && st->done) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* coef = reinterpret_cast<double*>(smem_raw);
  __shared__ double red[4];
  const double c = 1.0 / (lam[ell - 1] + mu);
  for (int i = threadIdx.x; i < ell; i += blockDim.x) coef[i] = (1.0 / (lam[i] + mu) - c) * s[i];
  __syncthreads();
  const int64_t j = (int64_t)bid * blockDim.x + threadIdx.x;
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
  double tot;
  if (!publish_and_reduce(rz, rz_part, (int)bid, &st->counter, (unsigned)(nb), red, &tot)) return;
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

// (D) for one problem: a workgroup of kApWaves waves owns kApCols columns; wave w adds the rows
// w, w + kApWaves, ... of U (two adjacent columns per lane, read as one 2-element vector when VEC),
// the waves' sums meet in LDS. The coefficients are (1/(lam_i + mu) - c) s_i with s_i the sum of the
// dot chunks. Then z, r^T z and beta as in the batched form.
constexpr int kApWaves = 8, kApCols = 128;

template <typename T> struct Pair;
template <> struct Pair<float> { typedef float type __attribute__((ext_vector_type(2))); };
template <> struct Pair<double> { typedef double type __attribute__((ext_vector_type(2))); };

template <typename T, bool VEC>
__global__ __launch_bounds__(64 * kApWaves) void precond_apply_cols_kernel(
    const T* __restrict__ U, int64_t ldU, int64_t P, int ell, const double* __restrict__ lam,
    const double* __restrict__ part, int nchunk, const double* __restrict__ r, double* __restrict__ z,
    double* __restrict__ rz_part, PcgState* __restrict__ st) {
  if (st->done) return;
  const double mu = st->lambda;  // the solve's damping (set on the device by the damping rule)
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* coef = reinterpret_cast<double*>(smem_raw);
  __shared__ double wsum[kApWaves][kApCols];
  __shared__ double red[kApWaves];
  const double c = 1.0 / (lam[ell - 1] + mu);
  for (int i = threadIdx.x; i < ell; i += blockDim.x) {
    double si = 0.0;
    for (int q = 0; q < nchunk; ++q) si += part[(int64_t)q * ell + i];
    coef[i] = (1.0 / (lam[i] + mu) - c) * si;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t j = (int64_t)blockIdx.x * kApCols + 2 * lane;  // this lane's columns j, j + 1
  double a0 = 0.0, a1 = 0.0;
  if (j < P) {
    if constexpr (VEC) {  // j even and ldU even: the pair is aligned and j + 1 < ldU
      using V2 = typename Pair<T>::type;
#pragma unroll 8
      for (int i = w; i < ell; i += kApWaves) {
        const V2 u = *reinterpret_cast<const V2*>(U + (int64_t)i * ldU + j);
        a0 += coef[i] * (double)u.x;
        a1 += coef[i] * (double)u.y;
      }
    } else {
      const bool two = j + 1 < P;
#pragma unroll 8
      for (int i = w; i < ell; i += kApWaves) {
        const T* u = U + (int64_t)i * ldU + j;
        a0 += coef[i] * (double)u[0];
        if (two) a1 += coef[i] * (double)u[1];
      }
    }
  }
  wsum[w][2 * lane] = a0;
  wsum[w][2 * lane + 1] = a1;
  __syncthreads();
  double rz = 0.0;
  if (threadIdx.x < kApCols) {
    const int64_t jj = (int64_t)blockIdx.x * kApCols + threadIdx.x;
    if (jj < P) {
      double acc = 0.0;
#pragma unroll
      for (int q = 0; q < kApWaves; ++q) acc += wsum[q][threadIdx.x];
      const double zj = c * r[jj] + acc;
      z[jj] = zj;
      rz = zj * r[jj];
    }
  }
  rz = block_sum(rz, red);
  const int nb = (int)gridDim.x;
  double tot;
  if (!publish_and_reduce(rz, rz_part, (int)blockIdx.x, &st->counter, (unsigned)(nb), red, &tot)) return;
  if (threadIdx.x == 0) {
    if (st->iters == 0 && st->beta == 0.0) {
      st->rz = tot;  // initial z_0 = P^{-1} r_0
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
__device__ __forceinline__ void pcg_init_body(const double* __restrict__ g, int64_t P, double* __restrict__ x,
                                              double* __restrict__ r, double* __restrict__ p_prev,
                                              double* __restrict__ part, PcgState* __restrict__ st, double rtol,
                                              int plain_cg, int bid, int nb) {
  __shared__ double red[4];
  const int64_t j = (int64_t)bid * blockDim.x + threadIdx.x;
  double gg = 0;
  if (j < P) {
    const double gj = g[j];
    x[j] = 0.0;
    r[j] = gj;
    p_prev[j] = 0.0;
    gg = gj * gj;
  }
  gg = block_sum(gg, red);
  double tot;
  if (!publish_and_reduce(gg, part, (int)bid, &st->counter, (unsigned)(nb), red, &tot)) return;
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

__global__ __launch_bounds__(256) void pcg_init_kernel(const double* __restrict__ g, int64_t P, double* __restrict__ x,
                                                       double* __restrict__ r, double* __restrict__ p_prev,
                                                       double* __restrict__ part, PcgState* __restrict__ st,
                                                       double rtol, int plain_cg) {
  pcg_init_body(g, P, x, r, p_prev, part, st, rtol, plain_cg, blockIdx.x, gridDim.x);
}

// small FP64 vector helpers
__global__ void dot_stage_kernel(const double* __restrict__ a, const double* __restrict__ b, int64_t n,
                                 double* __restrict__ part, double* __restrict__ out, unsigned* counter) {
  __shared__ double red[4];
  double acc = 0;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x)
    acc += a[j] * b[j];
  acc = block_sum(acc, red);
  double tot;
  if (!publish_and_reduce(acc, part, (int)blockIdx.x, counter, (unsigned)(gridDim.x), red, &tot)) return;
  if (threadIdx.x == 0) *out = tot;
}

__global__ void scale_by_rsqrt_kernel(const double* __restrict__ w, const double* __restrict__ ww, int64_t n,
                                      double* __restrict__ v) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n) v[j] = w[j] / sqrt(*ww);
}

// ---------------- batched PCG: several problems per launch ----------------
// Item `it` of a launch belongs to the last problem whose first item of that kind is <= it (problems
// with no items of a kind share their successor's first item and are never chosen).
template <typename Key>
__device__ __forceinline__ int find_problem(int n, int it, Key first) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (first(mid) <= it) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__global__ __launch_bounds__(256) void pcg_batch_init_kernel(const PcgBatchItem* __restrict__ items, int n) {
  const int it = blockIdx.x;
  const PcgBatchItem& b = items[find_problem(n, it, [&](int q) { return items[q].item0_elem; })];
  pcg_init_body(b.g, b.P, b.x, b.r, b.p0, b.part, b.st, b.rtol, b.plain, it - b.item0_elem, (int)((b.P + 255) / 256));
}

template <typename T, int NK, int R, int B>
__global__ __launch_bounds__(B) void pcg_batch_rows_kernel(const PcgBatchItem* __restrict__ items, int n) {
  const int it = blockIdx.x;
  const PcgBatchItem& b = items[find_problem(n, it, [&](int q) { return items[q].item0_rows; })];
  // iteration parity: the direction of the previous iteration and the slot for this one
  const bool odd = (b.st->iters & 1) != 0;
  pcg_rows_body<T, NK, R, B>((const T*)b.J, b.ldJ, b.N, b.P, b.plain ? b.r : b.z, odd ? b.p1 : b.p0,
                             odd ? b.p0 : b.p1, b.st, (T*)b.partial, b.tsq, it - b.item0_rows, b.nwg);
}

template <typename T>
__global__ __launch_bounds__(256) void pcg_batch_update_kernel(const PcgBatchItem* __restrict__ items, int n) {
  const int it = blockIdx.x;
  const PcgBatchItem& b = items[find_problem(n, it, [&](int q) { return items[q].item0_upd; })];
  const bool odd = (b.st->iters & 1) != 0;
  pcg_update_body<T>((const T*)b.partial, b.nwg, b.ldJ, b.P, odd ? b.p0 : b.p1, b.tsq, b.x, b.r, b.part, b.st,
                     b.plain, it - b.item0_upd, (int)((b.P + kRedCols - 1) / kRedCols));
}

template <typename T>
__global__ __launch_bounds__(256) void pcg_batch_dots_kernel(const PcgBatchItem* __restrict__ items, int n) {
  const int it = blockIdx.x;
  const PcgBatchItem& b = items[find_problem(n, it, [&](int q) { return items[q].item0_dots; })];
  precond_dots_body<T>((const T*)b.U, b.ldU, b.P, b.r, b.s, b.st, it - b.item0_dots);
}

template <typename T>
__global__ __launch_bounds__(256) void pcg_batch_apply_kernel(const PcgBatchItem* __restrict__ items, int n) {
  const int it = blockIdx.x;
  const PcgBatchItem& b = items[find_problem(n, it, [&](int q) { return items[q].item0_apply; })];
  precond_apply_body<T>((const T*)b.U, b.ldU, b.P, b.ell, b.lam, b.st->lambda, b.s, b.r, b.z, b.part, b.st,
                        it - b.item0_apply, (int)((b.P + 255) / 256));
}

// the damping rule of Section 4.3 for every problem of a batch (one thread per problem)
__global__ void pcg_batch_damping_kernel(const PcgBatchItem* __restrict__ items, PcgState* __restrict__ states, int n,
                                         double c_lam, double c_loss) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double l = items[i].loss != nullptr ? items[i].loss[0] : 0.0;
  states[i].lambda = fmax(c_lam * items[i].lam[0], c_loss * (l * l));
}

// one thread: the damping rule of Section 4.3 evaluated on the device, and the sketch's error words
__global__ void pcg_setup_kernel(PcgState* __restrict__ st, const double* __restrict__ lam_hat, double c_lam,
                                 const double* __restrict__ loss, double c_loss, const int* __restrict__ eig_err,
                                 const unsigned* __restrict__ chol_err) {
  if (lam_hat != nullptr) st->lambda = fmax(c_lam * lam_hat[0], c_loss * (loss[0] * loss[0]));
  int e = 0;
  if (eig_err != nullptr && *eig_err != 0) e |= 1;
  if (chol_err != nullptr && *chol_err != 0u) e |= 2;
  st->sketch_err = e;
}

}  // namespace

// ---------------- host launchers ----------------

ngd_status pcg_launch_setup(PcgState* st, const double* lam_hat, double c_lam, const double* loss, double c_loss,
                            const int* eig_err, const unsigned* chol_err, hipStream_t s) {
  hipLaunchKernelGGL(pcg_setup_kernel, dim3(1), dim3(1), 0, s, st, lam_hat, c_lam, loss, c_loss, eig_err, chol_err);
  NGD_HIP_TRY(hipGetLastError());
  return NGD_OK;
}

// One-pass configurations (block, NK, R): a workgroup per CU, so a lane may hold 256 VGPRs; R rows
// per step are chosen so that the 2R row buffers and the accumulator, (2R + 1) NK 16-byte chunks,
// fit beside the addressing registers. Rows longer than 512 x 18 chunks (147 KB) are not supported.
#define NGD_ROWS_CONFIGS(X)                                                                     \
  X(0, 256, 1, 4) X(1, 256, 2, 4) X(2, 256, 3, 4) X(3, 256, 4, 4) X(4, 512, 2, 4) X(5, 512, 3, 4) \
  X(6, 512, 4, 4) X(7, 512, 5, 4) X(8, 512, 6, 2) X(9, 512, 7, 2) X(10, 512, 8, 2)              \
  X(11, 512, 9, 2) X(12, 512, 10, 2) X(13, 512, 12, 1) X(14, 512, 14, 1) X(15, 512, 16, 1)     \
  X(16, 512, 17, 1) X(17, 512, 18, 1) X(18, 512, 5, 2)

struct RowsCfg {
  int id, block, nk, r;
};

static bool rows_cfg(int dtype, int64_t ldJ, RowsCfg* c) {
  const int vn = dtype == NGD_F64 ? 2 : 4;
  const int64_t nchunk = ldJ / vn;
  static const RowsCfg table[] = {
#define NGD_ROW(ID, B, NK, R) {ID, B, NK, R},
      NGD_ROWS_CONFIGS(NGD_ROW)
#undef NGD_ROW
  };
  // FP32 rows of 2,049 - 2,560 chunks (P about 8.2k - 10.2k): five chunks per thread and two rows per
  // step, few enough registers for two workgroups per CU (measured faster than four rows per step
  // with one workgroup per CU)
  if (dtype == NGD_F32 && nchunk > 2048 && nchunk <= 2560) {
    *c = table[18];
    return true;
  }
  for (const RowsCfg& t : table) {
    if ((int64_t)t.block * t.nk >= nchunk && (t.block == 512 || nchunk <= 256 * 4)) {
      *c = t;
      return true;
    }
  }
  return false;
}

int gram_rows_grid(int dtype, int64_t N, int64_t P) {
  // one workgroup per CU, or two where the row configuration leaves registers for two
  RowsCfg c;
  const int64_t ld = (P + 63) / 64 * 64;
  const int64_t cap = rows_cfg(dtype, ld, &c) && c.nk * c.r <= 10 && c.block == 512 ? 512 : 256;
  int64_t g = N < cap ? N : cap;
  return (int)(g < 1 ? 1 : g);
}

bool gram_rows_supported(int dtype, int64_t ldJ) {
  RowsCfg c;
  return rows_cfg(dtype, ldJ, &c) && (size_t)ldJ * (dtype == NGD_F64 ? 8 : 4) <= 150 * 1024;
}

#define NGD_CFG_DISPATCH(ID, CALL)                      \
  switch (ID) {                                         \
    NGD_ROWS_CONFIGS(CALL)                              \
    default: break;                                     \
  }

template <typename T>
static ngd_status gram_rows_t(const T* J, int64_t ldJ, int64_t N, int64_t P, const double* v, T* partial,
                              double* tsq, int nwg, hipStream_t s, LaunchEvents ev) {
  RowsCfg c;
  if (!rows_cfg(sizeof(T) == 8 ? NGD_F64 : NGD_F32, ldJ, &c)) {
    set_error("Jacobian row too long for the one-pass matvec");
    return NGD_ERR_INVALID;
  }
  const size_t lds = (size_t)ldJ * sizeof(T);
#define NGD_CALL(ID, B, NK, R)                                                                          \
  case ID: {                                                                                            \
    auto k = gram_rows_kernel<T, NK, R, B>;                                                             \
    NGD_HIP_TRY(hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds)); \
    hipExtLaunchKernelGGL(k, dim3(nwg), dim3(B), (uint32_t)lds, s, ev.start, ev.stop, 0u, J, ldJ, N, P, v,  \
                          partial, tsq);                                                                \
    break;                                                                                              \
  }
  NGD_CFG_DISPATCH(c.id, NGD_CALL)
#undef NGD_CALL
  NGD_HIP_TRY(hipGetLastError());
  return NGD_OK;
}

template <typename T>
static ngd_status grad_rows_t(const T* J, int64_t ldJ, int64_t N, const T* r, T* partial, int nwg, hipStream_t s) {
  RowsCfg c;
  if (!rows_cfg(sizeof(T) == 8 ? NGD_F64 : NGD_F32, ldJ, &c)) {
    set_error("Jacobian row too long for the one-pass gradient");
    return NGD_ERR_INVALID;
  }
  // rows per workgroup (the balanced split of row_range), staged in LDS up to 16 KB
  const int64_t per = (N + nwg - 1) / nwg;
  const int max_staged = per * (int64_t)sizeof(T) <= 16 * 1024 ? (int)per : 0;
  const size_t lds = (size_t)max_staged * sizeof(T);
#define NGD_CALL(ID, B, NK, R)                                                            \
  case ID: {                                                                              \
    hipLaunchKernelGGL((grad_rows_kernel<T, NK, R, B>), dim3(nwg), dim3(B), lds, s, J, ldJ, N, r, partial,      \
                       max_staged);                                                       \
    break;                                                                                \
  }
  NGD_CFG_DISPATCH(c.id, NGD_CALL)
#undef NGD_CALL
  NGD_HIP_TRY(hipGetLastError());
  return NGD_OK;
}

ngd_status launch_grad_rows(int dtype, const void* J, int64_t ldJ, int64_t N, const void* r, void* partial, int nwg,
                            hipStream_t s) {
  if (dtype == NGD_F64) return grad_rows_t<double>((const double*)J, ldJ, N, (const double*)r, (double*)partial, nwg, s);
  return grad_rows_t<float>((const float*)J, ldJ, N, (const float*)r, (float*)partial, nwg, s);
}

ngd_status launch_gram_rows(int dtype, const void* J, int64_t ldJ, int64_t N, int64_t P, const double* v,
                            void* partial, double* tsq, int nwg, hipStream_t s, LaunchEvents ev) {
  if (dtype == NGD_F64)
    return gram_rows_t<double>((const double*)J, ldJ, N, P, v, (double*)partial, tsq, nwg, s, ev);
  return gram_rows_t<float>((const float*)J, ldJ, N, P, v, (float*)partial, tsq, nwg, s, ev);
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

ngd_status pcg_launch_direction(int dtype, const double* z, const double* p_prev, int64_t P, double* p_cur, void* p_t,
                                double* part, PcgState* st, hipStream_t s) {
  dim3 grid((unsigned)((P + 255) / 256));
  if (dtype == NGD_F64)
    hipLaunchKernelGGL(pcg_direction_kernel<double>, grid, dim3(256), 0, s, z, p_prev, P, p_cur, (double*)p_t, part,
                       st);
  else
    hipLaunchKernelGGL(pcg_direction_kernel<float>, grid, dim3(256), 0, s, z, p_prev, P, p_cur, (float*)p_t, part, st);
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
                             double* p_cur, PcgState* st, T* partial, double* tsq, int nwg, hipStream_t s,
                             LaunchEvents ev) {
  RowsCfg c;
  if (!rows_cfg(sizeof(T) == 8 ? NGD_F64 : NGD_F32, ldJ, &c)) {
    set_error("Jacobian row too long for the one-pass matvec");
    return NGD_ERR_INVALID;
  }
  const size_t lds = (size_t)ldJ * sizeof(T);
#define NGD_CALL(ID, B, NK, R)                                                                          \
  case ID: {                                                                                            \
    auto k = pcg_rows_kernel<T, NK, R, B>;                                                              \
    NGD_HIP_TRY(hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds)); \
    hipExtLaunchKernelGGL(k, dim3(nwg), dim3(B), (uint32_t)lds, s, ev.start, ev.stop, 0u, J, ldJ, N, P, z, \
                          p_prev, p_cur, st, partial, tsq);                                             \
    break;                                                                                              \
  }
  NGD_CFG_DISPATCH(c.id, NGD_CALL)
#undef NGD_CALL
  NGD_HIP_TRY(hipGetLastError());
  return NGD_OK;
}

ngd_status pcg_launch_rows(int dtype, const void* J, int64_t ldJ, int64_t N, int64_t P, const double* z,
                           const double* p_prev, double* p_cur, PcgState* st, void* partial, double* tsq, int nwg,
                           hipStream_t s, LaunchEvents ev) {
  if (dtype == NGD_F64)
    return pcg_rows_t<double>((const double*)J, ldJ, N, P, z, p_prev, p_cur, st, (double*)partial, tsq, nwg, s, ev);
  return pcg_rows_t<float>((const float*)J, ldJ, N, P, z, p_prev, p_cur, st, (float*)partial, tsq, nwg, s, ev);
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

// column chunks of the preconditioner dots: enough workgroups to cover the device, chunks of at
// least 1024 columns, at most kDotChunksMax (the size of the partial buffer, kDotChunksMax x ell)
int precond_dot_chunks(int64_t P, int ell) {
  const int64_t rowblocks = (ell + kDotRows - 1) / kDotRows;
  int64_t nc = (1024 + rowblocks - 1) / rowblocks;
  if (nc > P / 1024) nc = P / 1024;
  if (nc > kDotChunksMax) nc = kDotChunksMax;
  return (int)(nc < 1 ? 1 : nc);
}

ngd_status pcg_launch_precond(int dtype, const void* U, int64_t ldU, int64_t P, int ell, const double* lam,
                              double* sbuf, const double* r, double* z, double* rz_part, PcgState* st, hipStream_t s) {
  if (ell < 1 || P < 1) {
    set_error("preconditioner with no rows or no columns");
    return NGD_ERR_INVALID;
  }
  const size_t lds = (size_t)ell * sizeof(double);
  const int nchunk = precond_dot_chunks(P, ell);
  const int64_t chunk = (P + nchunk - 1) / nchunk;
  const dim3 dgrid((unsigned)((ell + kDotRows - 1) / kDotRows), (unsigned)nchunk);
  const dim3 agrid((unsigned)((P + kApCols - 1) / kApCols));
  const size_t esz = dtype == NGD_F64 ? 8 : 4;
  const bool vec = ldU % 2 == 0 && (reinterpret_cast<uintptr_t>(U) % (2 * esz)) == 0;
#define NGD_APPLY(TT, VV)                                                                                      \
  do {                                                                                                         \
    auto k = precond_apply_cols_kernel<TT, VV>;                                                                \
    NGD_HIP_TRY(hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));   \
    hipLaunchKernelGGL(k, agrid, dim3(64 * kApWaves), lds, s, (const TT*)U, ldU, P, ell, lam, sbuf, nchunk,     \
                       r, z, rz_part, st);                                                                     \
  } while (0)
  if (dtype == NGD_F64) {
    hipLaunchKernelGGL(precond_dots_chunk_kernel<double>, dgrid, dim3(256), 0, s, (const double*)U, ldU, P, ell, chunk,
                       r, sbuf, st);
    if (vec) NGD_APPLY(double, true); else NGD_APPLY(double, false);
  } else {
    hipLaunchKernelGGL(precond_dots_chunk_kernel<float>, dgrid, dim3(256), 0, s, (const float*)U, ldU, P, ell, chunk,
                       r, sbuf, st);
    if (vec) NGD_APPLY(float, true); else NGD_APPLY(float, false);
  }
#undef NGD_APPLY
  NGD_HIP_TRY(hipGetLastError());
  return NGD_OK;
}

// ---------------- batched PCG launchers ----------------

ngd_status pcg_batch_launch_init(int dtype, const PcgBatchItem* items, int n, int total_elem, hipStream_t s) {
  (void)dtype;
  if (total_elem <= 0) return NGD_OK;
  hipLaunchKernelGGL(pcg_batch_init_kernel, dim3((unsigned)total_elem), dim3(256), 0, s, items, n);
  NGD_HIP_TRY(hipGetLastError());
  return NGD_OK;
}

ngd_status pcg_batch_launch_damping(const PcgBatchItem* items, PcgState* states, int n, double c_lam, double c_loss,
                                    hipStream_t s) {
  if (n <= 0) return NGD_OK;
  hipLaunchKernelGGL(pcg_batch_damping_kernel, dim3((unsigned)((n + 63) / 64)), dim3(64), 0, s, items, states, n, c_lam,
                     c_loss);
  NGD_HIP_TRY(hipGetLastError());
  return NGD_OK;
}

ngd_status pcg_batch_prepare(int dtype, int64_t max_ldJ, int max_ell) {
  RowsCfg c;
  if (!rows_cfg(dtype, max_ldJ, &c)) {
    set_error("Jacobian row too long for the one-pass matvec");
    return NGD_ERR_INVALID;
  }
  const int lds = (int)(max_ldJ * (dtype == NGD_F64 ? 8 : 4));
#define NGD_CALL(ID, B, NK, R)                                                                                   \
  case ID: {                                                                                                     \
    if (dtype == NGD_F64)                                                                                        \
      NGD_HIP_TRY(hipFuncSetAttribute((const void*)pcg_batch_rows_kernel<double, NK, R, B>,                     \
                                      hipFuncAttributeMaxDynamicSharedMemorySize, lds));                        \
    else                                                                                                         \
      NGD_HIP_TRY(hipFuncSetAttribute((const void*)pcg_batch_rows_kernel<float, NK, R, B>,                      \
                                      hipFuncAttributeMaxDynamicSharedMemorySize, lds));                        \
    break;                                                                                                       \
  }
  NGD_CFG_DISPATCH(c.id, NGD_CALL)
#undef NGD_CALL
  const int plds = (int)(max_ell * sizeof(double));
  NGD_HIP_TRY(hipFuncSetAttribute((const void*)pcg_batch_apply_kernel<double>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, plds));
  NGD_HIP_TRY(hipFuncSetAttribute((const void*)pcg_batch_apply_kernel<float>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, plds));
  return NGD_OK;
}

ngd_status pcg_batch_launch_rows(int dtype, const PcgBatchItem* items, int n, int total_rows, int64_t max_ldJ,
                                 hipStream_t s) {
  RowsCfg c;
  if (!rows_cfg(dtype, max_ldJ, &c)) {
    set_error("Jacobian row too long for the one-pass matvec");
    return NGD_ERR_INVALID;
  }
  const size_t lds = (size_t)max_ldJ * (dtype == NGD_F64 ? 8 : 4);
#define NGD_CALL(ID, B, NK, R)                                                                            \
  case ID: {                                                                                              \
    if (dtype == NGD_F64)                                                                                 \
      hipLaunchKernelGGL((pcg_batch_rows_kernel<double, NK, R, B>), dim3((unsigned)total_rows), dim3(B), lds, s, \
                         items, n);                                                                      \
    else                                                                                                  \
      hipLaunchKernelGGL((pcg_batch_rows_kernel<float, NK, R, B>), dim3((unsigned)total_rows), dim3(B), lds, s, \
                         items, n);                                                                      \
    break;                                                                                                \
  }
  NGD_CFG_DISPATCH(c.id, NGD_CALL)
#undef NGD_CALL
  NGD_HIP_TRY(hipGetLastError());
  return NGD_OK;
}

ngd_status pcg_batch_launch_update(int dtype, const PcgBatchItem* items, int n, int total_upd, hipStream_t s) {
  if (dtype == NGD_F64)
    hipLaunchKernelGGL(pcg_batch_update_kernel<double>, dim3((unsigned)total_upd), dim3(256), 0, s, items, n);
  else
    hipLaunchKernelGGL(pcg_batch_update_kernel<float>, dim3((unsigned)total_upd), dim3(256), 0, s, items, n);
  NGD_HIP_TRY(hipGetLastError());
  return NGD_OK;
}

ngd_status pcg_batch_launch_precond(int dtype, const PcgBatchItem* items, int n, int total_dots, int total_apply,
                                    int max_ell, hipStream_t s) {
  if (total_dots <= 0) return NGD_OK;
  const size_t lds = (size_t)max_ell * sizeof(double);
  if (dtype == NGD_F64) {
    hipLaunchKernelGGL(pcg_batch_dots_kernel<double>, dim3((unsigned)total_dots), dim3(256), 0, s, items, n);
    hipLaunchKernelGGL(pcg_batch_apply_kernel<double>, dim3((unsigned)total_apply), dim3(256), lds, s, items, n);
  } else {
    hipLaunchKernelGGL(pcg_batch_dots_kernel<float>, dim3((unsigned)total_dots), dim3(256), 0, s, items, n);
    hipLaunchKernelGGL(pcg_batch_apply_kernel<float>, dim3((unsigned)total_apply), dim3(256), lds, s, items, n);
  }
  NGD_HIP_TRY(hipGetLastError());
  return NGD_OK;
}

}  // namespace ngd
