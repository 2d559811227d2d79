// Dense contractions on the MFMA matrix cores: C(m,n) = alpha sum_k A(m,k) B(k,n) + beta C(m,n).
//
// Used for the sketch products Z = J_w Omega and J_w^T Q (the ell simultaneous matvecs of the
// "Precompute Jacobian only" strategy, Section 4.1.2 / Table tab:matvec_costs, and Alg. 6's
// Y = G Omega), and for the FP64 products of the ell x ell Nystrom core. Operands are read with
// either layout (K-contiguous or M/N-contiguous), converted to the compute type while they are
// staged in LDS (FP32 -> BF16 for the BF16 sketch, FP32 -> FP64 for the FP64 core), and multiplied
// with v_mfma_f64_16x16x4f64, v_mfma_f32_16x16x4f32 or v_mfma_f32_16x16x32_bf16.
//
// Tiling: 256 threads = 4 wave64s in a 2 x 2 arrangement; workgroup tile BM x BN = 64 x 64, each
// wave a 32 x 32 block of 2 x 2 MFMA tiles. The next K-slab is fetched into registers while the
// current one is multiplied out of LDS. Blocks that share an A row-panel are adjacent in launch
// order so the panel is reused from L2. FP64 compute has its own kernel (dgemm_kernel: double-
// buffered LDS, vector loads, and a symmetric mode for the Gram matrices of the core).
#include "common.h"

namespace ngd {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef double d4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

constexpr int BM = 64, BN = 64, NT = 256;

template <typename E> struct Cfg;
template <> struct Cfg<float> { static constexpr int BK = 16; };
template <> struct Cfg<__bf16> { static constexpr int BK = 32; };

template <typename TS>
__device__ __forceinline__ TS ldg(const TS* p) { return *p; }

// Stage a BM x BK tile of A (or BN x BK of B^T) into registers: element (row, k) of the tile.
// kmajor: X(row, k) = X[row*ld + k]; otherwise X[k*ld + row].
template <typename TS, typename E, int BK, int ROWS>
struct Stager {
  static constexpr int PER = ROWS * BK / NT;
  E v[PER];
  __device__ __forceinline__ void load(const TS* __restrict__ X, int64_t ld, bool kmajor, int64_t row0, int64_t nrows,
                                       int64_t k0, int64_t K) {
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      const int idx = threadIdx.x + e * NT;
      int r, k;
      if (kmajor) { k = idx % BK; r = idx / BK; }
      else { r = idx % ROWS; k = idx / ROWS; }
      const int64_t gr = row0 + r, gk = k0 + k;
      E val = E(0);
      if (gr < nrows && gk < K) val = (E)(kmajor ? ldg(X + gr * ld + gk) : ldg(X + gk * ld + gr));
      v[e] = val;
    }
  }
  // LDS layout: [row][BK + PAD] (k contiguous) for bf16, [k][ROWS + PAD] otherwise
  __device__ __forceinline__ void store(E* lds, bool kmajor) const {
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      const int idx = threadIdx.x + e * NT;
      int r, k;
      if (kmajor) { k = idx % BK; r = idx / BK; }
      else { r = idx % ROWS; k = idx / ROWS; }
      if constexpr (sizeof(E) == 2) lds[r * (BK + 8) + k] = v[e];
      else lds[k * (ROWS + 4) + r] = v[e];
    }
  }
};

template <typename TA, typename TB, typename TC, typename E>
__global__ __launch_bounds__(NT) void gemm_kernel(int64_t M, int64_t N, int64_t K, const TA* __restrict__ A,
                                                  int64_t lda, int a_kmajor, const TB* __restrict__ B, int64_t ldb,
                                                  int b_kmajor, TC* __restrict__ C, int64_t ldc, double alpha,
                                                  double beta, int n_tiles_n, int64_t kchunk,
                                                  double* __restrict__ work) {
  constexpr int BK = Cfg<E>::BK;
  constexpr bool IS_BF = sizeof(E) == 2;
  constexpr int A_ELEMS = IS_BF ? BM * (BK + 8) : BK * (BM + 4);
  constexpr int B_ELEMS = IS_BF ? BN * (BK + 8) : BK * (BN + 4);
  __shared__ __align__(16) E As[A_ELEMS];
  __shared__ __align__(16) E Bs[B_ELEMS];
  using Acc = f4;

  const int tile = blockIdx.x;
  const int64_t m0 = (int64_t)(tile / n_tiles_n) * BM;
  const int64_t n0 = (int64_t)(tile % n_tiles_n) * BN;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int wm = (wid >> 1) * 32, wn = (wid & 1) * 32;

  Acc acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = Acc{};

  Stager<TA, E, BK, BM> sa;
  Stager<TB, E, BK, BN> sb;
  const int64_t kbeg = (int64_t)blockIdx.y * kchunk;
  const int64_t kend = (kbeg + kchunk) < K ? (kbeg + kchunk) : K;
  sa.load(A, lda, a_kmajor, m0, M, kbeg, kend);
  sb.load(B, ldb, b_kmajor, n0, N, kbeg, kend);
  for (int64_t k0 = kbeg; k0 < kend; k0 += BK) {
    __syncthreads();
    sa.store(As, a_kmajor);
    sb.store(Bs, b_kmajor);
    __syncthreads();
    if (k0 + BK < kend) {
      sa.load(A, lda, a_kmajor, m0, M, k0 + BK, kend);
      sb.load(B, ldb, b_kmajor, n0, N, k0 + BK, kend);
    }
    if constexpr (IS_BF) {
      bf8 a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const E* pa = As + (wm + i * 16 + (lane & 15)) * (BK + 8) + 8 * (lane >> 4);
        const E* pb = Bs + (wn + i * 16 + (lane & 15)) * (BK + 8) + 8 * (lane >> 4);
        a[i] = *reinterpret_cast<const bf8*>(pa);
        b[i] = *reinterpret_cast<const bf8*>(pb);
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    } else {
#pragma unroll
      for (int kk = 0; kk < BK; kk += 4) {
        const int kr = kk + (lane >> 4);
        E a[2], b[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          a[i] = As[kr * (BM + 4) + wm + i * 16 + (lane & 15)];
          b[i] = Bs[kr * (BN + 4) + wn + i * 16 + (lane & 15)];
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
      }
    }
  }
  // epilogue: lane holds column lane % 16 of each 16 x 16 tile, rows 4*(lane/16) + r (the lane
  // layout of the FP32-accumulating instructions)
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row_in_tile = 4 * (lane >> 4) + r;
        const int64_t gm = m0 + wm + i * 16 + row_in_tile;
        const int64_t gn = n0 + wn + j * 16 + (lane & 15);
        if (gm < M && gn < N) {
          if (work != nullptr) {  // split-K: raw partial sum of this K-slice
            work[((int64_t)blockIdx.y * M + gm) * N + gn] = (double)acc[i][j][r];
          } else {
            double v = alpha * (double)acc[i][j][r];
            if (beta != 0.0) v += beta * (double)C[gm * ldc + gn];
            C[gm * ldc + gn] = (TC)v;
          }
        }
      }
}

// sum over the ks slices (stride `count`) of element idx, added in slice order (deterministic), with
// eight loads in flight
template <typename T>
__device__ __forceinline__ T sum_slices(const T* __restrict__ work, int ks, int64_t count, int64_t idx) {
  T acc = 0;
  int s = 0;
  for (; s + 8 <= ks; s += 8) {
    T v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = work[(int64_t)(s + u) * count + idx];
#pragma unroll
    for (int u = 0; u < 8; ++u) acc += v[u];
  }
  for (; s < ks; ++s) acc += work[(int64_t)s * count + idx];
  return acc;
}

// C = alpha * sum_s work[s] + beta * C, slices summed in a fixed order (deterministic)
template <typename TC>
__global__ void splitk_reduce_kernel(const double* __restrict__ work, int ks, int64_t M, int64_t N, TC* __restrict__ C,
                                     int64_t ldc, double alpha, double beta) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= M * N) return;
  const int64_t m = idx / N, n = idx - m * N;
  const double acc = sum_slices(work, ks, M * N, idx);
  double v = alpha * acc;
  if (beta != 0.0) v += beta * (double)C[m * ldc + n];
  C[m * ldc + n] = (TC)v;
}

// ---- FP64 compute (v_mfma_f64_16x16x4f64) ----
// Same tiling (64 x 64 per workgroup, 32 x 32 per wave), with K-slabs of 16 double-buffered in LDS
// (one barrier per slab), operands fetched four consecutive elements at a time (one vector load
// where the layout and alignment allow it) and converted to FP64 on the way into LDS. With `sym`,
// only the tiles on and below the diagonal of C = A A^T are formed.
constexpr int kDK = 16, kDPad = 4, kDLd = BM + kDPad;

template <typename TS>
struct DStage {
  double v[4];
  int r, k;
  __device__ __forceinline__ void setup(bool kmajor) {
    const int t = threadIdx.x;
    if (kmajor) { r = t >> 2; k = (t & 3) * 4; }   // 4 consecutive k of one row
    else { k = t >> 4; r = (t & 15) * 4; }         // 4 consecutive rows at one k
  }
  __device__ __forceinline__ void load(const TS* __restrict__ X, int64_t ld, bool kmajor, bool vec, int64_t row0,
                                       int64_t nrows, int64_t k0, int64_t kend) {
    const int64_t gr = row0 + r, gk = k0 + k;
    if (kmajor) {
      const TS* p = X + gr * ld + gk;
      if (vec && gr < nrows && gk + 3 < kend) {
        if constexpr (sizeof(TS) == 4) {
          const float4 q = *reinterpret_cast<const float4*>(p);
          v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
        } else {
          const double2 q0 = *reinterpret_cast<const double2*>(p), q1 = *reinterpret_cast<const double2*>(p + 2);
          v[0] = q0.x; v[1] = q0.y; v[2] = q1.x; v[3] = q1.y;
        }
      } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) v[j] = (gr < nrows && gk + j < kend) ? (double)p[j] : 0.0;
      }
    } else {
      const TS* p = X + gk * ld + gr;
      if (vec && gk < kend && gr + 3 < nrows) {
        if constexpr (sizeof(TS) == 4) {
          const float4 q = *reinterpret_cast<const float4*>(p);
          v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
        } else {
          const double2 q0 = *reinterpret_cast<const double2*>(p), q1 = *reinterpret_cast<const double2*>(p + 2);
          v[0] = q0.x; v[1] = q0.y; v[2] = q1.x; v[3] = q1.y;
        }
      } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) v[j] = (gk < kend && gr + j < nrows) ? (double)p[j] : 0.0;
      }
    }
  }
  // LDS tile [k][row] (pitch kDLd)
  __device__ __forceinline__ void store(double* lds, bool kmajor) const {
    if (kmajor) {
#pragma unroll
      for (int j = 0; j < 4; ++j) lds[(k + j) * kDLd + r] = v[j];
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j) lds[k * kDLd + r + j] = v[j];
    }
  }
};

// lower tile t (row-major over the lower triangle) -> (tile row, tile column)
__device__ __forceinline__ void lower_tile(int t, int& tm, int& tn) {
  int m = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
  while ((m + 1) * (m + 2) / 2 <= t) ++m;
  while (m * (m + 1) / 2 > t) --m;
  tm = m;
  tn = t - m * (m + 1) / 2;
}

template <typename TA, typename TB, typename TC>
__global__ __launch_bounds__(NT) void dgemm_kernel(int64_t M, int64_t N, int64_t K, const TA* __restrict__ A,
                                                   int64_t lda, int a_kmajor, int a_vec, const TB* __restrict__ B,
                                                   int64_t ldb, int b_kmajor, int b_vec, TC* __restrict__ C,
                                                   int64_t ldc, double alpha, double beta, int n_tiles_n, int sym,
                                                   int64_t kchunk, double* __restrict__ work) {
  __shared__ __align__(16) double As[2][kDK * kDLd];
  __shared__ __align__(16) double Bs[2][kDK * kDLd];
  int tm, tn;
  if (sym) lower_tile((int)blockIdx.x, tm, tn);
  else { tm = (int)blockIdx.x / n_tiles_n; tn = (int)blockIdx.x % n_tiles_n; }
  const int64_t m0 = (int64_t)tm * BM, n0 = (int64_t)tn * BN;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int wm = (wid >> 1) * 32, wn = (wid & 1) * 32;
  d4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};
  DStage<TA> sa;
  DStage<TB> sb;
  sa.setup(a_kmajor);
  sb.setup(b_kmajor);
  const int64_t kbeg = (int64_t)blockIdx.y * kchunk;
  const int64_t kend = (kbeg + kchunk) < K ? (kbeg + kchunk) : K;
  sa.load(A, lda, a_kmajor, a_vec, m0, M, kbeg, kend);
  sb.load(B, ldb, b_kmajor, b_vec, n0, N, kbeg, kend);
  sa.store(As[0], a_kmajor);
  sb.store(Bs[0], b_kmajor);
  __syncthreads();
  int buf = 0;
  for (int64_t k0 = kbeg; k0 < kend; k0 += kDK) {
    const bool more = k0 + kDK < kend;
    if (more) {
      sa.load(A, lda, a_kmajor, a_vec, m0, M, k0 + kDK, kend);
      sb.load(B, ldb, b_kmajor, b_vec, n0, N, k0 + kDK, kend);
    }
    const double* as = As[buf];
    const double* bs = Bs[buf];
#pragma unroll
    for (int kk = 0; kk < kDK; kk += 4) {
      const int kr = kk + (lane >> 4);
      double a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        a[i] = as[kr * kDLd + wm + i * 16 + (lane & 15)];
        b[i] = bs[kr * kDLd + wn + i * 16 + (lane & 15)];
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    if (more) {
      sa.store(As[buf ^ 1], a_kmajor);
      sb.store(Bs[buf ^ 1], b_kmajor);
    }
    __syncthreads();
    buf ^= 1;
  }
  // lane holds column lane % 16 of each 16 x 16 tile, rows lane / 16 + 4 r
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t gm = m0 + wm + i * 16 + (lane >> 4) + 4 * r;
        const int64_t gn = n0 + wn + j * 16 + (lane & 15);
        if (gm < M && gn < N) {
          if (work != nullptr) {
            work[((int64_t)blockIdx.y * M + gm) * N + gn] = acc[i][j][r];
          } else {
            double v = alpha * acc[i][j][r];
            if (beta != 0.0) v += beta * (double)C[gm * ldc + gn];
            C[gm * ldc + gn] = (TC)v;
            if (sym == 1 && tm != tn) {
              double w = alpha * acc[i][j][r];
              if (beta != 0.0) w += beta * (double)C[gn * ldc + gm];
              C[gn * ldc + gm] = (TC)w;
            }
          }
        }
      }
}

// split-K reduction of a symmetric product: only the tiles on and below the diagonal are read (the
// partials hold nothing else), each element summed once; with sym == 1 a thread also writes the
// mirror of an element below the diagonal tiles, with sym == 2 the upper tiles are left untouched
template <typename TC>
__global__ void splitk_reduce_sym_kernel(const double* __restrict__ work, int ks, int64_t M, TC* __restrict__ C,
                                         int64_t ldc, double alpha, double beta, int sym) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= M * M) return;
  const int64_t m = idx / M, n = idx - m * M;
  if (m / BM < n / BN) return;  // an upper tile: no partials here
  const double acc = sum_slices(work, ks, M * M, idx);
  double v = alpha * acc;
  if (beta != 0.0) v += beta * (double)C[m * ldc + n];
  C[m * ldc + n] = (TC)v;
  if (sym == 1 && m / BM > n / BN) {
    double w = alpha * acc;
    if (beta != 0.0) w += beta * (double)C[n * ldc + m];
    C[n * ldc + m] = (TC)w;
  }
}

template <typename TS>
bool vec_ok(const void* p, int64_t ld) {
  const int per = sizeof(TS) == 4 ? 4 : 2;
  return (reinterpret_cast<uintptr_t>(p) & 15u) == 0 && ld % per == 0;
}

template <typename TA, typename TB, typename TC>
ngd_status run_f64(const GemmArgs& g, hipStream_t s) {
  const int tn = (int)((g.N + BN - 1) / BN), tm = (int)((g.M + BM - 1) / BM);
  if (g.sym && (g.M != g.N || tm != tn)) {
    set_error("gemm: a symmetric product must be square");
    return NGD_ERR_INVALID;
  }
  const int64_t tiles = g.sym ? (int64_t)tm * (tm + 1) / 2 : (int64_t)tn * tm;
  if (tiles == 0) return NGD_OK;
  int ks = 1;
  if (g.work != nullptr && g.work_elems > 0) {
    // a workgroup keeps one 16-deep slab of each operand in flight, so a long K over few output tiles (the
    // sketch products at small ell) needs several workgroups per CU to cover the memory latency
    while (tiles * ks * 2 <= 4096 && g.K / (ks * 2) >= 8 * kDK && (int64_t)ks * 2 * g.M * g.N <= g.work_elems) ks *= 2;
  }
  const int64_t kchunk = ks == 1 ? g.K : ((g.K + ks - 1) / ks + kDK - 1) / kDK * kDK;
  const int av = vec_ok<TA>(g.A, g.lda), bv = vec_ok<TB>(g.B, g.ldb);
  hipLaunchKernelGGL((dgemm_kernel<TA, TB, TC>), dim3((unsigned)tiles, (unsigned)ks), dim3(NT), 0, s, g.M, g.N, g.K,
                     (const TA*)g.A, g.lda, (int)g.a_kmajor, av, (const TB*)g.B, g.ldb, (int)g.b_kmajor, bv,
                     (TC*)g.C, g.ldc, g.alpha, g.beta, tn, g.sym, kchunk, ks > 1 ? g.work : nullptr);
  NGD_HIP_TRY(hipGetLastError());
  if (ks > 1) {
    const int64_t mn = g.M * g.N;
    if (g.sym)
      hipLaunchKernelGGL(splitk_reduce_sym_kernel<TC>, dim3((unsigned)((mn + 255) / 256)), dim3(256), 0, s, g.work, ks,
                         g.M, (TC*)g.C, g.ldc, g.alpha, g.beta, g.sym);
    else
      hipLaunchKernelGGL(splitk_reduce_kernel<TC>, dim3((unsigned)((mn + 255) / 256)), dim3(256), 0, s, g.work, ks,
                         g.M, g.N, (TC*)g.C, g.ldc, g.alpha, g.beta);
    NGD_HIP_TRY(hipGetLastError());
  }
  return NGD_OK;
}

template <typename TA, typename TB, typename TC, typename E>
ngd_status run(const GemmArgs& g, hipStream_t s) {
  const int tn = (int)((g.N + BN - 1) / BN), tm = (int)((g.M + BM - 1) / BM);
  const int64_t tiles = (int64_t)tn * tm;
  if (tiles == 0) return NGD_OK;
  constexpr int BK = Cfg<E>::BK;
  // split K when the output has too few tiles to fill the chip (Gram matrices of the ell x ell core)
  int ks = 1;
  if (g.work != nullptr && g.work_elems > 0) {
    while (tiles * ks * 2 <= 1024 && g.K / (ks * 2) >= 8 * BK && (int64_t)ks * 2 * g.M * g.N <= g.work_elems) ks *= 2;
  }
  const int64_t kchunk = ks == 1 ? g.K : ((g.K + ks - 1) / ks + BK - 1) / BK * BK;
  hipLaunchKernelGGL((gemm_kernel<TA, TB, TC, E>), dim3((unsigned)tiles, (unsigned)ks), dim3(NT), 0, s, g.M, g.N, g.K,
                     (const TA*)g.A, g.lda, (int)g.a_kmajor, (const TB*)g.B, g.ldb, (int)g.b_kmajor, (TC*)g.C, g.ldc,
                     g.alpha, g.beta, tn, kchunk, ks > 1 ? g.work : nullptr);
  NGD_HIP_TRY(hipGetLastError());
  if (ks > 1) {
    const int64_t mn = g.M * g.N;
    hipLaunchKernelGGL(splitk_reduce_kernel<TC>, dim3((unsigned)((mn + 255) / 256)), dim3(256), 0, s, g.work, ks, g.M,
                       g.N, (TC*)g.C, g.ldc, g.alpha, g.beta);
    NGD_HIP_TRY(hipGetLastError());
  }
  return NGD_OK;
}

template <typename E>
ngd_status dispatch_types(const GemmArgs& g, hipStream_t s) {
  const bool a64 = g.a_type == NGD_F64, b64 = g.b_type == NGD_F64, c64 = g.c_type == NGD_F64;
  if constexpr (sizeof(E) == 8) {
    if (a64 && b64 && c64) return run_f64<double, double, double>(g, s);
    if (!a64 && !b64 && !c64) return run_f64<float, float, float>(g, s);
    if (!a64 && !b64 && c64) return run_f64<float, float, double>(g, s);
    if (!a64 && b64 && c64) return run_f64<float, double, double>(g, s);
    if (!a64 && b64 && !c64) return run_f64<float, double, float>(g, s);
    if (a64 && !b64 && !c64) return run_f64<double, float, float>(g, s);
    if (a64 && !b64 && c64) return run_f64<double, float, double>(g, s);
    return run_f64<double, double, float>(g, s);
  } else {
    if (g.sym) {
      set_error("gemm: symmetric products need FP64 compute");
      return NGD_ERR_INVALID;
    }
    if (a64 && b64 && c64) return run<double, double, double, E>(g, s);
    if (!a64 && !b64 && !c64) return run<float, float, float, E>(g, s);
    if (!a64 && !b64 && c64) return run<float, float, double, E>(g, s);
    if (!a64 && b64 && c64) return run<float, double, double, E>(g, s);
    if (!a64 && b64 && !c64) return run<float, double, float, E>(g, s);
    if (a64 && !b64 && !c64) return run<double, float, float, E>(g, s);
    if (a64 && !b64 && c64) return run<double, float, double, E>(g, s);
    return run<double, double, float, E>(g, s);
  }
}

}  // namespace

ngd_status launch_gemm(const GemmArgs& g, hipStream_t s) {
  if (g.M < 0 || g.N < 0 || g.K < 0) {
    set_error("gemm: negative size");
    return NGD_ERR_INVALID;
  }
  switch (g.compute) {
    case G_F64: return dispatch_types<double>(g, s);
    case G_F32: return dispatch_types<float>(g, s);
    default: return dispatch_types<__bf16>(g, s);
  }
}

}  // namespace ngd
