// Internal declarations shared by the libngd HIP sources (not part of the public ABI).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <type_traits>

#include "../../include/ngd.h"

namespace ngd {

constexpr int kMaxLayers = 8;   // affine layers
constexpr int kMaxDim = 6;      // input dimension d
constexpr int kMaxWidth = 256;
constexpr int kMaxEll = 1024;   // sketch size: the ell x ell core kernels hold their operands in registers
constexpr int kMaxChan = 8;     // value + |S| gradient + Laplacian + time <= 1 + 5 + 1 + 1

// Network and PDE description passed by value to the kernels.
struct NetDesc {
  int n_layers;                  // affine layers
  int widths[kMaxLayers + 1];
  int64_t woff[kMaxLayers];      // offset of W_l in theta
  int64_t boff[kMaxLayers];      // offset of b_l in theta
  int d;                         // input dimension
  int nS;                        // Laplacian coordinates (first nS inputs)
  int has_t;                     // heat: input d-1 is time
  int C;                         // channels: 1 + nS + 1 + has_t
  int pde;
  int max_width;
  int64_t P;
};

// Two networks of the Navier-Stokes rows (velocity: widths[n_layers] = 2 outputs; pressure: the same
// input and hidden widths, one output), theta = [theta_u, theta_p].
struct NsDesc {
  int n_layers;                  // affine layers of each network
  int widths[kMaxLayers + 1];    // the velocity network
  int64_t toff[2];               // start of each network's parameters in theta
  int64_t tl[2][kMaxLayers];     // offset of layer l's W within its network's parameters
  int wl[2][kMaxLayers];         // LDS offset of layer l's staged rows (n_out x (n_in + 1))
  int w_elems;                   // LDS elements of both networks' staged weights
  int64_t P;
  double nu;                     // viscosity
};

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): 10 rounds of two 32x32->64 multiplications,
// word recombination with the key, and a Weyl increment of the key between rounds.
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
  constexpr uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u, W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += W0;
      k1 += W1;
    }
    const uint64_t p0 = (uint64_t)M0 * c[0];
    const uint64_t p1 = (uint64_t)M1 * c[2];
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
  }
}

__device__ __forceinline__ double u53(uint32_t a, uint32_t b) {
  const uint64_t v = ((uint64_t)(a >> 5) << 26) + (uint64_t)(b >> 6);
  return ((double)v + 0.5) * 1.1102230246251565e-16;  // 2^-53
}

// Device-side solver state of one PCG solve (FP64 scalars).
struct PcgState {
  double rz;        // r^T z of the current iterate
  double rr;        // r^T r
  double bnorm2;    // ||g||^2
  double alpha;
  double beta;      // used to form the next search direction
  double pp;        // ||p||^2 of the current search direction
  double lambda;
  double rtol2bb;   // rtol^2 ||g||^2
  double mu_c;      // preconditioner: 1 / (lam_ell + mu)
  long long iters;
  long long maxit;
  int done;
  int converged;
  int breakdown;
  unsigned counter; // arrival counter for last-block reductions
  int sketch_err;   // the core of the sketch behind the preconditioner timed out (checked when asked)
};

void set_error(const std::string& msg);

#define NGD_HIP_TRY(expr)                                                        \
  do {                                                                           \
    hipError_t e_ = (expr);                                                      \
    if (e_ != hipSuccess) {                                                      \
      ::ngd::set_error(std::string(#expr) + ": " + hipGetErrorString(e_));       \
      (void)hipGetLastError(); /* leave no stale error for the caller's checks */ \
      return NGD_ERR_HIP;                                                        \
    }                                                                            \
  } while (0)

// propagate a non-OK status
#define NGD_TRY(expr)                 \
  do {                                \
    ngd_status st_ = (expr);          \
    if (st_ != NGD_OK) return st_;    \
  } while (0)

// ---- device helpers -----------------------------------------------------------------------------

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Wave-wide sum by DPP row operations (quad permutes, row mirrors, then row broadcasts 15 and 31;
// the total lands in lane 63 and is read from there): a few VALU cycles per step instead of an LDS
// permute. Every lane of the wave must be active.
template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ float dpp_move(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, ROW_MASK, 0xf, false));
}
template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ double dpp_move(double x) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), CTRL, ROW_MASK, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), CTRL, ROW_MASK, 0xf, false);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float lane63(float x) { return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 63)); }
__device__ __forceinline__ double lane63(double x) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(x), 63),
                          __builtin_amdgcn_readlane(__double2loint(x), 63));
}
template <typename T>
__device__ __forceinline__ T wave_sum_dpp(T x) {
  x += dpp_move<0xb1>(x);         // quad_perm [1, 0, 3, 2]
  x += dpp_move<0x4e>(x);         // quad_perm [2, 3, 0, 1]
  x += dpp_move<0x141>(x);        // row_half_mirror
  x += dpp_move<0x140>(x);        // row_mirror: every lane holds its row's sum
  x += dpp_move<0x142, 0xa>(x);   // row_bcast:15 into rows 1 and 3
  x += dpp_move<0x143, 0xc>(x);   // row_bcast:31 into rows 2 and 3
  return lane63(x);
}

// Block sum with wave_sum_dpp (every lane of every wave active)
template <typename T>
__device__ __forceinline__ T block_sum_dpp(T v, T* red) {
  v = wave_sum_dpp(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  T s = 0;
  for (int i = 0; i < nw; ++i) s += red[i];
  return s;
}

// Block-wide sum; `red` must hold blockDim.x/64 elements. Result is returned to every thread.
template <typename T>
__device__ __forceinline__ T block_sum(T v, T* red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  T s = 0;
  for (int i = 0; i < nw; ++i) s += red[i];
  return s;
}

// Sum of a[0..n) by the whole block in a fixed order (strided per-thread sums, then block_sum):
// deterministic for a given blockDim. Every thread gets the result.
__device__ __forceinline__ double block_sum_array(const double* __restrict__ a, int n, double* red) {
  double s = 0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) s += a[i];
  return block_sum(s, red);
}

// Deterministic two-stage reduction inside one launch. Block `bid` publishes its partial v (the same
// value in every thread) to part[bid] with a device-coherent (sc1) store, waits for that store to
// complete, and counts itself in; the block that arrives last reads all partials with
// device-coherent loads and returns true with their fixed-order sum in *total (every thread), then
// re-arms the counter for the next launch. No L2 write-back or invalidate is involved.
__device__ __forceinline__ bool publish_and_reduce(double v, double* part, int bid, unsigned* counter,
                                                   unsigned nblocks, double* red, double* total) {
  __shared__ int last;
  if (threadIdx.x == 0) {
    __hip_atomic_store(part + bid, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    const unsigned prev = __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    last = prev == nblocks - 1;
  }
  __syncthreads();
  if (!last) return false;
  double s = 0;
  for (int i = threadIdx.x; i < (int)nblocks; i += blockDim.x)
    s += __hip_atomic_load(part + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  *total = block_sum(s, red);
  if (threadIdx.x == 0) __hip_atomic_store(counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return true;
}

// ---- launchers (defined in the .hip files) ------------------------------------------------------

// ns.hip
ngd_status ns_describe(int n_layers, const int* widths, double nu, NsDesc* nd);
size_t ns_lds_bytes(const NsDesc& nd, int dtype);
int ns_blocks(int64_t N);
ngd_status launch_ns_residual(const NsDesc& nd, int dtype, const void* theta, int64_t theta_stride, int n_theta,
                              int64_t N, const void* X, const void* w, const void* f, const void* g,
                              const int8_t* kind, void* r_w, void* J, int64_t ldJ, double* loss_partial,
                              hipStream_t s);
ngd_status launch_ns_velocity_error(const NsDesc& nd, int dtype, const void* theta, const void* X, int64_t n,
                                    const void* u_ref, const void* grad_ref, double* part, int max_blocks,
                                    double* sums, hipStream_t s);

// residual.hip
ngd_status launch_residual_jacobian(const NetDesc& net, int dtype, const void* theta, int64_t N,
                                    const void* X, const void* w, const void* f, const void* g,
                                    const int8_t* kind, void* r_w, void* J, int64_t ldJ, double* loss_partial,
                                    int64_t theta_stride, int n_theta, hipStream_t s, int* n_blocks_out);
ngd_status launch_reduce_sum(const double* partial, int64_t n_per, int n_sets, double scale, double* out,
                             hipStream_t s);
// recompute mode: J_w^T wv accumulated into nwg partial rows (ld) and sum wv^2 into tsq[nwg];
// J_w u_j for k directions into out[r * ldo + j * cs]
int vjp_grid(const NetDesc& net, int dtype, int64_t N, int max_wg);
ngd_status launch_vjp(const NetDesc& net, int dtype, const void* theta, int64_t N, const void* X, const void* w,
                      const void* f, const void* g, const int8_t* kind, const double* wv, int64_t wv_stride,
                      void* partial, int64_t ld, double* tsq, int nwg, hipStream_t s);
ngd_status launch_jvp(const NetDesc& net, int dtype, const void* theta, const void* U, int64_t ldU, int64_t k,
                      int64_t N, const void* X, const void* w, const int8_t* kind, int out_type, void* out,
                      int64_t ldo, int64_t cs, hipStream_t s);
ngd_status launch_gradient(int dtype, const void* J, int64_t ldJ, int64_t N, int64_t P, const void* r,
                           double* work, double* grad, hipStream_t s);
int gradient_chunks(int64_t N);

// Events that, when set, the runtime stamps with the start and end of one kernel's own dispatch
// (hipExtLaunchKernel), so that a timer measures the kernel and not the markers around it.
struct LaunchEvents {
  hipEvent_t start = nullptr, stop = nullptr;
};

// matvec.hip
int gram_rows_grid(int dtype, int64_t N, int64_t P);
ngd_status launch_gram_rows(int dtype, const void* J, int64_t ldJ, int64_t N, int64_t P, const double* v,
                            void* partial, double* tsq, int nwg, hipStream_t s, LaunchEvents ev = {});
ngd_status launch_grad_rows(int dtype, const void* J, int64_t ldJ, int64_t N, const void* r, void* partial, int nwg,
                            hipStream_t s);
ngd_status launch_gram_reduce(int dtype, const void* partial, int nwg, int64_t ld, int64_t P, const double* v,
                              double lambda, double* y, hipStream_t s);

// gemm.hip: C(m,n) = alpha * sum_k A(m,k) B(k,n) (+ beta C), row-major C with ldc.
enum GemmType { G_F64 = 0, G_F32 = 1, G_BF16 = 2 };
struct GemmArgs {
  int64_t M, N, K;
  const void* A; int64_t lda; bool a_kmajor;   // A(m,k) = A[m*lda+k] if kmajor else A[k*lda+m]
  const void* B; int64_t ldb; bool b_kmajor;   // B(k,n) = B[n*ldb+k] if kmajor else B[k*ldb+n]
  void* C; int64_t ldc;
  int a_type, b_type, c_type;                  // storage types: NGD_F64 / NGD_F32
  int compute;                                 // GemmType
  double alpha, beta;
  double* work = nullptr;                      // optional split-K workspace (FP64)
  int64_t work_elems = 0;                      // its size in doubles
  // C = A B with B = A^T (M == N), FP64 compute only: 1 = only the tiles on and below the diagonal
  // are formed and mirrored, 2 = only those tiles are formed (the upper part of C is left untouched)
  int sym = 0;
};
ngd_status launch_gemm(const GemmArgs& a, hipStream_t s);

// sketch_gemm.hip: C = alpha A B^T with A (M x K) and B (N x K) K-contiguous (FP32 or BF16 storage),
// FP32 output, C^T stored when trans_c; a_kmajor: A is given as an FP32 K x M matrix (A[m][k] at
// k lda + m) and read without a transposed copy. Also transposed precision copies.
bool nt_gemm_supported(int a_type, int b_type, int compute, int64_t M, int64_t N, int64_t K, int64_t lda,
                       int64_t ldb, bool a_kmajor = false);
ngd_status launch_nt_gemm(int a_type, const void* A, int64_t lda, int b_type, const void* B, int64_t ldb,
                          int compute, int64_t M, int64_t N, int64_t K, int c_type, void* C, int64_t ldc,
                          bool trans_c, double alpha, float* work, int64_t work_elems, hipStream_t s,
                          bool a_kmajor = false);
ngd_status launch_cast_rows(int src_type, const void* src, int64_t ld_s, int64_t rows, int64_t cols, int dst_type,
                            void* dst, int64_t ld_d, hipStream_t s);
ngd_status launch_transpose_cast(int src_type, const void* src, int64_t ld_s, int64_t rows, int64_t cols,
                                 int dst_type, void* dst, int64_t ld_d, hipStream_t s);

// eig.hip: symmetric eigendecomposition of an n x n FP64 matrix (row-major, ld = n), in place.
// Eigenpairs below drop_rel * ||T|| (Gershgorin bound) are returned as zeros. A is overwritten.
// keep_err: leave the error word of an earlier call on the same workspace as it is (its flags are
// cleared either way).
size_t eig_workspace_bytes(int n);
// side, fork, join: a second stream and two events for the part that overlaps (side may be NULL)
ngd_status launch_sym_eig(double* A, int n, double drop_rel, double* evals_desc, double* evecs_rows, void* work,
                          hipStream_t s, hipStream_t side = nullptr, hipEvent_t fork = nullptr,
                          hipEvent_t join = nullptr, bool keep_err = false);
const int* eig_error_flag(void* work, int n);
// The same eigensolver for several matrices: launch_sym_eig_tridiag_batch clears each job's words and
// tridiagonalises every matrix in batched launches on s (one per register shape, the workgroups of
// each matrix meeting only among themselves); launch_sym_eig_finish then completes one job (after
// its tridiagonalisation, on any stream ordered after s). Together they compute what launch_sym_eig
// computes, bitwise.
struct EigJob {
  double* A;
  int n;
  void* work;
  bool keep_err;
  double drop_rel;
  hipStream_t side;   // the job's own second stream for the explicit Q (may be NULL)
  hipEvent_t fork, join;
};
ngd_status launch_sym_eig_tridiag_batch(const EigJob* jobs, int n, hipStream_t s);
// After launch_sym_eig_tridiag_batch: every job's explicit Q on its side stream, then multisection,
// inverse iteration and the cluster orthogonalisation of all jobs in one launch each on s;
// launch_sym_eig_rest then completes one job on any stream ordered after s. Together with the
// tridiagonalisation these compute what launch_sym_eig computes, bitwise.
ngd_status launch_sym_eig_middle_batch(const EigJob* jobs, int n, hipStream_t s);
ngd_status launch_sym_eig_rest(int n, double drop_rel, double* evals_desc, double* evecs_rows, void* work,
                               hipStream_t s, hipStream_t side = nullptr, hipEvent_t join = nullptr);
ngd_status launch_sym_eig_finish(int n, double drop_rel, double* evals_desc, double* evecs_rows, void* work,
                                 hipStream_t s, hipStream_t side = nullptr, hipEvent_t fork = nullptr,
                                 hipEvent_t join = nullptr);

// misc.hip
ngd_status launch_gaussian_omega(int dtype, uint64_t seed, uint64_t counter, int64_t P, int64_t ell, void* out,
                                 int64_t ld, hipStream_t s);
ngd_status launch_cast(int src_type, const void* src, int dst_type, void* dst, int64_t n, hipStream_t s);
// out[t * out_stride + j] = theta[j] - alpha_t d[j], alpha_t = alphas[t] (device), or alpha0 when
// alphas is NULL
ngd_status launch_axpy_theta(int dtype, const void* theta, const double* d, const double* alphas, int n_alpha,
                             int64_t P, void* out, int64_t out_stride, hipStream_t s, double alpha0 = 0.0);
ngd_status launch_sketch_info(const double* lam, int L, const double* core, const int* eig_err, const int* chol_err,
                              double* out, hipStream_t s);
// Armijo decision for nt trials on the device: st = [found, alpha, loss, index] (left as it is once found)
ngd_status launch_woodbury_lam(double* lam, int n, hipStream_t s);
ngd_status launch_lm_damping(const double* gd, const double* dgd, double alpha, double loss0, double loss1, double mu,
                             double floor_mu, double* out, hipStream_t s);
ngd_status launch_armijo(const double* alphas, const double* losses, const double* slope, double loss0, double c1,
                         int nt, int tried, double* st, hipStream_t s);
ngd_status launch_zero(void* p, size_t bytes, hipStream_t s);
// the damping rule of Section 4.3 for n problems (pointer tables in device memory), and Alg. 4's
// sketch-size update (out: device int64)
// the two-level eigendecomposition of the Nystrom core (FP64 problems): split off the pairs that the
// first level resolves, and merge the ones recomputed from the projected B
ngd_status launch_split_top(const double* lam, const double* Ev, int L, double tau, double* lam_t, double* Evt,
                            hipStream_t s);
ngd_status launch_merge_small(int dtype, const double* lam_t, const double* mu, const void* U2, int64_t ld2, int L,
                              int64_t P, double floor_rel, void* U, int64_t ldU, double* lam_hat, hipStream_t s);
ngd_status launch_damping1(const double* lam1, const double* loss, double c_lam, double c_loss, double* mu,
                           hipStream_t s);
ngd_status launch_damping(const double* const* lam1, const double* const* loss, double c_lam, double c_loss,
                          double* const* mu, int n, hipStream_t s);
ngd_status launch_next_rank(const double* lam, int64_t ell, double mu, int64_t dell, int64_t offset,
                            int64_t ell_max, int64_t* out, hipStream_t s);

// pivots.hip: out (+)= column sums of squares of J (N x P, ldJ) through `work` (work_elems doubles);
// ns samples of indices in [0, P) with probability proportional to max(w, 0) (Philox substream q;
// sorted and without duplicates when `unique`; count on the device); gather of columns.
constexpr int kDiagChunks = 64;
constexpr int kRpBlockMax = 64;  // largest RPCholesky block
constexpr int64_t kMaxSamples = 4096;
ngd_status launch_colsq(int dtype, const void* J, int64_t ldJ, int64_t N, int64_t P, double* work,
                        int64_t work_elems, int accumulate, double* out, hipStream_t s);
ngd_status launch_sample_pivots(const double* w, int64_t P, uint64_t seed, uint64_t counter, uint32_t q, int64_t ns,
                                int unique, int64_t* idx, int* count, hipStream_t s, const int64_t* done = nullptr);
// block RPCholesky pieces: W = F[idx, :kmax] (b x ldw) from the rows of F^T; the pivot block's
// Cholesky with dependent pivots dropped, the new rows of F^T, the diagonal downdate and the
// stopping rule. st = {rank, done, kept} (device int64), part = ceil(P/256) doubles.
ngd_status launch_rp_gather_f(const double* Ft, int64_t ldF, const int64_t* idx, int b, int64_t kmax, double* W,
                              int64_t ldw, hipStream_t s);
ngd_status launch_rp_block(const double* Ct, int64_t ldc, const int64_t* idx, const int* count, int64_t* st,
                           int64_t cap, double* Rt, int* keep_rows, int64_t P, double* Ft, int64_t ldF, double* d,
                           double* part, double eps, int b, double* trace_out, hipStream_t s);
ngd_status launch_gather_cols(int dtype, const void* J, int64_t ldJ, int64_t rows, const int64_t* cols, int64_t ncol,
                              void* out, int64_t ld_out, hipStream_t s);

// eval.hip: the four sums of the relative L2 / H1 error of u_theta against (u_ref, grad u_ref) at n
// points: sum (u - u_ref)^2, sum |grad u - grad u_ref|^2, sum u_ref^2, sum |grad u_ref|^2 (FP64,
// device). `part` holds 4 * kEvalBlocks doubles of workgroup partial sums.
constexpr int kEvalBlocks = 1024;
ngd_status launch_solution_error(const NetDesc& net, int dtype, const void* theta, const void* X, int64_t n,
                                 const void* u_ref, const void* grad_u_ref, double* part, double* sums,
                                 hipStream_t s);

// matvec.hip (continued)
bool gram_rows_supported(int dtype, int64_t ldJ);
ngd_status launch_dot(const double* a, const double* b, int64_t n, double* work, double* out, hipStream_t s);
ngd_status launch_scale_rsqrt(const double* w, const double* ww, int64_t n, double* v, hipStream_t s);
ngd_status pcg_launch_init(const double* g, int64_t P, double* x, double* r, double* p_prev, double* part,
                           PcgState* st, double rtol, int plain, hipStream_t s);
ngd_status pcg_launch_rows(int dtype, const void* J, int64_t ldJ, int64_t N, int64_t P, const double* z,
                           const double* p_prev, double* p_cur, PcgState* st, void* partial, double* tsq, int nwg,
                           hipStream_t s, LaunchEvents ev = {});
ngd_status pcg_launch_update(int dtype, const void* partial, int nwg, int64_t ld, int64_t P, const double* p,
                             const double* tsq, double* x, double* r, double* rr_part, PcgState* st, int plain,
                             hipStream_t s);
ngd_status pcg_launch_direction(int dtype, const double* z, const double* p_prev, int64_t P, double* p_cur, void* p_t,
                                double* part, PcgState* st, hipStream_t s);
// column chunks of the preconditioner dots (the partial buffer holds kDotChunksMax x ell doubles)
constexpr int kDotChunksMax = 16;
int precond_dot_chunks(int64_t P, int ell);
// before PCG initialisation: lambda from the damping rule max(c_lam lam_hat[0], c_loss loss^2) when
// lam_hat != NULL, and the sketch's error words (either pointer may be NULL) into st->sketch_err
ngd_status pcg_launch_setup(PcgState* st, const double* lam_hat, double c_lam, const double* loss, double c_loss,
                            const int* eig_err, const unsigned* chol_err, hipStream_t s);
ngd_status pcg_launch_precond(int dtype, const void* U, int64_t ldU, int64_t P, int ell, const double* lam,
                              double* sbuf, const double* r, double* z, double* rz_part, PcgState* st, hipStream_t s);

// Batched PCG (several independent problems per launch): one entry per problem, in device memory.
// The work items of a launch are numbered problem by problem; item0_* is the first item of this
// problem in each kind of launch (row workgroups, update column blocks of 32, preconditioner rows,
// element blocks of 256).
struct PcgBatchItem {
  const void* J;
  int64_t ldJ, N, P;
  const double* g;
  double *x, *r, *z, *p0, *p1, *s, *part;
  void* partial;
  double* tsq;
  PcgState* st;
  const void* U;  // NULL: plain CG
  int64_t ldU;
  const double* lam;
  const double* loss;  // the problem's loss (device) for the damping rule, or NULL
  double mu;
  double rtol;
  int ell, nwg, plain;
  int item0_rows, item0_upd, item0_dots, item0_elem, item0_apply;
};
ngd_status pcg_batch_launch_init(int dtype, const PcgBatchItem* items, int n, int total_elem, hipStream_t s);
ngd_status pcg_batch_launch_precond(int dtype, const PcgBatchItem* items, int n, int total_dots, int total_apply,
                                    int max_ell, hipStream_t s);
ngd_status pcg_batch_launch_rows(int dtype, const PcgBatchItem* items, int n, int total_rows, int64_t max_ldJ,
                                 hipStream_t s);
ngd_status pcg_batch_launch_update(int dtype, const PcgBatchItem* items, int n, int total_upd, hipStream_t s);
// make the kernels of a batched launch ready for stream capture (function attributes set up front)
ngd_status pcg_batch_prepare(int dtype, int64_t max_ldJ, int max_ell);
// the damping rule of Section 4.3 for every problem of a batch: states[i].lambda =
// max(c_lam items[i].lam[0], c_loss items[i].loss[0]^2)
ngd_status pcg_batch_launch_damping(const PcgBatchItem* items, PcgState* states, int n, double c_lam, double c_loss,
                                    hipStream_t s);

// residual.hip: several problems' residuals, Jacobians and loss partials in one launch
struct BatchResidualItem {
  NetDesc net;
  const void *theta, *X, *w, *f, *g;
  const int8_t* kind;
  void *r_w, *J;
  int64_t ldJ, N, first_tile;
  int TP;
  double* loss_part;
};
ngd_status launch_batch_residual_jacobian(int dtype, const BatchResidualItem* items, int n, int64_t total_tiles,
                                          size_t lds_bytes, hipStream_t s);
size_t residual_lds_bytes(const NetDesc& net, int dtype, int* tp);

// chol.hip: blocked shifted Cholesky of the core and the right triangular solve X <- X L^{-T}
ngd_status launch_shifted_cholesky(double* M, int n, double shift_rel, double floor_rel, double* scal, int* nmod,
                                   unsigned* sync, unsigned epoch, hipStream_t s);
ngd_status launch_trsm_q(const double* L, int ell, int z_type, const void* Z, int64_t N, double* Q, int qt_type,
                         void* Qt, int64_t ldqt, hipStream_t s);

// nystrom helpers (misc.hip)
ngd_status launch_whitening(const double* evals, const double* evec_rows, int ell, double* F, hipStream_t s);

// direct.hip: the full-Gramian solve (Alg. 2): blocked Cholesky of a P x P FP64 matrix and the two
// substitutions with it.
size_t direct_panel_inverse_bytes(int64_t P);
size_t direct_stage_bytes(int64_t P);
size_t direct_part_bytes(int64_t P);
ngd_status launch_add_diag(double* A, int64_t ld, int64_t n, double mu, hipStream_t s);
ngd_status launch_blocked_cholesky(double* A, int64_t ld, int64_t P, double* Linv, double* stage, int* info,
                                   hipStream_t s);
ngd_status launch_cholesky_solve(const double* L, int64_t ld, int64_t P, const double* Linv, const double* g,
                                 double* y, double* part, double* d, hipStream_t s);
ngd_status launch_add_scaled(int dtype, const void* X, int64_t ldx, double a, void* Y, int64_t ldy, int64_t rows,
                             int64_t cols, hipStream_t s);
int residual_block_rows(const NetDesc& net, int dtype);
// workgroups (one loss partial each) of a residual launch over N points, with or without the Jacobian
int residual_blocks(const NetDesc& net, int dtype, int64_t N, bool with_jacobian);
// line-search trials (residual-only sweeps) per launch: as many as occupy the device about as long as
// one (1 when a single trial already fills it), at most max_trials
int residual_trials_per_launch(const NetDesc& net, int dtype, int64_t N, int max_trials);

}  // namespace ngd
