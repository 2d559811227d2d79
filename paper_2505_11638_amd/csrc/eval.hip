// Accuracy of the network against a reference solution: u_theta and its input gradient at
// evaluation points, reduced to the four sums behind the relative L2 and H1 errors by which the
// experiments of Section 5 measure accuracy (Monte Carlo over uniform random points; the evaluation
// sets of the appendix's discretisation table). Evaluation only; no part of an NGD step.
#include "common.h"

namespace ngd {
namespace {

constexpr int kEvThreads = 256;
constexpr int kEvMaxD = 8;
constexpr size_t kEvLdsBudget = 64 * 1024;

// One workgroup per tile of tp points, the tiles dealt grid-stride. The activations h (width) and
// their input gradients G (width x d) of every point of the tile live in LDS, one layer at a time;
// each thread forms the next layer's values for one (point, neuron) pair:
//   z = W h + b,  Gz = W G,  a = tanh z,  h' = a,  G' = (1 - a^2) Gz,
// starting from h = x, G = I. The last, linear layer gives u and grad u. Each point's four terms
//   (u - u_ref)^2, |grad u - grad u_ref|^2, u_ref^2, |grad u_ref|^2
// are added to the workgroup's sums by one thread in point order (FP64 throughout), so the result
// does not depend on timing.
template <typename T>
__global__ __launch_bounds__(kEvThreads) void solution_error_kernel(NetDesc net, const T* __restrict__ theta,
                                                                    const T* __restrict__ X, int64_t n, int tp,
                                                                    const T* __restrict__ u_ref,
                                                                    const T* __restrict__ gu_ref,
                                                                    double* __restrict__ part) {
  extern __shared__ double sm[];
  const int d = net.d, mw = net.max_width;
  const int stride = mw * (1 + d);  // per point: h (mw), then G (mw x d, row = neuron)
  double* bufA = sm;
  double* bufB = sm + (size_t)tp * stride;
  double* terms = bufB + (size_t)tp * stride;  // tp x 4
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  const int64_t ntiles = (n + tp - 1) / tp;
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t p0 = tile * tp;
    for (int idx = threadIdx.x; idx < tp * d; idx += blockDim.x) {
      const int p = idx / d, k = idx - p * d;
      const int64_t gp = p0 + p;
      double* hp = bufA + (size_t)p * stride;
      hp[k] = gp < n ? (double)X[gp * d + k] : 0.0;
      for (int c = 0; c < d; ++c) hp[mw + k * d + c] = k == c ? 1.0 : 0.0;
    }
    __syncthreads();
    double* cur = bufA;
    double* nxt = bufB;
    for (int l = 0; l + 1 < net.n_layers; ++l) {
      const int nin = net.widths[l], nout = net.widths[l + 1];
      const T* W = theta + net.woff[l];
      const T* b = theta + net.boff[l];
      for (int idx = threadIdx.x; idx < tp * nout; idx += blockDim.x) {
        const int p = idx / nout, o = idx - p * nout;
        const double* hp = cur + (size_t)p * stride;
        double z = (double)b[o];
        double gz[kEvMaxD];
#pragma unroll
        for (int c = 0; c < kEvMaxD; ++c) gz[c] = 0.0;
        for (int k = 0; k < nin; ++k) {
          const double w = (double)W[(int64_t)o * nin + k];
          z = fma(w, hp[k], z);
#pragma unroll
          for (int c = 0; c < kEvMaxD; ++c)
            if (c < d) gz[c] = fma(w, hp[mw + k * d + c], gz[c]);
        }
        const double a = tanh(z), s1 = 1.0 - a * a;
        double* hq = nxt + (size_t)p * stride;
        hq[o] = a;
#pragma unroll
        for (int c = 0; c < kEvMaxD; ++c)
          if (c < d) hq[mw + o * d + c] = s1 * gz[c];
      }
      __syncthreads();
      double* t = cur;
      cur = nxt;
      nxt = t;
    }
    {
      const int l = net.n_layers - 1, nin = net.widths[l];
      const T* W = theta + net.woff[l];
      const T* b = theta + net.boff[l];
      for (int p = threadIdx.x; p < tp; p += blockDim.x) {
        const int64_t gp = p0 + p;
        double t4[4] = {0.0, 0.0, 0.0, 0.0};
        if (gp < n) {
          const double* hp = cur + (size_t)p * stride;
          double u = (double)b[0];
          double gu[kEvMaxD];
#pragma unroll
          for (int c = 0; c < kEvMaxD; ++c) gu[c] = 0.0;
          for (int k = 0; k < nin; ++k) {
            const double w = (double)W[k];
            u = fma(w, hp[k], u);
#pragma unroll
            for (int c = 0; c < kEvMaxD; ++c)
              if (c < d) gu[c] = fma(w, hp[mw + k * d + c], gu[c]);
          }
          const double ur = (double)u_ref[gp];
          t4[0] = (u - ur) * (u - ur);
          t4[2] = ur * ur;
#pragma unroll
          for (int c = 0; c < kEvMaxD; ++c)
            if (c < d) {
              const double gr = (double)gu_ref[gp * d + c], e = gu[c] - gr;
              t4[1] += e * e;
              t4[3] += gr * gr;
            }
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) terms[p * 4 + k] = t4[k];
      }
      __syncthreads();
      if (threadIdx.x == 0)
        for (int p = 0; p < tp; ++p)
#pragma unroll
          for (int k = 0; k < 4; ++k) acc[k] += terms[p * 4 + k];
      __syncthreads();
    }
  }
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < 4; ++k) part[(int64_t)k * gridDim.x + blockIdx.x] = acc[k];
}

}  // namespace

ngd_status launch_solution_error(const NetDesc& net, int dtype, const void* theta, const void* X, int64_t n,
                                 const void* u_ref, const void* grad_u_ref, double* part, double* sums,
                                 hipStream_t s) {
  if (net.d > kEvMaxD) {
    set_error("solution error: input dimension above 8");
    return NGD_ERR_INVALID;
  }
  if (n == 0) return launch_zero(sums, 4 * sizeof(double), s);
  const size_t stride = (size_t)net.max_width * (1 + net.d);
  int tp = (int)std::min<size_t>(32, kEvLdsBudget / (2 * stride * sizeof(double) + 4 * sizeof(double)));
  if (tp < 1) tp = 1;
  const size_t lds = (2 * (size_t)tp * stride + 4 * (size_t)tp) * sizeof(double);
  const int64_t ntiles = (n + tp - 1) / tp;
  const int grid = (int)std::min<int64_t>(kEvalBlocks, ntiles);
  if (dtype == NGD_F64) {
    NGD_HIP_TRY(hipFuncSetAttribute((const void*)solution_error_kernel<double>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL(solution_error_kernel<double>, dim3(grid), dim3(kEvThreads), lds, s, net,
                       (const double*)theta, (const double*)X, n, tp, (const double*)u_ref,
                       (const double*)grad_u_ref, part);
  } else {
    NGD_HIP_TRY(hipFuncSetAttribute((const void*)solution_error_kernel<float>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL(solution_error_kernel<float>, dim3(grid), dim3(kEvThreads), lds, s, net, (const float*)theta,
                       (const float*)X, n, tp, (const float*)u_ref, (const float*)grad_u_ref, part);
  }
  NGD_HIP_TRY(hipGetLastError());
  return launch_reduce_sum(part, grid, 4, 1.0, sums, s);
}

}  // namespace ngd
