// Residual rows, loss and Gauss-Newton Jacobian of the steady incompressible Navier-Stokes problem
// (the Kovasznay flow of Section 5.1.3, eq. navier_residual): a velocity network with two outputs and
// a pressure network with one, theta = [theta_u, theta_p] (Section 5.1.3), both tanh MLPs (Section 2.3).
//
// Rows: momentum k (k = 1, 2): -nu Laplace u_k + u_1 d_x u_k + u_2 d_y u_k + d_k p - f; continuity
// d_x u_1 + d_y u_2; boundary u_k - g; each times sqrt(w). The Jacobian row is the reverse sweep of the
// Taylor-mode channels (value, d/dx, d/dy, Laplacian) seeded with the derivative of the row's residual
// with respect to the networks' output channels: the Gauss-Newton linearisation of the convective term
// puts the row's own velocity and velocity gradient into the seeds.
//
// Layout: one workgroup stages both networks' weights in LDS once; each of its waves (eight where the
// LDS allows, else four) takes one row at a time, one lane per hidden unit (widths <= 64), the hidden
// layers' output channels in a per-wave LDS scratch with the four channels of a unit side by side (one
// vector read per unit), the pre-activation channels in registers (the depth is a template parameter). The waves of a workgroup never wait for
// each other between rows; lanes of one wave exchange values through LDS behind a wave barrier. The
// Jacobian row is written layer by layer with consecutive lanes on consecutive parameters.
#include "common.h"

namespace ngd {
namespace {

constexpr int kNsWavesMax = 8;

template <typename T>
struct V4t;
template <>
struct V4t<float> {
  typedef float type __attribute__((ext_vector_type(4)));
};
template <>
struct V4t<double> {
  typedef double type __attribute__((ext_vector_type(4)));
};
template <typename T>
using V4 = typename V4t<T>::type;

// LDS writes of one lane made visible to the other lanes of its wave (and the compiler kept from
// moving LDS accesses across the point)
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// sum_i w[i] h[i] + y0 over i < n: four products in flight per step (the LDS reads of a step issue
// together instead of one latency each), two partial sums
template <typename T>
__device__ __forceinline__ V4<T> ns_dot(const T* __restrict__ w, const V4<T>* __restrict__ h, int n, V4<T> y0) {
  V4<T> y1 = {T(0), T(0), T(0), T(0)};
  int i = 0;
  for (; i + 4 <= n; i += 4) {
    const T w0 = w[i], w1 = w[i + 1], w2 = w[i + 2], w3 = w[i + 3];
    const V4<T> h0 = h[i], h1 = h[i + 1], h2 = h[i + 2], h3 = h[i + 3];
    y0 += w0 * h0;
    y1 += w1 * h1;
    y0 += w2 * h2;
    y1 += w3 * h3;
  }
  for (; i < n; ++i) y0 += w[i] * h[i];
  return y0 + y1;
}

__host__ __device__ inline int ns_out_width(const NsDesc& nd, int net, int l) {
  return l == nd.n_layers - 1 ? (net == 0 ? nd.widths[nd.n_layers] : 1) : nd.widths[l + 1];
}

// Both networks' layers into LDS: layer l of network n at Ws + wl[n][l] as n_out rows of n_in + 1
// (the weights, then the bias).
template <typename T>
__device__ void ns_stage_weights(const NsDesc& nd, const T* __restrict__ theta, T* Ws) {
  for (int n = 0; n < 2; ++n) {
    for (int l = 0; l < nd.n_layers; ++l) {
      const int n_in = nd.widths[l], n_out = ns_out_width(nd, n, l), pitch = n_in + 1;
      const T* src = theta + nd.toff[n] + nd.tl[n][l];
      T* dst = Ws + nd.wl[n][l];
      const int tot = n_out * pitch;
      for (int e = threadIdx.x; e < tot; e += blockDim.x) {
        const int o = e / pitch, i = e - o * pitch;
        dst[e] = i < n_in ? src[(int64_t)o * n_in + i] : src[(int64_t)n_out * n_in + o];
      }
    }
  }
}

// Per-wave scratch (V4 units): hid[l][64] for l < n_layers - 1 (the channels of hidden layer l's outputs,
// the inputs of layer l + 1), adj[64] (adjoint of a layer's outputs) and zb[64] (adjoint of its
// pre-activations). The input layer's channels are (x, 1, 0, 0) and (y, 0, 1, 0) and are formed in
// place; each hidden unit's pre-activation derivative channels stay in its lane's registers.
__host__ __device__ inline int ns_scratch_v4(int n_layers) { return 64 * (n_layers + 1); }

// Output channels of network n at (x0, x1): out[k] = (value, d/dx, d/dy, Laplacian) of output k, in
// every lane; pre[l] = the pre-activation channels of hidden layer l in lane = unit. Hidden layers:
// z = W h + b on the value channel, W h on the others, then a = tanh z, s1 = 1 - a^2, s2 = -2 a s1:
// (a, s1 Gz, s1 Lz + s2 |Gz|^2).
template <typename T, int NL>
__device__ void ns_forward(const NsDesc& nd, int n, const T* Ws, V4<T>* sc, T x0, T x1, V4<T> (&pre)[NL - 1],
                           V4<T> out[2]) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int l = 0; l < NL - 1; ++l) {
    const int n_in = nd.widths[l], n_out = nd.widths[l + 1];
    if (lane < n_out) {
      const T* wr = Ws + nd.wl[n][l] + lane * (n_in + 1);
      V4<T> z;
      if (l == 0) {  // inputs (x, y): n_in = 2, the bias at wr[2]
        const T w0 = wr[0], w1 = wr[1];
        z = V4<T>{wr[2] + w0 * x0 + w1 * x1, w0, w1, T(0)};
      } else {
        z = ns_dot(wr, sc + 64 * (l - 1), n_in, V4<T>{wr[n_in], T(0), T(0), T(0)});
      }
      pre[l] = z;
      const T a = tanh(z.x), s1 = T(1) - a * a, s2 = T(-2) * a * s1;
      sc[64 * l + lane] = V4<T>{a, s1 * z.y, s1 * z.z, s1 * z.w + s2 * (z.y * z.y + z.z * z.z)};
    }
    wave_sync();
  }
  const int l = NL - 1, n_in = nd.widths[l], n_out = ns_out_width(nd, n, l);
  V4<T> y = {T(0), T(0), T(0), T(0)};
  if (lane < n_out) {
    const T* wr = Ws + nd.wl[n][l] + lane * (n_in + 1);
    y = ns_dot(wr, sc + 64 * (l - 1), n_in, V4<T>{wr[n_in], T(0), T(0), T(0)});
  }
  for (int k = 0; k < 2; ++k)
    out[k] = V4<T>{__shfl(y.x, k), __shfl(y.y, k), __shfl(y.z, k), __shfl(y.w, k)};
}

// Reverse sweep of network n seeded with seed[k] = d r / d(value, d/dx, d/dy, Laplacian of output k),
// writing the parameter derivatives into Jn (the row's columns of network n). The forward sweep of the
// same network must have filled the scratch and pre. For z = W h + b with pre-activation adjoint zbar:
// dW[o][i] = sum_c zbar_c[o] h_c[i], db[o] = zbar_value[o]; hidden-layer zbar from the output adjoint
// abar by the tanh channel rules (s3 = -2 s1 (s1 - 2 a^2)):
//   zbar_L = s1 abar_L, zbar_G = s1 abar_G + 2 s2 abar_L Gz,
//   zbar_v = s1 abar_v + s2 Gz . abar_G + (s2 Lz + s3 |Gz|^2) abar_L.
template <typename T, int NL>
__device__ void ns_reverse(const NsDesc& nd, int n, const T* Ws, V4<T>* sc, const V4<T> (&pre)[NL - 1], T x0, T x1,
                           const V4<T> seed[2], T* __restrict__ Jn) {
  const int lane = threadIdx.x & 63;
  V4<T>* adj = sc + 64 * (NL - 1);
  V4<T>* zb = sc + 64 * NL;
  {
    const int n_out = ns_out_width(nd, n, NL - 1);
    if (lane < n_out) zb[lane] = lane == 0 ? seed[0] : seed[1];
    wave_sync();
  }
#pragma unroll
  for (int l = NL - 1; l >= 0; --l) {
    const int n_in = nd.widths[l], n_out = ns_out_width(nd, n, l), pitch = n_in + 1;
    const T* W = Ws + nd.wl[n][l];
    if (l < NL - 1) {
      if (lane < n_out) {
        const T a = sc[64 * l + lane].x;
        const T s1 = T(1) - a * a, s2 = T(-2) * a * s1, s3 = T(-2) * s1 * (s1 - T(2) * a * a);
        const V4<T> p = pre[l];
        const V4<T> ab = adj[lane];
        const T gsq = p.y * p.y + p.z * p.z;
        zb[lane] = V4<T>{s1 * ab.x + s2 * (p.y * ab.y + p.z * ab.z) + (s2 * p.w + s3 * gsq) * ab.w,
                         s1 * ab.y + T(2) * s2 * ab.w * p.y, s1 * ab.z + T(2) * s2 * ab.w * p.z, s1 * ab.w};
      }
      wave_sync();
    }
    // the layer's weight block (n_out x n_in, row-major) and then its bias
    T* dst = Jn + nd.tl[n][l];
    const int tot = n_out * n_in;
    if (l == 0) {  // inputs (x, 1, 0, 0) and (y, 0, 1, 0)
      for (int e = lane; e < tot; e += 64) {
        const V4<T> z = zb[e >> 1];
        dst[e] = (e & 1) ? z.x * x1 + z.z : z.x * x0 + z.y;
      }
    } else {
      const V4<T>* h = sc + 64 * (l - 1);
      const int q = 64 / n_in, rm = 64 - q * n_in;
      int o = lane / n_in, i = lane - o * n_in;
#pragma unroll 2
      for (int e = lane; e < tot; e += 64) {
        const V4<T> z = zb[o], hv = h[i];
        dst[e] = z.x * hv.x + z.y * hv.y + z.z * hv.z + z.w * hv.w;
        o += q;
        i += rm;
        if (i >= n_in) {
          i -= n_in;
          ++o;
        }
      }
    }
    if (lane < n_out) dst[tot + lane] = zb[lane].x;
    if (l > 0) {
      // adjoint of the layer's inputs: abar_c[i] = sum_o zbar_c[o] W[o][i]
      if (lane < n_in) {
        V4<T> a0 = {T(0), T(0), T(0), T(0)}, a1 = a0;
        int o2 = 0;
        for (; o2 + 4 <= n_out; o2 += 4) {
          const T w0 = W[o2 * pitch + lane], w1 = W[(o2 + 1) * pitch + lane];
          const T w2 = W[(o2 + 2) * pitch + lane], w3 = W[(o2 + 3) * pitch + lane];
          const V4<T> z0 = zb[o2], z1 = zb[o2 + 1], z2 = zb[o2 + 2], z3 = zb[o2 + 3];
          a0 += w0 * z0;
          a1 += w1 * z1;
          a0 += w2 * z2;
          a1 += w3 * z3;
        }
        for (; o2 < n_out; ++o2) a0 += W[o2 * pitch + lane] * zb[o2];
        adj[lane] = a0 + a1;
      }
      wave_sync();
    }
  }
  wave_sync();  // the caller's next forward sweep overwrites what the last layer's stores read
}

// One wave per row, blockDim.x / 64 (4 or 8) waves per workgroup sharing the staged weights.
template <typename T, int NL>
__global__ void __launch_bounds__(64 * kNsWavesMax) ns_residual_kernel(NsDesc nd, const T* __restrict__ theta,
                                                                        int64_t theta_stride, int64_t N,
                                                                        const T* __restrict__ X, const T* __restrict__ w,
                                                                        const T* __restrict__ f, const T* __restrict__ g,
                                                                        const int8_t* __restrict__ kind,
                                                                        T* __restrict__ r_w, T* __restrict__ J,
                                                                        int64_t ldJ, double* loss_partial,
                                                                        int rows_per_block) {
  extern __shared__ __align__(32) unsigned char ns_smem[];
  __shared__ double red[kNsWavesMax];
  theta += blockIdx.y * theta_stride;
  T* Ws = reinterpret_cast<T*>(ns_smem);
  const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = blockDim.x >> 6;
  V4<T>* sc = reinterpret_cast<V4<T>*>(ns_smem + (size_t)nd.w_elems * sizeof(T)) + wid * ns_scratch_v4(NL);
  ns_stage_weights(nd, theta, Ws);
  __syncthreads();
  const T nu = (T)nd.nu;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
  const int64_t r1 = r0 + rows_per_block < N ? r0 + rows_per_block : N;
  double lsum = 0.0;
  V4<T> pre[NL - 1];
  for (int64_t r = r0 + wid; r < r1; r += nw) {
    const int k = kind[r];
    const T sw = sqrt(w[r]);
    const T x0 = X[2 * r], x1 = X[2 * r + 1];
    V4<T> U[2];  // U[k] = (u_k, d_x u_k, d_y u_k, Laplace u_k)
    ns_forward<T, NL>(nd, 0, Ws, sc, x0, x1, pre, U);
    const bool mom = k == NGD_ROW_NS_MOMENTUM_X || k == NGD_ROW_NS_MOMENTUM_Y;
    const int c = k == NGD_ROW_NS_MOMENTUM_Y ? 1 : 0;
    T* Jr = J ? J + r * ldJ : nullptr;
    if (Jr) {
      const V4<T> zero = {T(0), T(0), T(0), T(0)};
      V4<T> s[2] = {zero, zero};
      if (mom) {
        // d/du_j = d_j u_c, d/d(d_j u_c) = u_j, d/d(Laplace u_c) = -nu
        s[0].x = U[c].y;
        s[1].x = U[c].z;
        s[c].y = U[0].x;
        s[c].z = U[1].x;
        s[c].w = -nu;
      } else if (k == NGD_ROW_NS_CONTINUITY) {
        s[0].y = T(1);
        s[1].z = T(1);
      } else if (k == NGD_ROW_NS_BOUNDARY_U) {
        s[0].x = T(1);
      } else if (k == NGD_ROW_NS_BOUNDARY_V) {
        s[1].x = T(1);
      }
      s[0] *= sw;
      s[1] *= sw;
      ns_reverse<T, NL>(nd, 0, Ws, sc, pre, x0, x1, s, Jr + nd.toff[0]);
    }
    T res = T(0);
    if (mom) {
      V4<T> Pc[2];
      ns_forward<T, NL>(nd, 1, Ws, sc, x0, x1, pre, Pc);
      const T dp = c == 0 ? Pc[0].y : Pc[0].z;
      res = -nu * U[c].w + (U[0].x * U[c].y + U[1].x * U[c].z) + dp - f[r];
      if (Jr) {
        const V4<T> zero = {T(0), T(0), T(0), T(0)};
        V4<T> s[2] = {zero, zero};
        if (c == 0) s[0].y = sw;
        else s[0].z = sw;
        ns_reverse<T, NL>(nd, 1, Ws, sc, pre, x0, x1, s, Jr + nd.toff[1]);
      }
    } else {
      if (k == NGD_ROW_NS_CONTINUITY) res = U[0].y + U[1].z;
      else if (k == NGD_ROW_NS_BOUNDARY_U) res = U[0].x - g[r];
      else if (k == NGD_ROW_NS_BOUNDARY_V) res = U[1].x - g[r];
      if (Jr)  // the pressure network does not enter these rows
        for (int64_t e = lane; e < nd.P - nd.toff[1]; e += 64) Jr[nd.toff[1] + e] = T(0);
    }
    if (Jr)
      for (int64_t e = nd.P + lane; e < ldJ; e += 64) Jr[e] = T(0);
    const T rw = sw * res;
    if (r_w && lane == 0) r_w[r] = rw;
    lsum += (double)rw * (double)rw;
    wave_sync();  // the next row's forward sweep overwrites the scratch this one read
  }
  if (lane == 0) red[wid] = lsum;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < nw; ++i) s += red[i];
    loss_partial[(size_t)blockIdx.y * gridDim.x + blockIdx.x] = s;
  }
}

// Velocity error sums at evaluation points (relative L2 / H1 errors on u of Section 5.1.3): one wave
// per point, per-wave partials, workgroup partials in a fixed order, [|u - u_ref|^2, |grad u -
// grad u_ref|^2, |u_ref|^2, |grad u_ref|^2].
template <typename T, int NL>
__global__ void __launch_bounds__(64 * kNsWavesMax) ns_velocity_error_kernel(NsDesc nd, const T* __restrict__ theta,
                                                                              const T* __restrict__ X, int64_t n,
                                                                              const T* __restrict__ u_ref,
                                                                              const T* __restrict__ grad_ref,
                                                                              double* part) {
  extern __shared__ __align__(32) unsigned char ns_smem[];
  __shared__ double red[4 * kNsWavesMax];
  T* Ws = reinterpret_cast<T*>(ns_smem);
  const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = blockDim.x >> 6;
  V4<T>* sc = reinterpret_cast<V4<T>*>(ns_smem + (size_t)nd.w_elems * sizeof(T)) + wid * ns_scratch_v4(NL);
  ns_stage_weights(nd, theta, Ws);
  __syncthreads();
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  V4<T> pre[NL - 1];
  for (int64_t p = (int64_t)blockIdx.x * nw + wid; p < n; p += (int64_t)gridDim.x * nw) {
    V4<T> U[2];
    ns_forward<T, NL>(nd, 0, Ws, sc, X[2 * p], X[2 * p + 1], pre, U);
    for (int k = 0; k < 2; ++k) {
      const double ur = u_ref[2 * p + k], gx = grad_ref[4 * p + 2 * k], gy = grad_ref[4 * p + 2 * k + 1];
      const double du = (double)U[k].x - ur, dx = (double)U[k].y - gx, dy = (double)U[k].z - gy;
      s[0] += du * du;
      s[1] += dx * dx + dy * dy;
      s[2] += ur * ur;
      s[3] += gx * gx + gy * gy;
    }
    wave_sync();
  }
  if (lane == 0)
    for (int j = 0; j < 4; ++j) red[4 * wid + j] = s[j];
  __syncthreads();
  if (threadIdx.x < 4) {
    double t = 0.0;
    for (int i = 0; i < nw; ++i) t += red[4 * i + threadIdx.x];
    part[4 * (size_t)blockIdx.x + threadIdx.x] = t;
  }
}

__global__ void ns_error_reduce_kernel(const double* part, int nblocks, double* sums) {
  if (threadIdx.x < 4) {
    double t = 0.0;
    for (int b = 0; b < nblocks; ++b) t += part[4 * b + threadIdx.x];
    sums[threadIdx.x] = t;
  }
}

}  // namespace

ngd_status ns_describe(int n_layers, const int* widths, double nu, NsDesc* nd) {
  NsDesc d{};
  d.n_layers = n_layers;
  for (int l = 0; l <= n_layers; ++l) d.widths[l] = widths[l];
  int64_t woff = 0;
  int lds = 0;
  for (int n = 0; n < 2; ++n) {
    d.toff[n] = woff;
    int64_t t = 0;
    for (int l = 0; l < n_layers; ++l) {
      const int n_in = widths[l], n_out = ns_out_width(d, n, l);
      d.tl[n][l] = t;
      t += (int64_t)n_out * n_in + n_out;
      d.wl[n][l] = lds;
      lds += n_out * (n_in + 1);
    }
    woff += t;
  }
  // the per-wave scratch starts on a 32-byte boundary
  d.w_elems = (lds + 3) / 4 * 4;
  d.P = woff;
  d.nu = nu;
  *nd = d;
  return NGD_OK;
}

// Waves per workgroup: eight where their scratch fits beside the weights, else four.
static int ns_waves(const NsDesc& nd, int dtype) {
  const size_t e = dtype == NGD_F64 ? 8 : 4;
  const size_t per_wave = (size_t)ns_scratch_v4(nd.n_layers) * 4 * e;
  return (size_t)nd.w_elems * e + kNsWavesMax * per_wave <= 160 * 1024 ? kNsWavesMax : 4;
}

size_t ns_lds_bytes(const NsDesc& nd, int dtype) {
  const size_t e = dtype == NGD_F64 ? 8 : 4;
  return (size_t)nd.w_elems * e + (size_t)ns_waves(nd, dtype) * ns_scratch_v4(nd.n_layers) * 4 * e;
}

int ns_rows_per_block(int64_t N) {
  // about a thousand workgroups, whole rounds of the widest workgroup's waves
  int64_t rpb = (N + 1023) / 1024;
  rpb = (rpb + kNsWavesMax - 1) / kNsWavesMax * kNsWavesMax;
  return (int)(rpb < kNsWavesMax ? kNsWavesMax : rpb);
}

int ns_blocks(int64_t N) {
  const int rpb = ns_rows_per_block(N);
  return (int)((N + rpb - 1) / rpb);
}

namespace {

// the kernel instance for the networks' depth (2 .. 8 affine layers)
template <typename T, int NL>
const void* ns_res_ptr() { return (const void*)ns_residual_kernel<T, NL>; }
template <typename T, int NL>
const void* ns_err_ptr() { return (const void*)ns_velocity_error_kernel<T, NL>; }

template <typename T>
const void* ns_residual_for(int nl) {
  switch (nl) {
    case 2: return ns_res_ptr<T, 2>();
    case 3: return ns_res_ptr<T, 3>();
    case 4: return ns_res_ptr<T, 4>();
    case 5: return ns_res_ptr<T, 5>();
    case 6: return ns_res_ptr<T, 6>();
    case 7: return ns_res_ptr<T, 7>();
    case 8: return ns_res_ptr<T, 8>();
    default: return nullptr;
  }
}

template <typename T>
const void* ns_error_for(int nl) {
  switch (nl) {
    case 2: return ns_err_ptr<T, 2>();
    case 3: return ns_err_ptr<T, 3>();
    case 4: return ns_err_ptr<T, 4>();
    case 5: return ns_err_ptr<T, 5>();
    case 6: return ns_err_ptr<T, 6>();
    case 7: return ns_err_ptr<T, 7>();
    case 8: return ns_err_ptr<T, 8>();
    default: return nullptr;
  }
}

}  // namespace

ngd_status launch_ns_residual(const NsDesc& nd, int dtype, const void* theta, int64_t theta_stride, int n_theta,
                              int64_t N, const void* X, const void* w, const void* f, const void* g,
                              const int8_t* kind, void* r_w, void* J, int64_t ldJ, double* loss_partial,
                              hipStream_t s) {
  const size_t bytes = ns_lds_bytes(nd, dtype);
  if (bytes > 160 * 1024) {
    set_error("Navier-Stokes networks too large for the residual kernel's LDS budget");
    return NGD_ERR_INVALID;
  }
  const void* k = dtype == NGD_F64 ? ns_residual_for<double>(nd.n_layers) : ns_residual_for<float>(nd.n_layers);
  if (k == nullptr) {
    set_error("Navier-Stokes networks need 2 to 8 affine layers");
    return NGD_ERR_INVALID;
  }
  if (N <= 0) return NGD_OK;
  const int rpb = ns_rows_per_block(N);
  dim3 grid((unsigned)((N + rpb - 1) / rpb), (unsigned)n_theta);
  NGD_HIP_TRY(hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
  NsDesc ndc = nd;
  int64_t ts = theta_stride, n = N, ld = ldJ;
  int rp = rpb;
  void* args[] = {&ndc, (void*)&theta, &ts, &n, (void*)&X, (void*)&w, (void*)&f, (void*)&g, (void*)&kind,
                  &r_w, &J, &ld, &loss_partial, &rp};
  NGD_HIP_TRY(hipLaunchKernel(k, grid, dim3(64 * ns_waves(nd, dtype)), args, bytes, s));
  return NGD_OK;
}

ngd_status launch_ns_velocity_error(const NsDesc& nd, int dtype, const void* theta, const void* X, int64_t n,
                                    const void* u_ref, const void* grad_ref, double* part, int max_blocks,
                                    double* sums, hipStream_t s) {
  const size_t bytes = ns_lds_bytes(nd, dtype);
  if (bytes > 160 * 1024) {
    set_error("Navier-Stokes networks too large for the evaluation kernel's LDS budget");
    return NGD_ERR_INVALID;
  }
  const void* k = dtype == NGD_F64 ? ns_error_for<double>(nd.n_layers) : ns_error_for<float>(nd.n_layers);
  if (k == nullptr) {
    set_error("Navier-Stokes networks need 2 to 8 affine layers");
    return NGD_ERR_INVALID;
  }
  const int nw = ns_waves(nd, dtype);
  int64_t nb = (n + 8 * nw - 1) / (8 * nw);
  nb = nb < 1 ? 1 : (nb > max_blocks ? max_blocks : nb);
  if (n > 0) {
    NGD_HIP_TRY(hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
    NsDesc ndc = nd;
    int64_t nn = n;
    void* args[] = {&ndc, (void*)&theta, (void*)&X, &nn, (void*)&u_ref, (void*)&grad_ref, &part};
    NGD_HIP_TRY(hipLaunchKernel(k, dim3((unsigned)nb), dim3(64 * nw), args, bytes, s));
  } else {
    nb = 0;
  }
  hipLaunchKernelGGL(ns_error_reduce_kernel, dim3(1), dim3(64), 0, s, part, (int)nb, sums);
  NGD_HIP_TRY(hipGetLastError());
  return NGD_OK;
}

}  // namespace ngd
