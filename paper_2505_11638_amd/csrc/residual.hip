// Residuals, parameter Jacobian, gradient and loss of the PINN least-squares problem.
//
// One workgroup owns a tile of TP collocation points. Per point it propagates C channels through
// the tanh MLP (value, gradient with respect to the Laplacian coordinates, Laplacian, time
// derivative: Taylor-mode forward Laplacian), forms the residual of the Poisson / heat energy and,
// for the Jacobian, runs the reverse sweep of those channels. The parameter derivative of a layer
// z = W h + b is the channel sum dW[o,i] = sum_c zbar_c[o] h_c[i], written row by row with
// coalesced stores (consecutive lanes -> consecutive parameters of one point's Jacobian row).
// Pre-activations of every hidden layer stay in LDS between the sweeps; post-activations are
// recomputed elementwise from them. (Jacobian of eq. G_matrixfree, Section 4.1.1; network of
// Section 2.3; residuals of eq. energy_poisson and eq. heat_energy.)
#include "common.h"

namespace ngd {
namespace {

template <typename T>
struct Lds {
  T* Ws;    // current layer weights, n_out x (n_in + 1)
  T* pre;   // pre-activation channels of every hidden layer: [layer][p][c][n]
  T* hb;    // input channels of the current layer: [p][c][nmax]
  T* ab;    // adjoint of the current layer outputs: [p][c][nmax]
  T* zb;    // adjoint of the current layer pre-activations: [p][c][nmax]
  T* ub;    // output-layer channel values / adjoint seeds: [p][kMaxChan]
  T* red;   // reduction scratch
};

// Row pitch of the per-channel buffers (h, abar, zbar): the widest layer plus one, so that the 16 rows
// an MFMA operand read touches at one k fall in distinct LDS banks.
__host__ __device__ inline int chan_pitch(const NetDesc& net) { return net.max_width + 1; }

__host__ __device__ inline int64_t pre_offset(const NetDesc& net, int layer, int TP) {
  // start of hidden layer `layer` (affine index, < n_layers-1) in the pre buffer
  int64_t off = 0;
  for (int l = 0; l < layer; ++l) off += (int64_t)TP * net.C * net.widths[l + 1];
  return off;
}

__host__ __device__ inline size_t lds_elems(const NetDesc& net, int TP) {
  size_t ws = 0;
  for (int l = 0; l < net.n_layers; ++l) {
    size_t s = (size_t)net.widths[l + 1] * (net.widths[l] + 1);
    ws = s > ws ? s : ws;
  }
  size_t pre = (size_t)pre_offset(net, net.n_layers - 1, TP);
  size_t buf = (size_t)TP * net.C * chan_pitch(net);
  return ws + pre + 3 * buf + (size_t)TP * kMaxChan + 32;
}

// Residuals only (no Jacobian): the forward sweep needs one layer's pre-activations at a time and no
// adjoint buffers, so more points fit per workgroup.
__host__ __device__ inline size_t lds_elems_fwd(const NetDesc& net, int TP) {
  size_t ws = 0;
  for (int l = 0; l < net.n_layers; ++l) {
    size_t s = (size_t)net.widths[l + 1] * (net.widths[l] + 1);
    ws = s > ws ? s : ws;
  }
  return ws + (size_t)TP * net.C * net.max_width + (size_t)TP * net.C * chan_pitch(net) + (size_t)TP * kMaxChan + 32;
}

// Stage W_l (n_out x n_in, row-major in theta) into LDS with a padded row pitch n_in + 1. Each thread
// issues its loads in batches of kLoadBatch before storing any, so a batch costs one L2 round trip.
constexpr int kLoadBatch = 16;
template <typename T>
__device__ void load_weights(const NetDesc& net, const T* theta, int l, T* Ws) {
  const int n_in = net.widths[l], n_out = net.widths[l + 1];
  const int total = n_out * n_in;
  const T* W = theta + net.woff[l];
  const int step = blockDim.x;
  for (int base = threadIdx.x; base < total; base += step * kLoadBatch) {
    T v[kLoadBatch];
#pragma unroll
    for (int u = 0; u < kLoadBatch; ++u) {
      const int e = base + u * step;
      v[u] = e < total ? W[e] : T(0);
    }
#pragma unroll
    for (int u = 0; u < kLoadBatch; ++u) {
      const int e = base + u * step;
      if (e < total) {
        const int o = e / n_in, i = e - o * n_in;
        Ws[o * (n_in + 1) + i] = v[u];
      }
    }
  }
}

// ---- 16 x 16 MFMA tiles for the per-point products ----
// One wave computes C = sum_k A(m, k) B(k, n) for a 16 x 16 tile with v_mfma_f32_16x16x4f32 (or the
// FP64 form): in each K-step of 4, lane l supplies A(l % 16, k0 + l / 16) and B(k0 + l / 16, l % 16).
// The operands come from LDS through the functors (which return 0 outside the problem's extents);
// `store(row, col, value)` receives the lane's four results. The accumulator layout is row
// 4 (l / 16) + r for the FP32 form and l / 16 + 4 r for the FP64 form, column l % 16.
typedef float mf4 __attribute__((ext_vector_type(4)));
typedef double md4 __attribute__((ext_vector_type(4)));

template <typename T, typename FA, typename FB, typename FS>
__device__ __forceinline__ void mfma_tile(int K, FA&& a, FB&& b, FS&& store) {
  const int lane = threadIdx.x & 63, r16 = lane & 15, kq = lane >> 4;
  if constexpr (sizeof(T) == 8) {
    md4 acc = {0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < K; k0 += 4)
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a(r16, k0 + kq), b(k0 + kq, r16), acc, 0, 0, 0);
#pragma unroll
    for (int r = 0; r < 4; ++r) store(kq + 4 * r, r16, acc[r]);
  } else {
    mf4 acc = {0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < K; k0 += 4)
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a(r16, k0 + kq), b(k0 + kq, r16), acc, 0, 0, 0);
#pragma unroll
    for (int r = 0; r < 4; ++r) store(4 * kq + r, r16, acc[r]);
  }
}

// Two products summed in one tile: C = A1 B1 + A2 B2 (the tangent of a layer product)
template <typename T, typename FA1, typename FB1, typename FA2, typename FB2, typename FS>
__device__ __forceinline__ void mfma_tile2(int K, FA1&& a1, FB1&& b1, FA2&& a2, FB2&& b2, FS&& store) {
  const int lane = threadIdx.x & 63, r16 = lane & 15, kq = lane >> 4;
  if constexpr (sizeof(T) == 8) {
    md4 acc = {0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < K; k0 += 4) {
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a1(r16, k0 + kq), b1(k0 + kq, r16), acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a2(r16, k0 + kq), b2(k0 + kq, r16), acc, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) store(kq + 4 * r, r16, acc[r]);
  } else {
    mf4 acc = {0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < K; k0 += 4) {
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a1(r16, k0 + kq), b1(k0 + kq, r16), acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a2(r16, k0 + kq), b2(k0 + kq, r16), acc, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) store(4 * kq + r, r16, acc[r]);
  }
}

// pre[pc][o] = sum_i W[o][i] h[pc][i] (+ b[o] on value channels) for pc < npc, o < n_out (row pitch ldo)
template <typename T>
__device__ __forceinline__ void mfma_forward(const T* Ws, int n_in, int n_out, const T* hb, int nm, int npc, int C,
                                             const T* __restrict__ b, T* pre, int ldo = 0) {
  if (ldo == 0) ldo = n_out;
  // the tile index is wave-uniform: scalar registers keep its divisions off the vector ALUs
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), nw = blockDim.x >> 6;
  const int tm = (npc + 15) / 16, tn = (n_out + 15) / 16;
  // the lane's accumulator rows are r0, r0 + rs, r0 + 2 rs, r0 + 3 rs of the tile (the MFMA layouts)
  const int kq = (threadIdx.x & 63) >> 4;
  const int r0 = sizeof(T) == 8 ? kq : 4 * kq, rs = sizeof(T) == 8 ? 4 : 1;
  for (int t = wid; t < tm * tn; t += nw) {
    const int m0 = (t / tn) * 16, n0 = (t % tn) * 16;
    // channel of the lane's first row (pc % C, the value channel takes the bias), then stepped by rs
    int ch = (m0 + r0) % C;
    mfma_tile<T>(
        n_in, [&](int r, int k) { const int pc = m0 + r; return (pc < npc && k < n_in) ? hb[pc * nm + k] : T(0); },
        [&](int k, int c) { const int o = n0 + c; return (o < n_out && k < n_in) ? Ws[o * (n_in + 1) + k] : T(0); },
        [&](int r, int c, T v) {
          const int pc = m0 + r, o = n0 + c;
          if (pc < npc && o < n_out) pre[pc * ldo + o] = v + (ch == 0 ? b[o] : T(0));
          ch += rs;
          while (ch >= C) ch -= C;
        });
  }
}

// the tangent of mfma_forward: zd[pc][o] = sum_i W[o][i] hd[pc][i] + Wd[o][i] h[pc][i] (+ bd[o])
template <typename T>
__device__ __forceinline__ void mfma_forward_tangent(const T* Ws, const T* Wd, int n_in, int n_out, const T* hb,
                                                     const T* hd, int nm, int npc, int C, const T* __restrict__ bd,
                                                     T* zd) {
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), nw = blockDim.x >> 6;
  const int tm = (npc + 15) / 16, tn = (n_out + 15) / 16;
  for (int t = wid; t < tm * tn; t += nw) {
    const int m0 = (t / tn) * 16, n0 = (t % tn) * 16;
    auto w_of = [&](const T* Wm) {
      return [=](int k, int c) { const int o = n0 + c; return (o < n_out && k < n_in) ? Wm[o * (n_in + 1) + k] : T(0); };
    };
    auto h_of = [&](const T* Hm) {
      return [=](int r, int k) { const int pc = m0 + r; return (pc < npc && k < n_in) ? Hm[pc * nm + k] : T(0); };
    };
    mfma_tile2<T>(n_in, h_of(hd), w_of(Ws), h_of(hb), w_of(Wd), [&](int r, int c, T v) {
      const int pc = m0 + r, o = n0 + c;
      if (pc < npc && o < n_out) zd[pc * nm + o] = v + (pc % C == 0 ? bd[o] : T(0));
    });
  }
}

// ab[pc][i] = sum_o W[o][i] zb[pc][o] for pc < npc, i < n_in (the adjoint product W^T z)
template <typename T>
__device__ __forceinline__ void mfma_adjoint(const T* Ws, int n_in, int n_out, const T* zb, int nm, int npc, T* ab) {
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), nw = blockDim.x >> 6;
  const int tm = (npc + 15) / 16, tn = (n_in + 15) / 16;
  for (int t = wid; t < tm * tn; t += nw) {
    const int m0 = (t / tn) * 16, n0 = (t % tn) * 16;
    mfma_tile<T>(
        n_out, [&](int r, int k) { const int pc = m0 + r; return (pc < npc && k < n_out) ? zb[pc * nm + k] : T(0); },
        [&](int k, int c) { const int i = n0 + c; return (i < n_in && k < n_out) ? Ws[k * (n_in + 1) + i] : T(0); },
        [&](int r, int c, T v) {
          const int pc = m0 + r, i = n0 + c;
          if (pc < npc && i < n_in) ab[pc * nm + i] = v;
        });
  }
}

// input channels of layer 0 for the tile
template <typename T>
__device__ void input_channels(const NetDesc& net, const T* X, int64_t row0, int64_t N, int TP, T* hb) {
  const int d = net.d, C = net.C, nm = chan_pitch(net);
  for (int e = threadIdx.x; e < TP * C * d; e += blockDim.x) {
    int i = e % d, pc = e / d, c = pc % C, p = pc / C;
    int64_t row = row0 + p;
    T v = 0;
    if (c == 0) {
      v = row < N ? X[row * d + i] : T(0);
    } else if (c <= net.nS) {
      v = (i == c - 1) ? T(1) : T(0);
    } else if (c == net.nS + 1) {
      v = 0;
    } else {
      v = (i == d - 1) ? T(1) : T(0);
    }
    hb[pc * nm + i] = v;
  }
}

// post-activation channels of hidden layer `l` (affine index) from its pre-activations
template <typename T>
__device__ void activate(const NetDesc& net, const T* pre_l, int n, int TP, T* hb) {
  const int C = net.C, nS = net.nS, nm = chan_pitch(net);
  for (int e = threadIdx.x; e < TP * n; e += blockDim.x) {
    int p = e / n, i = e - p * n;
    const T* z = pre_l + (int64_t)p * C * n;
    T a = tanh(z[i]);
    T s1 = T(1) - a * a;
    T s2 = T(-2) * a * s1;
    T gsq = 0;
    T* h = hb + (int64_t)p * C * nm;
    h[i] = a;
    for (int k = 1; k <= nS; ++k) {
      T gz = z[k * n + i];
      gsq += gz * gz;
      h[k * nm + i] = s1 * gz;
    }
    h[(nS + 1) * nm + i] = s1 * z[(nS + 1) * n + i] + s2 * gsq;
    if (net.has_t) h[(nS + 2) * nm + i] = s1 * z[(nS + 2) * n + i];
  }
}

// MODE kJacobian: one tile of TP points per workgroup; writes r_w, the loss partial and (J != NULL)
// the Jacobian rows. MODE kVjp: the workgroup loops over tiles blockIdx.x, blockIdx.x + gridDim.x,
// ... and accumulates sum_r wv[r] dr_w[r]/dtheta into its own row of `J` (then a partial-sum buffer
// with leading dimension ldJ), plus sum_r wv[r]^2 into tsq_out[blockIdx.x]: the adjoint product
// J_w^T wv without storing J_w (the reverse sweep with its seeds scaled by wv).
enum { kJacobian = 0, kVjp = 1 };

// The workgroup's share of the work: tiles tile_first, tile_first + tile_step, ... of one problem.
// write_r: store r_w; loss_slot: this workgroup's loss partial (kJacobian); part_row: its partial
// row (kVjp); tsq_slot: its sum of wv^2 (kVjp).
template <typename T, int MODE>
__device__ void residual_body(const NetDesc& net, const T* __restrict__ theta, int64_t N, const T* __restrict__ X,
                              const T* __restrict__ w, const T* __restrict__ f, const T* __restrict__ g,
                              const int8_t* __restrict__ kind, T* __restrict__ r_w, T* __restrict__ J, int64_t ldJ,
                              int TP, int64_t tile_first, int64_t tile_step, const double* __restrict__ wv,
                              int64_t wv_stride, bool write_r, double* loss_slot, T* part_row, double* tsq_slot,
                              bool acc_in_lds = false, bool fwd_only = false) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* smem = reinterpret_cast<T*>(smem_raw);
  const int C = net.C, nS = net.nS, nm = chan_pitch(net), L = net.n_layers;
  const int64_t ntiles = (N + TP - 1) / TP;
  double tsq_acc = 0.0;
  bool first = true;
  for (int64_t tile = tile_first; tile < ntiles; tile += tile_step, first = false) {
  const int64_t row0 = tile * TP;

  Lds<T> s;
  {
    size_t ws = 0;
    for (int l = 0; l < L; ++l) {
      size_t q = (size_t)net.widths[l + 1] * (net.widths[l] + 1);
      ws = q > ws ? q : ws;
    }
    s.Ws = smem;
    s.pre = s.Ws + ws;
    if (fwd_only) {  // residuals only: one layer of pre-activations, no adjoint buffers
      s.hb = s.pre + (size_t)TP * C * net.max_width;
      s.ab = s.zb = nullptr;
      s.ub = s.hb + (size_t)TP * C * nm;
    } else {
      s.hb = s.pre + pre_offset(net, L - 1, TP);
      s.ab = s.hb + (size_t)TP * C * nm;
      s.zb = s.ab + (size_t)TP * C * nm;
      s.ub = s.zb + (size_t)TP * C * nm;
    }
    s.red = s.ub + TP * kMaxChan;
  }

  // ---------------- forward sweep ----------------
  input_channels(net, X, row0, N, TP, s.hb);
  for (int l = 0; l < L - 1; ++l) {
    const int n_in = net.widths[l], n_out = net.widths[l + 1];
    __syncthreads();
    load_weights(net, theta, l, s.Ws);
    __syncthreads();
    T* pre_l = s.pre + (fwd_only ? 0 : pre_offset(net, l, TP));
    const T* b = theta + net.boff[l];
    mfma_forward(s.Ws, n_in, n_out, s.hb, nm, TP * C, C, b, pre_l);
    __syncthreads();
    activate(net, pre_l, n_out, TP, s.hb);
  }
  // output layer: channel values of u
  const int n_last = net.widths[L - 1];
  const T* Wout = theta + net.woff[L - 1];
  const T bout = theta[net.boff[L - 1]];
  __syncthreads();
  for (int pc = threadIdx.x; pc < TP * C; pc += blockDim.x) {
    const T* h = s.hb + pc * nm;
    T acc = 0;
    for (int i = 0; i < n_last; ++i) acc += Wout[i] * h[i];
    int p = pc / C, c = pc % C;
    s.ub[p * kMaxChan + c] = acc + (c == 0 ? bout : T(0));
  }
  __syncthreads();
  // residuals, loss and adjoint seeds (overwrite ub with the seeds after reading the values)
  T lsum = 0;
  if (threadIdx.x < TP) {
    const int p = threadIdx.x;
    const int64_t row = row0 + p;
    T seed[kMaxChan];
    for (int c = 0; c < kMaxChan; ++c) seed[c] = 0;
    if (row < N) {
      const T u = s.ub[p * kMaxChan], lap = s.ub[p * kMaxChan + nS + 1];
      const T ut = net.has_t ? s.ub[p * kMaxChan + nS + 2] : T(0);
      const T sw = sqrt(w[row]);
      T res;
      if (kind[row] == NGD_ROW_INTERIOR) {
        if (net.pde == NGD_PDE_POISSON) {
          res = lap + f[row];
          seed[nS + 1] = sw;
        } else {
          res = ut - lap - f[row];
          seed[nS + 1] = -sw;
          seed[nS + 2] = sw;
        }
      } else {
        res = u - g[row];
        seed[0] = sw;
      }
      const T rw = sw * res;
      if constexpr (MODE == kJacobian) {
        if (r_w != nullptr && write_r) r_w[row] = rw;
        lsum = rw * rw;
      } else {
        const double wvr = wv[row * wv_stride];
        tsq_acc += wvr * wvr;
        for (int c = 0; c < kMaxChan; ++c) seed[c] *= (T)wvr;
      }
    }
    for (int c = 0; c < kMaxChan; ++c) s.ub[p * kMaxChan + c] = seed[c];
  }
  if constexpr (MODE == kJacobian) {
    __shared__ double red_d[16];
    double tot = block_sum<double>((double)lsum, red_d);
    if (threadIdx.x == 0 && loss_slot != nullptr) *loss_slot = tot;
    if (J == nullptr) return;
  }
  __syncthreads();
  // accumulate into this workgroup's partial row (kVjp), in LDS past the tile buffers when it fits
  // there (written out once after the last tile); a thread always owns the same entries
  T* acc_lds = (MODE == kVjp && acc_in_lds) ? smem + lds_elems(net, TP) : nullptr;
  auto put = [&](int64_t idx, T v) {
    T* q = acc_lds != nullptr ? acc_lds + idx : part_row + idx;
    *q = first ? v : *q + v;
  };
  (void)put;

  // ---------------- reverse sweep and Jacobian rows ----------------
  const int64_t P = net.P;
  const int nvalid = (int)((N - row0) < TP ? (N - row0) : TP);
  // output layer: dr/dW_out[i] = sum_c seed_c h_c[i], dr/db_out = seed_value; zero padding
  if constexpr (MODE == kJacobian) {
    for (int p = 0; p < nvalid; ++p) {
      T* Jrow = J + (row0 + p) * ldJ;
      const T* sd = s.ub + p * kMaxChan;
      for (int i = threadIdx.x; i < n_last; i += blockDim.x) {
        T acc = 0;
        for (int c = 0; c < C; ++c) acc += sd[c] * s.hb[(p * C + c) * nm + i];
        Jrow[net.woff[L - 1] + i] = acc;
      }
      if (threadIdx.x == 0) Jrow[net.boff[L - 1]] = sd[0];
      for (int64_t j = P + threadIdx.x; j < ldJ; j += blockDim.x) Jrow[j] = 0;
    }
  } else {
    for (int i = threadIdx.x; i < n_last; i += blockDim.x) {
      T acc = 0;
      for (int p = 0; p < nvalid; ++p)
        for (int c = 0; c < C; ++c) acc += s.ub[p * kMaxChan + c] * s.hb[(p * C + c) * nm + i];
      put(net.woff[L - 1] + i, acc);
    }
    if (threadIdx.x == 0) {
      T acc = 0;
      for (int p = 0; p < nvalid; ++p) acc += s.ub[p * kMaxChan];
      put(net.boff[L - 1], acc);
    }
    if (first && acc_lds == nullptr)
      for (int64_t j = P + threadIdx.x; j < ldJ; j += blockDim.x) part_row[j] = 0;
  }
  // adjoint of the last hidden layer outputs: ab = W_out^T seed
  for (int e = threadIdx.x; e < TP * C * n_last; e += blockDim.x) {
    int i = e % n_last, pc = e / n_last, p = pc / C, c = pc % C;
    s.ab[pc * nm + i] = Wout[i] * s.ub[p * kMaxChan + c];
  }
  for (int l = L - 2; l >= 0; --l) {
    const int n_in = net.widths[l], n_out = net.widths[l + 1];
    const T* pre_l = s.pre + pre_offset(net, l, TP);
    __syncthreads();
    // zbar from abar through tanh (channel rules of the forward Laplacian)
    for (int e = threadIdx.x; e < TP * n_out; e += blockDim.x) {
      int p = e / n_out, o = e - p * n_out;
      const T* z = pre_l + (int64_t)p * C * n_out;
      const T* a_ = s.ab + (int64_t)p * C * nm;
      T* zb = s.zb + (int64_t)p * C * nm;
      T a = tanh(z[o]);
      T s1 = T(1) - a * a;
      T s2 = T(-2) * a * s1;
      T s3 = T(-2) * s1 * (s1 - T(2) * a * a);
      T aL = a_[(nS + 1) * nm + o];
      T gsq = 0, gdot = 0;
      for (int k = 1; k <= nS; ++k) {
        T gz = z[k * n_out + o];
        T ag = a_[k * nm + o];
        gsq += gz * gz;
        gdot += gz * ag;
        zb[k * nm + o] = s1 * ag + T(2) * s2 * aL * gz;
      }
      T Lz = z[(nS + 1) * n_out + o];
      zb[(nS + 1) * nm + o] = s1 * aL;
      T zv = s1 * a_[o] + s2 * gdot + (s2 * Lz + s3 * gsq) * aL;
      if (net.has_t) {
        T aT = a_[(nS + 2) * nm + o];
        zb[(nS + 2) * nm + o] = s1 * aT;
        zv += s2 * z[(nS + 2) * n_out + o] * aT;
      }
      zb[o] = zv;
    }
    // input channels of this layer
    if (l == 0)
      input_channels(net, X, row0, N, TP, s.hb);
    else
      activate(net, s.pre + pre_offset(net, l - 1, TP), n_in, TP, s.hb);
    __syncthreads();
    // Jacobian segments of W_l and b_l
    const int64_t wo = net.woff[l], bo = net.boff[l];
    const int nel = n_out * n_in;
    const int wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int tmo = (n_out + 15) / 16, tni = (n_in + 15) / 16;
    if constexpr (MODE == kVjp) {
      // dW[o][i] = sum over the tile's points and channels of zbar[pc][o] h[pc][i]: one contraction
      // with K = nvalid C (seeds of rows past N are zero)
      const int kk = nvalid * C;
      for (int t = wid; t < tmo * tni; t += nw) {
        const int o0 = (t / tni) * 16, i0 = (t % tni) * 16;
        mfma_tile<T>(
            kk, [&](int r, int k) { const int o = o0 + r; return (o < n_out && k < kk) ? s.zb[k * nm + o] : T(0); },
            [&](int k, int c) { const int i = i0 + c; return (i < n_in && k < kk) ? s.hb[k * nm + i] : T(0); },
            [&](int r, int c, T v) {
              const int o = o0 + r, i = i0 + c;
              if (o < n_out && i < n_in) put(wo + o * n_in + i, v);
            });
      }
      (void)nel;
      for (int o = threadIdx.x; o < n_out; o += blockDim.x) {
        T acc = 0;
        for (int p = 0; p < nvalid; ++p) acc += s.zb[(int64_t)p * C * nm + o];
        put(bo + o, acc);
      }
    } else {
      // per point p: the W_l block of J_p is zbar_p (n_out x C) times h_p^T (C x n_in), K = C. The tile
      // index is the same in every lane of a wave: kept in scalar registers, so that its divisions do
      // not occupy the vector ALUs
      const int tpp = tmo * tni, wid_s = __builtin_amdgcn_readfirstlane(wid);
      for (int t = wid_s; t < nvalid * tpp; t += nw) {
        const int p = t / tpp, tt = t - p * tpp;
        const int o0 = (tt / tni) * 16, i0 = (tt % tni) * 16;
        const T* zbp = s.zb + (int64_t)p * C * nm;
        const T* hbp = s.hb + (int64_t)p * C * nm;
        T* Jrow = J + (row0 + p) * ldJ + wo;
        mfma_tile<T>(
            C, [&](int r, int k) { const int o = o0 + r; return (o < n_out && k < C) ? zbp[k * nm + o] : T(0); },
            [&](int k, int c) { const int i = i0 + c; return (i < n_in && k < C) ? hbp[k * nm + i] : T(0); },
            [&](int r, int c, T v) {
              const int o = o0 + r, i = i0 + c;
              if (o < n_out && i < n_in) Jrow[o * n_in + i] = v;
            });
      }
      (void)nel;
    }
    if constexpr (MODE == kJacobian) {
      for (int p = 0; p < nvalid; ++p) {
        T* Jrow = J + (row0 + p) * ldJ + bo;
        for (int o = threadIdx.x; o < n_out; o += blockDim.x) Jrow[o] = s.zb[(int64_t)p * C * nm + o];
      }
    }
    if (l == 0) break;
    // abar of the layer inputs: ab = W_l^T zbar
    __syncthreads();
    load_weights(net, theta, l, s.Ws);
    __syncthreads();
    mfma_adjoint(s.Ws, n_in, n_out, s.zb, nm, TP * C, s.ab);
  }
  __syncthreads();
  }  // tile loop
  if constexpr (MODE == kVjp) {
    __shared__ double red_t[16];
    const double t = block_sum(tsq_acc, red_t);
    if (threadIdx.x == 0 && tsq_slot != nullptr) *tsq_slot = t;
    if (acc_in_lds) {
      const T* acc = smem + lds_elems(net, TP);
      for (int64_t j = threadIdx.x; j < ldJ; j += blockDim.x) part_row[j] = j < net.P ? acc[j] : T(0);
    }
  }
}

template <typename T, int MODE, int NT = 256>
__global__ __launch_bounds__(NT) void residual_jacobian_kernel(
    NetDesc net, const T* __restrict__ theta0, int64_t theta_stride, int64_t N, const T* __restrict__ X,
    const T* __restrict__ w, const T* __restrict__ f, const T* __restrict__ g, const int8_t* __restrict__ kind,
    T* __restrict__ r_w, T* __restrict__ J, int64_t ldJ, double* __restrict__ loss_partial, int TP,
    const double* __restrict__ wv, int64_t wv_stride, double* __restrict__ tsq_out, int acc_in_lds,
    int fwd_only) {
  const T* theta = theta0 + (int64_t)blockIdx.y * theta_stride;
  const int64_t ntiles = (N + TP - 1) / TP;
  const int64_t tile_step = MODE == kVjp ? (int64_t)gridDim.x : ntiles;
  double* loss_slot =
      loss_partial != nullptr ? loss_partial + (int64_t)blockIdx.y * gridDim.x + blockIdx.x : nullptr;
  T* part_row = MODE == kVjp ? J + (int64_t)blockIdx.x * ldJ : nullptr;
  double* tsq_slot = tsq_out != nullptr ? tsq_out + blockIdx.x : nullptr;
  residual_body<T, MODE>(net, theta, N, X, w, f, g, kind, r_w, J, ldJ, TP, blockIdx.x, tile_step, wv, wv_stride,
                         blockIdx.y == 0, loss_slot, part_row, tsq_slot, acc_in_lds != 0,
                         MODE == kJacobian && fwd_only != 0 && J == nullptr);
}

// Several problems in one launch: work item i is tile (i - first_tile[q]) of the problem q whose
// tile range holds i; workgroups stride over the items (a persistent grid). loss_part has one slot
// per tile of the problem.
template <typename T, int NT = 256>
__global__ __launch_bounds__(NT) void batch_residual_jacobian_kernel(const BatchResidualItem* __restrict__ items,
                                                                      int n_prob, int64_t total_tiles) {
  for (int64_t it = blockIdx.x; it < total_tiles; it += gridDim.x) {
    int lo = 0, hi = n_prob - 1;  // last problem whose first tile is <= it
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (items[mid].first_tile <= it) lo = mid; else hi = mid - 1;
    }
    const BatchResidualItem& b = items[lo];
    const int64_t tile = it - b.first_tile;
    const int64_t ntiles = (b.N + b.TP - 1) / b.TP;
    residual_body<T, kJacobian>(b.net, (const T*)b.theta, b.N, (const T*)b.X, (const T*)b.w, (const T*)b.f,
                                (const T*)b.g, b.kind, (T*)b.r_w, (T*)b.J, b.ldJ, b.TP, tile, ntiles, nullptr, 0, true,
                                b.loss_part + tile, nullptr, nullptr);
    __syncthreads();
  }
}

// Forward-mode product with the parameter Jacobian: out[r * ldo + j * cs] = (J_w u_j)[r] for the
// direction u_j = U + j * ldU (j = blockIdx.y). Every channel of the forward Laplacian sweep carries a
// tangent: for z = W h + b, zdot = W hdot + Wdot h (+ bdot on the value channel), and the tanh
// channel rules are differentiated once more (s1' = -2 a a', s2' = -2 (a' s1 + a s1')). The
// residual's tangent is read from the output channels as the residual itself is (eq. energy_poisson,
// eq. heat_energy) and scaled by sqrt(w).
template <typename T, typename TO>
__global__ __launch_bounds__(256) void jvp_kernel(NetDesc net, const T* __restrict__ theta, const T* __restrict__ U,
                                                  int64_t ldU, int64_t N, const T* __restrict__ X,
                                                  const T* __restrict__ w, const int8_t* __restrict__ kind,
                                                  TO* __restrict__ out, int64_t ldo, int64_t cs, int TP) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* smem = reinterpret_cast<T*>(smem_raw);
  const int C = net.C, nS = net.nS, nm = chan_pitch(net), L = net.n_layers;
  const int64_t row0 = (int64_t)blockIdx.x * TP;
  const T* dth = U + (int64_t)blockIdx.y * ldU;
  size_t ws = 0;
  for (int l = 0; l < L; ++l) {
    size_t q = (size_t)net.widths[l + 1] * (net.widths[l] + 1);
    ws = q > ws ? q : ws;
  }
  const size_t buf = (size_t)TP * C * nm;
  T* Ws = smem;
  T* Wd = Ws + ws;
  T* hb = Wd + ws;     // [p][c][nm] channels entering the layer
  T* hd = hb + buf;    // their tangents
  T* zb = hd + buf;    // pre-activation channels
  T* zd = zb + buf;    // their tangents
  T* ud = zd + buf;    // output-channel tangents [p][kMaxChan]

  input_channels(net, X, row0, N, TP, hb);
  for (size_t e = threadIdx.x; e < buf; e += blockDim.x) hd[e] = 0;
  for (int l = 0; l < L - 1; ++l) {
    const int n_in = net.widths[l], n_out = net.widths[l + 1];
    __syncthreads();
    load_weights(net, theta, l, Ws);
    load_weights(net, dth, l, Wd);
    __syncthreads();
    const T* b = theta + net.boff[l];
    const T* bd = dth + net.boff[l];
    mfma_forward(Ws, n_in, n_out, hb, nm, TP * C, C, b, zb, nm);
    mfma_forward_tangent(Ws, Wd, n_in, n_out, hb, hd, nm, TP * C, C, bd, zd);
    __syncthreads();
    for (int e = threadIdx.x; e < TP * n_out; e += blockDim.x) {
      const int p = e / n_out, o = e - p * n_out;
      const T* z = zb + (int64_t)p * C * nm;
      const T* zt = zd + (int64_t)p * C * nm;
      T* h = hb + (int64_t)p * C * nm;
      T* ht = hd + (int64_t)p * C * nm;
      const T a = tanh(z[o]);
      const T s1 = T(1) - a * a, s2 = T(-2) * a * s1;
      const T ad = s1 * zt[o];
      const T s1d = T(-2) * a * ad;
      const T s2d = T(-2) * (ad * s1 + a * s1d);
      h[o] = a;
      ht[o] = ad;
      T gsq = 0, gsqd = 0;
      for (int k = 1; k <= nS; ++k) {
        const T gz = z[k * nm + o], gzd = zt[k * nm + o];
        gsq += gz * gz;
        gsqd += T(2) * gz * gzd;
        h[k * nm + o] = s1 * gz;
        ht[k * nm + o] = s1d * gz + s1 * gzd;
      }
      const T lz = z[(nS + 1) * nm + o], lzd = zt[(nS + 1) * nm + o];
      h[(nS + 1) * nm + o] = s1 * lz + s2 * gsq;
      ht[(nS + 1) * nm + o] = s1d * lz + s1 * lzd + s2d * gsq + s2 * gsqd;
      if (net.has_t) {
        const T tz = z[(nS + 2) * nm + o], tzd = zt[(nS + 2) * nm + o];
        h[(nS + 2) * nm + o] = s1 * tz;
        ht[(nS + 2) * nm + o] = s1d * tz + s1 * tzd;
      }
    }
  }
  // output layer (linear): udot_c = w_out . hdot_c + wdot_out . h_c (+ bdot on the value channel)
  const int n_last = net.widths[L - 1];
  const T* Wout = theta + net.woff[L - 1];
  const T* Wdout = dth + net.woff[L - 1];
  const T bdout = dth[net.boff[L - 1]];
  __syncthreads();
  for (int pc = threadIdx.x; pc < TP * C; pc += blockDim.x) {
    const T* h = hb + pc * nm;
    const T* ht = hd + pc * nm;
    T dacc = 0;
    for (int i = 0; i < n_last; ++i) dacc += Wout[i] * ht[i] + Wdout[i] * h[i];
    const int p = pc / C, c = pc % C;
    ud[p * kMaxChan + c] = dacc + (c == 0 ? bdout : T(0));
  }
  __syncthreads();
  if (threadIdx.x < TP) {
    const int p = threadIdx.x;
    const int64_t row = row0 + p;
    if (row < N) {
      const T* u = ud + p * kMaxChan;
      T rd;
      if (kind[row] == NGD_ROW_INTERIOR)
        rd = net.pde == NGD_PDE_POISSON ? u[nS + 1] : u[nS + 2] - u[nS + 1];
      else
        rd = u[0];
      out[row * ldo + (int64_t)blockIdx.y * cs] = (TO)(sqrt(w[row]) * rd);
    }
  }
}

__host__ inline size_t jvp_lds_elems(const NetDesc& net, int TP) {
  size_t ws = 0;
  for (int l = 0; l < net.n_layers; ++l) {
    size_t s = (size_t)net.widths[l + 1] * (net.widths[l] + 1);
    ws = s > ws ? s : ws;
  }
  return 2 * ws + 4 * (size_t)TP * net.C * chan_pitch(net) + (size_t)TP * kMaxChan;
}

// sum of n_per partials for each of n_sets sets, scaled: out[s] = scale * sum_i partial[s*n_per + i]
__global__ void reduce_sum_kernel(const double* __restrict__ partial, int64_t n_per, double scale,
                                  double* __restrict__ out) {
  __shared__ double red[16];
  const double* p = partial + (int64_t)blockIdx.x * n_per;
  double acc = 0;
  for (int64_t i = threadIdx.x; i < n_per; i += blockDim.x) acc += p[i];
  acc = block_sum(acc, red);
  if (threadIdx.x == 0) out[blockIdx.x] = scale * acc;
}

// gradient: grad[j] = sum_r r[r] J[r, j]; stage 1 per row chunk, stage 2 over chunks (FP64)
template <typename T>
__global__ __launch_bounds__(256) void colsum_stage1(const T* __restrict__ J, int64_t ldJ, int64_t N, int64_t P,
                                                     const T* __restrict__ r, int64_t rows_per,
                                                     double* __restrict__ work) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t r0 = (int64_t)blockIdx.y * rows_per;
  const int64_t r1 = (r0 + rows_per) < N ? (r0 + rows_per) : N;
  if (j >= P) return;
  double acc = 0;
  for (int64_t i = r0; i < r1; ++i) acc += (double)r[i] * (double)J[i * ldJ + j];
  work[(int64_t)blockIdx.y * P + j] = acc;
}

__global__ void colsum_stage2(const double* __restrict__ work, int nchunk, int64_t P, double* __restrict__ out) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= P) return;
  double acc = 0;
  for (int c = 0; c < nchunk; ++c) acc += work[(int64_t)c * P + j];
  out[j] = acc;
}

}  // namespace

static int choose_tp(const NetDesc& net, size_t elem, size_t* bytes, bool fwd_only = false);

int residual_block_rows(const NetDesc& net, int dtype) {
  size_t b = 0;
  return choose_tp(net, dtype == NGD_F64 ? 8 : 4, &b);
}

int residual_trials_per_launch(const NetDesc& net, int dtype, int64_t N, int max_trials) {
  size_t bytes = 0;
  const int tp = choose_tp(net, dtype == NGD_F64 ? 8 : 4, &bytes, true);
  const int64_t per_trial = (N + tp - 1) / tp;
  int dev = 0, cus = 0, per_cu = 0;
  const void* k = dtype == NGD_F64 ? (const void*)residual_jacobian_kernel<double, kJacobian>
                                   : (const void*)residual_jacobian_kernel<float, kJacobian>;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, 256, bytes) != hipSuccess || per_cu < 1)
    return 1;
  // trials that run in about four rounds of resident workgroups cost little more than one
  const int64_t fit = 4 * (int64_t)cus * per_cu / (per_trial > 0 ? per_trial : 1);
  return (int)(fit < 1 ? 1 : (fit > max_trials ? max_trials : fit));
}

int residual_blocks(const NetDesc& net, int dtype, int64_t N, bool with_jacobian) {
  size_t b = 0;
  const int tp = choose_tp(net, dtype == NGD_F64 ? 8 : 4, &b, !with_jacobian);
  return (int)((N + tp - 1) / tp);
}

static int choose_tp(const NetDesc& net, size_t elem, size_t* bytes, bool fwd_only) {
  auto need = [&](int t) { return (fwd_only ? lds_elems_fwd(net, t) : lds_elems(net, t)) * elem; };
  // small tiles (more workgroups, several per CU) measured fastest; the residual-only layout starts
  // from the same size, so that both sweeps group the loss partials alike (bitwise the same loss)
  int tp = 4;
  while (tp > 1 && need(tp) > 96 * 1024) tp >>= 1;
  // wide layers: trade occupancy for more points per staged weight matrix
  while (tp < 4 && need(2 * tp) <= 150 * 1024) tp <<= 1;
  *bytes = need(tp);
  return tp;
}

// Threads per workgroup of the Jacobian sweep: the tile's LDS decides how many workgroups share a CU;
// where that is one or two, wider workgroups (1,024 or 512 threads) keep more waves in flight for the
// row stores and the per-point products (every loop of the sweep strides over the workgroup).
static int jacobian_threads(size_t lds_bytes) {
  const size_t per_cu = lds_bytes > 0 ? (160 * 1024) / lds_bytes : 8;
  return per_cu <= 1 ? 1024 : (per_cu <= 3 ? 512 : 256);
}

ngd_status launch_residual_jacobian(const NetDesc& net, int dtype, const void* theta, int64_t N, const void* X,
                                    const void* w, const void* f, const void* g, const int8_t* kind, void* r_w,
                                    void* J, int64_t ldJ, double* loss_partial, int64_t theta_stride, int n_theta,
                                    hipStream_t s, int* n_blocks_out) {
  size_t elem = dtype == NGD_F64 ? 8 : 4;
  size_t bytes = 0;
  const int fwd_only = J == nullptr ? 1 : 0;
  int tp = choose_tp(net, elem, &bytes, fwd_only != 0);
  if (bytes > 160 * 1024) {
    set_error("network too wide for the residual kernel's LDS budget");
    return NGD_ERR_INVALID;
  }
  dim3 grid((unsigned)((N + tp - 1) / tp), (unsigned)n_theta);
  if (n_blocks_out) *n_blocks_out = (int)grid.x;
  const int nt = fwd_only ? 256 : jacobian_threads(bytes);
  auto go = [&](auto k, auto tag) -> ngd_status {
    using T = decltype(tag);
    NGD_HIP_TRY(hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
    hipLaunchKernelGGL(k, grid, dim3(nt), bytes, s, net, (const T*)theta, theta_stride, N, (const T*)X, (const T*)w,
                       (const T*)f, (const T*)g, kind, (T*)r_w, (T*)J, ldJ, loss_partial, tp, nullptr, (int64_t)0,
                       nullptr, 0, fwd_only);
    return NGD_OK;
  };
  ngd_status st;
  if (dtype == NGD_F64) {
    st = nt == 1024 ? go(residual_jacobian_kernel<double, kJacobian, 1024>, 0.0)
                    : (nt == 512 ? go(residual_jacobian_kernel<double, kJacobian, 512>, 0.0)
                                 : go(residual_jacobian_kernel<double, kJacobian>, 0.0));
  } else {
    st = nt == 1024 ? go(residual_jacobian_kernel<float, kJacobian, 1024>, 0.f)
                    : (nt == 512 ? go(residual_jacobian_kernel<float, kJacobian, 512>, 0.f)
                                 : go(residual_jacobian_kernel<float, kJacobian>, 0.f));
  }
  NGD_TRY(st);
  NGD_HIP_TRY(hipGetLastError());
  return NGD_OK;
}

int vjp_grid(const NetDesc& net, int dtype, int64_t N, int max_wg) {
  size_t bytes = 0;
  const int tp = choose_tp(net, dtype == NGD_F64 ? 8 : 4, &bytes);
  const int64_t tiles = (N + tp - 1) / tp;
  return (int)(tiles < max_wg ? tiles : max_wg);
}

ngd_status launch_vjp(const NetDesc& net, int dtype, const void* theta, int64_t N, const void* X, const void* w,
                      const void* f, const void* g, const int8_t* kind, const double* wv, int64_t wv_stride,
                      void* partial, int64_t ld, double* tsq, int nwg, hipStream_t s) {
  size_t elem = dtype == NGD_F64 ? 8 : 4;
  size_t bytes = 0;
  int tp = choose_tp(net, elem, &bytes);
  const int64_t tiles = (N + tp - 1) / tp;
  if (nwg < 1 || nwg > tiles) {
    set_error("vjp: workgroup count out of range");
    return NGD_ERR_INVALID;
  }
  // the workgroup's P accumulators in LDS too when they fit beside the tile buffers
  const size_t with_acc = (bytes + 15) / 16 * 16 + (size_t)net.P * elem;
  const int acc_in_lds = with_acc <= 150 * 1024 && bytes % elem == 0 ? 1 : 0;
  if (acc_in_lds) bytes = (size_t)(lds_elems(net, tp) + net.P) * elem;
  if (dtype == NGD_F64) {
    auto k = residual_jacobian_kernel<double, kVjp>;
    NGD_HIP_TRY(hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
    hipLaunchKernelGGL(k, dim3(nwg), dim3(256), bytes, s, net, (const double*)theta, (int64_t)0, N, (const double*)X,
                       (const double*)w, (const double*)f, (const double*)g, kind, nullptr, (double*)partial, ld,
                       nullptr, tp, wv, wv_stride, tsq, acc_in_lds, 0);
  } else {
    auto k = residual_jacobian_kernel<float, kVjp>;
    NGD_HIP_TRY(hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
    hipLaunchKernelGGL(k, dim3(nwg), dim3(256), bytes, s, net, (const float*)theta, (int64_t)0, N, (const float*)X,
                       (const float*)w, (const float*)f, (const float*)g, kind, nullptr, (float*)partial, ld, nullptr,
                       tp, wv, wv_stride, tsq, acc_in_lds, 0);
  }
  NGD_HIP_TRY(hipGetLastError());
  return NGD_OK;
}

ngd_status launch_jvp(const NetDesc& net, int dtype, const void* theta, const void* U, int64_t ldU, int64_t k,
                      int64_t N, const void* X, const void* w, const int8_t* kind, int out_type, void* out,
                      int64_t ldo, int64_t cs, hipStream_t s) {
  if (k <= 0 || N <= 0) return NGD_OK;
  const size_t elem = dtype == NGD_F64 ? 8 : 4;
  int tp = 16;
  while (tp > 1 && jvp_lds_elems(net, tp) * elem > 64 * 1024) tp >>= 1;
  const size_t bytes = jvp_lds_elems(net, tp) * elem;
  if (bytes > 150 * 1024) {
    set_error("network too wide for the JVP kernel's LDS budget");
    return NGD_ERR_INVALID;
  }
  dim3 grid((unsigned)((N + tp - 1) / tp), (unsigned)k);
#define NGD_JVP(T, TO)                                                                                          \
  do {                                                                                                         \
    auto kf = jvp_kernel<T, TO>;                                                                               \
    NGD_HIP_TRY(hipFuncSetAttribute((const void*)kf, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes)); \
    hipLaunchKernelGGL(kf, grid, dim3(256), bytes, s, net, (const T*)theta, (const T*)U, ldU, N, (const T*)X,    \
                       (const T*)w, kind, (TO*)out, ldo, cs, tp);                                              \
  } while (0)
  if (dtype == NGD_F64 && out_type == NGD_F64) NGD_JVP(double, double);
  else if (dtype == NGD_F32 && out_type == NGD_F32) NGD_JVP(float, float);
  else if (dtype == NGD_F32 && out_type == NGD_F64) NGD_JVP(float, double);
  else {
    set_error("jvp: unsupported output type");
    return NGD_ERR_INVALID;
  }
#undef NGD_JVP
  NGD_HIP_TRY(hipGetLastError());
  return NGD_OK;
}

size_t residual_lds_bytes(const NetDesc& net, int dtype, int* tp) {
  size_t bytes = 0;
  *tp = choose_tp(net, dtype == NGD_F64 ? 8 : 4, &bytes);
  return bytes;
}

ngd_status launch_batch_residual_jacobian(int dtype, const BatchResidualItem* items, int n, int64_t total_tiles,
                                          size_t lds_bytes, hipStream_t s) {
  if (total_tiles <= 0) return NGD_OK;
  if (lds_bytes > 160 * 1024) {
    set_error("network too wide for the residual kernel's LDS budget");
    return NGD_ERR_INVALID;
  }
  // a persistent grid: a few workgroups per CU, striding over all tiles of all problems
  const int64_t grid = total_tiles < 2048 ? total_tiles : 2048;
  const int nt = jacobian_threads(lds_bytes);
  auto go = [&](auto k) -> ngd_status {
    NGD_HIP_TRY(hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes));
    hipLaunchKernelGGL(k, dim3((unsigned)grid), dim3(nt), lds_bytes, s, items, n, total_tiles);
    return NGD_OK;
  };
  ngd_status st;
  if (dtype == NGD_F64)
    st = nt == 1024 ? go(batch_residual_jacobian_kernel<double, 1024>)
                    : (nt == 512 ? go(batch_residual_jacobian_kernel<double, 512>) : go(batch_residual_jacobian_kernel<double>));
  else
    st = nt == 1024 ? go(batch_residual_jacobian_kernel<float, 1024>)
                    : (nt == 512 ? go(batch_residual_jacobian_kernel<float, 512>) : go(batch_residual_jacobian_kernel<float>));
  NGD_TRY(st);
  NGD_HIP_TRY(hipGetLastError());
  return NGD_OK;
}

ngd_status launch_reduce_sum(const double* partial, int64_t n_per, int n_sets, double scale, double* out,
                             hipStream_t s) {
  hipLaunchKernelGGL(reduce_sum_kernel, dim3(n_sets), dim3(256), 0, s, partial, n_per, scale, out);
  NGD_HIP_TRY(hipGetLastError());
  return NGD_OK;
}

int gradient_chunks(int64_t N) {
  int64_t c = (N + 255) / 256;
  return (int)(c < 64 ? c : 64);
}

ngd_status launch_gradient(int dtype, const void* J, int64_t ldJ, int64_t N, int64_t P, const void* r,
                           double* work, double* grad, hipStream_t s) {
  const int nchunk = gradient_chunks(N);
  const int64_t rows_per = (N + nchunk - 1) / nchunk;
  dim3 grid((unsigned)((P + 255) / 256), (unsigned)nchunk);
  if (dtype == NGD_F64)
    hipLaunchKernelGGL(colsum_stage1<double>, grid, dim3(256), 0, s, (const double*)J, ldJ, N, P,
                       (const double*)r, rows_per, work);
  else
    hipLaunchKernelGGL(colsum_stage1<float>, grid, dim3(256), 0, s, (const float*)J, ldJ, N, P, (const float*)r,
                       rows_per, work);
  hipLaunchKernelGGL(colsum_stage2, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, s, work, nchunk, P, grad);
  NGD_HIP_TRY(hipGetLastError());
  return NGD_OK;
}

}  // namespace ngd
