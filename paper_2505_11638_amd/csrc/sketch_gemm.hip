// The two large sketch contractions on the MFMA matrix cores, in "NT" form: C = alpha A B^T with
// A (M x K) and B (N x K) both K-contiguous. Z = J_w Omega uses A = J_w (N x P, the stored FP32
// Jacobian, converted to the compute type while it is staged) and B = Omega^T (ell x P); the
// second product B^T = Q^T J_w of the structured Alg. 6 runs as (J_w^T Q)^T with A = J_w^T and
// B = Q^T, both transposed copies in the compute type, and the result written transposed. These
// are the ell simultaneous Gramian matvecs of the sketch (Section 4.1.2, Table tab:matvec_costs).
// The second product can also take A = J_w^T straight from the stored J_w (A "K-major": A[m][k] at
// k lda + m), so that no transposed copy of J_w is made: the loader then reads 16-byte runs along m
// from four K-rows and writes them to LDS as 4-k chunks of one m in a chunk-major layout.
//
// Tiling for gfx950: a 256 x 128 workgroup tile, 4 wave64s in a 2 x 2 arrangement, so each wave
// owns a 128 x 64 block of 8 x 4 MFMA tiles (v_mfma_f32_16x16x32_bf16 for BF16, or
// v_mfma_f32_16x16x4f32 for FP32). One K-slab is 64 bytes per row in either type (32 BF16 or 16
// FP32 values), staged in LDS with an 80-byte row pitch (conflict-free 16-byte operand reads) and
// double-buffered: the next slab's global loads are in flight while the current one is multiplied
// out, with a single barrier per slab. Registers are capped for two workgroups per CU (the other
// workgroup's MFMA work covers this one's load latency). Tiles are numbered so that the workgroups that share an A
// row panel run on the same XCD (workgroups are dealt to the 8 XCDs round-robin), where the panel
// is then read from that XCD's L2.
#include <algorithm>
#include <mutex>
#include <type_traits>

#include "common.h"

namespace ngd {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned u4 __attribute__((ext_vector_type(4)));
typedef unsigned u2 __attribute__((ext_vector_type(2)));

constexpr int kBM = 256, kBN = 128, kThreads = 256;
constexpr int kRowBytes = 64;                 // one K-slab of one row
constexpr int kPitch = 80;                    // LDS row pitch in bytes
constexpr int kXcd = 8;

template <typename E> struct Slab { static constexpr int BK = kRowBytes / (int)sizeof(E); };

// One 16-byte LDS chunk (8 BF16 or 4 FP32 compute values) of a staged row, from the source type.
template <typename TS, typename E> struct Chunk;
template <> struct Chunk<float, __bf16> {
  static constexpr int N_LD = 2;  // two 16-byte global loads per chunk
  static __device__ __forceinline__ u4 convert(const u4* raw) {
    const f4 a = __builtin_bit_cast(f4, raw[0]), b = __builtin_bit_cast(f4, raw[1]);
    bf8 o;
    o[0] = (__bf16)a.x; o[1] = (__bf16)a.y; o[2] = (__bf16)a.z; o[3] = (__bf16)a.w;
    o[4] = (__bf16)b.x; o[5] = (__bf16)b.y; o[6] = (__bf16)b.z; o[7] = (__bf16)b.w;
    return __builtin_bit_cast(u4, o);
  }
};
template <> struct Chunk<__bf16, __bf16> {
  static constexpr int N_LD = 1;
  static __device__ __forceinline__ u4 convert(const u4* raw) { return raw[0]; }
};
template <> struct Chunk<float, float> {
  static constexpr int N_LD = 1;
  static __device__ __forceinline__ u4 convert(const u4* raw) { return raw[0]; }
};

// Registers holding this thread's chunks of one ROWS x BK slab of a K-contiguous operand.
// Chunk q = threadIdx.x + kThreads * i covers row q / 4, compute columns (q % 4) * CE ...
template <typename TS, typename E, int ROWS>
struct SlabLoader {
  static constexpr int CHUNKS = ROWS * 4 / kThreads;
  static constexpr int CE = 16 / (int)sizeof(E);             // compute values per chunk
  static constexpr int LD_BYTES = CE * (int)sizeof(TS) / Chunk<TS, E>::N_LD;
  u4 raw[CHUNKS][Chunk<TS, E>::N_LD];

  // rsrc spans this tile's rows only, so rows past the operand's end read as zero; columns at or
  // past K are zeroed explicitly in the last slab (they may hold the next row or padding).
  __device__ __forceinline__ void load(__amdgpu_buffer_rsrc_t rsrc, int64_t ld, int64_t k0, int64_t K) {
    const int c = threadIdx.x & 3;
#pragma unroll
    for (int i = 0; i < CHUNKS; ++i) {
      const int row = (threadIdx.x >> 2) + i * (kThreads / 4);
      const uint32_t off = (uint32_t)(((int64_t)row * ld + k0 + c * CE) * (int64_t)sizeof(TS));
#pragma unroll
      for (int h = 0; h < Chunk<TS, E>::N_LD; ++h)
        raw[i][h] = __builtin_amdgcn_raw_buffer_load_b128(rsrc, off + h * LD_BYTES, 0, 0);
    }
    if (k0 + Slab<E>::BK > K) {  // last, partial slab
#pragma unroll
      for (int i = 0; i < CHUNKS; ++i)
#pragma unroll
        for (int h = 0; h < Chunk<TS, E>::N_LD; ++h) {
          constexpr int PER = LD_BYTES / (int)sizeof(TS);
          TS v[PER];
          __builtin_memcpy(v, &raw[i][h], 16);
#pragma unroll
          for (int e = 0; e < PER; ++e)
            if (k0 + c * CE + h * PER + e >= K) v[e] = TS(0);
          __builtin_memcpy(&raw[i][h], v, 16);
        }
    }
  }
  __device__ __forceinline__ void store(unsigned char* lds) const {
    const int c = threadIdx.x & 3;
#pragma unroll
    for (int i = 0; i < CHUNKS; ++i) {
      const int row = (threadIdx.x >> 2) + i * (kThreads / 4);
      *reinterpret_cast<u4*>(lds + row * kPitch + c * 16) = Chunk<TS, E>::convert(raw[i]);
    }
  }
};

// LDS layout of a K-major A slab: 16-byte chunk (kc, m) holds compute values k = kc CE .. kc CE + CE - 1
// of row m at kc * kKcStride + 16 m. The stride is 16 (256 + 1) bytes, so the 16 lanes that the LDS
// serves together (chunks kc + 4 i, m = 4 j + e in the writes; kc, m0 + r16 in the MFMA reads) fall
// in 16 distinct 16-byte bank groups.
constexpr int kKcStride = 16 * (kBM + 1);

// Registers holding this thread's part of one BK x 256 slab of a K-major operand (m contiguous in
// memory): lane l of wave w covers k-chunk kc = l % 4 and columns m = 4 (16 w + l / 4) .. + 3, that
// is CE rows of 16 bytes (4 source values along m) each, converted to CE-value chunks along k.
template <typename TS, typename E>
struct KMajorLoader {
  static_assert(sizeof(TS) == 4, "K-major operands are stored in FP32");
  static constexpr int CE = 16 / (int)sizeof(E);  // compute values per chunk = source rows per thread
  u4 raw[CE];

  // The resource covers this slab's rows only (k0 .. min(k0 + BK, K) - 1 from column m0 on), so rows
  // at or past K read as zero; columns past the operand's M hold values that only reach rows of C
  // that are not stored.
  __device__ __forceinline__ void load(const TS* tile, int64_t lda, int64_t k0, int64_t K) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int kc = lane & 3, mq = 16 * w + (lane >> 2);
    constexpr int BK = Slab<E>::BK;
    const int64_t rows = K - k0 < BK ? K - k0 : BK;
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        (void*)(tile + k0 * lda), (short)0, (int)(rows * lda * (int64_t)sizeof(TS)), 0x00020000);
#pragma unroll
    for (int e = 0; e < CE; ++e) {
      const uint32_t off = (uint32_t)(((int64_t)(kc * CE + e) * lda + 4 * mq) * (int64_t)sizeof(TS));
      raw[e] = __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0);
    }
  }
  __device__ __forceinline__ void store(unsigned char* lds) const {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int kc = lane & 3, mq = 16 * w + (lane >> 2);
#pragma unroll
    for (int j = 0; j < 4; ++j) {  // column m = 4 mq + j: the CE values of k-chunk kc
      u4 o;
      if constexpr (sizeof(E) == 4) {
        o = u4{raw[0][j], raw[1][j], raw[2][j], raw[3][j]};
      } else {  // the 8 FP32 values of k-chunk kc, rounded as the row loader rounds them
        const u4 two[2] = {u4{raw[0][j], raw[1][j], raw[2][j], raw[3][j]}, u4{raw[4][j], raw[5][j], raw[6][j], raw[7][j]}};
        o = Chunk<float, __bf16>::convert(two);
      }
      *reinterpret_cast<u4*>(lds + kc * kKcStride + 16 * (4 * mq + j)) = o;
    }
  }
};

// Buffer resource over the tile's rows of an operand whose pointer has been advanced by `kbeg`
// columns (a split-K slice): the extent ends where the operand's last row of the tile ends.
template <typename T>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t tile_rsrc(const T* base, int64_t row0, int64_t rows_total,
                                                            int64_t rows_tile, int64_t ld, int64_t kbeg) {
  const int64_t rows = rows_total - row0 < rows_tile ? rows_total - row0 : rows_tile;
  return __builtin_amdgcn_make_buffer_rsrc((void*)(base + row0 * ld), (short)0,
                                           (int)((rows * ld - kbeg) * (int64_t)sizeof(T)), 0x00020000);
}

// Multiply one staged slab: acc[i][j] (16 x 16 tiles) += A_slab(wave rows) B_slab(wave cols)^T, for
// the tiles i < imax, j < jmax that hold rows and columns of C (wave-uniform bounds: the MFMAs of
// tiles wholly past the end of C are skipped, which frees the matrix core for the other waves)
template <typename E, bool FULL, bool AK>
__device__ __forceinline__ void slab_mfma(const unsigned char* As, const unsigned char* Bs, int wm, int wn,
                                          int imax, int jmax, f4 (&acc)[8][4]) {
  const int lane = threadIdx.x & 63;
  const int r16 = lane & 15, kq = lane >> 4;
  u4 b[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) b[j] = *reinterpret_cast<const u4*>(Bs + (wn + 16 * j + r16) * kPitch + 16 * kq);
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    if (!FULL && i >= imax) break;
    const u4 a = AK ? *reinterpret_cast<const u4*>(As + kq * kKcStride + 16 * (wm + 16 * i + r16))
                    : *reinterpret_cast<const u4*>(As + (wm + 16 * i + r16) * kPitch + 16 * kq);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (!FULL && j >= jmax) break;
      if constexpr (sizeof(E) == 2) {
        // lane holds k = 8 kq .. 8 kq + 7 of row r16 for both operands
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, a), __builtin_bit_cast(bf8, b[j]),
                                                            acc[i][j], 0, 0, 0);
      } else {
        // four K-steps; in step s lane supplies k = 4 kq + s for both operands (the same
        // permutation of the slab's 16 k on both sides leaves the sum unchanged)
        const f4 av = __builtin_bit_cast(f4, a), bv = __builtin_bit_cast(f4, b[j]);
#pragma unroll
        for (int s = 0; s < 4; ++s)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[s], bv[s], acc[i][j], 0, 0, 0);
      }
    }
  }
}

// C (M x N, ldc) = alpha A B^T, or C^T stored (C[n * ldc + m]) when trans_c. With split K
// (gridDim.y slices of kchunk), slice s writes its partial product to C + s * slice_stride.
template <typename TA, typename TB, typename E, typename TC, bool AK>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2, 2))) void nt_gemm_kernel(int64_t M, int64_t N, int64_t K, const TA* __restrict__ A,
                                                           int64_t lda, const TB* __restrict__ B, int64_t ldb,
                                                           TC* __restrict__ C, int64_t ldc, int trans_c, float alpha,
                                                           int tiles_n, int tiles, int per_xcd, int64_t kchunk,
                                                           int64_t slice_stride) {
  __shared__ __align__(16) unsigned char As[2][kBM * kPitch];
  __shared__ __align__(16) unsigned char Bs[2][kBN * kPitch];
  const int t = (int)(blockIdx.x % kXcd) * per_xcd + (int)(blockIdx.x / kXcd);
  if (t >= tiles) return;
  const int64_t m0 = (int64_t)(t / tiles_n) * kBM;
  const int64_t n0 = (int64_t)(t % tiles_n) * kBN;
  const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int wm = (wid >> 1) * 128, wn = (wid & 1) * 64;
  constexpr int BK = Slab<E>::BK;

  // this slice's K range: the operands are offset to its start, K becomes its length
  const int64_t kbeg = (int64_t)blockIdx.y * kchunk;
  A += AK ? kbeg * lda : kbeg;
  B += kbeg;
  C += (int64_t)blockIdx.y * slice_stride;
  K = (K - kbeg) < kchunk ? (K - kbeg) : kchunk;
  // a K-major A is addressed per slab from the tile's first column
  const TA* const at = A + m0;
  const __amdgpu_buffer_rsrc_t rb = tile_rsrc(B, n0, N, kBN, ldb, kbeg);
  const __amdgpu_buffer_rsrc_t ra = AK ? rb : tile_rsrc(A, m0, M, kBM, lda, kbeg);  // (unused when AK)
  // two register sets per operand: the slab after next is loaded while the next one waits in
  // registers for its LDS buffer, so two slabs of global loads are in flight behind the MFMAs
  typename std::conditional<AK, KMajorLoader<TA, E>, SlabLoader<TA, E, kBM>>::type la0, la1;
  SlabLoader<TB, E, kBN> lb0, lb1;
  f4 acc[8][4];
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};

  const int64_t nk = (K + BK - 1) / BK;
  const int imax = (int)((M - m0 - wm + 15) / 16), jmax = (int)((N - n0 - wn + 15) / 16);
  // (FP32 only: the BF16 instantiations are large enough that a second copy of the loop costs more
  // in instruction fetch than the skipped edge tiles save)
  const bool full = sizeof(E) == 2 || (imax >= 8 && jmax >= 4);
  auto load_a = [&](auto& la, int64_t k0) {
    if constexpr (AK) la.load(at, lda, k0, K);
    else la.load(ra, lda, k0, K);
  };
  load_a(la0, 0);
  lb0.load(rb, ldb, 0, K);
  if (nk > 1) {
    load_a(la1, BK);
    lb1.load(rb, ldb, BK, K);
  }
  la0.store(As[0]);
  lb0.store(Bs[0]);
  __syncthreads();
  // the K loop, with the tile bounds checked only in workgroups that hold an edge of C (the branch
  // is taken once, outside the loop, so the loads in flight across iterations are not waited for).
  // Step kt multiplies LDS buffer kt % 2; the register set that held slab kt is free and takes
  // slab kt + 2; the other set holds slab kt + 1 and goes to the other LDS buffer.
  auto kloop = [&](auto full_tag) {
    constexpr bool FULL = decltype(full_tag)::value;
    auto step = [&](int64_t kt, int cur, auto& la_free, auto& lb_free, auto& la_next, auto& lb_next) {
      if (kt + 2 < nk) {
        load_a(la_free, (kt + 2) * BK);
        lb_free.load(rb, ldb, (kt + 2) * BK, K);
      }
      slab_mfma<E, FULL, AK>(As[cur], Bs[cur], wm, wn, imax, jmax, acc);
      if (kt + 1 < nk) {
        la_next.store(As[cur ^ 1]);
        lb_next.store(Bs[cur ^ 1]);
      }
      __syncthreads();
    };
    for (int64_t kt = 0; kt < nk; kt += 2) {
      step(kt, 0, la0, lb0, la1, lb1);
      if (kt + 1 < nk) step(kt + 1, 1, la1, lb1, la0, lb0);
    }
  };
  if constexpr (sizeof(E) == 2) {
    kloop(std::true_type{});
  } else {
    if (full) kloop(std::true_type{});
    else kloop(std::false_type{});
  }

  // epilogue: lane holds column lane % 16 and rows 4 (lane / 16) + r of each 16 x 16 tile
  const int cn = lane & 15, rq = 4 * (lane >> 4);
  const bool vec_ok = (ldc & 3) == 0 && (reinterpret_cast<uintptr_t>(C) & 15) == 0;
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t gm = m0 + wm + 16 * i + rq;
      const int64_t gn = n0 + wn + 16 * j + cn;
      if (gn >= N) continue;
      if (trans_c) {
        TC* dst = C + gn * ldc + gm;
        if constexpr (sizeof(TC) == 4) {
          if (gm + 3 < M && vec_ok) {
            *reinterpret_cast<f4*>(dst) = alpha * acc[i][j];
            continue;
          }
        }
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (gm + r < M) dst[r] = (TC)(alpha * acc[i][j][r]);
      } else {
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (gm + r < M) C[(gm + r) * ldc + gn] = (TC)(alpha * acc[i][j][r]);
      }
    }
}

// dst (cols x rows, ld_d) = src (rows x cols, ld_s)^T converted to TD, through a 64 x 64 LDS tile
template <typename TS, typename TD>
__global__ __launch_bounds__(256) void transpose_cast_kernel(const TS* __restrict__ src, int64_t ld_s, int64_t rows,
                                                             int64_t cols, TD* __restrict__ dst, int64_t ld_d) {
  // staged in FP32 (the value is rounded to TD anyway), in FP64 for an FP64 destination
  using TT = typename std::conditional<std::is_same<TD, double>::value, double, float>::type;
  __shared__ TT tile[64][65];
  const int64_t r0 = (int64_t)blockIdx.y * 64, c0 = (int64_t)blockIdx.x * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const int r = ty + 4 * k;
    const int64_t gr = r0 + r, gc = c0 + tx;
    tile[r][tx] = (gr < rows && gc < cols) ? (TT)src[gr * ld_s + gc] : TT(0);
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const int c = ty + 4 * k;
    const int64_t gc = c0 + c, gr = r0 + tx;
    if (gc < cols && gr < rows) dst[gc * ld_d + gr] = (TD)tile[tx][c];
  }
}

// out = alpha sum_s work[s] over ks slices of `count` elements each, in a fixed order; out is laid out
// as `rows` x `cols` with leading dimension ld_out, the slices as rows x cols packed.
__global__ void splitk_sum_kernel(const float* __restrict__ work, int ks, int64_t rows, int64_t cols,
                                  float* __restrict__ out, int64_t ld_out, float alpha) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t count = rows * cols;
  if (idx >= count) return;
  // slices added in order, eight loads in flight
  float acc = 0.f;
  int q = 0;
  for (; q + 8 <= ks; q += 8) {
    float v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = work[(int64_t)(q + u) * count + idx];
#pragma unroll
    for (int u = 0; u < 8; ++u) acc += v[u];
  }
  for (; q < ks; ++q) acc += work[(int64_t)q * count + idx];
  const int64_t r = idx / cols, c = idx - r * cols;
  out[r * ld_out + c] = alpha * acc;
}

// Split-K choice from a small model of the launch. Workgroups are dealt to the XCDs round-robin in
// launch order (x fastest), and each XCD starts its next workgroup in the first of its resident
// slots (two per CU) that comes free. A workgroup lasts (its slabs) x (one slab's time with two
// workgroups per CU) x (its tile's weight): 1 for a full tile, less for an edge tile, whose MFMAs
// outside C are skipped but whose loads and barriers are not. Slices add their partial products'
// round trip through HBM (written by the GEMM, read by the ordered sum). The slab times are those
// measured on MI355X for the two compute types (FP32 runs near 78% of the MFMA peak, BF16 is bound
// by the L2 -> CU traffic of its FP32 operand).
constexpr double kSlabUsF32 = 4.4, kSlabUsBf16 = 1.5;
constexpr double kSumBytesPerUs = 5.0e6;  // 5 TB/s
constexpr int kXcdSlotsMax = 256;

double tile_weight(int64_t M, int64_t N, int64_t t, int64_t tiles_n) {
  const int64_t m0 = (t / tiles_n) * kBM, n0 = (t % tiles_n) * kBN;
  const double fm = (double)std::min<int64_t>(kBM, M - m0) / kBM, fn = (double)std::min<int64_t>(kBN, N - n0) / kBN;
  return 0.35 + 0.65 * fm * fn;
}

double predict_us(int64_t M, int64_t N, int64_t nk, int q, double slab_us, int64_t tiles_n, int64_t tiles,
                  int64_t per, int slots) {
  const int per_xcd_slots = std::max(1, std::min(kXcdSlotsMax, slots / kXcd));
  const int64_t slabs = (nk + q - 1) / q;
  double worst = 0.0;
  double free_at[kXcdSlotsMax];
  for (int x = 0; x < kXcd; ++x) {
    for (int i = 0; i < per_xcd_slots; ++i) free_at[i] = 0.0;
    for (int y = 0; y < q; ++y)
      for (int64_t j = 0; j < per; ++j) {
        const int64_t t = (int64_t)x * per + j;
        if (t >= tiles) break;
        int best = 0;
        for (int i = 1; i < per_xcd_slots; ++i)
          if (free_at[i] < free_at[best]) best = i;
        free_at[best] += (double)slabs * slab_us * tile_weight(M, N, t, tiles_n);
      }
    for (int i = 0; i < per_xcd_slots; ++i) worst = std::max(worst, free_at[i]);
  }
  if (q > 1) worst += (double)q * M * N * 8.0 / kSumBytesPerUs;
  return worst;
}

int choose_split(int64_t M, int64_t N, int64_t K, int BK, double slab_us, int64_t tiles_n, int64_t tiles, int64_t per,
                 int slots, int64_t work_elems) {
  // the prediction costs up to a few ms of host time for large grids, so it is made once per shape (a
  // batch of uneven problems brings two shapes per member)
  constexpr int kCache = 512;
  struct Entry { int64_t M, N, K, work; int BK, slots, ks; };
  static Entry cache[kCache];
  static int used = 0;
  static int next = 0;  // round-robin slot for a new shape once the table is full
  static std::mutex mu;
  std::lock_guard<std::mutex> lock(mu);
  for (int i = 0; i < used; ++i)
    if (cache[i].M == M && cache[i].N == N && cache[i].K == K && cache[i].work == work_elems && cache[i].BK == BK &&
        cache[i].slots == slots)
      return cache[i].ks;
  const int64_t nk = (K + BK - 1) / BK;
  int ks = 1;
  double best = predict_us(M, N, nk, 1, slab_us, tiles_n, tiles, per, slots);
  for (int q = 2; q <= 16; ++q) {
    if (nk / q < 8 || (int64_t)q * M * N > work_elems) break;
    const double c = predict_us(M, N, nk, q, slab_us, tiles_n, tiles, per, slots);
    if (c < best) {
      best = c;
      ks = q;
    }
  }
  if (used < kCache) {
    cache[used++] = Entry{M, N, K, work_elems, BK, slots, ks};
  } else {
    cache[next] = Entry{M, N, K, work_elems, BK, slots, ks};
    next = (next + 1) % kCache;
  }
  return ks;
}

template <typename TA, typename TB, typename E, typename TC, bool AK = false>
ngd_status run_nt(int64_t M, int64_t N, int64_t K, const void* A, int64_t lda, const void* B, int64_t ldb, void* C,
                  int64_t ldc, bool trans_c, double alpha, float* work, int64_t work_elems, hipStream_t s) {
  const int64_t tm = (M + kBM - 1) / kBM, tn = (N + kBN - 1) / kBN;
  const int64_t tiles = tm * tn;
  if (tiles == 0) return NGD_OK;
  const int64_t per = (tiles + kXcd - 1) / kXcd;
  constexpr int BK = Slab<E>::BK;
  // split K by the count of slices with the shortest predicted time (kept per shape)
  int ks = 1;
  if (work != nullptr) {
    // two resident workgroups per compute unit (initialised once, thread-safe)
    static const int slots = [] {
      int dev = 0, cus = 0;
      if (hipGetDevice(&dev) != hipSuccess ||
          hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
      return 2 * (cus > 0 ? cus : 1);
    }();
    if (slots == 0) {
      set_error("hipDeviceGetAttribute (compute unit count) failed");
      return NGD_ERR_HIP;
    }
    ks = choose_split(M, N, K, BK, sizeof(E) == 2 ? kSlabUsBf16 : kSlabUsF32, tn, tiles, per, slots, work_elems);
  }
  const int64_t kchunk = ks == 1 ? K : ((K + ks - 1) / ks + BK - 1) / BK * BK;
  if (ks == 1) {
    hipLaunchKernelGGL((nt_gemm_kernel<TA, TB, E, TC, AK>), dim3((unsigned)(per * kXcd), 1), dim3(kThreads), 0, s, M, N,
                       K, (const TA*)A, lda, (const TB*)B, ldb, (TC*)C, ldc, (int)trans_c, (float)alpha, (int)tn,
                       (int)tiles, (int)per, kchunk, (int64_t)0);
    NGD_HIP_TRY(hipGetLastError());
    return NGD_OK;
  }
  // slices in the output's own orientation (rows x cols packed), then one ordered sum
  const int64_t rows = trans_c ? N : M, cols = trans_c ? M : N;
  hipLaunchKernelGGL((nt_gemm_kernel<TA, TB, E, float, AK>), dim3((unsigned)(per * kXcd), (unsigned)ks), dim3(kThreads), 0,
                     s, M, N, K, (const TA*)A, lda, (const TB*)B, ldb, work, cols, (int)trans_c, 1.0f, (int)tn,
                     (int)tiles, (int)per, kchunk, rows * cols);
  NGD_HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(splitk_sum_kernel, dim3((unsigned)((rows * cols + 255) / 256)), dim3(256), 0, s, work, ks, rows,
                     cols, (float*)C, ldc, (float)alpha);
  NGD_HIP_TRY(hipGetLastError());
  return NGD_OK;
}

template <typename TS, typename TD>
__global__ void cast_rows_kernel(const TS* __restrict__ src, int64_t ld_s, int64_t rows, int64_t cols,
                                 TD* __restrict__ dst, int64_t ld_d) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t r = blockIdx.y;
  if (c < cols && r < rows) dst[r * ld_d + c] = (TD)src[r * ld_s + c];
}

}  // namespace

bool nt_gemm_supported(int a_type, int b_type, int compute, int64_t M, int64_t N, int64_t K, int64_t lda,
                       int64_t ldb, bool a_kmajor) {
  auto sz = [](int t) { return t == NGD_BF16 ? 2 : (t == NGD_F32 ? 4 : 8); };
  if (compute == G_F64 || a_type == NGD_F64 || b_type == NGD_F64) return false;
  if (compute == G_F32 && (a_type != NGD_F32 || b_type != NGD_F32)) return false;
  if (a_kmajor && a_type != NGD_F32) return false;
  // 16-byte aligned rows, and 32-bit byte offsets within one tile's rows (one slab's rows for a
  // K-major A, whose rows are M long)
  if ((lda * sz(a_type)) % 16 != 0 || (ldb * sz(b_type)) % 16 != 0) return false;
  if ((a_kmajor ? lda < M : lda < K) || ldb < K) return false;
  const int64_t a_rows = a_kmajor ? 32 : kBM;
  if (a_rows * lda * sz(a_type) >= (int64_t)1 << 31 || (int64_t)kBN * ldb * sz(b_type) >= (int64_t)1 << 31)
    return false;
  const int64_t tiles = ((M + kBM - 1) / kBM) * ((N + kBN - 1) / kBN);
  return tiles > 0 && tiles < ((int64_t)1 << 30);
}

ngd_status launch_nt_gemm(int a_type, const void* A, int64_t lda, int b_type, const void* B, int64_t ldb,
                          int compute, int64_t M, int64_t N, int64_t K, int c_type, void* C, int64_t ldc,
                          bool trans_c, double alpha, float* work, int64_t work_elems, hipStream_t s, bool a_kmajor) {
  if (!nt_gemm_supported(a_type, b_type, compute, M, N, K, lda, ldb, a_kmajor) || c_type != NGD_F32 ||
      (trans_c ? (ldc < M || ldc % 4 != 0) : ldc < N)) {
    set_error("nt_gemm: unsupported operand types or layout");
    return NGD_ERR_INVALID;
  }
  if (a_kmajor) {  // A = an FP32 matrix read K-major (no transposed copy)
    if (compute == G_F32)
      return run_nt<float, float, float, float, true>(M, N, K, A, lda, B, ldb, C, ldc, trans_c, alpha, work,
                                                      work_elems, s);
    if (b_type == NGD_BF16)
      return run_nt<float, __bf16, __bf16, float, true>(M, N, K, A, lda, B, ldb, C, ldc, trans_c, alpha, work,
                                                        work_elems, s);
    set_error("nt_gemm: unsupported operand types for a K-major A");
    return NGD_ERR_INVALID;
  }
  if (compute == G_F32) return run_nt<float, float, float, float>(M, N, K, A, lda, B, ldb, C, ldc, trans_c, alpha, work, work_elems, s);
  if (a_type == NGD_F32 && b_type == NGD_BF16)
    return run_nt<float, __bf16, __bf16, float>(M, N, K, A, lda, B, ldb, C, ldc, trans_c, alpha, work, work_elems, s);
  if (a_type == NGD_BF16 && b_type == NGD_BF16)
    return run_nt<__bf16, __bf16, __bf16, float>(M, N, K, A, lda, B, ldb, C, ldc, trans_c, alpha, work, work_elems, s);
  if (a_type == NGD_F32 && b_type == NGD_F32)
    return run_nt<float, float, __bf16, float>(M, N, K, A, lda, B, ldb, C, ldc, trans_c, alpha, work, work_elems, s);
  set_error("nt_gemm: unsupported operand types");
  return NGD_ERR_INVALID;
}

ngd_status launch_cast_rows(int src_type, const void* src, int64_t ld_s, int64_t rows, int64_t cols, int dst_type,
                            void* dst, int64_t ld_d, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return NGD_OK;
  dim3 grid((unsigned)((cols + 255) / 256), (unsigned)rows);
  if (src_type == NGD_F32 && dst_type == NGD_BF16)
    hipLaunchKernelGGL((cast_rows_kernel<float, __bf16>), grid, dim3(256), 0, s, (const float*)src, ld_s, rows, cols,
                       (__bf16*)dst, ld_d);
  else if (src_type == NGD_F64 && dst_type == NGD_F32)
    hipLaunchKernelGGL((cast_rows_kernel<double, float>), grid, dim3(256), 0, s, (const double*)src, ld_s, rows, cols,
                       (float*)dst, ld_d);
  else if (src_type == NGD_F64 && dst_type == NGD_F64)
    hipLaunchKernelGGL((cast_rows_kernel<double, double>), grid, dim3(256), 0, s, (const double*)src, ld_s, rows,
                       cols, (double*)dst, ld_d);
  else {
    set_error("cast_rows: unsupported types");
    return NGD_ERR_INVALID;
  }
  NGD_HIP_TRY(hipGetLastError());
  return NGD_OK;
}

ngd_status launch_transpose_cast(int src_type, const void* src, int64_t ld_s, int64_t rows, int64_t cols,
                                 int dst_type, void* dst, int64_t ld_d, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return NGD_OK;
  dim3 grid((unsigned)((cols + 63) / 64), (unsigned)((rows + 63) / 64));
#define NGD_TC(TS, TD)                                                                                         \
  hipLaunchKernelGGL((transpose_cast_kernel<TS, TD>), grid, dim3(256), 0, s, (const TS*)src, ld_s, rows, cols, \
                     (TD*)dst, ld_d)
  if (src_type == NGD_F32 && dst_type == NGD_BF16) NGD_TC(float, __bf16);
  else if (src_type == NGD_F32 && dst_type == NGD_F32) NGD_TC(float, float);
  else if (src_type == NGD_F64 && dst_type == NGD_BF16) NGD_TC(double, __bf16);
  else if (src_type == NGD_F64 && dst_type == NGD_F32) NGD_TC(double, float);
  else if (src_type == NGD_F64 && dst_type == NGD_F64) NGD_TC(double, double);
  else {
    set_error("transpose_cast: unsupported types");
    return NGD_ERR_INVALID;
  }
#undef NGD_TC
  NGD_HIP_TRY(hipGetLastError());
  return NGD_OK;
}

}  // namespace ngd
