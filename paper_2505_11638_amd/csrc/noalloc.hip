// The damped Gramian product of a stored J_w without a problem handle and without any allocation:
// the one-pass matvec's workgroup partials, its FP64 copies of v and y and its row sums live in a
// file-scope device array, whose address is looked up once per device.
#include <mutex>

#include "common.h"

using namespace ngd;

namespace {

constexpr size_t kScratchBytes = (size_t)NGD_NOALLOC_SCRATCH_BYTES;

// One copy per GPU, held until the process ends. Host code never passes this name to a kernel: it
// uses the per-device address from hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

size_t up256(size_t x) { return (x + 255) / 256 * 256; }

#define NGD_CHECK_ARG(cond, msg) \
  do {                           \
    if (!(cond)) {               \
      ::ngd::set_error(msg);     \
      return NGD_ERR_INVALID;    \
    }                            \
  } while (0)

// Scratch bytes of one call: the workgroup partials (nwg x ldJ, dtype), v and y in FP64, the
// workgroups' row sums. Every size the one-pass matvec accepts (ldJ * elem <= 150 KB, nwg <= 256)
// needs less than 40 MiB.
size_t scratch_bytes(int32_t dtype, int64_t n_rows, int64_t ldJ) {
  const size_t elem = dtype == NGD_F64 ? 8 : 4;
  const size_t nwg = (size_t)gram_rows_grid(dtype, n_rows, ldJ);
  return up256(nwg * (size_t)ldJ * elem) + 2 * up256((size_t)ldJ * 8) + up256(nwg * 8);
}

// The scratch array's address on the current device (looked up on the first call on that device).
ngd_status scratch_ptr(void** out) {
  int dev = 0;
  NGD_HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("device ordinal out of range for the static scratch table");
    return NGD_ERR_INVALID;
  }
  std::lock_guard<std::mutex> lock(g_mu);
  if (g_ptr[dev] == nullptr) {
    void* p = nullptr;
    NGD_HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return NGD_OK;
}

}  // namespace

extern "C" {

ngd_status ngd_gramian_matvec_noalloc(int32_t dtype, const void* J, int64_t ldJ, int64_t n_rows, int64_t n_params,
                                      const void* v, double lambda, void* y, void* stream) {
  NGD_CHECK_ARG(J != nullptr && v != nullptr && y != nullptr, "NULL argument");
  NGD_CHECK_ARG(dtype == NGD_F64 || dtype == NGD_F32, "dtype must be NGD_F64 or NGD_F32");
  NGD_CHECK_ARG(n_rows >= 1 && n_params >= 1, "n_rows and n_params must be >= 1");
  NGD_CHECK_ARG(ldJ >= n_params, "ldJ < n_params");
  const int vn = dtype == NGD_F64 ? 2 : 4;
  NGD_CHECK_ARG(ldJ % vn == 0, "ldJ must be a multiple of 16 bytes / element size");
  NGD_CHECK_ARG((reinterpret_cast<uintptr_t>(J) & 15u) == 0, "J must be 16-byte aligned");
  NGD_CHECK_ARG(gram_rows_supported(dtype, ldJ), "ldJ too large for the one-pass matvec");
  NGD_CHECK_ARG(lambda >= 0.0, "lambda must be >= 0");
  NGD_CHECK_ARG(v != y, "y must not alias v");
  const size_t need = scratch_bytes(dtype, n_rows, ldJ);
  if (need > kScratchBytes) {
    set_error("ngd_gramian_matvec_noalloc: this size needs " + std::to_string(need) +
              " bytes of scratch, more than the static maximum of " + std::to_string(kScratchBytes));
    return NGD_ERR_INVALID;
  }
  void* base = nullptr;
  NGD_TRY(scratch_ptr(&base));
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const int nwg = gram_rows_grid(dtype, n_rows, ldJ);
  const size_t elem = dtype == NGD_F64 ? 8 : 4;
  char* q = static_cast<char*>(base);
  void* partial = q;
  q += up256((size_t)nwg * ldJ * elem);
  double* v64 = reinterpret_cast<double*>(q);
  q += up256((size_t)ldJ * 8);
  double* y64 = reinterpret_cast<double*>(q);
  q += up256((size_t)ldJ * 8);
  double* tsq = reinterpret_cast<double*>(q);
  // every scratch word a kernel reads was written earlier in this call: nothing needs clearing
  NGD_TRY(launch_cast(dtype, v, NGD_F64, v64, n_params, s));
  NGD_TRY(launch_gram_rows(dtype, J, ldJ, n_rows, n_params, v64, partial, tsq, nwg, s, LaunchEvents{}));
  NGD_TRY(launch_gram_reduce(dtype, partial, nwg, ldJ, n_params, v64, lambda, y64, s));
  return launch_cast(NGD_F64, y64, dtype, y, n_params, s);
}

}  // extern "C"
