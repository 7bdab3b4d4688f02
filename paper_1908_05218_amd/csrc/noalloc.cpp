// Allocation-free exact H^2 mat-vec (h2_matvec_noalloc) for callers that
// cannot allocate device memory: its temporaries live in a file-scope device
// array, located once per device when the first context on that device is
// created.  The computation is h2_matvec's (same kernels, same order).
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "internal.h"

namespace {

// One copy per device, held until the process ends.  Host code never uses
// the array's name as an address (it is a host-side stand-in): the device
// address comes from hipGetSymbolAddress below.
static __device__ __align__(256) char scratch[H2_MATVEC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};

}  // namespace

namespace h2 {

h2_status noalloc_setup(int device) {
  if (device < 0 || device >= kMaxDevices)
    return set_error(H2_ERR_DEVICE, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_scratch[device]) return H2_OK;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) {
    (void)hipGetLastError();
    return set_error(H2_ERR_DEVICE, std::string("hipGetSymbolAddress of the scratch array: ") +
                                        hipGetErrorString(e));
  }
  g_scratch[device] = ptr;
  return H2_OK;
}

}  // namespace h2

extern "C" h2_status h2_matvec_noalloc(h2_ctx ctx, h2_mat M, const double* x_dev, double* y_dev,
                                       int64_t nrhs, hipStream_t stream) {
  using namespace h2;
  if (!ctx || !M || !x_dev || !y_dev || nrhs < 1) return set_error(H2_ERR_ARG, "bad argument");
  ctx = home_of(ctx, M);
  if (!ctx) return set_error(H2_ERR_ARG, "M belongs to another context");
  std::lock_guard<std::recursive_mutex> lk(ctx->mu);
  try {
    if (!M->mv) return set_error(H2_ERR_ARG, "M has no mat-vec task lists");
    void* scr = nullptr;
    {
      std::lock_guard<std::mutex> g(g_mu);
      scr = ctx->device < kMaxDevices ? g_scratch[ctx->device] : nullptr;
    }
    if (!scr) return set_error(H2_ERR_DEVICE, "no scratch array on this device");
    const size_t need = matvec_scratch_bytes(M, nrhs);
    if (need > H2_MATVEC_SCRATCH_BYTES)
      return set_error(H2_ERR_UNSUPPORTED,
                       "the mat-vec temporaries need " + std::to_string(need) +
                           " bytes, beyond the scratch array of " +
                           std::to_string((size_t)H2_MATVEC_SCRATCH_BYTES) + " bytes");
    H2_HIP(hipSetDevice(ctx->device));
    matvec_impl(ctx, M, x_dev, y_dev, nrhs, stream ? stream : ctx->stream, scr,
                H2_MATVEC_SCRATCH_BYTES);
    return H2_OK;
  } catch (const Error& e) {
    (void)hipGetLastError();
    return set_error(e.code, e.msg);
  } catch (const std::exception& e) {
    return set_error(H2_ERR_INTERNAL, e.what());
  }
}
