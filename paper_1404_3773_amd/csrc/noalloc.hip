// H*X for callers that cannot allocate device memory (code under HIP graph
// capture, tight serving loops): ces_apply_H_noalloc runs the same kernels as
// ces_apply_H with its scratch regions carved from a fixed, file-scope device
// array instead of a caller workspace.
//
// The array is a device symbol: host code never uses its name as an address.
// Its device address is looked up with hipGetSymbolAddress once per device,
// with that device current, on the first call there, and kept per device; every
// later call on that device passes the stored address to the kernels.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "ces_internal.h"

namespace {

// Largest scratch one call may use: 256 MiB per device, held from the first
// call on a device until the process ends.  An H*X of k columns needs the
// regions of ces::hx_layout (about 2 n_r L^2 k + n_r n_theta (2L - 1) k
// elements, plus 2 d k FP32 copies in mixed precision): k = 32 on a basis of
// L_max = 30, N = 60 with a 90 x 62 x 124 grid fits in both precisions.
constexpr size_t kScratchBytes = CES_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

std::mutex g_mu;
void* g_dev_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up once per
// device and cached).
ces_status scratch_address(void** out) {
  int dev = 0;
  CES_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices)
    return ces::fail(CES_ERR_DEVICE, "device ordinal beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_dev_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return ces::fail(CES_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch): ") +
                                           hipGetErrorString(e));
    g_dev_ptr[dev] = p;
  }
  *out = g_dev_ptr[dev];
  return CES_OK;
}

}  // namespace

extern "C" ces_status ces_apply_H_noalloc(ces_ham hh, int k, const double* d_X, int64_t ldx,
                                         double* d_Y, int64_t ldy, int prec, void* stream) {
  using namespace ces;
  CES_TRY(check_ham(hh));
  Ham& h = hh->h;
  CES_TRY(check_block(h, k, d_X, ldx, "X"));
  CES_TRY(check_block(h, k, d_Y, ldy, "Y"));
  if (prec != CES_PREC_FP64 && prec != CES_PREC_MIXED)
    return fail(CES_ERR_INVALID_ARG, "unknown precision");
  const Layout ly = hx_layout(h, k, prec);
  if (ly.total > kScratchBytes)
    return fail(CES_ERR_WORKSPACE, "H*X of " + std::to_string(k) + " columns needs " +
                                       std::to_string(ly.total) +
                                       " bytes of scratch, above the fixed " +
                                       std::to_string(kScratchBytes));
  void* work = nullptr;
  CES_TRY(scratch_address(&work));
  // Every region is written before it is read (padding columns included), so
  // nothing left by an earlier call needs clearing.
  return apply_H_impl(h, ly, work, k, d_X, ldx, d_Y, ldy, prec,
                      static_cast<hipStream_t>(stream));
}
