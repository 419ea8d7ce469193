// bsm_match without any allocation.
//
// Some callers cannot allocate device memory while they run (work under HIP
// graph capture, tight serving loops, harnesses that forbid hipMalloc).  For
// them bsm_match_noalloc runs the same kernels as bsm_match, with the pair's
// scratch (two colour planes and three descriptor planes) in one fixed
// device array of this library instead of context memory.
//
// The array is a file-scope __device__ variable.  In host code its name
// stands for a host-side shadow, not a device address, so host code never
// passes it to a kernel: bsm_create calls noalloc_setup with its device
// current, which takes the array's device address on that device once with
// hipGetSymbolAddress and keeps it per device.  Every device holds its own
// copy of the array until the process ends.
#include "bsm_internal.h"

static __device__ __align__(256) unsigned char scratch[bsm::kNoAllocScratchBytes];

namespace bsm {
namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;                         // guards g_ptr
void *g_ptr[kMaxDevices] = {};           // device address of `scratch`, per device

void *scratch_on(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_mu);
  return g_ptr[device];
}

}  // namespace

hipError_t noalloc_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_ptr[device]) return hipSuccess;
  void *p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (!p) return hipErrorInvalidSymbol;
  g_ptr[device] = p;
  return hipSuccess;
}

}  // namespace bsm

using namespace bsm;

extern "C" bsm_status bsm_match_noalloc(bsm_ctx *ctx, const uint8_t *left, const uint8_t *right,
                                        int32_t W, int32_t H, int32_t stride, int32_t dmax,
                                        int32_t *disp, int16_t *cost, void *hip_stream) {
  clear_error();
  bsm_status st;
  if ((st = check_alive(ctx)) != BSM_OK) return st;
  if ((st = validate_image(left, W, H, stride)) != BSM_OK) return st;
  if ((st = validate_image(right, W, H, stride)) != BSM_OK) return st;
  if ((st = validate_dmax(W, dmax)) != BSM_OK) return st;
  if (!disp || (reinterpret_cast<uintptr_t>(disp) & 3u) || (reinterpret_cast<uintptr_t>(cost) & 3u))
    return fail(BSM_EINVAL, "disp must be a 4-byte aligned device pointer (cost too)");
  const size_t need = match_scratch_bytes(ctx, W, H);
  if (need > kNoAllocScratchBytes)
    return fail(BSM_ETOOBIG,
                "a %d x %d pair at n = %d needs %zu scratch bytes; bsm_match_noalloc holds at "
                "most %zu (use bsm_match)",
                W, H, ctx->n, need, kNoAllocScratchBytes);
  void *buf = scratch_on(ctx->device);
  if (!buf)
    return fail(BSM_EDEVICE, "no scratch address for device %d (context set-up did not run)",
                ctx->device);
  DeviceGuard g(ctx->device);
  if (g.err() != hipSuccess) return device_fail(ctx, g.err(), "hipSetDevice");
  // Everything on the caller's stream: no side stream, no event.
  return match_on_stream(ctx, left, right, W, H, stride, dmax, disp, cost, buf,
                         static_cast<hipStream_t>(hip_stream), nullptr, false);
}
