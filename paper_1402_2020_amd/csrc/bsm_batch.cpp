// Batched matching of many uneven pairs (bsm_match_batch).
#include "bsm_internal.h"

namespace bsm {

struct BatchState {
  Scratch scratch;
};

void batch_state_free(BatchState *b) { delete b; }

}  // namespace bsm

using namespace bsm;

extern "C" bsm_status bsm_match_batch(bsm_ctx *ctx, const bsm_pair *pairs, int32_t npairs,
                                      void *hip_stream) {
  clear_error();
  bsm_status st;
  if ((st = check_alive(ctx)) != BSM_OK) return st;
  if (npairs < 0 || (npairs > 0 && !pairs)) return fail(BSM_EINVAL, "invalid pair list");
  size_t need = 0;
  for (int i = 0; i < npairs; ++i) {
    const bsm_pair &p = pairs[i];
    if ((st = validate_image(p.left, p.width, p.height, p.stride)) != BSM_OK ||
        (st = validate_image(p.right, p.width, p.height, p.stride)) != BSM_OK ||
        (st = validate_dmax(p.width, p.dmax)) != BSM_OK)
      return fail(st, "pair %d: %s", i, bsm_last_error());
    if (!p.disp || (reinterpret_cast<uintptr_t>(p.disp) & 3u) ||
        (reinterpret_cast<uintptr_t>(p.cost) & 3u))
      return fail(BSM_EINVAL, "pair %d: misaligned or NULL output", i);
    need = std::max(need, match_scratch_bytes(ctx, p.width, p.height));
  }
  if (npairs == 0) return BSM_OK;
  if (!ctx->batch) ctx->batch = new BatchState;
  int prev = -1;
  (void)hipGetDevice(&prev);
  if (prev != ctx->device) (void)hipSetDevice(ctx->device);
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  hipError_t e;
  void *buf = ctx->batch->scratch.acquire(need, s, &e);
  if (!buf) st = device_fail(ctx, e, "batch scratch");
  for (int i = 0; st == BSM_OK && i < npairs; ++i) {
    const bsm_pair &p = pairs[i];
    st = match_on_stream(ctx, p.left, p.right, p.width, p.height, p.stride, p.dmax, p.disp,
                         p.cost, buf, s);
  }
  if (st == BSM_OK && (e = ctx->batch->scratch.release(s)) != hipSuccess)
    st = device_fail(ctx, e, "batch scratch event");
  if (prev >= 0 && prev != ctx->device) (void)hipSetDevice(prev);
  return st;
}
