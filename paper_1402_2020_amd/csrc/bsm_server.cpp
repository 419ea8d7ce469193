// Serving: continuous batching of pairs submitted from the host.
#include "bsm_internal.h"

namespace bsm {
struct Server {};
void server_stop(Server *s) { delete s; }
}  // namespace bsm

using namespace bsm;

extern "C" {
bsm_status bsm_serve_config(bsm_ctx *ctx, size_t, int32_t) {
  clear_error();
  return fail(BSM_EINVAL, "serving is not available in this build");
}
bsm_status bsm_submit(bsm_ctx *ctx, const bsm_pair *, uint64_t *) {
  clear_error();
  return fail(BSM_EINVAL, "serving is not available in this build");
}
bsm_status bsm_poll(bsm_ctx *, uint64_t, int32_t *, bsm_times *) {
  clear_error();
  return fail(BSM_ENOTFOUND, "serving is not available in this build");
}
bsm_status bsm_drain(bsm_ctx *) {
  clear_error();
  return BSM_OK;
}
}
