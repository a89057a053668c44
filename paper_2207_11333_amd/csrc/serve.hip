// Serving scheduler (continuous batching of inference requests).
#include "runtime.hpp"

namespace hgnn {
void serve_shutdown(hgnn_ctx *) {}
} // namespace hgnn

using namespace hgnn;

extern "C" {
int hgnn_serve_start(hgnn_ctx *, const hgnn_serve_config *) {
  return set_error(HGNN_EINVAL, "serving not built yet");
}
int hgnn_serve_submit(hgnn_ctx *, const hgnn_batch *, uint64_t *) {
  return set_error(HGNN_EINVAL, "serving not started");
}
int hgnn_serve_poll(hgnn_ctx *, uint64_t, float *, int32_t *) {
  return set_error(HGNN_EINVAL, "serving not started");
}
int hgnn_serve_stats_get(hgnn_ctx *, hgnn_serve_stats *) {
  return set_error(HGNN_EINVAL, "serving not started");
}
int hgnn_serve_stop(hgnn_ctx *) { return HGNN_OK; }
}
