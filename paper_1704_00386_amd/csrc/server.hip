// server.hip -- request loop with continuous batching (placeholder until the
// server lands).
#include "api_util.h"
#include "internal.h"

using namespace nd;

extern "C" {
nd_status nd_server_create(nd_ctx *, int32_t, int32_t, nd_server **) {
  set_error("nd_server: not available in this build");
  return ND_ERR_UNSUPPORTED;
}
nd_status nd_server_submit(nd_server *, nd_graph *, nd_kind, const nd_opts *,
                           int32_t *, uint64_t *) {
  return ND_ERR_UNSUPPORTED;
}
nd_status nd_server_wait(nd_server *, uint64_t, int64_t, nd_result *, double *) {
  return ND_ERR_UNSUPPORTED;
}
nd_status nd_server_cancel(nd_server *, uint64_t) { return ND_ERR_UNSUPPORTED; }
void nd_server_destroy(nd_server *) {}
}
