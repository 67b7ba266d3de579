// batch.hip -- several graphs swept together (placeholder until the batched
// driver lands).
#include "api_util.h"
#include "internal.h"

using namespace nd;

extern "C" nd_status nd_batch_decompose(nd_ctx *ctx, int32_t count,
                                        nd_graph *const *graphs, nd_kind kind,
                                        const nd_opts *opts,
                                        int32_t *const *kappas, int on_device,
                                        void *stream, nd_result *res) {
  (void)ctx; (void)count; (void)graphs; (void)kind; (void)opts; (void)kappas;
  (void)on_device; (void)stream; (void)res;
  set_error("nd_batch_decompose: not available in this build");
  return ND_ERR_UNSUPPORTED;
}
