// api_util.h -- turning internal exceptions into nd_status at the ABI.
#pragma once

#include <exception>
#include <new>

#include "internal.h"

namespace nd {

// Run f; map every failure to a status (never let an exception cross the
// C ABI).
template <class F>
nd_status guarded(F &&f) {
  try {
    f();
    return ND_OK;
  } catch (const Err &e) {
    return e.code;
  } catch (const std::bad_alloc &) {
    set_error("host allocation failed");
    return ND_ERR_OOM;
  } catch (const std::exception &e) {
    set_error("internal error: %s", e.what());
    return ND_ERR_DEVICE;
  } catch (...) {
    set_error("internal error");
    return ND_ERR_DEVICE;
  }
}

// Build what `kind` needs (idempotent).
void prepare(nd_graph *g, nd_kind kind, hipStream_t s);
// ND_ERR_INVALID unless 0 <= tau <= d_s everywhere.
void check_tau_range(nd_graph *g, const KindState &ks, const int32_t *tau,
                     hipStream_t s);

}  // namespace nd
