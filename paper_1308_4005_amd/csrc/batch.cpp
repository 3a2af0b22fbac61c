// Batched evaluation of many independent periodic boxes (placeholder until
// the persistent batched path lands).
#include "mls_internal.h"

using namespace mls;

struct mls_batch_s {
  int nbox = 0;
};

extern "C" {

mls_status mls_batch_create(int, const mls_params*, const int64_t*, int, mls_batch_t* out) {
  if (out) *out = nullptr;
  set_error("batched evaluation is not available in this build");
  return MLS_ERR_UNSUPPORTED;
}

mls_status mls_batch_evaluate(mls_batch_t, const double*, const double*, double*, double*, double*, void*) {
  set_error("batched evaluation is not available in this build");
  return MLS_ERR_UNSUPPORTED;
}

mls_status mls_batch_get_tuning(mls_batch_t, int*, int*, double*) {
  set_error("batched evaluation is not available in this build");
  return MLS_ERR_UNSUPPORTED;
}

mls_status mls_batch_destroy(mls_batch_t) { return MLS_OK; }

}  // extern "C"
