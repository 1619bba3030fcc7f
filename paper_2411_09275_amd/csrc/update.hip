// Batch updates (placeholder until the update path lands).
#include "pkd_internal.h"

namespace pkd {
int run_insert(pkd_tree*, hipStream_t, const int64_t*, const int64_t*, int64_t) { return PKD_ERR_UNSUPPORTED; }
int run_delete(pkd_tree*, hipStream_t, const int64_t*, const int64_t*, int64_t, int64_t*) {
  return PKD_ERR_UNSUPPORTED;
}
}  // namespace pkd
