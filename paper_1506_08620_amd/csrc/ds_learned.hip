// Learned monotone CDF method (placeholder until the model kernels land).
#include "ds_internal.h"

namespace ds {

struct LearnedModel {};

ds_status learned_build(ds_index*, const ds_build_opts*, hipStream_t) { return DS_ERR_UNSUPPORTED; }
ds_status learned_search(ds_index*, const void*, int64_t, int32_t*, hipStream_t) { return DS_ERR_UNSUPPORTED; }
void learned_free(ds_index* h) {
  delete h->learned;
  h->learned = nullptr;
}

}  // namespace ds
