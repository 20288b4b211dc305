// Batched ragged build + search (placeholder until the batched kernels land).
#include "ds_internal.h"

extern "C" {

size_t ds_batch_workspace_bytes(int32_t, int64_t, int64_t) { return 0; }
ds_status ds_search_batched(const ds_batch_desc*, hipStream_t) { return DS_ERR_UNSUPPORTED; }
ds_status ds_batch_report(const ds_batch_desc*, int32_t*, int64_t*, hipStream_t) { return DS_ERR_UNSUPPORTED; }

}  // extern "C"
