// Temporary: entry points not implemented yet.
#include "common.h"
extern "C" {
int gq_join_build(gq_ctx*, const gq_batch*, const int32_t*, int, const gq_pred*, int, const gq_join_opts*, hipStream_t, gq_join_table**) { return GQ_ERR_UNSUPPORTED; }
int gq_join_probe(gq_ctx*, const gq_join_table*, const gq_batch*, const int32_t*, int, const gq_pred*, int, int32_t*, int32_t*, int64_t, int64_t*, hipStream_t) { return GQ_ERR_UNSUPPORTED; }
const int64_t* gq_join_table_count_ptr(const gq_join_table*) { return nullptr; }
int gq_join_table_free(gq_ctx*, gq_join_table*, hipStream_t) { return GQ_ERR_UNSUPPORTED; }
int gq_gather(gq_ctx*, const gq_batch*, const int32_t*, int, const int32_t*, int64_t, gq_batch*, hipStream_t) { return GQ_ERR_UNSUPPORTED; }
int gq_groupby_agg(gq_ctx*, const gq_batch*, const int32_t*, int, const gq_pred*, int, const gq_agg*, int, const gq_groupby_opts*, gq_batch*, int64_t*, hipStream_t) { return GQ_ERR_UNSUPPORTED; }
int gq_pipeline(gq_ctx*, const gq_plan*, const gq_batch*, gq_batch*, int64_t*, hipStream_t) { return GQ_ERR_UNSUPPORTED; }
}
