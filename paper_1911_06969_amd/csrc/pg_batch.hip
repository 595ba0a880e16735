// Batched and served motif counting over many small graphs (placeholder
// until the kernels land).
#include "pg_internal.h"

extern "C" {
int pg_batch_load(int64_t, const int64_t*, const int64_t*, const int32_t*, unsigned, void*, pg_batch**) {
    pg::set_error("batch mode not built yet");
    return PG_EUNSUPPORTED;
}
int pg_batch_free(pg_batch*) { return PG_OK; }
int pg_batch_count_motifs(pg_batch*, int, const int64_t*, int64_t, uint64_t*) {
    pg::set_error("batch mode not built yet");
    return PG_EUNSUPPORTED;
}
int pg_batch_count_motifs_async(pg_batch*, int, const int64_t*, int64_t, uint64_t*, void*) {
    pg::set_error("batch mode not built yet");
    return PG_EUNSUPPORTED;
}
int pg_batch_work_estimate(const pg_batch*, double*) { return PG_EUNSUPPORTED; }
int pg_batch_set_params(pg_batch*, int, double, int) { return PG_EUNSUPPORTED; }
}
