// Frequent subgraph mining (placeholder until the kernels land).
#include "pg_internal.h"

namespace pg {
uint64_t fsm_num_patterns(int max_edges, int n_labels) {
    (void)max_edges; (void)n_labels;
    return 0;
}
int fsm_pattern_key(uint64_t, int, int, int*, int32_t*) { return PG_EUNSUPPORTED; }
void run_fsm(pg_graph*, int, uint64_t, uint64_t*, size_t, size_t*) {
    throw Error{PG_EUNSUPPORTED, "FSM not built yet"};
}
}  // namespace pg
