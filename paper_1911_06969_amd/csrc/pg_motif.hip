// Vertex-induced motif counting (placeholder until the kernels land).
#include "pg_internal.h"

namespace pg {
void count_motifs(pg_graph* g, int k, uint64_t* counts) {
    (void)g; (void)k; (void)counts;
    throw Error{PG_EUNSUPPORTED, "motif counting not built yet"};
}
}  // namespace pg
