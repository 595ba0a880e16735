// The extern "C" boundary: argument checks, error codes, per-call device
// memory growth, and dispatch to the mining pipelines.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>

#include "pg_internal.h"

namespace pg {
const char* last_error();
void set_allocator(void* (*a)(size_t, void*), void (*f)(void*, void*), void* ctx);
void prof_enable(bool on);
void prof_reset();
bool prof_query(const char* name, double* ms, uint64_t* launches, double* units);
std::string prof_list();
int fsm_pattern_key(uint64_t index, int max_edges, int n_labels, int* shape, int32_t* labels5);

static int g_live_objects = 0;

// PG_TRACE_ARENA=1: report on stderr each time a call is rerun with a larger arena
static bool trace_arena() {
    static const bool on = [] {
        const char* e = std::getenv("PG_TRACE_ARENA");
        return e != nullptr && e[0] == '1';
    }();
    return on;
}

static void require_device() {
    static int have = -1;
    if (have < 0) {
        int n = 0;
        hipError_t e = hipGetDeviceCount(&n);
        have = (e == hipSuccess && n > 0) ? 1 : 0;
        if (e != hipSuccess) (void)hipGetLastError();
    }
    if (!have) throw Error{PG_EDEVICE, "no HIP device available"};
}

// Runs one mining call.  Per-call device memory comes from the graph's
// arena; when a call needs more than the arena holds, the arena grows (up
// to the memory budget) and the call is run again from the start.
template <class F>
static void run_with_arena(pg_graph* g, F&& body) {
    g->arena.need = 0;
    for (int attempt = 0;; ++attempt) {
        g->arena.begin_call();
        try {
            body();
            PG_HIP(hipStreamSynchronize(g->stream));
            prof_flush();
            return;
        } catch (const Error& e) {
            (void)hipStreamSynchronize(g->stream);
            prof_flush();
            if (e.code == PG_ENOMEM && e.msg == "arena" && attempt < 32) {
                const size_t cap = g->budget + (size_t(64) << 20);
                if (g->arena.need > cap)
                    throw Error{PG_ENOMEM, "memory budget too small for the embedding levels (need " +
                                               std::to_string(g->arena.need) + " bytes)"};
                // at least four times the last size and at least 64 MiB (within
                // the budget): a call finds its needs one push at a time, and
                // each retry runs it from the start
                const size_t floor_bytes = std::min<size_t>(cap, size_t(64) << 20);
                g->arena.want = std::min(std::max({g->arena.want, 4 * g->arena.buf.bytes, floor_bytes}),
                                         std::max(g->arena.need, cap));
                if (trace_arena())
                    std::fprintf(stderr, "[pangolin] call retried with an arena of %zu bytes (attempt %d)\n",
                                 g->arena.want, attempt + 1);
                g->arena.buf.release();
                continue;
            }
            throw;
        }
    }
}

}  // namespace pg

using namespace pg;

extern "C" {

const char* pg_version(void) { return "pangolin-hip 0.1 (gfx950)"; }

const char* pg_last_error(void) { return pg::last_error(); }

int pg_set_allocator(void* (*alloc)(size_t, void*), void (*free_)(void*, void*), void* ctx) {
    return guarded([&] {
        PG_REQUIRE((alloc == nullptr) == (free_ == nullptr), PG_EINVAL, "alloc and free must both be set or both NULL");
        PG_REQUIRE(g_live_objects == 0, PG_EINVAL, "allocator can only change while no graph or batch is loaded");
        set_allocator(alloc, free_, ctx);
    });
}

int pg_graph_load_csr(int64_t n, int64_t nnz, const int64_t* row_ptr, const int32_t* col_idx,
                      const int32_t* labels, int32_t n_labels, unsigned flags, void* stream, pg_graph** out) {
    return guarded([&] {
        PG_REQUIRE(out != nullptr, PG_EINVAL, "out is NULL");
        PG_REQUIRE((flags & ~(PG_DEVICE_PTRS | PG_CANONICALIZE)) == 0, PG_EINVAL, "unknown flag");
        require_device();
        pg_graph* g = new pg_graph();
        g->stream = static_cast<hipStream_t>(stream);
        try {
            PG_HIP(hipGetDevice(&g->device));
            g->budget = device_info().total_mem / 4;
            graph_load(g, n, nnz, row_ptr, col_idx, labels, n_labels, flags);
        } catch (...) {
            (void)hipStreamSynchronize(g->stream);
            delete g;
            throw;
        }
        ++g_live_objects;
        *out = g;
    });
}

int pg_graph_free(pg_graph* g) {
    return guarded([&] {
        if (!g) return;
        (void)hipStreamSynchronize(g->stream);
        delete g;
        --g_live_objects;
    });
}

int pg_graph_set_stream(pg_graph* g, void* stream) {
    return guarded([&] {
        PG_REQUIRE(g != nullptr, PG_EINVAL, "graph is NULL");
        PG_HIP(hipStreamSynchronize(g->stream));
        g->stream = static_cast<hipStream_t>(stream);
    });
}

int pg_graph_info(const pg_graph* g, int64_t* n, int64_t* nnz, int64_t* max_degree) {
    return guarded([&] {
        PG_REQUIRE(g != nullptr, PG_EINVAL, "graph is NULL");
        if (n) *n = g->n;
        if (nnz) *nnz = g->nnz;
        if (max_degree) *max_degree = g->max_deg;
    });
}

int pg_set_memory_budget(pg_graph* g, uint64_t bytes) {
    return guarded([&] {
        PG_REQUIRE(g != nullptr, PG_EINVAL, "graph is NULL");
        if (bytes == 0) bytes = device_info().total_mem / 4;
        g->budget = std::max<uint64_t>(bytes, uint64_t(1) << 20);
        g->arena.want = 0;
        g->arena.buf.release();
    });
}

int pg_graph_set_option(pg_graph* g, int option, int64_t value) {
    return guarded([&] {
        PG_REQUIRE(g != nullptr, PG_EINVAL, "graph is NULL");
        switch (option) {
            case PG_OPT_CLIQUE_MASKS: g->force_generic = (value == 0); break;
            case PG_OPT_FSM_BIT_KEYS: g->fsm_bit_keys = (value != 0); break;
            default: throw Error{PG_EINVAL, "unknown option " + std::to_string(option)};
        }
    });
}

int pg_count_cliques(pg_graph* g, int k, uint64_t* count) {
    return guarded([&] {
        PG_REQUIRE(g != nullptr && count != nullptr, PG_EINVAL, "NULL argument");
        PG_REQUIRE(k >= 1 && k <= PG_KMAX, PG_EUNSUPPORTED, "k must be in [1, 8]");
        require_device();
        uint64_t c = 0;
        run_with_arena(g, [&] { c = count_cliques(g, k); });
        *count = c;
    });
}

int pg_list_cliques(pg_graph* g, int k, int32_t* out, uint64_t capacity, uint64_t* total) {
    return guarded([&] {
        PG_REQUIRE(g != nullptr && total != nullptr, PG_EINVAL, "NULL argument");
        PG_REQUIRE(capacity == 0 || out != nullptr, PG_EINVAL, "out is NULL with a non-zero capacity");
        PG_REQUIRE(k >= 1 && k <= PG_KMAX, PG_EUNSUPPORTED, "k must be in [1, 8]");
        require_device();
        uint64_t c = 0;
        run_with_arena(g, [&] { c = list_cliques(g, k, out, capacity); });
        *total = c;
    });
}

int pg_count_motifs(pg_graph* g, int k, uint64_t* counts) {
    return guarded([&] {
        PG_REQUIRE(g != nullptr && counts != nullptr, PG_EINVAL, "NULL argument");
        PG_REQUIRE(k >= 3 && k <= 5, PG_EUNSUPPORTED, "motif size must be 3, 4 or 5");
        require_device();
        uint64_t c[21] = {0};
        run_with_arena(g, [&] { count_motifs(g, k, c); });
        std::memcpy(counts, c, sizeof(uint64_t) * (k == 3 ? 2 : (k == 4 ? 6 : 21)));
    });
}

int pg_fsm(pg_graph* g, int max_edges, uint64_t min_support, uint64_t* supports, size_t supports_len,
           size_t* n_frequent) {
    return guarded([&] {
        PG_REQUIRE(g != nullptr && supports != nullptr, PG_EINVAL, "NULL argument");
        PG_REQUIRE(max_edges >= 1 && max_edges <= 4, PG_EUNSUPPORTED, "max_edges must be in [1, 4]");
        PG_REQUIRE(g->n_labels > 0, PG_EINVAL, "FSM needs a labelled graph");
        PG_REQUIRE(fsm_num_patterns(max_edges, g->n_labels) > 0, PG_EUNSUPPORTED,
                   "patterns of four edges need at most 32 labels");
        const uint64_t np = fsm_num_patterns(max_edges, g->n_labels);
        PG_REQUIRE(supports_len >= np, PG_EINVAL, "supports array too short");
        require_device();
        std::vector<uint64_t> sup(np, 0);
        size_t nf = 0;
        run_with_arena(g, [&] { run_fsm(g, max_edges, min_support, sup.data(), np, &nf); });
        std::memcpy(supports, sup.data(), sizeof(uint64_t) * np);
        if (n_frequent) *n_frequent = nf;
    });
}

uint64_t pg_fsm_num_patterns(int max_edges, int n_labels) {
    if (max_edges < 1 || max_edges > 4 || n_labels < 1 || n_labels > 64) return 0;
    return fsm_num_patterns(max_edges, n_labels);
}

int pg_fsm_pattern_key(uint64_t index, int max_edges, int n_labels, int* shape, int32_t* labels5) {
    return guarded([&] {
        PG_REQUIRE(shape != nullptr && labels5 != nullptr, PG_EINVAL, "NULL argument");
        PG_REQUIRE(max_edges >= 1 && max_edges <= 4 && n_labels >= 1 && n_labels <= 64, PG_EINVAL,
                   "arguments out of range");
        PG_REQUIRE(index < fsm_num_patterns(max_edges, n_labels), PG_EINVAL, "index out of range");
        fsm_pattern_key(index, max_edges, n_labels, shape, labels5);
    });
}

int pg_profile_enable(int on) {
    prof_enable(on != 0);
    return PG_OK;
}

int pg_profile_reset(void) {
    prof_reset();
    return PG_OK;
}

int pg_profile_query(const char* kernel, double* total_ms, uint64_t* launches, double* units) {
    return guarded([&] {
        PG_REQUIRE(kernel != nullptr, PG_EINVAL, "kernel is NULL");
        PG_REQUIRE(prof_query(kernel, total_ms, launches, units), PG_EINVAL, std::string("no record for ") + kernel);
    });
}

int pg_profile_list(char* buf, size_t cap) {
    return guarded([&] {
        PG_REQUIRE(buf != nullptr && cap > 0, PG_EINVAL, "bad buffer");
        std::string s = prof_list();
        size_t n = std::min(cap - 1, s.size());
        std::memcpy(buf, s.data(), n);
        buf[n] = 0;
    });
}

}  // extern "C"

namespace pg {
void note_object(int delta) { g_live_objects += delta; }
}  // namespace pg
