// Internal declarations shared by the HIP sources of the mining library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "pangolin_hip.h"

namespace pg {

// ------------------------------------------------------------ error state

void set_error(const std::string& msg);

struct Error {
    int code;
    std::string msg;
};

#define PG_HIP(call)                                                                   \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess)                                                          \
            throw ::pg::Error{PG_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)}; \
    } while (0)

#define PG_REQUIRE(cond, code, msg)                     \
    do {                                                \
        if (!(cond)) throw ::pg::Error{(code), (msg)};  \
    } while (0)

// Runs body, converting exceptions to a status code.
template <class F>
int guarded(F&& body) {
    try {
        body();
        return PG_OK;
    } catch (const Error& e) {
        set_error(e.msg);
        return e.code;
    } catch (const std::bad_alloc&) {
        set_error("host allocation failed");
        return PG_ENOMEM;
    } catch (const std::exception& e) {
        set_error(e.what());
        return PG_EINVAL;
    }
}

// ---------------------------------------------------------------- memory

void* dev_alloc(size_t bytes);       // throws Error{PG_ENOMEM}
void dev_free(void* p);

// Grow-only device buffer.
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    void reserve(size_t need);
    void release();
    template <class T> T* as() const { return static_cast<T*>(p); }
    ~DevBuf() { release(); }
};

// Stack allocator over one device buffer: per-call temporaries are pushed
// and popped in LIFO order; the buffer grows only between calls.
struct Arena {
    DevBuf buf;
    size_t top = 0;
    size_t high = 0;   // high-water mark of the last call
    size_t want = 0;   // capacity to grow to before the next call
    size_t need = 0;   // largest size a push of this call required
    void begin_call();
    void* push(size_t bytes);   // 256-byte aligned; throws PG_ENOMEM when full
    // throws as push would if `bytes` more could not be pushed: a call checks
    // up front for room it needs later, so a short arena reruns it early
    void ensure(size_t bytes);
    size_t mark() const { return top; }
    void reset(size_t m) { top = m; }
    size_t avail() const { return buf.bytes > top ? buf.bytes - top : 0; }
};

template <class T>
T* push(Arena& a, size_t count) {
    return static_cast<T*>(a.push(count * sizeof(T)));
}

// --------------------------------------------------------------- profiling

bool prof_on();
// Brackets one kernel launch with events on `s` when profiling is on.
struct ProfScope {
    int slot = -1;
    hipStream_t s;
    ProfScope(const char* kernel, hipStream_t s, double units = 0.0);
    ~ProfScope();
};
void prof_flush();   // resolves pending events; stream must be synchronised

// ------------------------------------------------------------- device info

struct DeviceInfo {
    int device = 0;
    int n_cu = 256;
    size_t total_mem = 0;
};
const DeviceInfo& device_info();

// --------------------------------------------------------------- graph

// Layout and schedule of the 4-clique sibling-mask path.  They depend on
// the DAG's out-degrees only, so they are built once, beside the DAG.
// Roots whose out-degree exceeds the masks' limit (heavy roots) go through
// the general level kernels, over a CSR of their out-lists alone.
struct MaskPlan {
    bool built = false;
    int64_t words = 0;       // mask words of all light roots
    int64_t items = 0;       // count-pass work items
    int round = 64;          // level-1 entries per count-pass item (16 on small graphs)
    int64_t windows = 0;     // windows of roots for the fused last level
    int64_t heavy_edges = 0; // DAG edges of heavy roots
    DevBuf moff;             // uint64[n+1]: first mask word of each root (heavy roots: none)
    DevBuf item;             // uint64[items]: (light root, round of `round` level-1 entries)
    DevBuf wfirst;           // int64[windows+1]: first root of each window; wfirst[windows] = n
    DevBuf hrp;              // uint64[n+1]: heavy roots' out-lists in hcol (empty for light roots)
    DevBuf hcol;             // int32[heavy_edges]
    // heavy roots through wide rows in device memory (k <= 4)
    int64_t n_heavy = 0;     // heavy roots
    int64_t hwords = 0;      // their row words in all
    int64_t hitems = 0;      // work items (heavy root, block of rows)
    DevBuf hroot;            // int32[n_heavy]: the heavy roots (DAG ranks), ascending
    DevBuf hoff;             // uint64[n_heavy+1]: first row word of each
    DevBuf hitem;            // uint64[hitems]
};

struct Dag {
    bool built = false;
    int64_t n_edges = 0;     // directed DAG edges (= undirected edges)
    int64_t max_out = 0;
    DevBuf rank_of;          // int32[n]: rank of each original vertex in the degree order
    DevBuf rp;               // int64[n+1] over ranks
    DevBuf col;              // int32[n_edges], out-neighbours (ranks), ascending
    DevBuf src;              // int32[n_edges], source rank of every DAG edge (level-1 idx)
    MaskPlan plan;
};

struct MotifL1 {
    bool built = false;
    int64_t n_edges = 0;     // undirected edges (u < v)
    DevBuf seg;              // int64[n+1]: edges of vertex u are seg[u]..seg[u+1]-1
    DevBuf src;              // int32[n_edges] = u
    DevBuf dst;              // int32[n_edges] = v (> u), ascending within u
    DevBuf rev;              // int32[n_edges]: place after u in v's row, from the row's start
    // dense adjacency rows of high-degree vertices (membership in O(1))
    bool hubs_built = false;
    int64_t n_hubs = 0, hub_words = 0;
    DevBuf hub_id;           // int32[n]: row of the vertex, or -1
    DevBuf hub_bits;         // uint32[n_hubs][hub_words]
};

// The graph with its vertices renamed by decreasing degree (ties by id),
// for the 4-motif path.  Motif counts do not depend on vertex names; under
// this naming the smallest vertex of an embedding (its first vertex in the
// canonical order) is its highest-degree one, so the hub lists are the ones
// shared by many embeddings.
struct MotifGraph {
    bool built = false;
    int64_t n = 0, nnz = 0, max_deg = 0;
    DevBuf rp;               // int64[n+1]
    DevBuf col;              // int32[nnz], ascending per row
    MotifL1 ml1;
};

// The CSR a motif pipeline runs on: the input graph or the renamed one.
struct MotifView {
    int64_t n, nnz, max_deg;
    const int64_t* rp;
    const int32_t* col;
    MotifL1* ml1;
};

}  // namespace pg

struct pg_graph {
    int device = 0;
    hipStream_t stream = nullptr;
    int64_t n = 0, nnz = 0, max_deg = 0;
    int32_t n_labels = 0;
    pg::DevBuf rp, col, labels;
    pg::Dag dag;
    pg::MotifL1 ml1;
    pg::MotifGraph mg;
    uint64_t budget = 0;     // bytes for materialised levels
    bool force_generic = false;   // cliques: skip the sibling-mask path
    bool fsm_bit_keys = true;     // FSM: sorted bit keys for three-edge domains
    pg::Arena arena;
};

struct pg_batch;

namespace pg {

// ----------------------------------------------------------- primitives

// Exclusive prefix sum of m uint32 values into out[0..m] (out[m] = total),
// returns nothing; temporaries come from the arena.
void scan_u32(const uint32_t* in, int64_t m, uint64_t* out, Arena& a, hipStream_t s);
void scan_u64(const uint64_t* in, int64_t m, uint64_t* out, Arena& a, hipStream_t s);

// Stable LSD radix sort of uint64 keys on bits [lo_bit, hi_bit).  keys and
// tmp hold m entries; the sorted keys end in keys.
void radix_sort_u64(uint64_t* keys, uint64_t* tmp, int64_t m, int lo_bit, int hi_bit, Arena& a,
                    hipStream_t s);

// Sets n uint64 values to v (a kernel, so it is safe under graph capture).
void fill_u64(uint64_t* p, int64_t n, uint64_t v, hipStream_t s);
void fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t s);

uint64_t read_u64(const uint64_t* dev, hipStream_t s);   // synchronous

// Work items for load balance: segment p in [p_lo, p_lo + n_seg), whose
// children are seg[p] .. seg[p+1] (any offset base), is cut into rounds of
// `per` children; item = (p << ROUND_BITS) | round, in segment order.
// Returns the number of items; the array comes from the arena.  A caller
// that knows the children in all (total = seg[p_lo + n_seg] - seg[p_lo])
// passes it: the array is then sized by a bound and filled in one pass.
// With count_dev as well, the number of items is written there (on the
// stream) instead of being read back, and the bound is returned.
constexpr int ROUND_BITS = 24;
__host__ __device__ inline int64_t item_seg(uint64_t it) { return (int64_t)(it >> ROUND_BITS); }
__host__ __device__ inline int64_t item_round(uint64_t it) { return (int64_t)(it & ((1ull << ROUND_BITS) - 1)); }
int64_t round_items(const int64_t* seg, int64_t p_lo, int64_t n_seg, int per, Arena& a, hipStream_t s,
                    uint64_t** items, int64_t total = -1, uint64_t* count_dev = nullptr);
int64_t round_items(const uint64_t* seg, int64_t p_lo, int64_t n_seg, int per, Arena& a, hipStream_t s,
                    uint64_t** items, int64_t total = -1, uint64_t* count_dev = nullptr);
// The same over the segments with cmin <= children < cmax only.
int64_t round_items_between(const uint64_t* seg, int64_t p_lo, int64_t n_seg, int per, int64_t cmin, int64_t cmax,
                            Arena& a, hipStream_t s, uint64_t** items);

// ------------------------------------------------------------- pipelines

void graph_load(pg_graph* g, int64_t n, int64_t nnz, const int64_t* rp, const int32_t* col,
                const int32_t* labels, int32_t n_labels, unsigned flags);
void build_dag(pg_graph* g);
void build_motif_l1(pg_graph* g);
void build_motif_l1(pg_graph* g, const MotifView& v);
void build_motif_graph(pg_graph* g);
MotifView motif_view(pg_graph* g, bool renamed);
uint64_t count_cliques(pg_graph* g, int k);
uint64_t list_cliques(pg_graph* g, int k, int32_t* out, uint64_t capacity);
void count_motifs(pg_graph* g, int k, uint64_t* counts);
void run_fsm(pg_graph* g, int max_edges, uint64_t min_support, uint64_t* supports, size_t len,
             size_t* n_frequent);

uint64_t fsm_num_patterns(int max_edges, int n_labels);

int64_t grid_waves(int waves_per_cu);

}  // namespace pg
