/*
 * pangolin_hip.h -- C ABI of an MI355X (gfx950) graph pattern mining library.
 *
 * The library implements the extend-reduce-filter mining model of Pangolin
 * (Chen, Dathathri, Gill, Pingali, VLDB 2020): embeddings grow level by
 * level over a CSR graph (section 3.1, Algorithms 1-2), each level is kept
 * as a structure of arrays and built by a count pass, an exclusive prefix
 * sum and a write pass (sections 5.1 and 5.3), and the last level is fused
 * with pattern classification and reduction (section 5.2).  Counts are exact
 * unsigned 64-bit integers.
 *
 * Conventions for every call:
 *  - The return value is PG_OK (0) or a negative pg_status.  Outputs are
 *    written only when PG_OK is returned.  pg_last_error() describes the
 *    most recent failure of the calling thread.
 *  - Pointers documented as host memory are plain host pointers owned by
 *    the caller.  With PG_DEVICE_PTRS the graph arrays are device pointers
 *    owned by the caller and read only during the call.
 *  - The library owns every device buffer it allocates.  The graph is copied
 *    to device memory at load time and freed by pg_graph_free.
 *  - Mining calls are synchronous: they enqueue their kernels on the
 *    graph's stream and return after the results are on the host.  A graph
 *    is never modified after loading; several threads may mine one graph
 *    concurrently only if each uses its own graph handle.
 *  - There is no CPU fallback: without a usable HIP device every call that
 *    needs one returns PG_EDEVICE.
 */
#ifndef PANGOLIN_HIP_H
#define PANGOLIN_HIP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PG_OK = 0,
    PG_EINVAL = -1,        /* invalid argument or CSR violating the input rules */
    PG_ENOMEM = -2,        /* device allocation failed or budget too small */
    PG_EUNSUPPORTED = -3,  /* size k / max_edges outside the supported range */
    PG_EDEVICE = -4,       /* HIP runtime error or no device */
    PG_EOVERFLOW = -5      /* an index or count exceeded its integer width */
} pg_status;

typedef struct pg_graph pg_graph;   /* opaque, device resident */
typedef struct pg_batch pg_batch;   /* opaque, many small graphs, device resident */

/* flags for pg_graph_load_csr / pg_batch_load */
#define PG_DEVICE_PTRS 1u   /* the CSR arrays are device pointers */
#define PG_CANONICALIZE 2u  /* pg_graph_load_csr only: make the CSR canonical on the device */

#define PG_KMAX 8           /* largest clique size */

/* ----------------------------------------------------------------- graphs */

/*
 * Loads an undirected graph in CSR form (the input format of section 6.1:
 * symmetric, no self-loops, no duplicate edges, each neighbour list sorted
 * ascending).
 *   n         number of vertices, 0 <= n < 2^31
 *   nnz       number of directed entries (twice the edges), < 2^40
 *   row_ptr   int64[n+1], row_ptr[0] = 0, row_ptr[n] = nnz, non-decreasing
 *   col_idx   int32[nnz], neighbours of v at row_ptr[v] .. row_ptr[v+1]-1
 *   labels    int32[n] vertex labels in [0, n_labels), or NULL (unlabelled)
 *   n_labels  number of labels (0 when labels == NULL), at most 64
 *   flags     PG_DEVICE_PTRS and/or PG_CANONICALIZE, or 0
 *   stream    hipStream_t for all work on this graph, or NULL (null stream)
 *   out       receives the handle
 * The CSR is validated on the device; a violation returns PG_EINVAL.  With
 * PG_CANONICALIZE the library first rebuilds the rows on the device as the
 * symmetric closure of the entries, sorted ascending, without self-loops
 * and duplicates (the input itself is not modified); row_ptr must still be
 * non-decreasing from 0 to nnz and every id in [0, n), else PG_EINVAL.
 * pg_graph_info then reports the canonical nnz.
 */
int pg_graph_load_csr(int64_t n, int64_t nnz, const int64_t* row_ptr, const int32_t* col_idx,
                      const int32_t* labels, int32_t n_labels, unsigned flags, void* stream,
                      pg_graph** out);

/* Frees the graph and every device buffer it owns.  NULL is accepted. */
int pg_graph_free(pg_graph* g);

/* Replaces the stream the graph's work is enqueued on. */
int pg_graph_set_stream(pg_graph* g, void* stream);

/* Vertex count, directed entry count and maximum degree (host outputs,
 * any may be NULL). */
int pg_graph_info(const pg_graph* g, int64_t* n, int64_t* nnz, int64_t* max_degree);

/*
 * Bound on the device bytes one mining call may hold for materialised
 * embedding levels.  When a level would exceed it, the initial single-edge
 * embeddings are processed in chunks through all levels (edge blocking,
 * section 5.2) and the results summed.  0 restores the default (a quarter
 * of the device memory).  Values below 1 MiB are raised to 1 MiB.
 */
int pg_set_memory_budget(pg_graph* g, uint64_t bytes);

/*
 * Per-graph switches.
 *   PG_OPT_CLIQUE_MASKS  1 (default): k-cliques with k >= 3 on graphs
 *                        whose DAG out-degree is at most 768 record each
 *                        level-1 entry's children (its triangles) as a
 *                        bitmask over its root's out-list; k = 3 is their
 *                        number, and deeper levels count with popcounts;
 *                        0: the general level kernels for every k.
 *   PG_OPT_FSM_BIT_KEYS  1 (default): FSM sets the domain bits of patterns
 *                        of three edges (section 5.3) by writing one key
 *                        (bitmap word, bit) per embedding vertex, sorting
 *                        the keys by 64 KB bitmap block and OR-ing each
 *                        block in LDS, when the keys fit the memory budget
 *                        (32 B per embedding, twice); 0: an atomic OR per
 *                        embedding vertex into the bitmaps.  Supports are
 *                        the same either way.
 * Unknown options return PG_EINVAL.
 */
#define PG_OPT_CLIQUE_MASKS 1
#define PG_OPT_FSM_BIT_KEYS 2
int pg_graph_set_option(pg_graph* g, int option, int64_t value);

/*
 * Number of k-cliques (k pairwise adjacent vertices; section 2.2, with
 * triangle counting as k = 3).  Vertex-induced extension of the last vertex
 * only (eager pruning, section 4.1) on the degree-ordered DAG (section 4.1:
 * each edge points to the endpoint of higher degree, ties to the larger
 * id), toAdd = adjacency to every earlier vertex (the clique listing of
 * section 3.3).
 *   k      1 <= k <= PG_KMAX (k = 1 gives n, k = 2 the number of edges)
 *   count  host uint64, receives the count
 * The first call builds and caches the DAG on the device.
 */
int pg_count_cliques(pg_graph* g, int k, uint64_t* count);

/*
 * The k-cliques themselves (clique listing, section 3.3: the clique program
 * with the last level written out instead of counted).  The levels are
 * materialised as in pg_count_cliques (count pass, exclusive scan, write)
 * up to the last one, whose entries are the cliques.
 *   k         1 <= k <= PG_KMAX
 *   out       host int32[capacity * k], caller-owned: row i holds the i-th
 *             clique's vertex ids (original numbering), its lowest vertex
 *             in the degree order first, then one vertex per level; the
 *             order of the rows is that of the levels (by that lowest
 *             vertex, then level by level) and is the same on every call.
 *             May be NULL when capacity is 0.
 *   capacity  rows of out; cliques past it are counted, not written
 *   total     host uint64, receives the number of k-cliques
 * Errors: PG_EINVAL for NULL total, or NULL out with capacity > 0;
 * PG_EUNSUPPORTED for k out of range.
 */
int pg_list_cliques(pg_graph* g, int k, int32_t* out, uint64_t capacity, uint64_t* total);

/*
 * Vertex-induced motif counts for k = 3, 4 or 5 (section 2.2 motif
 * counting, section 3.3 Listing of motif counting with customised
 * classification, section 4.2).  Every connected induced k-vertex subgraph
 * is counted once, in the slot of its isomorphism class:
 *   k = 3: counts[0] wedge (path on 3 vertices), counts[1] triangle
 *   k = 4: counts[0] path, [1] 3-star, [2] 4-cycle, [3] paw (triangle with
 *          a pendant edge), [4] diamond (4-cycle with one chord), [5] 4-clique
 *   k = 5: the 21 connected graphs on five vertices, ordered by edge count,
 *          ties by the smallest 10-bit adjacency mask over all orderings of
 *          the five vertices (bit b(b-1)/2 + a set iff vertices a < b are
 *          adjacent); [0] the 4-star, [2] the path, [20] the 5-clique
 *   counts  host uint64[2], uint64[6] or uint64[21]
 * Errors: PG_EINVAL for NULL g or counts, PG_EUNSUPPORTED for k outside
 * 3..5.
 */
int pg_count_motifs(pg_graph* g, int k, uint64_t* counts);

/*
 * Frequent subgraph mining with minimum-image (domain) support (sections
 * 2.2 and 3.3, Listing of FSM): edge-induced embeddings over a labelled
 * graph, extended one edge per level up to max_edges edges (the paper's
 * "k-FSM" mines patterns of k-1 edges, so k-FSM is max_edges = k-1).  Before
 * each extension the embeddings of patterns whose support is below
 * min_support are dropped (Filter; pattern is frequent iff support >=
 * min_support).
 *   max_edges     1..4 (4 needs n_labels <= 32, else PG_EUNSUPPORTED)
 *   min_support   threshold sigma
 *   supports      host uint64[supports_len]; supports[i] = support of the
 *                 pattern with dense index i if it is frequent, else 0
 *   supports_len  >= pg_fsm_num_patterns(max_edges, n_labels)
 *   n_frequent    host, receives the number of frequent patterns (may be NULL)
 * Requires a labelled graph.
 */
int pg_fsm(pg_graph* g, int max_edges, uint64_t min_support, uint64_t* supports,
           size_t supports_len, size_t* n_frequent);

/*
 * Size of the dense pattern index used by pg_fsm for n_labels labels.  A
 * labelled pattern is a shape whose numbered vertex positions carry labels;
 * label tuples that a symmetry of the shape maps onto each other name one
 * pattern, represented by the lexicographically smallest of them.  The
 * index enumerates the shapes in this order, and within a shape its
 * representative tuples in lexicographic order:
 *   shape 0  single edge (a, b)                                   [1 edge]
 *   shape 1  wedge (centre, leaf, leaf)                           [2 edges]
 *   shape 2  triangle (a, b, c)                                   [3 edges]
 *   shape 3  path on 4 vertices, labels along the path
 *   shape 4  3-star (centre, three leaves)
 *   shape 5  path on 5 vertices, labels along the path            [4 edges]
 *   shape 6  4-star (centre, four leaves)
 *   shape 7  fork (the vertex of degree 3, its two leaves, the middle vertex
 *            of its leg of length 2, the end of that leg)
 *   shape 8  4-cycle, labels around the cycle
 *   shape 9  paw (the triangle vertex of degree 3, its pendant vertex, the
 *            two other triangle vertices)
 * so that, for instance, a wedge is (c, a, b) with a <= b and a path
 * (a, b, c, d) is read from the end that gives the smaller tuple.  Returns
 * 0 for arguments out of range.
 */
uint64_t pg_fsm_num_patterns(int max_edges, int n_labels);

/* Decodes a dense index into its shape (0..9) and the labels of its 2-5
 * positions (host outputs; labels5 is int32[5], unused slots are set to
 * -1). */
int pg_fsm_pattern_key(uint64_t index, int max_edges, int n_labels, int* shape, int32_t* labels5);

/* ---------------------------------------------------- many small graphs */

/*
 * Loads a batch of small graphs into one device allocation.  Graph g owns
 * vertices voff[g] .. voff[g+1]-1; row_ptr (int64[voff[n_graphs]+1]) gives
 * positions in col (int32, total row_ptr[voff[n_graphs]] entries); col
 * holds graph-local vertex ids.  Each graph must follow the CSR rules of
 * pg_graph_load_csr and have at most PG_BATCH_MAX_VERTICES vertices.
 * voff is host memory (int64[n_graphs+1]) in every case; row_ptr and col are
 * device pointers when PG_DEVICE_PTRS is set.
 */
#define PG_BATCH_MAX_VERTICES 512
int pg_batch_load(int64_t n_graphs, const int64_t* voff, const int64_t* row_ptr,
                  const int32_t* col, unsigned flags, void* stream, pg_batch** out);
int pg_batch_free(pg_batch* b);

/*
 * 4-motif (k = 4) or 3-motif (k = 3) counts of the graphs ids[0..n_ids) of a
 * batch (all graphs when ids == NULL, then n_ids is ignored), computed in
 * one persistent launch that takes graphs from a work queue, largest
 * estimated work first.  counts (host) receives n_ids rows of 6 (k = 4) or 2
 * (k = 3) uint64, in the order of ids.  Same slot order as pg_count_motifs.
 */
int pg_batch_count_motifs(pg_batch* b, int k, const int64_t* ids, int64_t n_ids, uint64_t* counts);

/*
 * Allocation-free form of pg_batch_count_motifs, for callers that cannot
 * allocate device memory during the call (tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments, results and errors, and it runs
 * the same kernel.  It calls no device allocation routine: its temporaries
 * (the ids, the queue items, the output rows and the queue counter) live in
 * one fixed device array of 2 MiB per GPU, set up on the GPU's first call
 * and held until the process ends.
 * Limits: n_ids (the batch size when ids == NULL) at most
 * PG_BATCH_STATIC_MAX_IDS, else PG_EINVAL; each graph is split into at most
 * 4 queue items.
 * Every call on a GPU uses that GPU's one array, which keeps the previous
 * call's contents (the call clears what must start at zero).  Calls that
 * overlapped on one GPU would race on it, so the library serialises them
 * with a per-device lock: a concurrent caller waits.  The batch's device is
 * made current for the call and the caller's current device is restored.
 */
#define PG_BATCH_STATIC_MAX_IDS 16384
int pg_batch_count_motifs_noalloc(pg_batch* b, int k, const int64_t* ids, int64_t n_ids, uint64_t* counts);

/*
 * Asynchronous slots for a serving loop.  A slot owns pinned host buffers,
 * device buffers for up to max_ids graphs and a captured HIP graph of one
 * batched launch (copy in, clear, count, copy out), replayed on the slot's
 * stream for every submission.  Slots on different streams run
 * concurrently; they share only the read-only batch.
 *   pg_batch_slot_create  max_ids >= 1; stream: hipStream_t; NULL makes the
 *                         slot create (and later destroy) a non-blocking
 *                         stream of its own, since the null stream cannot
 *                         be captured
 *   pg_batch_slot_submit  enqueues the counts of ids[0..n_ids) (host array,
 *                         n_ids <= max_ids) and returns at once; the slot
 *                         must be idle (PG_EINVAL otherwise)
 *   pg_batch_slot_query   1 when the last submission has finished (or none
 *                         is pending), 0 while it runs
 *   pg_batch_slot_wait    waits for the last submission and copies its rows
 *                         (n_ids x 6 for k = 4, x 2 for k = 3) to counts
 *                         (host); the slot becomes idle
 *   pg_batch_slot_free    waits, then releases the slot
 */
typedef struct pg_batch_slot pg_batch_slot;
int pg_batch_slot_create(pg_batch* b, int64_t max_ids, void* stream, pg_batch_slot** out);
int pg_batch_slot_submit(pg_batch_slot* s, int k, const int64_t* ids, int64_t n_ids);
int pg_batch_slot_query(pg_batch_slot* s);
int pg_batch_slot_wait(pg_batch_slot* s, uint64_t* counts);
int pg_batch_slot_free(pg_batch_slot* s);

/* Estimated device work of each graph (host double[n_graphs]), the
 * quantity the batch scheduler orders graphs by. */
int pg_batch_work_estimate(const pg_batch* b, double* work);

/* Tile/work-split parameters of the batch kernel (the values an autotuner
 * picks).  0 keeps the current value.  block_threads in {64, 128, 256,
 * 512}; split_work is the estimated work above which a graph is split into
 * several queue items; grid_blocks is the persistent grid size.  They apply
 * to every later pg_batch_count_motifs call, and slots re-capture their
 * launch with them at their next submission. */
int pg_batch_set_params(pg_batch* b, int block_threads, double split_work, int grid_blocks);

/* --------------------------------------------------------------- runtime */

/* Text of the last failure on this thread (never NULL). */
const char* pg_last_error(void);

/*
 * Routes the library's device allocations through alloc/free_ (for example
 * a caching allocator).  alloc(bytes, ctx) returns device memory or NULL;
 * free_(ptr, ctx) releases it.  Passing NULL for both restores hipMalloc /
 * hipFree.  Must be called while no graph or batch is loaded.
 */
int pg_set_allocator(void* (*alloc)(size_t bytes, void* ctx), void (*free_)(void* ptr, void* ctx),
                     void* ctx);

/*
 * Kernel timing.  When enabled, every kernel launch is bracketed by HIP
 * events on the stream it runs on and its duration is added to the named
 * kernel's total.  pg_profile_query returns the total milliseconds, the
 * number of launches and the work units reported for `kernel` (returns
 * PG_EINVAL for an unknown name).  pg_profile_list writes up to `cap`
 * kernel names, separated by newlines, into buf.
 */
int pg_profile_enable(int on);
int pg_profile_reset(void);
int pg_profile_query(const char* kernel, double* total_ms, uint64_t* launches, double* units);
int pg_profile_list(char* buf, size_t cap);

/* Library version string. */
const char* pg_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PANGOLIN_HIP_H */
