// k-clique counting: vertex-induced extension of the last vertex only, on
// the degree-ordered DAG (Pangolin sections 3.3 and 4.1, clique Listing).
//
// Embedding list.  Level L1 holds the single-edge embeddings (the DAG
// edges); level L_i holds (i+1)-cliques.  Each level is a structure of
// arrays: vid[] (the newest vertex of every embedding) plus the offsets
// seg[] of the children of every embedding of the previous level, which is
// the prefix sum the count pass produces (section 5.3) and encodes the
// idx[] column of section 5.1 in compressed form: the parent of entry x is
// the p with seg[p] <= x < seg[p+1].
//
// Extension.  toExtend = last vertex only, toAdd = adjacent to every earlier
// vertex.  The siblings of an entry x (the children of x's parent) are
// exactly the vertices adjacent to all of x's earlier vertices and later in
// the order; so the children of x are out(vid[x]) intersected with the
// siblings after x.  One wave takes one parent segment, stages the sibling
// list in LDS, streams the out-lists of the siblings from HBM (coalesced,
// several siblings per 64-lane step) and tests each candidate by a
// branch-free binary search in the LDS copy.
//
// Three modes share the kernel: COUNT (children per entry, for the scan),
// WRITE (children at their scanned offsets, ascending) and LAST (the fused
// last level: candidates are tested and counted, never stored; each wave
// keeps its count in a register and adds it once, section 5.2).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>
#include <vector>

#include "pg_device.h"
#include "pg_internal.h"

namespace pg {

constexpr int CQ_THREADS = 256;
constexpr int CQ_WAVES = CQ_THREADS / WAVE;
constexpr int CQ_SMAX = 1024;          // sibling lists up to this length live in LDS
constexpr int CQ_ROUND = 256;          // entries of a segment per work item (long segments spread over waves)
constexpr int CQ_TRIM_MIN = 48;        // out-lists at least this long are trimmed to max(S)

enum { MODE_COUNT = 0, MODE_WRITE = 1, MODE_LAST = 2 };

struct CliqueArgs {
    XcdQueue Q;                         // over items[], or parent segments [p_lo, p_lo + n_items) if null
    const uint64_t* items;              // (parent, round of CQ_ROUND entries of its segment)
    int64_t p_lo;
    const int64_t* seg;                 // seg[p] - seg_base = first entry of segment p
    int64_t seg_base;
    const int32_t* vid;                 // entries of this level
    int64_t x_lo, x_hi;                 // only entries in [x_lo, x_hi) are extended
    const int64_t* rp;                  // DAG
    const int32_t* col;
    uint32_t* count;                    // COUNT: children of entry x
    const uint64_t* start;              // WRITE: children of x begin at start[x] - start_base
    uint64_t start_base;
    int32_t* out_vid;                   // WRITE
    unsigned long long* stats;          // LAST: [0] cliques, [1] input entries, [2] sum of out-degrees
};

struct CliqueLds {
    int32_t S[CQ_WAVES][CQ_SMAX];
    uint32_t pre[CQ_WAVES][WAVE];
    int64_t lo[CQ_WAVES][WAVE];
    uint32_t cnt[CQ_WAVES][WAVE];
};

struct CliqueAcc {
    uint64_t found = 0, n_in = 0, deg_sum = 0;
};

// Extends the entries of one parent segment whose sibling list is S
// (LDS or global; the pointer's address space is known after inlining).
template <int MODE, class SPtr>
__device__ __forceinline__ void clique_segment(const CliqueArgs& A, CliqueLds& L, int w, SPtr S, int32_t s,
                                               int64_t b, int32_t r0, int32_t r1, CliqueAcc& acc) {
    const int32_t s_last = S[s - 1];
    const int32_t x0 = (int32_t)max64(r0, A.x_lo - b);
    const int32_t x1 = (int32_t)min64(min(s, r1), A.x_hi - b);
    for (int32_t xc = x0; xc < x1; xc += WAVE) {
        const int32_t x = xc + lane();
        int64_t lo = 0;
        uint32_t d = 0;
        if (x < x1) {
            const int32_t v = S[x];
            const int64_t r0 = A.rp[v], r1 = A.rp[v + 1];
            if (MODE == MODE_LAST) {
                acc.n_in += 1;
                acc.deg_sum += (uint64_t)(r1 - r0);
            }
            if (x < s - 1) {
                // candidates lie in (S[x], S[s-1]]: out(v) is above v already
                const int64_t hi = (r1 - r0 >= CQ_TRIM_MIN) ? upper_bound(A.col, r0, r1, s_last) : r1;
                lo = r0;
                d = (uint32_t)(hi - r0);
            }
        }
        const uint32_t inc = wave_incl_scan(d);
        const uint32_t W = bcast(inc, WAVE - 1);
        L.pre[w][lane()] = inc - d;
        L.lo[w][lane()] = lo;
        if (MODE != MODE_LAST) L.cnt[w][lane()] = 0;
        wave_sync();
        const int nx = min(WAVE, x1 - xc);
        for (uint32_t t0 = 0; t0 < W; t0 += WAVE) {
            const uint32_t t = t0 + lane();
            const bool valid = t < W;
            // xi: the entry whose candidate range holds t
            int xi = 0;
            {
                int n_i = nx;
                while (n_i > 1) {
                    const int half = n_i >> 1;
                    if (L.pre[w][xi + half] <= t) xi += half;
                    n_i -= half;
                }
            }
            bool found = false;
            int32_t u = 0;
            if (valid) {
                u = A.col[L.lo[w][xi] + (t - L.pre[w][xi])];
                const int32_t after = xc + xi + 1;
                found = contains(S + after, s - after, u);
            }
            if (MODE == MODE_LAST) {
                acc.found += found;
            } else if (MODE == MODE_COUNT) {
                if (found) atomicAdd(&L.cnt[w][xi], 1u);
            } else {
                // lanes of one entry are contiguous; rank found candidates in lane order
                const int key = valid ? xi : WAVE;   // invalid lanes form their own group
                const int prev = __shfl_up(key, 1, WAVE);
                const bool head = lane() == 0 || prev != key;
                const uint64_t H = ballot(head);
                const uint64_t F = ballot(found);
                const uint64_t le = lanemask_lt() | (1ull << lane());
                const int h = 63 - __clzll(H & le);
                const uint64_t grp = le & ~((1ull << h) - 1ull);
                const uint32_t base = valid ? L.cnt[w][xi] : 0u;
                if (found) {
                    const uint64_t dst = A.start[b + xc + xi] - A.start_base + base +
                                         (uint64_t)popc64(F & grp & lanemask_lt());
                    A.out_vid[dst] = u;
                }
                const bool next_head = (lane() == WAVE - 1) || ((H >> (lane() + 1)) & 1ull);
                wave_sync();
                if (valid && next_head) L.cnt[w][xi] = base + (uint32_t)popc64(F & grp);
                wave_sync();
            }
        }
        if (MODE == MODE_COUNT) {
            wave_sync();
            if (x < x1) A.count[b + x] = L.cnt[w][lane()];
        }
        wave_sync();
    }
}

template <int MODE>
__global__ __launch_bounds__(CQ_THREADS) void k_clique_ext(CliqueArgs A) {
    __shared__ CliqueLds L;
    const int w = threadIdx.x / WAVE;
    CliqueAcc acc;
    QueueCursor cur = queue_start();
    int64_t it_end = 0;
    for (int64_t it = queue_next(A.Q, cur, it_end); it >= 0; it = queue_next(A.Q, cur, it_end)) {
        for (int64_t j = it; j < it_end; ++j) {
            int64_t p = A.p_lo + j;
            int32_t r0 = 0, r1 = 0x7fffffff;
            if (A.items) {
                const uint64_t item = (uint64_t)uniform64((int64_t)A.items[j]);
                p = item_seg(item);
                r0 = (int32_t)item_round(item) * CQ_ROUND;
                r1 = r0 + CQ_ROUND;
            }
            const int64_t b = A.seg[p] - A.seg_base;
            const int64_t e = A.seg[p + 1] - A.seg_base;
            const int32_t s = (int32_t)(e - b);
            if (s <= 0) continue;
            if (s <= CQ_SMAX) {
                for (int i = lane(); i < s; i += WAVE) L.S[w][i] = A.vid[b + i];
                wave_sync();
                clique_segment<MODE>(A, L, w, &L.S[w][0], s, b, r0, r1, acc);
            } else {
                clique_segment<MODE>(A, L, w, A.vid + b, s, b, r0, r1, acc);
            }
            wave_sync();
        }
    }
    if (MODE == MODE_LAST) {
        const uint64_t f = wave_sum_u64(acc.found);
        const uint64_t ni = wave_sum_u64(acc.n_in);
        const uint64_t ds = wave_sum_u64(acc.deg_sum);
        if (lane() == 0 && (f | ni)) {
            atomicAdd(&A.stats[0], (unsigned long long)f);
            atomicAdd(&A.stats[1], (unsigned long long)ni);
            atomicAdd(&A.stats[2], (unsigned long long)ds);
        }
    }
}

// Chunk boundaries for edge blocking: entry c_j = largest c with
// start[c] <= j * cap (j = 1..nb-1), plus the segment of the previous level
// that holds entry c_j.
__global__ void k_chunk_bounds(const uint64_t* __restrict__ start, int64_t m, uint64_t cap, int64_t nb,
                               const int64_t* __restrict__ seg, int64_t seg_base, int64_t n_seg,
                               int64_t* __restrict__ out_c, int64_t* __restrict__ out_p,
                               uint64_t* __restrict__ out_s) {
    const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (j > nb) return;
    int64_t c;
    if (j == 0) c = 0;
    else if (j == nb) c = m;
    else {
        const uint64_t target = start[0] + (uint64_t)j * cap;
        int64_t lo = 0, hi = m;   // largest c in [0, m] with start[c] <= target
        while (lo < hi) {
            const int64_t mid = (lo + hi + 1) >> 1;
            if (start[mid] <= target) lo = mid; else hi = mid - 1;
        }
        c = lo;
    }
    // segment p with seg[p] - seg_base <= c < seg[p+1] - seg_base (last such p)
    int64_t lo = 0, hi = n_seg;
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (seg[mid] - seg_base <= c) lo = mid; else hi = mid - 1;
    }
    out_c[j] = c;
    out_p[j] = lo;
    out_s[j] = start[c];
}

// One materialised level as the general path holds it: the vertex of each
// entry, and the segments of the parent level that give each entry's parent
// (the largest p in [p_lo, p_hi) with seg[p] - seg_base <= entry).  At
// level 1 the parents are the roots.
struct LevelRef {
    const int32_t* vid = nullptr;
    const int64_t* seg = nullptr;
    int64_t seg_base = 0, p_lo = 0, p_hi = 0;
};

struct LevelChain {
    LevelRef l[PG_KMAX];
};

// Listing: where the cliques go (host rows of k vertex ids).
struct ListOut {
    int32_t* host = nullptr;
    uint64_t capacity = 0;       // rows
    uint64_t found = 0;          // cliques met so far (also past capacity)
    const int32_t* vertex_of_rank = nullptr;
};

struct CliqueRun {
    pg_graph* g;
    int k;
    hipStream_t s;
    unsigned long long* stats;
    unsigned long long* qctr;   // Q_WORDS words of queue counters
    int64_t waves;
    int blocks;
    uint64_t mwords = 0;        // mask path: words of all mask rows
    bool long_segments = false; // general path: segments may exceed CQ_ROUND entries
    ListOut* list = nullptr;    // listing instead of counting (general path)
    LevelChain chain;           // general path: the levels above the current one
};

// Writes the k-cliques of entries [y0, y1) of level L = k - 1 as rows of
// original vertex ids (root first, then one vertex per level), out[(y - y0)
// * k + j].  Each thread walks one entry's parents up to its root.
__global__ void k_clique_emit(LevelChain C, int L, int64_t y0, int64_t y1, const int32_t* __restrict__ vertex_of_rank,
                              int32_t* __restrict__ out) {
    for (int64_t y = y0 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; y < y1;
         y += (int64_t)gridDim.x * blockDim.x) {
        int32_t* row = out + (y - y0) * (L + 1);
        int64_t e = y;
        for (int l = L; l >= 1; --l) {
            const LevelRef& R = C.l[l - 1];
            row[l] = vertex_of_rank[R.vid[e]];
            // the parent: the last segment starting at or before e
            int64_t lo = R.p_lo, hi = R.p_hi - 1;
            while (lo < hi) {
                const int64_t mid = (lo + hi + 1) >> 1;
                if (R.seg[mid] - R.seg_base <= e) lo = mid; else hi = mid - 1;
            }
            e = lo;
        }
        row[0] = vertex_of_rank[e];
    }
}

constexpr int64_t LIST_ROWS = 1 << 20;   // cliques per copy to the host

// Cliques are entries [y0, y1) of the last level: those that still fit the
// caller's rows are copied there (in pieces of LIST_ROWS), all are counted.
static void emit_cliques(CliqueRun& R, int64_t y0, int64_t y1) {
    ListOut& O = *R.list;
    Arena& ar = R.g->arena;
    const uint64_t before = O.found;
    const uint64_t room = O.capacity > before ? O.capacity - before : 0;
    const int64_t copy_end = y0 + (int64_t)std::min<uint64_t>((uint64_t)(y1 - y0), room);
    for (int64_t a = y0; a < copy_end; a += LIST_ROWS) {
        const int64_t b = std::min<int64_t>(copy_end, a + LIST_ROWS);
        const size_t mk = ar.mark();
        int32_t* rows = push<int32_t>(ar, (size_t)(b - a) * R.k);
        const unsigned blocks = (unsigned)std::min<int64_t>((b - a + 255) / 256, 65535);
        k_clique_emit<<<blocks, 256, 0, R.s>>>(R.chain, R.k - 1, a, b, O.vertex_of_rank, rows);
        PG_HIP(hipGetLastError());
        PG_HIP(hipMemcpyAsync(O.host + (before + (uint64_t)(a - y0)) * R.k, rows,
                              sizeof(int32_t) * (size_t)(b - a) * R.k, hipMemcpyDeviceToHost, R.s));
        PG_HIP(hipStreamSynchronize(R.s));
        ar.reset(mk);
    }
    O.found = before + (uint64_t)(y1 - y0);
}

// Work items are parent segments, or rounds of CQ_ROUND entries of them
// when some segment is longer than a round (a segment's entries are then
// spread over several waves).
template <int MODE>
static void launch(CliqueRun& R, CliqueArgs A, int64_t p_lo, int64_t n_seg, const char* name, double units) {
    if (n_seg <= 0) return;
    Arena& ar = R.g->arena;
    const size_t mk = ar.mark();
    int64_t n_items = n_seg;
    A.items = nullptr;
    if (R.long_segments) {
        uint64_t* items = nullptr;
        n_items = round_items(A.seg, p_lo, n_seg, CQ_ROUND, ar, R.s, &items);
        A.items = items;
        p_lo = 0;
    }
    if (n_items > 0) {
        fill_u64(reinterpret_cast<uint64_t*>(R.qctr), Q_WORDS, 0, R.s);
        A.Q.next = R.qctr;
        A.Q.n_items = n_items;
        A.Q.chunk = n_items >= R.waves * 64 ? 16 : (n_items >= R.waves * 8 ? 4 : 1);
        A.p_lo = p_lo;
        A.stats = R.stats;
        ProfScope ps(name, R.s, units);
        k_clique_ext<MODE><<<R.blocks, CQ_THREADS, 0, R.s>>>(A);
        PG_HIP(hipGetLastError());
    }
    ar.reset(mk);
}

// Extends the entries [x_lo, x_hi) of level `lev` (segments [p_lo, p_hi) of
// its parents cover them) through the remaining levels.
static void extend_level(CliqueRun& R, int lev, const int64_t* seg, int64_t seg_base, int64_t p_lo, int64_t p_hi,
                         const int32_t* vid, int64_t x_lo, int64_t x_hi) {
    pg_graph* g = R.g;
    Arena& ar = g->arena;
    R.chain.l[lev - 1] = LevelRef{vid, seg, seg_base, p_lo, p_hi};
    if (R.list && lev == R.k - 1) {   // listing: the entries of this level are the cliques
        emit_cliques(R, x_lo, x_hi);
        return;
    }
    CliqueArgs A{};
    A.seg = seg;
    A.seg_base = seg_base;
    A.vid = vid;
    A.x_lo = x_lo;
    A.x_hi = x_hi;
    A.rp = g->dag.rp.as<int64_t>();
    A.col = g->dag.col.as<int32_t>();
    if (lev == R.k - 2 && !R.list) {
        launch<MODE_LAST>(R, A, p_lo, p_hi - p_lo, "clique_last", 0.0);
        return;
    }
    const int64_t m = x_hi - x_lo;
    if (m <= 0) return;
    const size_t mk = ar.mark();
    // count pass (inspection) -> exclusive prefix sum -> exact allocation -> write pass
    uint32_t* cnt = push<uint32_t>(ar, m);
    uint64_t* start = push<uint64_t>(ar, m + 1);
    A.count = cnt - x_lo;   // indexed by entry id
    launch<MODE_COUNT>(R, A, p_lo, p_hi - p_lo, "clique_count", (double)m);
    scan_u32(cnt, m, start, ar, R.s);
    const uint64_t total = read_u64(start + m, R.s);
    if (total == 0) {
        ar.reset(mk);
        return;
    }
    PG_REQUIRE(total < (uint64_t(1) << 40), PG_EOVERFLOW, "level size exceeds 2^40 entries");
    const bool next_last = (lev + 1 == R.k - 2) && !R.list;
    // bytes per entry of the next level: vid, plus count + start if it is
    // extended again
    const uint64_t per = next_last ? 4 : 4 + 4 + 8;
    const uint64_t room = g->budget > ar.mark() ? (g->budget - ar.mark()) : 0;
    uint64_t cap = std::max<uint64_t>(room / (per * (next_last ? 1 : 2)), (uint64_t)R.g->dag.max_out + 1);
    int64_t nb = (int64_t)((total + cap - 1) / cap);
    std::vector<int64_t> hc(nb + 1), hp(nb + 1);
    std::vector<uint64_t> hs(nb + 1);
    if (nb == 1) {
        hc[0] = 0; hc[1] = m;
        hp[0] = p_lo; hp[1] = p_hi - 1;
        hs[0] = 0; hs[1] = total;
    } else {
        const size_t mk2 = ar.mark();
        int64_t* dc = push<int64_t>(ar, nb + 1);
        int64_t* dp = push<int64_t>(ar, nb + 1);
        uint64_t* ds = push<uint64_t>(ar, nb + 1);
        k_chunk_bounds<<<(unsigned)((nb + 1 + 255) / 256), 256, 0, R.s>>>(start, m, cap, nb, seg + p_lo,
                                                                         seg_base + x_lo, p_hi - p_lo, dc, dp, ds);
        PG_HIP(hipGetLastError());
        PG_HIP(hipMemcpyAsync(hc.data(), dc, sizeof(int64_t) * (nb + 1), hipMemcpyDeviceToHost, R.s));
        PG_HIP(hipMemcpyAsync(hp.data(), dp, sizeof(int64_t) * (nb + 1), hipMemcpyDeviceToHost, R.s));
        PG_HIP(hipMemcpyAsync(hs.data(), ds, sizeof(uint64_t) * (nb + 1), hipMemcpyDeviceToHost, R.s));
        PG_HIP(hipStreamSynchronize(R.s));
        ar.reset(mk2);
        for (int64_t j = 0; j <= nb; ++j) hp[j] += p_lo;
    }
    uint64_t biggest = 0;
    for (int64_t j = 0; j < nb; ++j) biggest = std::max<uint64_t>(biggest, hs[j + 1] - hs[j]);
    int32_t* next_vid = push<int32_t>(ar, std::max<uint64_t>(biggest, 1));
    for (int64_t j = 0; j < nb; ++j) {
        const int64_t c0 = hc[j], c1 = hc[j + 1];
        if (c1 <= c0) continue;
        // write pass for entries [x_lo + c0, x_lo + c1): their segments run
        // from the one holding c0 to the one holding c1 - 1
        CliqueArgs W = A;
        W.x_lo = x_lo + c0;
        W.x_hi = x_lo + c1;
        W.start = start - x_lo;
        W.start_base = hs[j];
        W.out_vid = next_vid;
        int64_t q_lo = hp[j], q_hi;
        if (nb == 1) q_hi = p_hi;
        else {
            // the segment holding entry c1 - 1 is the last p with seg[p] <= c1 - 1
            q_hi = (j + 1 == nb) ? p_hi : hp[j + 1] + 1;
        }
        launch<MODE_WRITE>(R, W, q_lo, q_hi - q_lo, "clique_write", (double)(hs[j + 1] - hs[j]));
        // next level: segments are the entries [c0, c1) of this level, whose
        // children offsets (rebased by hs[j]) are start[c0..c1]
        extend_level(R, lev + 1, reinterpret_cast<const int64_t*>(start), (int64_t)hs[j], c0, c1, next_vid, 0,
                     (int64_t)(hs[j + 1] - hs[j]));
    }
    ar.reset(mk);
}

// ---------------------------------------------------------------------
// 4-cliques with per-root sibling masks.
//
// Every level-2 sibling list (the children of an edge (r, v1)) is a subset
// of out(r).  So the count pass over the out-list of root r records, for
// each of r's level-1 entries i, its children as a bitmask over the
// positions of out(r) (row i of r's mask block) together with their number.
// The write pass emits the level-2 structure of arrays from the masks:
// idx = parent entry and pos = the new vertex's position in out(r), which
// names the vertex (out(r)[pos]) and memoizes where its own row is, so no
// vid column is stored.  The fused last level then counts, for
// every level-2 entry (r, v1, w) at positions i1, j, the common later
// neighbours of r, v1 and w as popcount(row i1 AND row j): bits of row j are
// positions above j, so every 4-clique is counted once.

constexpr int BM_MAXD = 768;             // roots with out-degree up to this use masks
constexpr int BM_W = BM_MAXD / 64;       // 64-bit words per mask row
constexpr int BM_UNROLL = 4;             // out-list elements per lane per step (double-buffered)

// Level-1 entry e = (r, S[i]) is described by one word: the first mask word
// of r's block, i, and the row width W (words):  base << 14 | i << 4 | W.
__host__ __device__ constexpr uint64_t row_info(uint64_t base, int i, int W) {
    return (base << 14) | ((uint64_t)i << 4) | (uint64_t)W;
}
__device__ __forceinline__ int info_w(uint64_t info) { return (int)(info & 15); }
__device__ __forceinline__ int info_i(uint64_t info) { return (int)((info >> 4) & 1023); }
__device__ __forceinline__ uint64_t info_base(uint64_t info) { return info >> 14; }

constexpr int BM_CHUNK = 8;              // most count-pass items a wave takes at once
constexpr int64_t BM_SMALL_E = int64_t(1) << 20;   // DAG edges below which count-pass items are short
constexpr int BM_SMALL_ROUND = 16;                 // their level-1 entries per item

struct BmLds {
    int32_t S[CQ_WAVES][BM_MAXD];
    unsigned long long row[CQ_WAVES][BM_W];
    uint4 item[CQ_WAVES][BM_CHUNK];      // b, d | round << 16, mask base (low, high)
};

// Search of NK <= BM_UNROLL keys in S[x+1, d), x and d wave-uniform and
// LG = floor(log2(len)), len = d - x - 1 >= 1: for each key u the last
// element P of S[x, d) with P = S + x or *P <= u.  With m = 2^LG, one probe
// at x + m decides whether the answer lies among the first m positions or
// the last m; strides m/2 .. 1 finish it (Shar's method).  Every probe stays
// inside S[x+1, d); all strides are immediates (LDS offsets) and the chain
// is straight-line code, so a step costs one add, compare and select.
template <int LG, int NK>
__device__ __forceinline__ void bs_find(const int32_t* S, int32_t x, int32_t d, const int32_t* (&P)[BM_UNROLL],
                                        const int32_t (&u)[BM_UNROLL]) {
    constexpr int32_t m = 1 << LG;
    const int32_t pivot = S[x + m];
#pragma unroll
    for (int q = 0; q < NK; ++q) P[q] = (pivot <= u[q]) ? S + (d - m) : S + x;
#pragma unroll
    for (int st = m / 2; st >= 1; st >>= 1)
#pragma unroll
        for (int q = 0; q < NK; ++q) P[q] = (P[q][st] <= u[q]) ? P[q] + st : P[q];
}

// Looks up keys u[0, NK) in S[x+1, d) (LG as for bs_find); hits set bits of
// the LDS row.  Returns the number of hits (wave-uniform).  No key equals
// S[x], so a search ending at S + x is a miss.
template <int LG, int NK>
__device__ __forceinline__ uint32_t search_keys(const int32_t* S, int32_t x, int32_t d,
                                                const int32_t (&u)[BM_UNROLL], unsigned long long* row) {
    const int32_t* P[BM_UNROLL];
    bs_find<LG, NK>(S, x, d, P, u);
    uint32_t c = 0;
#pragma unroll
    for (int q = 0; q < NK; ++q) {
        const bool f = *P[q] == u[q];
        c += (uint32_t)popc64(ballot(f));
        if (f) {
            // byte offset in S: LDS addresses are 32-bit
            const uint32_t off = (uint32_t)(reinterpret_cast<uintptr_t>(P[q]) - reinterpret_cast<uintptr_t>(S));
            atomicOr(&row[off >> 8], 1ull << ((off >> 2) & 63));
        }
    }
    return c;
}

struct BmArgs {
    XcdQueue Q;                 // over items[]: (root, round of `round` level-1 entries), highest ranks first
    const uint64_t* items;
    const int64_t* rp;          // DAG
    const int32_t* col;
    const uint64_t* moff;       // first mask word of each root
    uint64_t* M;                // mask rows
    uint32_t* count;            // children of each level-1 entry
    uint64_t* info;             // row_info of each level-1 entry
    unsigned long long* stats;  // [3] += out-list entries streamed
    int round;                  // level-1 entries per item (64 or 16)
};

// count pass: a work item is one round of 64 level-1 entries of a root r
// (16 on graphs of fewer than 2^20 DAG edges), so no wave holds a heavy
// root for long, with out(r) staged in LDS.  The
// wave walks the round's entries in order; for entry i (vertex v = S[i]) all 64 lanes
// stream out(v) together, BM_UNROLL coalesced loads per lane in flight,
// and look each candidate up in S[i+1, d) with a branch-free binary search
// whose trip count is the same for every lane.  Hits set bits of row i in
// LDS; the finished row goes to HBM and its popcount is i's child count.
// The stream stops once it passes the root's last out-neighbour.
// Streams out(v) of level-1 entry x (n_cand > 0 elements from cp) against
// S[x+1, d): BM_UNROLL loads per lane per step, double-buffered (the next
// step's loads fly during this step's search, the two buffers alternate),
// hits set bits of the LDS row.  Stops once the list passes s_last.
// Returns the number of hits (wave-uniform).
//
// A step is read through a buffer descriptor over its valid elements: the
// address arithmetic is scalar, and lanes past the end read 0, which is
// never in S (out(r) holds ranks above r, so its elements are at least 1).
// Every step issues its loads (after the final step they repeat its first
// element), so the number of loads in flight is known at compile time and
// the search waits for its own step's data only.

template <int LG>
__device__ __forceinline__ uint32_t stream_entry(const int32_t* cp, int64_t left, const int32_t* S, int32_t x,
                                                 int32_t d, int32_t s_last, unsigned long long* row,
                                                 uint64_t& streamed) {
    constexpr int STEP = WAVE * BM_UNROLL;
    uint32_t c = 0;
    int32_t ua[BM_UNROLL], ub[BM_UNROLL];
    int32_t la = 0, lb = 0;   // valid elements of each buffer (wave-uniform)
    // lim >= 1 elements valid from p
    auto load = [&](int32_t (&u)[BM_UNROLL], const int32_t* p, int32_t lim) {
        const __amdgpu_buffer_rsrc_t rs =
            __builtin_amdgcn_make_buffer_rsrc(const_cast<int32_t*>(p), (short)0, lim * 4, BUF_WORD3);
#pragma unroll
        for (int q = 0; q < BM_UNROLL; ++q)
            u[q] = __builtin_amdgcn_raw_buffer_load_b32(rs, (q * WAVE + lane()) * 4, 0, 0);
    };
    // A step is sorted: once the first key of a row of 64 exceeds s_last
    // (or the row is past the list), no key of it or of a later row hits.
    static_assert(BM_UNROLL == 4, "the row cases below are written out for four rows");
    auto search = [&](const int32_t (&u)[BM_UNROLL], int32_t lim) {
        auto live = [&](int q) { return q * WAVE < lim && readlane(u[q], 0) <= s_last; };
        if (live(3)) c += search_keys<LG, 4>(S, x, d, u, row);
        else if (live(2)) c += search_keys<LG, 3>(S, x, d, u, row);
        else if (live(1)) c += search_keys<LG, 2>(S, x, d, u, row);
        else if (live(0)) c += search_keys<LG, 1>(S, x, d, u, row);
    };
    // the next step's loads: of cp + STEP if there is one, else of cp again
    auto next = [&](int32_t (&u)[BM_UNROLL], int32_t& lim, bool more) {
        lim = more ? (int32_t)min64(left - STEP, STEP) : 1;
        load(u, more ? cp + STEP : cp, lim);
    };
    la = (int32_t)min64(left, STEP);
    load(ua, cp, la);
    while (true) {
        // ua holds the current step; ub gets the next one
        bool more = left > STEP && readlane(ua[BM_UNROLL - 1], WAVE - 1) <= s_last;
        next(ub, lb, more);
        search(ua, la);
        streamed += (uint64_t)min64(left, STEP);
        if (!more) break;
        cp += STEP;
        left -= STEP;
        // ub holds the current step; ua gets the next one
        more = left > STEP && readlane(ub[BM_UNROLL - 1], WAVE - 1) <= s_last;
        next(ua, la, more);
        search(ub, lb);
        streamed += (uint64_t)min64(left, STEP);
        if (!more) break;
        cp += STEP;
        left -= STEP;
    }
    return c;
}

__global__ __launch_bounds__(CQ_THREADS, 7) void k_clique_count_masks(BmArgs A) {
    __shared__ BmLds L;
    const int w = threadIdx.x / WAVE;
    int32_t* S = L.S[w];
    unsigned long long* row = L.row[w];
    if (lane() < BM_W) row[lane()] = 0ull;   // every entry leaves it zero again
    uint64_t streamed = 0;   // wave-uniform
    QueueCursor cur = queue_start();
    int64_t it_end = 0;
    for (int64_t it = queue_next(A.Q, cur, it_end); it >= 0; it = queue_next(A.Q, cur, it_end)) {
        // the chunk's item descriptors, loaded side by side (one item per
        // lane) and kept in LDS.  The DAG has at most 2^31 - 1 edges and
        // out-degrees of at most BM_MAXD here, so b fits 32 bits and d and
        // the round share a word.
        const int nj = (int)(it_end - it);   // <= BM_CHUNK
        wave_sync();                         // the previous chunk's reads are done
        if (lane() < nj) {
            const uint64_t item = A.items[A.Q.n_items - 1 - (it + lane())];
            const int64_t r = item_seg(item);
            const int64_t b0 = A.rp[r];
            const uint64_t mb = A.moff[r];
            L.item[w][lane()] = make_uint4((uint32_t)b0,
                                           (uint32_t)(A.rp[r + 1] - b0) | ((uint32_t)item_round(item) << 16),
                                           (uint32_t)mb, (uint32_t)(mb >> 32));
        }
        wave_sync();
        for (int jj = 0; jj < nj; ++jj) {
            // everything per item and per entry is wave-uniform: keep it scalar
            const uint4 desc = L.item[w][jj];
            const int64_t b = uniform((int32_t)desc.x);
            const int32_t dr = uniform((int32_t)desc.y);
            const int32_t d = dr & 0xffff;
            if (d < 2) continue;   // counts are pre-zeroed; rows and infos are never read
            const int W = (d + 63) >> 6;
            const int32_t xc = (dr >> 16) * A.round;
            const int nx = min(A.round, d - xc);
            // out-list bounds of the round's entries, one per lane; the
            // entry's vertex comes from HBM, so these loads fly with the staging
            const int32_t xl = xc + lane();
            int64_t lo = 0;
            int32_t nl = 0;   // out-degree (the DAG has fewer than 2^31 edges)
            if (lane() < nx && xl < d - 1) {
                const int32_t v = A.col[b + xl];
                lo = A.rp[v];
                nl = (int32_t)(A.rp[v + 1] - lo);
            }
            wave_sync();           // the previous item's reads of S are done
            for (int k = lane(); k < d; k += WAVE) S[k] = A.col[b + k];
            wave_sync();
            const int32_t s_last = uniform(S[d - 1]);
            const uint64_t base = ((uint64_t)(uint32_t)uniform((int32_t)desc.w) << 32) | (uint32_t)uniform((int32_t)desc.z);
            uint64_t* Mr = A.M + base;
            uint32_t mine = 0;
            for (int xi = 0; xi < nx; ++xi) {
                const int32_t x = xc + xi;
                const int64_t l = (int64_t)readlane64((uint64_t)lo, xi);
                const int64_t n_cand = readlane(nl, xi);
                uint32_t c = 0;   // hits = children of x (wave-uniform)
                // the row is all zero here; with no candidates it stays so
                if (n_cand <= 0) {
                    if (lane() < W) Mr[(uint64_t)x * W + lane()] = 0ull;
                    continue;
                }
                // n_cand > 0 only when x < d - 1, so S[x+1, d) is non-empty
                static_assert(BM_MAXD <= 1024, "depths below cover len < 1024");
                const int lg = 31 - __clz(d - x - 1);
                switch (lg) {
                    case 0: c = stream_entry<0>(A.col + l, n_cand, S, x, d, s_last, row, streamed); break;
                    case 1: c = stream_entry<1>(A.col + l, n_cand, S, x, d, s_last, row, streamed); break;
                    case 2: c = stream_entry<2>(A.col + l, n_cand, S, x, d, s_last, row, streamed); break;
                    case 3: c = stream_entry<3>(A.col + l, n_cand, S, x, d, s_last, row, streamed); break;
                    case 4: c = stream_entry<4>(A.col + l, n_cand, S, x, d, s_last, row, streamed); break;
                    case 5: c = stream_entry<5>(A.col + l, n_cand, S, x, d, s_last, row, streamed); break;
                    case 6: c = stream_entry<6>(A.col + l, n_cand, S, x, d, s_last, row, streamed); break;
                    case 7: c = stream_entry<7>(A.col + l, n_cand, S, x, d, s_last, row, streamed); break;
                    case 8: c = stream_entry<8>(A.col + l, n_cand, S, x, d, s_last, row, streamed); break;
                    default: c = stream_entry<9>(A.col + l, n_cand, S, x, d, s_last, row, streamed); break;
                }
                wave_sync();      // every lane's hits are in the row
                if (lane() < W) {
                    Mr[(uint64_t)x * W + lane()] = row[lane()];
                    row[lane()] = 0ull;
                }
                if (lane() == xi) mine = c;
                wave_sync();      // cleared before the next entry's hits
            }
            if (lane() < nx) {
                A.count[b + xl] = mine;
                A.info[b + xl] = row_info(base, xl, W);
            }
        }
    }
    if (lane() == 0 && streamed) atomicAdd(&A.stats[3], (unsigned long long)streamed);
}

// write pass: a wave takes 64 consecutive level-1 entries (one per lane,
// which loads its row), then, entry by entry, compacts the set bits of the
// row a word at a time with a ballot (lane j handles bit j; words that are
// zero, such as all those below the entry's own position, are skipped with a
// scalar branch).  The children of the wave's entries fill one contiguous
// output range, so they gather in a buffer in LDS and leave in full 64-lane
// coalesced stores.  A level-2 entry is (parent level-1 entry, position in
// the root's out-list); its vertex is the root's out-neighbour at that
// position.
constexpr int WR_THREADS = 256;

__global__ __launch_bounds__(WR_THREADS) void k_clique_write_masks(int64_t e_lo, int64_t e_hi,
                                                                   const uint64_t* __restrict__ info,
                                                                   const uint64_t* __restrict__ M,
                                                                   const uint64_t* __restrict__ start,
                                                                   uint64_t start_base,
                                                                   int32_t* __restrict__ out_idx,
                                                                   uint16_t* __restrict__ out_pos,
                                                                   unsigned long long* __restrict__ stats) {
    // fill < 64 before a word adds at most 64 children
    __shared__ int32_t buf_idx[WR_THREADS / WAVE][2 * WAVE];
    __shared__ uint16_t buf_pos[WR_THREADS / WAVE][2 * WAVE];
    int32_t* bi = buf_idx[threadIdx.x / WAVE];
    uint16_t* bp = buf_pos[threadIdx.x / WAVE];
    uint64_t read = 0;   // info and row bytes of the entries with children
    const int64_t n_waves = (int64_t)gridDim.x * (blockDim.x / WAVE);
    const int64_t wave_id = (int64_t)blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE;
    // A batch's starts and row infos are loaded together (lanes past e_hi
    // load the last entry's and drop them), one batch ahead: the next
    // batch's loads fly while this one is compacted.
    const int64_t stride = n_waves * WAVE;
    uint64_t ns0 = 0, ns1 = 0, nf = 0;
    auto meta = [&](int64_t b0) {
        const int64_t e = b0 + lane();
        const int64_t ec = e < e_hi ? e : e_hi - 1;
        ns0 = start[ec];
        ns1 = start[ec + 1];
        nf = info[ec];
        if (e >= e_hi) ns1 = ns0;
    };
    int64_t e0 = e_lo + wave_id * WAVE;
    if (e0 < e_hi) meta(e0);
    for (; e0 < e_hi; e0 += stride) {
        const uint64_t s0 = ns0 - start_base, s1 = ns1 - start_base;
        const uint64_t fcur = nf;
        const bool has = s1 > s0;
        int Wl = 0;
        uint64_t words[BM_W];
        {
            const uint64_t f = has ? fcur : 0;
            Wl = info_w(f);
            const uint64_t* rowp = M + info_base(f) + (uint64_t)info_i(f) * Wl;
            // in 16-byte pairs (half the scattered load instructions)
            static_assert(BM_W % 2 == 0, "rows are read in word pairs");
#pragma unroll
            for (int q = 0; q < BM_W; q += 2) {
                if (q + 1 < Wl) {
                    const ulonglong2 pr = *reinterpret_cast<const ulonglong2*>(rowp + q);
                    words[q] = pr.x;
                    words[q + 1] = pr.y;
                } else {
                    words[q] = q < Wl ? rowp[q] : 0ull;
                    words[q + 1] = 0ull;
                }
            }
            if (has) read += 8u + 8u * (uint64_t)Wl;
        }
        meta(e0 + stride < e_hi ? e0 + stride : e0);
        // lane 0's entry e0 < e_hi opens the wave's output range
        uint64_t out_at = readlane64(s0, 0);
        int fill = 0;   // children in the buffer (wave-uniform)
        // the words of entry li's row, for a row of NW words (unrolled)
        auto emit = [&](auto nw, int li, int32_t parent) {
            constexpr int NW = decltype(nw)::value;
#pragma unroll
            for (int q = 0; q < NW; ++q) {
                const uint64_t wq = readlane64(words[q], li);
                if (wq == 0) continue;
                if ((wq >> lane()) & 1ull) {
                    const int slot = fill + __popcll(wq & lanemask_lt());
                    bi[slot] = parent;
                    bp[slot] = (uint16_t)(q * 64 + lane());
                }
                fill += __popcll(wq);
                if (fill >= WAVE) {
                    wave_sync();
                    out_idx[out_at + lane()] = bi[lane()];
                    out_pos[out_at + lane()] = bp[lane()];
                    const int32_t ti = bi[WAVE + lane()];
                    const uint16_t tp = bp[WAVE + lane()];
                    wave_sync();
                    bi[lane()] = ti;
                    bp[lane()] = tp;
                    fill -= WAVE;
                    out_at += WAVE;
                }
            }
        };
        static_assert(BM_W == 12, "the row widths below run to 12 words");
        uint64_t todo = ballot(has);
        while (todo) {
            const int li = __ffsll((unsigned long long)todo) - 1;
            todo &= todo - 1;
            const int32_t parent = (int32_t)(e0 + li);
            switch (readlane(Wl, li)) {
                case 1: emit(std::integral_constant<int, 1>{}, li, parent); break;
                case 2: emit(std::integral_constant<int, 2>{}, li, parent); break;
                case 3: emit(std::integral_constant<int, 3>{}, li, parent); break;
                case 4: emit(std::integral_constant<int, 4>{}, li, parent); break;
                case 5: emit(std::integral_constant<int, 5>{}, li, parent); break;
                case 6: emit(std::integral_constant<int, 6>{}, li, parent); break;
                case 7: emit(std::integral_constant<int, 7>{}, li, parent); break;
                case 8: emit(std::integral_constant<int, 8>{}, li, parent); break;
                case 9: emit(std::integral_constant<int, 9>{}, li, parent); break;
                case 10: emit(std::integral_constant<int, 10>{}, li, parent); break;
                case 11: emit(std::integral_constant<int, 11>{}, li, parent); break;
                default: emit(std::integral_constant<int, 12>{}, li, parent); break;
            }
        }
        wave_sync();
        if (lane() < fill) {
            out_idx[out_at + lane()] = bi[lane()];
            out_pos[out_at + lane()] = bp[lane()];
        }
        wave_sync();   // the buffer is refilled by the next batch
    }
    read = wave_sum_u64(read);
    if (lane() == 0 && read) atomicAdd(&stats[4], (unsigned long long)read);
}

// fused last level: a level-2 entry (r, S[i], S[j]), i < j, extends to the
// 4-cliques given by the set bits of row i AND row j (row j only has bits
// above j, so each is counted once); a thread takes one entry at a time.
// The mask rows are read from LDS.  The mask blocks of consecutive roots are
// consecutive in M, so a run of roots (a window) is one word range of M.  A root whose block has LW_BIG words or more is a
// window of its own; the others are grouped while their blocks start in the
// same LW_SPAN-word stretch of M.  A window then spans fewer than
// LW_SPAN + LW_BIG words, or one block (at most BM_MAXD * BM_W words).  A
// work item is a round of at most LW_PER of a window's level-2 entries
// (those of the current chunk of level-1 entries); a workgroup stages the
// window's words in LDS, in 16-byte pieces, and counts its entries from
// there.  Items are taken from a counter, one workgroup at a time.
constexpr int LW_THREADS = 512;
constexpr int LW_BIG = 3072;
constexpr int LW_SPAN = 6144;
constexpr int LW_CAP = BM_MAXD * BM_W + 2;   // +1 word when the range starts at an odd word, even
constexpr int LW_PER = 1 << 15;
static_assert(LW_SPAN + LW_BIG <= BM_MAXD * BM_W, "a window of small roots fits the LDS buffer");

// window starts: mark[r] = 1 if root r opens a window
__global__ void k_last_marks(int64_t n, const uint64_t* __restrict__ moff, uint32_t* __restrict__ mark) {
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t m0 = moff[r];
        bool st = r == 0 || moff[r + 1] - m0 >= (uint64_t)LW_BIG;
        if (!st) {
            const uint64_t pm = moff[r - 1];
            st = m0 - pm >= (uint64_t)LW_BIG || m0 / LW_SPAN != pm / LW_SPAN;
        }
        mark[r] = st ? 1u : 0u;
    }
}

// first root of each window (woff = exclusive scan of mark); first[nw] = n
__global__ void k_last_first(int64_t n, const uint32_t* __restrict__ mark, const uint64_t* __restrict__ woff,
                             int64_t* __restrict__ first) {
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
        if (mark[r]) first[woff[r]] = r;
        if (r == n - 1) first[woff[n]] = n;
    }
}

// level-2 entries of each window within the chunk of level-1 entries
// [c0, c1): seg[w] .. seg[w + 1], counted from the chunk's first entry
__global__ void k_last_segs(int64_t nw, const int64_t* __restrict__ first, const int64_t* __restrict__ rp,
                            const uint64_t* __restrict__ start, int64_t c0, int64_t c1, uint64_t* __restrict__ seg) {
    for (int64_t w = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; w <= nw; w += (int64_t)gridDim.x * blockDim.x) {
        const int64_t e = min64(max64(rp[first[w]], c0), c1);
        seg[w] = start[e] - start[c0];
    }
}

// Entries e0 + threadIdx.x, ... < e1 (e0 < e1), LW_B at a time per thread:
// their loads are clamped into [e0, e1) and issued together, so a thread
// waits for one round trip per LW_B entries.
constexpr int LW_B = 16;

template <bool LDS>
__device__ __forceinline__ void last_count(const uint64_t* base, uint64_t m_al, uint64_t e0, uint64_t e1,
                                           const int32_t* __restrict__ idx, const uint16_t* __restrict__ pos,
                                           const uint64_t* __restrict__ info, uint64_t& found, uint64_t& words) {
    for (uint64_t x0 = e0 + threadIdx.x; x0 < e1; x0 += LW_B * LW_THREADS) {
        int32_t p[LW_B];
        int j[LW_B];
#pragma unroll
        for (int u = 0; u < LW_B; ++u) {
            const uint64_t x = x0 + (uint64_t)u * LW_THREADS;
            const uint64_t xc = x < e1 ? x : e1 - 1;
            p[u] = idx[xc];
            j[u] = pos[xc];
        }
        uint64_t f[LW_B];
#pragma unroll
        for (int u = 0; u < LW_B; ++u) f[u] = info[p[u]];
#pragma unroll
        for (int u = 0; u < LW_B; ++u) {
            if (x0 + (uint64_t)u * LW_THREADS >= e1) break;
            const int W = info_w(f[u]);
            const uint64_t* blk = base + (info_base(f[u]) - m_al);
            const uint64_t* r1 = blk + (uint64_t)info_i(f[u]) * W;
            const uint64_t* r2 = blk + (uint64_t)j[u] * W;
            for (int q = j[u] >> 6; q < W; ++q) found += (uint64_t)__popcll(r1[q] & r2[q]);
            words += (uint64_t)(W - (j[u] >> 6));
        }
    }
}

__global__ __launch_bounds__(LW_THREADS) void k_clique_last_lds(const uint64_t* __restrict__ items,
                                                                const unsigned long long* __restrict__ n_items_dev,
                                                                const uint64_t* __restrict__ seg,
                                                                const int64_t* __restrict__ first,
                                                                const uint64_t* __restrict__ moff,
                                                                const int32_t* __restrict__ idx,
                                                                const uint16_t* __restrict__ pos,
                                                                const uint64_t* __restrict__ info,
                                                                const uint64_t* __restrict__ M,
                                                                unsigned long long* __restrict__ next,
                                                                unsigned long long* __restrict__ stats) {
    __shared__ __align__(16) uint64_t R[LW_CAP];
    __shared__ int64_t s_item;
    const int64_t n_items = (int64_t)*n_items_dev;
    uint64_t found = 0, words = 0;
    while (true) {
        // every thread is done with the previous item's words here
        if (threadIdx.x == 0) s_item = (int64_t)atomicAdd(next, 1ull);
        __syncthreads();
        const int64_t it = s_item;
        if (it >= n_items) break;
        const uint64_t item = items[it];
        const int64_t w = item_seg(item);
        const uint64_t e0 = seg[w] + item_round(item) * (uint64_t)LW_PER;
        const uint64_t e1 = e0 + LW_PER < seg[w + 1] ? e0 + LW_PER : seg[w + 1];
        const uint64_t m_al = moff[first[w]] & ~1ull;   // M is 16-byte aligned
        const uint64_t span = moff[first[w + 1]] - m_al;
        if (span <= (uint64_t)LW_CAP) {
            const int64_t np = (int64_t)(span / 2);
            const ulonglong2* src = reinterpret_cast<const ulonglong2*>(M + m_al);
            ulonglong2* dst = reinterpret_cast<ulonglong2*>(R);
            // three 16-byte loads in flight per thread
            for (int64_t k = threadIdx.x; k < np; k += 3 * LW_THREADS) {
                const int64_t kb = k + LW_THREADS, kc = k + 2 * LW_THREADS;
                const ulonglong2 va = src[k];
                const ulonglong2 vb = kb < np ? src[kb] : va;
                const ulonglong2 vc = kc < np ? src[kc] : va;
                dst[k] = va;
                if (kb < np) dst[kb] = vb;
                if (kc < np) dst[kc] = vc;
            }
            if ((span & 1) && threadIdx.x == 0) R[span - 1] = M[m_al + span - 1];
            __syncthreads();
            last_count<true>(R, m_al, e0, e1, idx, pos, info, found, words);
        } else {
            // not reached for blocks laid out as above; kept for safety
            last_count<false>(M + m_al, m_al, e0, e1, idx, pos, info, found, words);
        }
    }
    found = wave_sum_u64(found);
    words = wave_sum_u64(words);
    if (lane() == 0 && (found | words)) {
        atomicAdd(&stats[0], (unsigned long long)found);
        atomicAdd(&stats[2], (unsigned long long)words);
    }
}

// Deeper levels with masks (k >= 5).  An entry's children are the positions
// set in the AND of the mask rows of all its vertices after the root; for a
// parent segment that AND is shared, so a child only adds its own row.
struct MaskChain {
    const int32_t* idx[PG_KMAX + 1];    // level l >= 2: parent index (level 2: level-1 entry)
    const uint16_t* pos[PG_KMAX + 1];   // level l >= 2: position in the root's out-list
};

struct MaskArgs {
    XcdQueue Q;                  // over parents: a parent has at most BM_MAXD children
    int64_t p_lo;                // parents (level lev-1 entries)
    const uint64_t* seg;         // COUNT, WRITE: children of parent p: seg[p] - seg_base .. seg[p+1] - seg_base
    uint64_t seg_base;
    int lev;                     // level of the children
    MaskChain ch;
    int64_t x_lo, x_hi;          // children extended (WRITE chunks)
    const uint64_t* info;        // row_info of each level-1 entry
    const uint64_t* M;
    uint32_t* count;             // COUNT: per child
    const uint64_t* start;       // WRITE: grandchildren of child x at start[x] - start_base
    uint64_t start_base;
    int32_t* out_idx;
    uint16_t* out_pos;
    unsigned long long* stats;
};

__device__ __forceinline__ int32_t lanes_below(uint64_t m) {
    return (int32_t)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// COUNT and WRITE take a parent's children from the stored level `lev`.
// LAST never stores that level: a parent's children are the positions set
// in its set (every position in it extends the parent to a clique of the
// level), packed into LDS with ballots, and each adds the popcount of its
// row AND the set, which counts its own children (the k-cliques).
template <int MODE>
__global__ __launch_bounds__(CQ_THREADS, MODE == MODE_LAST ? 6 : 1) void k_clique_mask_level(MaskArgs A) {
    __shared__ uint16_t kids[MODE == MODE_LAST ? CQ_WAVES : 1][MODE == MODE_LAST ? BM_MAXD : 1];
    uint64_t acc = 0;
    // LAST: parents with children, words of their sets, children, and row
    // words read (each child reads the words of the pairs where its
    // parent's set is non-empty)
    uint32_t lw_par = 0, lw_set = 0, lw_ent = 0;
    uint64_t lw_row = 0;
    QueueCursor cur = queue_start();
    int64_t it_end = 0;
    for (int64_t it = queue_next(A.Q, cur, it_end); it >= 0; it = queue_next(A.Q, cur, it_end)) {
        // set-up of up to 64 parents side by side: lane l walks the ancestry
        // of parent it + l and forms its set S (the AND of the rows of its
        // vertices after the root), word q in sp[q]
        const int64_t p = A.p_lo + it + lane();
        int64_t px0 = 0, px1 = 0;
        int Wl = 0;
        uint64_t bl = 0;
        uint64_t sp[BM_W];
#pragma unroll
        for (int q = 0; q < BM_W; ++q) sp[q] = 0ull;
        if (it + lane() < it_end) {
            if constexpr (MODE == MODE_LAST) {
                px1 = 1;   // decided by the set below
            } else {
                const int64_t b = (int64_t)(A.seg[p] - A.seg_base);
                const int64_t e2 = (int64_t)(A.seg[p + 1] - A.seg_base);
                // the parent's children within the launch's window [x_lo, x_hi)
                px0 = max64(b, A.x_lo);
                px1 = min64(e2, A.x_hi);
            }
            if (px0 < px1) {
                int32_t apos[PG_KMAX];
                int na = 0;
                int64_t c = p;
                for (int l = A.lev - 1; l >= 2; --l) {
                    apos[na++] = A.ch.pos[l][c];
                    c = A.ch.idx[l][c];
                }
                const uint64_t f = A.info[c];         // c: the level-1 entry
                Wl = info_w(f);
                bl = info_base(f);
                const uint64_t* blk = A.M + bl;
                // a row at a time, its words loaded together
                const uint64_t* ri = blk + (uint64_t)info_i(f) * Wl;
#pragma unroll
                for (int q = 0; q < BM_W; ++q)
                    if (q < Wl) sp[q] = ri[q];
                for (int a2 = 0; a2 < na; ++a2) {
                    const uint64_t* ra = blk + (uint64_t)apos[a2] * Wl;
#pragma unroll
                    for (int q = 0; q < BM_W; ++q)
                        if (q < Wl) sp[q] &= ra[q];
                }
                if constexpr (MODE == MODE_LAST) {
                    uint32_t nch = 0, nzw = 0;
#pragma unroll
                    for (int q = 0; q < BM_W; q += 2) {
                        const uint64_t s0 = q < Wl ? sp[q] : 0ull, s1 = q + 1 < Wl ? sp[q + 1] : 0ull;
                        nch += (uint32_t)(__popcll(s0) + __popcll(s1));
                        nzw += ((s0 | s1) != 0ull) ? ((q + 1 < Wl) ? 2u : 1u) : 0u;
                    }
                    if (nch == 0) px1 = 0;
                    else {
                        lw_par += 1;
                        lw_set += (uint32_t)Wl * (uint32_t)(A.lev - 1);   // the parent's rows
                        lw_ent += nch;
                        lw_row += (uint64_t)nch * nzw;
                    }
                }
            }
        }
        uint64_t todo_p = ballot(px0 < px1);
        while (todo_p) {
            const int pi = __ffsll((unsigned long long)todo_p) - 1;
            todo_p &= todo_p - 1;
            const int W = readlane(Wl, pi);
            const uint64_t* blk = A.M + readlane64(bl, pi);
            uint64_t s[BM_W];
            // the words below W, a pair at a time (the others are zero)
#pragma unroll
            for (int q = 0; q < BM_W; q += 2) {
                s[q] = s[q + 1] = 0ull;
                if (q < W) {
                    s[q] = readlane64(sp[q], pi);
                    s[q + 1] = readlane64(sp[q + 1], pi);
                }
            }
            int64_t x0 = 0, x1 = 0;
            uint32_t acc_p = 0;   // LAST: this parent's count in this lane (at most 12 rounds of 768)
            // pairs of words where the parent's set is non-empty, one bit each
            uint32_t nzp = 0;
#pragma unroll
            for (int q = 0; q < BM_W; q += 2) nzp |= ((s[q] | s[q + 1]) != 0ull) ? (1u << (q / 2)) : 0u;
            uint16_t* kl = kids[MODE == MODE_LAST ? threadIdx.x / WAVE : 0];
            if constexpr (MODE == MODE_LAST) {
                // the set's positions, in order
                int32_t n = 0;
#pragma unroll
                for (int q = 0; q < BM_W; ++q) {
                    if (s[q] != 0ull) {
                        if ((s[q] >> lane()) & 1ull) kl[n + lanes_below(s[q])] = (uint16_t)(q * 64 + lane());
                        n += popc64(s[q]);
                    }
                }
                wave_sync();
                x1 = n;
            } else {
                x0 = (int64_t)readlane64((uint64_t)px0, pi);
                x1 = (int64_t)readlane64((uint64_t)px1, pi);
            }
            for (int64_t xb = x0; xb < x1; xb += WAVE) {
                const int64_t x = xb + lane();
                const bool valid = x < x1;
                // idle lanes take the last entry's row and drop the result,
                // so the loads below need no per-lane branches
                const int64_t xs = valid ? x : x1 - 1;
                int32_t px = 0;
                if constexpr (MODE == MODE_LAST) px = (int32_t)kl[xs];
                else px = A.ch.pos[A.lev][xs];
                const uint64_t* row = blk + (uint64_t)px * W;
                // only the pairs of words where the parent's set is non-empty
                // (a wave-uniform test) are read, 16 bytes each and all in
                // flight together (the word after an odd-width row's last is
                // M's next word or its padding, and its set word is zero)
                ulonglong2 pr[BM_W / 2];
#pragma unroll
                for (int q = 0; q < BM_W; q += 2) {
                    pr[q / 2] = make_ulonglong2(0ull, 0ull);
                    if ((nzp >> (q / 2)) & 1u) pr[q / 2] = *reinterpret_cast<const ulonglong2*>(row + q);
                }
                uint64_t words[MODE == MODE_WRITE ? BM_W : 1];
                uint32_t cnt = 0;
#pragma unroll
                for (int q = 0; q < BM_W; q += 2) {
                    uint64_t w0 = 0ull, w1 = 0ull;
                    if ((nzp >> (q / 2)) & 1u) {   // the same uniform test as the loads
                        w0 = s[q] & pr[q / 2].x;
                        w1 = s[q + 1] & pr[q / 2].y;
                        cnt += (uint32_t)(__popcll(w0) + __popcll(w1));
                    }
                    if constexpr (MODE == MODE_WRITE) {
                        words[q] = w0;
                        words[q + 1] = w1;
                    }
                }
                if (!valid) cnt = 0;
                if (MODE == MODE_COUNT && valid) A.count[x] = cnt;
                if (MODE == MODE_LAST) acc_p += cnt;
                if (MODE == MODE_WRITE) {
                    // children of the wave's entries, entry by entry, each
                    // word compacted by a ballot (coalesced stores)
                    const uint64_t s0 = valid ? A.start[x] - A.start_base : 0;
                    uint64_t todo = ballot(cnt != 0);
                    while (todo) {
                        const int li = __ffsll((unsigned long long)todo) - 1;
                        todo &= todo - 1;
                        uint64_t o = readlane64(s0, li);
                        const int32_t parent = (int32_t)(xb + li);
#pragma unroll
                        for (int q = 0; q < BM_W; ++q) {
                            if (q < W) {
                                const uint64_t wq = readlane64(words[q], li);
                                if ((wq >> lane()) & 1ull) {
                                    const uint64_t slot = o + (uint64_t)__popcll(wq & lanemask_lt());
                                    A.out_idx[slot] = parent;
                                    A.out_pos[slot] = (uint16_t)(q * 64 + lane());
                                }
                                o += (uint64_t)__popcll(wq);
                            }
                        }
                    }
                }
            }
            if constexpr (MODE == MODE_LAST) {
                acc += acc_p;
                wave_sync();   // the list is read before the next parent's
            }
        }
    }
    if (MODE == MODE_LAST) {
        acc = wave_sum_u64(acc);
        if (lane() == 0 && acc) atomicAdd(&A.stats[0], (unsigned long long)acc);
        const uint64_t t_par = wave_sum_u64(lw_par), t_set = wave_sum_u64(lw_set);
        const uint64_t t_ent = wave_sum_u64(lw_ent), t_row = wave_sum_u64(lw_row);
        if (lane() == 0 && t_par) {
            atomicAdd(&A.stats[8], (unsigned long long)t_par);
            atomicAdd(&A.stats[9], (unsigned long long)t_set);
            atomicAdd(&A.stats[10], (unsigned long long)t_ent);
            atomicAdd(&A.stats[11], (unsigned long long)t_row);
        }
    }
}

// Per root: its mask words and its out-degree split by whether the root is
// light (out-degree at most BM_MAXD: sibling masks) or heavy (the general
// level kernels).
__global__ void k_mask_words(int64_t n, const int64_t* __restrict__ rp, uint32_t* __restrict__ words,
                             uint32_t* __restrict__ light, uint32_t* __restrict__ heavy) {
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
        const int64_t d = rp[r + 1] - rp[r];
        const bool lt = d <= BM_MAXD;
        words[r] = lt ? (uint32_t)(d * ((d + 63) >> 6)) : 0u;
        light[r] = lt ? (uint32_t)d : 0u;
        heavy[r] = lt ? 0u : (uint32_t)d;
    }
}

// The heavy roots' out-lists, packed: hcol[hrp[r] ..) = col[rp[r] ..) when
// root r is heavy (hrp[r + 1] > hrp[r]).  One wave per root.
__global__ void k_heavy_lists(int64_t n, const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                              const uint64_t* __restrict__ hrp, int32_t* __restrict__ hcol) {
    const int64_t n_waves = (int64_t)gridDim.x * (blockDim.x / WAVE);
    for (int64_t r = (int64_t)blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE; r < n; r += n_waves) {
        const int64_t len = (int64_t)(hrp[r + 1] - hrp[r]);
        for (int64_t k = lane(); k < len; k += WAVE) hcol[hrp[r] + k] = col[rp[r] + k];
    }
}

// ------------------------------------------------ heavy roots, k = 3 and 4
//
// Roots of out-degree D above BM_MAXD (up to HM_MAXD) keep their sibling
// rows in device memory: row i of root r is the set of positions j of
// out(r) whose vertex is an out-neighbour of out(r)[i] (all above i), in
// W = ceil(D / 64) words.  The triangles at r are the rows' set bits; its
// 4-cliques are the popcounts of row i AND row j over every set bit j of
// row i (bits of row j lie above j, so each 4-clique is counted once).
constexpr int HM_MAXD = 8192;
constexpr int HM_WMAX = HM_MAXD / 64;    // row words at most (two per lane)
constexpr int HM_THREADS = 256;
constexpr int HM_WAVES = HM_THREADS / WAVE;
constexpr int HM_BLOCK = 64;             // rows per work item

struct HmArgs {
    XcdQueue Q;
    const uint64_t* items;        // (heavy root index, block of HM_BLOCK rows)
    const int32_t* hroot;
    const uint64_t* hoff;
    const int64_t* rp;            // DAG
    const int32_t* col;
    uint64_t* rows;               // row words; NULL: triangles only
    unsigned long long* stats;    // [0] += cliques, [5] += out-list elements streamed, [6] += row pairs
};

// heavy root flags and sizes: out-degree, and row words D * W
__global__ void k_heavy_flags(int64_t n, const int64_t* __restrict__ rp, uint32_t* __restrict__ flag) {
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x)
        flag[r] = (rp[r + 1] - rp[r] > BM_MAXD) ? 1u : 0u;
}

__global__ void k_heavy_fill(int64_t n, const int64_t* __restrict__ rp, const uint64_t* __restrict__ pos,
                             int32_t* __restrict__ hroot, uint32_t* __restrict__ hdeg, uint64_t* __restrict__ hw) {
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x)
        if (pos[r + 1] > pos[r]) {
            const int64_t d = rp[r + 1] - rp[r];
            hroot[pos[r]] = (int32_t)r;
            hdeg[pos[r]] = (uint32_t)d;
            hw[pos[r]] = (uint64_t)d * (uint64_t)((d + 63) >> 6);
        }
}

// Rows: a workgroup stages out(r) in LDS for an item; each wave builds rows
// of the item's block, all lanes streaming out(v) (cut at out(r)'s last
// vertex) and searching each element among out(r)'s later positions.
__global__ __launch_bounds__(HM_THREADS) void k_heavy_rows(HmArgs A) {
    __shared__ int32_t S[HM_MAXD];
    __shared__ unsigned long long row[HM_WAVES][HM_WMAX];
    __shared__ int64_t s_next[2];
    const int w = threadIdx.x / WAVE;
    for (int k = lane(); k < HM_WMAX; k += WAVE) row[w][k] = 0ull;
    uint64_t found = 0, streamed = 0;
    QueueCursor cur = queue_start();
    while (true) {
        __syncthreads();
        if (w == 0) {
            int64_t e = 0;
            const int64_t f = queue_next(A.Q, cur, e);
            if (lane() == 0) {
                s_next[0] = f;
                s_next[1] = e;
            }
        }
        __syncthreads();
        const int64_t first = s_next[0], last = s_next[1];
        if (first < 0) break;
        for (int64_t jt = first; jt < last; ++jt) {
            const uint64_t item = A.items[jt];
            const int64_t h = item_seg(item);
            const int32_t r = A.hroot[h];
            const int64_t b = A.rp[r];
            const int32_t D = (int32_t)(A.rp[r + 1] - b);
            const int32_t W = (D + 63) >> 6;
            __syncthreads();   // the previous item's searches are done
            for (int k = threadIdx.x; k < D; k += HM_THREADS) S[k] = A.col[b + k];
            __syncthreads();
            const int32_t s_last = S[D - 1];
            const int32_t i0 = (int32_t)item_round(item) * HM_BLOCK;
            const int32_t i1 = min(i0 + HM_BLOCK, D);
            uint64_t* R = A.rows ? A.rows + A.hoff[h] : nullptr;
            for (int32_t i = i0 + w; i < i1; i += HM_WAVES) {
                const int32_t v = S[i];
                const int64_t lo = A.rp[v];
                const int64_t hi = upper_bound(A.col, lo, A.rp[v + 1], s_last);
                streamed += (uint64_t)(hi - lo);
                for (int64_t t0 = lo; t0 < hi; t0 += WAVE) {
                    const int64_t t = t0 + lane();
                    if (t < hi) {
                        const int32_t u = A.col[t];
                        const int32_t j = (int32_t)lower_bound(S, (int64_t)i + 1, (int64_t)D, u);
                        if (j < D && S[j] == u) atomicOr(&row[w][j >> 6], 1ull << (j & 63));
                    }
                }
                wave_sync();
                for (int k = lane(); k < W; k += WAVE) {
                    const unsigned long long x = row[w][k];
                    found += (uint64_t)__popcll(x);
                    if (R) R[(int64_t)i * W + k] = x;
                    row[w][k] = 0ull;
                }
                wave_sync();
            }
        }
    }
    found = wave_sum_u64(found);
    if (lane() == 0) {
        if (!A.rows && found) atomicAdd(&A.stats[0], (unsigned long long)found);
        if (streamed) atomicAdd(&A.stats[5], (unsigned long long)streamed);
    }
}

// 4-cliques: a wave takes an item and, row by row, holds row i in
// registers (lane l: words l and l + 64), walks its set bits j in order and
// adds popcount(row i AND row j); row j's words below j's own are zero and
// are not read.  Four rows j are loaded before their popcounts are taken.
__global__ __launch_bounds__(HM_THREADS) void k_heavy_last(HmArgs A) {
    uint64_t acc = 0, pairs = 0;
    QueueCursor cur = queue_start();
    int64_t it_end = 0;
    for (int64_t it = queue_next(A.Q, cur, it_end); it >= 0; it = queue_next(A.Q, cur, it_end)) {
        for (int64_t jt = it; jt < it_end; ++jt) {
            const uint64_t item = (uint64_t)uniform64((int64_t)A.items[jt]);
            const int64_t h = item_seg(item);
            const int32_t r = uniform(A.hroot[h]);
            const int32_t D = uniform((int32_t)(A.rp[r + 1] - A.rp[r]));
            const int32_t W = (D + 63) >> 6;
            const uint64_t* R = A.rows + uniform64((int64_t)A.hoff[h]);
            const int32_t i0 = (int32_t)item_round(item) * HM_BLOCK;
            const int32_t i1 = min(i0 + HM_BLOCK, D);
            for (int32_t i = i0; i < i1; ++i) {
                const uint64_t* ri = R + (int64_t)i * W;
                const uint64_t a0 = lane() < W ? ri[lane()] : 0ull;
                const uint64_t a1 = lane() + WAVE < W ? ri[lane() + WAVE] : 0ull;
                for (int32_t wd = i >> 6; wd < W; ++wd) {
                    uint64_t bits = wd < WAVE ? readlane64(a0, wd) : readlane64(a1, wd - WAVE);
                    while (bits) {
                        int32_t js[4];
                        int nj = 0;
                        while (bits && nj < 4) {
                            js[nj++] = wd * 64 + __builtin_ctzll(bits);
                            bits &= bits - 1;
                        }
                        uint64_t b0[4], b1[4];
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const bool on = q < nj;
                            const uint64_t* rj = R + (int64_t)(on ? js[q] : i) * W;
                            const int32_t low = on ? (js[q] >> 6) : W;   // words below are zero
                            b0[q] = (lane() >= low && lane() < W) ? rj[lane()] : 0ull;
                            b1[q] = (lane() + WAVE >= low && lane() + WAVE < W) ? rj[lane() + WAVE] : 0ull;
                        }
#pragma unroll
                        for (int q = 0; q < 4; ++q)
                            acc += (uint64_t)(__popcll(a0 & b0[q]) + __popcll(a1 & b1[q]));
                        pairs += (uint64_t)nj;
                    }
                }
            }
        }
    }
    acc = wave_sum_u64(acc);
    if (lane() == 0) {
        if (acc) atomicAdd(&A.stats[0], (unsigned long long)acc);
        if (pairs) atomicAdd(&A.stats[6], (unsigned long long)pairs);
    }
}

static unsigned grid_threads(int64_t items) {
    int64_t b = (items + 255) / 256;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(b, (int64_t)device_info().n_cu * 32));
}

struct MaskCtx {
    const uint64_t* info;
    const uint64_t* M;
};

template <int MODE>
static void launch_mask(CliqueRun& R, MaskArgs A, int64_t p_lo, int64_t n_par, const char* name, double units) {
    if (n_par <= 0) return;
    fill_u64(reinterpret_cast<uint64_t*>(R.qctr), Q_WORDS, 0, R.s);
    A.Q.next = R.qctr;
    A.Q.n_items = n_par;
    // a wave sets up at most 64 parents at once (one per lane)
    A.Q.chunk = n_par >= R.waves * 64 ? WAVE : (n_par >= R.waves * 8 ? 8 : 1);
    A.p_lo = p_lo;
    A.stats = R.stats;
    ProfScope ps(name, R.s, units);
    k_clique_mask_level<MODE><<<R.blocks, CQ_THREADS, 0, R.s>>>(A);
    PG_HIP(hipGetLastError());
}

// Level `lev` (>= 2) entries [0, m), in segments of parents [p_lo, p_hi) at
// level lev-1, extended through the remaining levels with masks.
static void mask_levels(CliqueRun& R, const MaskCtx& X, int lev, MaskChain ch, const uint64_t* seg,
                        uint64_t seg_base, int64_t p_lo, int64_t p_hi, int64_t m) {
    pg_graph* g = R.g;
    Arena& ar = g->arena;
    MaskArgs A{};
    A.seg = seg;
    A.seg_base = seg_base;
    A.lev = lev;
    A.ch = ch;
    A.x_lo = 0;
    A.x_hi = m;
    A.info = X.info;
    A.M = X.M;
    if (m <= 0) return;
    if (lev + 1 == R.k - 2) {
        // the next level's entries are the last level's inputs: they are never
        // stored, the last level finds them in the sets of this level's entries
        A.lev = lev + 1;
        launch_mask<MODE_LAST>(R, A, 0, m, "clique_last", 0.0);
        return;
    }
    const size_t mk = ar.mark();
    uint32_t* cnt = push<uint32_t>(ar, m);
    uint64_t* start = push<uint64_t>(ar, m + 1);
    A.count = cnt;
    launch_mask<MODE_COUNT>(R, A, p_lo, p_hi - p_lo, "clique_count_l", (double)m);
    scan_u32(cnt, m, start, ar, R.s);
    const uint64_t total = read_u64(start + m, R.s);
    if (total == 0) {
        ar.reset(mk);
        return;
    }
    // a stored level is extended in turn: its entries (6 B), counts (4 B)
    // and starts (8 B), twice over for its own children
    const uint64_t per = 6 + 4 + 8;
    const uint64_t room = g->budget > ar.mark() ? g->budget - ar.mark() : 0;
    const uint64_t cap = std::max<uint64_t>(room / (per * 2), (uint64_t)g->dag.max_out + 1);
    const int64_t nb = (int64_t)((total + cap - 1) / cap);
    std::vector<int64_t> hc(nb + 1), hp(nb + 1);
    std::vector<uint64_t> hs(nb + 1);
    if (nb == 1) {
        hc[0] = 0; hc[1] = m;
        hp[0] = p_lo; hp[1] = p_hi - 1;
        hs[0] = 0; hs[1] = total;
    } else {
        const size_t mk2 = ar.mark();
        int64_t* dc = push<int64_t>(ar, nb + 1);
        int64_t* dp = push<int64_t>(ar, nb + 1);
        uint64_t* ds = push<uint64_t>(ar, nb + 1);
        k_chunk_bounds<<<(unsigned)((nb + 1 + 255) / 256), 256, 0, R.s>>>(
            start, m, cap, nb, reinterpret_cast<const int64_t*>(seg) + p_lo, (int64_t)seg_base, p_hi - p_lo, dc, dp, ds);
        PG_HIP(hipGetLastError());
        PG_HIP(hipMemcpyAsync(hc.data(), dc, sizeof(int64_t) * (nb + 1), hipMemcpyDeviceToHost, R.s));
        PG_HIP(hipMemcpyAsync(hp.data(), dp, sizeof(int64_t) * (nb + 1), hipMemcpyDeviceToHost, R.s));
        PG_HIP(hipMemcpyAsync(hs.data(), ds, sizeof(uint64_t) * (nb + 1), hipMemcpyDeviceToHost, R.s));
        PG_HIP(hipStreamSynchronize(R.s));
        ar.reset(mk2);
        for (int64_t j = 0; j <= nb; ++j) hp[j] += p_lo;
    }
    uint64_t biggest = 0;
    for (int64_t j = 0; j < nb; ++j) biggest = std::max<uint64_t>(biggest, hs[j + 1] - hs[j]);
    int32_t* n_idx = push<int32_t>(ar, std::max<uint64_t>(biggest, 1));
    uint16_t* n_pos = push<uint16_t>(ar, std::max<uint64_t>(biggest, 1));
    for (int64_t j = 0; j < nb; ++j) {
        const int64_t c0 = hc[j], c1 = hc[j + 1];
        const uint64_t mm = hs[j + 1] - hs[j];
        if (c1 <= c0 || mm == 0) continue;
        MaskArgs W = A;
        W.x_lo = c0;
        W.x_hi = c1;
        W.start = start;
        W.start_base = hs[j];
        W.out_idx = n_idx;
        W.out_pos = n_pos;
        const int64_t q_lo = hp[j];
        const int64_t q_hi = (nb == 1 || j + 1 == nb) ? p_hi : hp[j + 1] + 1;
        launch_mask<MODE_WRITE>(R, W, q_lo, q_hi - q_lo, "clique_write_l", (double)mm);
        MaskChain nc = ch;
        nc.idx[lev + 1] = n_idx;
        nc.pos[lev + 1] = n_pos;
        mask_levels(R, X, lev + 1, nc, start, hs[j], c0, c1, (int64_t)mm);
    }
    ar.reset(mk);
}

// The mask path's layout and schedule, built once per graph beside the DAG
// (they depend on its out-degrees only): each light root's first mask
// word, the windows of roots for the fused last level, the count pass's
// work items (rounds of 64 or 16 level-1 entries of light roots), and the heavy
// roots' out-lists as a CSR of their own for the general kernels.
static void build_mask_plan(pg_graph* g) {
    MaskPlan& P = g->dag.plan;
    if (P.built) return;
    const int64_t n = g->n;
    const int64_t E = g->dag.n_edges;
    const int64_t* rp = g->dag.rp.as<int64_t>();
    hipStream_t s = g->stream;
    // temporaries in an arena of their own (the call's arena grows by need),
    // none released before the end: four uint32[n] arrays and three
    // uint64[n+1] offset arrays (40 B per root), the items at their bound
    // (round_items' bound), and the scans' tile sums
    // small graphs take rounds of 16 entries, so that the few waves holding
    // a hub's entries do not serialise the whole pass
    P.round = (E < BM_SMALL_E) ? BM_SMALL_ROUND : WAVE;
    const int64_t cap = E / P.round + n + 1;
    Arena ar;
    ar.buf.reserve(sizeof(uint64_t) * (size_t)(9 * (n + 1) + cap + 16 * ((n + 2047) / 2048)) + (size_t(1) << 20));
    P.moff.reserve(sizeof(uint64_t) * (n + 1));
    uint64_t* moff = P.moff.as<uint64_t>();
    uint64_t* lseg = push<uint64_t>(ar, n + 1);
    P.hrp.reserve(sizeof(uint64_t) * (n + 1));
    uint64_t* hrp = P.hrp.as<uint64_t>();
    {
        uint32_t* words = push<uint32_t>(ar, n);
        uint32_t* light = push<uint32_t>(ar, n);
        uint32_t* heavy = push<uint32_t>(ar, n);
        k_mask_words<<<grid_threads(n), 256, 0, s>>>(n, rp, words, light, heavy);
        PG_HIP(hipGetLastError());
        scan_u32(words, n, moff, ar, s);
        scan_u32(light, n, lseg, ar, s);
        scan_u32(heavy, n, hrp, ar, s);
    }
    const int64_t words = (int64_t)read_u64(moff + n, s);
    const int64_t e_heavy = (int64_t)read_u64(hrp + n, s);
    P.hcol.reserve(sizeof(int32_t) * (size_t)std::max<int64_t>(e_heavy, 1));
    if (e_heavy > 0) {
        k_heavy_lists<<<grid_threads(n * WAVE), 256, 0, s>>>(n, rp, g->dag.col.as<int32_t>(), hrp,
                                                             P.hcol.as<int32_t>());
        PG_HIP(hipGetLastError());
    }
    int64_t nw = 0;
    {
        uint32_t* mark = push<uint32_t>(ar, n);
        uint64_t* woff = push<uint64_t>(ar, n + 1);
        k_last_marks<<<grid_threads(n), 256, 0, s>>>(n, moff, mark);
        PG_HIP(hipGetLastError());
        scan_u32(mark, n, woff, ar, s);
        nw = (int64_t)read_u64(woff + n, s);
        P.wfirst.reserve(sizeof(int64_t) * (nw + 1));
        k_last_first<<<grid_threads(n), 256, 0, s>>>(n, mark, woff, P.wfirst.as<int64_t>());
        PG_HIP(hipGetLastError());
    }
    uint64_t* items = nullptr;
    const int64_t m = round_items(lseg, 0, n, P.round, ar, s, &items, E - e_heavy);
    P.item.reserve(sizeof(uint64_t) * std::max<int64_t>(m, 1));
    if (m > 0)
        PG_HIP(hipMemcpyAsync(P.item.as<uint64_t>(), items, sizeof(uint64_t) * m, hipMemcpyDeviceToDevice, s));
    // heavy roots for the wide rows: their list, row-word offsets and items
    // of HM_BLOCK rows
    P.n_heavy = P.hwords = P.hitems = 0;
    if (e_heavy > 0) {
        uint32_t* flag = push<uint32_t>(ar, n);
        uint64_t* pos = push<uint64_t>(ar, n + 1);
        k_heavy_flags<<<grid_threads(n), 256, 0, s>>>(n, rp, flag);
        PG_HIP(hipGetLastError());
        scan_u32(flag, n, pos, ar, s);
        const int64_t nh = (int64_t)read_u64(pos + n, s);
        P.hroot.reserve(sizeof(int32_t) * std::max<int64_t>(nh, 1));
        P.hoff.reserve(sizeof(uint64_t) * (nh + 1));
        uint32_t* hdeg = push<uint32_t>(ar, std::max<int64_t>(nh, 1));
        uint64_t* hw = push<uint64_t>(ar, std::max<int64_t>(nh, 1));
        uint64_t* hseg = push<uint64_t>(ar, nh + 1);
        k_heavy_fill<<<grid_threads(n), 256, 0, s>>>(n, rp, pos, P.hroot.as<int32_t>(), hdeg, hw);
        PG_HIP(hipGetLastError());
        scan_u32(hdeg, nh, hseg, ar, s);
        scan_u64(hw, nh, P.hoff.as<uint64_t>(), ar, s);
        uint64_t* hitems = nullptr;
        const int64_t mh = round_items(hseg, 0, nh, HM_BLOCK, ar, s, &hitems);
        P.hitem.reserve(sizeof(uint64_t) * std::max<int64_t>(mh, 1));
        if (mh > 0)
            PG_HIP(hipMemcpyAsync(P.hitem.as<uint64_t>(), hitems, sizeof(uint64_t) * mh, hipMemcpyDeviceToDevice, s));
        P.n_heavy = nh;
        P.hitems = mh;
        P.hwords = (int64_t)read_u64(P.hoff.as<uint64_t>() + nh, s);
    }
    PG_HIP(hipStreamSynchronize(s));
    P.words = words;
    P.windows = nw;
    P.items = m;
    P.heavy_edges = e_heavy;
    P.built = true;
}

// Triangles (k = 3) or 4-cliques (k = 4) at the heavy roots through wide
// rows; the count goes to stats[0].
static void heavy_masks(CliqueRun& R, const MaskPlan& P) {
    pg_graph* g = R.g;
    hipStream_t s = R.s;
    Arena& ar = g->arena;
    HmArgs A{};
    A.items = P.hitem.as<uint64_t>();
    A.hroot = P.hroot.as<int32_t>();
    A.hoff = P.hoff.as<uint64_t>();
    A.rp = g->dag.rp.as<int64_t>();
    A.col = g->dag.col.as<int32_t>();
    A.stats = R.stats;
    A.rows = R.k == 4 ? push<uint64_t>(ar, (size_t)std::max<int64_t>(P.hwords, 1)) : nullptr;
    A.Q.n_items = P.hitems;
    A.Q.chunk = 1;
    if (P.hitems == 0) return;
    fill_u64(reinterpret_cast<uint64_t*>(R.qctr), Q_WORDS, 0, s);
    A.Q.next = R.qctr;
    {
        ProfScope ps("clique_heavy_rows", s, (double)P.n_heavy);
        k_heavy_rows<<<(unsigned)(4 * device_info().n_cu), HM_THREADS, 0, s>>>(A);
        PG_HIP(hipGetLastError());
    }
    if (R.k == 4) {
        fill_u64(reinterpret_cast<uint64_t*>(R.qctr), Q_WORDS, 0, s);
        ProfScope ps("clique_heavy_last", s, (double)P.n_heavy);
        k_heavy_last<<<(unsigned)(8 * device_info().n_cu), HM_THREADS, 0, s>>>(A);
        PG_HIP(hipGetLastError());
    }
}

// Returns the number of level-2 entries: the triangles, which are the
// count for k = 3 (the count pass alone) and the last level's inputs for
// k = 4.
static uint64_t count_cliques4_masks(pg_graph* g, CliqueRun& R) {
    hipStream_t s = R.s;
    Arena& ar = g->arena;
    const int64_t n = g->n;
    const int64_t E = g->dag.n_edges;
    const int64_t* rp = g->dag.rp.as<int64_t>();
    const int32_t* col = g->dag.col.as<int32_t>();
    PG_REQUIRE(E <= INT32_MAX, PG_EUNSUPPORTED, "level-2 parent indices are 32-bit: too many DAG edges");
    build_mask_plan(g);
    const MaskPlan& P = g->dag.plan;
    const uint64_t* moff = P.moff.as<uint64_t>();
    const uint64_t mwords = (uint64_t)P.words;
    // two words of padding: the deeper levels read rows in 16-byte pairs
    uint64_t* M = push<uint64_t>(ar, mwords + 2);
    uint32_t* cnt = push<uint32_t>(ar, E);
    uint64_t* info = push<uint64_t>(ar, E);
    uint64_t* start = push<uint64_t>(ar, E + 1);
    fill_u32(cnt, E, 0, s);
    R.mwords = mwords;
    // k = 4: windows of roots for the fused last level (first root of each)
    const int64_t nw = P.windows;
    const int64_t* wfirst = P.wfirst.as<int64_t>();
    {
        BmArgs A;
        const uint64_t* items = P.item.as<uint64_t>();
        const int64_t n_items = P.items;
        fill_u64(reinterpret_cast<uint64_t*>(R.qctr), Q_WORDS, 0, s);
        A.Q.next = R.qctr;
        A.Q.n_items = n_items;
        A.Q.chunk = n_items >= R.waves * 64 ? 4 : 1;   // at most BM_CHUNK
        A.items = items;
        A.rp = rp;
        A.col = col;
        A.moff = moff;
        A.M = M;
        A.count = cnt;
        A.info = info;
        A.stats = R.stats;
        A.round = P.round;
        if (n_items > 0) {
            ProfScope ps("clique_count", s, (double)E);
            k_clique_count_masks<<<R.blocks, CQ_THREADS, 0, s>>>(A);
            PG_HIP(hipGetLastError());
        }
    }
    scan_u32(cnt, E, start, ar, s);
    const uint64_t total = read_u64(start + E, s);
    // level 2 holds the triangles (r, S[i], S[j]), i < j, each once
    if (total == 0 || R.k == 3) return total;
    // edge blocking over level-1 entries: 6 bytes per level-2 entry, and
    // for k >= 5 its child count and offset (12 B) plus room for a chunk of
    // the next level
    const uint64_t room = g->budget > ar.mark() ? g->budget - ar.mark() : 0;
    const uint64_t per = R.k == 4 ? 6 : 6 + 4 + 8;
    const uint64_t cap = std::max<uint64_t>(room / (per * (R.k == 4 ? 1 : 2)), (uint64_t)g->dag.max_out + 1);
    const int64_t nb = (int64_t)((total + cap - 1) / cap);
    std::vector<int64_t> hc(nb + 1), hp(nb + 1);
    std::vector<uint64_t> hs(nb + 1);
    if (nb == 1) {
        hc[0] = 0; hc[1] = E;
        hs[0] = 0; hs[1] = total;
    } else {
        const size_t mk2 = ar.mark();
        int64_t* dc = push<int64_t>(ar, nb + 1);
        int64_t* dp = push<int64_t>(ar, nb + 1);
        uint64_t* ds = push<uint64_t>(ar, nb + 1);
        k_chunk_bounds<<<(unsigned)((nb + 1 + 255) / 256), 256, 0, s>>>(start, E, cap, nb, rp, 0, n, dc, dp, ds);
        PG_HIP(hipGetLastError());
        PG_HIP(hipMemcpyAsync(hc.data(), dc, sizeof(int64_t) * (nb + 1), hipMemcpyDeviceToHost, s));
        PG_HIP(hipMemcpyAsync(hs.data(), ds, sizeof(uint64_t) * (nb + 1), hipMemcpyDeviceToHost, s));
        PG_HIP(hipStreamSynchronize(s));
        ar.reset(mk2);
    }
    uint64_t biggest = 0;
    for (int64_t j = 0; j < nb; ++j) biggest = std::max<uint64_t>(biggest, hs[j + 1] - hs[j]);
    int32_t* l2_idx = push<int32_t>(ar, std::max<uint64_t>(biggest, 1));
    uint16_t* l2_pos = push<uint16_t>(ar, std::max<uint64_t>(biggest, 1));
    for (int64_t j = 0; j < nb; ++j) {
        const int64_t c0 = hc[j], c1 = hc[j + 1];
        const uint64_t m2 = hs[j + 1] - hs[j];
        if (c1 <= c0 || m2 == 0) continue;
        {
            ProfScope ps("clique_write", s, (double)m2);
            k_clique_write_masks<<<grid_threads(c1 - c0), WR_THREADS, 0, s>>>(c0, c1, info, M, start, hs[j], l2_idx, l2_pos,
                                                                       R.stats);
            PG_HIP(hipGetLastError());
        }
        if (R.k == 4) {
            const size_t mk = ar.mark();
            uint64_t* wseg = push<uint64_t>(ar, nw + 1);
            k_last_segs<<<grid_threads(nw + 1), 256, 0, s>>>(nw, wfirst, rp, start, c0, c1, wseg);
            PG_HIP(hipGetLastError());
            // the item count stays on the device (stats[7]): no round trip
            uint64_t* items = nullptr;
            round_items(wseg, 0, nw, LW_PER, ar, s, &items, (int64_t)m2, reinterpret_cast<uint64_t*>(R.stats + 7));
            fill_u64(reinterpret_cast<uint64_t*>(R.qctr), Q_WORDS, 0, s);
            {
                ProfScope ps("clique_last", s, 0.0);
                k_clique_last_lds<<<(unsigned)(2 * device_info().n_cu), LW_THREADS, 0, s>>>(
                    items, R.stats + 7, wseg, wfirst, moff, l2_idx, l2_pos, info, M, R.qctr, R.stats);
                PG_HIP(hipGetLastError());
            }
            ar.reset(mk);
        } else {
            MaskCtx X{info, M};
            MaskChain ch{};
            ch.idx[2] = l2_idx;
            ch.pos[2] = l2_pos;
            mask_levels(R, X, 2, ch, start, hs[j], c0, c1, (int64_t)m2);
        }
    }
    // input entries of the last level (the level-2 entries)
    return total;
}

uint64_t count_cliques(pg_graph* g, int k) {
    PG_REQUIRE(k >= 1 && k <= PG_KMAX, PG_EUNSUPPORTED, "k must be in [1, PG_KMAX]");
    if (k == 1) return (uint64_t)g->n;
    if (k == 2) return (uint64_t)(g->nnz / 2);
    build_dag(g);
    if (g->dag.n_edges == 0) return 0;
    hipStream_t s = g->stream;
    Arena& ar = g->arena;
    CliqueRun R;
    R.g = g;
    R.k = k;
    R.s = s;
    R.waves = grid_waves(32);
    R.blocks = (int)(R.waves / CQ_WAVES);
    R.long_segments = g->dag.max_out > CQ_ROUND;
    uint64_t* small = push<uint64_t>(ar, 12 + Q_WORDS);
    R.stats = reinterpret_cast<unsigned long long*>(small);
    R.qctr = reinterpret_cast<unsigned long long*>(small + 12);
    fill_u64(small, 12, 0, s);
    const bool masks = k >= 3 && !g->force_generic;
    uint64_t n2 = 0;
    if (masks) {
        // every clique is counted at its lowest vertex (its root): roots of
        // out-degree above BM_MAXD through the general kernels, over the
        // CSR of their out-lists, the others through the sibling masks
        build_mask_plan(g);
        const MaskPlan& P = g->dag.plan;
        if (P.heavy_edges > 0) {
            // the count pass below needs the mask rows and per-entry counts,
            // infos and offsets: if the arena cannot hold them, rerun the call
            // now rather than after the heavy roots' levels
            const uint64_t E1 = (uint64_t)g->dag.n_edges;
            const size_t light = 8 * std::max<uint64_t>((uint64_t)P.words, 1) + 20 * E1 + 8 + 4 * 256;
            ar.ensure(light);
            const size_t mk = ar.mark();
            // k = 3, 4: wide rows in device memory when every heavy root
            // fits them and they fit the budget; otherwise the general kernels
            const uint64_t room = g->budget > ar.mark() ? g->budget - ar.mark() : 0;
            if (k <= 4 && g->dag.max_out <= HM_MAXD && (k == 3 || (uint64_t)P.hwords * 8 <= room / 2)) {
                heavy_masks(R, P);
            } else {
                extend_level(R, 1, reinterpret_cast<const int64_t*>(P.hrp.as<uint64_t>()), 0, 0, g->n,
                             P.hcol.as<int32_t>(), 0, P.heavy_edges);
            }
            ar.reset(mk);
        }
        n2 = count_cliques4_masks(g, R);
    } else {
        // level L1: entries = DAG edges, parents = vertices (segment = out-list)
        extend_level(R, 1, g->dag.rp.as<int64_t>(), 0, 0, g->n, g->dag.col.as<int32_t>(), 0, g->dag.n_edges);
    }
    uint64_t st[12] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    PG_HIP(hipMemcpyAsync(st, small, sizeof(st), hipMemcpyDeviceToHost, s));
    PG_HIP(hipStreamSynchronize(s));
    if (masks) st[1] = n2;
    if (prof_on()) {
        // algorithmic bytes of one call, per kernel
        const double E = (double)g->dag.n_edges;
        if (!masks) {
            // last level: per input entry its SoA entry and a row-pointer
            // pair (16 B), and the out-list of its newest vertex (4 B each)
            ProfScope ps("clique_last_work", s, 16.0 * (double)st[1] + 4.0 * (double)st[2]);
        } else {
            // count pass: per level-1 entry its vertex, row-pointer pair,
            // count and row info (32 B) and its mask row; 4 B per streamed
            // out-list element
            ProfScope pc("clique_count_work", s, 32.0 * E + 8.0 * (double)R.mwords + 4.0 * (double)st[3]);
            // write pass: a start pair per level-1 entry, info and row of
            // every entry with children, 6 B per level-2 entry written
            if (k >= 4) ProfScope pw("clique_write_work", s, 16.0 * E + (double)st[4] + 6.0 * (double)st[1]);
            if (k == 4)   // last level: 6 B SoA + 8 B info per entry, 16 B per pair of row words
                ProfScope pl("clique_last_work", s, 14.0 * (double)st[1] + 16.0 * (double)st[2]);
            if (k >= 5) {
                // last mask level: per parent its level-1 info (8 B), its
                // ancestry (idx and pos, 6 B per level) and the words of its
                // set (8 B each); per child the row words read (8 B each)
                const double na = (double)(k - 4);
                ProfScope pl("clique_last_work", s,
                             (8.0 + 6.0 * na) * (double)st[8] + 8.0 * (double)st[9] + 8.0 * (double)st[11]);
            }
        }
    }
    // k = 3 on the mask path: the light roots' triangles are the level-2
    // entries; the heavy roots' are in st[0]
    return (masks && k == 3 ? n2 : 0) + st[0];
}

__global__ void k_vertex_of_rank(int64_t n, const int32_t* __restrict__ rank_of, int32_t* __restrict__ vor) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
        vor[rank_of[v]] = (int32_t)v;
}

// Lists the k-cliques through the general level kernels: the last level is
// materialised like the others (count pass, scan, write) and each of its
// entries, walked up to its root, is one clique.  Rows of k original vertex
// ids, the root (lowest in the degree order) first, then one vertex per
// level; cliques in the order of the levels (by root, then level by level).
// The first `capacity` go to `out`; returns the number of k-cliques.
uint64_t list_cliques(pg_graph* g, int k, int32_t* out, uint64_t capacity) {
    PG_REQUIRE(k >= 1 && k <= PG_KMAX, PG_EUNSUPPORTED, "k must be in [1, PG_KMAX]");
    build_dag(g);
    const int64_t n = g->n;
    hipStream_t s = g->stream;
    Arena& ar = g->arena;
    int32_t* vor = push<int32_t>(ar, (size_t)std::max<int64_t>(n, 1));
    if (n > 0) {
        k_vertex_of_rank<<<grid_threads(n), 256, 0, s>>>(n, g->dag.rank_of.as<int32_t>(), vor);
        PG_HIP(hipGetLastError());
    }
    if (k == 1) {   // the vertices, in the degree order
        const uint64_t c = std::min<uint64_t>((uint64_t)n, capacity);
        if (c > 0) PG_HIP(hipMemcpyAsync(out, vor, sizeof(int32_t) * c, hipMemcpyDeviceToHost, s));
        PG_HIP(hipStreamSynchronize(s));
        return (uint64_t)n;
    }
    if (g->dag.n_edges == 0) return 0;
    CliqueRun R;
    R.g = g;
    R.k = k;
    R.s = s;
    R.waves = grid_waves(32);
    R.blocks = (int)(R.waves / CQ_WAVES);
    R.long_segments = g->dag.max_out > CQ_ROUND;
    uint64_t* small = push<uint64_t>(ar, 12 + Q_WORDS);
    R.stats = reinterpret_cast<unsigned long long*>(small);
    R.qctr = reinterpret_cast<unsigned long long*>(small + 12);
    fill_u64(small, 12, 0, s);
    ListOut O;
    O.host = out;
    O.capacity = out ? capacity : 0;
    O.vertex_of_rank = vor;
    R.list = &O;
    extend_level(R, 1, g->dag.rp.as<int64_t>(), 0, 0, n, g->dag.col.as<int32_t>(), 0, g->dag.n_edges);
    PG_HIP(hipStreamSynchronize(s));
    return O.found;
}

}  // namespace pg
