// Vertex-induced motif counting for k = 3, 4 and 5 (Pangolin sections 2.2,
// 3.3 motif Listing, 4.2).
//
// Canonical test (isAutoCanonical for vertex extension).  An embedding is
// kept in one order only: the breadth-first order from its smallest
// vertex, neighbours of one vertex taken in increasing id.  With p(j) the
// position of v_j's first earlier neighbour, a sequence is canonical iff
// v0 is the minimum, p is non-decreasing and p(j) = p(j+1) implies
// v_j < v_{j+1}.  Extending a canonical sequence by u is canonical iff
// u > v0, u is not in it, and with s = the first position adjacent to u:
// s >= p(last), and s = p(last) implies u > v_last.
//
// Levels.  L1 = every edge once as (v0 < v1) (p(1) = 0).  L2 = canonical
// connected 3-sets (v0, v1, v2) built by count / scan / write, each entry
// with a 2-bit connectivity code memoising its pattern (bit 0: v2 ~ v0,
// bit 1: v2 ~ v1; section 4.2 memoisation).  The last level is fused with
// classification and reduction.
//
// Fused last level.  For an embedding E and a candidate u let the mask be
// the set of E's vertices adjacent to u.  The canonical test depends only on
// the mask and on whether u lies above a threshold (v_last or v0); the
// pattern of E + u is the connectivity bitmap of E plus the mask, looked up
// in a 64-entry table.  So instead of testing every candidate one by one,
// the kernel counts candidates per exact mask and per threshold range from
// set intersections (each computed by iterating the smaller list and
// binary-searching the larger one), then applies the canonical rule and the
// table to the counts.  This is the same reduction (Algorithm 2 Reduce with
// support 1 and Aggregate = sum) without enumerating candidates.
//
// Output order: k = 3: wedge, triangle; k = 4: path, star, cycle, paw,
// diamond, 4-clique; k = 5: the 21 classes described at k_motif_last5.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "pg_device.h"
#include "pg_internal.h"

namespace pg {

constexpr int MO_THREADS = 128;
constexpr int MO_WAVES = MO_THREADS / WAVE;
constexpr int MO_STAGE = 512;     // adjacency lists up to this long are staged in LDS
constexpr int MO_CMAX = 512;      // common-neighbour lists up to this long live in LDS
constexpr int MO_FLAT = 1024;     // children streaming fewer candidates share wave steps
constexpr int MO5_WAVES_PER_CU = 32;   // k = 5 last level: at most this many waves per CU (latency-bound lanes)

enum { ML1_COUNT = 0, ML1_WRITE = 1, ML1_LAST3 = 2 };

// Pattern table for 4 vertices.  Bit i of the index is pair i of
// (01, 02, 12, 03, 13, 23).  Value: 0 path, 1 star, 2 cycle, 3 paw,
// 4 diamond, 5 4-clique, -1 disconnected.
struct Lut4 {
    int8_t v[64];
};

__host__ __device__ constexpr Lut4 make_lut4() {
    Lut4 t{};
    const int pa[6] = {0, 0, 1, 0, 1, 2};
    const int pb[6] = {1, 2, 2, 3, 3, 3};
    for (int m = 0; m < 64; ++m) {
        int deg[4] = {0, 0, 0, 0};
        int e = 0;
        for (int i = 0; i < 6; ++i)
            if ((m >> i) & 1) {
                deg[pa[i]]++;
                deg[pb[i]]++;
                e++;
            }
        int dmin = 4, dmax = 0;
        for (int a = 0; a < 4; ++a) {
            dmin = deg[a] < dmin ? deg[a] : dmin;
            dmax = deg[a] > dmax ? deg[a] : dmax;
        }
        int8_t c = -1;
        if (dmin > 0) {
            if (e == 3) c = (dmax == 3) ? 1 : (e == 3 && dmax == 2 ? 0 : -1);
            else if (e == 4) c = (dmax == 3) ? 3 : 2;
            else if (e == 5) c = 4;
            else if (e == 6) c = 5;
        }
        t.v[m] = c;
    }
    return t;
}

__constant__ Lut4 c_lut4 = make_lut4();

struct MotifArgs {
    XcdQueue Q;                 // over items[]: (segment, round of 64 children)
    const uint64_t* items;
    const int64_t* rp;          // undirected CSR
    const int32_t* col;
    // level-1 segments: vertex v0 owns L1 entries l1_seg[v0] .. l1_seg[v0+1]-1
    const int64_t* l1_seg;
    const int32_t* l1_src;
    const int32_t* l1_dst;
    const int32_t* l1_rev;      // first place in l1_dst's row past l1_src (row-relative)
    int64_t x_lo, x_hi;         // L1 entries extended (count / write / last3)
    uint32_t* count;            // ML1_COUNT: L2 children per L1 entry (indexed by entry)
    const uint64_t* start;      // ML1_WRITE: children of entry x at start[x] - start_base
    uint64_t start_base;
    // ML1_WRITE: entries with at least this many children go to the map
    // kernel, which tells from its map whether a child of A0 is adjacent to
    // v1, so their codes are not computed here
    uint64_t heavy_min;
    int32_t* out_vid;
    uint8_t* out_code;
    // last level of k = 4: segment p (an L1 entry) owns L2 entries
    // seg2[p] - seg2_base .. seg2[p+1] - seg2_base - 1
    const uint64_t* seg2;
    uint64_t seg2_base;
    const int32_t* vid2;
    const uint8_t* code2;
    int32_t* scratch;           // per-wave common-neighbour lists longer than MO_CMAX
    int64_t scratch_per_wave;
    unsigned long long* out;    // pattern counters (6) + work stats
    // dense rows of high-degree vertices: hub_id[v] >= 0 selects row
    // hub_bits + hub_id[v] * hub_words (bit u set iff u ~ v)
    const int32_t* hub_id;
    const uint32_t* hub_bits;
    int64_t hub_words;
};

// --------------------------------------------------------------- helpers

template <class P>
__device__ __forceinline__ bool member(P a, int32_t len, int32_t key) {
    return contains(a, len, key);
}

__device__ __forceinline__ const uint32_t* hub_row(const MotifArgs& A, int32_t v) {
    const int32_t h = A.hub_id[v];
    return h >= 0 ? A.hub_bits + (int64_t)h * A.hub_words : nullptr;
}

__device__ __forceinline__ bool bit_has(const uint32_t* row, int32_t u) {
    return (row[(uint32_t)u >> 5] >> (u & 31)) & 1u;
}

// membership in a sorted list, through its dense row when it has one
template <class P>
__device__ __forceinline__ bool adj_has(const uint32_t* row, P a, int32_t len, int32_t u) {
    return row ? bit_has(row, u) : member(a, len, u);
}

// the same for a wave-uniform len (unrolled search)
template <class P>
__device__ __forceinline__ bool adj_has_u(const uint32_t* row, P a, int32_t len, int32_t u) {
    return row ? bit_has(row, u) : member_u(a, len, u);
}

// relative cost of one membership test: 1 through LDS or a dense row,
// otherwise the depth of a binary search in global memory
__device__ __forceinline__ int32_t probe_cost(bool cheap, int32_t len) {
    return cheap ? 1 : 32 - __clz(max(len, 1));
}

// ---------------------------------------------------------- level 1 -> 2

struct L1Lds {
    int32_t A0[MO_WAVES][MO_STAGE];
    uint32_t pre[MO_WAVES][WAVE];
    int64_t lo1[MO_WAVES][WAVE];    // first entry of A1 above v0 (global index)
    int32_t d1[MO_WAVES][WAVE];     // |A1 above v0|
    int32_t v1[MO_WAVES][WAVE];
    int32_t na[MO_WAVES][WAVE];     // |A0 above v1|
    int32_t opt[MO_WAVES][WAVE];    // COUNT/LAST3: 0 iterate A0', 1 iterate A1'; WRITE: 1 no codes (map kernel)
    int32_t hb1[MO_WAVES][WAVE];    // dense row of v1, or -1
    uint32_t c_all[MO_WAVES][WAVE];
    uint32_t c_hi[MO_WAVES][WAVE];
};

// L1 entries [xc, x1) of vertex v0 (at most 64: one work item)
template <int MODE, class P0>
__device__ __forceinline__ void motif_l1_segment(const MotifArgs& A, L1Lds& L, int w, int32_t v0, P0 A0,
                                                 int32_t d0, int64_t r0, int64_t b, int32_t xc, int32_t x1,
                                                 uint64_t (&acc)[6], const uint32_t* h0, bool a0_cheap) {
    // A0' = A0 above v0, at positions [a0lo, d0)
    const int32_t a0lo = (int32_t)upper_bound(A0, 0, d0, v0);
    {
        const int32_t x = xc + lane();
        uint32_t work = 0;
        if (x < x1) {
            const int32_t v1 = A.l1_dst[b + x];
            const int64_t q0 = A.rp[v1], q1 = A.rp[v1 + 1];
            const int64_t lo1 = upper_bound(A.col, q0, q1, v0);
            const int32_t d1p = (int32_t)(q1 - lo1);
            const int32_t na = d0 - (int32_t)upper_bound(A0, a0lo, d0, v1);
            const int32_t d0p = d0 - a0lo;
            const int32_t hb1 = A.hub_id[v1];
            int opt = 0;
            if (MODE == ML1_WRITE) {
                work = (uint32_t)(na + d1p);
                opt = (A.start[b + x + 1] - A.start[b + x] >= A.heavy_min) ? 1 : 0;
            } else {
                // iterate A0' probing A1, or A1' probing A0: the cheaper total
                const int64_t c0 = (int64_t)d0p * probe_cost(hb1 >= 0, (int32_t)(q1 - q0));
                const int64_t c1 = (int64_t)d1p * probe_cost(a0_cheap, d0);
                opt = (c0 <= c1) ? 0 : 1;
                work = (uint32_t)(opt == 0 ? d0p : d1p);
            }
            L.lo1[w][lane()] = lo1;
            L.d1[w][lane()] = d1p;
            L.v1[w][lane()] = v1;
            L.na[w][lane()] = na;
            L.opt[w][lane()] = opt;
            L.hb1[w][lane()] = hb1;
        }
        const uint32_t inc = wave_incl_scan(work);
        const uint32_t W = bcast(inc, WAVE - 1);
        if (MODE == ML1_LAST3 && lane() == 0) {
            acc[2] += W;                     // list elements iterated
            acc[3] += (uint64_t)(x1 - xc);   // level-1 entries
        }
        L.pre[w][lane()] = inc - work;
        L.c_all[w][lane()] = 0;
        L.c_hi[w][lane()] = 0;
        wave_sync();
        const int nx = min(WAVE, x1 - xc);
        for (uint32_t t0 = 0; t0 < W; t0 += WAVE) {
            const uint32_t t = t0 + lane();
            const bool valid = t < W;
            int xi = 0;
            {
                int n_i = nx;
                while (n_i > 1) {
                    const int half = n_i >> 1;
                    if (L.pre[w][xi + half] <= t) xi += half;
                    n_i -= half;
                }
            }
            if (MODE != ML1_WRITE) {
                if (valid) {
                    const uint32_t j = t - L.pre[w][xi];
                    const int32_t v1 = L.v1[w][xi];
                    const int32_t hb1 = L.hb1[w][xi];
                    int32_t u;
                    bool f;
                    if (L.opt[w][xi] == 0) {
                        u = A0[a0lo + j];
                        if (hb1 >= 0) {
                            f = bit_has(A.hub_bits + (int64_t)hb1 * A.hub_words, u);
                        } else {
                            const int64_t q0 = A.rp[v1], q1 = A.rp[v1 + 1];
                            f = member(A.col + q0, (int32_t)(q1 - q0), u);
                        }
                    } else {
                        u = A.col[L.lo1[w][xi] + j];
                        f = adj_has(h0, A0, d0, u);
                    }
                    if (f) {
                        atomicAdd(&L.c_all[w][xi], 1u);
                        if (u > v1) atomicAdd(&L.c_hi[w][xi], 1u);
                    }
                }
            } else {
                // children of (v0, v1): u in A0 above v1 (code bit 0 set, bit 1 =
                // u ~ v1), then u in A1 above v0 not adjacent to v0 (code 2)
                bool emit = false;
                int32_t u = 0;
                uint8_t code = 0;
                if (valid) {
                    const uint32_t j = t - L.pre[w][xi];
                    const int32_t v1 = L.v1[w][xi];
                    const int32_t na = L.na[w][xi];
                    const int32_t hb1 = L.hb1[w][xi];
                    if ((int32_t)j < na) {
                        u = A0[d0 - na + (int32_t)j];
                        bool a12 = false;
                        if (L.opt[w][xi]) {
                            // the map kernel finds u ~ v1 in its map
                        } else if (hb1 >= 0) {
                            a12 = bit_has(A.hub_bits + (int64_t)hb1 * A.hub_words, u);
                        } else {
                            const int64_t q0 = A.rp[v1], q1 = A.rp[v1 + 1];
                            a12 = member(A.col + q0, (int32_t)(q1 - q0), u);
                        }
                        code = 1 | (a12 ? 2 : 0);
                        emit = true;
                    } else {
                        u = A.col[L.lo1[w][xi] + (j - (uint32_t)na)];
                        emit = !adj_has(h0, A0, d0, u);
                        code = 2;
                    }
                }
                const int key = valid ? xi : WAVE;
                const int prev = __shfl_up(key, 1, WAVE);
                const bool head = lane() == 0 || prev != key;
                const uint64_t H = ballot(head);
                const uint64_t F = ballot(emit);
                const uint64_t le = lanemask_lt() | (1ull << lane());
                const int h = 63 - __clzll(H & le);
                const uint64_t grp = le & ~((1ull << h) - 1ull);
                const uint32_t base = valid ? L.c_all[w][xi] : 0u;
                if (emit) {
                    const uint64_t dst = A.start[b + xc + xi] - A.start_base + base +
                                         (uint64_t)popc64(F & grp & lanemask_lt());
                    A.out_vid[dst] = u;
                    A.out_code[dst] = code;
                }
                const bool next_head = (lane() == WAVE - 1) || ((H >> (lane() + 1)) & 1ull);
                wave_sync();
                if (valid && next_head) L.c_all[w][xi] = base + (uint32_t)popc64(F & grp);
                wave_sync();
            }
        }
        wave_sync();
        if (x < x1) {
            const uint32_t ca = L.c_all[w][lane()], ch = L.c_hi[w][lane()];
            const int32_t na = L.na[w][lane()], d1p = L.d1[w][lane()];
            if (MODE == ML1_COUNT) {
                A.count[b + x] = (uint32_t)(na + d1p) - ca;
            } else if (MODE == ML1_LAST3) {
                acc[1] += ch;                                  // triangles
                acc[0] += (uint64_t)(na - (int32_t)ch) + (uint64_t)(d1p - (int32_t)ca);   // wedges
            }
        }
        wave_sync();
    }
}

template <int MODE>
__global__ __launch_bounds__(MO_THREADS) void k_motif_l1(MotifArgs A) {
    __shared__ L1Lds L;
    const int w = threadIdx.x / WAVE;
    uint64_t acc[6] = {0, 0, 0, 0, 0, 0};
    QueueCursor cur = queue_start();
    int64_t it_end = 0;
    for (int64_t it = queue_next(A.Q, cur, it_end); it >= 0; it = queue_next(A.Q, cur, it_end)) {
        for (int64_t j = it; j < it_end; ++j) {
            const uint64_t item = A.items[j];
            const int64_t p = item_seg(item);
            const int32_t v0 = (int32_t)p;
            const int64_t b = A.l1_seg[p], e = A.l1_seg[p + 1];
            const int32_t s = (int32_t)(e - b);
            // this item's entries, within the launch's window [x_lo, x_hi)
            const int32_t xa = (int32_t)max64(item_round(item) * WAVE, A.x_lo - b);
            const int32_t xb = (int32_t)min64(min64(item_round(item) * WAVE + WAVE, s), A.x_hi - b);
            if (xa >= xb) continue;
            const int64_t r0 = A.rp[v0], r1 = A.rp[v0 + 1];
            const int32_t d0 = (int32_t)(r1 - r0);
            if (MODE == ML1_LAST3 && lane() == 0) acc[4] += (uint64_t)d0 + 4;   // v0's row pointers and list
            if (d0 <= MO_STAGE) {
                for (int i = lane(); i < d0; i += WAVE) L.A0[w][i] = A.col[r0 + i];
                wave_sync();
                motif_l1_segment<MODE>(A, L, w, v0, &L.A0[w][0], d0, r0, b, xa, xb, acc, nullptr, true);
            } else {
                const uint32_t* h0 = hub_row(A, v0);
                motif_l1_segment<MODE>(A, L, w, v0, A.col + r0, d0, r0, b, xa, xb, acc, h0, h0 != nullptr);
            }
            wave_sync();
        }
    }
    if (MODE == ML1_LAST3) {
        const uint64_t wd = wave_sum_u64(acc[0]), tr = wave_sum_u64(acc[1]);
        if (lane() == 0) {
            if (wd) atomicAdd(&A.out[0], (unsigned long long)wd);
            if (tr) atomicAdd(&A.out[1], (unsigned long long)tr);
            // work (lane 0 holds it): elements iterated, entries, 4-byte words of staging
            if (acc[2]) atomicAdd(&A.out[12], (unsigned long long)acc[2]);
            if (acc[3]) atomicAdd(&A.out[13], (unsigned long long)acc[3]);
            if (acc[4]) atomicAdd(&A.out[14], (unsigned long long)acc[4]);
        }
    }
}

// ------------------------------------------------------- last level, k = 4

struct L4Lds {
    int32_t A0[MO_WAVES][MO_STAGE];
    int32_t A1[MO_WAVES][MO_STAGE];
    int32_t A2[MO_WAVES][MO_STAGE];  // the current child's list, when staged
    int32_t C[MO_WAVES][MO_CMAX];
};

// Adds the hits of one 64-candidate step to the six counters: [0, 1] u ~ v0
// and v2, [2, 3] u ~ v1 and v2, [4, 5] all three, each split into (v0, v2]
// and above v2.  Ballots make the counts wave-uniform.
__device__ __forceinline__ void tally(uint32_t (&c)[6], bool in02, bool in12, bool in012, bool hi) {
    c[0] += (uint32_t)popc64(ballot(in02 && !hi));
    c[1] += (uint32_t)popc64(ballot(in02 && hi));
    c[2] += (uint32_t)popc64(ballot(in12 && !hi));
    c[3] += (uint32_t)popc64(ballot(in12 && hi));
    c[4] += (uint32_t)popc64(ballot(in012 && !hi));
    c[5] += (uint32_t)popc64(ballot(in012 && hi));
}

// Children [xc, xc + 64) of one L1 entry (v0, v1).  A0/A1: the two adjacency lists (LDS or
// global) with their dense rows h0/h1 when they have one, C: A0 and A1
// above v0 intersected (sorted, LDS or scratch).
//
// The lanes first read 64 children's parameters and pick, per child, the
// cheaper way to get its counts: stream A2' (v2's list above v0) probing A0
// and A1, or stream A0' and A1' probing A2 (through v2's dense row, or a
// copy staged in LDS).  Then the wave takes the children one at a time:
// every lane probes one candidate of the child's stream, all lanes follow
// the same strategy, binary searches run the same number of steps in every
// lane, and the counts are ballot popcounts.
template <class P0, class P1, class PC>
__device__ __forceinline__ void motif_last4_segment(const MotifArgs& A, L4Lds& L, int w, int32_t v0, int32_t v1,
                                                    P0 A0, int32_t d0, P1 A1, int32_t d1, PC C, int32_t nc,
                                                    int64_t b, int32_t xc, int32_t s, uint64_t (&acc)[6],
                                                    uint64_t& items, const uint32_t* h0, const uint32_t* h1,
                                                    bool cheap0, bool cheap1) {
    const int32_t a0lo = (int32_t)upper_bound(A0, 0, d0, v0);
    const int32_t a1lo = (int32_t)upper_bound(A1, 0, d1, v0);
    const int32_t d0p = d0 - a0lo, d1p = d1 - a1lo;
    const int32_t pc0 = probe_cost(cheap0, d0), pc1 = probe_cost(cheap1, d1);
    int32_t* S2 = &L.A2[w][0];
    {   // children [xc, min(xc + 64, s)): one work item
        const int32_t x = xc + lane();
        int32_t v2 = 0, code = 0, hb2 = -1, opt = 0;
        int64_t s0 = 0, s1 = 0, lo2 = 0;
        if (x < s) {
            v2 = A.vid2[b + x];
            code = A.code2[b + x];
            s0 = A.rp[v2];
            s1 = A.rp[v2 + 1];
            lo2 = upper_bound(A.col, s0, s1, v0);
            const int32_t d2 = (int32_t)(s1 - s0), d2p = (int32_t)(s1 - lo2);
            hb2 = A.hub_id[v2];
            const bool stage2 = hb2 < 0 && d2 <= MO_STAGE;
            const int32_t pc2 = probe_cost(hb2 >= 0 || stage2, d2);
            const int64_t cost0 = (int64_t)d2p * (pc0 + pc1);
            const int64_t cost1 = (int64_t)d0p * (pc2 + pc1) + (int64_t)d1p * pc2 + (stage2 ? d2 : 0);
            opt = (cost0 <= cost1) ? 0 : 1;
            items += (uint64_t)(opt == 0 ? d2p : d0p + d1p);
        }
        uint32_t cnt[6] = {0, 0, 0, 0, 0, 0};   // lane x: its child's counters
        const int nx = min(WAVE, s - xc);
        // Children that stream their own list and have fewer than MO_FLAT
        // candidates: their lists are laid end to end and the wave takes 64
        // candidates a step, so several short children share a step.  A
        // lane finds its child in the prefix of the lengths; a child's lanes
        // are contiguous, and the last of them adds the child's counts
        // (ballot popcounts over its lanes, below v2 | above v2 << 16).  The
        // per-wave child staging area holds the prefix, list starts, v2 and
        // counts until they are read back.
        const bool flat = x < s && opt == 0 && (s1 - lo2) < MO_FLAT;
        {
            uint32_t* fpre = reinterpret_cast<uint32_t*>(S2);
            int64_t* flo = reinterpret_cast<int64_t*>(fpre + WAVE);
            int32_t* fv2 = reinterpret_cast<int32_t*>(flo + WAVE);
            uint32_t* fcc = reinterpret_cast<uint32_t*>(fv2 + WAVE);   // [3][WAVE]
            const uint32_t my = flat ? (uint32_t)(s1 - lo2) : 0u;
            const uint32_t inc = wave_incl_scan(my);
            const uint32_t total = bcast(inc, WAVE - 1);
            wave_sync();   // the previous item's use of the staging area is over
            fpre[lane()] = inc - my;
            flo[lane()] = lo2;
            fv2[lane()] = v2;
            fcc[lane()] = 0;
            fcc[WAVE + lane()] = 0;
            fcc[2 * WAVE + lane()] = 0;
            wave_sync();
            for (uint32_t t0 = 0; t0 < total; t0 += WAVE) {
                const uint32_t t = t0 + lane();
                const bool valid = t < total;
                // the child of candidate t: the last lane whose prefix is <= t
                int xi = 0;
                {
                    int n_i = nx;
                    while (n_i > 1) {
                        const int half = n_i >> 1;
                        if (fpre[xi + half] <= t) xi += half;
                        n_i -= half;
                    }
                }
                int32_t u = 0, cv = 0;
                if (valid) {
                    u = A.col[flo[xi] + (int64_t)(t - fpre[xi])];
                    cv = fv2[xi];
                }
                const bool in0 = valid && adj_has_u(h0, A0, d0, u);
                const bool in1 = valid && adj_has_u(h1, A1, d1, u);
                const bool hi = u > cv;
                const int key = valid ? xi : WAVE;
                const int prev = __shfl_up(key, 1, WAVE);
                const bool head = lane() == 0 || prev != key;
                const uint64_t H = ballot(head);
                const uint64_t le = lanemask_lt() | (1ull << lane());
                const int hd = 63 - __clzll(H & le);
                const uint64_t grp = le & ~((1ull << hd) - 1ull);
                const bool last = lane() == WAVE - 1 || ((H >> (lane() + 1)) & 1ull);
                const uint64_t B0l = ballot(in0 && !hi), B0h = ballot(in0 && hi);
                const uint64_t B1l = ballot(in1 && !hi), B1h = ballot(in1 && hi);
                const uint64_t B2l = ballot(in0 && in1 && !hi), B2h = ballot(in0 && in1 && hi);
                if (valid && last) {
                    fcc[xi] += (uint32_t)popc64(B0l & grp) | ((uint32_t)popc64(B0h & grp) << 16);
                    fcc[WAVE + xi] += (uint32_t)popc64(B1l & grp) | ((uint32_t)popc64(B1h & grp) << 16);
                    fcc[2 * WAVE + xi] += (uint32_t)popc64(B2l & grp) | ((uint32_t)popc64(B2h & grp) << 16);
                }
                wave_sync();
            }
            if (flat) {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const uint32_t v = fcc[c * WAVE + lane()];
                    cnt[2 * c] = v & 0xffffu;
                    cnt[2 * c + 1] = v >> 16;
                }
            }
            wave_sync();   // read back before the staging area is reused
        }
        for (int xi = 0; xi < nx; ++xi) {
            if (ballot(flat) >> xi & 1ull) continue;   // counted above
            const int32_t cv2 = readlane(v2, xi);
            uint32_t c6[6] = {0, 0, 0, 0, 0, 0};
            if (readlane(opt, xi) == 0) {
                const int64_t l = (int64_t)readlane64((uint64_t)lo2, xi);
                const int64_t h = (int64_t)readlane64((uint64_t)s1, xi);
                for (int64_t t0 = l; t0 < h; t0 += 2 * WAVE) {
                    const int64_t ta = t0 + lane(), tb = ta + WAVE;
                    const bool va = ta < h, vb = tb < h;
                    const int32_t ua = va ? A.col[ta] : 0;
                    const int32_t ub = vb ? A.col[tb] : 0;
                    const bool a0 = va && adj_has_u(h0, A0, d0, ua);
                    const bool b0 = vb && adj_has_u(h0, A0, d0, ub);
                    const bool a1 = va && adj_has_u(h1, A1, d1, ua);
                    const bool b1 = vb && adj_has_u(h1, A1, d1, ub);
                    tally(c6, a0, a1, a0 && a1, ua > cv2);
                    tally(c6, b0, b1, b0 && b1, ub > cv2);
                }
            } else {
                const int32_t hb = readlane(hb2, xi);
                const int64_t base = (int64_t)readlane64((uint64_t)s0, xi);
                const int32_t len2 = (int32_t)((int64_t)readlane64((uint64_t)s1, xi) - base);
                const uint32_t* h2 = hb >= 0 ? A.hub_bits + (int64_t)hb * A.hub_words : nullptr;
                const bool staged = h2 == nullptr && len2 <= MO_STAGE;
                if (staged) {
                    wave_sync();   // the previous child's probes are done
                    for (int k = lane(); k < len2; k += WAVE) S2[k] = A.col[base + k];
                    wave_sync();
                }
                const int32_t tot = d0p + d1p;
                for (int32_t t0 = 0; t0 < tot; t0 += WAVE) {
                    const int32_t t = t0 + lane();
                    const bool from0 = t < d0p;
                    bool in2 = false, in1 = false;
                    int32_t u = 0;
                    if (t < tot) {
                        u = from0 ? A0[a0lo + t] : A1[a1lo + (t - d0p)];
                        in2 = staged ? member_u(S2, len2, u) : adj_has_u(h2, A.col + base, len2, u);
                        in1 = from0 && in2 && adj_has_u(h1, A1, d1, u);
                    }
                    tally(c6, from0 && in2, !from0 && in2, in1, u > cv2);
                }
            }
            if (lane() == xi) {
#pragma unroll
                for (int c = 0; c < 6; ++c) cnt[c] = c6[c];
            }
        }
        if (x < s) {
            const int a02 = code & 1, a12 = (code >> 1) & 1;
            const int p = a02 ? 0 : 1;
            // "at least" counts per range: [0] = (v0, v2], [1] = above v2
            const int32_t u0 = (int32_t)upper_bound(A0, a0lo, d0, v2);
            const int32_t u1 = (int32_t)upper_bound(A1, a1lo, d1, v2);
            const int64_t u2 = upper_bound(A.col, lo2, s1, v2);
            const int32_t uc = (int32_t)upper_bound(C, 0, nc, v2);
            // per-child counts are bounded by a degree: 32-bit (fewer registers)
            const int32_t I0[2] = {u0 - a0lo, d0 - u0};
            const int32_t I1[2] = {u1 - a1lo, d1 - u1};
            const int32_t I2[2] = {(int32_t)(u2 - lo2), (int32_t)(s1 - u2)};
            const int32_t I01[2] = {uc, nc - uc};
            int32_t N[2][8];
#pragma unroll
            for (int r = 0; r < 2; ++r) {
                const int32_t i02 = (int32_t)cnt[0 + r], i12 = (int32_t)cnt[2 + r];
                const int32_t i012 = (int32_t)cnt[4 + r];
                N[r][0] = 0;
                N[r][7] = i012;
                N[r][3] = I01[r] - i012;
                N[r][5] = i02 - i012;
                N[r][6] = i12 - i012;
                N[r][1] = I0[r] - I01[r] - i02 + i012;
                N[r][2] = I1[r] - I01[r] - i12 + i012;
                N[r][4] = I2[r] - i02 - i12 + i012;
            }
            // the embedding's own vertices are not candidates: v1 (adjacent
            // to v0, to v2 iff a12) and v2 (adjacent to v0 iff a02, to v1 iff
            // a12); constant indices keep N and acc in registers
            const int r1 = v1 > v2 ? 1 : 0, m1 = 1 | (a12 ? 4 : 0), m2 = a02 | (a12 << 1);
#pragma unroll
            for (int r = 0; r < 2; ++r)
#pragma unroll
                for (int m = 0; m < 8; ++m) N[r][m] -= (int32_t)((r == r1 && m == m1) + (r == 0 && m == m2));
            const int ebits = 1 | (a02 << 1) | (a12 << 2);
#pragma unroll
            for (int m = 1; m < 8; ++m) {
                const int sbit = (m & 1) ? 0 : ((m & 2) ? 1 : 2);   // first adjacent position
                if (sbit < p) continue;
                const int64_t c = (sbit == p) ? (int64_t)N[1][m] : (int64_t)N[0][m] + N[1][m];
                const int pid = c_lut4.v[ebits | (m << 3)];
#pragma unroll
                for (int q = 0; q < 6; ++q) acc[q] += (pid == q) ? (uint64_t)c : 0ull;
            }
        }
        wave_sync();
    }
}

__global__ __launch_bounds__(MO_THREADS) void k_motif_last4(MotifArgs A) {
    __shared__ L4Lds L;
    const int w = threadIdx.x / WAVE;
    const int64_t wave_id = (int64_t)blockIdx.x * MO_WAVES + w;
    int32_t* scratch = A.scratch + wave_id * A.scratch_per_wave;
    uint64_t acc[6] = {0, 0, 0, 0, 0, 0};
    uint64_t items = 0, n_in = 0, deg_sum = 0;
    QueueCursor cur = queue_start();
    int64_t it_end = 0;
    for (int64_t it = queue_next(A.Q, cur, it_end); it >= 0; it = queue_next(A.Q, cur, it_end)) {
        for (int64_t j = it; j < it_end; ++j) {
            // per item everything is wave-uniform: keep it in scalar registers
            const uint64_t item = (uint64_t)uniform64((int64_t)A.items[j]);
            const int64_t p = item_seg(item);
            const int32_t xc = (int32_t)item_round(item) * WAVE;
            const int64_t b = uniform64((int64_t)(A.seg2[p] - A.seg2_base));
            const int32_t s = uniform((int32_t)(A.seg2[p + 1] - A.seg2[p]));
            if (xc >= s) continue;
            const int32_t v0 = uniform(A.l1_src[p]), v1 = uniform(A.l1_dst[p]);
            const int64_t r0 = uniform64(A.rp[v0]), q0 = uniform64(A.rp[v1]);
            const int32_t d0 = uniform((int32_t)(A.rp[v0 + 1] - r0)), d1 = uniform((int32_t)(A.rp[v1 + 1] - q0));
            const uint64_t n_here = (uint64_t)(min(xc + WAVE, s) - xc);
            n_in += (lane() == 0) ? n_here : 0;
            deg_sum += (lane() == 0) ? n_here * (uint64_t)(d0 + d1) : 0;
            const bool st0 = d0 <= MO_STAGE, st1 = d1 <= MO_STAGE;
            if (st0) for (int i = lane(); i < d0; i += WAVE) L.A0[w][i] = A.col[r0 + i];
            if (st1) for (int i = lane(); i < d1; i += WAVE) L.A1[w][i] = A.col[q0 + i];
            wave_sync();
            // C = A0 and A1 above v0, intersected: iterate the shorter, search the longer
            const int32_t* gA0 = A.col + r0;
            const int32_t* gA1 = A.col + q0;
            const uint32_t* h0 = st0 ? nullptr : hub_row(A, v0);
            const uint32_t* h1 = st1 ? nullptr : hub_row(A, v1);
            const bool it0 = d0 <= d1;
            const int32_t di = it0 ? d0 : d1;
            int32_t nc = 0;
            bool c_in_lds = true;
            for (int32_t j0 = 0; j0 < di; j0 += WAVE) {
                const int32_t j = j0 + lane();
                bool f = false;
                int32_t u = 0;
                if (j < di) {
                    if (it0) {
                        u = st0 ? L.A0[w][j] : gA0[j];
                        f = u > v0 && (st1 ? member_u(&L.A1[w][0], d1, u) : adj_has_u(h1, gA1, d1, u));
                    } else {
                        u = st1 ? L.A1[w][j] : gA1[j];
                        f = u > v0 && (st0 ? member_u(&L.A0[w][0], d0, u) : adj_has_u(h0, gA0, d0, u));
                    }
                }
                const uint64_t F = ballot(f);
                const int32_t pos = nc + popc64(F & lanemask_lt());
                if (f) {
                    scratch[pos] = u;
                    if (pos < MO_CMAX) L.C[w][pos] = u;
                }
                nc += popc64(F);
            }
            c_in_lds = nc <= MO_CMAX;
            __threadfence_block();
            wave_sync();
            // dispatch on where each list lives (all wave-uniform)
            const bool ch0 = st0 || h0 != nullptr, ch1 = st1 || h1 != nullptr;
            const int32_t* sc = scratch;
            if (st0 && st1) {
                if (c_in_lds) motif_last4_segment(A, L, w, v0, v1, &L.A0[w][0], d0, &L.A1[w][0], d1, &L.C[w][0], nc, b, xc, s, acc, items, h0, h1, ch0, ch1);
                else motif_last4_segment(A, L, w, v0, v1, &L.A0[w][0], d0, &L.A1[w][0], d1, sc, nc, b, xc, s, acc, items, h0, h1, ch0, ch1);
            } else if (st0) {
                if (c_in_lds) motif_last4_segment(A, L, w, v0, v1, &L.A0[w][0], d0, gA1, d1, &L.C[w][0], nc, b, xc, s, acc, items, h0, h1, ch0, ch1);
                else motif_last4_segment(A, L, w, v0, v1, &L.A0[w][0], d0, gA1, d1, sc, nc, b, xc, s, acc, items, h0, h1, ch0, ch1);
            } else if (st1) {
                if (c_in_lds) motif_last4_segment(A, L, w, v0, v1, gA0, d0, &L.A1[w][0], d1, &L.C[w][0], nc, b, xc, s, acc, items, h0, h1, ch0, ch1);
                else motif_last4_segment(A, L, w, v0, v1, gA0, d0, &L.A1[w][0], d1, sc, nc, b, xc, s, acc, items, h0, h1, ch0, ch1);
            } else {
                if (c_in_lds) motif_last4_segment(A, L, w, v0, v1, gA0, d0, gA1, d1, &L.C[w][0], nc, b, xc, s, acc, items, h0, h1, ch0, ch1);
                else motif_last4_segment(A, L, w, v0, v1, gA0, d0, gA1, d1, sc, nc, b, xc, s, acc, items, h0, h1, ch0, ch1);
            }
            wave_sync();
        }
    }
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        const uint64_t v = wave_sum_u64(acc[c]);
        if (lane() == 0 && v) atomicAdd(&A.out[c], (unsigned long long)v);
    }
    const uint64_t it_sum = wave_sum_u64(items);
    const uint64_t ni = wave_sum_u64(n_in), ds = wave_sum_u64(deg_sum);
    if (lane() == 0) {
        if (it_sum) atomicAdd(&A.out[6], (unsigned long long)it_sum);
        if (ni) atomicAdd(&A.out[7], (unsigned long long)ni);
        if (ds) atomicAdd(&A.out[8], (unsigned long long)ds);
    }
}

// --------------------------------------- last level, k = 4, many children
//
// L1 entries (v0, v1) with many children are taken by whole workgroups.  The
// workgroup marks the lists of v0 and v1 above v0 in a map in LDS with two
// bits per vertex (bit 0: u ~ v0, bit 1: u ~ v1), so testing a candidate u
// of a child's list against both lists is one LDS read.  The marks stay
// while consecutive items share v0 (only v1's are redone) or the whole entry
// (a long entry is cut into items of MM_CHILDREN children).  The waves take
// an item's children 64 at a time from a counter in LDS, so a wave that
// drew children with long lists does not hold the others at the next
// entry's barrier for more than one such group.  Per entry the
// workgroup also records, for every position j of v1's list above v0, how
// many of the elements before j are adjacent to v0 (cum), which gives the
// common neighbours of v0 and v1 up to any child v2 with one lookup.
//
// Each wave takes 64 children, one per lane: the lane finds the ranks of
// v2 in the lists of v0 and v1 (in v0's list by position for the children
// that are A0's elements above v1).  Children with
// fewer than 64 candidates are streamed by their own lane (four loads in
// flight); longer ones by the whole wave, 256 candidates per step, counted
// with ballots.  The counts per adjacency mask and range then go through
// the same canonical rule and pattern table as in k_motif_last4.
constexpr int MM_THREADS = 512;
constexpr int MM_WAVES = MM_THREADS / WAVE;
constexpr int MM_CHILDREN = 4096;              // children per item, taken by the waves 64 at a time
constexpr int64_t MM_HEAVY = 256;              // entries with at least this many children use the map
constexpr int MM_G = 8;                        // 64-candidate chunks loaded at once by a wave
constexpr int32_t MM_LONG = 1024;              // children with this many candidates are streamed by the whole wave
constexpr int MM_E = 16;                       // candidates a lane counts per round (a multiple of 4)
constexpr int MM_FLUSH = 252 / MM_E;           // rounds between moves of the byte counts

__device__ __forceinline__ uint32_t map_bits(const uint32_t* map, int32_t u) {
    return (map[(uint32_t)u >> 4] >> (((uint32_t)u & 15u) << 1)) & 3u;
}

// Adds this entry's (r = 0: candidates u <= v2, r = 1: above v2) counts to
// the pattern counters.  k: [0, 1] u ~ v0 and v2, [2, 3] u ~ v1 and v2,
// [4, 5] all three, [6, 7] v2's list per range; I*: list sizes per range.
__device__ __forceinline__ void motif4_classify(uint64_t (&acc)[6], const uint32_t (&k)[8],
                                                const int32_t (&I0)[2], const int32_t (&I1)[2],
                                                const int32_t (&I01)[2], int32_t v1, int32_t v2, int code) {
    const int a02 = code & 1, a12 = (code >> 1) & 1;
    const int p = a02 ? 0 : 1;
    const int32_t I2[2] = {(int32_t)k[6], (int32_t)k[7]};
    int32_t N[2][8];
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        const int32_t i02 = (int32_t)k[0 + r], i12 = (int32_t)k[2 + r], i012 = (int32_t)k[4 + r];
        N[r][0] = 0;
        N[r][7] = i012;
        N[r][3] = I01[r] - i012;
        N[r][5] = i02 - i012;
        N[r][6] = i12 - i012;
        N[r][1] = I0[r] - I01[r] - i02 + i012;
        N[r][2] = I1[r] - I01[r] - i12 + i012;
        N[r][4] = I2[r] - i02 - i12 + i012;
    }
    const int r1 = v1 > v2 ? 1 : 0, m1 = 1 | (a12 ? 4 : 0), m2 = a02 | (a12 << 1);
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int m = 0; m < 8; ++m) N[r][m] -= (int32_t)((r == r1 && m == m1) + (r == 0 && m == m2));
    const int ebits = 1 | (a02 << 1) | (a12 << 2);
#pragma unroll
    for (int m = 1; m < 8; ++m) {
        const int sbit = (m & 1) ? 0 : ((m & 2) ? 1 : 2);
        if (sbit < p) continue;
        const int64_t c = (sbit == p) ? (int64_t)N[1][m] : (int64_t)N[0][m] + N[1][m];
        const int pid = c_lut4.v[ebits | (m << 3)];
#pragma unroll
        for (int q = 0; q < 6; ++q) acc[q] += (pid == q) ? (uint64_t)c : 0ull;
    }
}

template <int LOGV>
__global__ __launch_bounds__(MM_THREADS) void k_motif_last4_map(MotifArgs A, int32_t* __restrict__ cum_all,
                                                                int64_t cum_stride) {
    constexpr int WORDS = (1 << LOGV) / 16;
    __shared__ uint32_t map[WORDS];
    __shared__ int64_t s_next[2];
    __shared__ uint32_t s_tot[MM_WAVES];
    __shared__ int32_t s_grab;
    const int w = threadIdx.x / WAVE;
    int32_t* cum = cum_all + (int64_t)blockIdx.x * cum_stride;
    const int32_t* __restrict__ col = A.col;
    for (int i = threadIdx.x; i < WORDS; i += MM_THREADS) map[i] = 0;
    // the marked lists: A0' = col[m0b, m0e), A1' = col[m1b, m1e)
    int32_t mv0 = -1, mv1 = -1;
    int64_t m0b = 0, m0e = 0, m1b = 0, m1e = 0;
    int32_t nc = 0, mna = 0;   // |A0' ∩ A1'|; |A0 above v1| (the first children, in A0's order)
    uint64_t acc[6] = {0, 0, 0, 0, 0, 0};
    uint64_t streamed = 0, n_in = 0, marked = 0;
    QueueCursor cur = queue_start();
    while (true) {
        __syncthreads();   // every wave is done with the previous chunk's s_next
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
        for (int64_t j = first; j < last; ++j) {
            const uint64_t item = (uint64_t)uniform64((int64_t)A.items[j]);
            const int64_t p = item_seg(item);
            const int32_t xa = (int32_t)item_round(item) * MM_CHILDREN;
            const int64_t b = uniform64((int64_t)(A.seg2[p] - A.seg2_base));
            const int32_t s = uniform((int32_t)(A.seg2[p + 1] - A.seg2[p]));
            if (xa >= s) continue;
            const int32_t v0 = uniform(A.l1_src[p]), v1 = uniform(A.l1_dst[p]);
            __syncthreads();   // every wave is done with the previous item's children
            if (threadIdx.x == 0) s_grab = 0;
            if (v0 != mv0 || v1 != mv1) {
                // L1 entries are the rows' upper halves in order: A0 above v0
                // starts where v0's entries begin to count, and v1 sits at the
                // entry's rank among them; v0's place in v1's row is stored
                const int64_t s0 = uniform64(A.l1_seg[v0]), s0e = uniform64(A.l1_seg[v0 + 1]);
                const int64_t r1 = uniform64(A.rp[v0 + 1]);
                const int64_t q0 = uniform64(A.rp[v1]), q1 = uniform64(A.rp[v1 + 1]);
                const int64_t a0b = r1 - (s0e - s0);
                const int64_t a1b = q0 + uniform(A.l1_rev[p]);
                if (v0 != mv0) {
                    for (int64_t t = m0b + threadIdx.x; t < m0e; t += MM_THREADS) map[(uint32_t)col[t] >> 4] = 0u;
                    for (int64_t t = m1b + threadIdx.x; t < m1e; t += MM_THREADS) map[(uint32_t)col[t] >> 4] = 0u;
                    __syncthreads();
                    for (int64_t t = a0b + threadIdx.x; t < r1; t += MM_THREADS) {
                        const uint32_t u = (uint32_t)col[t];
                        atomicOr(&map[u >> 4], 1u << ((u & 15u) << 1));
                    }
                    marked += (uint64_t)(r1 - a0b);
                } else {
                    for (int64_t t = m1b + threadIdx.x; t < m1e; t += MM_THREADS) {
                        const uint32_t u = (uint32_t)col[t];
                        atomicAnd(&map[u >> 4], ~(2u << ((u & 15u) << 1)));
                    }
                }
                __syncthreads();
                for (int64_t t = a1b + threadIdx.x; t < q1; t += MM_THREADS) {
                    const uint32_t u = (uint32_t)col[t];
                    atomicOr(&map[u >> 4], 2u << ((u & 15u) << 1));
                }
                marked += (uint64_t)(q1 - a1b);
                __syncthreads();
                // cum over A1' in MM_WAVES slices: counts, then positions
                const int32_t d1p = (int32_t)(q1 - a1b);
                const int32_t per = (d1p + MM_WAVES - 1) / MM_WAVES;
                const int32_t sb = min(w * per, d1p), se = min(sb + per, d1p);
                uint32_t c = 0;
                for (int32_t t0 = sb; t0 < se; t0 += WAVE) {
                    const int32_t t = t0 + lane();
                    const bool h = t < se && (map_bits(map, col[a1b + (t < se ? t : sb)]) & 1u);
                    c += (uint32_t)popc64(ballot(h));
                }
                if (lane() == 0) s_tot[w] = c;
                __syncthreads();
                uint32_t base = 0, total = 0;
                for (int k = 0; k < MM_WAVES; ++k) {
                    const uint32_t tk = s_tot[k];
                    base += k < w ? tk : 0u;
                    total += tk;
                }
                for (int32_t t0 = sb; t0 < se; t0 += WAVE) {
                    const int32_t t = t0 + lane();
                    const bool h = t < se && (map_bits(map, col[a1b + (t < se ? t : sb)]) & 1u);
                    const uint64_t B = ballot(h);
                    if (t < se) cum[t] = (int32_t)(base + (uint32_t)popc64(B & lanemask_lt()));
                    base += (uint32_t)popc64(B);
                }
                if (threadIdx.x == 0) cum[d1p] = (int32_t)total;
                __syncthreads();
                mv0 = v0;
                mv1 = v1;
                m0b = a0b;
                m0e = r1;
                m1b = a1b;
                m1e = q1;
                nc = (int32_t)total;
                mna = (int32_t)(s0e - p - 1);   // A0's elements above v1
            }
            __syncthreads();   // the counter is reset (and the marks are in place)
            const int32_t xend = min(xa + MM_CHILDREN, s);
            while (true) {
                // the wave's next 64 children [xw, xe)
                int32_t g = 0;
                if (lane() == 0) g = atomicAdd(&s_grab, 1);
                const int32_t xw = xa + uniform(bcast(g, 0)) * WAVE;
                if (xw >= xend) break;
                const int32_t xe = min(xw + WAVE, xend);
                const int32_t x = xw + lane();
                const bool valid = x < xe;
                int32_t v2 = 0, code = 0;
                int64_t lo2 = 0, s1 = 0;
                int32_t I0[2] = {0, 0}, I1[2] = {0, 0}, I01[2] = {0, 0};
                if (valid) {
                    v2 = A.vid2[b + x];
                    // the first mna children are A0's (code bit 0), and v2 ~ v1
                    // is bit 1 of v2's pair in the map; the others are A1's only
                    code = x < mna ? (1 | (int32_t)(map_bits(map, v2) & 2u)) : 2;
                    const int64_t s0 = A.rp[v2];
                    s1 = A.rp[v2 + 1];
                    lo2 = upper_bound(col, s0, s1, v0);
                    // the first mna children are A0's elements above v1, in order
                    const int64_t u0 = x < mna ? m0e - mna + x + 1 : upper_bound(col, m0b, m0e, v2);
                    const int64_t u1 = upper_bound(col, m1b, m1e, v2);
                    I0[0] = (int32_t)(u0 - m0b);
                    I0[1] = (int32_t)(m0e - u0);
                    I1[0] = (int32_t)(u1 - m1b);
                    I1[1] = (int32_t)(m1e - u1);
                    I01[0] = cum[u1 - m1b];
                    I01[1] = nc - I01[0];
                }
                // candidates: v2's list above v0
                const int32_t len = (int32_t)(s1 - lo2);
                uint32_t k[8] = {0, 0, 0, 0, 0, 0, 0, 0};
                // children with fewer than MM_LONG candidates: the lane streams
                // its own list, MM_E candidates (16-byte loads) at a time.  The
                // children of an entry come in the order of their names, which is
                // the order of decreasing degree, so the lists of a group of 64
                // are of similar lengths.  A candidate u falls in one of eight
                // classes (u above v2 or not, times its two map bits); the lane
                // counts them in the eight bytes of a 64-bit word, one class bit
                // per candidate, and moves the bytes to 32-bit counts every
                // MM_FLUSH rounds (at most 252 per byte).  Lanes past the list
                // take vertex 0 (no bits, not above v2): its class is never read.
                {
                    const int32_t te = (valid && len < MM_LONG) ? len : 0;
                    const int32_t nit = (te + MM_E - 1) / MM_E;
                    const int32_t* cp = col + lo2;
                    uint32_t n8[8] = {0, 0, 0, 0, 0, 0, 0, 0};
                    int32_t i = 0;
                    // the next block is loaded before the current one is counted
                    // (it ends at most 2 * MM_E - 1 entries past the list: within
                    // the zeroed tail)
                    int32_t nu[MM_E];
                    __builtin_memcpy(nu, cp, 4 * MM_E);
                    while (ballot(i < nit)) {
                        uint64_t acc = 0;
                        const int32_t stop = i + MM_FLUSH;
                        do {
                            if (i < nit) {
                                int32_t u[MM_E];
#pragma unroll
                                for (int q = 0; q < MM_E; ++q) u[q] = nu[q];
                                __builtin_memcpy(nu, cp + MM_E * (i + 1), 4 * MM_E);
                                const int32_t r = te - MM_E * i;
#pragma unroll
                                for (int q = 1; q < MM_E; ++q) u[q] = r > q ? u[q] : 0;
                                uint32_t mw[MM_E];
#pragma unroll
                                for (int q = 0; q < MM_E; ++q) mw[q] = map[(uint32_t)u[q] >> 4];
#pragma unroll
                                for (int q = 0; q < MM_E; ++q) {
                                    // v_bfe takes the low five bits of its offset: 2 * (u mod 16)
                                    const uint32_t bits = __builtin_amdgcn_ubfe(mw[q], (uint32_t)u[q] << 1, 2u);
                                    const uint32_t sh = (bits << 3) | (u[q] > v2 ? 32u : 0u);
                                    acc += 1ull << sh;
                                }
                            }
                            ++i;
                        } while (i < stop && ballot(i < nit));
#pragma unroll
                        for (int c = 0; c < 8; ++c) n8[c] += (uint32_t)(acc >> (8 * c)) & 255u;
                    }
                    // class c = 4 * above + bits; bit 0: u ~ v0, bit 1: u ~ v1
                    k[0] += n8[1] + n8[3];
                    k[1] += n8[5] + n8[7];
                    k[2] += n8[2] + n8[3];
                    k[3] += n8[6] + n8[7];
                    k[4] += n8[3];
                    k[5] += n8[7];
                    k[7] += n8[4] + n8[5] + n8[6] + n8[7];
                }
                // long children: the wave streams their lists as one sequence of
                // 64-candidate chunks, MM_G chunks (of one or several children)
                // loaded before any is counted.  A chunk is read from a uniform
                // base with one lane offset (the column array has a zeroed tail of
                // 64 entries, so the lanes past a list read in bounds) and those
                // lanes then take vertex 0, which is never marked and lies below
                // every v2; all map words of the group are read before any is
                // used.  A chunk adds to its child's lane the candidates above v2
                // and, per range, those adjacent to v0, to v1 and to both; the
                // candidates at or below v2 follow from the list length.
                uint64_t longm = ballot(valid && len >= MM_LONG);
                int cxi = -1;
                const int32_t* cb = col;   // the current child's list (wave-uniform)
                int32_t co = 0, cl = 0;    // its next chunk and length
                int32_t cv2 = 0;
                auto next_child = [&]() {
                    cxi = -1;
                    if (longm) {
                        cxi = __builtin_ctzll(longm);
                        longm &= longm - 1;
                        cb = col + (int64_t)readlane64((uint64_t)lo2, cxi);
                        cl = readlane(len, cxi);
                        cv2 = readlane(v2, cxi);
                        co = 0;
                    }
                };
                next_child();
                while (cxi >= 0) {
                    int qx[MM_G];
                    int32_t qn[MM_G], qv[MM_G];
                    const int32_t* qp[MM_G];
#pragma unroll
                    for (int q = 0; q < MM_G; ++q) {
                        qx[q] = cxi;
                        qn[q] = cxi < 0 ? 0 : min(WAVE, cl - co);
                        qp[q] = cxi < 0 ? col : cb + co;
                        qv[q] = cv2;
                        if (cxi >= 0) {
                            co += WAVE;
                            if (co >= cl) next_child();
                        }
                    }
                    int32_t u[MM_G];
#pragma unroll
                    for (int q = 0; q < MM_G; ++q) u[q] = qp[q][lane()];
                    uint32_t mw[MM_G];
#pragma unroll
                    for (int q = 0; q < MM_G; ++q) {
                        u[q] = lane() < qn[q] ? u[q] : 0;
                        mw[q] = map[(uint32_t)u[q] >> 4];
                    }
#pragma unroll
                    for (int q = 0; q < MM_G; ++q) {
                        if (qx[q] < 0) continue;   // an unused slot of the last group
                        const uint32_t bits = mw[q] >> (((uint32_t)u[q] & 15u) << 1);
                        const uint64_t B0 = ballot(bits & 1u), B1 = ballot(bits & 2u);
                        const uint64_t Hi = ballot(u[q] > qv[q]);
                        const uint64_t B01 = B0 & B1;
                        if (lane() == qx[q]) {
                            k[0] += (uint32_t)popc64(B0 & ~Hi);
                            k[1] += (uint32_t)popc64(B0 & Hi);
                            k[2] += (uint32_t)popc64(B1 & ~Hi);
                            k[3] += (uint32_t)popc64(B1 & Hi);
                            k[4] += (uint32_t)popc64(B01 & ~Hi);
                            k[5] += (uint32_t)popc64(B01 & Hi);
                            k[7] += (uint32_t)popc64(Hi);
                        }
                    }
                }
                if (valid) k[6] = (uint32_t)len - k[7];
                if (valid) {
                    streamed += (uint64_t)len;
                    n_in += 1;
                    motif4_classify(acc, k, I0, I1, I01, v1, v2, code);
                }
            }   // groups of 64 children
        }
    }
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        const uint64_t v = wave_sum_u64(acc[c]);
        if (lane() == 0 && v) atomicAdd(&A.out[c], (unsigned long long)v);
    }
    const uint64_t st = wave_sum_u64(streamed), ni = wave_sum_u64(n_in);
    if (lane() == 0) {
        if (st) atomicAdd(&A.out[9], (unsigned long long)st);
        if (ni) atomicAdd(&A.out[10], (unsigned long long)ni);
        if (w == 0 && marked) atomicAdd(&A.out[11], (unsigned long long)marked);
    }
}

// ------------------------------------------------------- last level, k = 5
//
// Five vertices: a pattern is the 10-bit mask of adjacent position pairs,
// bit b(b-1)/2 + a for a < b (the 4-vertex order followed by 04, 14, 24,
// 34).  Classes are the 21 connected graphs numbered by (edge count,
// smallest mask over the relabellings of the positions); the table maps a
// mask to its class (-1 when disconnected).
//
// Level 3 (four vertices) is not materialised.  A wave takes 64 L2 entries
// (v0, v1, v2) of one L1 entry (v0, v1), one per lane.  In rounds, every
// lane walks its entry's canonical extensions u by the rule above and
// queues each (v2, u, pair mask, p(3)) in the wave's LDS queue until the
// queue is full (a lane whose push does not fit retries that u in the next
// round); then the lanes take the queued 4-sets one each, walk their
// canonical extensions w and add one to the class of each 10-bit mask.  So
// lanes wait on the degrees of single 4-sets, not of whole subtrees.
// Adjacency is a binary search in the CSR.

constexpr int M5_Q = 512;       // queued 4-sets per wave
constexpr int M5_STAGE = 256;   // lists of v0 and v1 up to this long are staged in LDS

struct M5Lds {
    int32_t s0[MO_WAVES][M5_STAGE];
    int32_t s1[MO_WAVES][M5_STAGE];
    int32_t v2[MO_WAVES][M5_Q];
    int32_t u[MO_WAVES][M5_Q];
    int32_t m[MO_WAVES][M5_Q];   // pair mask of the 4-set | p(3) << 8
    uint32_t n[MO_WAVES];
    unsigned long long cnt[21];
};

__device__ __forceinline__ bool adj_g(const MotifArgs& A, int32_t a, int32_t u) {
    const int64_t r0 = A.rp[a];
    return member(A.col + r0, (int32_t)(A.rp[a + 1] - r0), u);
}

// the lists of v0 and v1 (shared by the wave's entries): LDS copies or the CSR
struct M5Lists {
    const int32_t* l0;
    const int32_t* l1;
    int32_t d0, d1;
};

// canonical extensions w of the 4-set (v0, v1, x2, x3) with pair mask m4 and
// p(3) = p3, from the lists of positions p3..3
__device__ __forceinline__ void last5_walk(const MotifArgs& A, const M5Lists& S, const int8_t* __restrict__ lut,
                                           int32_t v0, int32_t v1, int32_t x2, int32_t x3, int m4, int p3,
                                           unsigned long long* cnt, uint64_t& walked) {
    for (int J = p3; J < 4; ++J) {
        const int32_t xj = J == 0 ? v0 : (J == 1 ? v1 : (J == 2 ? x2 : x3));
        const int64_t t0 = A.rp[xj], t1 = A.rp[xj + 1];
        walked += (uint64_t)(t1 - t0);
        for (int64_t t = t0; t < t1; ++t) {
            const int32_t w = A.col[t];
            if (w <= v0 || w == v1 || w == x2 || w == x3) continue;
            if (J == p3 && w <= x3) continue;
            if (J > 0 && member(S.l0, S.d0, w)) continue;
            if (J > 1 && member(S.l1, S.d1, w)) continue;
            if (J > 2 && adj_g(A, x2, w)) continue;
            const int a0 = J == 0 ? 1 : 0;
            const int a1 = J == 1 ? 1 : (J < 1 ? (int)member(S.l1, S.d1, w) : 0);
            const int a2 = J == 2 ? 1 : (J < 2 ? (int)adj_g(A, x2, w) : 0);
            const int a3 = J == 3 ? 1 : (int)adj_g(A, x3, w);
            const int c = lut[m4 | (a0 << 6) | (a1 << 7) | (a2 << 8) | (a3 << 9)];
            if (c >= 0) atomicAdd(&cnt[c], 1ull);   // always connected; the test keeps LDS in bounds
        }
    }
}

__global__ __launch_bounds__(MO_THREADS) void k_motif_last5(MotifArgs A, const int8_t* __restrict__ lut) {
    __shared__ M5Lds L;
    const int w = threadIdx.x / WAVE;
    for (int i = threadIdx.x; i < 21; i += blockDim.x) L.cnt[i] = 0;
    __syncthreads();
    uint64_t walked = 0, n2 = 0, n3 = 0;   // work record: list elements walked, entries
    QueueCursor cur = queue_start();
    int64_t it_end = 0;
    for (int64_t it = queue_next(A.Q, cur, it_end); it >= 0; it = queue_next(A.Q, cur, it_end)) {
        for (int64_t j = it; j < it_end; ++j) {
            const uint64_t item = A.items[j];
            const int64_t p = item_seg(item);
            const int32_t x = (int32_t)item_round(item) * WAVE + lane();
            const int32_t s = (int32_t)(A.seg2[p + 1] - A.seg2[p]);
            const int32_t v0 = A.l1_src[p], v1 = A.l1_dst[p];
            M5Lists S;
            {
                const int64_t r0 = A.rp[v0], q0 = A.rp[v1];
                S.d0 = (int32_t)(A.rp[v0 + 1] - r0);
                S.d1 = (int32_t)(A.rp[v1 + 1] - q0);
                S.l0 = A.col + r0;
                S.l1 = A.col + q0;
                if (S.d0 <= M5_STAGE) {
                    for (int i = lane(); i < S.d0; i += WAVE) L.s0[w][i] = A.col[r0 + i];
                    S.l0 = &L.s0[w][0];
                }
                if (S.d1 <= M5_STAGE) {
                    for (int i = lane(); i < S.d1; i += WAVE) L.s1[w][i] = A.col[q0 + i];
                    S.l1 = &L.s1[w][0];
                }
                __threadfence_block();
                wave_sync();
            }
            bool done = x >= s;
            int32_t v2 = 0;
            int m3 = 0, I = 3;
            int64_t t = 0, t1 = 0;
            if (!done) {
                const int64_t e = (int64_t)(A.seg2[p] - A.seg2_base) + x;
                v2 = A.vid2[e];
                const int code = A.code2[e];
                m3 = 1 | ((code & 1) << 1) | (((code >> 1) & 1) << 2);
                I = (code & 1) ? 0 : 1;   // p(2): v2's first adjacent position
                const int32_t vi = I == 0 ? v0 : v1;
                t = A.rp[vi];
                t1 = A.rp[vi + 1];
                walked += (uint64_t)(t1 - t);
                ++n2;
            }
            const int p2 = (I == 0) ? 0 : 1;
            while (ballot(!done) != 0ull) {
                if (lane() == 0) L.n[w] = 0u;
                __threadfence_block();
                wave_sync();
                // level 3: queue extensions u until the queue is full
                while (!done) {
                    if (t >= t1) {   // the next list: positions I + 1 .. 2
                        if (++I > 2) {
                            done = true;
                            break;
                        }
                        const int32_t vi = I == 1 ? v1 : v2;
                        t = A.rp[vi];
                        t1 = A.rp[vi + 1];
                        walked += (uint64_t)(t1 - t);
                        continue;
                    }
                    const int32_t u = A.col[t];
                    bool ok = u > v0 && u != v1 && u != v2 && !(I == p2 && u <= v2);
                    ok = ok && !(I > 0 && member(S.l0, S.d0, u)) && !(I > 1 && member(S.l1, S.d1, u));
                    if (ok) {
                        const int a0 = I == 0 ? 1 : 0;
                        const int a1 = I == 1 ? 1 : (I < 1 ? (int)member(S.l1, S.d1, u) : 0);
                        const int a2 = I == 2 ? 1 : (int)adj_g(A, v2, u);
                        const uint32_t slot = atomicAdd(&L.n[w], 1u);
                        if (slot >= (uint32_t)M5_Q) break;   // full: retry u next round
                        L.v2[w][slot] = v2;
                        L.u[w][slot] = u;
                        L.m[w][slot] = (m3 | (a0 << 3) | (a1 << 4) | (a2 << 5)) | (I << 8);
                        ++n3;
                    }
                    ++t;
                }
                __threadfence_block();
                wave_sync();
                // level 4: one queued 4-set per lane
                const uint32_t nq = min(L.n[w], (uint32_t)M5_Q);
                for (uint32_t q = lane(); q < nq; q += WAVE) {
                    const int mq = L.m[w][q];
                    last5_walk(A, S, lut, v0, v1, L.v2[w][q], L.u[w][q], mq & 255, mq >> 8, L.cnt, walked);
                }
                wave_sync();
            }
            wave_sync();   // the next item overwrites the staged lists
        }
    }
    const uint64_t ws = wave_sum_u64(walked), s2 = wave_sum_u64(n2), s3 = wave_sum_u64(n3);
    if (lane() == 0) {
        if (ws) atomicAdd(&A.out[24], (unsigned long long)ws);
        if (s2) atomicAdd(&A.out[25], (unsigned long long)s2);
        if (s3) atomicAdd(&A.out[26], (unsigned long long)s3);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < 21; i += blockDim.x)
        if (L.cnt[i]) atomicAdd(&A.out[i], L.cnt[i]);
}

// The 1024-entry class table of five vertices (see above), built once.
struct Lut5 {
    int8_t v[1024];
};

static const Lut5& lut5_host() {
    static const Lut5 t = [] {
        Lut5 r{};
        int pos[5] = {0, 1, 2, 3, 4};
        int best[1024];
        for (int m = 0; m < 1024; ++m) best[m] = 1024;
        do {   // every relabelling of the positions
            for (int m = 0; m < 1024; ++m) {
                int q = 0;
                for (int b = 1; b < 5; ++b)
                    for (int a = 0; a < b; ++a) {
                        if (!((m >> (b * (b - 1) / 2 + a)) & 1)) continue;
                        const int x = std::min(pos[a], pos[b]), y = std::max(pos[a], pos[b]);
                        q |= 1 << (y * (y - 1) / 2 + x);
                    }
                best[m] = std::min(best[m], q);
            }
        } while (std::next_permutation(pos, pos + 5));
        std::vector<int> classes;
        std::vector<bool> conn(1024);
        for (int m = 0; m < 1024; ++m) {
            int reach = 1;   // vertices reachable from position 0
            for (int round = 0; round < 4; ++round)
                for (int b = 1; b < 5; ++b)
                    for (int a = 0; a < b; ++a)
                        if (((m >> (b * (b - 1) / 2 + a)) & 1) && ((reach >> a) & 1 || (reach >> b) & 1))
                            reach |= (1 << a) | (1 << b);
            conn[m] = reach == 31;
            if (conn[m] && best[m] == m) classes.push_back(m);
        }
        std::sort(classes.begin(), classes.end(), [](int a, int b) {
            const int ea = __builtin_popcount(a), eb = __builtin_popcount(b);
            return ea != eb ? ea < eb : a < b;
        });
        for (int m = 0; m < 1024; ++m) {
            r.v[m] = -1;
            if (!conn[m]) continue;
            const auto it = std::lower_bound(classes.begin(), classes.end(), best[m], [](int a, int b) {
                const int ea = __builtin_popcount(a), eb = __builtin_popcount(b);
                return ea != eb ? ea < eb : a < b;
            });
            r.v[m] = (int8_t)(it - classes.begin());
        }
        return r;
    }();
    return t;
}

// ------------------------------------------------------------------ host

struct MotifRun {
    pg_graph* g;
    hipStream_t s;
    unsigned long long* out;    // 16 counters
    unsigned long long* qctr;
    int64_t waves;
    int blocks;
};

static MotifArgs base_args(const MotifView& V) {
    MotifArgs A{};
    A.rp = V.rp;
    A.col = V.col;
    A.l1_seg = V.ml1->seg.as<int64_t>();
    A.l1_src = V.ml1->src.as<int32_t>();
    A.l1_dst = V.ml1->dst.as<int32_t>();
    A.l1_rev = V.ml1->rev.as<int32_t>();
    A.heavy_min = UINT64_MAX;
    A.hub_id = V.ml1->hub_id.as<int32_t>();
    A.hub_bits = V.ml1->hub_bits.as<uint32_t>();
    A.hub_words = V.ml1->hub_words;
    return A;
}

__global__ __launch_bounds__(256) void k_hub_rows(int64_t n_hubs, const int32_t* __restrict__ hubs,
                                                  const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                                                  int64_t words, uint32_t* __restrict__ bits) {
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x / WAVE);
    for (int64_t h = blockIdx.x * (int64_t)(blockDim.x / WAVE) + threadIdx.x / WAVE; h < n_hubs; h += waves) {
        const int32_t v = hubs[h];
        uint32_t* row = bits + h * words;
        for (int64_t j = rp[v] + lane(); j < rp[v + 1]; j += WAVE) {
            const uint32_t u = (uint32_t)col[j];
            atomicOr(row + (u >> 5), 1u << (u & 31));
        }
    }
}

// Dense adjacency rows for the vertices whose lists are too long to stage in
// LDS (degree > MO_STAGE), within a memory cap (the highest degrees first
// when the cap binds).
static void build_hubs(pg_graph* g, const MotifView& V) {
    MotifL1& L = *V.ml1;
    if (L.hubs_built) return;
    hipStream_t s = g->stream;
    const int64_t n = V.n;
    std::vector<int64_t> hrp((size_t)n + 1);
    PG_HIP(hipMemcpyAsync(hrp.data(), V.rp, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToHost, s));
    PG_HIP(hipStreamSynchronize(s));
    const int64_t words = (n + 31) / 32;
    const uint64_t cap = std::min<uint64_t>(uint64_t(2) << 30, std::max<uint64_t>(g->budget / 8, 1));
    int64_t thr = MO_STAGE + 1;
    std::vector<int32_t> hubs;
    while (true) {
        hubs.clear();
        for (int64_t v = 0; v < n; ++v)
            if (hrp[v + 1] - hrp[v] >= thr) hubs.push_back((int32_t)v);
        if ((uint64_t)hubs.size() * (uint64_t)words * 4 <= cap) break;
        thr *= 2;
    }
    std::vector<int32_t> id((size_t)std::max<int64_t>(n, 1), -1);
    for (size_t h = 0; h < hubs.size(); ++h) id[(size_t)hubs[h]] = (int32_t)h;
    L.hub_id.reserve(sizeof(int32_t) * id.size());
    PG_HIP(hipMemcpyAsync(L.hub_id.p, id.data(), sizeof(int32_t) * id.size(), hipMemcpyHostToDevice, s));
    L.n_hubs = (int64_t)hubs.size();
    L.hub_words = words;
    L.hub_bits.reserve(sizeof(uint32_t) * std::max<int64_t>(L.n_hubs * words, 1));
    if (L.n_hubs > 0) {
        DevBuf hl;
        hl.reserve(sizeof(int32_t) * hubs.size());
        PG_HIP(hipMemcpyAsync(hl.p, hubs.data(), sizeof(int32_t) * hubs.size(), hipMemcpyHostToDevice, s));
        fill_u32(L.hub_bits.as<uint32_t>(), L.n_hubs * words, 0, s);
        k_hub_rows<<<(unsigned)std::min<int64_t>((L.n_hubs + 3) / 4, 4096), 256, 0, s>>>(
            L.n_hubs, hl.as<int32_t>(), V.rp, V.col, words, L.hub_bits.as<uint32_t>());
        PG_HIP(hipGetLastError());
        PG_HIP(hipStreamSynchronize(s));
    }
    PG_HIP(hipStreamSynchronize(s));
    L.hubs_built = true;
}

static void set_queue(MotifRun& R, MotifArgs& A, const uint64_t* items, int64_t n_items) {
    fill_u64(reinterpret_cast<uint64_t*>(R.qctr), Q_WORDS, 0, R.s);
    A.Q.next = R.qctr;
    A.Q.n_items = n_items;
    A.Q.chunk = n_items >= R.waves * 64 ? 4 : 1;
    A.items = items;
    A.out = R.out;
}

// a level-1 pass over the vertices [v_lo, v_hi), in items of 64 L1 entries
template <int MODE>
static void launch_l1(MotifRun& R, MotifArgs A, int64_t v_lo, int64_t v_hi, const char* name, double units) {
    if (v_hi <= v_lo) return;
    Arena& ar = R.g->arena;
    const size_t mk = ar.mark();
    uint64_t* items = nullptr;
    const int64_t m = round_items(A.l1_seg, v_lo, v_hi - v_lo, WAVE, ar, R.s, &items);
    if (m > 0) {
        set_queue(R, A, items, m);
        ProfScope ps(name, R.s, units);
        k_motif_l1<MODE><<<R.blocks, MO_THREADS, 0, R.s>>>(A);
        PG_HIP(hipGetLastError());
    }
    ar.reset(mk);
}

// first vertex whose L1 segment holds entry x: largest v with l1_seg[v] <= x
__global__ void k_vertex_of_entry(const int64_t* __restrict__ seg, int64_t n, const int64_t* __restrict__ xs,
                                  int64_t nq, int64_t* __restrict__ out) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= nq) return;
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (seg[mid] <= xs[i]) lo = mid; else hi = mid - 1;
    }
    out[i] = lo;
}

__global__ void k_chunk_entries(const uint64_t* __restrict__ start, int64_t m, uint64_t cap, int64_t nb,
                                int64_t* __restrict__ out_c, uint64_t* __restrict__ out_s) {
    const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (j > nb) return;
    int64_t c;
    if (j == 0) c = 0;
    else if (j == nb) c = m;
    else {
        const uint64_t target = (uint64_t)j * cap;
        int64_t lo = 0, hi = m;
        while (lo < hi) {
            const int64_t mid = (lo + hi + 1) >> 1;
            if (start[mid] <= target) lo = mid; else hi = mid - 1;
        }
        c = lo;
    }
    out_c[j] = c;
    out_s[j] = start[c];
}

static int motif_classes(int k) {
    return k == 3 ? 2 : (k == 4 ? 6 : 21);
}

// Launch shape of the map kernel: the smallest map (2^logv vertices) that
// holds the graph, and as many workgroups as fit on the device at once.
struct MapLaunch {
    int logv = 0;        // 0: the graph is too large for a map in LDS
    int blocks = 0;
    int32_t* cum = nullptr;
    int64_t cum_stride = 0;
};

static MapLaunch plan_map(int64_t n) {
    MapLaunch M;
    int logv = 16;
    while (logv <= 19 && (int64_t(1) << logv) < n) ++logv;
    if (logv > 19) return M;
    M.logv = logv;
    int per_cu = 0;
    hipError_t e = hipSuccess;
    switch (logv) {
        case 16: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_motif_last4_map<16>, MM_THREADS, 0); break;
        case 17: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_motif_last4_map<17>, MM_THREADS, 0); break;
        case 18: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_motif_last4_map<18>, MM_THREADS, 0); break;
        default: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_motif_last4_map<19>, MM_THREADS, 0); break;
    }
    if (e != hipSuccess) {
        (void)hipGetLastError();
        per_cu = 1;
    }
    M.blocks = device_info().n_cu * std::max(1, per_cu);
    return M;
}

static void launch_map(const MapLaunch& M, const MotifArgs& L, hipStream_t s) {
    switch (M.logv) {
        case 16: k_motif_last4_map<16><<<M.blocks, MM_THREADS, 0, s>>>(L, M.cum, M.cum_stride); break;
        case 17: k_motif_last4_map<17><<<M.blocks, MM_THREADS, 0, s>>>(L, M.cum, M.cum_stride); break;
        case 18: k_motif_last4_map<18><<<M.blocks, MM_THREADS, 0, s>>>(L, M.cum, M.cum_stride); break;
        default: k_motif_last4_map<19><<<M.blocks, MM_THREADS, 0, s>>>(L, M.cum, M.cum_stride); break;
    }
    PG_HIP(hipGetLastError());
}

void count_motifs(pg_graph* g, int k, uint64_t* counts) {
    PG_REQUIRE(k >= 3 && k <= 5, PG_EUNSUPPORTED, "motif size must be 3, 4 or 5");
    // k = 4 runs on the graph renamed by decreasing degree
    const MotifView V = motif_view(g, k == 4);
    build_motif_l1(g, V);
    build_hubs(g, V);
    const int64_t E = V.ml1->n_edges;
    const int nc = motif_classes(k);
    for (int i = 0; i < nc; ++i) counts[i] = 0;
    if (E == 0) return;
    hipStream_t s = g->stream;
    Arena& ar = g->arena;
    MotifRun R;
    R.g = g;
    R.s = s;
    R.waves = grid_waves(16);
    R.blocks = (int)(R.waves / MO_WAVES);
    uint64_t* small = push<uint64_t>(ar, 32 + Q_WORDS);
    R.out = reinterpret_cast<unsigned long long*>(small);
    R.qctr = reinterpret_cast<unsigned long long*>(small + 32);
    fill_u64(small, 32, 0, s);
    // k = 5: lanes wait on dependent searches, so more waves per CU hide them
    // k = 5: as many workgroups per CU as its LDS and registers let reside,
    // up to MO5_WAVES_PER_CU waves
    int blocks5 = (int)(grid_waves(MO5_WAVES_PER_CU) / MO_WAVES);
    if (k == 5) {
        int per_cu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_motif_last5, MO_THREADS, 0) == hipSuccess &&
            per_cu > 0)
            blocks5 = device_info().n_cu * std::min(per_cu, MO5_WAVES_PER_CU / MO_WAVES);
        else
            (void)hipGetLastError();
    }
    int8_t* lut5 = nullptr;
    if (k == 5) {
        lut5 = push<int8_t>(ar, 1024);
        PG_HIP(hipMemcpyAsync(lut5, lut5_host().v, 1024, hipMemcpyHostToDevice, s));
    }
    MotifArgs A = base_args(V);
    A.x_lo = 0;
    A.x_hi = E;
    if (k == 3) {
        launch_l1<ML1_LAST3>(R, A, 0, g->n, "motif_last", 0.0);
    } else {
        // level 2: count pass -> scan -> write, in chunks of L1 entries that fit the budget
        uint32_t* cnt = push<uint32_t>(ar, E);
        uint64_t* start = push<uint64_t>(ar, E + 1);
        A.count = cnt;
        launch_l1<ML1_COUNT>(R, A, 0, g->n, "motif_count", (double)E);
        scan_u32(cnt, E, start, ar, s);
        const uint64_t total = read_u64(start + E, s);
        const int64_t scratch_per_wave = std::max<int64_t>(g->max_deg, 1);
        int32_t* scratch = push<int32_t>(ar, (size_t)(R.waves * scratch_per_wave));
        MapLaunch map;
        if (k == 4) {
            map = plan_map(V.n);
            if (map.logv > 0) {
                map.cum_stride = V.max_deg + 1;
                map.cum = push<int32_t>(ar, (size_t)map.blocks * (size_t)map.cum_stride);
            }
        }
        const uint64_t per = 5;   // vid + code per L2 entry
        const uint64_t room = g->budget > ar.mark() ? g->budget - ar.mark() : 0;
        const uint64_t cap = std::max<uint64_t>(room / per, (uint64_t)(2 * g->max_deg + 1));
        const int64_t nb = total == 0 ? 0 : (int64_t)((total + cap - 1) / cap);
        std::vector<int64_t> hc(nb + 1, 0), hv(nb + 1, 0);
        std::vector<uint64_t> hs(nb + 1, 0);
        if (nb >= 1) {
            const size_t mk = ar.mark();
            int64_t* dc = push<int64_t>(ar, nb + 1);
            uint64_t* ds = push<uint64_t>(ar, nb + 1);
            int64_t* dv = push<int64_t>(ar, nb + 1);
            k_chunk_entries<<<(unsigned)((nb + 256) / 256), 256, 0, s>>>(start, E, cap, nb, dc, ds);
            PG_HIP(hipGetLastError());
            k_vertex_of_entry<<<(unsigned)((nb + 256) / 256), 256, 0, s>>>(A.l1_seg, g->n, dc, nb + 1, dv);
            PG_HIP(hipGetLastError());
            PG_HIP(hipMemcpyAsync(hc.data(), dc, sizeof(int64_t) * (nb + 1), hipMemcpyDeviceToHost, s));
            PG_HIP(hipMemcpyAsync(hs.data(), ds, sizeof(uint64_t) * (nb + 1), hipMemcpyDeviceToHost, s));
            PG_HIP(hipMemcpyAsync(hv.data(), dv, sizeof(int64_t) * (nb + 1), hipMemcpyDeviceToHost, s));
            PG_HIP(hipStreamSynchronize(s));
            ar.reset(mk);
        }
        uint64_t biggest = 0;
        for (int64_t j = 0; j < nb; ++j) biggest = std::max<uint64_t>(biggest, hs[j + 1] - hs[j]);
        int32_t* vid2 = push<int32_t>(ar, std::max<uint64_t>(biggest, 1));
        uint8_t* code2 = push<uint8_t>(ar, std::max<uint64_t>(biggest, 1));
        for (int64_t j = 0; j < nb; ++j) {
            const int64_t c0 = hc[j], c1 = hc[j + 1];
            if (c1 <= c0) continue;
            MotifArgs W = A;
            W.x_lo = c0;
            W.x_hi = c1;
            W.start = start;
            W.start_base = hs[j];
            W.out_vid = vid2;
            W.out_code = code2;
            if (k == 4 && map.logv > 0) W.heavy_min = (uint64_t)MM_HEAVY;
            const int64_t v_lo = hv[j];
            const int64_t v_hi = (j + 1 == nb) ? g->n : std::min<int64_t>(g->n, hv[j + 1] + 1);
            launch_l1<ML1_WRITE>(R, W, v_lo, v_hi, "motif_write", (double)(hs[j + 1] - hs[j]));
            // fused last level over the L1 entries [c0, c1) (segments of L2)
            MotifArgs L = A;
            L.seg2 = start;
            L.seg2_base = hs[j];
            L.vid2 = vid2;
            L.code2 = code2;
            L.scratch = scratch;
            L.scratch_per_wave = scratch_per_wave;
            const size_t mk = ar.mark();
            uint64_t* items = nullptr;
            // k = 4: entries with many children go to the map kernel, the
            // others to the per-wave kernel
            const int64_t light_max = (k == 4 && map.logv > 0) ? MM_HEAVY : INT64_MAX;
            const int64_t m = round_items_between(start, c0, c1 - c0, WAVE, 0, light_max, ar, s, &items);
            if (m > 0) {
                set_queue(R, L, items, m);
                ProfScope ps("motif_last", s, 0.0);
                if (k == 4) k_motif_last4<<<R.blocks, MO_THREADS, 0, s>>>(L);
                else k_motif_last5<<<blocks5, MO_THREADS, 0, s>>>(L, lut5);
                PG_HIP(hipGetLastError());
            }
            if (light_max != INT64_MAX) {
                uint64_t* hitems = nullptr;
                const int64_t mh = round_items_between(start, c0, c1 - c0, MM_CHILDREN, light_max, INT64_MAX, ar, s,
                                                       &hitems);
                if (mh > 0) {
                    set_queue(R, L, hitems, mh);
                    L.Q.chunk = std::max<int64_t>(1, std::min<int64_t>(8, mh / ((int64_t)map.blocks * 4)));
                    ProfScope ps("motif_last_map", s, 0.0);
                    launch_map(map, L, s);
                }
            }
            ar.reset(mk);
        }
    }
    uint64_t h[32];
    PG_HIP(hipMemcpyAsync(h, small, sizeof(h), hipMemcpyDeviceToHost, s));
    PG_HIP(hipStreamSynchronize(s));
    for (int i = 0; i < nc; ++i) counts[i] = h[i];
    if (prof_on() && k == 4) {
        // algorithmic bytes of the fused last level.  Per-wave kernel: per
        // input embedding the SoA entry (5 B), the three row-pointer pairs
        // (48 B) and one 4-byte probe per intersection item.  Map kernel: per
        // input embedding its vertex and v2's row-pointer pair (20 B: the code
        // comes from the map) and 4 B per candidate of its list; 4 B per list
        // element marked.
        ProfScope ps("motif_last_work", s, 53.0 * (double)h[7] + 4.0 * (double)h[6]);
        ProfScope pm("motif_last_map_work", s, 20.0 * (double)h[10] + 4.0 * (double)(h[9] + h[11]));
    }
    if (prof_on() && k == 3) {
        // fused level 2: per level-1 entry v1 and its row-pointer pair
        // (20 B), 4 B per list element iterated (A0' probing A1 or A1'
        // probing A0, the cheaper), and per item v0's row pointers and list
        ProfScope ps("motif_last_work", s, 20.0 * (double)h[13] + 4.0 * (double)h[12] + 4.0 * (double)h[14]);
    }
    if (prof_on() && k == 5) {
        // k = 5: per level-2 entry its SoA entry and a row-pointer pair
        // (16 B), per level-3 extension a row-pointer pair (16 B), and 4 B
        // per element of every list walked at levels 3 and 4
        ProfScope ps("motif_last_work", s, 16.0 * (double)(h[25] + h[26]) + 4.0 * (double)h[24]);
    }
}

}  // namespace pg
