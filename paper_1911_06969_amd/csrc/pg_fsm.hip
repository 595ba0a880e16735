// Frequent subgraph mining with minimum-image (domain) support, edge-induced
// embeddings of up to three edges over a vertex-labelled graph (Pangolin
// sections 2.1-2.2, 3.3 FSM Listing, 5.3).
//
// Levels (Algorithm 1 with Reduce and Filter on, also right after Init):
//   L1  every edge e = (u < v), identified by its rank in (u, v) order;
//   Reduce L1, Filter L1 -> frequent edges;
//   L2  (e1, e2): count / scan / write from the frequent edges, each entry
//       storing its pattern id (memoisation, section 4.2);
//   Reduce L2, Filter L2 -> frequent wedges;
//   L3  generated from the frequent wedges and reduced on the fly (the last
//       level is never stored).
//
// Canonical test (isAutoCanonical for edge extension).  An embedding is kept
// only in greedy order: g1 is its smallest edge, then repeatedly the
// smallest remaining edge adjacent to those chosen.  Extending a greedy
// sequence (g1..gj) by an edge e keeps it greedy iff e is adjacent to the
// chosen edges, e > g1, and e > g_i for every i >= 2 such that e is adjacent
// to g1..g_{i-1}.
//
// Patterns are numbered by the dense index of the public header (shape,
// then labels); their vertices fall in orbits (vertices swapped by a
// label-preserving automorphism).  The domain of an orbit is the set of
// graph vertices any embedding places in it; the support of a pattern is
// the smallest orbit domain, which equals the minimum-image support over all
// subgraph isomorphisms.
//
// Reduce.  A histogram of embeddings per pattern bounds each support
// (support <= embeddings x largest orbit), so bitmaps are kept only for
// patterns that can reach the threshold; every embedding sets the bits of
// its vertices in its pattern's orbit bitmaps (one bit per graph vertex),
// and popcounts give the domain sizes.  When the bitmaps of one level do not
// fit the memory budget, the candidate patterns are processed in groups.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "pg_device.h"
#include "pg_internal.h"

namespace pg {

// ----------------------------------------------------- pattern numbering

struct PatBase {
    int64_t L;
    int64_t p2, t3, paths;
    int64_t edge, wedge, tri, path, star;
    // four edges: 5-path, 4-star, fork, 4-cycle, paw
    int64_t q4, s4n, p5n, fkn, c4n, pwn;
    int64_t p5, star4, fork, cyc, paw;
    int64_t total;
};

__host__ __device__ inline PatBase pat_base(int64_t L, int max_edges) {
    PatBase B;
    B.L = L;
    B.p2 = L * (L + 1) / 2;
    B.t3 = L * (L + 1) * (L + 2) / 6;
    B.paths = (L * L * L * L + L * L) / 2;
    B.edge = 0;
    B.wedge = B.p2;
    B.tri = B.wedge + L * B.p2;
    B.path = B.tri + B.t3;
    B.star = B.path + B.paths;
    // label multisets of four leaves; palindromic 5-sequences; cycles up to
    // rotation and reflection (Burnside over the 8 symmetries of a square)
    B.q4 = L * (L + 1) * (L + 2) * (L + 3) / 24;
    B.p5n = (L * L * L * L * L + L * L * L) / 2;
    B.s4n = L * B.q4;
    B.fkn = L * B.p2 * L * L;
    B.c4n = (L * L * L * L + 2 * L * L * L + 3 * L * L + 2 * L) / 8;
    B.pwn = L * L * B.p2;
    B.p5 = B.star + L * B.t3;
    B.star4 = B.p5 + B.p5n;
    B.fork = B.star4 + B.s4n;
    B.cyc = B.fork + B.fkn;
    B.paw = B.cyc + B.c4n;
    B.total = max_edges >= 4 ? B.paw + B.pwn
              : max_edges == 3 ? B.p5 : (max_edges == 2 ? B.tri : B.p2);
    return B;
}

// rank of a <= b among label pairs in lexicographic order
__host__ __device__ inline int64_t pair_rank(int64_t a, int64_t b, int64_t L) {
    return a * L - a * (a - 1) / 2 + (b - a);
}

// rank of a <= b <= c among sorted label triples in lexicographic order
__host__ __device__ inline int64_t triple_rank(int64_t a, int64_t b, int64_t c, int64_t L) {
    int64_t r = 0;
    for (int64_t x = 0; x < a; ++x) r += (L - x) * (L - x + 1) / 2;
    for (int64_t y = a; y < b; ++y) r += L - y;
    return r + (c - b);
}

// Largest label count for patterns of four edges: the 5-path table has
// n_labels^5 entries.
constexpr int FSM4_MAX_LABELS = 32;

uint64_t fsm_num_patterns(int max_edges, int n_labels) {
    if (max_edges < 1 || max_edges > 4 || n_labels < 1) return 0;
    if (max_edges == 4 && n_labels > FSM4_MAX_LABELS) return 0;
    return (uint64_t)pat_base(n_labels, max_edges).total;
}

// Representative label tuples of the table-ranked shapes, as host checks of
// a tuple code (digits base L, first position most significant).
static bool path_rep(int64_t x, int64_t L, int n) {   // x <= its reversal
    int64_t d[5];
    for (int i = n - 1; i >= 0; --i) { d[i] = x % L; x /= L; }
    for (int i = 0; i < n; ++i) {
        if (d[i] != d[n - 1 - i]) return d[i] < d[n - 1 - i];
    }
    return true;
}

static bool sorted_rep(int64_t x, int64_t L) {   // non-decreasing 4-tuple
    int64_t d[4];
    for (int i = 3; i >= 0; --i) { d[i] = x % L; x /= L; }
    return d[0] <= d[1] && d[1] <= d[2] && d[2] <= d[3];
}

static bool cycle_rep(int64_t x, int64_t L) {    // smallest of the 8 readings
    int64_t d[4];
    for (int i = 3; i >= 0; --i) { d[i] = x % L; x /= L; }
    for (int r = 0; r < 4; ++r)
        for (int dir = 0; dir < 2; ++dir) {
            for (int i = 0; i < 4; ++i) {
                const int64_t c = dir ? d[(r - i + 4) % 4] : d[(r + i) % 4];
                if (c != d[i]) {
                    if (c < d[i]) return false;
                    break;
                }
            }
        }
    return true;
}

// the r-th representative code of a table-ranked shape (host, by walking)
template <class Rep>
static int64_t nth_rep(int64_t r, int64_t count, Rep&& rep) {
    for (int64_t x = 0; x < count; ++x)
        if (rep(x)) {
            if (r == 0) return x;
            --r;
        }
    return -1;
}

static void digits(int64_t x, int64_t L, int n, int32_t* out) {
    for (int i = n - 1; i >= 0; --i) { out[i] = (int32_t)(x % L); x /= L; }
}

int fsm_pattern_key(uint64_t index, int max_edges, int n_labels, int* shape, int32_t* lab) {
    const PatBase B = pat_base(n_labels, max_edges);
    const int64_t L = n_labels;
    int64_t i = (int64_t)index;
    for (int j = 0; j < 5; ++j) lab[j] = -1;
    auto pair_of = [&](int64_t r, int32_t* out) {
        for (int64_t a = 0; a < L; ++a)
            for (int64_t b = a; b < L; ++b)
                if (pair_rank(a, b, L) == r) { out[0] = (int32_t)a; out[1] = (int32_t)b; return; }
    };
    auto triple_of = [&](int64_t r, int32_t* out) {
        for (int64_t a = 0; a < L; ++a)
            for (int64_t b = a; b < L; ++b)
                for (int64_t c = b; c < L; ++c)
                    if (triple_rank(a, b, c, L) == r) { out[0] = (int32_t)a; out[1] = (int32_t)b; out[2] = (int32_t)c; return; }
    };
    if (i < B.wedge) { *shape = 0; pair_of(i, lab); return PG_OK; }
    if (i < B.tri) {
        *shape = 1;
        const int64_t r = i - B.wedge;
        lab[0] = (int32_t)(r / B.p2);
        pair_of(r % B.p2, lab + 1);
        return PG_OK;
    }
    if (i < B.path) { *shape = 2; triple_of(i - B.tri, lab); return PG_OK; }
    if (i < B.star) {
        *shape = 3;
        digits(nth_rep(i - B.path, L * L * L * L, [&](int64_t x) { return path_rep(x, L, 4); }), L, 4, lab);
        return PG_OK;
    }
    if (i < B.p5) {
        *shape = 4;
        const int64_t r = i - B.star;
        lab[0] = (int32_t)(r / B.t3);
        triple_of(r % B.t3, lab + 1);
        return PG_OK;
    }
    if (i < B.star4) {
        *shape = 5;
        digits(nth_rep(i - B.p5, L * L * L * L * L, [&](int64_t x) { return path_rep(x, L, 5); }), L, 5, lab);
        return PG_OK;
    }
    if (i < B.fork) {
        *shape = 6;
        const int64_t r = i - B.star4;
        lab[0] = (int32_t)(r / B.q4);
        digits(nth_rep(r % B.q4, L * L * L * L, [&](int64_t x) { return sorted_rep(x, L); }), L, 4, lab + 1);
        return PG_OK;
    }
    if (i < B.cyc) {
        *shape = 7;
        int64_t r = i - B.fork;
        lab[4] = (int32_t)(r % L);
        r /= L;
        lab[3] = (int32_t)(r % L);
        r /= L;
        pair_of(r % B.p2, lab + 1);
        lab[0] = (int32_t)(r / B.p2);
        return PG_OK;
    }
    if (i < B.paw) {
        *shape = 8;
        digits(nth_rep(i - B.cyc, L * L * L * L, [&](int64_t x) { return cycle_rep(x, L); }), L, 4, lab);
        return PG_OK;
    }
    *shape = 9;
    const int64_t r = i - B.paw;
    pair_of(r % B.p2, lab + 2);
    lab[1] = (int32_t)((r / B.p2) % L);
    lab[0] = (int32_t)(r / B.p2 / L);
    return PG_OK;
}

// ------------------------------------------------------ device classifiers

struct FsmCtx {
    const int64_t* rp;
    const int32_t* col;
    const int32_t* eid;      // undirected edge id of every CSR entry
    const int32_t* esrc;     // edge -> smaller endpoint
    const int32_t* edst;     // edge -> larger endpoint
    const int32_t* lab;
    const int32_t* path_rank;   // rank of every canonical label sequence of a path
    // four edges (NULL below): ranks of the representative 5-paths, sorted
    // leaf quadruples and 4-cycle readings, indexed by their tuple code
    const int32_t* p5_rank;
    const int32_t* q4_rank;
    const int32_t* c4_rank;
    PatBase B;
};

constexpr int FSM_MAXV = 5;   // vertices of a pattern of at most four edges

struct Emb {
    int32_t pid;
    int nv;
    int32_t v[FSM_MAXV];
    int8_t orb[FSM_MAXV];
};

__device__ __forceinline__ void sort3(int32_t& a, int32_t& b, int32_t& c) {
    if (a > b) { int32_t t = a; a = b; b = t; }
    if (b > c) { int32_t t = b; b = c; c = t; }
    if (a > b) { int32_t t = a; a = b; b = t; }
}

// single edge (u, v)
__device__ __forceinline__ Emb classify_edge(const FsmCtx& C, int32_t u, int32_t v) {
    Emb E;
    const int32_t lu = C.lab[u], lv = C.lab[v];
    const int32_t a = min(lu, lv), b = max(lu, lv);
    E.pid = (int32_t)(C.B.edge + pair_rank(a, b, C.B.L));
    E.nv = 2;
    E.v[0] = u; E.v[1] = v;
    // equal labels: one orbit; otherwise the smaller label is orbit 0
    E.orb[0] = (lu == a) ? 0 : 1;
    E.orb[1] = (lv == a) ? 0 : 1;
    return E;
}

// wedge: centre s, leaves o and t
__device__ __forceinline__ Emb classify_wedge(const FsmCtx& C, int32_t s, int32_t o, int32_t t) {
    Emb E;
    const int32_t ls = C.lab[s], lo = C.lab[o], lt = C.lab[t];
    const int32_t a = min(lo, lt), b = max(lo, lt);
    E.pid = (int32_t)(C.B.wedge + (int64_t)ls * C.B.p2 + pair_rank(a, b, C.B.L));
    E.nv = 3;
    E.v[0] = s; E.v[1] = o; E.v[2] = t;
    // centre: orbit 0; leaves: one orbit if their labels agree, else the
    // smaller label is orbit 1
    E.orb[0] = 0;
    E.orb[1] = (lo == a) ? 1 : 2;
    E.orb[2] = (lt == a) ? 1 : 2;
    return E;
}

__device__ __forceinline__ Emb classify_triangle(const FsmCtx& C, int32_t x, int32_t y, int32_t z) {
    Emb E;
    int32_t l[3] = {C.lab[x], C.lab[y], C.lab[z]};
    int32_t a = l[0], b = l[1], c = l[2];
    sort3(a, b, c);
    E.pid = (int32_t)(C.B.tri + triple_rank(a, b, c, C.B.L));
    E.nv = 3;
    E.v[0] = x; E.v[1] = y; E.v[2] = z;
    for (int i = 0; i < 3; ++i) E.orb[i] = (l[i] == a) ? 0 : ((l[i] == b) ? 1 : 2);
    return E;
}

// star: centre s, leaves p, q, r
__device__ __forceinline__ Emb classify_star(const FsmCtx& C, int32_t s, int32_t p, int32_t q, int32_t r) {
    Emb E;
    int32_t l[3] = {C.lab[p], C.lab[q], C.lab[r]};
    int32_t a = l[0], b = l[1], c = l[2];
    sort3(a, b, c);
    E.pid = (int32_t)(C.B.star + (int64_t)C.lab[s] * C.B.t3 + triple_rank(a, b, c, C.B.L));
    E.nv = 4;
    E.v[0] = s; E.v[1] = p; E.v[2] = q; E.v[3] = r;
    E.orb[0] = 0;
    for (int i = 0; i < 3; ++i) E.orb[i + 1] = 1 + ((l[i] == a) ? 0 : ((l[i] == b) ? 1 : 2));
    return E;
}

// path w0 - w1 - w2 - w3
__device__ __forceinline__ Emb classify_path(const FsmCtx& C, int32_t w0, int32_t w1, int32_t w2, int32_t w3) {
    Emb E;
    const int64_t L = C.B.L;
    const int32_t l0 = C.lab[w0], l1 = C.lab[w1], l2 = C.lab[w2], l3 = C.lab[w3];
    const int64_t f = ((int64_t)(l0 * L + l1) * L + l2) * L + l3;
    const int64_t r = ((int64_t)(l3 * L + l2) * L + l1) * L + l0;
    E.pid = (int32_t)(C.B.path + C.path_rank[f <= r ? f : r]);
    E.nv = 4;
    E.v[0] = w0; E.v[1] = w1; E.v[2] = w2; E.v[3] = w3;
    if (f == r) {
        E.orb[0] = 0; E.orb[1] = 1; E.orb[2] = 1; E.orb[3] = 0;
    } else if (f < r) {
        E.orb[0] = 0; E.orb[1] = 1; E.orb[2] = 2; E.orb[3] = 3;
    } else {
        E.orb[0] = 3; E.orb[1] = 2; E.orb[2] = 1; E.orb[3] = 0;
    }
    return E;
}

// ----------------------------------------------- four-edge classifiers
//
// Orbits are numbered by the smallest canonical position they contain.

// 5-path w0 - w1 - w2 - w3 - w4
__device__ __forceinline__ Emb classify_path5(const FsmCtx& C, const int32_t (&w)[5]) {
    Emb E;
    const int64_t L = C.B.L;
    int32_t l[5];
    for (int i = 0; i < 5; ++i) l[i] = C.lab[w[i]];
    int64_t f = 0, r = 0;
    for (int i = 0; i < 5; ++i) {
        f = f * L + l[i];
        r = r * L + l[4 - i];
    }
    E.pid = (int32_t)(C.B.p5 + C.p5_rank[f <= r ? f : r]);
    E.nv = 5;
    const bool rev = r < f;
    for (int i = 0; i < 5; ++i) {
        E.v[i] = w[i];
        const int pos = rev ? 4 - i : i;
        E.orb[i] = (int8_t)((f == r) ? (pos < 4 - pos ? pos : 4 - pos) : pos);
    }
    return E;
}

// 4-star: centre c, leaves q[0..3]
__device__ __forceinline__ Emb classify_star4(const FsmCtx& C, int32_t c, const int32_t (&q)[4]) {
    Emb E;
    const int64_t L = C.B.L;
    int32_t l[4];
    for (int i = 0; i < 4; ++i) l[i] = C.lab[q[i]];
    int32_t t[4] = {l[0], l[1], l[2], l[3]};
    for (int i = 1; i < 4; ++i)
        for (int j = i; j > 0 && t[j - 1] > t[j]; --j) { const int32_t x = t[j]; t[j] = t[j - 1]; t[j - 1] = x; }
    const int64_t code = ((t[0] * L + t[1]) * L + t[2]) * L + t[3];
    E.pid = (int32_t)(C.B.star4 + (int64_t)C.lab[c] * C.B.q4 + C.q4_rank[code]);
    E.nv = 5;
    E.v[0] = c;
    E.orb[0] = 0;
    for (int i = 0; i < 4; ++i) {
        E.v[i + 1] = q[i];
        int first = 0;
        while (t[first] != l[i]) ++first;
        E.orb[i + 1] = (int8_t)(1 + first);   // first sorted position with this label
    }
    return E;
}

// fork: c of degree 3, its leaves a and b, the middle m of its long leg and the end e
__device__ __forceinline__ Emb classify_fork(const FsmCtx& C, int32_t c, int32_t a, int32_t b, int32_t m, int32_t e) {
    Emb E;
    const int64_t L = C.B.L;
    const int32_t la = C.lab[a], lb = C.lab[b];
    const int32_t x = min(la, lb), y = max(la, lb);
    E.pid = (int32_t)(C.B.fork + (((int64_t)C.lab[c] * C.B.p2 + pair_rank(x, y, L)) * L + C.lab[m]) * L + C.lab[e]);
    E.nv = 5;
    E.v[0] = c; E.v[1] = a; E.v[2] = b; E.v[3] = m; E.v[4] = e;
    E.orb[0] = 0;
    E.orb[1] = (la == x) ? 1 : 2;
    E.orb[2] = (lb == x) ? 1 : 2;
    E.orb[3] = 3;
    E.orb[4] = 4;
    return E;
}

// 4-cycle w0 - w1 - w2 - w3 - w0
__device__ __forceinline__ Emb classify_cycle4(const FsmCtx& C, const int32_t (&w)[4]) {
    Emb E;
    const int64_t L = C.B.L;
    int32_t l[4];
    for (int i = 0; i < 4; ++i) l[i] = C.lab[w[i]];
    // reading (r, dir): position i holds vertex (r + i) mod 4, or (r - i) mod 4
    int64_t best = -1;
    for (int r = 0; r < 4; ++r)
        for (int dir = 0; dir < 2; ++dir) {
            int64_t code = 0;
            for (int i = 0; i < 4; ++i) code = code * L + l[dir ? (r - i + 4) & 3 : (r + i) & 3];
            if (best < 0 || code < best) best = code;
        }
    E.pid = (int32_t)(C.B.cyc + C.c4_rank[best]);
    E.nv = 4;
    for (int j = 0; j < 4; ++j) {
        E.v[j] = w[j];
        E.orb[j] = 4;
    }
    // a vertex's orbit: its smallest position over the readings that give the canonical tuple
    for (int r = 0; r < 4; ++r)
        for (int dir = 0; dir < 2; ++dir) {
            int64_t code = 0;
            for (int i = 0; i < 4; ++i) code = code * L + l[dir ? (r - i + 4) & 3 : (r + i) & 3];
            if (code != best) continue;
            for (int j = 0; j < 4; ++j) {
                const int pos = dir ? (r - j + 4) & 3 : (j - r + 4) & 3;
                if (pos < E.orb[j]) E.orb[j] = (int8_t)pos;
            }
        }
    return E;
}

// paw: x of degree 3, its pendant y, the triangle's other vertices p and q
__device__ __forceinline__ Emb classify_paw(const FsmCtx& C, int32_t x, int32_t y, int32_t p, int32_t q) {
    Emb E;
    const int64_t L = C.B.L;
    const int32_t lp = C.lab[p], lq = C.lab[q];
    const int32_t a = min(lp, lq), b = max(lp, lq);
    E.pid = (int32_t)(C.B.paw + ((int64_t)C.lab[x] * L + C.lab[y]) * C.B.p2 + pair_rank(a, b, L));
    E.nv = 4;
    E.v[0] = x; E.v[1] = y; E.v[2] = p; E.v[3] = q;
    E.orb[0] = 0;
    E.orb[1] = 1;
    E.orb[2] = (lp == a) ? 2 : 3;
    E.orb[3] = (lq == a) ? 2 : 3;
    return E;
}

// Pattern of a connected set of three or four edges (graph edge ids).  The
// shape follows from the vertex count and the degrees inside the set; paths
// and cycles are walked from an end or any vertex.
__device__ __forceinline__ Emb classify_edges(const FsmCtx& C, const int32_t* es, int ne) {
    int32_t vs[FSM_MAXV];
    int deg[FSM_MAXV];
    uint32_t adj[FSM_MAXV];
    int nv = 0;
    for (int i = 0; i < FSM_MAXV; ++i) { deg[i] = 0; adj[i] = 0u; vs[i] = -1; }
    for (int k = 0; k < ne; ++k) {
        const int32_t ends[2] = {C.esrc[es[k]], C.edst[es[k]]};
        int at[2];
        for (int h = 0; h < 2; ++h) {
            int f = -1;
            for (int i = 0; i < nv; ++i)
                if (vs[i] == ends[h]) f = i;
            if (f < 0 && nv < FSM_MAXV) { f = nv; vs[nv++] = ends[h]; }
            at[h] = f < 0 ? 0 : f;
            deg[at[h]]++;
        }
        adj[at[0]] |= 1u << at[1];
        adj[at[1]] |= 1u << at[0];
    }
    int dmax = 0, imax = 0;
    for (int i = 0; i < nv; ++i)
        if (deg[i] > dmax) { dmax = deg[i]; imax = i; }
    // the other end of a walk step from `cur` that does not go back to `prev`
    auto step = [&](int cur, int prev) {
        const uint32_t m = adj[cur] & ~(prev >= 0 ? 1u << prev : 0u);
        return m ? __builtin_ctz(m) : -1;
    };
    if (ne == 3) {
        if (nv == 3) return classify_triangle(C, vs[0], vs[1], vs[2]);
        if (dmax == 3) {
            int32_t lv[3];
            int k = 0;
            for (int i = 0; i < 4; ++i)
                if (i != imax) lv[k++] = vs[i];
            return classify_star(C, vs[imax], lv[0], lv[1], lv[2]);
        }
        int e0 = 0;
        while (deg[e0] != 1) ++e0;
        int w[4];
        w[0] = e0;
        w[1] = step(w[0], -1);
        w[2] = step(w[1], w[0]);
        w[3] = step(w[2], w[1]);
        return classify_path(C, vs[w[0]], vs[w[1]], vs[w[2]], vs[w[3]]);
    }
    // four edges
    if (nv == 5) {
        if (dmax == 4) {
            int32_t q[4];
            int k = 0;
            for (int i = 0; i < 5; ++i)
                if (i != imax) q[k++] = vs[i];
            return classify_star4(C, vs[imax], q);
        }
        if (dmax == 3) {
            int leaves[2], k = 0, mid = -1;
            for (int i = 0; i < 5; ++i)
                if ((adj[imax] >> i) & 1u) {
                    if (deg[i] == 1) leaves[k++] = i;
                    else mid = i;
                }
            const int end = step(mid, imax);
            return classify_fork(C, vs[imax], vs[leaves[0]], vs[leaves[1]], vs[mid], vs[end]);
        }
        int e0 = 0;
        while (deg[e0] != 1) ++e0;
        int w[5];
        w[0] = e0;
        w[1] = step(w[0], -1);
        for (int i = 2; i < 5; ++i) w[i] = step(w[i - 1], w[i - 2]);
        const int32_t path[5] = {vs[w[0]], vs[w[1]], vs[w[2]], vs[w[3]], vs[w[4]]};
        return classify_path5(C, path);
    }
    if (dmax == 2) {
        int w[4];
        w[0] = 0;
        w[1] = step(0, -1);
        w[2] = step(w[1], w[0]);
        w[3] = step(w[2], w[1]);
        const int32_t cyc[4] = {vs[w[0]], vs[w[1]], vs[w[2]], vs[w[3]]};
        return classify_cycle4(C, cyc);
    }
    int pend = 0;
    while (deg[pend] != 1) ++pend;
    int tri[2], k = 0;
    for (int i = 0; i < 4; ++i)
        if (i != imax && i != pend) tri[k++] = i;
    return classify_paw(C, vs[imax], vs[pend], vs[tri[0]], vs[tri[1]]);
}

// ---------------------------------------------------------------- kernels

__global__ void k_path_flags(int64_t L, uint32_t* __restrict__ flag) {
    const int64_t N = L * L * L * L;
    for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < N; x += (int64_t)gridDim.x * blockDim.x) {
        const int64_t a = x / (L * L * L), b = (x / (L * L)) % L, c = (x / L) % L, d = x % L;
        const int64_t rev = ((d * L + c) * L + b) * L + a;
        flag[x] = x <= rev ? 1u : 0u;
    }
}

// representative flags of the table-ranked shapes of four edges (see
// path_rep / sorted_rep / cycle_rep on the host)
enum { REP_PATH5 = 0, REP_SORTED4 = 1, REP_CYCLE4 = 2 };

__global__ void k_rep_flags(int64_t L, int kind, int64_t N, uint32_t* __restrict__ flag) {
    for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < N; x += (int64_t)gridDim.x * blockDim.x) {
        const int n = kind == REP_PATH5 ? 5 : 4;
        int64_t d[5];
        int64_t y = x;
        for (int i = n - 1; i >= 0; --i) { d[i] = y % L; y /= L; }
        bool rep = true;
        if (kind == REP_PATH5) {
            for (int i = 0; i < n; ++i)
                if (d[i] != d[n - 1 - i]) { rep = d[i] < d[n - 1 - i]; break; }
        } else if (kind == REP_SORTED4) {
            rep = d[0] <= d[1] && d[1] <= d[2] && d[2] <= d[3];
        } else {
            for (int r = 0; r < 4 && rep; ++r)
                for (int dir = 0; dir < 2 && rep; ++dir)
                    for (int i = 0; i < 4; ++i) {
                        const int64_t c = dir ? d[(r - i + 4) & 3] : d[(r + i) & 3];
                        if (c != d[i]) {
                            rep = c > d[i];
                            break;
                        }
                    }
        }
        flag[x] = rep ? 1u : 0u;
    }
}

__global__ void k_u64_to_i32(int64_t n, const uint64_t* __restrict__ in, int32_t* __restrict__ out) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = (int32_t)in[i];
}

// undirected edge id of every CSR entry: entry (u, w) with w > u is edge
// seg[u] + its position among u's larger neighbours; w < u takes the id of
// the mirrored entry.
__global__ __launch_bounds__(256) void k_edge_ids(int64_t n, const int64_t* __restrict__ rp,
                                                  const int32_t* __restrict__ col,
                                                  const int64_t* __restrict__ seg, int32_t* __restrict__ eid) {
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x / WAVE);
    for (int64_t u = blockIdx.x * (int64_t)(blockDim.x / WAVE) + threadIdx.x / WAVE; u < n; u += waves) {
        const int64_t r0 = rp[u], r1 = rp[u + 1];
        const int64_t up_u = r1 - (seg[u + 1] - seg[u]);   // first entry above u
        for (int64_t j = r0 + lane(); j < r1; j += WAVE) {
            const int32_t w = col[j];
            if (w > u) {
                eid[j] = (int32_t)(seg[u] + (j - up_u));
            } else {
                const int64_t q1 = rp[w + 1];
                const int64_t up_w = q1 - (seg[w + 1] - seg[w]);
                const int64_t pos = lower_bound(col, up_w, q1, (int32_t)u);
                eid[j] = (int32_t)(seg[w] + (pos - up_w));
            }
        }
    }
}

// Histogram of m values into counts[].  Values in [lo, lo + nb) with nb <=
// HIST_LDS bins gather in a histogram of the workgroup's own in LDS (few
// global counters would otherwise take every element's atomic), which is
// added to counts once per workgroup; other values go to counts directly.
constexpr int HIST_LDS = 8192;

__global__ __launch_bounds__(256) void k_hist(int64_t m, const int32_t* __restrict__ val, uint32_t* __restrict__ counts,
                                              int32_t lo, int32_t nb) {
    __shared__ uint32_t h[HIST_LDS];
    const bool local = nb <= HIST_LDS;
    if (local) {
        for (int b = threadIdx.x; b < nb; b += blockDim.x) h[b] = 0u;
        __syncthreads();
    }
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t v = val[i];
        const uint32_t b = (uint32_t)(v - lo);
        if (local && b < (uint32_t)nb) atomicAdd(&h[b], 1u);
        else atomicAdd(&counts[v], 1u);
    }
    if (local) {
        __syncthreads();
        for (int b = threadIdx.x; b < nb; b += blockDim.x)
            if (h[b]) atomicAdd(&counts[lo + b], h[b]);
    }
}

static unsigned hist_blocks(int64_t m) {
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>((m + 255) / 256, (int64_t)device_info().n_cu * 2));
}

// candidate flag: the pattern has enough embeddings to possibly reach sigma
__global__ void k_candidates(int64_t np, int64_t p_lo, const uint32_t* __restrict__ counts, PatBase B,
                             uint64_t sigma, uint32_t* __restrict__ flag) {
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < np; p += (int64_t)gridDim.x * blockDim.x) {
        // dense index: triangles and 3-stars have orbits of up to 3 vertices,
        // 4-stars and 4-cycles of up to 4
        const int64_t q = p + p_lo;
        const uint64_t maxorb = (q >= B.star4 && q < B.fork) || (q >= B.cyc && q < B.paw) ? 4
                                : ((q >= B.tri && q < B.path) || (q >= B.star && q < B.p5) ? 3 : 2);
        flag[p] = (counts[p] > 0 && (uint64_t)counts[p] * maxorb >= sigma) ? 1u : 0u;
    }
}

__global__ void k_slots(int64_t np, const uint32_t* __restrict__ flag, const uint64_t* __restrict__ pos,
                        int32_t* __restrict__ slot, int32_t* __restrict__ pid_of_slot) {
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < np; p += (int64_t)gridDim.x * blockDim.x) {
        if (flag[p]) {
            slot[p] = (int32_t)pos[p];
            pid_of_slot[pos[p]] = (int32_t)p;
        } else {
            slot[p] = -1;
        }
    }
}

struct Bits {
    uint32_t* bm;          // [slot - s_lo][orbit][word]
    int64_t words;         // words per bitmap
    int norb;              // bitmaps per slot: 4, or 5 with patterns of four edges
    const int32_t* slot;   // pattern -> slot or -1
    int32_t s_lo, s_hi;    // slots of this group
    const int32_t* lrank;  // vertex -> its rank among the vertices of its label
};

__device__ __forceinline__ void set_bits(const Bits& Bt, const Emb& E) {
    const int32_t sl = Bt.slot[E.pid];
    if (sl < Bt.s_lo || sl >= Bt.s_hi) return;
    uint32_t* base = Bt.bm + (int64_t)(sl - Bt.s_lo) * Bt.norb * Bt.words;
    // every vertex of an orbit has the orbit's label, so its bit is indexed
    // by its rank within that label (bitmaps of max-label-count bits)
    // Most embeddings meet bits that are set already (a domain holds at most
    // one bit per vertex, and each vertex lies in many embeddings): the word
    // is read first and the atomic skipped when the bit is there.  Bits only
    // go from 0 to 1, so a stale read can only cost a redundant atomic.
    for (int i = 0; i < E.nv; ++i) {
        const uint32_t v = (uint32_t)Bt.lrank[E.v[i]];
        uint32_t* w = base + E.orb[i] * Bt.words + (v >> 5);
        const uint32_t bit = 1u << (v & 31);
        if ((__hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & bit) == 0u) atomicOr(w, bit);
    }
}

// The domain bits of one embedding of at most four vertices as sort keys:
// (bitmap word << 5 | bit) per vertex, all ones where there is none (fewer
// vertices, or a pattern without a slot in this group), four keys per
// embedding at a 32-byte aligned place.
__device__ __forceinline__ void bit_keys(const Bits& Bt, const Emb& E, uint64_t* __restrict__ out) {
    const int32_t sl = Bt.slot[E.pid];
    const bool in = sl >= Bt.s_lo && sl < Bt.s_hi;
    const uint64_t base = in ? (uint64_t)(sl - Bt.s_lo) * Bt.norb : 0;
    uint64_t k[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        k[i] = ~0ull;
        if (in && i < E.nv) {
            const uint32_t v = (uint32_t)Bt.lrank[E.v[i]];
            k[i] = (((base + (uint64_t)E.orb[i]) * (uint64_t)Bt.words + (v >> 5)) << 5) | (v & 31u);
        }
    }
    __builtin_memcpy(__builtin_assume_aligned(out, 32), k, 32);
}

// Bitmap blocks of FB_WORDS words (64 KB): the keys are sorted by block
// (key >> FB_SHIFT), then one workgroup per block ORs its keys into LDS
// and stores the block's words.  The all-ones keys sort after every block
// (the sort covers enough bits to tell the last block from them).
constexpr int FB_WORDS = 16384;
constexpr int FB_SHIFT = 5 + 14;
constexpr int FB_THREADS = 1024;

__device__ __forceinline__ int64_t first_key_at_least(const uint64_t* __restrict__ keys, int64_t m, uint64_t t) {
    int64_t lo = 0, hi = m;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (keys[mid] < t) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

__global__ __launch_bounds__(FB_THREADS) void k_bits_apply(const uint64_t* __restrict__ keys, int64_t m,
                                                           int64_t total_words, uint32_t* __restrict__ bm) {
    __shared__ uint32_t w[FB_WORDS];
    __shared__ int64_t rng[2];
    const int64_t b = blockIdx.x;
    for (int i = threadIdx.x; i < FB_WORDS; i += FB_THREADS) w[i] = 0;
    if (threadIdx.x < 2) rng[threadIdx.x] = first_key_at_least(keys, m, (uint64_t)(b + threadIdx.x) << FB_SHIFT);
    __syncthreads();
    for (int64_t i = rng[0] + threadIdx.x; i < rng[1]; i += FB_THREADS) {
        const uint64_t k = keys[i];
        atomicOr(&w[(uint32_t)(k >> 5) & (FB_WORDS - 1)], 1u << (uint32_t)(k & 31u));
    }
    __syncthreads();
    const int64_t w0 = b * FB_WORDS;
    const int nw = (int)min64(FB_WORDS, total_words - w0);
    for (int i = threadIdx.x; i < nw; i += FB_THREADS) bm[w0 + i] = w[i];
}

// level 1: patterns of every edge, or domain bits
template <bool BITS>
__global__ void k_fsm_l1(FsmCtx C, int64_t E, int32_t* __restrict__ pid, Bits Bt) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < E; e += (int64_t)gridDim.x * blockDim.x) {
        const Emb Em = classify_edge(C, C.esrc[e], C.edst[e]);
        if (BITS) set_bits(Bt, Em);
        else pid[e] = Em.pid;
    }
}

// stream compaction by a frequent flag on the entries' pattern
__global__ void k_keep_flags(int64_t m, const int32_t* __restrict__ pid, const uint8_t* __restrict__ freq,
                             uint32_t* __restrict__ keep) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
        keep[i] = freq[pid[i]] ? 1u : 0u;
}

__global__ void k_compact2(int64_t m, const uint32_t* __restrict__ keep, const uint64_t* __restrict__ pos,
                           const int32_t* __restrict__ a, const int32_t* __restrict__ b, int32_t* __restrict__ oa,
                           int32_t* __restrict__ ob) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
        if (keep[i]) {
            oa[pos[i]] = a ? a[i] : (int32_t)i;
            if (b) ob[pos[i]] = b[i];
        }
}

// level 2 from frequent edges: COUNT children, or WRITE (e1, e2, pid)
template <bool WRITE>
__global__ void k_fsm_l2(FsmCtx C, int64_t m, const int32_t* __restrict__ e1s, uint32_t* __restrict__ cnt,
                         const uint64_t* __restrict__ start, int32_t* __restrict__ o1, int32_t* __restrict__ o2,
                         int32_t* __restrict__ opid) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t e1 = e1s[i];
        const int32_t a = C.esrc[e1], b = C.edst[e1];
        uint64_t pos = WRITE ? start[i] : 0;
        uint32_t c = 0;
        for (int side = 0; side < 2; ++side) {
            const int32_t s = side ? b : a, o = side ? a : b;
            for (int64_t j = C.rp[s]; j < C.rp[s + 1]; ++j) {
                const int32_t e = C.eid[j];
                if (e <= e1) continue;       // canonical: e > g1 (and e != e1)
                if (WRITE) {
                    const Emb Em = classify_wedge(C, s, o, C.col[j]);
                    o1[pos] = e1;
                    o2[pos] = e;
                    opid[pos] = Em.pid;
                    ++pos;
                } else {
                    ++c;
                }
            }
        }
        if (!WRITE) cnt[i] = c;
    }
}

// Level 3 from frequent wedges.  L3_HIST / L3_BITS: fused with Reduce (a
// histogram of patterns, with the children per parent when nch is given,
// or domain bits); L3_KEYS: the domain bits as sort keys at the parent's
// offset; L3_COUNT / L3_WRITE: the materialised level of four-edge mining
// (children per parent, then (e1, e2, e3, pattern) at the parent's offset).
enum { L3_HIST = 0, L3_BITS = 1, L3_COUNT = 2, L3_WRITE = 3, L3_KEYS = 4 };

// A wave takes 64 parents (frequent wedges e1, e2 with shared vertex s,
// other ends o of e1 and t of e2) a round and lays their candidate edges
// end to end: the lists of s, o and t.  Each step the 64 lanes take 64
// consecutive candidates, so a list is read by neighbouring lanes, and a
// lane finds its parent in the prefix of the parents' list lengths.  A
// candidate edge (x, w) extends the wedge when the canonical order admits
// it: at s a new leaf (a star) and at o (a triangle or a path) only edges
// after e2, at t (a path) edges after e1.  A child's place among its
// parent's children is the children the parent had before this step plus
// those of its lanes below it in the step (a parent's lanes are
// contiguous), so the children of a parent are written side by side.
constexpr int F3_THREADS = 256;
constexpr int F3_WAVES = F3_THREADS / WAVE;

struct F3Lds {
    uint32_t pre[F3_WAVES][WAVE];   // first candidate of each parent
    uint32_t ns[F3_WAVES][WAVE], no[F3_WAVES][WAVE];
    uint32_t cnt[F3_WAVES][WAVE];   // children found so far
    int32_t s[F3_WAVES][WAVE], o[F3_WAVES][WAVE], t[F3_WAVES][WAVE];
    int32_t e1[F3_WAVES][WAVE], e2[F3_WAVES][WAVE];
    int64_t bs[F3_WAVES][WAVE], bo[F3_WAVES][WAVE], bt[F3_WAVES][WAVE];
};

template <int MODE>
__global__ __launch_bounds__(F3_THREADS) void k_fsm_l3(FsmCtx C, int64_t m, const int32_t* __restrict__ e1s,
                                                      const int32_t* __restrict__ e2s, uint32_t* __restrict__ counts,
                                                      Bits Bt, unsigned long long* __restrict__ n_emb,
                                                      const uint64_t* __restrict__ start, int32_t* __restrict__ o1,
                                                      int32_t* __restrict__ o2, int32_t* __restrict__ o3,
                                                      int32_t* __restrict__ opid, uint32_t* __restrict__ nch,
                                                      uint64_t* __restrict__ keys) {
    __shared__ F3Lds L;
    const int w = threadIdx.x / WAVE;
    uint64_t local = 0, scanned = 0;
    const int64_t stride = (int64_t)gridDim.x * F3_WAVES * WAVE;
    for (int64_t r0 = ((int64_t)blockIdx.x * F3_WAVES + w) * WAVE; r0 < m; r0 += stride) {
        const int64_t i = r0 + lane();
        uint32_t tot = 0;
        {
            int32_t e1 = 0, e2 = 0, sv = 0, ov = 0, tv = 0;
            int64_t bs = 0, bo = 0, bt = 0;
            uint32_t ns = 0, no = 0, nt = 0;
            if (i < m) {
                e1 = e1s[i];
                e2 = e2s[i];
                const int32_t a = C.esrc[e1], b = C.edst[e1], c = C.esrc[e2], d = C.edst[e2];
                sv = (a == c || a == d) ? a : b;
                ov = (sv == a) ? b : a;
                tv = (sv == c) ? d : c;
                bs = C.rp[sv];
                ns = (uint32_t)(C.rp[sv + 1] - bs);
                bo = C.rp[ov];
                no = (uint32_t)(C.rp[ov + 1] - bo);
                bt = C.rp[tv];
                nt = (uint32_t)(C.rp[tv + 1] - bt);
            }
            tot = ns + no + nt;
            const uint32_t inc = wave_incl_scan(tot);
            L.pre[w][lane()] = inc - tot;
            L.ns[w][lane()] = ns;
            L.no[w][lane()] = no;
            L.cnt[w][lane()] = 0;
            L.s[w][lane()] = sv;
            L.o[w][lane()] = ov;
            L.t[w][lane()] = tv;
            L.e1[w][lane()] = e1;
            L.e2[w][lane()] = e2;
            L.bs[w][lane()] = bs;
            L.bo[w][lane()] = bo;
            L.bt[w][lane()] = bt;
        }
        if (MODE == L3_HIST) scanned += tot;
        const uint32_t total = bcast(wave_incl_scan(tot), WAVE - 1);
        const int np = (int)min64(WAVE, m - r0);
        wave_sync();
        for (uint32_t c0 = 0; c0 < total; c0 += WAVE) {
            const uint32_t cidx = c0 + lane();
            const bool valid = cidx < total;
            // the parent of candidate cidx: the last lane whose prefix is <= cidx
            int xi = 0;
            {
                int n_i = np;
                while (n_i > 1) {
                    const int half = n_i >> 1;
                    if (L.pre[w][xi + half] <= cidx) xi += half;
                    n_i -= half;
                }
            }
            bool child = false;
            Emb Em;
            Em.pid = 0;
            Em.nv = 0;
            int32_t e3 = 0;
            if (valid) {
                const uint32_t off = cidx - L.pre[w][xi];
                const uint32_t ns = L.ns[w][xi], no = L.no[w][xi];
                const int32_t sv = L.s[w][xi], ov = L.o[w][xi], tv = L.t[w][xi];
                if (off < ns) {
                    const int64_t j = L.bs[w][xi] + off;
                    const int32_t x = C.col[j];
                    e3 = C.eid[j];
                    child = x != ov && x != tv && e3 > L.e2[w][xi];
                    if (child && MODE != L3_COUNT) Em = classify_star(C, sv, ov, tv, x);
                } else if (off < ns + no) {
                    const int64_t j = L.bo[w][xi] + (off - ns);
                    const int32_t x = C.col[j];
                    e3 = C.eid[j];
                    child = x != sv && e3 > L.e2[w][xi];
                    if (child && MODE != L3_COUNT)
                        Em = (x == tv) ? classify_triangle(C, sv, ov, tv) : classify_path(C, x, ov, sv, tv);
                } else {
                    const int64_t j = L.bt[w][xi] + (off - ns - no);
                    const int32_t x = C.col[j];
                    e3 = C.eid[j];
                    child = x != sv && x != ov && e3 > L.e1[w][xi];
                    if (child && MODE != L3_COUNT) Em = classify_path(C, ov, sv, tv, x);
                }
            }
            // the child's place among its parent's children
            const uint64_t V = ballot(child);
            const int key = valid ? xi : WAVE;
            const int prev = __shfl_up(key, 1, WAVE);
            const bool head = lane() == 0 || prev != key;
            const uint64_t H = ballot(head);
            const uint64_t lt = lanemask_lt();
            const int hd = 63 - __clzll(H & (lt | (1ull << lane())));
            const uint64_t seg_lt = lt & ~((1ull << hd) - 1ull);
            const uint32_t before = L.cnt[w][xi] + (uint32_t)popc64(V & seg_lt);
            const bool last = lane() == WAVE - 1 || ((H >> (lane() + 1)) & 1ull);
            if (child) {
                ++local;
                if (MODE == L3_HIST) atomicAdd(&counts[Em.pid], 1u);
                if (MODE == L3_BITS) set_bits(Bt, Em);
                if (MODE == L3_KEYS) bit_keys(Bt, Em, keys + ((start[r0 + xi] + before) << 2));
                if (MODE == L3_WRITE) {
                    const uint64_t pos = start[r0 + xi] + before;
                    o1[pos] = L.e1[w][xi];
                    o2[pos] = L.e2[w][xi];
                    o3[pos] = e3;
                    opid[pos] = Em.pid;
                }
            }
            wave_sync();   // every lane has read the counts before they move on
            if (valid && last) L.cnt[w][xi] = before + (uint32_t)(child ? 1 : 0);
            wave_sync();
        }
        if (i < m) {
            if (MODE == L3_COUNT) counts[i] = L.cnt[w][lane()];
            if (MODE == L3_HIST && nch) nch[i] = L.cnt[w][lane()];
        }
        wave_sync();   // the round's LDS is read before the next round writes it
    }
    if (MODE == L3_HIST) {
        local = wave_sum_u64(local);
        scanned = wave_sum_u64(scanned);
        if (lane() == 0 && local) atomicAdd(&n_emb[0], (unsigned long long)local);
        if (lane() == 0 && scanned) atomicAdd(&n_emb[1], (unsigned long long)scanned);
    }
}

// domain bits of stored level-3 entries
__global__ void k_fsm_l3_bits_stored(FsmCtx C, int64_t m, const int32_t* __restrict__ e1s,
                                     const int32_t* __restrict__ e2s, const int32_t* __restrict__ e3s, Bits Bt) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t es[3] = {e1s[i], e2s[i], e3s[i]};
        set_bits(Bt, classify_edges(C, es, 3));
    }
}

// Level 4 from frequent level-3 entries (g1, g2, g3 in greedy order), fused
// with Reduce: every edge e at a vertex of the embedding, not in it, keeps
// the greedy order iff e > g1, e > g2 when e touches g1, and e > g3 when e
// touches g1 or g2.  An edge joining two vertices of the embedding is seen
// from both ends and taken from the smaller one.
template <bool BITS>
__global__ void k_fsm_l4(FsmCtx C, int64_t m, const int32_t* __restrict__ e1s, const int32_t* __restrict__ e2s,
                         const int32_t* __restrict__ e3s, uint32_t* __restrict__ counts, Bits Bt,
                         unsigned long long* __restrict__ n_emb) {
    uint64_t local = 0, scanned = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
        int32_t es[4] = {e1s[i], e2s[i], e3s[i], 0};
        int32_t vs[4];
        int nv = 0;
        for (int k = 0; k < 3; ++k) {
            const int32_t ends[2] = {C.esrc[es[k]], C.edst[es[k]]};
            for (int h = 0; h < 2; ++h) {
                bool seen = false;
                for (int q = 0; q < nv; ++q) seen |= vs[q] == ends[h];
                if (!seen && nv < 4) vs[nv++] = ends[h];
            }
        }
        const int32_t a1 = C.esrc[es[0]], b1 = C.edst[es[0]];
        const int32_t a2 = C.esrc[es[1]], b2 = C.edst[es[1]];
        for (int k = 0; k < nv; ++k) {
            const int32_t x = vs[k];
            if (!BITS) scanned += (uint64_t)(C.rp[x + 1] - C.rp[x]);
            for (int64_t j = C.rp[x]; j < C.rp[x + 1]; ++j) {
                const int32_t e = C.eid[j];
                if (e <= es[0] || e == es[1] || e == es[2]) continue;
                const int32_t w = C.col[j];
                bool inside = false;
                for (int q = 0; q < nv; ++q) inside |= vs[q] == w;
                if (inside && w < x) continue;
                const bool t1 = x == a1 || x == b1 || w == a1 || w == b1;
                const bool t12 = t1 || x == a2 || x == b2 || w == a2 || w == b2;
                if (t1 && e <= es[1]) continue;
                if (t12 && e <= es[2]) continue;
                es[3] = e;
                const Emb Em = classify_edges(C, es, 4);
                ++local;
                if (BITS) set_bits(Bt, Em); else atomicAdd(&counts[Em.pid], 1u);
            }
        }
    }
    if (!BITS) {
        local = wave_sum_u64(local);
        scanned = wave_sum_u64(scanned);
        if (lane() == 0 && local) atomicAdd(&n_emb[2], (unsigned long long)local);
        if (lane() == 0 && scanned) atomicAdd(&n_emb[3], (unsigned long long)scanned);
    }
}

// level 2 domain bits from the stored entries
__global__ void k_fsm_l2_bits(FsmCtx C, int64_t m, const int32_t* __restrict__ e1s, const int32_t* __restrict__ e2s,
                              Bits Bt) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t e1 = e1s[i], e2 = e2s[i];
        const int32_t a = C.esrc[e1], b = C.edst[e1], c = C.esrc[e2], d = C.edst[e2];
        const int32_t s = (a == c || a == d) ? a : b;
        const int32_t o = (s == a) ? b : a;
        const int32_t t = (s == c) ? d : c;
        set_bits(Bt, classify_wedge(C, s, o, t));
    }
}

// support of each slot of the group: the smallest non-empty orbit domain
// one wave per orbit bitmap (blockDim = norb waves)
__global__ __launch_bounds__(FSM_MAXV * WAVE) void k_supports(const uint32_t* __restrict__ bm, int64_t words,
                                                              int norb, int32_t s_lo, int32_t s_hi,
                                                              uint64_t* __restrict__ sup_slot) {
    __shared__ unsigned long long pop[FSM_MAXV];
    const int32_t sl = s_lo + blockIdx.x;
    if (sl >= s_hi) return;
    const int o = threadIdx.x / WAVE;
    const uint32_t* base = bm + ((int64_t)(sl - s_lo) * norb + o) * words;
    uint64_t c = 0;
    for (int64_t i = lane(); i < words; i += WAVE) c += (uint64_t)__popc(base[i]);
    c = wave_sum_u64(c);
    if (lane() == 0) pop[o] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t best = 0;
        for (int k = 0; k < norb; ++k)
            if (pop[k] && (best == 0 || pop[k] < best)) best = pop[k];
        sup_slot[sl] = best;
    }
}

__global__ void k_frequent(int64_t np, const int32_t* __restrict__ slot, const uint64_t* __restrict__ sup_slot,
                           uint64_t sigma, uint64_t* __restrict__ sup_pat, uint8_t* __restrict__ freq) {
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < np; p += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t s = slot[p] >= 0 ? sup_slot[slot[p]] : 0;
        const bool f = slot[p] >= 0 && s >= sigma && s > 0;
        freq[p] = f ? 1 : 0;
        sup_pat[p] = f ? s : 0;
    }
}

// ------------------------------------------------------------------ host

static unsigned grid1(int64_t items) {
    int64_t b = (items + 255) / 256;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(b, (int64_t)device_info().n_cu * 16));
}

// Reduce over one level: supports of its patterns [p_lo, p_hi) (dense
// index), frequent flags, and the host copy of the supports.
template <class SetBits>
static void reduce_level(pg_graph* g, FsmCtx& C, const int32_t* lrank, int64_t label_max, int64_t p_lo,
                         int64_t p_hi, const uint32_t* counts, uint64_t sigma, uint8_t* freq, uint64_t* sup_pat,
                         SetBits&& set_bits_pass) {
    hipStream_t s = g->stream;
    Arena& ar = g->arena;
    const int64_t np = p_hi - p_lo;
    const size_t mk = ar.mark();
    uint32_t* flag = push<uint32_t>(ar, np);
    uint64_t* pos = push<uint64_t>(ar, np + 1);
    int32_t* slot = push<int32_t>(ar, C.B.total);
    fill_u32(reinterpret_cast<uint32_t*>(slot), C.B.total, 0xffffffffu, s);
    k_candidates<<<grid1(np), 256, 0, s>>>(np, p_lo, counts + p_lo, C.B, sigma, flag);
    PG_HIP(hipGetLastError());
    scan_u32(flag, np, pos, ar, s);
    const int64_t ns = (int64_t)read_u64(pos + np, s);
    int32_t* pid_of_slot = push<int32_t>(ar, std::max<int64_t>(ns, 1));
    k_slots<<<grid1(np), 256, 0, s>>>(np, flag, pos, slot + p_lo, pid_of_slot);
    PG_HIP(hipGetLastError());
    uint64_t* sup_slot = push<uint64_t>(ar, std::max<int64_t>(ns, 1));
    if (ns > 0) {
        const int64_t words = (label_max + 31) / 32;
        const int norb = C.B.total > C.B.p5 ? FSM_MAXV : 4;
        const uint64_t per_slot = (uint64_t)words * norb * sizeof(uint32_t);
        const uint64_t room = g->budget > ar.mark() ? g->budget - ar.mark() : 0;
        const int64_t group = std::max<int64_t>(1, std::min<int64_t>(ns, (int64_t)(room / std::max<uint64_t>(per_slot, 1))));
        uint32_t* bm = push<uint32_t>(ar, (size_t)group * norb * words);
        for (int64_t g0 = 0; g0 < ns; g0 += group) {
            const int64_t g1 = std::min(ns, g0 + group);
            fill_u32(bm, (g1 - g0) * norb * words, 0, s);
            Bits Bt{bm, words, norb, slot, (int32_t)g0, (int32_t)g1, lrank};
            set_bits_pass(Bt);
            ProfScope ps("fsm_support", s, (double)(g1 - g0));
            k_supports<<<(unsigned)(g1 - g0), norb * WAVE, 0, s>>>(bm, words, norb, (int32_t)g0, (int32_t)g1,
                                                                   sup_slot);
            PG_HIP(hipGetLastError());
        }
    }
    // the slot table covers the whole index; only this level's range is read
    k_frequent<<<grid1(np), 256, 0, s>>>(np, slot + p_lo, sup_slot, sigma, sup_pat + p_lo, freq + p_lo);
    PG_HIP(hipGetLastError());
    ar.reset(mk);
}

__global__ void k_label_keys(int64_t n, const int32_t* __restrict__ lab, uint64_t* __restrict__ keys) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
        keys[v] = ((uint64_t)(uint32_t)lab[v] << 32) | (uint64_t)v;
}

__global__ void k_label_ranks(int64_t n, const uint64_t* __restrict__ sorted, const uint64_t* __restrict__ first,
                              int32_t* __restrict__ lrank) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t k = sorted[i];
        lrank[(uint32_t)k] = (int32_t)((uint64_t)i - first[k >> 32]);
    }
}

// Rank of every vertex among the vertices of its label (stable by id);
// returns the largest label class.
static int64_t label_ranks(pg_graph* g, int32_t* lrank) {
    hipStream_t s = g->stream;
    Arena& ar = g->arena;
    const int64_t n = g->n, L = g->n_labels;
    if (n == 0) return 0;
    const size_t mk = ar.mark();
    uint64_t* keys = push<uint64_t>(ar, n);
    uint64_t* tmp = push<uint64_t>(ar, n);
    uint32_t* hist = push<uint32_t>(ar, L);
    uint64_t* first = push<uint64_t>(ar, L + 1);
    fill_u32(hist, L, 0, s);
    k_label_keys<<<grid1(n), 256, 0, s>>>(n, g->labels.as<int32_t>(), keys);
    PG_HIP(hipGetLastError());
    k_hist<<<hist_blocks(n), 256, 0, s>>>(n, g->labels.as<int32_t>(), hist, 0, (int32_t)L);
    PG_HIP(hipGetLastError());
    int lb = 1;
    while ((int64_t(1) << lb) < L) ++lb;
    radix_sort_u64(keys, tmp, n, 0, 32 + lb, ar, s);
    scan_u32(hist, L, first, ar, s);
    k_label_ranks<<<grid1(n), 256, 0, s>>>(n, keys, first, lrank);
    PG_HIP(hipGetLastError());
    std::vector<uint32_t> h((size_t)L);
    PG_HIP(hipMemcpyAsync(h.data(), hist, sizeof(uint32_t) * L, hipMemcpyDeviceToHost, s));
    PG_HIP(hipStreamSynchronize(s));
    ar.reset(mk);
    int64_t mx = 0;
    for (uint32_t c : h) mx = std::max<int64_t>(mx, c);
    return mx;
}

void run_fsm(pg_graph* g, int max_edges, uint64_t min_support, uint64_t* supports, size_t len, size_t* n_frequent) {
    PG_REQUIRE(max_edges >= 1 && max_edges <= 4, PG_EUNSUPPORTED, "max_edges must be in [1, 4]");
    PG_REQUIRE(g->n_labels > 0, PG_EINVAL, "FSM needs a labelled graph");
    PG_REQUIRE(max_edges < 4 || g->n_labels <= FSM4_MAX_LABELS, PG_EUNSUPPORTED,
               "patterns of four edges need at most 32 labels");
    build_motif_l1(g);
    PG_REQUIRE(g->ml1.n_edges < INT32_MAX, PG_EOVERFLOW, "FSM supports fewer than 2^31 edges");
    hipStream_t s = g->stream;
    Arena& ar = g->arena;
    const int64_t L = g->n_labels;
    const int64_t E = g->ml1.n_edges;
    FsmCtx C;
    C.B = pat_base(L, max_edges);
    const int64_t np = C.B.total;
    PG_REQUIRE((uint64_t)np <= len, PG_EINVAL, "supports array too short");
    C.rp = g->rp.as<int64_t>();
    C.col = g->col.as<int32_t>();
    C.esrc = g->ml1.src.as<int32_t>();
    C.edst = g->ml1.dst.as<int32_t>();
    C.lab = g->labels.as<int32_t>();
    // edge ids of CSR entries
    int32_t* eid = push<int32_t>(ar, std::max<int64_t>(g->nnz, 1));
    if (g->n > 0) {
        k_edge_ids<<<grid1(g->n * 64 / 4), 256, 0, s>>>(g->n, C.rp, C.col, g->ml1.seg.as<int64_t>(), eid);
        PG_HIP(hipGetLastError());
    }
    C.eid = eid;
    // path label ranks
    int32_t* prank = nullptr;
    if (max_edges >= 3) {
        const int64_t N4 = L * L * L * L;
        prank = push<int32_t>(ar, N4);
        const size_t mk = ar.mark();
        uint32_t* pf = push<uint32_t>(ar, N4);
        uint64_t* pr = push<uint64_t>(ar, N4 + 1);
        k_path_flags<<<grid1(N4), 256, 0, s>>>(L, pf);
        PG_HIP(hipGetLastError());
        scan_u32(pf, N4, pr, ar, s);
        k_u64_to_i32<<<grid1(N4), 256, 0, s>>>(N4, pr, prank);
        PG_HIP(hipGetLastError());
        ar.reset(mk);
    }
    C.path_rank = prank;
    C.p5_rank = C.q4_rank = C.c4_rank = nullptr;
    if (max_edges >= 4) {
        // rank tables of the 5-path, 4-star and 4-cycle blocks: representative
        // flags over all tuple codes, then their exclusive prefix sum
        auto table = [&](int kind, int64_t N) {
            int32_t* rank = push<int32_t>(ar, N);
            const size_t mk = ar.mark();
            uint32_t* f = push<uint32_t>(ar, N);
            uint64_t* r = push<uint64_t>(ar, N + 1);
            k_rep_flags<<<grid1(N), 256, 0, s>>>(L, kind, N, f);
            PG_HIP(hipGetLastError());
            scan_u32(f, N, r, ar, s);
            k_u64_to_i32<<<grid1(N), 256, 0, s>>>(N, r, rank);
            PG_HIP(hipGetLastError());
            ar.reset(mk);
            return rank;
        };
        C.p5_rank = table(REP_PATH5, L * L * L * L * L);
        C.q4_rank = table(REP_SORTED4, L * L * L * L);
        C.c4_rank = table(REP_CYCLE4, L * L * L * L);
    }
    int32_t* lrank = push<int32_t>(ar, std::max<int64_t>(g->n, 1));
    const int64_t label_max = label_ranks(g, lrank);
    uint32_t* counts = push<uint32_t>(ar, np);
    uint8_t* freq = push<uint8_t>(ar, np);
    uint64_t* sup_pat = push<uint64_t>(ar, np);
    fill_u32(counts, np, 0, s);
    fill_u64(sup_pat, np, 0, s);
    fill_u32(reinterpret_cast<uint32_t*>(freq), (np + 3) / 4, 0, s);
    unsigned long long* n_emb = reinterpret_cast<unsigned long long*>(push<uint64_t>(ar, 4));
    fill_u64(reinterpret_cast<uint64_t*>(n_emb), 4, 0, s);

    int64_t n2_total = 0, m2_total = 0, l3_passes = 0, l3_key_passes = 0, n3_stored = 0;
    double apply_keys = 0.0, apply_words = 0.0;
    // ---------------- level 1: every edge; Reduce; Filter
    int32_t* pid1 = push<int32_t>(ar, std::max<int64_t>(E, 1));
    {
        ProfScope ps("fsm_l1", s, (double)E);
        k_fsm_l1<false><<<grid1(E), 256, 0, s>>>(C, E, pid1, Bits{});
        PG_HIP(hipGetLastError());
        k_hist<<<hist_blocks(E), 256, 0, s>>>(E, pid1, counts, (int32_t)C.B.edge, (int32_t)(C.B.wedge - C.B.edge));
        PG_HIP(hipGetLastError());
    }
    reduce_level(g, C, lrank, label_max, C.B.edge, C.B.wedge, counts, min_support, freq, sup_pat, [&](const Bits& Bt) {
        k_fsm_l1<true><<<grid1(E), 256, 0, s>>>(C, E, nullptr, Bt);
        PG_HIP(hipGetLastError());
    });
    if (max_edges >= 2) {
        // Filter: frequent edges, in id order
        uint32_t* keep = push<uint32_t>(ar, std::max<int64_t>(E, 1));
        uint64_t* kpos = push<uint64_t>(ar, E + 1);
        k_keep_flags<<<grid1(E), 256, 0, s>>>(E, pid1, freq, keep);
        PG_HIP(hipGetLastError());
        scan_u32(keep, E, kpos, ar, s);
        const int64_t m1 = (int64_t)read_u64(kpos + E, s);
        int32_t* f1 = push<int32_t>(ar, std::max<int64_t>(m1, 1));
        k_compact2<<<grid1(E), 256, 0, s>>>(E, keep, kpos, nullptr, nullptr, f1, nullptr);
        PG_HIP(hipGetLastError());

        // ---------------- level 2: count / scan / write with memoised pattern ids
        uint32_t* c2 = push<uint32_t>(ar, std::max<int64_t>(m1, 1));
        uint64_t* st2 = push<uint64_t>(ar, m1 + 1);
        if (m1 > 0) {
            ProfScope ps("fsm_l2_count", s, (double)m1);
            k_fsm_l2<false><<<grid1(m1), 256, 0, s>>>(C, m1, f1, c2, nullptr, nullptr, nullptr, nullptr);
            PG_HIP(hipGetLastError());
        }
        scan_u32(c2, m1, st2, ar, s);
        const int64_t n2 = (int64_t)read_u64(st2 + m1, s);
        n2_total = n2;
        int32_t* a2 = push<int32_t>(ar, std::max<int64_t>(n2, 1));
        int32_t* b2 = push<int32_t>(ar, std::max<int64_t>(n2, 1));
        int32_t* p2 = push<int32_t>(ar, std::max<int64_t>(n2, 1));
        if (m1 > 0) {
            ProfScope ps("fsm_l2_write", s, (double)n2);
            k_fsm_l2<true><<<grid1(m1), 256, 0, s>>>(C, m1, f1, nullptr, st2, a2, b2, p2);
            PG_HIP(hipGetLastError());
            k_hist<<<hist_blocks(n2), 256, 0, s>>>(n2, p2, counts, (int32_t)C.B.wedge, (int32_t)(C.B.tri - C.B.wedge));
            PG_HIP(hipGetLastError());
        }
        reduce_level(g, C, lrank, label_max, C.B.wedge, C.B.tri, counts, min_support, freq, sup_pat, [&](const Bits& Bt) {
            if (n2 > 0) {
                k_fsm_l2_bits<<<grid1(n2), 256, 0, s>>>(C, n2, a2, b2, Bt);
                PG_HIP(hipGetLastError());
            }
        });
        if (max_edges >= 3) {
            // Filter: frequent wedges
            uint32_t* keep2 = push<uint32_t>(ar, std::max<int64_t>(n2, 1));
            uint64_t* kpos2 = push<uint64_t>(ar, n2 + 1);
            k_keep_flags<<<grid1(n2), 256, 0, s>>>(n2, p2, freq, keep2);
            PG_HIP(hipGetLastError());
            scan_u32(keep2, n2, kpos2, ar, s);
            const int64_t m2 = (int64_t)read_u64(kpos2 + n2, s);
            m2_total = m2;
            int32_t* fa = push<int32_t>(ar, std::max<int64_t>(m2, 1));
            int32_t* fb = push<int32_t>(ar, std::max<int64_t>(m2, 1));
            k_compact2<<<grid1(n2), 256, 0, s>>>(n2, keep2, kpos2, a2, b2, fa, fb);
            PG_HIP(hipGetLastError());
            if (max_edges == 3) {
                // ---------------- level 3, fused with Reduce (never stored)
                uint32_t* nch = push<uint32_t>(ar, std::max<int64_t>(m2, 1));
                uint64_t* st3 = push<uint64_t>(ar, m2 + 1);
                if (m2 > 0) {
                    ProfScope ps("fsm_l3_hist", s, (double)m2);
                    k_fsm_l3<L3_HIST><<<grid1(m2), 256, 0, s>>>(C, m2, fa, fb, counts, Bits{}, n_emb, nullptr,
                                                                nullptr, nullptr, nullptr, nullptr, nch, nullptr);
                    PG_HIP(hipGetLastError());
                }
                // every embedding's place among the level's, for the bit keys
                scan_u32(nch, m2, st3, ar, s);
                const int64_t n3 = (int64_t)read_u64(st3 + m2, s);
                reduce_level(g, C, lrank, label_max, C.B.tri, C.B.total, counts, min_support, freq, sup_pat,
                             [&](const Bits& Bt) {
                    if (m2 == 0) return;
                    // sorted keys need 2 x 32 B per embedding and the sort's tile
                    // histograms (12 B per digit per 2,048 keys)
                    const int64_t nk = 4 * n3;
                    const uint64_t need = 64ull * (uint64_t)n3 + 12ull * 256 * (uint64_t)(nk / 2048 + 2) +
                                          (uint64_t(64) << 20);
                    const uint64_t room = g->budget > ar.mark() ? g->budget - ar.mark() : 0;
                    if (g->fsm_bit_keys && n3 > 0 && need <= room) {
                        ar.ensure(need);
                        const size_t mk = ar.mark();
                        const int64_t total_words = (int64_t)(Bt.s_hi - Bt.s_lo) * Bt.norb * Bt.words;
                        const int64_t nblk = (total_words + FB_WORDS - 1) / FB_WORDS;
                        // sort digits enough for 2^bits > nblk: the all-ones keys
                        // then sort after the last block
                        int bits = 1;
                        while ((int64_t(1) << bits) <= nblk) ++bits;
                        uint64_t* keys = push<uint64_t>(ar, nk);
                        uint64_t* tmp = push<uint64_t>(ar, nk);
                        {
                            ProfScope ps("fsm_l3_keys", s, (double)m2);
                            k_fsm_l3<L3_KEYS><<<grid1(m2), 256, 0, s>>>(C, m2, fa, fb, nullptr, Bt, nullptr, st3,
                                                                        nullptr, nullptr, nullptr, nullptr, nullptr,
                                                                        keys);
                            PG_HIP(hipGetLastError());
                        }
                        radix_sort_u64(keys, tmp, nk, FB_SHIFT, FB_SHIFT + bits, ar, s);
                        {
                            ProfScope ps("fsm_bits_apply", s, (double)nk);
                            k_bits_apply<<<(unsigned)nblk, FB_THREADS, 0, s>>>(keys, nk, total_words, Bt.bm);
                            PG_HIP(hipGetLastError());
                        }
                        ar.reset(mk);
                        ++l3_key_passes;   // one per group of candidate patterns
                        apply_keys += (double)nk;
                        apply_words += (double)total_words;
                    } else {
                        ++l3_passes;
                        ProfScope ps("fsm_l3_bits", s, (double)m2);
                        k_fsm_l3<L3_BITS><<<grid1(m2), 256, 0, s>>>(C, m2, fa, fb, nullptr, Bt, nullptr, nullptr,
                                                                    nullptr, nullptr, nullptr, nullptr, nullptr,
                                                                    nullptr);
                        PG_HIP(hipGetLastError());
                    }
                });
            } else {
                // ---------------- level 3 materialised: count / scan / write
                uint32_t* c3 = push<uint32_t>(ar, std::max<int64_t>(m2, 1));
                uint64_t* st3 = push<uint64_t>(ar, m2 + 1);
                if (m2 > 0) {
                    ProfScope ps("fsm_l3_count", s, (double)m2);
                    k_fsm_l3<L3_COUNT><<<grid1(m2), 256, 0, s>>>(C, m2, fa, fb, c3, Bits{}, nullptr, nullptr,
                                                                 nullptr, nullptr, nullptr, nullptr, nullptr,
                                                                 nullptr);
                    PG_HIP(hipGetLastError());
                }
                scan_u32(c3, m2, st3, ar, s);
                const int64_t n3 = (int64_t)read_u64(st3 + m2, s);
                PG_REQUIRE(n3 < INT32_MAX, PG_EOVERFLOW, "level 3 exceeds 2^31 embeddings");
                n3_stored = n3;
                int32_t* x3 = push<int32_t>(ar, std::max<int64_t>(n3, 1));
                int32_t* y3 = push<int32_t>(ar, std::max<int64_t>(n3, 1));
                int32_t* z3 = push<int32_t>(ar, std::max<int64_t>(n3, 1));
                int32_t* p3 = push<int32_t>(ar, std::max<int64_t>(n3, 1));
                if (m2 > 0) {
                    ProfScope ps("fsm_l3_write", s, (double)n3);
                    k_fsm_l3<L3_WRITE><<<grid1(m2), 256, 0, s>>>(C, m2, fa, fb, nullptr, Bits{}, nullptr, st3, x3,
                                                                 y3, z3, p3, nullptr, nullptr);
                    PG_HIP(hipGetLastError());
                    k_hist<<<hist_blocks(n3), 256, 0, s>>>(n3, p3, counts, (int32_t)C.B.tri,
                                                           (int32_t)(C.B.p5 - C.B.tri));
                    PG_HIP(hipGetLastError());
                }
                reduce_level(g, C, lrank, label_max, C.B.tri, C.B.p5, counts, min_support, freq, sup_pat,
                             [&](const Bits& Bt) {
                    if (n3 > 0) {
                        k_fsm_l3_bits_stored<<<grid1(n3), 256, 0, s>>>(C, n3, x3, y3, z3, Bt);
                        PG_HIP(hipGetLastError());
                    }
                });
                // Filter: frequent patterns of three edges
                uint32_t* keep3 = push<uint32_t>(ar, std::max<int64_t>(n3, 1));
                uint64_t* kpos3 = push<uint64_t>(ar, n3 + 1);
                k_keep_flags<<<grid1(n3), 256, 0, s>>>(n3, p3, freq, keep3);
                PG_HIP(hipGetLastError());
                scan_u32(keep3, n3, kpos3, ar, s);
                const int64_t m3 = (int64_t)read_u64(kpos3 + n3, s);
                int32_t* fx = push<int32_t>(ar, std::max<int64_t>(m3, 1));
                int32_t* fy = push<int32_t>(ar, std::max<int64_t>(m3, 1));
                int32_t* fz = push<int32_t>(ar, std::max<int64_t>(m3, 1));
                k_compact2<<<grid1(n3), 256, 0, s>>>(n3, keep3, kpos3, x3, y3, fx, fy);
                PG_HIP(hipGetLastError());
                k_compact2<<<grid1(n3), 256, 0, s>>>(n3, keep3, kpos3, z3, nullptr, fz, nullptr);
                PG_HIP(hipGetLastError());
                // ---------------- level 4, fused with Reduce (never stored)
                if (m3 > 0) {
                    ProfScope ps("fsm_l4_hist", s, (double)m3);
                    k_fsm_l4<false><<<grid1(m3), 256, 0, s>>>(C, m3, fx, fy, fz, counts, Bits{}, n_emb);
                    PG_HIP(hipGetLastError());
                }
                reduce_level(g, C, lrank, label_max, C.B.p5, C.B.total, counts, min_support, freq, sup_pat,
                             [&](const Bits& Bt) {
                    if (m3 > 0) {
                        ProfScope ps("fsm_l4_bits", s, (double)m3);
                        k_fsm_l4<true><<<grid1(m3), 256, 0, s>>>(C, m3, fx, fy, fz, nullptr, Bt, nullptr);
                        PG_HIP(hipGetLastError());
                    }
                });
            }
        }
    }
    std::vector<uint64_t> h((size_t)np);
    uint64_t n3s[4] = {0, 0, 0, 0};
    PG_HIP(hipMemcpyAsync(h.data(), sup_pat, sizeof(uint64_t) * np, hipMemcpyDeviceToHost, s));
    PG_HIP(hipMemcpyAsync(n3s, n_emb, sizeof(n3s), hipMemcpyDeviceToHost, s));
    PG_HIP(hipStreamSynchronize(s));
    const uint64_t n3 = max_edges == 4 ? (uint64_t)n3_stored : n3s[0];
    if (prof_on()) {
        // embeddings generated at every level (levels 2, 3 and 4 from the
        // filtered parents)
        ProfScope ps("fsm_embeddings", s, (double)E + (double)n2_total + (double)n3 + (double)n3s[2]);
        // algorithmic bytes of one domain-bit pass over level 3: per
        // parent its two edge ids, their four endpoints and three
        // row-pointer pairs (72 B); per scanned list element its vertex and
        // edge id (8 B); per embedding the new vertex's label (4 B) and a
        // read-modify-write of one domain word per vertex (4 x 8 B)
        const double walk = 72.0 * (double)m2_total + 8.0 * (double)n3s[1];
        if (l3_passes > 0) ProfScope pw("fsm_l3_bits_work", s, (double)l3_passes * (walk + 36.0 * (double)n3));
        if (max_edges == 3 && m2_total > 0) {
            // the histogram pass: the same walk, per embedding the new
            // vertex's label and a histogram update (4 + 8 B), per parent its
            // child count (4 B)
            ProfScope ph("fsm_l3_hist_work", s, walk + 12.0 * (double)n3 + 4.0 * (double)m2_total);
        }
        // the key pass: the walk, per parent its offset (8 B), per embedding
        // the new vertex's label and four 8-byte keys; the block pass: each
        // key read once and every bitmap word written once
        if (l3_key_passes > 0) {
            ProfScope pk("fsm_l3_keys_work", s,
                         (double)l3_key_passes * (walk + 8.0 * (double)m2_total + 36.0 * (double)n3));
            ProfScope pa("fsm_bits_apply_work", s, 8.0 * apply_keys + 4.0 * apply_words);
        }
    }
    size_t nf = 0;
    for (int64_t p = 0; p < np; ++p) {
        supports[p] = h[p];
        nf += h[p] > 0;
    }
    if (n_frequent) *n_frequent = nf;
}

}  // namespace pg
