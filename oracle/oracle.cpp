/*
 * CPU oracle for graph pattern mining counts -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, obviously correct reference computations used to check the
 * HIP path.  Only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark may load this library.  It shares no code with the HIP
 * library.
 *
 * Definitions followed (Pangolin, VLDB 2020):
 *  - k-clique count: number of k-vertex subsets that are pairwise adjacent
 *    (section 2.2; TC is the case k = 3).  Each clique is counted once by
 *    enumerating it in the order of a total vertex order: the degree order
 *    of section 4.1 (higher degree later, ties broken by larger id).
 *  - k-motif counts: for each connected k-vertex pattern, the number of
 *    vertex-induced k-subsets whose induced subgraph is isomorphic to it
 *    (section 2.1 vertex-induced embeddings, section 2.2 motif counting).
 *    Enumeration by ESU (Wernicke 2006), which visits every connected
 *    induced subset exactly once; classification by edge count and maximum
 *    degree for k = 3, 4; for k = 5 by the smallest relabelled pair mask.
 *  - Closed-form pieces for 4-motifs: non-induced pattern counts from
 *    degrees, per-edge triangle counts and common-neighbour counts.
 *  - Frequent subgraph mining: edge-induced embeddings (section 2.1) are
 *    connected edge subsets, enumerated once each by ESU on the line graph;
 *    their labelled pattern is found by trying every vertex permutation;
 *    minimum-image (domain) support (section 2.2) is the smallest number
 *    of distinct graph vertices any pattern vertex is mapped to, over all
 *    label-preserving subgraph isomorphisms.
 */
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>
#include <parallel/algorithm>
#include <omp.h>

typedef int64_t i64;
typedef int32_t i32;
typedef uint64_t u64;

/* The thread count asked for one call (0 = all), restored when it ends so
 * that a call on a tiny graph does not leave later calls single-threaded. */
struct ThreadScope {
    int prev;
    explicit ThreadScope(int nthreads) : prev(omp_get_max_threads()) {
        if (nthreads > 0) omp_set_num_threads(nthreads);
    }
    ~ThreadScope() { omp_set_num_threads(prev); }
};

extern "C" int or_max_threads(void) { return omp_get_max_threads(); }

/* ================================================================ cliques */

/* Counts cliques of size `left` more vertices inside candidate set `cand`
 * (all of whose members are adjacent to every vertex chosen so far and come
 * later in the order).  out[w] holds w's later neighbours, sorted by id. */
static u64 clique_rec(const std::vector<i32>& cand, int left,
                      const std::vector<std::vector<i32>>& out) {
    if (left == 1) return (u64)cand.size();
    u64 total = 0;
    std::vector<i32> next;
    for (i32 w : cand) {
        next.clear();
        std::set_intersection(cand.begin(), cand.end(), out[w].begin(), out[w].end(),
                              std::back_inserter(next));
        if ((int)next.size() >= left - 1) total += clique_rec(next, left - 1, out);
    }
    return total;
}

static std::vector<std::vector<i32>> degree_order_out(i64 n, const i64* rp, const i32* col) {
    std::vector<std::vector<i32>> out((size_t)n);
    for (i64 u = 0; u < n; ++u) {
        i64 du = rp[u + 1] - rp[u];
        for (i64 j = rp[u]; j < rp[u + 1]; ++j) {
            i32 v = col[j];
            i64 dv = rp[v + 1] - rp[v];
            /* u -> v iff (deg u, u) < (deg v, v) */
            if (du < dv || (du == dv && u < v)) out[u].push_back(v);
        }
    }
    return out;
}

extern "C" u64 or_clique_count(i64 n, const i64* rp, const i32* col, int k, int nthreads) {
    ThreadScope threads(nthreads);
    if (k <= 0) return 0;
    if (k == 1) return (u64)n;
    auto out = degree_order_out(n, rp, col);
    u64 total = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : total)
    for (i64 v = 0; v < n; ++v) total += clique_rec(out[v], k - 1, out);
    return total;
}

/* Same count restricted to cliques whose first vertex in the degree order is
 * one of roots[0..nr); per-root counts go to per_root[]. */
extern "C" u64 or_clique_count_roots(i64 n, const i64* rp, const i32* col, int k,
                                     const i64* roots, i64 nr, u64* per_root, int nthreads) {
    ThreadScope threads(nthreads);
    auto out = degree_order_out(n, rp, col);
    u64 total = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : total)
    for (i64 i = 0; i < nr; ++i) {
        u64 c = (k == 1) ? 1 : clique_rec(out[roots[i]], k - 1, out);
        if (per_root) per_root[i] = c;
        total += c;
    }
    return total;
}

/* ================================================================= motifs */

static inline bool adjacent(const i64* rp, const i32* col, i32 u, i32 v) {
    return std::binary_search(col + rp[u], col + rp[u + 1], v);
}

/* Pattern of an induced k-subset, k = 3 or 4:
 *   k=3: 0 wedge, 1 triangle
 *   k=4: 0 path P4, 1 star, 2 cycle C4, 3 paw, 4 diamond, 5 clique K4
 * decided from the number of edges and the largest degree. */
static int classify(const i32* vs, int k, const i64* rp, const i32* col) {
    int deg[4] = {0, 0, 0, 0}, edges = 0;
    for (int a = 0; a < k; ++a)
        for (int b = a + 1; b < k; ++b)
            if (adjacent(rp, col, vs[a], vs[b])) { deg[a]++; deg[b]++; edges++; }
    int dmax = 0;
    for (int a = 0; a < k; ++a) dmax = std::max(dmax, deg[a]);
    if (k == 3) return edges == 3 ? 1 : 0;
    switch (edges) {
        case 3: return dmax == 3 ? 1 : 0;
        case 4: return dmax == 3 ? 3 : 2;
        case 5: return 4;
        case 6: return 5;
    }
    return -1; /* disconnected: never reached by ESU */
}

/* k=5: the class of an induced 5-subset is found from its 10-bit pair mask
 * (bit b(b-1)/2 + a for positions a < b).  Classes are the connected
 * 5-vertex graphs numbered by (edge count, smallest mask over all 120
 * relabellings); the table is built once by trying every relabelling. */
/* Classes of 5-vertex graphs, built by discovery: the 1024 pair masks are
 * visited by increasing (edge count, mask value); a connected mask that is
 * isomorphic to no class found so far opens a new class.  So classes come
 * out ordered by edge count, and each class's first mask is its smallest,
 * which is the documented order.  of[m] = the class isomorphic to m (-1 for
 * a disconnected mask).  Isomorphism is tested on 5x5 adjacency matrices
 * under all 120 vertex orders. */
struct Class5 {
    signed char of[1024];
    static void matrix(int m, bool a[5][5]) {
        int bit = 0;
        for (int j = 0; j < 5; ++j)
            for (int i = 0; i < 5; ++i) a[i][j] = false;
        for (int j = 1; j < 5; ++j)
            for (int i = 0; i < j; ++i, ++bit) a[i][j] = a[j][i] = (m >> bit) & 1;
    }
    static bool isomorphic(int x, int y) {
        if (__builtin_popcount(x) != __builtin_popcount(y)) return false;
        bool A[5][5], B[5][5];
        matrix(x, A);
        matrix(y, B);
        int p[5] = {0, 1, 2, 3, 4};
        do {
            bool same = true;
            for (int i = 0; i < 5 && same; ++i)
                for (int j = 0; j < 5 && same; ++j) same = A[i][j] == B[p[i]][p[j]];
            if (same) return true;
        } while (std::next_permutation(p, p + 5));
        return false;
    }
    static bool connected(int m) {
        bool A[5][5];
        matrix(m, A);
        bool seen[5] = {true, false, false, false, false};
        int stack[5] = {0}, top = 1, count = 1;
        while (top) {
            int v = stack[--top];
            for (int u = 0; u < 5; ++u)
                if (A[v][u] && !seen[u]) {
                    seen[u] = true;
                    stack[top++] = u;
                    ++count;
                }
        }
        return count == 5;
    }
    Class5() {
        std::vector<int> order(1024);
        for (int m = 0; m < 1024; ++m) order[m] = m;
        std::stable_sort(order.begin(), order.end(),
                         [](int x, int y) { return __builtin_popcount(x) < __builtin_popcount(y); });
        std::vector<int> reps;
        for (int m : order) {
            if (!connected(m)) continue;
            bool known = false;
            for (int r : reps)
                if (isomorphic(m, r)) { known = true; break; }
            if (!known) reps.push_back(m);
        }
        for (int m = 0; m < 1024; ++m) {
            of[m] = -1;
            if (!connected(m)) continue;
            for (size_t c = 0; c < reps.size(); ++c)
                if (isomorphic(m, reps[c])) { of[m] = (signed char)c; break; }
        }
    }
};

static int classify5(const i32* vs, const i64* rp, const i32* col) {
    static const Class5 table;
    int m = 0;
    for (int b = 1; b < 5; ++b)
        for (int a = 0; a < b; ++a)
            if (adjacent(rp, col, vs[a], vs[b])) m |= 1 << (b * (b - 1) / 2 + a);
    return table.of[m];
}

struct Esu {
    const i64* rp; const i32* col; int k; u64* counts;
};

/* ESU: sub holds the current connected subset (sub[0] is its smallest
 * vertex), ext the extension set. */
static void esu_rec(const Esu& E, std::vector<i32>& sub, std::vector<i32> ext) {
    if ((int)sub.size() == E.k) {
        int p = E.k == 5 ? classify5(sub.data(), E.rp, E.col) : classify(sub.data(), E.k, E.rp, E.col);
        E.counts[p]++;
        return;
    }
    const i32 root = sub[0];
    while (!ext.empty()) {
        i32 w = ext.back();
        ext.pop_back();
        std::vector<i32> ext2 = ext;
        /* exclusive neighbours of w: not in sub, not adjacent to sub */
        for (i64 j = E.rp[w]; j < E.rp[w + 1]; ++j) {
            i32 u = E.col[j];
            if (u <= root) continue;
            bool bad = false;
            for (i32 s : sub)
                if (s == u || adjacent(E.rp, E.col, s, u)) { bad = true; break; }
            if (bad) continue;
            if (std::find(ext2.begin(), ext2.end(), u) == ext2.end()) ext2.push_back(u);
        }
        sub.push_back(w);
        esu_rec(E, sub, ext2);
        sub.pop_back();
    }
}

/* counts[] receives 2 (k=3), 6 (k=4) or 21 (k=5) values. */
extern "C" void or_motif_esu(i64 n, const i64* rp, const i32* col, int k, u64* counts, int nthreads) {
    ThreadScope threads(nthreads);
    const int np = (k == 3) ? 2 : (k == 4 ? 6 : 21);
    for (int p = 0; p < np; ++p) counts[p] = 0;
#pragma omp parallel
    {
        u64 local[21] = {0};
        Esu E{rp, col, k, local};
#pragma omp for schedule(dynamic, 16)
        for (i64 v = 0; v < n; ++v) {
            std::vector<i32> sub{(i32)v};
            std::vector<i32> ext;
            for (i64 j = rp[v]; j < rp[v + 1]; ++j)
                if (col[j] > v) ext.push_back(col[j]);
            esu_rec(E, sub, ext);
        }
#pragma omp critical
        for (int p = 0; p < np; ++p) counts[p] += local[p];
    }
}

/* ESU restricted to subsets whose smallest vertex is in roots[]. */
extern "C" void or_motif_esu_roots(i64 n, const i64* rp, const i32* col, int k, const i64* roots,
                                   i64 nr, u64* counts, int nthreads) {
    (void)n;
    ThreadScope threads(nthreads);
    const int np = (k == 3) ? 2 : (k == 4 ? 6 : 21);
    for (int p = 0; p < np; ++p) counts[p] = 0;
#pragma omp parallel
    {
        u64 local[21] = {0};
        Esu E{rp, col, k, local};
#pragma omp for schedule(dynamic, 1)
        for (i64 i = 0; i < nr; ++i) {
            i32 v = (i32)roots[i];
            std::vector<i32> sub{v};
            std::vector<i32> ext;
            for (i64 j = rp[v]; j < rp[v + 1]; ++j)
                if (col[j] > v) ext.push_back(col[j]);
            esu_rec(E, sub, ext);
        }
#pragma omp critical
        for (int p = 0; p < np; ++p) counts[p] += local[p];
    }
}

/* Pieces of the closed-form 4-motif counts (all exact integers):
 *   parts[0] = sum_v C(d_v, 2)                 (non-induced wedges)
 *   parts[1] = T, number of triangles
 *   parts[2] = sum_v C(d_v, 3)                 (non-induced 3-stars)
 *   parts[3] = sum_{uv in E} (d_u-1)(d_v-1)    (before removing triangles)
 *   parts[4] = sum_{u<w} C(c(u,w), 2)          (twice the non-induced 4-cycles)
 *   parts[5] = sum_v t_v (d_v - 2)             (non-induced paws)
 *   parts[6] = sum_{uv in E} C(t_uv, 2)        (non-induced diamonds)
 * where t_uv = common neighbours of an edge, t_v = triangles at v and
 * c(u,w) = common neighbours of a vertex pair. */
extern "C" void or_motif_parts(i64 n, const i64* rp, const i32* col, u64* parts, int nthreads) {
    ThreadScope threads(nthreads);
    u64 wedges = 0, star = 0, p4raw = 0, tri3 = 0, dia = 0;
    std::vector<u64> tv((size_t)n, 0);
    /* per-edge triangles by merging the two sorted lists */
#pragma omp parallel for schedule(dynamic, 256) reduction(+ : wedges, star, p4raw, tri3, dia)
    for (i64 u = 0; u < n; ++u) {
        u64 du = (u64)(rp[u + 1] - rp[u]);
        wedges += du * (du - (du > 0)) / 2;
        if (du >= 3) star += du * (du - 1) * (du - 2) / 6;
        for (i64 j = rp[u]; j < rp[u + 1]; ++j) {
            i32 v = col[j];
            u64 dv = (u64)(rp[v + 1] - rp[v]);
            /* t_uv, computed from u's side for every directed entry */
            const i32* a = col + rp[u]; const i32* ae = col + rp[u + 1];
            const i32* b = col + rp[v]; const i32* be = col + rp[v + 1];
            u64 t = 0;
            while (a < ae && b < be) {
                if (*a < *b) ++a; else if (*b < *a) ++b; else { ++t; ++a; ++b; }
            }
            tv[u] += t;        /* each triangle at u seen twice (two edges at u) */
            if (u < v) {
                p4raw += (du - 1) * (dv - 1);
                tri3 += t;
                dia += t * (t - (t > 0)) / 2;
            }
        }
    }
    u64 paw = 0;
#pragma omp parallel for schedule(static) reduction(+ : paw)
    for (i64 v = 0; v < n; ++v) {
        u64 d = (u64)(rp[v + 1] - rp[v]);
        u64 t = tv[v] / 2;
        if (d >= 2) paw += t * (d - 2);
    }
    /* common-neighbour pair counts: for each u, count paths u-v-w with w > u */
    u64 c4twice = 0;
#pragma omp parallel reduction(+ : c4twice)
    {
        std::vector<u64> cnt((size_t)n, 0);
        std::vector<i32> touched;
#pragma omp for schedule(dynamic, 64)
        for (i64 u = 0; u < n; ++u) {
            touched.clear();
            for (i64 j = rp[u]; j < rp[u + 1]; ++j) {
                i32 v = col[j];
                for (i64 l = rp[v]; l < rp[v + 1]; ++l) {
                    i32 w = col[l];
                    if (w <= u) continue;
                    if (cnt[w]++ == 0) touched.push_back(w);
                }
            }
            for (i32 w : touched) {
                u64 c = cnt[w];
                c4twice += c * (c - 1) / 2;
                cnt[w] = 0;
            }
        }
    }
    parts[0] = wedges;
    parts[1] = tri3 / 3;
    parts[2] = star;
    parts[3] = p4raw;
    parts[4] = c4twice;
    parts[5] = paw;
    parts[6] = dia;
}

/* ==================================================================== FSM */

/* Labelled patterns with 1..4 edges.  A shape is a connected unlabelled
 * graph with numbered vertices (positions); a labelled pattern is a shape
 * with one label per position.  Tuples that a symmetry of the shape maps
 * onto each other name one pattern, represented by the tuple that
 * canonical_tuple() returns.  The dense index lists the shapes in the order
 * below and, inside a shape, its representative tuples in lexicographic
 * order:
 *   0 edge        (a, b)
 *   1 wedge       (centre, leaf, leaf)
 *   2 triangle    (a, b, c)
 *   3 path P4     labels along the path
 *   4 star K1,3   (centre, leaf, leaf, leaf)
 *   5 path P5     labels along the path
 *   6 star K1,4   (centre, four leaves)
 *   7 fork        (vertex of degree 3, its two leaves, the middle vertex of
 *                  its leg of length 2, the end of that leg)
 *   8 cycle C4    labels around the cycle
 *   9 paw         (triangle vertex of degree 3, its pendant vertex, the two
 *                  other triangle vertices)
 * Shapes 0, 1-2, 3-4 and 5-9 have 1, 2, 3 and 4 edges. */
static const int SHAPE_NV[10] = {2, 3, 3, 4, 4, 5, 5, 5, 4, 4};
static const int SHAPE_NE[10] = {1, 2, 3, 3, 3, 4, 4, 4, 4, 4};
static const int N_SHAPES = 10;

/* the representative of label tuple t of shape s, in place */
static void canonical_tuple(int s, int* t) {
    const int n = SHAPE_NV[s];
    switch (s) {
        case 0: case 2:                      /* every position alike */
            std::sort(t, t + n);
            break;
        case 1: case 4: case 6:              /* leaves of a star */
            std::sort(t + 1, t + n);
            break;
        case 3: case 5: {                    /* a path read from either end */
            int r[5];
            for (int i = 0; i < n; ++i) r[i] = t[n - 1 - i];
            if (std::lexicographical_compare(r, r + n, t, t + n)) std::copy(r, r + n, t);
            break;
        }
        case 7:                              /* the fork's two leaves */
            std::sort(t + 1, t + 3);
            break;
        case 8: {                            /* a cycle: rotations and reflections */
            int best[4] = {t[0], t[1], t[2], t[3]};
            for (int rot = 0; rot < 4; ++rot)
                for (int dir = 0; dir < 2; ++dir) {
                    int c[4];
                    for (int i = 0; i < 4; ++i) c[i] = dir ? t[(rot - i + 4) % 4] : t[(rot + i) % 4];
                    if (std::lexicographical_compare(c, c + 4, best, best + 4)) std::copy(c, c + 4, best);
                }
            std::copy(best, best + 4, t);
            break;
        }
        case 9:                              /* the paw's two triangle vertices of degree 2 */
            std::sort(t + 2, t + 4);
            break;
    }
}

/* Index tables by enumeration: every label tuple of a shape, in
 * lexicographic order, is tested for being its own representative; the
 * representatives get consecutive numbers. */
struct PatternIndex {
    int L = -1, max_edges = -1;
    u64 base[N_SHAPES + 1];
    std::vector<int32_t> rank[N_SHAPES];     /* tuple code -> rank in its block, or -1 */

    static u64 code_of(const int* t, int n, u64 L) {
        u64 c = 0;
        for (int i = 0; i < n; ++i) c = c * L + (u64)t[i];
        return c;
    }
    void build(int L_, int me) {
        if (L_ == L && me == max_edges) return;
        L = L_;
        max_edges = me;
        base[0] = 0;
        for (int s = 0; s < N_SHAPES; ++s) {
            rank[s].clear();
            u64 count = 0;
            if (SHAPE_NE[s] <= me) {
                const int n = SHAPE_NV[s];
                u64 size = 1;
                for (int i = 0; i < n; ++i) size *= (u64)L;
                rank[s].assign((size_t)size, -1);
                int t[5], c[5];
                for (u64 x = 0; x < size; ++x) {
                    u64 r = x;
                    for (int i = n - 1; i >= 0; --i) { t[i] = (int)(r % (u64)L); r /= (u64)L; }
                    std::copy(t, t + n, c);
                    canonical_tuple(s, c);
                    if (std::equal(t, t + n, c)) rank[s][(size_t)x] = (int32_t)count++;
                }
            }
            base[s + 1] = base[s] + count;
        }
    }
    u64 total() const { return base[N_SHAPES]; }
    /* index of the pattern of shape s whose positions carry labels lab */
    u64 index(int s, const int* lab) const {
        int t[5];
        std::copy(lab, lab + SHAPE_NV[s], t);
        canonical_tuple(s, t);
        return base[s] + (u64)rank[s][(size_t)code_of(t, SHAPE_NV[s], (u64)L)];
    }
};

static PatternIndex g_index;

/* label tuples of 5 positions are enumerated in full: keep the tables small */
static bool index_fits(int max_edges, int L) {
    const double size = std::pow((double)L, max_edges >= 4 ? 5.0 : 4.0);
    return L >= 1 && max_edges >= 1 && max_edges <= 4 && size <= (double)(1 << 26);
}

extern "C" u64 or_fsm_num_patterns(int max_edges, int L) {
    if (!index_fits(max_edges, L)) return 0;
    g_index.build(L, max_edges);
    return g_index.total();
}

extern "C" u64 or_fsm_pattern_index(int shape, const int* lab, int L) {
    if (shape < 0 || shape >= N_SHAPES || !index_fits(SHAPE_NE[shape], L)) return ~0ULL;
    g_index.build(L, std::max(g_index.max_edges, SHAPE_NE[shape]));
    return g_index.index(shape, lab);
}

struct FsmCtx {
    i64 n;
    const i64* rp; const i32* col; const i32* lab; int L; int K;
    const i32* eu; const i32* ev;             /* undirected edges, id order */
    const i64* inc_ptr; const i64* inc;       /* edges incident to a vertex */
    const PatternIndex* index;
    std::vector<u64>* keys;                   /* (pattern, position, vertex) */
    u64* emb_count;                           /* embeddings per level */
};

static inline bool share(const FsmCtx& C, i64 x, i64 y) {
    return C.eu[x] == C.eu[y] || C.eu[x] == C.ev[y] || C.ev[x] == C.eu[y] || C.ev[x] == C.ev[y];
}

/* Shape of a connected edge set on vertices 0..nv-1 with adjacency adj and
 * degrees deg, and its vertices in the shape's position order. */
static int shape_positions(int ne, int nv, int adj[5][5], const int* deg, int* pos) {
    int dmax = 0;
    for (int i = 0; i < nv; ++i) dmax = std::max(dmax, deg[i]);
    auto first_of_degree = [&](int d, int skip) {
        for (int i = 0; i < nv; ++i) if (deg[i] == d && i != skip) return i;
        return -1;
    };
    auto walk = [&](int start) {     /* a path or a cycle, from start */
        int prev = -1, cur = start;
        for (int s = 0; s < nv; ++s) {
            pos[s] = cur;
            int nxt = -1;
            for (int j = 0; j < nv; ++j)
                if (j != prev && j != cur && adj[cur][j]) { nxt = j; break; }
            prev = cur;
            cur = nxt;
        }
    };
    auto star = [&](int centre) {
        int k = 1;
        pos[0] = centre;
        for (int i = 0; i < nv; ++i) if (i != centre) pos[k++] = i;
    };
    if (ne == 1) { pos[0] = 0; pos[1] = 1; return 0; }
    if (ne == 2) { star(first_of_degree(2, -1)); return 1; }
    if (ne == 3 && nv == 3) { pos[0] = 0; pos[1] = 1; pos[2] = 2; return 2; }
    if (ne == 3) {
        if (dmax == 3) { star(first_of_degree(3, -1)); return 4; }
        walk(first_of_degree(1, -1));
        return 3;
    }
    /* four edges */
    if (nv == 5) {
        if (dmax == 4) { star(first_of_degree(4, -1)); return 6; }
        if (dmax == 2) { walk(first_of_degree(1, -1)); return 5; }
        const int c = first_of_degree(3, -1);
        int k = 1, x = -1;
        pos[0] = c;
        for (int j = 0; j < nv; ++j) {
            if (!adj[c][j]) continue;
            if (deg[j] == 1) pos[k++] = j;
            else x = j;
        }
        pos[3] = x;
        for (int j = 0; j < nv; ++j) if (j != c && adj[x][j]) pos[4] = j;
        return 7;
    }
    if (dmax == 2) { walk(0); return 8; }
    pos[0] = first_of_degree(3, -1);
    pos[1] = first_of_degree(1, -1);
    pos[2] = first_of_degree(2, -1);
    pos[3] = first_of_degree(2, pos[2]);
    return 9;
}

/* Classify one connected edge set and emit its domain keys. */
static void fsm_emit(const FsmCtx& C, const std::vector<i64>& es) {
    i32 vs[5]; int nv = 0;
    auto addv = [&](i32 v) {
        for (int i = 0; i < nv; ++i) if (vs[i] == v) return;
        vs[nv++] = v;
    };
    for (i64 e : es) { addv(C.eu[e]); addv(C.ev[e]); }
    int adj[5][5] = {{0}};
    auto at = [&](i32 v) { for (int i = 0; i < nv; ++i) if (vs[i] == v) return i; return -1; };
    for (i64 e : es) {
        int a = at(C.eu[e]), b = at(C.ev[e]);
        adj[a][b] = adj[b][a] = 1;
    }
    int deg[5] = {0, 0, 0, 0, 0};
    for (int i = 0; i < nv; ++i)
        for (int j = 0; j < nv; ++j) deg[i] += adj[i][j];
    const int ne = (int)es.size();
    int pos[5];
    const int shape = shape_positions(ne, nv, adj, deg, pos);
    int lab[5];
    for (int i = 0; i < nv; ++i) lab[i] = C.lab[vs[pos[i]]];
    const u64 pid = C.index->index(shape, lab);
    C.emb_count[ne - 1]++;
    /* domains: a canonical code per vertex order (labels in order, then the
     * absent pairs in order); the orders that minimise it differ by the
     * pattern's label-preserving automorphisms, so vertex vs[pp[i]] of any
     * minimising order pp belongs to the domain of code position i */
    int perm[5] = {0, 1, 2, 3, 4};
    u64 best = ~0ULL;
    std::vector<std::vector<int>> best_perms;
    do {
        u64 code = 0;
        for (int i = 0; i < nv; ++i) code = code * 64 + (u64)C.lab[vs[perm[i]]];
        for (int i = 0; i < nv; ++i)
            for (int j = i + 1; j < nv; ++j) code = code * 2 + (u64)(1 - adj[perm[i]][perm[j]]);
        if (code < best) { best = code; best_perms.clear(); }
        if (code == best) best_perms.push_back(std::vector<int>(perm, perm + nv));
    } while (std::next_permutation(perm, perm + nv));
    for (const auto& pp : best_perms)
        for (int i = 0; i < nv; ++i)
            C.keys->push_back(((pid * 8 + (u64)i) << 32) | (u64)(uint32_t)vs[pp[i]]);
}

static void fsm_esu(const FsmCtx& C, std::vector<i64>& sub, std::vector<i64> ext) {
    fsm_emit(C, sub);
    if ((int)sub.size() == C.K) return;
    const i64 root = sub[0];
    while (!ext.empty()) {
        i64 w = ext.back();
        ext.pop_back();
        std::vector<i64> ext2 = ext;
        /* line-graph neighbours of w that are exclusive w.r.t. sub */
        const i32 ends[2] = {C.eu[w], C.ev[w]};
        for (int t = 0; t < 2; ++t) {
            i32 x = ends[t];
            for (i64 j = C.inc_ptr[x]; j < C.inc_ptr[x + 1]; ++j) {
                i64 u = C.inc[j];
                if (u <= root || u == w) continue;
                bool bad = false;
                for (i64 s : sub) if (s == u || share(C, s, u)) { bad = true; break; }
                if (bad) continue;
                if (std::find(ext2.begin(), ext2.end(), u) == ext2.end()) ext2.push_back(u);
            }
        }
        sub.push_back(w);
        fsm_esu(C, sub, ext2);
        sub.pop_back();
    }
}

/* Unfiltered MNI supports of every labelled connected pattern with
 * 1..max_edges edges (max_edges <= 4), written at the dense index.
 * emb_count[j] = number of (j+1)-edge embeddings (j < 4).  Returns -1 for
 * sizes the index tables do not cover. */
extern "C" int or_fsm_supports(i64 n, const i64* rp, const i32* col, const i32* labels, int L,
                               int max_edges, u64* supports, u64* emb_count, int nthreads) {
    ThreadScope threads(nthreads);
    if (!index_fits(max_edges, L)) return -1;
    std::vector<i32> eu, ev;
    for (i64 u = 0; u < n; ++u)
        for (i64 j = rp[u]; j < rp[u + 1]; ++j)
            if (col[j] > u) { eu.push_back((i32)u); ev.push_back(col[j]); }
    const i64 E = (i64)eu.size();
    std::vector<i64> inc_ptr((size_t)n + 1, 0), inc((size_t)(2 * E));
    for (i64 e = 0; e < E; ++e) { inc_ptr[eu[e] + 1]++; inc_ptr[ev[e] + 1]++; }
    for (i64 v = 0; v < n; ++v) inc_ptr[v + 1] += inc_ptr[v];
    {
        std::vector<i64> fill(inc_ptr.begin(), inc_ptr.end() - 1);
        for (i64 e = 0; e < E; ++e) { inc[fill[eu[e]]++] = e; inc[fill[ev[e]]++] = e; }
    }
    g_index.build(L, max_edges);
    const u64 np = g_index.total();
    for (u64 i = 0; i < np; ++i) supports[i] = 0;
    for (int j = 0; j < 4; ++j) emb_count[j] = 0;

    int nt = omp_get_max_threads();
    std::vector<std::vector<u64>> keys((size_t)nt);
    std::vector<u64> cnt((size_t)nt * 4, 0);
#pragma omp parallel
    {
        int t = omp_get_thread_num();
        FsmCtx C{n, rp, col, labels, L, max_edges, eu.data(), ev.data(), inc_ptr.data(), inc.data(),
                 &g_index, &keys[t], &cnt[(size_t)t * 4]};
#pragma omp for schedule(dynamic, 256)
        for (i64 e = 0; e < E; ++e) {
            std::vector<i64> sub{e};
            std::vector<i64> ext;
            for (int s = 0; s < 2; ++s) {
                i32 x = s ? ev[e] : eu[e];
                for (i64 j = inc_ptr[x]; j < inc_ptr[x + 1]; ++j)
                    if (inc[j] > e && std::find(ext.begin(), ext.end(), inc[j]) == ext.end())
                        ext.push_back(inc[j]);
            }
            fsm_esu(C, sub, ext);
        }
    }
    for (int t = 0; t < nt; ++t)
        for (int j = 0; j < 4; ++j) emb_count[j] += cnt[(size_t)t * 4 + j];
    size_t total = 0;
    for (auto& k : keys) total += k.size();
    std::vector<u64> all;
    all.reserve(total);
    for (auto& k : keys) { all.insert(all.end(), k.begin(), k.end()); std::vector<u64>().swap(k); }
    __gnu_parallel::sort(all.begin(), all.end());
    all.erase(std::unique(all.begin(), all.end()), all.end());
    /* keys are sorted by (pattern, position): the distinct vertices of each
     * position are a run; the support is the smallest run of the pattern */
    size_t i = 0;
    while (i < all.size()) {
        const u64 pp = all[i] >> 32;
        size_t j = i;
        while (j < all.size() && (all[j] >> 32) == pp) ++j;
        const u64 pid = pp / 8, run = (u64)(j - i);
        if (supports[pid] == 0 || run < supports[pid]) supports[pid] = run;
        i = j;
    }
    return 0;
}
