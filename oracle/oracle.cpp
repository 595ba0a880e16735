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
struct Class5 {
    signed char of[1024];
    Class5() {
        int perm[5] = {0, 1, 2, 3, 4};
        std::vector<int> canon(1024, 1 << 20);
        do {
            for (int m = 0; m < 1024; ++m) {
                int r = 0;
                for (int b = 1; b < 5; ++b)
                    for (int a = 0; a < b; ++a)
                        if ((m >> (b * (b - 1) / 2 + a)) & 1) {
                            int x = std::min(perm[a], perm[b]), y = std::max(perm[a], perm[b]);
                            r |= 1 << (y * (y - 1) / 2 + x);
                        }
                canon[m] = std::min(canon[m], r);
            }
        } while (std::next_permutation(perm, perm + 5));
        std::vector<int> codes;
        for (int m = 0; m < 1024; ++m) {
            /* connected: grow the component of vertex 0 */
            int comp = 1, grew = 1;
            while (grew) {
                grew = 0;
                for (int b = 1; b < 5; ++b)
                    for (int a = 0; a < b; ++a)
                        if (((m >> (b * (b - 1) / 2 + a)) & 1) && (((comp >> a) ^ (comp >> b)) & 1)) {
                            comp |= (1 << a) | (1 << b);
                            grew = 1;
                        }
            }
            of[m] = -1;
            if (comp == 31) codes.push_back(canon[m]);
        }
        std::sort(codes.begin(), codes.end(), [](int x, int y) {
            int px = __builtin_popcount(x), py = __builtin_popcount(y);
            return px != py ? px < py : x < y;
        });
        codes.erase(std::unique(codes.begin(), codes.end()), codes.end());
        /* isomorphic masks share the code, so only connected masks match one */
        for (int m = 0; m < 1024; ++m)
            for (size_t c = 0; c < codes.size(); ++c)
                if (codes[c] == canon[m]) of[m] = (signed char)c;
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

/* Dense index of a labelled pattern with at most 3 edges over L labels.
 * shape: 0 edge (a<=b), 1 wedge (centre c; leaves a<=b), 2 triangle
 * (a<=b<=c), 3 path (a,b,c,d) read from the end that gives the smaller
 * sequence, 4 star (centre c; leaves a<=b<=c).  Blocks are laid out in
 * that order. */
static u64 pairs_count(u64 L) { return L * (L + 1) / 2; }
static u64 triples_count(u64 L) { return L * (L + 1) * (L + 2) / 6; }
/* rank of a multiset a<=b<=c in lexicographic order of sorted triples */
static u64 triple_rank(u64 a, u64 b, u64 c, u64 L) {
    u64 r = 0;
    for (u64 x = 0; x < a; ++x) r += (L - x) * (L - x + 1) / 2;
    for (u64 y = a; y < b; ++y) r += (L - y);
    r += c - b;
    return r;
}
static u64 pair_rank(u64 a, u64 b, u64 L) {
    u64 r = 0;
    for (u64 x = 0; x < a; ++x) r += L - x;
    return r + (b - a);
}

extern "C" u64 or_fsm_num_patterns(int max_edges, int L_) {
    u64 L = (u64)L_;
    u64 t = 0;
    if (max_edges >= 1) t += pairs_count(L);
    if (max_edges >= 2) t += L * pairs_count(L);
    if (max_edges >= 3) t += triples_count(L) + (L * L * L * L + L * L) / 2 + L * triples_count(L);
    return t;
}

/* Rank of a path label sequence among the sequences x with x <= reverse(x)
 * (each path pattern read from the end giving the smaller sequence), in
 * lexicographic order.  Built once per label count by walking all L^4
 * sequences in order. */
static std::vector<u64> g_path_rank;
static u64 g_path_rank_L = 0;
static void build_path_rank(u64 L) {
    if (g_path_rank_L == L) return;
    g_path_rank.assign((size_t)(L * L * L * L), ~0ULL);
    u64 r = 0;
    for (u64 x = 0; x < L * L * L * L; ++x) {
        u64 p0 = x / (L * L * L), p1 = (x / (L * L)) % L, p2 = (x / L) % L, p3 = x % L;
        u64 rev = ((p3 * L + p2) * L + p1) * L + p0;
        if (x <= rev) g_path_rank[x] = r++;
    }
    g_path_rank_L = L;
}
static u64 path_rank(u64 a, u64 b, u64 c, u64 d, u64 L) {
    return g_path_rank[(size_t)(((a * L + b) * L + c) * L + d)];
}

static u64 pattern_index(int shape, const int* lab, u64 L) {
    u64 base = 0;
    if (shape == 0) {
        u64 a = std::min(lab[0], lab[1]), b = std::max(lab[0], lab[1]);
        return pair_rank(a, b, L);
    }
    base += pairs_count(L);
    if (shape == 1) { /* lab = centre, leaf, leaf */
        u64 a = std::min(lab[1], lab[2]), b = std::max(lab[1], lab[2]);
        return base + (u64)lab[0] * pairs_count(L) + pair_rank(a, b, L);
    }
    base += L * pairs_count(L);
    if (shape == 2) {
        int s[3] = {lab[0], lab[1], lab[2]};
        std::sort(s, s + 3);
        return base + triple_rank(s[0], s[1], s[2], L);
    }
    base += triples_count(L);
    if (shape == 3) { /* lab = a,b,c,d along the path */
        u64 f = ((u64)lab[0] * L + lab[1]) * L * L + (u64)lab[2] * L + lab[3];
        u64 r = ((u64)lab[3] * L + lab[2]) * L * L + (u64)lab[1] * L + lab[0];
        if (r < f) return base + path_rank(lab[3], lab[2], lab[1], lab[0], L);
        return base + path_rank(lab[0], lab[1], lab[2], lab[3], L);
    }
    base += (L * L * L * L + L * L) / 2;
    /* shape 4: lab = centre, leaf, leaf, leaf */
    int s[3] = {lab[1], lab[2], lab[3]};
    std::sort(s, s + 3);
    return base + (u64)lab[0] * triples_count(L) + triple_rank(s[0], s[1], s[2], L);
}

extern "C" u64 or_fsm_pattern_index(int shape, const int* lab, int L) {
    build_path_rank((u64)L);
    return pattern_index(shape, lab, (u64)L);
}

struct FsmCtx {
    i64 n;
    const i64* rp; const i32* col; const i32* lab; int L; int K;
    const i32* eu; const i32* ev;             /* undirected edges, id order */
    const i64* inc_ptr; const i64* inc;       /* edges incident to a vertex */
    std::vector<u64>* keys;                   /* (pattern, position, vertex) */
    u64* emb_count;                           /* embeddings per level */
};

static inline bool share(const FsmCtx& C, i64 x, i64 y) {
    return C.eu[x] == C.eu[y] || C.eu[x] == C.ev[y] || C.ev[x] == C.eu[y] || C.ev[x] == C.ev[y];
}

/* Classify one connected edge set and emit its domain keys. */
static void fsm_emit(const FsmCtx& C, const std::vector<i64>& es) {
    i32 vs[4]; int nv = 0;
    auto addv = [&](i32 v) {
        for (int i = 0; i < nv; ++i) if (vs[i] == v) return;
        vs[nv++] = v;
    };
    for (i64 e : es) { addv(C.eu[e]); addv(C.ev[e]); }
    int adj[4][4] = {{0}};
    auto pos = [&](i32 v) { for (int i = 0; i < nv; ++i) if (vs[i] == v) return i; return -1; };
    for (i64 e : es) {
        int a = pos(C.eu[e]), b = pos(C.ev[e]);
        adj[a][b] = adj[b][a] = 1;
    }
    /* canonical code: minimum over vertex permutations of
     * (labels in order, adjacency bits in order) */
    int perm[4] = {0, 1, 2, 3};
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
    /* shape and labels of canonical positions */
    const std::vector<int>& p0 = best_perms[0];
    int deg[4] = {0, 0, 0, 0};
    for (int i = 0; i < nv; ++i)
        for (int j = 0; j < nv; ++j) deg[i] += adj[p0[i]][p0[j]];
    int lab[4];
    int ne = (int)es.size();
    int shape = -1;
    if (ne == 1) { shape = 0; lab[0] = C.lab[vs[p0[0]]]; lab[1] = C.lab[vs[p0[1]]]; }
    else if (ne == 2) {
        shape = 1;
        int c = 0; for (int i = 0; i < 3; ++i) if (deg[i] == 2) c = i;
        int k = 1; lab[0] = C.lab[vs[p0[c]]];
        for (int i = 0; i < 3; ++i) if (i != c) lab[k++] = C.lab[vs[p0[i]]];
    } else if (nv == 3) {
        shape = 2; for (int i = 0; i < 3; ++i) lab[i] = C.lab[vs[p0[i]]];
    } else {
        int dmax = 0; for (int i = 0; i < 4; ++i) dmax = std::max(dmax, deg[i]);
        if (dmax == 3) {
            shape = 4;
            int c = 0; for (int i = 0; i < 4; ++i) if (deg[i] == 3) c = i;
            int k = 1; lab[0] = C.lab[vs[p0[c]]];
            for (int i = 0; i < 4; ++i) if (i != c) lab[k++] = C.lab[vs[p0[i]]];
        } else {
            shape = 3;  /* walk the path from one end */
            int cur = 0; for (int i = 0; i < 4; ++i) if (deg[i] == 1) { cur = i; break; }
            int prev = -1;
            for (int s = 0; s < 4; ++s) {
                lab[s] = C.lab[vs[p0[cur]]];
                int nxt = -1;
                for (int j = 0; j < 4; ++j) if (j != prev && j != cur && adj[p0[cur]][p0[j]]) nxt = j;
                prev = cur; cur = nxt;
            }
        }
    }
    u64 pid = pattern_index(shape, lab, (u64)C.L);
    C.emb_count[ne - 1]++;
    /* every minimising permutation maps canonical position i to a vertex of
     * the orbit of that position: all of them enter the domain of i */
    for (const auto& pp : best_perms)
        for (int i = 0; i < nv; ++i)
            C.keys->push_back(((pid * 4 + (u64)i) << 32) | (u64)(uint32_t)vs[pp[i]]);
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
 * 1..max_edges edges (max_edges <= 3), written at the dense index.
 * emb_count[j] = number of (j+1)-edge embeddings. */
extern "C" int or_fsm_supports(i64 n, const i64* rp, const i32* col, const i32* labels, int L,
                               int max_edges, u64* supports, u64* emb_count, int nthreads) {
    ThreadScope threads(nthreads);
    if (max_edges < 1 || max_edges > 3) return -1;
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
    const u64 np = or_fsm_num_patterns(max_edges, L);
    build_path_rank((u64)L);
    for (u64 i = 0; i < np; ++i) supports[i] = 0;
    for (int j = 0; j < 3; ++j) emb_count[j] = 0;

    int nt = omp_get_max_threads();
    std::vector<std::vector<u64>> keys((size_t)nt);
    std::vector<u64> cnt((size_t)nt * 3, 0);
#pragma omp parallel
    {
        int t = omp_get_thread_num();
        FsmCtx C{n, rp, col, labels, L, max_edges, eu.data(), ev.data(), inc_ptr.data(), inc.data(),
                 &keys[t], &cnt[(size_t)t * 3]};
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
        for (int j = 0; j < 3; ++j) emb_count[j] += cnt[(size_t)t * 3 + j];
    size_t total = 0;
    for (auto& k : keys) total += k.size();
    std::vector<u64> all;
    all.reserve(total);
    for (auto& k : keys) { all.insert(all.end(), k.begin(), k.end()); std::vector<u64>().swap(k); }
    __gnu_parallel::sort(all.begin(), all.end());
    all.erase(std::unique(all.begin(), all.end()), all.end());
    /* distinct vertices per (pattern, position); support = min over positions */
    std::vector<u64> dom((size_t)np * 4, 0);
    std::vector<uint8_t> has((size_t)np * 4, 0);
    for (u64 key : all) { dom[key >> 32]++; has[key >> 32] = 1; }
    for (u64 p = 0; p < np; ++p) {
        u64 s = ~0ULL; bool any = false;
        for (int i = 0; i < 4; ++i)
            if (has[p * 4 + i]) { s = std::min(s, dom[p * 4 + i]); any = true; }
        supports[p] = any ? s : 0;
    }
    return 0;
}
