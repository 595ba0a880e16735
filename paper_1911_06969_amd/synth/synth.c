/*
 * Seeded synthetic graph generators.
 *
 * This file produces inputs only.  It contains none of the mining
 * arithmetic (no orientation, no intersection, no classification, no
 * support computation): it draws random graphs and writes them as the
 * canonical CSR the mining method assumes (symmetric, no self-loops, no
 * duplicate edges, neighbour lists ascending; Pangolin section 6.1).
 * Both the HIP path and the CPU oracle consume what it writes.
 *
 * Randomness is counter based: every draw is splitmix64 of (seed, stream,
 * counter), so results do not depend on the number of threads.
 *
 * Generators:
 *   - R-MAT (Chakrabarti et al.): edge_factor * 2^scale sampled pairs, each
 *     choosing one quadrant per bit with probabilities a, b, c, d=1-a-b-c,
 *     followed by a seeded uniform vertex permutation; loops and duplicate
 *     pairs are removed when the CSR is built.
 *   - Erdos-Renyi G(n, p) by geometric skipping (Batagelj and Brandes 2005).
 *   - A batch of G(n_g, p_g) graphs with n_g uniform on [nmin, nmax] and
 *     p_g uniform on [pmin, pmax].
 *   - Vertex labels i.i.d. uniform over [0, L).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#include <omp.h>

static inline uint64_t mix64(uint64_t z) {
    z += 0x9e3779b97f4a7c15ULL;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

/* counter-based draw: stream separates independent uses of one seed */
static inline uint64_t draw64(uint64_t seed, uint64_t stream, uint64_t ctr) {
    return mix64(mix64(seed ^ (stream * 0xd1b54a32d192ed03ULL)) + ctr * 0x9e3779b97f4a7c15ULL);
}

static inline double draw_u01(uint64_t seed, uint64_t stream, uint64_t ctr) {
    return (double)(draw64(seed, stream, ctr) >> 11) * (1.0 / 9007199254740992.0);
}

/* ---------------------------------------------------------------- R-MAT */

/* Writes m sampled (src, dst) pairs over 2^scale vertices, already passed
 * through a seeded uniform permutation of the vertex ids. */
void synth_rmat_pairs(int scale, int64_t m, double a, double b, double c,
                      uint64_t seed, int32_t* src, int32_t* dst) {
    const int64_t n = (int64_t)1 << scale;
    const double ab = a + b;
    const double d = 1.0 - a - b - c;
    const double p_dst_given_src0 = b / ab;        /* quadrant b vs a */
    const double p_dst_given_src1 = d / (c + d);   /* quadrant d vs c */
    int32_t* perm = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    for (int64_t i = 0; i < n; ++i) perm[i] = (int32_t)i;
    for (int64_t i = n - 1; i > 0; --i) {        /* Fisher-Yates, stream 1 */
        uint64_t r = draw64(seed, 1, (uint64_t)i) % (uint64_t)(i + 1);
        int32_t t = perm[i]; perm[i] = perm[r]; perm[r] = t;
    }
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < m; ++e) {
        int64_t u = 0, v = 0;
        for (int bit = 0; bit < scale; ++bit) {
            uint64_t ctr = ((uint64_t)e * (uint64_t)scale + (uint64_t)bit) * 2u;
            double r1 = draw_u01(seed, 2, ctr);
            double r2 = draw_u01(seed, 2, ctr + 1);
            int sbit = r1 >= ab;
            int dbit = sbit ? (r2 < p_dst_given_src1) : (r2 < p_dst_given_src0);
            u |= (int64_t)sbit << bit;
            v |= (int64_t)dbit << bit;
        }
        src[e] = perm[u];
        dst[e] = perm[v];
    }
    free(perm);
}

static int cmp_i32(const void* x, const void* y) {
    int32_t a = *(const int32_t*)x, b = *(const int32_t*)y;
    return (a > b) - (a < b);
}

/* Builds the canonical symmetric CSR of an undirected pair list: drops
 * loops, symmetrises, sorts each row and removes duplicates.
 * row_ptr has n+1 entries; col must hold 2*m entries.  Returns nnz. */
int64_t synth_csr_from_pairs(int64_t n, int64_t m, const int32_t* src,
                             const int32_t* dst, int64_t* row_ptr, int32_t* col) {
    int64_t* cnt = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    for (int64_t e = 0; e < m; ++e) {
        if (src[e] == dst[e]) continue;
        cnt[src[e] + 1]++;
        cnt[dst[e] + 1]++;
    }
    for (int64_t i = 0; i < n; ++i) cnt[i + 1] += cnt[i];
    int64_t* pos = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    memcpy(pos, cnt, sizeof(int64_t) * (size_t)n);
    for (int64_t e = 0; e < m; ++e) {
        if (src[e] == dst[e]) continue;
        col[pos[src[e]]++] = dst[e];
        col[pos[dst[e]]++] = src[e];
    }
    free(pos);
    int64_t* keep = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t v = 0; v < n; ++v) {
        int32_t* row = col + cnt[v];
        int64_t len = cnt[v + 1] - cnt[v];
        if (len > 1) qsort(row, (size_t)len, sizeof(int32_t), cmp_i32);
        int64_t k = 0;
        for (int64_t i = 0; i < len; ++i)
            if (k == 0 || row[i] != row[k - 1]) row[k++] = row[i];
        keep[v] = k;
    }
    row_ptr[0] = 0;
    for (int64_t v = 0; v < n; ++v) row_ptr[v + 1] = row_ptr[v] + keep[v];
    for (int64_t v = 0; v < n; ++v)   /* in place: destinations never pass sources */
        memmove(col + row_ptr[v], col + cnt[v], sizeof(int32_t) * (size_t)keep[v]);
    free(keep);
    free(cnt);
    return row_ptr[n];
}

/* ------------------------------------------------------------ Erdos-Renyi */

/* Geometric skipping over the pairs (v, w), w < v, in order of (v, w).
 * With rows == NULL only counts.  Otherwise fills a CSR whose rows come out
 * sorted: row v receives its smaller neighbours while v is the current row
 * and its larger ones afterwards, both ascending. */
static int64_t er_one(int64_t n, double p, uint64_t seed, uint64_t stream,
                      int64_t* row_ptr, int32_t* col) {
    if (n < 2 || p <= 0.0) {
        if (row_ptr) for (int64_t i = 0; i <= n; ++i) row_ptr[i] = 0;
        return 0;
    }
    const double lq = log1p(-p);
    int64_t m = 0;
    int64_t* fill = NULL;
    if (row_ptr) fill = (int64_t*)calloc((size_t)n, sizeof(int64_t));
    for (int pass = 0; pass < (row_ptr ? 2 : 1); ++pass) {
        int64_t v = 1, w = -1;
        uint64_t ctr = 0;
        m = 0;
        while (v < n) {
            double r = draw_u01(seed, stream, ctr++);
            int64_t skip = (p >= 1.0) ? 0 : (int64_t)floor(log1p(-r) / lq);
            w += 1 + skip;
            while (w >= v && v < n) { w -= v; v += 1; }
            if (v < n) {
                if (row_ptr && pass == 0) { fill[v]++; fill[w]++; }
                if (row_ptr && pass == 1) {
                    col[row_ptr[v] + fill[v]++] = (int32_t)w;
                    col[row_ptr[w] + fill[w]++] = (int32_t)v;
                }
                m++;
            }
        }
        if (row_ptr && pass == 0) {
            row_ptr[0] = 0;
            for (int64_t i = 0; i < n; ++i) row_ptr[i + 1] = row_ptr[i] + fill[i];
            memset(fill, 0, sizeof(int64_t) * (size_t)n);
        }
    }
    free(fill);
    return m;
}

/* Number of undirected edges G(n, p) draws for this seed. */
int64_t synth_er_count(int64_t n, double p, uint64_t seed) {
    return er_one(n, p, seed, 3, NULL, NULL);
}

/* Fills the CSR (row_ptr: n+1, col: 2*edges). */
void synth_er_fill(int64_t n, double p, uint64_t seed, int64_t* row_ptr, int32_t* col) {
    er_one(n, p, seed, 3, row_ptr, col);
}

void synth_labels(int64_t n, int32_t n_labels, uint64_t seed, int32_t* labels) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        labels[i] = (int32_t)(draw64(seed, 4, (uint64_t)i) % (uint64_t)n_labels);
}

/* ------------------------------------------------------- batch of G(n,p) */

/* Per-graph sizes and edge probabilities, then the per-graph edge counts. */
void synth_er_batch_params(int64_t G, int32_t nmin, int32_t nmax, double pmin, double pmax,
                           uint64_t seed, int32_t* n_out, double* p_out, int64_t* m_out) {
    for (int64_t g = 0; g < G; ++g) {
        n_out[g] = nmin + (int32_t)(draw64(seed, 5, (uint64_t)g) % (uint64_t)(nmax - nmin + 1));
        p_out[g] = pmin + (pmax - pmin) * draw_u01(seed, 6, (uint64_t)g);
    }
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t g = 0; g < G; ++g)
        m_out[g] = er_one(n_out[g], p_out[g], seed, 1000 + (uint64_t)g, NULL, NULL);
}

/* Fills the batched CSR.  Graph g owns vertices [voff[g], voff[g+1]) of the
 * global row_ptr (which holds positions into col) and its col entries are
 * local vertex ids 0..n_g-1. */
void synth_er_batch_fill(int64_t G, const int32_t* n_in, const double* p_in, uint64_t seed,
                         const int64_t* voff, const int64_t* eoff, int64_t* row_ptr, int32_t* col) {
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t g = 0; g < G; ++g) {
        int64_t n = n_in[g];
        int64_t* rp = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
        er_one(n, p_in[g], seed, 1000 + (uint64_t)g, rp, col + eoff[g]);
        for (int64_t i = 0; i < n; ++i) row_ptr[voff[g] + i] = eoff[g] + rp[i];
        free(rp);
    }
    int64_t total_v = voff[G];
    row_ptr[total_v] = eoff[G];
}
