// Graph ingest: copy, validate on the device, and the derived structures
// the mining pipelines start from (degree-ordered DAG for cliques, the
// single-edge embedding list for motifs).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "pg_device.h"
#include "pg_internal.h"

namespace pg {

enum : unsigned {
    BAD_ROWPTR = 1u,
    BAD_RANGE = 2u,
    BAD_LOOP = 4u,
    BAD_ORDER = 8u,
    BAD_SYMMETRY = 16u,
    BAD_LABEL = 32u,
};

// One wave per vertex: row bounds, entry range, no loop, strictly ascending,
// and the reverse entry exists (symmetry).  Also the maximum degree.
__global__ __launch_bounds__(256) void k_validate(int64_t n, int64_t nnz, const int64_t* __restrict__ rp,
                                                  const int32_t* __restrict__ col,
                                                  const int32_t* __restrict__ labels, int32_t n_labels,
                                                  unsigned* __restrict__ flags,
                                                  unsigned long long* __restrict__ max_deg, bool bounds_only) {
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x / WAVE);
    unsigned bad = 0;
    uint64_t dmax = 0;
    for (int64_t v = blockIdx.x * (int64_t)(blockDim.x / WAVE) + threadIdx.x / WAVE; v < n; v += waves) {
        const int64_t r0 = rp[v], r1 = rp[v + 1];
        if (v == 0 && r0 != 0) bad |= BAD_ROWPTR;
        if (v == n - 1 && r1 != nnz) bad |= BAD_ROWPTR;
        if (r0 < 0 || r1 < r0 || r1 > nnz) {
            bad |= BAD_ROWPTR;
            continue;
        }
        if (labels && lane() == 0 && (labels[v] < 0 || labels[v] >= n_labels)) bad |= BAD_LABEL;
        dmax = max(dmax, (uint64_t)(r1 - r0));
        for (int64_t j = r0 + lane(); j < r1; j += WAVE) {
            const int32_t u = col[j];
            if (u < 0 || u >= n) {
                bad |= BAD_RANGE;
                continue;
            }
            if (bounds_only) continue;
            if (u == v) bad |= BAD_LOOP;
            if (j > r0 && col[j - 1] >= u) bad |= BAD_ORDER;
            const int64_t q0 = rp[u], q1 = rp[u + 1];
            if (q0 < 0 || q1 < q0 || q1 > nnz) continue;   // reported by u's own wave
            if (!contains(col + q0, (int32_t)min64(q1 - q0, INT32_MAX), (int32_t)v))
                bad |= BAD_SYMMETRY;
        }
    }
    if (bad) atomicOr(flags, bad);
    if (dmax) atomicMax(max_deg, (unsigned long long)dmax);
}

static int bits_for(uint64_t x) {
    int b = 0;
    while (b < 64 && (x >> b) != 0) ++b;
    return b;
}

static unsigned grid_for(int64_t items, int per_block) {
    int64_t b = (items + per_block - 1) / per_block;
    b = std::max<int64_t>(1, std::min<int64_t>(b, (int64_t)device_info().n_cu * 32));
    return (unsigned)b;
}

// ------------------------------------------------------- canonical CSR
//
// PG_CANONICALIZE: the rows are rebuilt as the sorted, duplicate-free,
// loop-free neighbour lists of the symmetric closure: every entry (v, u)
// with u != v gives the keys (v, u) and (u, v); the keys are sorted and
// repeated ones dropped.  Row bounds and vertex ids must be valid already.

constexpr uint64_t NO_EDGE = ~0ull;

__global__ void k_canon_keys(int64_t n, const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                             uint64_t* __restrict__ keys) {
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x / WAVE);
    for (int64_t v = blockIdx.x * (int64_t)(blockDim.x / WAVE) + threadIdx.x / WAVE; v < n; v += waves)
        for (int64_t j = rp[v] + lane(); j < rp[v + 1]; j += WAVE) {
            const uint64_t u = (uint32_t)col[j];
            const bool loop = u == (uint64_t)v;
            keys[2 * j] = loop ? NO_EDGE : ((uint64_t)v << 32) | u;
            keys[2 * j + 1] = loop ? NO_EDGE : (u << 32) | (uint64_t)v;
        }
}

__global__ void k_canon_keep(int64_t m, const uint64_t* __restrict__ keys, uint32_t* __restrict__ keep) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
        keep[i] = (keys[i] != NO_EDGE && (i == 0 || keys[i - 1] != keys[i])) ? 1u : 0u;
}

__global__ void k_canon_write(int64_t m, const uint64_t* __restrict__ keys, const uint32_t* __restrict__ keep,
                              const uint64_t* __restrict__ pos, int32_t* __restrict__ col,
                              uint32_t* __restrict__ deg) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
        if (keep[i]) {
            col[pos[i]] = (int32_t)(uint32_t)keys[i];
            atomicAdd(&deg[keys[i] >> 32], 1u);
        }
}

static void canonicalize(pg_graph* g) {
    hipStream_t s = g->stream;
    const int64_t n = g->n, nnz = g->nnz;
    DevBuf scratch;
    scratch.reserve(256);
    unsigned* dflags = scratch.as<unsigned>();
    unsigned long long* dmax = reinterpret_cast<unsigned long long*>(scratch.as<char>() + 64);
    fill_u32(dflags, 1, 0, s);
    fill_u64(reinterpret_cast<uint64_t*>(dmax), 1, 0, s);
    if (n > 0) {
        const int64_t blocks = std::min<int64_t>((n + 3) / 4, (int64_t)device_info().n_cu * 16);
        k_validate<<<(unsigned)blocks, 256, 0, s>>>(n, nnz, g->rp.as<int64_t>(), g->col.as<int32_t>(), nullptr, 0,
                                                    dflags, dmax, true);
        PG_HIP(hipGetLastError());
    }
    unsigned hf = 0;
    PG_HIP(hipMemcpyAsync(&hf, dflags, sizeof(hf), hipMemcpyDeviceToHost, s));
    PG_HIP(hipStreamSynchronize(s));
    if (n == 0 && nnz != 0) hf |= BAD_ROWPTR;
    PG_REQUIRE(hf == 0, PG_EINVAL,
               std::string("invalid CSR (canonicalising needs valid row bounds and vertex ids):") +
                   ((hf & BAD_ROWPTR) ? " row_ptr not monotone or not ending at nnz;" : "") +
                   ((hf & BAD_RANGE) ? " neighbour id out of range;" : ""));
    if (nnz == 0) return;
    const int64_t m = 2 * nnz;
    DevBuf keys, tmp, keep, pos, deg;
    keys.reserve(sizeof(uint64_t) * m);
    tmp.reserve(sizeof(uint64_t) * m);
    keep.reserve(sizeof(uint32_t) * m);
    pos.reserve(sizeof(uint64_t) * (m + 1));
    deg.reserve(sizeof(uint32_t) * std::max<int64_t>(n, 1));
    Arena ar;
    ar.buf.reserve(sizeof(uint64_t) * (size_t)(256 * ((m + 2047) / 2048) * 3 + (1 << 20)));
    k_canon_keys<<<grid_for(n, 4), 256, 0, s>>>(n, g->rp.as<int64_t>(), g->col.as<int32_t>(), keys.as<uint64_t>());
    PG_HIP(hipGetLastError());
    const int nb = std::max(1, bits_for((uint64_t)(n - 1)));
    radix_sort_u64(keys.as<uint64_t>(), tmp.as<uint64_t>(), m, 0, nb, ar, s);
    radix_sort_u64(keys.as<uint64_t>(), tmp.as<uint64_t>(), m, 32, 32 + nb, ar, s);
    k_canon_keep<<<grid_for(m, 256), 256, 0, s>>>(m, keys.as<uint64_t>(), keep.as<uint32_t>());
    PG_HIP(hipGetLastError());
    scan_u32(keep.as<uint32_t>(), m, pos.as<uint64_t>(), ar, s);
    const int64_t nnz2 = (int64_t)read_u64(pos.as<uint64_t>() + m, s);
    fill_u32(deg.as<uint32_t>(), n, 0, s);
    DevBuf col2;
    col2.reserve(sizeof(int32_t) * std::max<int64_t>(nnz2, 1));
    k_canon_write<<<grid_for(m, 256), 256, 0, s>>>(m, keys.as<uint64_t>(), keep.as<uint32_t>(), pos.as<uint64_t>(),
                                                   col2.as<int32_t>(), deg.as<uint32_t>());
    PG_HIP(hipGetLastError());
    scan_u32(deg.as<uint32_t>(), n, g->rp.as<uint64_t>(), ar, s);
    PG_HIP(hipStreamSynchronize(s));
    std::swap(g->col.p, col2.p);
    std::swap(g->col.bytes, col2.bytes);
    g->nnz = nnz2;
}

void graph_load(pg_graph* g, int64_t n, int64_t nnz, const int64_t* rp, const int32_t* col,
                const int32_t* labels, int32_t n_labels, unsigned flags) {
    PG_REQUIRE(n >= 0 && n < INT32_MAX, PG_EINVAL, "n out of range");
    PG_REQUIRE(nnz >= 0 && nnz < (int64_t(1) << 40), PG_EINVAL, "nnz out of range");
    PG_REQUIRE(rp != nullptr && (col != nullptr || nnz == 0), PG_EINVAL, "null CSR array");
    PG_REQUIRE((labels == nullptr) == (n_labels == 0), PG_EINVAL, "labels and n_labels disagree");
    PG_REQUIRE(n_labels >= 0 && n_labels <= 64, PG_EINVAL, "n_labels must be in [0, 64]");
    hipStream_t s = g->stream;
    g->n = n;
    g->nnz = nnz;
    g->n_labels = n_labels;
    const hipMemcpyKind kind = (flags & PG_DEVICE_PTRS) ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    g->rp.reserve(sizeof(int64_t) * (n + 1));
    g->col.reserve(sizeof(int32_t) * std::max<int64_t>(nnz, 1));
    PG_HIP(hipMemcpyAsync(g->rp.p, rp, sizeof(int64_t) * (n + 1), kind, s));
    if (nnz) PG_HIP(hipMemcpyAsync(g->col.p, col, sizeof(int32_t) * nnz, kind, s));
    if (labels) {
        g->labels.reserve(sizeof(int32_t) * std::max<int64_t>(n, 1));
        if (n) PG_HIP(hipMemcpyAsync(g->labels.p, labels, sizeof(int32_t) * n, kind, s));
    }
    if (flags & PG_CANONICALIZE) {
        canonicalize(g);
        nnz = g->nnz;
    }
    DevBuf scratch;
    scratch.reserve(256);
    unsigned* dflags = scratch.as<unsigned>();
    unsigned long long* dmax = reinterpret_cast<unsigned long long*>(scratch.as<char>() + 64);
    PG_HIP(hipMemsetAsync(scratch.p, 0, 256, s));
    if (n > 0) {
        const int64_t blocks = std::min<int64_t>((n + 3) / 4, (int64_t)device_info().n_cu * 16);
        ProfScope ps("validate", s, (double)nnz);
        k_validate<<<(unsigned)blocks, 256, 0, s>>>(n, nnz, g->rp.as<int64_t>(), g->col.as<int32_t>(),
                                                    labels ? g->labels.as<int32_t>() : nullptr, n_labels,
                                                    dflags, dmax, false);
        PG_HIP(hipGetLastError());
    }
    unsigned hf = 0;
    unsigned long long hm = 0;
    PG_HIP(hipMemcpyAsync(&hf, dflags, sizeof(hf), hipMemcpyDeviceToHost, s));
    PG_HIP(hipMemcpyAsync(&hm, dmax, sizeof(hm), hipMemcpyDeviceToHost, s));
    PG_HIP(hipStreamSynchronize(s));
    prof_flush();
    if (n == 0 && nnz != 0) hf |= BAD_ROWPTR;
    if (hf) {
        std::string why;
        if (hf & BAD_ROWPTR) why += " row_ptr not monotone or not ending at nnz;";
        if (hf & BAD_RANGE) why += " neighbour id out of range;";
        if (hf & BAD_LOOP) why += " self-loop;";
        if (hf & BAD_ORDER) why += " neighbour list not strictly ascending (or duplicate);";
        if (hf & BAD_SYMMETRY) why += " not symmetric;";
        if (hf & BAD_LABEL) why += " label out of range;";
        throw Error{PG_EINVAL, "invalid CSR:" + why};
    }
    g->max_deg = (int64_t)hm;
}

// ------------------------------------------------------------------- DAG
//
// Orientation of section 4.1: an edge points to the endpoint of higher
// degree, ties to the larger vertex id.  Vertices are renamed by their rank
// in that (degree, id) order, so every DAG edge goes from a smaller to a
// larger rank and each out-list is ascending in rank.

__global__ void k_degree_keys(int64_t n, const int64_t* __restrict__ rp, uint64_t* __restrict__ keys) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
        keys[v] = ((uint64_t)(rp[v + 1] - rp[v]) << 32) | (uint64_t)v;
}

__global__ void k_rank_of(int64_t n, const uint64_t* __restrict__ sorted, int32_t* __restrict__ rank_of) {
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x)
        rank_of[(uint32_t)sorted[r]] = (int32_t)r;
}

// out-degree of every vertex, stored at its rank
__global__ __launch_bounds__(256) void k_dag_outdeg(int64_t n, const int64_t* __restrict__ rp,
                                                    const int32_t* __restrict__ col,
                                                    const int32_t* __restrict__ rank_of,
                                                    uint32_t* __restrict__ dout_at_rank,
                                                    unsigned* __restrict__ max_out) {
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x / WAVE);
    uint32_t mx = 0;
    for (int64_t v = blockIdx.x * (int64_t)(blockDim.x / WAVE) + threadIdx.x / WAVE; v < n; v += waves) {
        const int32_t rv = rank_of[v];
        uint32_t c = 0;
        for (int64_t j = rp[v] + lane(); j < rp[v + 1]; j += WAVE) c += rank_of[col[j]] > rv;
        c = wave_sum_u32(c);
        if (lane() == 0) dout_at_rank[rv] = c;
        mx = max(mx, c);
    }
    if (lane() == 0 && mx) atomicMax(max_out, mx);
}

// (rank(v) << 32 | rank(u)) for every DAG edge, placed in v's rank row
__global__ __launch_bounds__(256) void k_dag_emit(int64_t n, const int64_t* __restrict__ rp,
                                                  const int32_t* __restrict__ col,
                                                  const int32_t* __restrict__ rank_of,
                                                  const uint64_t* __restrict__ dag_rp,
                                                  uint64_t* __restrict__ keys) {
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x / WAVE);
    for (int64_t v = blockIdx.x * (int64_t)(blockDim.x / WAVE) + threadIdx.x / WAVE; v < n; v += waves) {
        const int32_t rv = rank_of[v];
        uint64_t pos = dag_rp[rv];
        for (int64_t j0 = rp[v]; j0 < rp[v + 1]; j0 += WAVE) {
            const int64_t j = j0 + lane();
            int32_t ru = -1;
            if (j < rp[v + 1]) ru = rank_of[col[j]];
            const bool keep = ru > rv;
            const uint64_t m = ballot(keep);
            if (keep) keys[pos + popc64(m & lanemask_lt())] = ((uint64_t)(uint32_t)rv << 32) | (uint32_t)ru;
            pos += popc64(m);
        }
    }
}

__global__ void k_split_low(int64_t m, const uint64_t* __restrict__ keys, int32_t* __restrict__ low,
                            int32_t* __restrict__ high) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
        low[i] = (int32_t)(uint32_t)keys[i];
        high[i] = (int32_t)(uint32_t)(keys[i] >> 32);
    }
}

void build_dag(pg_graph* g) {
    if (g->dag.built) return;
    hipStream_t s = g->stream;
    const int64_t n = g->n;
    Dag& D = g->dag;
    const int64_t m = g->nnz / 2;
    D.rank_of.reserve(sizeof(int32_t) * std::max<int64_t>(n, 1));
    D.rp.reserve(sizeof(int64_t) * (n + 1));
    D.col.reserve(sizeof(int32_t) * std::max<int64_t>(m, 1));
    D.src.reserve(sizeof(int32_t) * std::max<int64_t>(m, 1));
    DevBuf t1, t2, t3;
    t1.reserve(sizeof(uint64_t) * std::max<int64_t>(std::max(n, m), 1));
    t2.reserve(sizeof(uint64_t) * std::max<int64_t>(std::max(n, m), 1));
    t3.reserve(sizeof(uint32_t) * std::max<int64_t>(n, 1) + 512);
    Arena tmp;
    tmp.buf.reserve(sizeof(uint64_t) * (size_t)(256 * ((std::max(n, m) + 2047) / 2048) * 3 + (1 << 20)));
    ProfScope ps("dag_build", s, (double)g->nnz);
    if (n > 0) {
        // 1. degree order: stable sort of (deg << 32 | v) on the degree bits
        uint64_t* keys = t1.as<uint64_t>();
        k_degree_keys<<<grid_for(n, 256), 256, 0, s>>>(n, g->rp.as<int64_t>(), keys);
        PG_HIP(hipGetLastError());
        const int db = std::max(1, bits_for((uint64_t)g->max_deg));
        radix_sort_u64(keys, t2.as<uint64_t>(), n, 32, 32 + db, tmp, s);
        k_rank_of<<<grid_for(n, 256), 256, 0, s>>>(n, keys, D.rank_of.as<int32_t>());
        PG_HIP(hipGetLastError());
        // 2. out-degrees at rank positions, then the DAG row pointers
        uint32_t* dout = t3.as<uint32_t>();
        unsigned* dmo = reinterpret_cast<unsigned*>(t3.as<char>() + ((sizeof(uint32_t) * n + 255) & ~size_t(255)));
        fill_u32(dmo, 1, 0, s);
        k_dag_outdeg<<<grid_for(n, 4), 256, 0, s>>>(n, g->rp.as<int64_t>(), g->col.as<int32_t>(),
                                                    D.rank_of.as<int32_t>(), dout, dmo);
        PG_HIP(hipGetLastError());
        unsigned hmo = 0;
        PG_HIP(hipMemcpyAsync(&hmo, dmo, sizeof(hmo), hipMemcpyDeviceToHost, s));
        PG_HIP(hipStreamSynchronize(s));
        D.max_out = hmo;
        scan_u32(dout, n, D.rp.as<uint64_t>(), tmp, s);
        // 3. edges as (rank(src), rank(dst)) keys, sorted on both halves
        if (m > 0) {
            uint64_t* ek = t1.as<uint64_t>();
            k_dag_emit<<<grid_for(n, 4), 256, 0, s>>>(n, g->rp.as<int64_t>(), g->col.as<int32_t>(),
                                                      D.rank_of.as<int32_t>(), D.rp.as<uint64_t>(), ek);
            PG_HIP(hipGetLastError());
            const int nb = std::max(1, bits_for((uint64_t)(n - 1)));
            radix_sort_u64(ek, t2.as<uint64_t>(), m, 0, nb, tmp, s);
            radix_sort_u64(ek, t2.as<uint64_t>(), m, 32, 32 + nb, tmp, s);
            k_split_low<<<grid_for(m, 256), 256, 0, s>>>(m, ek, D.col.as<int32_t>(), D.src.as<int32_t>());
            PG_HIP(hipGetLastError());
        }
    } else {
        fill_u64(D.rp.as<uint64_t>(), 1, 0, s);
    }
    PG_HIP(hipStreamSynchronize(s));
    D.n_edges = m;
    D.built = true;
}

// ----------------------------------------------------- motif single edges
//
// The initial embedding list of vertex-induced mining (Algorithm 1, Init):
// every edge once, as (v0, v1) with v0 < v1.  Stored as the upper half of
// each adjacency row: segment of v0 = its neighbours larger than v0.

__global__ __launch_bounds__(256) void k_upper_count(int64_t n, const int64_t* __restrict__ rp,
                                                     const int32_t* __restrict__ col,
                                                     uint32_t* __restrict__ cnt) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r0 = rp[v], r1 = rp[v + 1];
        cnt[v] = (uint32_t)(r1 - upper_bound(col, r0, r1, (int32_t)v));
    }
}

__global__ __launch_bounds__(256) void k_upper_write(int64_t n, const int64_t* __restrict__ rp,
                                                     const int32_t* __restrict__ col,
                                                     const uint64_t* __restrict__ seg,
                                                     int32_t* __restrict__ src, int32_t* __restrict__ dst) {
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x / WAVE);
    for (int64_t v = blockIdx.x * (int64_t)(blockDim.x / WAVE) + threadIdx.x / WAVE; v < n; v += waves) {
        const int64_t r1 = rp[v + 1];
        const int64_t r0 = r1 - (int64_t)(seg[v + 1] - seg[v]);
        for (int64_t j = r0 + lane(); j < r1; j += WAVE) {
            const uint64_t o = seg[v] + (uint64_t)(j - r0);
            src[o] = (int32_t)v;
            dst[o] = col[j];
        }
    }
}

// for every L1 entry (u, v): the first place in v's row past u
__global__ __launch_bounds__(256) void k_upper_rev(int64_t m, const int64_t* __restrict__ rp,
                                                   const int32_t* __restrict__ col, const int32_t* __restrict__ src,
                                                   const int32_t* __restrict__ dst, int32_t* __restrict__ rev) {
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < m; p += (int64_t)gridDim.x * blockDim.x) {
        const int32_t v = dst[p];
        const int64_t q0 = rp[v];
        rev[p] = (int32_t)(upper_bound(col, q0, rp[v + 1], src[p]) - q0);
    }
}

void build_motif_l1(pg_graph* g, const MotifView& V) {
    MotifL1& L = *V.ml1;
    if (L.built) return;
    hipStream_t s = g->stream;
    const int64_t n = V.n, m = V.nnz / 2;
    L.seg.reserve(sizeof(int64_t) * (n + 1));
    L.src.reserve(sizeof(int32_t) * std::max<int64_t>(m, 1));
    L.dst.reserve(sizeof(int32_t) * std::max<int64_t>(m, 1));
    L.rev.reserve(sizeof(int32_t) * std::max<int64_t>(m, 1));
    DevBuf cnt;
    cnt.reserve(sizeof(uint32_t) * std::max<int64_t>(n, 1));
    Arena tmp;
    tmp.buf.reserve(sizeof(uint64_t) * (size_t)(2 * ((n + 2047) / 2048) + 64) + (1 << 16));
    if (n > 0) {
        k_upper_count<<<grid_for(n, 256), 256, 0, s>>>(n, V.rp, V.col, cnt.as<uint32_t>());
        PG_HIP(hipGetLastError());
        scan_u32(cnt.as<uint32_t>(), n, L.seg.as<uint64_t>(), tmp, s);
        k_upper_write<<<grid_for(n, 4), 256, 0, s>>>(n, V.rp, V.col, L.seg.as<uint64_t>(), L.src.as<int32_t>(),
                                                     L.dst.as<int32_t>());
        PG_HIP(hipGetLastError());
        if (m > 0) {
            k_upper_rev<<<grid_for(m, 256), 256, 0, s>>>(m, V.rp, V.col, L.src.as<int32_t>(), L.dst.as<int32_t>(),
                                                        L.rev.as<int32_t>());
            PG_HIP(hipGetLastError());
        }
    } else {
        fill_u64(L.seg.as<uint64_t>(), 1, 0, s);
    }
    PG_HIP(hipStreamSynchronize(s));
    L.n_edges = m;
    L.built = true;
}

void build_motif_l1(pg_graph* g) { build_motif_l1(g, motif_view(g, false)); }

// ------------------------------------------------- renamed graph (motifs)
//
// New name of v = its position in the order of decreasing degree, ties by
// increasing id.  Rows are the renamed neighbour lists, ascending.

__global__ void k_desc_degree_keys(int64_t n, const int64_t* __restrict__ rp, uint64_t max_deg,
                                   uint64_t* __restrict__ keys) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
        keys[v] = ((max_deg - (uint64_t)(rp[v + 1] - rp[v])) << 32) | (uint64_t)v;
}

// degree of the vertex named r (for the row pointers)
__global__ void k_renamed_degree(int64_t n, const uint64_t* __restrict__ sorted, const int64_t* __restrict__ rp,
                                 uint32_t* __restrict__ deg) {
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t v = (uint32_t)sorted[r];
        deg[r] = (uint32_t)(rp[v + 1] - rp[v]);
    }
}

// (name(v) << 32 | name(u)) for every directed entry (v, u), in input order
__global__ __launch_bounds__(256) void k_renamed_edges(int64_t n, const int64_t* __restrict__ rp,
                                                       const int32_t* __restrict__ col,
                                                       const int32_t* __restrict__ name,
                                                       uint64_t* __restrict__ keys) {
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x / WAVE);
    for (int64_t v = blockIdx.x * (int64_t)(blockDim.x / WAVE) + threadIdx.x / WAVE; v < n; v += waves) {
        const uint64_t hv = (uint64_t)(uint32_t)name[v] << 32;
        for (int64_t j = rp[v] + lane(); j < rp[v + 1]; j += WAVE) keys[j] = hv | (uint32_t)name[col[j]];
    }
}

void build_motif_graph(pg_graph* g) {
    MotifGraph& M = g->mg;
    if (M.built) return;
    hipStream_t s = g->stream;
    const int64_t n = g->n, nnz = g->nnz;
    M.n = n;
    M.nnz = nnz;
    M.max_deg = g->max_deg;
    M.rp.reserve(sizeof(int64_t) * (n + 1));
    // 64 zeroed entries past the end, so a wave may read a whole 64-entry
    // chunk from any list start
    M.col.reserve(sizeof(int32_t) * (nnz + WAVE));
    PG_HIP(hipMemsetAsync(M.col.as<int32_t>() + nnz, 0, sizeof(int32_t) * WAVE, s));
    DevBuf t1, t2, name, deg, hi;
    const int64_t big = std::max<int64_t>(std::max(n, nnz), 1);
    t1.reserve(sizeof(uint64_t) * big);
    t2.reserve(sizeof(uint64_t) * big);
    name.reserve(sizeof(int32_t) * std::max<int64_t>(n, 1));
    deg.reserve(sizeof(uint32_t) * std::max<int64_t>(n, 1));
    hi.reserve(sizeof(int32_t) * std::max<int64_t>(nnz, 1));
    Arena tmp;
    tmp.buf.reserve(sizeof(uint64_t) * (size_t)(256 * ((big + 2047) / 2048) * 3 + (1 << 20)));
    ProfScope ps("motif_rename", s, (double)nnz);
    if (n > 0) {
        uint64_t* keys = t1.as<uint64_t>();
        k_desc_degree_keys<<<grid_for(n, 256), 256, 0, s>>>(n, g->rp.as<int64_t>(), (uint64_t)g->max_deg, keys);
        PG_HIP(hipGetLastError());
        const int db = std::max(1, bits_for((uint64_t)g->max_deg));
        radix_sort_u64(keys, t2.as<uint64_t>(), n, 32, 32 + db, tmp, s);
        k_rank_of<<<grid_for(n, 256), 256, 0, s>>>(n, keys, name.as<int32_t>());
        PG_HIP(hipGetLastError());
        k_renamed_degree<<<grid_for(n, 256), 256, 0, s>>>(n, keys, g->rp.as<int64_t>(), deg.as<uint32_t>());
        PG_HIP(hipGetLastError());
        scan_u32(deg.as<uint32_t>(), n, M.rp.as<uint64_t>(), tmp, s);
        if (nnz > 0) {
            uint64_t* ek = t1.as<uint64_t>();
            k_renamed_edges<<<grid_for(n, 4), 256, 0, s>>>(n, g->rp.as<int64_t>(), g->col.as<int32_t>(),
                                                           name.as<int32_t>(), ek);
            PG_HIP(hipGetLastError());
            const int nb = std::max(1, bits_for((uint64_t)(n - 1)));
            radix_sort_u64(ek, t2.as<uint64_t>(), nnz, 0, nb, tmp, s);
            radix_sort_u64(ek, t2.as<uint64_t>(), nnz, 32, 32 + nb, tmp, s);
            k_split_low<<<grid_for(nnz, 256), 256, 0, s>>>(nnz, ek, M.col.as<int32_t>(), hi.as<int32_t>());
            PG_HIP(hipGetLastError());
        }
    } else {
        fill_u64(M.rp.as<uint64_t>(), 1, 0, s);
    }
    PG_HIP(hipStreamSynchronize(s));
    M.built = true;
}

MotifView motif_view(pg_graph* g, bool renamed) {
    if (renamed) {
        build_motif_graph(g);
        MotifGraph& M = g->mg;
        return MotifView{M.n, M.nnz, M.max_deg, M.rp.as<int64_t>(), M.col.as<int32_t>(), &M.ml1};
    }
    return MotifView{g->n, g->nnz, g->max_deg, g->rp.as<int64_t>(), g->col.as<int32_t>(), &g->ml1};
}

}  // namespace pg
