// Batched motif counting over many small graphs in one persistent launch
// (the graphs stay resident; a serving loop drives the asynchronous form).
//
// Every graph has at most PG_BATCH_MAX_VERTICES vertices, so a workgroup
// keeps the graph's adjacency as bitset rows in LDS.  The mining steps are
// those of the single-graph motif path (canonical breadth-first order from
// the smallest vertex, connectivity bitmap -> 64-entry pattern table,
// Pangolin sections 3.3 and 4.2), with set intersections done as masked
// popcounts over the rows:
//   level 1  edges (v0 < v1), one per lane;
//   level 2  the canonical third vertices v2 of an edge form a bitset:
//            (A0 above v1) | (A1 minus A0 above v0); they are iterated, never
//            stored;
//   level 3  fused with classification and reduction: for every (v0,v1,v2)
//            the candidates adjacent to exactly the vertex subset m of
//            {v0,v1,v2}, in the range above v0 or above v2, are popcounts of
//            row combinations; the canonical rule keeps the right ranges and
//            the pattern table turns (edges of v0v1v2, m) into the motif.
// Work items are (graph, range of edges) ordered by estimated work, largest
// first, and taken from an atomic queue by persistent workgroups; each item
// adds its per-pattern counts into the graph's row of the output.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <numeric>
#include <vector>

#include "pg_device.h"
#include "pg_internal.h"

namespace pg {

constexpr int BT_MAXN = PG_BATCH_MAX_VERTICES;
constexpr int BT_WORDS = BT_MAXN / 64;   // 64-bit words per adjacency row

// 4-vertex pattern of the connectivity bitmap (pairs 01 02 12 03 13 23):
// 0 path, 1 star, 2 cycle, 3 paw, 4 diamond, 5 4-clique, -1 disconnected
__host__ __device__ constexpr int8_t motif4_of(int m) {
    const int pa[6] = {0, 0, 1, 0, 1, 2};
    const int pb[6] = {1, 2, 2, 3, 3, 3};
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
    if (dmin == 0) return -1;
    if (e == 3) return dmax == 3 ? 1 : 0;
    if (e == 4) return dmax == 3 ? 3 : 2;
    return e == 5 ? 4 : 5;
}

struct BatchLut {
    int8_t v[64];
};

__host__ __device__ constexpr BatchLut make_batch_lut() {
    BatchLut t{};
    for (int m = 0; m < 64; ++m) t.v[m] = motif4_of(m);
    return t;
}

__constant__ BatchLut c_blut = make_batch_lut();

struct BatchItem {
    int32_t graph;     // index into the caller's id list
    int32_t e_lo, e_hi;  // edge range [e_lo, e_hi) in the graph's (v0 < v1) order
};

struct BatchArgs {
    const int64_t* voff;       // device: vertex offsets of the graphs
    const int64_t* rp;         // global row pointers (positions in col)
    const int32_t* col;        // local ids
    const int64_t* ids;        // graph of each output row
    const BatchItem* items;
    int64_t n_items;
    const int64_t* n_items_dev;   // when set, the item count is read from device memory
    unsigned long long* next;  // queue counter (zeroed before the launch)
    unsigned long long* out;   // rows of 6 (k = 4) or 2 (k = 3)
    int k;
};

__device__ __forceinline__ uint64_t above_mask(int w, int32_t v) {
    // bits of word w for vertices strictly greater than v
    const int32_t lo = w * 64;
    if (v < lo) return ~0ull;
    if (v >= lo + 63) return 0ull;
    return ~0ull << (v - lo + 1);
}

// One graph item per workgroup: rows as bitsets, then one lane per edge.
template <int NT>
__global__ __launch_bounds__(NT) void k_batch_motifs(BatchArgs A) {
    __shared__ uint64_t rows[BT_MAXN][BT_WORDS];
    __shared__ int32_t up_start[BT_MAXN + 1];   // first edge (v < u) of each vertex
    __shared__ int32_t s_item;
    __shared__ int32_t wave_tot[NT / WAVE];
    const int64_t n_items = A.n_items_dev ? *A.n_items_dev : A.n_items;
    while (true) {
        if (threadIdx.x == 0) s_item = (int32_t)min<unsigned long long>(atomicAdd(A.next, 1ull), (unsigned long long)INT32_MAX);
        __syncthreads();
        const int64_t it = s_item;
        __syncthreads();
        if (it >= n_items) break;
        const BatchItem I = A.items[it];
        const int64_t g = A.ids[I.graph];
        const int64_t v0g = A.voff[g];
        const int32_t n = (int32_t)(A.voff[g + 1] - v0g);
        const int W = (n + 63) / 64;
        const int64_t* rp = A.rp + v0g;
        // adjacency rows as bitsets
        for (int i = threadIdx.x; i < n * W; i += NT) rows[i / W][i % W] = 0;
        __syncthreads();
        for (int32_t v = threadIdx.x; v < n; v += NT)
            for (int64_t j = rp[v]; j < rp[v + 1]; ++j) {
                const int32_t u = A.col[j];
                rows[v][u >> 6] |= 1ull << (u & 63);
            }
        __syncthreads();
        // up_start: exclusive prefix over vertices of their larger neighbours
        {
            const int w = threadIdx.x / WAVE;
            int32_t carry = 0;
            for (int32_t c0 = 0; c0 < n; c0 += NT) {
                const int32_t v = c0 + threadIdx.x;
                uint32_t up = 0;
                if (v < n)
                    for (int x = 0; x < W; ++x) up += __popcll(rows[v][x] & above_mask(x, v));
                const uint32_t inc = wave_incl_scan(up);
                if (lane() == WAVE - 1) wave_tot[w] = (int32_t)inc;
                __syncthreads();
                int32_t before = carry;
                for (int j = 0; j < w; ++j) before += wave_tot[j];
                if (v < n) up_start[v] = before + (int32_t)(inc - up);
                int32_t total = 0;
                for (int j = 0; j < NT / WAVE; ++j) total += wave_tot[j];
                carry += total;
                __syncthreads();
            }
            if (threadIdx.x == 0) up_start[n] = carry;
            __syncthreads();
        }
        uint64_t acc[6] = {0, 0, 0, 0, 0, 0};
        for (int32_t e = I.e_lo + (int32_t)threadIdx.x; e < I.e_hi; e += NT) {
            // edge e = (a, b), a < b: a holds e in its upper range
            int32_t a = 0;
            {
                int32_t cnt = n;
                while (cnt > 1) {
                    const int32_t half = cnt >> 1;
                    if (up_start[a + half] <= e) a += half;
                    cnt -= half;
                }
            }
            const int64_t deg_a = rp[a + 1] - rp[a];
            const int32_t up_a = up_start[a + 1] - up_start[a];
            const int32_t b = A.col[rp[a] + (deg_a - up_a) + (e - up_start[a])];
            if (A.k == 3) {
                // u adjacent to a above b: triangle if also ~b, else wedge;
                // u adjacent to b only, above a: wedge
                for (int w = 0; w < W; ++w) {
                    const uint64_t ra = rows[a][w], rb = rows[b][w];
                    const uint64_t hb = above_mask(w, b), ha = above_mask(w, a);
                    acc[1] += __popcll(ra & rb & hb);
                    acc[0] += __popcll(ra & ~rb & hb) + __popcll(rb & ~ra & ha);
                }
                continue;
            }
            // canonical third vertices of (a, b)
            for (int w = 0; w < W; ++w) {
                const uint64_t ra = rows[a][w], rb = rows[b][w];
                uint64_t kids = (ra & above_mask(w, b)) | (rb & ~ra & above_mask(w, a));
                while (kids) {
                    const int bit = __ffsll((unsigned long long)kids) - 1;
                    kids &= kids - 1;
                    const int32_t c = w * 64 + bit;
                    const int a02 = (int)((ra >> bit) & 1), a12 = (int)((rb >> bit) & 1);
                    const int p = a02 ? 0 : 1;
                    const int ebits = 1 | (a02 << 1) | (a12 << 2);
                    // candidates u > a, u not in {a, b, c}, by exact mask and range
                    uint64_t N[2][8];
#pragma unroll
                    for (int r = 0; r < 2; ++r)
#pragma unroll
                        for (int m = 0; m < 8; ++m) N[r][m] = 0;
                    for (int x = 0; x < W; ++x) {
                        const uint64_t A0 = rows[a][x], A1 = rows[b][x], A2 = rows[c][x];
                        uint64_t own = 0;
                        if ((b >> 6) == x) own |= 1ull << (b & 63);
                        if ((c >> 6) == x) own |= 1ull << (c & 63);
                        const uint64_t hi = above_mask(x, c) & ~own;                   // above c
                        const uint64_t lo = above_mask(x, a) & ~above_mask(x, c) & ~own;   // (a, c]
#pragma unroll
                        for (int m = 1; m < 8; ++m) {
                            const uint64_t sel = ((m & 1) ? A0 : ~A0) & ((m & 2) ? A1 : ~A1) & ((m & 4) ? A2 : ~A2);
                            N[0][m] += __popcll(sel & lo);
                            N[1][m] += __popcll(sel & hi);
                        }
                    }
#pragma unroll
                    for (int m = 1; m < 8; ++m) {
                        const int sbit = (m & 1) ? 0 : ((m & 2) ? 1 : 2);
                        if (sbit < p) continue;
                        const uint64_t cnt = (sbit == p) ? N[1][m] : N[0][m] + N[1][m];
                        const int pid = c_blut.v[ebits | (m << 3)];
                        if (pid >= 0) acc[pid] += cnt;
                    }
                }
            }
        }
        // one add per pattern per wave
        const int width = A.k == 3 ? 2 : 6;
        for (int c = 0; c < width; ++c) {
            const uint64_t v = wave_sum_u64(acc[c]);
            if (lane() == 0 && v) atomicAdd(&A.out[(int64_t)I.graph * width + c], (unsigned long long)v);
        }
        __syncthreads();
    }
}

// Validation of every graph of a batch: one wave per vertex (global index);
// entries in [0, n_g), no loop, strictly ascending, reverse entry present.
__global__ __launch_bounds__(256) void k_batch_validate(int64_t n_graphs, const int64_t* __restrict__ voff,
                                                        const int64_t* __restrict__ rp,
                                                        const int32_t* __restrict__ col, int64_t nnz,
                                                        unsigned* __restrict__ bad_out) {
    const int64_t nv = voff[n_graphs];
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x / WAVE);
    unsigned bad = 0;
    for (int64_t v = blockIdx.x * (int64_t)(blockDim.x / WAVE) + threadIdx.x / WAVE; v < nv; v += waves) {
        int64_t lo = 0, hi = n_graphs - 1;   // graph of v: last g with voff[g] <= v
        while (lo < hi) {
            const int64_t mid = (lo + hi + 1) >> 1;
            if (voff[mid] <= v) lo = mid; else hi = mid - 1;
        }
        const int64_t g0 = voff[lo];
        const int32_t ng = (int32_t)(voff[lo + 1] - g0);
        const int32_t lv = (int32_t)(v - g0);
        const int64_t r0 = rp[v], r1 = rp[v + 1];
        if (r0 < 0 || r1 < r0 || r1 > nnz) { bad |= 1; continue; }
        for (int64_t j = r0 + lane(); j < r1; j += WAVE) {
            const int32_t u = col[j];
            if (u < 0 || u >= ng) { bad |= 2; continue; }
            if (u == lv) bad |= 4;
            if (j > r0 && col[j - 1] >= u) bad |= 8;
            const int64_t q0 = rp[g0 + u], q1 = rp[g0 + u + 1];
            if (q0 < 0 || q1 < q0 || q1 > nnz) continue;
            if (!contains(col + q0, (int32_t)(q1 - q0), lv)) bad |= 16;
        }
    }
    if (bad) atomicOr(bad_out, bad);
}

}  // namespace pg

using namespace pg;

struct pg_batch {
    int device = 0;
    hipStream_t stream = nullptr;
    int64_t n_graphs = 0, n_vertices = 0, nnz = 0;
    std::vector<int64_t> voff;     // host copy
    std::vector<int32_t> n_edges;  // per graph
    std::vector<double> work;      // per graph estimate
    DevBuf d_voff, d_rp, d_col, d_all_ids;
    int block_threads = 256;
    double split_work = 4.0e6;
    int grid_blocks = 0;
    int params_gen = 0;        // bumped by pg_batch_set_params; slots re-capture when it moves
    Arena arena;
};

namespace pg {

// Work estimate of a graph: connected 3-vertex subsets (the level-2
// entries) times the row words touched for each.
static double graph_work(int64_t n, int64_t m, const int64_t* rp_local_deg) {
    (void)rp_local_deg;
    if (n <= 0) return 0;
    const double d = 2.0 * (double)m / (double)n;
    const double words = std::ceil((double)n / 64.0);
    return ((double)n * d * d / 2.0 + (double)m) * words + 1.0;
}

static void build_items(pg_batch* b, const int64_t* ids, int64_t n_ids, std::vector<BatchItem>& items,
                        int max_parts = 1 << 20) {
    std::vector<std::pair<double, BatchItem>> tmp;
    tmp.reserve((size_t)n_ids);
    for (int64_t r = 0; r < n_ids; ++r) {
        const int64_t g = ids[r];
        const double w = b->work[(size_t)g];
        const int32_t E = b->n_edges[(size_t)g];
        int parts = (int)std::min<double>(std::max(1.0, std::ceil(w / b->split_work)), std::max(1, E));
        parts = std::min(parts, max_parts);
        for (int p = 0; p < parts; ++p) {
            BatchItem I;
            I.graph = (int32_t)r;
            I.e_lo = (int32_t)((int64_t)E * p / parts);
            I.e_hi = (int32_t)((int64_t)E * (p + 1) / parts);
            tmp.push_back({w / parts, I});
        }
    }
    std::stable_sort(tmp.begin(), tmp.end(), [](const auto& x, const auto& y) { return x.first > y.first; });
    items.resize(tmp.size());
    for (size_t i = 0; i < tmp.size(); ++i) items[i] = tmp[i].second;
}

// Persistent grid of the batch kernel: the tuned size, else one or two
// workgroups per CU; never more workgroups than items.
static int batch_grid(const pg_batch* b, int64_t n_items) {
    const int per_cu = b->block_threads >= 512 ? 1 : 2;
    const int blocks = b->grid_blocks > 0 ? b->grid_blocks : device_info().n_cu * per_cu;
    return (int)std::max<int64_t>(1, std::min<int64_t>(blocks, n_items));
}

static void launch_batch(pg_batch* b, int k, const int64_t* d_ids, const BatchItem* d_items, int64_t n_items,
                         uint64_t* d_out, unsigned long long* d_next, hipStream_t s) {
    BatchArgs A;
    A.voff = b->d_voff.as<int64_t>();
    A.rp = b->d_rp.as<int64_t>();
    A.col = b->d_col.as<int32_t>();
    A.ids = d_ids;
    A.items = d_items;
    A.n_items = n_items;
    A.n_items_dev = nullptr;
    A.next = d_next;
    A.out = reinterpret_cast<unsigned long long*>(d_out);
    A.k = k;
    fill_u64(reinterpret_cast<uint64_t*>(d_next), 1, 0, s);
    const int blocks = batch_grid(b, n_items);
    ProfScope ps("batch_motifs", s, (double)n_items);
    switch (b->block_threads) {
        case 64: k_batch_motifs<64><<<blocks, 64, 0, s>>>(A); break;
        case 128: k_batch_motifs<128><<<blocks, 128, 0, s>>>(A); break;
        case 512: k_batch_motifs<512><<<blocks, 512, 0, s>>>(A); break;
        default: k_batch_motifs<256><<<blocks, 256, 0, s>>>(A); break;
    }
    PG_HIP(hipGetLastError());
}

}  // namespace pg

namespace pg {
void note_object(int delta);
}

extern "C" {

int pg_batch_load(int64_t n_graphs, const int64_t* voff, const int64_t* row_ptr, const int32_t* col,
                  unsigned flags, void* stream, pg_batch** out) {
    return guarded([&] {
        PG_REQUIRE(out != nullptr && voff != nullptr && row_ptr != nullptr, PG_EINVAL, "NULL argument");
        PG_REQUIRE(n_graphs >= 0 && n_graphs < INT32_MAX, PG_EINVAL, "n_graphs out of range");
        PG_REQUIRE((flags & ~PG_DEVICE_PTRS) == 0, PG_EINVAL, "unknown flag");
        int ndev = 0;
        if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) {
            (void)hipGetLastError();
            throw Error{PG_EDEVICE, "no HIP device available"};
        }
        pg_batch* b = new pg_batch();
        try {
            b->stream = static_cast<hipStream_t>(stream);
            PG_HIP(hipGetDevice(&b->device));
            b->n_graphs = n_graphs;
            b->voff.assign(voff, voff + n_graphs + 1);
            PG_REQUIRE(b->voff[0] == 0, PG_EINVAL, "voff[0] must be 0");
            for (int64_t g = 0; g < n_graphs; ++g) {
                const int64_t n = b->voff[g + 1] - b->voff[g];
                PG_REQUIRE(n >= 0 && n <= PG_BATCH_MAX_VERTICES, PG_EINVAL,
                           "graph " + std::to_string(g) + " has more than PG_BATCH_MAX_VERTICES vertices");
            }
            const int64_t nv = b->voff[n_graphs];
            b->n_vertices = nv;
            // row pointers on the host (needed for per-graph edge counts)
            std::vector<int64_t> hrp((size_t)nv + 1);
            const hipMemcpyKind kind = (flags & PG_DEVICE_PTRS) ? hipMemcpyDeviceToHost : hipMemcpyHostToHost;
            PG_HIP(hipMemcpy(hrp.data(), row_ptr, sizeof(int64_t) * (nv + 1), kind));
            const int64_t nnz = hrp[(size_t)nv] - hrp[0];
            PG_REQUIRE(hrp[0] == 0 && nnz >= 0, PG_EINVAL, "row_ptr must start at 0");
            b->nnz = nnz;
            b->n_edges.resize((size_t)n_graphs);
            b->work.resize((size_t)n_graphs);
            for (int64_t g = 0; g < n_graphs; ++g) {
                const int64_t v0 = b->voff[g], v1 = b->voff[g + 1];
                const int64_t m2 = hrp[(size_t)v1] - hrp[(size_t)v0];
                PG_REQUIRE(m2 >= 0 && m2 % 2 == 0, PG_EINVAL, "graph rows not symmetric");
                b->n_edges[(size_t)g] = (int32_t)(m2 / 2);
                b->work[(size_t)g] = graph_work(v1 - v0, m2 / 2, nullptr);
            }
            b->d_voff.reserve(sizeof(int64_t) * (n_graphs + 1));
            b->d_rp.reserve(sizeof(int64_t) * (nv + 1));
            b->d_col.reserve(sizeof(int32_t) * std::max<int64_t>(nnz, 1));
            hipStream_t s = b->stream;
            PG_HIP(hipMemcpyAsync(b->d_voff.p, b->voff.data(), sizeof(int64_t) * (n_graphs + 1),
                                  hipMemcpyHostToDevice, s));
            PG_HIP(hipMemcpyAsync(b->d_rp.p, hrp.data(), sizeof(int64_t) * (nv + 1), hipMemcpyHostToDevice, s));
            const hipMemcpyKind ckind = (flags & PG_DEVICE_PTRS) ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
            if (nnz) PG_HIP(hipMemcpyAsync(b->d_col.p, col, sizeof(int32_t) * nnz, ckind, s));
            // identity id list for whole-batch calls
            std::vector<int64_t> all((size_t)std::max<int64_t>(n_graphs, 1));
            std::iota(all.begin(), all.end(), 0);
            b->d_all_ids.reserve(sizeof(int64_t) * all.size());
            PG_HIP(hipMemcpyAsync(b->d_all_ids.p, all.data(), sizeof(int64_t) * all.size(), hipMemcpyHostToDevice, s));
            PG_HIP(hipStreamSynchronize(s));
            // validate every graph on the device: symmetric, sorted, loop-free, in range
            if (nv > 0) {
                DevBuf flag;
                flag.reserve(256);
                fill_u32(flag.as<uint32_t>(), 1, 0, s);
                const int64_t blocks = std::min<int64_t>((nv + 3) / 4, (int64_t)device_info().n_cu * 16);
                k_batch_validate<<<(unsigned)blocks, 256, 0, s>>>(n_graphs, b->d_voff.as<int64_t>(),
                                                                  b->d_rp.as<int64_t>(), b->d_col.as<int32_t>(),
                                                                  nnz, flag.as<unsigned>());
                PG_HIP(hipGetLastError());
                unsigned hf = 0;
                PG_HIP(hipMemcpyAsync(&hf, flag.p, sizeof(hf), hipMemcpyDeviceToHost, s));
                PG_HIP(hipStreamSynchronize(s));
                PG_REQUIRE(hf == 0, PG_EINVAL, "invalid CSR in batch (code " + std::to_string(hf) + ")");
            }
        } catch (...) {
            delete b;
            throw;
        }
        note_object(1);
        *out = b;
    });
}

int pg_batch_free(pg_batch* b) {
    return guarded([&] {
        if (!b) return;
        (void)hipStreamSynchronize(b->stream);
        delete b;
        note_object(-1);
    });
}

int pg_batch_set_params(pg_batch* b, int block_threads, double split_work, int grid_blocks) {
    return guarded([&] {
        PG_REQUIRE(b != nullptr, PG_EINVAL, "batch is NULL");
        if (block_threads) {
            PG_REQUIRE(block_threads == 64 || block_threads == 128 || block_threads == 256 || block_threads == 512,
                       PG_EINVAL, "block_threads must be 64, 128, 256 or 512");
            b->block_threads = block_threads;
        }
        if (split_work > 0) b->split_work = split_work;
        if (grid_blocks > 0) b->grid_blocks = grid_blocks;
        b->params_gen++;
    });
}

int pg_batch_work_estimate(const pg_batch* b, double* work) {
    return guarded([&] {
        PG_REQUIRE(b != nullptr && work != nullptr, PG_EINVAL, "NULL argument");
        std::memcpy(work, b->work.data(), sizeof(double) * (size_t)b->n_graphs);
    });
}

int pg_batch_count_motifs(pg_batch* b, int k, const int64_t* ids, int64_t n_ids, uint64_t* counts) {
    return guarded([&] {
        PG_REQUIRE(b != nullptr && counts != nullptr, PG_EINVAL, "NULL argument");
        PG_REQUIRE(k == 3 || k == 4, PG_EUNSUPPORTED, "motif size must be 3 or 4");
        std::vector<int64_t> all;
        if (ids == nullptr) {
            n_ids = b->n_graphs;
            all.resize((size_t)n_ids);
            std::iota(all.begin(), all.end(), 0);
            ids = all.data();
        }
        PG_REQUIRE(n_ids >= 0, PG_EINVAL, "n_ids < 0");
        for (int64_t i = 0; i < n_ids; ++i)
            PG_REQUIRE(ids[i] >= 0 && ids[i] < b->n_graphs, PG_EINVAL, "graph id out of range");
        const int width = k == 3 ? 2 : 6;
        if (n_ids == 0) return;
        std::vector<BatchItem> items;
        build_items(b, ids, n_ids, items);
        hipStream_t s = b->stream;
        Arena& ar = b->arena;
        for (int attempt = 0;; ++attempt) {
            ar.want = std::max<size_t>(ar.want, (size_t)n_ids * (8 + 8 * width) + items.size() * sizeof(BatchItem) + 4096);
            ar.begin_call();
            try {
                int64_t* d_ids = push<int64_t>(ar, n_ids);
                BatchItem* d_items = static_cast<BatchItem*>(ar.push(items.size() * sizeof(BatchItem)));
                uint64_t* d_out = push<uint64_t>(ar, (size_t)n_ids * width);
                unsigned long long* d_next = reinterpret_cast<unsigned long long*>(push<uint64_t>(ar, 1));
                PG_HIP(hipMemcpyAsync(d_ids, ids, sizeof(int64_t) * n_ids, hipMemcpyHostToDevice, s));
                PG_HIP(hipMemcpyAsync(d_items, items.data(), items.size() * sizeof(BatchItem), hipMemcpyHostToDevice, s));
                fill_u64(d_out, (int64_t)n_ids * width, 0, s);
                launch_batch(b, k, d_ids, d_items, (int64_t)items.size(), d_out, d_next, s);
                PG_HIP(hipMemcpyAsync(counts, d_out, sizeof(uint64_t) * n_ids * width, hipMemcpyDeviceToHost, s));
                PG_HIP(hipStreamSynchronize(s));
                prof_flush();
                return;
            } catch (const Error& e) {
                (void)hipStreamSynchronize(s);
                if (e.code == PG_ENOMEM && e.msg == "arena" && attempt < 4) {
                    ar.buf.release();
                    continue;
                }
                throw;
            }
        }
    });
}

}  // extern "C"

// ----------------------------------------------- allocation-free entry point
//
// pg_batch_count_motifs_noalloc keeps its temporaries in one fixed device
// array instead of the batch's arena: the caller's ids, the queue items, the
// output rows and the queue counter.  Each GPU holds its own copy of the
// array (at its own address) until the process ends.  Host code never
// passes the array's name to a kernel or a copy: that name is a host-side
// stand-in, not a device address.  The device address is looked up once per
// device with hipGetSymbolAddress and kept.

namespace pg {

constexpr int64_t NA_MAX_IDS = PG_BATCH_STATIC_MAX_IDS;
constexpr int NA_PARTS = 4;   // queue items per graph at most
constexpr size_t na_align(size_t x) { return (x + 255) & ~size_t(255); }
constexpr size_t NA_IDS = 0;
constexpr size_t NA_ITEMS = NA_IDS + na_align(sizeof(int64_t) * NA_MAX_IDS);
constexpr size_t NA_OUT = NA_ITEMS + na_align(sizeof(BatchItem) * NA_MAX_IDS * NA_PARTS);
constexpr size_t NA_NEXT = NA_OUT + na_align(sizeof(uint64_t) * 6 * NA_MAX_IDS);
constexpr size_t NA_BYTES = NA_NEXT + 256;
static_assert(NA_BYTES <= (size_t(2) << 20), "the allocation-free scratch is 2 MiB at most");

static __device__ __align__(256) unsigned char scratch[NA_BYTES];

constexpr int NA_MAX_DEVICES = 64;
static std::mutex g_na_mu[NA_MAX_DEVICES];
static unsigned char* g_na_ptr[NA_MAX_DEVICES] = {};

// Device address of `scratch` on the current device (looked up on the
// device's first call); the caller holds g_na_mu[dev].
static unsigned char* scratch_ptr(int dev) {
    if (!g_na_ptr[dev]) {
        void* p = nullptr;
        PG_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        PG_REQUIRE(p != nullptr, PG_EDEVICE, "no device address for the static scratch array");
        g_na_ptr[dev] = static_cast<unsigned char*>(p);
    }
    return g_na_ptr[dev];
}

}  // namespace pg

extern "C" {

int pg_batch_count_motifs_noalloc(pg_batch* b, int k, const int64_t* ids, int64_t n_ids, uint64_t* counts) {
    return guarded([&] {
        PG_REQUIRE(b != nullptr && counts != nullptr, PG_EINVAL, "NULL argument");
        PG_REQUIRE(k == 3 || k == 4, PG_EUNSUPPORTED, "motif size must be 3 or 4");
        PG_REQUIRE(b->device >= 0 && b->device < NA_MAX_DEVICES, PG_EDEVICE, "device index out of range");
        std::vector<int64_t> all;
        if (ids == nullptr) {
            n_ids = b->n_graphs;
            all.resize((size_t)n_ids);
            std::iota(all.begin(), all.end(), 0);
            ids = all.data();
        }
        PG_REQUIRE(n_ids >= 0, PG_EINVAL, "n_ids < 0");
        PG_REQUIRE(n_ids <= NA_MAX_IDS, PG_EINVAL,
                   "n_ids exceeds PG_BATCH_STATIC_MAX_IDS (" + std::to_string(NA_MAX_IDS) + ")");
        for (int64_t i = 0; i < n_ids; ++i)
            PG_REQUIRE(ids[i] >= 0 && ids[i] < b->n_graphs, PG_EINVAL, "graph id out of range");
        if (n_ids == 0) return;
        const int width = k == 3 ? 2 : 6;
        std::vector<BatchItem> items;
        build_items(b, ids, n_ids, items, NA_PARTS);
        PG_REQUIRE((int64_t)items.size() <= NA_MAX_IDS * NA_PARTS, PG_EINVAL, "too many queue items");

        int prev = 0;
        PG_HIP(hipGetDevice(&prev));
        PG_HIP(hipSetDevice(b->device));
        struct Restore {
            int d;
            ~Restore() { (void)hipSetDevice(d); }
        } restore{prev};
        std::lock_guard<std::mutex> lock(g_na_mu[b->device]);
        unsigned char* base = scratch_ptr(b->device);
        int64_t* d_ids = reinterpret_cast<int64_t*>(base + NA_IDS);
        BatchItem* d_items = reinterpret_cast<BatchItem*>(base + NA_ITEMS);
        uint64_t* d_out = reinterpret_cast<uint64_t*>(base + NA_OUT);
        unsigned long long* d_next = reinterpret_cast<unsigned long long*>(base + NA_NEXT);
        hipStream_t s = b->stream;
        PG_HIP(hipMemcpyAsync(d_ids, ids, sizeof(int64_t) * n_ids, hipMemcpyHostToDevice, s));
        PG_HIP(hipMemcpyAsync(d_items, items.data(), items.size() * sizeof(BatchItem), hipMemcpyHostToDevice, s));
        // the array keeps the previous call's rows: clear this call's (a fill
        // kernel); launch_batch clears the queue counter the same way
        fill_u64(d_out, (int64_t)n_ids * width, 0, s);
        launch_batch(b, k, d_ids, d_items, (int64_t)items.size(), d_out, d_next, s);
        PG_HIP(hipMemcpyAsync(counts, d_out, sizeof(uint64_t) * n_ids * width, hipMemcpyDeviceToHost, s));
        PG_HIP(hipStreamSynchronize(s));
        prof_flush();
    });
}

}  // extern "C"

// ------------------------------------------------------------- slots

struct pg_batch_slot {
    pg_batch* b = nullptr;
    hipStream_t s = nullptr;
    int64_t max_ids = 0, max_items = 0;
    int64_t* h_ids = nullptr;          // pinned
    BatchItem* h_items = nullptr;      // pinned
    int64_t* h_n = nullptr;            // pinned: number of items
    uint64_t* h_out = nullptr;         // pinned: rows of 6
    DevBuf d_ids, d_items, d_n, d_out, d_next;
    hipGraph_t graph[2] = {nullptr, nullptr};          // k = 3, k = 4
    hipGraphExec_t exec[2] = {nullptr, nullptr};
    hipEvent_t done = nullptr;
    bool own_stream = false;           // created here because the caller passed the null stream
    bool pending = false;
    int pending_k = 4;
    int64_t pending_n = 0;
    int params_gen = -1;               // batch parameters the captured graphs were made with
    ~pg_batch_slot() {
        for (int i = 0; i < 2; ++i) {
            if (exec[i]) (void)hipGraphExecDestroy(exec[i]);
            if (graph[i]) (void)hipGraphDestroy(graph[i]);
        }
        if (done) (void)hipEventDestroy(done);
        if (h_ids) (void)hipHostFree(h_ids);
        if (h_items) (void)hipHostFree(h_items);
        if (h_n) (void)hipHostFree(h_n);
        if (h_out) (void)hipHostFree(h_out);
        if (own_stream && s) (void)hipStreamDestroy(s);
    }
};

namespace pg {

constexpr int SLOT_PARTS = 4;   // queue items per graph at most, in a slot

// Captures one replayable launch: copy ids, items and their number in, clear
// the outputs (fill kernels, no memset nodes), run the persistent kernel,
// copy the rows out.  Buffer sizes are the slot's maxima, so one graph
// serves every submission.
static void capture_slot(pg_batch_slot* S, int k) {
    pg_batch* b = S->b;
    hipStream_t s = S->s;
    const int width = 6;
    BatchArgs A;
    A.voff = b->d_voff.as<int64_t>();
    A.rp = b->d_rp.as<int64_t>();
    A.col = b->d_col.as<int32_t>();
    A.ids = S->d_ids.as<int64_t>();
    A.items = S->d_items.as<BatchItem>();
    A.n_items = 0;
    A.n_items_dev = S->d_n.as<int64_t>();
    A.next = S->d_next.as<unsigned long long>();
    A.out = S->d_out.as<unsigned long long>();
    A.k = k;
    // the same grid as a direct launch; the item count is only known on the
    // device, so the slot's maximum bounds it
    const int blocks = batch_grid(b, S->max_items);
    hipGraph_t gr = nullptr;
    PG_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    hipError_t err = hipSuccess;
    do {
        if ((err = hipMemcpyAsync(S->d_ids.p, S->h_ids, sizeof(int64_t) * S->max_ids, hipMemcpyHostToDevice, s))) break;
        if ((err = hipMemcpyAsync(S->d_items.p, S->h_items, sizeof(BatchItem) * S->max_items, hipMemcpyHostToDevice, s))) break;
        if ((err = hipMemcpyAsync(S->d_n.p, S->h_n, sizeof(int64_t), hipMemcpyHostToDevice, s))) break;
        fill_u64(S->d_out.as<uint64_t>(), S->max_ids * width, 0ull, s);
        fill_u64(S->d_next.as<uint64_t>(), 1, 0ull, s);
        switch (b->block_threads) {
            case 64: k_batch_motifs<64><<<blocks, 64, 0, s>>>(A); break;
            case 128: k_batch_motifs<128><<<blocks, 128, 0, s>>>(A); break;
            case 512: k_batch_motifs<512><<<blocks, 512, 0, s>>>(A); break;
            default: k_batch_motifs<256><<<blocks, 256, 0, s>>>(A); break;
        }
        if ((err = hipGetLastError())) break;
        err = hipMemcpyAsync(S->h_out, S->d_out.p, sizeof(uint64_t) * S->max_ids * width, hipMemcpyDeviceToHost, s);
    } while (false);
    hipError_t e2 = hipStreamEndCapture(s, &gr);
    if (err != hipSuccess || e2 != hipSuccess) {
        if (gr) (void)hipGraphDestroy(gr);
        throw Error{PG_EDEVICE, std::string("graph capture failed: ") + hipGetErrorString(err != hipSuccess ? err : e2)};
    }
    hipGraphExec_t ex = nullptr;
    hipError_t e3 = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
    if (e3 != hipSuccess) {
        (void)hipGraphDestroy(gr);
        throw Error{PG_EDEVICE, std::string("graph instantiate failed: ") + hipGetErrorString(e3)};
    }
    if (S->exec[k - 3]) (void)hipGraphExecDestroy(S->exec[k - 3]);
    if (S->graph[k - 3]) (void)hipGraphDestroy(S->graph[k - 3]);
    S->graph[k - 3] = gr;
    S->exec[k - 3] = ex;
}

// (Re)captures both graphs when the batch's parameters changed since the
// last capture; the slot must be idle.
static void ensure_captured(pg_batch_slot* S) {
    if (S->params_gen == S->b->params_gen) return;
    capture_slot(S, 3);
    capture_slot(S, 4);
    S->params_gen = S->b->params_gen;
}

}  // namespace pg

extern "C" {

int pg_batch_slot_create(pg_batch* b, int64_t max_ids, void* stream, pg_batch_slot** out) {
    return guarded([&] {
        PG_REQUIRE(b != nullptr && out != nullptr, PG_EINVAL, "NULL argument");
        PG_REQUIRE(max_ids >= 1 && max_ids <= (int64_t(1) << 24), PG_EINVAL, "max_ids out of range");
        pg_batch_slot* S = new pg_batch_slot();
        try {
            S->b = b;
            S->s = static_cast<hipStream_t>(stream);
            if (S->s == nullptr) {   // the null stream cannot be captured
                PG_HIP(hipStreamCreateWithFlags(&S->s, hipStreamNonBlocking));
                S->own_stream = true;
            }
            S->max_ids = max_ids;
            S->max_items = max_ids * SLOT_PARTS;
            PG_HIP(hipHostMalloc((void**)&S->h_ids, sizeof(int64_t) * max_ids, hipHostMallocDefault));
            PG_HIP(hipHostMalloc((void**)&S->h_items, sizeof(BatchItem) * S->max_items, hipHostMallocDefault));
            PG_HIP(hipHostMalloc((void**)&S->h_n, sizeof(int64_t), hipHostMallocDefault));
            PG_HIP(hipHostMalloc((void**)&S->h_out, sizeof(uint64_t) * max_ids * 6, hipHostMallocDefault));
            std::memset(S->h_ids, 0, sizeof(int64_t) * max_ids);
            std::memset(S->h_items, 0, sizeof(BatchItem) * S->max_items);
            *S->h_n = 0;
            S->d_ids.reserve(sizeof(int64_t) * max_ids);
            S->d_items.reserve(sizeof(BatchItem) * S->max_items);
            S->d_n.reserve(sizeof(int64_t));
            S->d_out.reserve(sizeof(uint64_t) * max_ids * 6);
            S->d_next.reserve(sizeof(uint64_t));
            PG_HIP(hipEventCreateWithFlags(&S->done, hipEventDisableTiming));
            ensure_captured(S);
        } catch (...) {
            delete S;
            throw;
        }
        note_object(1);
        *out = S;
    });
}

int pg_batch_slot_submit(pg_batch_slot* S, int k, const int64_t* ids, int64_t n_ids) {
    return guarded([&] {
        PG_REQUIRE(S != nullptr && (ids != nullptr || n_ids == 0), PG_EINVAL, "NULL argument");
        PG_REQUIRE(k == 3 || k == 4, PG_EUNSUPPORTED, "motif size must be 3 or 4");
        PG_REQUIRE(!S->pending, PG_EINVAL, "slot is busy");
        PG_REQUIRE(n_ids >= 0 && n_ids <= S->max_ids, PG_EINVAL, "too many ids for this slot");
        for (int64_t i = 0; i < n_ids; ++i)
            PG_REQUIRE(ids[i] >= 0 && ids[i] < S->b->n_graphs, PG_EINVAL, "graph id out of range");
        ensure_captured(S);   // pg_batch_set_params since the last submission
        std::vector<BatchItem> items;
        build_items(S->b, ids, n_ids, items, SLOT_PARTS);
        std::memcpy(S->h_ids, ids, sizeof(int64_t) * n_ids);
        std::memcpy(S->h_items, items.data(), sizeof(BatchItem) * items.size());
        *S->h_n = (int64_t)items.size();
        PG_HIP(hipGraphLaunch(S->exec[k - 3], S->s));
        PG_HIP(hipEventRecord(S->done, S->s));
        S->pending = true;
        S->pending_k = k;
        S->pending_n = n_ids;
    });
}

int pg_batch_slot_query(pg_batch_slot* S) {
    if (!S) return PG_EINVAL;
    if (!S->pending) return 1;
    hipError_t e = hipEventQuery(S->done);
    if (e == hipSuccess) return 1;
    if (e == hipErrorNotReady) return 0;
    pg::set_error(std::string("hipEventQuery: ") + hipGetErrorString(e));
    return PG_EDEVICE;
}

int pg_batch_slot_wait(pg_batch_slot* S, uint64_t* counts) {
    return guarded([&] {
        PG_REQUIRE(S != nullptr, PG_EINVAL, "slot is NULL");
        if (!S->pending) return;
        PG_HIP(hipEventSynchronize(S->done));
        // the kernel packs rows of the submission's width (2 for k = 3)
        const int width = S->pending_k == 3 ? 2 : 6;
        if (counts) std::memcpy(counts, S->h_out, sizeof(uint64_t) * S->pending_n * width);
        S->pending = false;
    });
}

int pg_batch_slot_free(pg_batch_slot* S) {
    return guarded([&] {
        if (!S) return;
        if (S->pending) (void)hipEventSynchronize(S->done);
        (void)hipStreamSynchronize(S->s);
        delete S;
        note_object(-1);
    });
}

}  // extern "C"
