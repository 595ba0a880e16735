// Runtime pieces of the mining library: error state, device memory,
// kernel timing, and the scan / radix-sort / fill primitives the level
// pipelines are built from.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "pg_device.h"
#include "pg_internal.h"

namespace pg {

// ------------------------------------------------------------ error state

static thread_local std::string t_last_error = "";

void set_error(const std::string& msg) { t_last_error = msg; }

const char* last_error() { return t_last_error.c_str(); }

// ---------------------------------------------------------------- memory

static void* (*g_alloc)(size_t, void*) = nullptr;
static void (*g_free)(void*, void*) = nullptr;
static void* g_alloc_ctx = nullptr;

void* dev_alloc(size_t bytes) {
    if (bytes == 0) bytes = 256;
    void* p = nullptr;
    if (g_alloc) {
        p = g_alloc(bytes, g_alloc_ctx);
        if (!p) throw Error{PG_ENOMEM, "allocator hook returned NULL for " + std::to_string(bytes) + " bytes"};
        return p;
    }
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        throw Error{PG_ENOMEM, "hipMalloc(" + std::to_string(bytes) + ") failed: " + hipGetErrorString(e)};
    }
    return p;
}

void dev_free(void* p) {
    if (!p) return;
    if (g_free) g_free(p, g_alloc_ctx);
    else (void)hipFree(p);
}

void set_allocator(void* (*a)(size_t, void*), void (*f)(void*, void*), void* ctx) {
    g_alloc = a;
    g_free = f;
    g_alloc_ctx = ctx;
}

void DevBuf::reserve(size_t need) {
    if (need <= bytes && p) return;
    release();
    p = dev_alloc(need);
    bytes = need;
}

void DevBuf::release() {
    if (p) dev_free(p);
    p = nullptr;
    bytes = 0;
}

void Arena::begin_call() {
    top = 0;
    high = 0;
    want = std::max<size_t>(want, size_t(4) << 20);
    if (want > buf.bytes) buf.reserve(want);
}

void Arena::ensure(size_t bytes) {
    if (top + bytes > buf.bytes) {
        // Remember the size this call needed; the caller retries after growth.
        need = std::max(need, top + bytes);
        want = std::max(want, need + need / 4);
        throw Error{PG_ENOMEM, "arena"};
    }
}

void* Arena::push(size_t bytes) {
    size_t b = (bytes + 255) & ~size_t(255);
    ensure(b);
    void* p = static_cast<char*>(buf.p) + top;
    top += b;
    high = std::max(high, top);
    return p;
}

// ------------------------------------------------------------- device info

const DeviceInfo& device_info() {
    static DeviceInfo info;
    static bool done = false;
    static std::mutex mu;
    std::lock_guard<std::mutex> lk(mu);
    if (!done) {
        int dev = 0;
        PG_HIP(hipGetDevice(&dev));
        hipDeviceProp_t prop;
        PG_HIP(hipGetDeviceProperties(&prop, dev));
        info.device = dev;
        info.n_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
        info.total_mem = prop.totalGlobalMem;
        done = true;
    }
    return info;
}

int64_t grid_waves(int waves_per_cu) { return (int64_t)device_info().n_cu * waves_per_cu; }

// --------------------------------------------------------------- profiling

struct ProfStat {
    double ms = 0;
    uint64_t launches = 0;
    double units = 0;
};
struct Pending {
    std::string name;
    hipEvent_t a, b;
    double units;
};
static std::mutex g_prof_mu;
static bool g_prof = false;
static std::map<std::string, ProfStat> g_stats;
static std::vector<Pending> g_pending;
static std::vector<hipEvent_t> g_event_pool;

bool prof_on() { return g_prof; }

static hipEvent_t get_event() {
    if (!g_event_pool.empty()) {
        hipEvent_t e = g_event_pool.back();
        g_event_pool.pop_back();
        return e;
    }
    hipEvent_t e;
    PG_HIP(hipEventCreate(&e));
    return e;
}

ProfScope::ProfScope(const char* kernel, hipStream_t st, double units) : s(st) {
    if (!g_prof) return;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    Pending p{kernel, get_event(), get_event(), units};
    PG_HIP(hipEventRecord(p.a, s));
    g_pending.push_back(p);
    slot = (int)g_pending.size() - 1;
}

ProfScope::~ProfScope() {
    if (slot < 0) return;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (slot < (int)g_pending.size()) (void)hipEventRecord(g_pending[slot].b, s);
}

void prof_flush() {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    for (auto& p : g_pending) {
        float ms = 0;
        if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            auto& st = g_stats[p.name];
            st.ms += ms;
            st.launches += 1;
            st.units += p.units;
        }
        g_event_pool.push_back(p.a);
        g_event_pool.push_back(p.b);
    }
    g_pending.clear();
}

void prof_enable(bool on) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof = on;
}

void prof_reset() {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_stats.clear();
}

bool prof_query(const char* name, double* ms, uint64_t* launches, double* units) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    auto it = g_stats.find(name);
    if (it == g_stats.end()) return false;
    if (ms) *ms = it->second.ms;
    if (launches) *launches = it->second.launches;
    if (units) *units = it->second.units;
    return true;
}

std::string prof_list() {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    std::string s;
    for (auto& kv : g_stats) {
        s += kv.first;
        s += "\n";
    }
    return s;
}

// ------------------------------------------------------------------ fill

template <class T>
__global__ void k_fill(T* p, int64_t n, T v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

void fill_u64(uint64_t* p, int64_t n, uint64_t v, hipStream_t s) {
    if (n <= 0) return;
    int blocks = (int)std::min<int64_t>((n + 255) / 256, 4096);
    k_fill<uint64_t><<<blocks, 256, 0, s>>>(p, n, v);
    PG_HIP(hipGetLastError());
}

void fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t s) {
    if (n <= 0) return;
    int blocks = (int)std::min<int64_t>((n + 255) / 256, 4096);
    k_fill<uint32_t><<<blocks, 256, 0, s>>>(p, n, v);
    PG_HIP(hipGetLastError());
}

// ------------------------------------------------------------ round items

// rounds of `per` children of each segment whose child count lies in
// [cmin, cmax); other segments get none
template <class T>
__global__ void k_round_counts(const T* __restrict__ seg, int64_t p_lo, int64_t n_seg, int per, int64_t cmin,
                               int64_t cmax, uint32_t* __restrict__ rounds) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n_seg;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = (int64_t)(seg[p_lo + i + 1] - seg[p_lo + i]);
        rounds[i] = (c >= cmin && c < cmax) ? (uint32_t)((c + per - 1) / per) : 0u;
    }
}

__global__ void k_round_emit(int64_t p_lo, int64_t n_seg, const uint64_t* __restrict__ pos,
                             uint64_t* __restrict__ items, uint64_t cap, uint64_t* __restrict__ count_dev) {
    if (count_dev && blockIdx.x == 0 && threadIdx.x == 0) *count_dev = pos[n_seg] < cap ? pos[n_seg] : cap;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n_seg;
         i += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t b = pos[i], e = pos[i + 1] < cap ? pos[i + 1] : cap;
        const uint64_t p = (uint64_t)(p_lo + i) << ROUND_BITS;
        for (uint64_t k = b; k < e; ++k) items[k] = p | (k - b);
    }
}

template <class T>
static int64_t round_items_impl(const T* seg, int64_t p_lo, int64_t n_seg, int per, int64_t total, Arena& a,
                                hipStream_t s, uint64_t** items, uint64_t* count_dev, int64_t cmin = 0,
                                int64_t cmax = INT64_MAX) {
    *items = nullptr;
    if (n_seg <= 0) {
        if (count_dev) fill_u64(count_dev, 1, 0, s);
        return 0;
    }
    PG_REQUIRE((uint64_t)(p_lo + n_seg) < (1ull << (64 - ROUND_BITS)), PG_EOVERFLOW, "too many segments");
    const unsigned blocks = (unsigned)std::min<int64_t>((n_seg + 255) / 256, 8192);
    if (total >= 0) {
        // sum of ceil(c / per) <= total / per + n_seg: the items go first,
        // at that bound, and one pass fills them
        const int64_t cap = total / per + n_seg + 1;
        uint64_t* out = push<uint64_t>(a, cap);
        const size_t mk = a.mark();
        uint32_t* rounds = push<uint32_t>(a, n_seg);
        uint64_t* pos = push<uint64_t>(a, n_seg + 1);
        k_round_counts<T><<<blocks, 256, 0, s>>>(seg, p_lo, n_seg, per, cmin, cmax, rounds);
        PG_HIP(hipGetLastError());
        scan_u32(rounds, n_seg, pos, a, s);
        k_round_emit<<<blocks, 256, 0, s>>>(p_lo, n_seg, pos, out, (uint64_t)cap, count_dev);
        PG_HIP(hipGetLastError());
        if (count_dev) {
            a.reset(mk);
            *items = out;
            return cap;
        }
        const int64_t m = (int64_t)read_u64(pos + n_seg, s);
        a.reset(mk);
        PG_REQUIRE(m <= cap, PG_EOVERFLOW, "work items exceed their bound: segment sizes disagree with the total");
        *items = out;
        return m;
    }
    const size_t mk = a.mark();
    uint32_t* rounds = push<uint32_t>(a, n_seg);
    uint64_t* pos = push<uint64_t>(a, n_seg + 1);
    k_round_counts<T><<<blocks, 256, 0, s>>>(seg, p_lo, n_seg, per, cmin, cmax, rounds);
    PG_HIP(hipGetLastError());
    scan_u32(rounds, n_seg, pos, a, s);
    const int64_t m = (int64_t)read_u64(pos + n_seg, s);
    // the items go below the temporaries' mark so that those can be dropped
    a.reset(mk);
    uint64_t* out = push<uint64_t>(a, std::max<int64_t>(m, 1));
    const size_t mk2 = a.mark();
    uint32_t* rounds2 = push<uint32_t>(a, n_seg);
    uint64_t* pos2 = push<uint64_t>(a, n_seg + 1);
    k_round_counts<T><<<blocks, 256, 0, s>>>(seg, p_lo, n_seg, per, cmin, cmax, rounds2);
    PG_HIP(hipGetLastError());
    scan_u32(rounds2, n_seg, pos2, a, s);
    k_round_emit<<<blocks, 256, 0, s>>>(p_lo, n_seg, pos2, out, (uint64_t)m, count_dev);
    PG_HIP(hipGetLastError());
    a.reset(mk2);
    *items = out;
    return m;
}

int64_t round_items(const int64_t* seg, int64_t p_lo, int64_t n_seg, int per, Arena& a, hipStream_t s,
                    uint64_t** items, int64_t total, uint64_t* count_dev) {
    return round_items_impl(seg, p_lo, n_seg, per, total, a, s, items, count_dev);
}

int64_t round_items(const uint64_t* seg, int64_t p_lo, int64_t n_seg, int per, Arena& a, hipStream_t s,
                    uint64_t** items, int64_t total, uint64_t* count_dev) {
    return round_items_impl(seg, p_lo, n_seg, per, total, a, s, items, count_dev);
}

int64_t round_items_between(const uint64_t* seg, int64_t p_lo, int64_t n_seg, int per, int64_t cmin, int64_t cmax,
                            Arena& a, hipStream_t s, uint64_t** items) {
    return round_items_impl(seg, p_lo, n_seg, per, -1, a, s, items, nullptr, cmin, cmax);
}

uint64_t read_u64(const uint64_t* dev, hipStream_t s) {
    uint64_t h = 0;
    PG_HIP(hipMemcpyAsync(&h, dev, sizeof(h), hipMemcpyDeviceToHost, s));
    PG_HIP(hipStreamSynchronize(s));
    return h;
}

// ------------------------------------------------------------------ scan
//
// Three phases (inspection-execution's prefix sum, section 5.3):
// per-tile sums, an exclusive scan of the tile sums (recursively), then a
// per-tile exclusive scan offset by the tile's base.  A tile is 256 threads
// x 8 consecutive items.  With few tiles each block adds up the sums of the
// tiles before it itself, and the scan takes two launches (one for a single
// tile).

constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int64_t SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;

template <class Tin>
__global__ __launch_bounds__(SCAN_THREADS) void k_scan_tile_sums(const Tin* __restrict__ in, int64_t m,
                                                                 uint64_t* __restrict__ sums) {
    __shared__ uint64_t part[SCAN_THREADS / WAVE];
    const int64_t base = blockIdx.x * SCAN_TILE + threadIdx.x * SCAN_ITEMS;
    uint64_t s = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i)
        if (base + i < m) s += (uint64_t)in[base + i];
    s = wave_sum_u64(s);
    if (lane() == 0) part[threadIdx.x / WAVE] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t t = 0;
        for (int w = 0; w < SCAN_THREADS / WAVE; ++w) t += part[w];
        sums[blockIdx.x] = t;
    }
}

// LOCAL: the tile's base is the sum of sums[0, blockIdx.x), added up by
// the block itself (for few tiles); else tile_base[blockIdx.x].
template <class Tin, bool LOCAL>
__global__ __launch_bounds__(SCAN_THREADS) void k_scan_tiles(const Tin* __restrict__ in, int64_t m,
                                                             const uint64_t* __restrict__ tile_base,
                                                             uint64_t* __restrict__ out) {
    __shared__ uint64_t wave_tot[SCAN_THREADS / WAVE];
    __shared__ uint64_t wave_pre[SCAN_THREADS / WAVE];
    const int64_t base = blockIdx.x * SCAN_TILE + threadIdx.x * SCAN_ITEMS;
    const int w = threadIdx.x / WAVE;
    uint64_t before = 0;
    if (LOCAL) {
        uint64_t acc = 0;
        for (int64_t i = threadIdx.x; i < (int64_t)blockIdx.x; i += SCAN_THREADS) acc += tile_base[i];
        acc = wave_sum_u64(acc);
        if (lane() == 0) wave_pre[w] = acc;
    }
    uint64_t v[SCAN_ITEMS];
    uint64_t s = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        v[i] = (base + i < m) ? (uint64_t)in[base + i] : 0;
        s += v[i];
    }
    // inclusive scan of per-thread sums within the wave
    uint64_t inc = s;
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
        uint64_t t = (uint64_t)__shfl_up((unsigned long long)inc, d, WAVE);
        if (lane() >= d) inc += t;
    }
    if (lane() == WAVE - 1) wave_tot[w] = inc;
    __syncthreads();
    if (LOCAL) {
        for (int j = 0; j < SCAN_THREADS / WAVE; ++j) before += wave_pre[j];
    } else {
        before = tile_base[blockIdx.x];
    }
    for (int j = 0; j < w; ++j) before += wave_tot[j];
    uint64_t run = before + inc - s;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        if (base + i < m) out[base + i] = run;
        run += v[i];
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == SCAN_THREADS - 1) out[m] = run;
}

// tiles up to this many add up their own bases (two launches in all)
constexpr int64_t SCAN_LOCAL_TILES = 2048;

template <class Tin>
static void scan_impl(const Tin* in, int64_t m, uint64_t* out, Arena& a, hipStream_t s) {
    if (m <= 0) {
        fill_u64(out, 1, 0, s);
        return;
    }
    const int64_t tiles = (m + SCAN_TILE - 1) / SCAN_TILE;
    size_t mk = a.mark();
    uint64_t* sums = push<uint64_t>(a, tiles);
    if (tiles > 1) {
        ProfScope ps("scan", s, (double)m);
        k_scan_tile_sums<Tin><<<(unsigned)tiles, SCAN_THREADS, 0, s>>>(in, m, sums);
        PG_HIP(hipGetLastError());
    }
    if (tiles <= SCAN_LOCAL_TILES) {
        ProfScope ps("scan", s, tiles > 1 ? 0.0 : (double)m);
        k_scan_tiles<Tin, true><<<(unsigned)tiles, SCAN_THREADS, 0, s>>>(in, m, sums, out);
        PG_HIP(hipGetLastError());
    } else {
        uint64_t* base = push<uint64_t>(a, tiles + 1);
        scan_impl<uint64_t>(sums, tiles, base, a, s);
        ProfScope ps("scan", s, 0.0);
        k_scan_tiles<Tin, false><<<(unsigned)tiles, SCAN_THREADS, 0, s>>>(in, m, base, out);
        PG_HIP(hipGetLastError());
    }
    a.reset(mk);
}

void scan_u32(const uint32_t* in, int64_t m, uint64_t* out, Arena& a, hipStream_t s) {
    scan_impl<uint32_t>(in, m, out, a, s);
}

void scan_u64(const uint64_t* in, int64_t m, uint64_t* out, Arena& a, hipStream_t s) {
    scan_impl<uint64_t>(in, m, out, a, s);
}

// ------------------------------------------------------------ radix sort
//
// Stable LSD radix sort, 8-bit digits.  Each pass: a digit histogram per
// tile (laid out digit-major), an exclusive scan of the histograms, then a
// stable scatter.  Inside a tile every wave owns a contiguous run of keys
// and ranks them in order; the ranks of equal digits within one 64-key
// step come from eight ballots (one per digit bit).  The ranked keys are
// first placed in LDS in digit order, then written out in that order, so
// that each digit's keys of a tile (32 on average) leave as one run.

constexpr int RS_THREADS = 512;    // at least 256: one thread per digit
constexpr int RS_WAVES = RS_THREADS / WAVE;
constexpr int RS_PER_WAVE = 1024;   // keys per wave per tile
constexpr int64_t RS_TILE = (int64_t)RS_WAVES * RS_PER_WAVE;

__global__ __launch_bounds__(RS_THREADS) void k_radix_hist(const uint64_t* __restrict__ keys, int64_t m,
                                                           int shift, int64_t n_tiles,
                                                           uint32_t* __restrict__ hist) {
    __shared__ uint32_t h[256];
    if (threadIdx.x < 256) h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t t0 = blockIdx.x * RS_TILE;
    for (int64_t i = threadIdx.x; i < RS_TILE; i += RS_THREADS) {
        int64_t j = t0 + i;
        if (j < m) atomicAdd(&h[(keys[j] >> shift) & 255u], 1u);
    }
    __syncthreads();
    if (threadIdx.x < 256) hist[(int64_t)threadIdx.x * n_tiles + blockIdx.x] = h[threadIdx.x];
}

__global__ __launch_bounds__(RS_THREADS) void k_radix_scatter(const uint64_t* __restrict__ keys, int64_t m,
                                                              int shift, int64_t n_tiles,
                                                              const uint64_t* __restrict__ offs,
                                                              uint64_t* __restrict__ out) {
    constexpr int KPL = RS_PER_WAVE / WAVE;   // keys per lane, held in registers
    // per wave and digit: its count, then (in place) its next place
    __shared__ uint32_t run[RS_WAVES][256];
    __shared__ uint32_t dstart[256];
    __shared__ uint64_t doff[256];   // the digit's first place in the output, for this tile
    __shared__ uint64_t sk[RS_TILE];
    const int w = threadIdx.x / WAVE;
    for (int d = lane(); d < 256; d += WAVE) run[w][d] = 0;
    if (threadIdx.x < 256) doff[threadIdx.x] = offs[(int64_t)threadIdx.x * n_tiles + blockIdx.x];
    const int64_t tbase = blockIdx.x * RS_TILE;
    const int64_t wbase = tbase + (int64_t)w * RS_PER_WAVE;
    uint64_t kk[KPL];
#pragma unroll
    for (int i = 0; i < KPL; ++i) {
        const int64_t j = wbase + i * WAVE + lane();
        kk[i] = j < m ? keys[j] : 0ull;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < KPL; ++i)
        if (wbase + i * WAVE + lane() < m) atomicAdd(&run[w][(kk[i] >> shift) & 255u], 1u);
    __syncthreads();
    // dstart[d]: first place of digit d in the tile's digit order (one
    // thread per digit, the 256 totals scanned by the first wave's lanes)
    if (threadIdx.x < 256) {
        const int d = threadIdx.x;
        uint32_t tot = 0;
        for (int ww = 0; ww < RS_WAVES; ++ww) tot += run[ww][d];
        dstart[d] = tot;
    }
    __syncthreads();
    if (w == 0) {
        uint32_t carry = 0;
        for (int c = 0; c < 256; c += WAVE) {
            const uint32_t v = dstart[c + lane()];
            const uint32_t inc = wave_incl_scan(v);
            dstart[c + lane()] = carry + inc - v;
            carry += bcast(inc, WAVE - 1);
        }
    }
    __syncthreads();
    // run[w][d] = place of wave w's first key of digit d
    if (threadIdx.x < 256) {
        const int d = threadIdx.x;
        uint32_t acc = dstart[d];
        for (int ww = 0; ww < RS_WAVES; ++ww) {
            const uint32_t c = run[ww][d];
            run[ww][d] = acc;
            acc += c;
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < KPL; ++i) {
        const bool valid = wbase + i * WAVE + lane() < m;
        const uint64_t k = kk[i];
        const uint32_t d = (uint32_t)((k >> shift) & 255u);
        uint64_t peers = ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const uint64_t mb = ballot(((d >> b) & 1u) != 0);
            peers &= ((d >> b) & 1u) ? mb : ~mb;
        }
        const uint32_t before = (uint32_t)popc64(peers & lanemask_lt());
        const uint32_t base = valid ? run[w][d] : 0;
        if (valid) sk[base + before] = k;
        // the highest lane of each digit group advances the running count
        const bool last = valid && ((peers >> lane()) == 1ull);
        if (last) run[w][d] = base + before + 1;
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    // out in digit order: a digit's keys go to consecutive places
    const int n = (int)min64(RS_TILE, m - tbase);
    for (int p = threadIdx.x; p < n; p += RS_THREADS) {
        const uint64_t k = sk[p];
        const uint32_t d = (uint32_t)((k >> shift) & 255u);
        out[doff[d] + (uint32_t)(p - (int)dstart[d])] = k;
    }
}

void radix_sort_u64(uint64_t* keys, uint64_t* tmp, int64_t m, int lo_bit, int hi_bit, Arena& a,
                    hipStream_t s) {
    if (m <= 1) return;
    const int64_t n_tiles = (m + RS_TILE - 1) / RS_TILE;
    size_t mk = a.mark();
    uint32_t* hist = push<uint32_t>(a, 256 * n_tiles);
    uint64_t* offs = push<uint64_t>(a, 256 * n_tiles + 1);
    uint64_t* src = keys;
    uint64_t* dst = tmp;
    for (int shift = lo_bit; shift < hi_bit; shift += 8) {
        ProfScope ps("radix_sort", s, (double)m);
        // per pass every key is read twice (histogram, scatter) and written once
        ProfScope pw("radix_sort_work", s, 24.0 * (double)m);
        k_radix_hist<<<(unsigned)n_tiles, RS_THREADS, 0, s>>>(src, m, shift, n_tiles, hist);
        PG_HIP(hipGetLastError());
        scan_u32(hist, 256 * n_tiles, offs, a, s);
        k_radix_scatter<<<(unsigned)n_tiles, RS_THREADS, 0, s>>>(src, m, shift, n_tiles, offs, dst);
        PG_HIP(hipGetLastError());
        std::swap(src, dst);
    }
    if (src != keys) PG_HIP(hipMemcpyAsync(keys, src, sizeof(uint64_t) * m, hipMemcpyDeviceToDevice, s));
    a.reset(mk);
}

}  // namespace pg
