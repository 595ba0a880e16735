// Device-side helpers for 64-lane CDNA wavefronts.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace pg {

constexpr int WAVE = 64;
constexpr int N_XCD = 8;   // MI355X: 8 accelerator complex dies, 32 CUs each

__device__ __forceinline__ int lane() { return __lane_id(); }

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

// Makes LDS writes of every lane visible to the other lanes of the wave.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint64_t lanemask_lt() {
    return (lane() == 0) ? 0ull : (~0ull >> (64 - lane()));
}

__device__ __forceinline__ int popc64(uint64_t x) { return __popcll(x); }

template <class T>
__device__ __forceinline__ T bcast(T v, int src) {
    return __shfl(v, src, WAVE);
}

__device__ __forceinline__ int64_t bcast64(int64_t v, int src) {
    return (int64_t)__shfl((long long)v, src, WAVE);
}

// 64-bit integer min / max by compare and select (HIP's generic min/max on
// 64-bit integers goes through double precision).
__host__ __device__ __forceinline__ int64_t min64(int64_t a, int64_t b) { return a < b ? a : b; }
__host__ __device__ __forceinline__ int64_t max64(int64_t a, int64_t b) { return a > b ? a : b; }

// Value of v in lane l, for a wave-uniform l (a scalar read of the lane's
// register, no LDS traffic).
__device__ __forceinline__ int32_t readlane(int32_t v, int l) {
    return __builtin_amdgcn_readlane(v, l);
}

__device__ __forceinline__ uint64_t readlane64(uint64_t v, int l) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), l);
    return ((uint64_t)hi << 32) | lo;
}

// Marks a value the same in every lane as such (it goes to a scalar
// register, and branches on it become scalar branches).
__device__ __forceinline__ int32_t uniform(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ int64_t uniform64(int64_t v) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Inclusive prefix sum across the wave.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
        uint32_t t = __shfl_up(v, d, WAVE);
        if (lane() >= d) v += t;
    }
    return v;
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
#pragma unroll
    for (int d = WAVE / 2; d > 0; d >>= 1) v += (uint64_t)__shfl_xor((unsigned long long)v, d, WAVE);
    return v;
}

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
#pragma unroll
    for (int d = WAVE / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, WAVE);
    return v;
}

// First index in [lo, hi) with a[i] >= key.
template <class P>
__device__ __forceinline__ int64_t lower_bound(P a, int64_t lo, int64_t hi, int32_t key) {
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (a[mid] < key) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// First index in [lo, hi) with a[i] > key.
template <class P>
__device__ __forceinline__ int64_t upper_bound(P a, int64_t lo, int64_t hi, int32_t key) {
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (a[mid] <= key) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// Branch-free membership test in a sorted array of length len (len >= 0).
template <class P>
__device__ __forceinline__ bool contains(P a, int32_t len, int32_t key) {
    if (len <= 0) return false;
    int32_t base = 0;
    int32_t n = len;
    while (n > 1) {
        int32_t half = n >> 1;
        base = (a[base + half] <= key) ? base + half : base;
        n -= half;
    }
    return a[base] == key;
}

// Membership of key in the sorted a[0, n) for n >= 1, LG = floor(log2(n)):
// Shar's search.  With m = 2^LG, one probe at m - 1 decides whether the
// last element <= key lies among the first m - 1 positions or the last m;
// strides m/2 .. 1 finish it.  Probes stay inside a[0, n), strides are
// immediates and the chain is straight-line code.
template <int LG, class P>
__device__ __forceinline__ bool member_shar(P a, int32_t n, int32_t key) {
    constexpr int32_t m = 1 << LG;
    P q = (a[m - 1] <= key) ? a + (n - m) : a - 1;   // last element <= key, or a - 1
#pragma unroll
    for (int st = m / 2; st >= 1; st >>= 1) q = (q[st] <= key) ? q + st : q;
    return q >= a && *(q >= a ? q : a) == key;
}

// Membership for a wave-uniform n (the depth switch is a scalar branch).
template <class P>
__device__ __forceinline__ bool member_u(P a, int32_t n, int32_t key) {
    if (n <= 0) return false;
    switch (31 - __clz(n)) {
        case 0: return member_shar<0>(a, n, key);
        case 1: return member_shar<1>(a, n, key);
        case 2: return member_shar<2>(a, n, key);
        case 3: return member_shar<3>(a, n, key);
        case 4: return member_shar<4>(a, n, key);
        case 5: return member_shar<5>(a, n, key);
        case 6: return member_shar<6>(a, n, key);
        case 7: return member_shar<7>(a, n, key);
        case 8: return member_shar<8>(a, n, key);
        case 9: return member_shar<9>(a, n, key);
        default: return contains(a, n, key);
    }
}

// Word 3 of a buffer resource for raw 32-bit loads (gfx9 family): with a
// record count in bytes, lanes past it read 0.
constexpr int BUF_WORD3 = 0x00020000;

// ---------------------------------------------------------- work queues
//
// Items [0, n_items) are split into Q_PARTS contiguous ranges, one per die,
// so that neighbouring items (which share adjacency lists) run on the same
// die and share its L2.  Workgroups are dispatched to dies round-robin, so
// workgroup b runs on die b % N_XCD and starts on range b % Q_PARTS.  A wave
// takes `chunk` items at a time from its range and, when that is exhausted,
// from the other ranges in turn; every wave stops after all ranges are
// exhausted.  The counters sit in cache lines of their own: atomics of all
// dies on one line serialise on it (sharing one line cost the 4-clique count
// pass a tenth of its time).  More ranges per die did not pay.
constexpr int Q_PARTS = N_XCD;
constexpr int Q_STRIDE = 16;   // counters 128 bytes apart
constexpr int Q_WORDS = Q_PARTS * Q_STRIDE;

struct XcdQueue {
    unsigned long long* next;   // Q_WORDS words, zeroed before the launch
    int64_t n_items;
    int64_t chunk;
};

struct QueueCursor {
    int start;    // first range
    int tried;    // ranges found exhausted
};

__device__ __forceinline__ int64_t xcd_lo(const XcdQueue& Q, int q) {
    return (Q.n_items * q) / Q_PARTS;
}

// the tried-th range to visit, starting from the wave's own
__device__ __forceinline__ int queue_range(const QueueCursor& c) {
    return (c.start + c.tried) % Q_PARTS;
}

// Returns the first item of the next chunk (its end is min(first + chunk,
// range end)) or -1 when all ranges are exhausted.  Wave-uniform.
__device__ __forceinline__ int64_t queue_next(const XcdQueue& Q, QueueCursor& c, int64_t& end) {
    while (c.tried < Q_PARTS) {
        const int q = queue_range(c);
        const int64_t lo = xcd_lo(Q, q), hi = xcd_lo(Q, q + 1);
        int64_t got = 0;
        if (lane() == 0) got = (int64_t)atomicAdd(&Q.next[q * Q_STRIDE], (unsigned long long)Q.chunk);
        got = bcast64(got, 0);
        const int64_t first = lo + got;
        if (first < hi) {
            end = min64(first + Q.chunk, hi);
            return first;
        }
        c.tried++;
    }
    return -1;
}

__device__ __forceinline__ QueueCursor queue_start() {
    QueueCursor c;
    c.start = blockIdx.x % Q_PARTS;
    c.tried = 0;
    return c;
}

}  // namespace pg
