// host_common.h -- host-side helpers shared by the single-cloud and the
// batched pipelines: grow-only device / pinned buffers, event timers, error
// macros and small index utilities.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <string>
#include <utility>
#include <vector>

#include "../../include/rpp.h"

namespace rpp {

// Capacity for a buffer that must hold `bytes` and held `old` before: at least
// 1.5x the old capacity, rounded up to 64 KiB, so a sequence of slowly
// growing requests reallocates O(log) times rather than on nearly every call
// (each reallocation is a device-wide synchronising free + malloc).
inline size_t grow_capacity(size_t old, size_t bytes)
{
    size_t b = bytes < 256 ? 256 : bytes;
    if (old) {
        const size_t g = old + old / 2;
        if (g > b)
            b = g;
    }
    return (b + 65535) & ~(size_t)65535;
}

// Where the device buffers of one workspace come from.
//  - Own allocations (the default): hipMalloc, with 1.5x growth headroom;
//    with a limit (a serving slot's reservation, RPP_DEVICE_BUDGET_BYTES)
//    every allocation is exact-sized and the buffers together never hold
//    more than the limit.
//  - A caller-provided arena (rpp_barcodes_device's workspace argument):
//    buffers are carved from it bottom-up and never freed; a buffer takes
//    its planned maximum for the call (its hint) on first use when that
//    still fits, so an arena of at least the sum of the hints never runs
//    out, and otherwise exactly what is asked.
struct DevPool {
    char *arena = nullptr;
    size_t arena_size = 0, arena_top = 0;
    size_t limit = SIZE_MAX;    // own allocations: most bytes held at once
    size_t held = 0;            // own allocations: bytes held now
    bool exhausted = false;     // the last failed request hit the arena end or the limit
};

// Device buffer; grows, never shrinks; movable, not copyable.
struct DevBuf {
    void *p = nullptr;
    size_t cap = 0;
    size_t hint = 0;            // planned maximum (arena mode)
    DevPool *pool = nullptr;    // allocation policy; null = plain hipMalloc
    bool owned = true;          // false: carved from an arena, never freed here
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    DevBuf(DevBuf &&o) noexcept
        : p(o.p), cap(o.cap), hint(o.hint), pool(o.pool), owned(o.owned)
    {
        o.p = nullptr;
        o.cap = 0;
        o.owned = true;
    }
    DevBuf &operator=(DevBuf &&o) noexcept
    {
        std::swap(p, o.p);
        std::swap(cap, o.cap);
        std::swap(hint, o.hint);
        std::swap(pool, o.pool);
        std::swap(owned, o.owned);
        return *this;
    }
    ~DevBuf() { release(); }
    // Free own memory (arena memory is simply forgotten).
    void release()
    {
        if (p && owned) {
            (void)hipFree(p);
            if (pool)
                pool->held -= cap;
        }
        p = nullptr;
        cap = 0;
        owned = true;
    }
    bool ensure(size_t bytes)
    {
        if (bytes <= cap && p)
            return true;
        if (pool && pool->arena) {
            const size_t left = pool->arena_size - pool->arena_top;
            size_t want = ((bytes > hint ? bytes : hint) + 255) & ~(size_t)255;
            if (want > left)
                want = (bytes + 255) & ~(size_t)255;
            if (want > left) {
                pool->exhausted = true;
                return false;
            }
            release();
            p = pool->arena + pool->arena_top;
            pool->arena_top += want;
            cap = want;
            owned = false;
            return true;
        }
        const size_t cap0 = (p && owned) ? cap : 0;
        const bool limited = pool && pool->limit != SIZE_MAX;
        size_t b = limited ? grow_capacity(0, bytes) : grow_capacity(cap0, bytes);
        if (limited && pool->held - cap0 + b > pool->limit) {
            pool->exhausted = true;
            return false;
        }
        release();
        if (hipMalloc(&p, b) != hipSuccess) {
            // The headroom may not fit where the exact size does.
            const size_t e = grow_capacity(0, bytes);
            p = nullptr;
            if (e >= b || hipMalloc(&p, e) != hipSuccess) {
                p = nullptr;
                return false;
            }
            b = e;
        }
        cap = b;
        if (pool)
            pool->held += b;
        return true;
    }
    template <typename T>
    T *as() const
    {
        return static_cast<T *>(p);
    }
};

// Owning pinned host buffer (hipHostMalloc); same rules as DevBuf.
struct HostBuf {
    void *p = nullptr;
    size_t cap = 0;
    HostBuf() = default;
    HostBuf(const HostBuf &) = delete;
    HostBuf &operator=(const HostBuf &) = delete;
    HostBuf(HostBuf &&o) noexcept : p(o.p), cap(o.cap)
    {
        o.p = nullptr;
        o.cap = 0;
    }
    HostBuf &operator=(HostBuf &&o) noexcept
    {
        std::swap(p, o.p);
        std::swap(cap, o.cap);
        return *this;
    }
    ~HostBuf()
    {
        if (p)
            (void)hipHostFree(p);
    }
    bool ensure(size_t bytes)
    {
        if (bytes <= cap && p)
            return true;
        const size_t cap0 = p ? cap : 0;
        if (p)
            (void)hipHostFree(p);
        p = nullptr;
        cap = 0;
        size_t b = grow_capacity(cap0, bytes);
        if (hipHostMalloc(&p, b, hipHostMallocDefault) != hipSuccess) {
            // The headroom may not fit where the exact size does.
            const size_t e = grow_capacity(0, bytes);
            p = nullptr;
            if (e >= b || hipHostMalloc(&p, e, hipHostMallocDefault) != hipSuccess) {
                p = nullptr;
                return false;
            }
            b = e;
        }
        cap = b;
        return true;
    }
    template <typename T>
    T *as() const
    {
        return static_cast<T *>(p);
    }
};

// ---------------------------------------------------------------------------
// error helpers
// ---------------------------------------------------------------------------
#define HIP_TRY(expr)                                                              \
    do {                                                                           \
        hipError_t e_ = (expr);                                                    \
        if (e_ != hipSuccess) {                                                    \
            err = std::string(#expr) + ": " + hipGetErrorString(e_);               \
            return RPP_E_DEVICE;                                                   \
        }                                                                          \
    } while (0)

#define ALLOC_TRY(buf, bytes)                                                      \
    do {                                                                           \
        if (!(buf).ensure(bytes)) {                                                \
            err = alloc_failure_text(buf, (size_t)(bytes));                        \
            return RPP_E_NOMEM;                                                    \
        }                                                                          \
    } while (0)

inline std::string alloc_failure_text(const DevBuf &b, size_t bytes)
{
    if (b.pool && b.pool->arena)
        return "caller workspace too small: " + std::to_string(bytes) + " more bytes needed with " +
               std::to_string(b.pool->arena_size - b.pool->arena_top) + " of " +
               std::to_string(b.pool->arena_size) + " left";
    if (b.pool && b.pool->exhausted)
        return "device memory limit of " + std::to_string(b.pool->limit) +
               " bytes reached (allocation of " + std::to_string(bytes) + " bytes)";
    return "allocation of " + std::to_string(bytes) + " bytes failed";
}

template <typename B>
inline std::string alloc_failure_text(const B &, size_t bytes)
{
    return "allocation of " + std::to_string(bytes) + " bytes failed";
}

struct GpuTimer {
    hipEvent_t a = nullptr, b = nullptr;
    hipStream_t s;
    explicit GpuTimer(hipStream_t st) : s(st)
    {
        (void)hipEventCreate(&a);
        (void)hipEventCreate(&b);
    }
    ~GpuTimer()
    {
        if (a)
            (void)hipEventDestroy(a);
        if (b)
            (void)hipEventDestroy(b);
    }
    void start() { (void)hipEventRecord(a, s); }
    void stop() { (void)hipEventRecord(b, s); }
    float ms()
    {
        float m = 0.0f;
        (void)hipEventSynchronize(b);
        (void)hipEventElapsedTime(&m, a, b);
        return m;
    }
};

// Distances as the host sees them: the n x n matrix, or, on the sparse
// path, packed neighbour rows -- bits (n x words u64: the neighbours of each
// vertex), npre (n x words u32: position in nbd of each word's first
// neighbour) and nbd (the neighbours' distances, row after row, ascending).
// Packed rows answer only for pairs within the threshold, which is every
// pair a simplex within the threshold has.
struct HostDist {
    const float *dsq = nullptr;
    int n = 0;
    const uint64_t *bits = nullptr;
    const uint32_t *npre = nullptr;
    const float *nbd = nullptr;
    int words = 0;
    float operator()(int a, int b) const
    {
        if (!nbd)
            return dsq[(size_t)a * n + b];
        if (a == b)
            return 0.0f;
        const size_t k = (size_t)a * words + (size_t)(b >> 6);
        return nbd[npre[k] + (uint32_t)__builtin_popcountll(bits[k] & ((1ull << (b & 63)) - 1))];
    }
};

// npre of packed rows from their bitsets: per vertex, a running count of
// neighbours over the words (out: n * words entries).
inline void packed_row_prefix(const uint64_t *bits, int n, int words, uint32_t *out)
{
    uint32_t run = 0;
    for (size_t k = 0; k < (size_t)n * words; ++k) {
        out[k] = run;
        run += (uint32_t)__builtin_popcountll(bits[k]);
    }
}

// Longest edge of the q-simplex c (cidx), the one of largest edge cidx
// among equally long edges.
inline uint64_t critical_edge(const HostDist &D, const uint64_t *binom, uint64_t c, int q)
{
    const int n = D.n;
    int v[8];
    int hi = n;
    for (int pos = 0; pos <= q; ++pos) {
        const int k = q + 1 - pos;
        int lo = k - 1, h = hi - 1;
        while (lo < h) {
            const int mid = (lo + h + 1) >> 1;
            if (binom[(size_t)k * (n + 1) + mid] <= c)
                lo = mid;
            else
                h = mid - 1;
        }
        v[pos] = lo;
        c -= binom[(size_t)k * (n + 1) + lo];
        hi = lo;
    }
    float best = -1.0f;
    uint64_t be = UINT64_MAX;
    for (int i = 0; i <= q; ++i)
        for (int j = i + 1; j <= q; ++j) {
            const float e = D(v[i], v[j]);
            const uint64_t ec = (uint64_t)v[i] * (v[i] - 1) / 2 + (uint64_t)v[j];  // v[i] > v[j]
            if (e > best || (e == best && ec > be)) {
                best = e;
                be = ec;
            }
        }
    return be;
}

inline uint64_t critical_edge(const float *dsq, int n, const uint64_t *binom, uint64_t c, int q)
{
    HostDist D;
    D.dsq = dsq;
    D.n = n;
    return critical_edge(D, binom, c, q);
}

inline int bit_length(uint64_t x)
{
    return x ? 64 - __builtin_clzll(x) : 0;
}


}  // namespace rpp
