// residual.cpp -- host reduction of the columns the GPU could not pair.
//
// Paper, "Reduction Matrix vs. Oblivious Matrix Reduction" (both techniques,
// Algorithm 2 for the oblivious one) and "Core System Optimizations"
// (two-layer pair store).  Columns arrive in coboundary order together with
// their lows (oldest cofacets), computed on the GPU.  A column whose low is
// not yet a pivot is paired at once, with no coboundary built (its
// unreduced column is already reduced: the emergent shortcut).  Otherwise
// its coboundary is regenerated from the distance matrix (implicit matrix
// reduction) as a stream of keys, oldest first; a column is a 4-ary min-heap
// over the fronts of the streams it has summed, so the heap top is its low;
// Z/2 addition adds the other column's streams, and equal entries cancel in
// pairs when the low is taken.
#include "residual.h"

#include <immintrin.h>
#include <sched.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <cstring>
#include <atomic>
#include <type_traits>
#include <condition_variable>
#include <functional>
#include <chrono>
#include <cmath>
#include <memory>
#include <new>
#include <stdexcept>
#include <mutex>
#include <thread>

namespace rpp {

namespace {

struct Entry {
    float diam;
    uint64_t cidx;
};

// Column entries are packed into one unsigned integer whose order is the
// filtration order of the cofacets: the diameter's bit pattern (monotone for
// non-negative floats) above (M - cidx), so a smaller key is older -- smaller
// diameter, then larger cidx.  K = uint64_t when every cofacet index fits in
// 32 bits, unsigned __int128 otherwise.
using u128 = unsigned __int128;
template <class K> struct KeyFmt;
template <> struct KeyFmt<uint64_t> {
    static constexpr int S = 32;
    static constexpr uint64_t M = 0xffffffffull;
};
template <> struct KeyFmt<u128> {
    static constexpr int S = 64;
    static constexpr uint64_t M = ~0ull;
};
// How a key is laid out: the diameter above an index field of `shift`
// bits holding (mask - cidx).  By default the diameter is its float bit
// pattern and the field is 32 or 64 bits wide (KeyFmt).  With rank-coded
// diameters (integer ranks held as floats) the rank itself is stored and
// the field is only as wide as the largest cofacet index needs, so 64-bit
// keys cover indices past 2^32.
struct KeyCodec {
    int shift = 32;
    uint64_t mask = 0xffffffffull;
    bool rank = false;
};
template <class K> inline KeyCodec default_codec()
{
    KeyCodec kc;
    kc.shift = KeyFmt<K>::S;
    kc.mask = KeyFmt<K>::M;
    return kc;
}
template <class K> inline K pack_key(const KeyCodec &kc, float d, uint64_t c)
{
    const uint32_t hi = kc.rank ? (uint32_t)d : __builtin_bit_cast(uint32_t, d);
    return ((K)hi << kc.shift) | (K)(kc.mask - c);
}
template <class K> inline Entry unpack_key(const KeyCodec &kc, K k)
{
    const uint32_t hi = (uint32_t)(k >> kc.shift);
    return Entry{kc.rank ? (float)hi : __builtin_bit_cast(float, hi),
                 kc.mask - (uint64_t)(k & (K)kc.mask)};
}

// Moves the c smallest of a[0..m) (distinct keys) to a[0..c), unordered:
// quickselect with a median-of-three pivot and a branch-free Lomuto
// partition (every element is swapped; the split index advances on the
// comparison result), which keeps the mispredictions of a comparison-driven
// partition out of the loop.
template <class K> void select_smallest(K *a, size_t m, size_t c)
{
    size_t lo = 0, hi = m;
    while (hi - lo > 24) {
        const size_t mid = lo + (hi - lo) / 2;
        K x = a[lo], y = a[mid], z = a[hi - 1];
        if (x > y)
            std::swap(x, y);
        if (y > z)
            y = z > x ? z : x;  // median of three
        // distinct keys and a median pivot: both sides are non-empty
        size_t j = lo;
        for (size_t i = lo; i < hi; ++i) {
            const K t = a[i];
            const bool lt = t < y;
            a[i] = a[j];
            a[j] = t;
            j += lt ? 1 : 0;
        }
        if (c < j)
            hi = j;
        else if (c > j)
            lo = j;
        else
            return;
    }
    std::sort(a + lo, a + hi);
}

// AVX-512 (F, VL, BW, VBMI2), checked once at load; the vector routines
// below are chosen at run time.
static bool cpu_has_avx512()
{
    return __builtin_cpu_supports("avx512f") && __builtin_cpu_supports("avx512vl") &&
           __builtin_cpu_supports("avx512bw") && __builtin_cpu_supports("avx512vbmi2");
}
static const bool HAVE_AVX512 = cpu_has_avx512();

// Index of the smallest of a[0..m) (distinct keys below 2^64 - 1): eight
// running minima with their indices, then a reduction.
__attribute__((target("avx512f"))) static size_t argmin_u64_avx512(const uint64_t *a, size_t m)
{
    const __m512i ones = _mm512_set1_epi64(-1);
    __m512i best = ones, bidx = _mm512_setzero_si512();
    __m512i idx = _mm512_set_epi64(7, 6, 5, 4, 3, 2, 1, 0);
    const __m512i step = _mm512_set1_epi64(8);
    size_t i = 0;
    for (; i + 8 <= m; i += 8) {
        const __m512i v = _mm512_loadu_si512(a + i);
        const __mmask8 lt = _mm512_cmplt_epu64_mask(v, best);
        best = _mm512_mask_mov_epi64(best, lt, v);
        bidx = _mm512_mask_mov_epi64(bidx, lt, idx);
        idx = _mm512_add_epi64(idx, step);
    }
    if (i < m) {
        const __mmask8 lm = (__mmask8)((1u << (m - i)) - 1u);
        const __m512i v = _mm512_mask_loadu_epi64(ones, lm, a + i);
        const __mmask8 lt = _mm512_mask_cmplt_epu64_mask(lm, v, best);
        best = _mm512_mask_mov_epi64(best, lt, v);
        bidx = _mm512_mask_mov_epi64(bidx, lt, idx);
    }
    const uint64_t mn = _mm512_reduce_min_epu64(best);
    const __mmask8 at = _mm512_cmpeq_epu64_mask(best, _mm512_set1_epi64((long long)mn));
    alignas(64) uint64_t ix[8];
    _mm512_store_si512(ix, bidx);
    return (size_t)ix[__builtin_ctz((unsigned)at)];
}

// Splits a[0..m) (u64 keys) into the keys <= y, moved to the front in
// order of appearance, and the others behind them; returns the count of the
// first group.  Eight keys per step: each group is compressed in registers
// and stored whole -- the low group in place (its write position never
// passes the read position, so only consumed slots are overwritten), the
// high group into tmp (m + 8 slots), copied back at the end.
__attribute__((target("avx512f"))) static size_t partition_le_u64_avx512(uint64_t *a, size_t m,
                                                                         uint64_t y,
                                                                         uint64_t *tmp)
{
    const __m512i vy = _mm512_set1_epi64((long long)y);
    size_t nl = 0, ng = 0, i = 0;
    for (; i + 8 <= m; i += 8) {
        const __m512i v = _mm512_loadu_si512(a + i);
        const __mmask8 le = _mm512_cmple_epu64_mask(v, vy);
        _mm512_storeu_si512(a + nl, _mm512_maskz_compress_epi64(le, v));
        _mm512_storeu_si512(tmp + ng, _mm512_maskz_compress_epi64((__mmask8)~le, v));
        const size_t k = (size_t)__builtin_popcount((unsigned)le);
        nl += k;
        ng += 8 - k;
    }
    for (; i < m; ++i) {
        const uint64_t x = a[i];
        if (x <= y)
            a[nl++] = x;
        else
            tmp[ng++] = x;
    }
    memcpy(a + nl, tmp, ng * sizeof(uint64_t));
    return nl;
}

// select_smallest for u64 keys with the vector partition: the pivot is the
// sample key nearest the target rank among 15 spread over the range, so a
// pass usually lands close to c and few passes follow.
static void select_smallest_u64_avx512(uint64_t *a, size_t m, size_t c)
{
    thread_local std::vector<uint64_t> tmp;
    if (tmp.size() < m + 8)
        tmp.resize(m + 8);
    size_t lo = 0, hi = m;
    while (hi - lo > 48) {
        const size_t len = hi - lo;
        uint64_t smp[15];
        for (int k = 0; k < 15; ++k)
            smp[k] = a[lo + (len * (2 * k + 1)) / 30];
        std::sort(smp, smp + 15);
        size_t q = ((c - lo) * 15) / len;
        q = q > 14 ? 14 : q;
        const uint64_t y = smp[q];
        size_t j = lo + partition_le_u64_avx512(a + lo, len, y, tmp.data());
        if (j == hi)  // y is the largest key of the range: set it apart
            j = lo + partition_le_u64_avx512(a + lo, len, y - 1, tmp.data());
        if (c < j)
            hi = j;
        else if (c > j)
            lo = j;
        else
            return;
    }
    std::sort(a + lo, a + hi);
}

// Index of the smallest of a[0..m), m >= 1.
template <class K> static inline size_t argmin_keys(const K *a, size_t m)
{
    if (std::is_same<K, uint64_t>::value && HAVE_AVX512)
        return argmin_u64_avx512(reinterpret_cast<const uint64_t *>(a), m);
    size_t b = 0;
    K best = a[0];
    for (size_t i = 1; i < m; ++i) {
        const K x = a[i];
        const bool lt = x < best;
        best = lt ? x : best;
        b = lt ? i : b;
    }
    return b;
}

// Stream storage.  Streams are bump-allocated from blocks that a reduction
// hands back to a process-wide pool when it ends, so a warm process neither
// calls malloc per stream nor writes to fresh pages: the first touch of a
// fresh page costs more than computing the coboundary written to it.
class BlockPool {
public:
    static constexpr size_t BLOCK = (size_t)4 << 20;     // bytes
    static constexpr size_t KEEP = (size_t)1 << 30;      // pooled bytes kept at most
    static BlockPool &get()
    {
        static BlockPool pool;
        return pool;
    }
    char *take()
    {
        {
            std::lock_guard<std::mutex> lk(mu_);
            if (!free_.empty()) {
                char *b = free_.back();
                free_.pop_back();
                return b;
            }
        }
        return static_cast<char *>(::operator new(BLOCK, std::align_val_t(64)));
    }
    void give(char *b)
    {
        {
            std::lock_guard<std::mutex> lk(mu_);
            if ((free_.size() + 1) * BLOCK <= KEEP) {
                free_.push_back(b);
                return;
            }
        }
        ::operator delete(b, std::align_val_t(64));
    }

private:
    BlockPool() = default;
    ~BlockPool()
    {
        for (char *b : free_)
            ::operator delete(b, std::align_val_t(64));
    }
    std::mutex mu_;
    std::vector<char *> free_;
};

// Blocks of a reduction that are in use; returned to the pool together.
struct BlockSink {
    std::mutex mu;
    std::vector<std::pair<char *, size_t>> blocks;  // size BLOCK: pooled
    ~BlockSink()
    {
        for (auto &b : blocks) {
            if (b.second == BlockPool::BLOCK)
                BlockPool::get().give(b.first);
            else
                ::operator delete(b.first, std::align_val_t(64));
        }
    }
};

// A bump allocator for one thread; its blocks go to the sink when it ends
// (the streams written into them live as long as the reduction).
class Arena {
public:
    explicit Arena(BlockSink *sink) : sink_(sink) {}
    Arena(const Arena &) = delete;
    Arena &operator=(const Arena &) = delete;
    ~Arena()
    {
        if (mine_.empty())
            return;
        std::lock_guard<std::mutex> lk(sink_->mu);
        sink_->blocks.insert(sink_->blocks.end(), mine_.begin(), mine_.end());
    }
    // Room for `count` keys; commit() takes what was used of it.
    template <class K> K *reserve(size_t count)
    {
        const size_t bytes = (count * sizeof(K) + 63) & ~(size_t)63;
        if (used_ + bytes > cap_) {
            if (bytes > BlockPool::BLOCK) {
                char *b = static_cast<char *>(::operator new(bytes, std::align_val_t(64)));
                mine_.push_back({b, bytes});
                cur_ = b;
                cap_ = bytes;
            } else {
                cur_ = BlockPool::get().take();
                mine_.push_back({cur_, BlockPool::BLOCK});
                cap_ = BlockPool::BLOCK;
            }
            used_ = 0;
        }
        return reinterpret_cast<K *>(cur_ + used_);
    }
    template <class K> void commit(size_t count)
    {
        used_ += (count * sizeof(K) + 63) & ~(size_t)63;
    }
    // Takes back the last commit (its keys stay readable until the next
    // reserve).
    template <class K> void uncommit(size_t count)
    {
        used_ -= (count * sizeof(K) + 63) & ~(size_t)63;
    }

private:
    BlockSink *sink_;
    std::vector<std::pair<char *, size_t>> mine_;
    char *cur_ = nullptr;
    size_t used_ = 0, cap_ = 0;
};

// One added coboundary, consumed oldest-first.  Only a sorted prefix is
// kept: the oldest `chunk` remaining keys are selected (linear on average)
// and sorted; when they run out the next, twice as large, chunk is
// selected.  A column's low usually lies a few dozen entries into each
// stream, so most keys are never ordered, and pops read memory in order.
template <class K> struct Stream {
    static constexpr int SINGLES = 8;  // keys taken one at a time before chunks
    K *e = nullptr;  // arena storage
    uint32_t len = 0, pos = 0, sorted = 0, chunk = 32;
    int singles = 0;
    bool empty() const { return pos >= len; }
    K front() const { return e[pos]; }
    // hot: order a first chunk now, while the keys are in cache, instead of
    // taking single keys later (each later scan reads the whole stream again)
    void prepare(bool hot, uint32_t ordered)
    {
        pos = 0;
        singles = hot ? SINGLES : 0;
        chunk = 32;
        sorted = ordered;  // an ordered prefix: nothing to do for it
        // a deep consumer with a short ordered prefix gets its first chunk
        // now, while the keys are in cache
        if (ordered == 0 || (hot && ordered < 32 && ordered < len))
            extend(ordered);
    }
    void refill() { extend(pos); }
    // Orders keys from `at` (= sorted): the next one alone, or a chunk.
    void extend(size_t at)
    {
        const size_t rem = len - at;
        if (rem == 0)
            return;
        if (singles < SINGLES && rem > 16) {
            // the next key alone, by a scan for the minimum: most streams
            // are consumed only a few keys deep
            const size_t j = at + argmin_keys(e + at, rem);
            std::swap(e[at], e[j]);
            sorted = (uint32_t)at + 1;
            ++singles;
            return;
        }
        const size_t c = std::min<size_t>(rem, chunk);
        if (c < rem) {
            if (std::is_same<K, uint64_t>::value && HAVE_AVX512)
                select_smallest_u64_avx512(reinterpret_cast<uint64_t *>(e + at), rem, c);
            else
                select_smallest(e + at, rem, c);
        }
        std::sort(e + at, e + at + c);
        sorted = (uint32_t)(at + c);
        chunk = chunk < (1u << 30) ? chunk * 2 : chunk;
    }
    void pop()
    {
        if (++pos == sorted)
            refill();
    }
};

// Whether new streams should be ordered up front (a dimension whose columns
// cancel deeply) or one key at a time (most streams are consumed only a few
// keys deep).  Decided by the share of this reduction's streams consumed
// past the single-key phase; before 64 streams are seen, by the dimension
// (edges' coboundaries cancel deeply, higher ones rarely).
struct DepthPolicy {
    std::atomic<uint64_t> streams{0}, deep{0};
    bool prior = false;
    bool hot() const
    {
        const uint64_t s = streams.load(std::memory_order_relaxed);
        if (s < 64)
            return prior;
        return deep.load(std::memory_order_relaxed) * 4 > s;
    }
};

// Hash map from cofacet indices (never ~0) to column positions: open
// addressing with linear probing over a power-of-two table, backward-shift
// deletion.  One flat array instead of a node per entry (the exact phase
// inserts a pivot for every nonzero column: 787k on the dimension-3
// sphere).
class FlatMap {
public:
    explicit FlatMap(size_t expected)
    {
        size_t c = 16;
        while (c < 2 * expected + 16)
            c *= 2;
        keys_.assign(c, EMPTY);
        vals_.resize(c);
        mask_ = c - 1;
    }
    // The value of key k, or nullptr.
    int64_t *find(uint64_t k)
    {
        for (size_t i = home(k);; i = (i + 1) & mask_) {
            if (keys_[i] == k)
                return &vals_[i];
            if (keys_[i] == EMPTY)
                return nullptr;
        }
    }
    // Inserts (k, v) unless k is present; the value slot and whether it was
    // inserted.
    std::pair<int64_t *, bool> emplace(uint64_t k, int64_t v)
    {
        if (2 * (size_ + 1) > keys_.size())
            grow();
        for (size_t i = home(k);; i = (i + 1) & mask_) {
            if (keys_[i] == k)
                return {&vals_[i], false};
            if (keys_[i] == EMPTY) {
                keys_[i] = k;
                vals_[i] = v;
                ++size_;
                return {&vals_[i], true};
            }
        }
    }
    void erase(uint64_t k)
    {
        size_t i = home(k);
        while (keys_[i] != k) {
            if (keys_[i] == EMPTY)
                return;
            i = (i + 1) & mask_;
        }
        // shift back the entries of the cluster that may fill the hole
        for (size_t j = (i + 1) & mask_; keys_[j] != EMPTY; j = (j + 1) & mask_) {
            const size_t h = home(keys_[j]);
            if (((j - h) & mask_) >= ((j - i) & mask_)) {
                keys_[i] = keys_[j];
                vals_[i] = vals_[j];
                i = j;
            }
        }
        keys_[i] = EMPTY;
        --size_;
    }

private:
    static constexpr uint64_t EMPTY = ~0ull;
    size_t home(uint64_t k) const
    {
        k ^= k >> 33;  // a 64-bit mixer (the MurmurHash3 finaliser)
        k *= 0xff51afd7ed558ccdull;
        k ^= k >> 33;
        k *= 0xc4ceb9fe1a85ec53ull;
        k ^= k >> 33;
        return (size_t)k & mask_;
    }
    void grow()
    {
        std::vector<uint64_t> ok;
        std::vector<int64_t> ov;
        ok.swap(keys_);
        ov.swap(vals_);
        keys_.assign(ok.size() * 2, EMPTY);
        vals_.resize(ok.size() * 2);
        mask_ = keys_.size() - 1;
        size_ = 0;
        for (size_t i = 0; i < ok.size(); ++i)
            if (ok[i] != EMPTY)
                emplace(ok[i], ov[i]);
    }
    std::vector<uint64_t> keys_;
    std::vector<int64_t> vals_;
    size_t mask_ = 0, size_ = 0;
};

// Radix heap over keys that never fall below the last minimum taken (the
// low of a column only grows as the reduction adds columns whose low is
// the current one).  Keys are read in 4-bit digits.  Bucket 0 holds copies
// of that minimum; a key that first differs from it in digit L, where its
// own digit is g, sits in bucket 1 + 16 L + g, and every key of a bucket
// is smaller than every key of a later one.  Taking the next minimum
// empties the lowest non-empty bucket into lower ones (a key moves at most
// once per digit, every move a sequential append) -- or, once that bucket
// is small, sorts it into the front run: distinct keys (pairs cancelled),
// in order, all below every bucket.  The low is then the run's first key,
// and a new key within the run's range is toggled into it in place.
template <class K> struct RadixHeap {
    static constexpr int DB = 4, DIG = 1 << DB;
    static constexpr int NB = 8 * (int)sizeof(K) / DB * DIG + 1;
    static constexpr size_t RUN = 48;  // largest bucket sorted into the run
    std::vector<K> b[NB];
    uint64_t busy[(NB + 63) / 64] = {};  // bit i: bucket i is not empty
    std::vector<K> run;                  // front run: run[rh..] ascending
    size_t rh = 0;
    K last = 0;
    int bucket(K k) const
    {
        const K x = k ^ last;
        if (x == 0)
            return 0;
        int hb;  // highest differing bit
        if (sizeof(K) == 8) {
            hb = 63 - __builtin_clzll((uint64_t)x);
        } else {
            const uint64_t hi = (uint64_t)(x >> 32 >> 32);
            hb = hi ? 127 - __builtin_clzll(hi) : 63 - __builtin_clzll((uint64_t)x);
        }
        const int L = hb / DB;
        return 1 + L * DIG + (int)((k >> (L * DB)) & (K)(DIG - 1));
    }
    void put(K k)
    {
        const int i = bucket(k);
        b[i].push_back(k);
        busy[i >> 6] |= 1ull << (i & 63);
    }
    void drop(int i)
    {
        b[i].clear();
        busy[i >> 6] &= ~(1ull << (i & 63));
    }
    // Lowest non-empty bucket above 0, or NB.
    int first_above_zero() const
    {
        for (int w = 0; w < (NB + 63) / 64; ++w) {
            const uint64_t m = w == 0 ? busy[0] & ~1ull : busy[w];
            if (m)
                return 64 * w + __builtin_ctzll(m);
        }
        return NB;
    }
    bool run_empty() const { return rh == run.size(); }
    // Z/2 add of k to the run (k within its range): removes an equal key,
    // else inserts k in order.
    void toggle(K k)
    {
        K *f = run.data() + rh, *e = run.data() + run.size();
        K *at = std::lower_bound(f, e, k);
        if (*at == k) {
            if (at == f) {
                ++rh;
            } else {
                std::move(at + 1, e, at);
                run.pop_back();
            }
            return;
        }
        if (rh > 0 && at - f < e - at) {
            std::move(f, at, f - 1);  // room in front: shift the lower part
            --rh;
            *(at - 1) = k;
        } else {
            const size_t pos = (size_t)(at - run.data());
            run.insert(run.begin() + (ptrdiff_t)pos, k);
        }
    }
    void add(K k)
    {
        if (!run_empty() && k <= run.back())
            toggle(k);
        else
            put(k);
    }
    // Adds keys; one below the last minimum (an addition whose low is older
    // than the column's) re-buckets everything around it.
    void push(const K *e, size_t len)
    {
        if (len == 0)
            return;
        K m = e[0];
        for (size_t i = 1; i < len; ++i)
            m = e[i] < m ? e[i] : m;
        if (m < last)
            rebase(m);
        for (size_t i = 0; i < len; ++i)
            add(e[i]);
    }
    // Adds every key of another heap (none lies below its last minimum).
    void merge(const RadixHeap &o)
    {
        if (o.size() == 0)
            return;
        if (o.last < last)
            rebase(o.last);
        o.for_each([&](K k) { add(k); });
    }
    void rebase(K m)
    {
        std::vector<K> all(run.begin() + (ptrdiff_t)rh, run.end());
        run.clear();
        rh = 0;
        for (int i = 0; i < NB; ++i) {
            all.insert(all.end(), b[i].begin(), b[i].end());
            drop(i);
        }
        last = m;
        for (K k : all)
            put(k);
    }
    // The smallest key present an odd number of times (the low of the Z/2
    // sum); false when every key cancels.
    bool low(K &out)
    {
        while (true) {
            if (!run_empty()) {
                out = run[rh];
                return true;
            }
            if (!b[0].empty()) {
                if (b[0].size() & 1) {
                    b[0].resize(1);
                    out = last;
                    return true;
                }
                drop(0);
            }
            const int i = first_above_zero();
            if (i == NB)
                return false;
            std::vector<K> &v = b[i];
            K m = v[0];
            for (K k : v)
                m = k < m ? k : m;
            last = m;
            if (v.size() <= RUN) {
                // sort, keep the keys of odd multiplicity
                std::sort(v.begin(), v.end());
                run.clear();
                rh = 0;
                for (size_t j = 0; j < v.size();) {
                    size_t e = j + 1;
                    while (e < v.size() && v[e] == v[j])
                        ++e;
                    if ((e - j) & 1)
                        run.push_back(v[j]);
                    j = e;
                }
                drop(i);
                continue;
            }
            for (K k : v)
                put(k);  // lands below i
            drop(i);
        }
    }
    // Keys just above the low, usually the next lows: up to w of the run
    // behind it, then, when the run holds fewer, the lowest bucket if it
    // holds at most bmax keys (unordered; out has room for w + bmax).
    size_t ahead(K *out, size_t w, size_t bmax) const
    {
        size_t c = 0;
        for (size_t j = rh + 1; j < run.size() && c < w; ++j)
            out[c++] = run[j];
        if (c < w) {
            const int i = first_above_zero();
            if (i < NB && b[i].size() <= bmax)
                for (K k : b[i])
                    out[c++] = k;
        }
        return c;
    }
    template <class F> void for_each(F f) const
    {
        for (size_t j = rh; j < run.size(); ++j)
            f(run[j]);
        for (int i = 0; i < NB; ++i)
            for (K k : b[i])
                f(k);
    }
    size_t size() const
    {
        size_t n = run.size() - rh;
        for (int i = 0; i < NB; ++i)
            n += b[i].size();
        return n;
    }
};

// Bucket queue over the keys' top bits, for the same long columns: slot
// (k - base) >> s of a power-of-two table laid over the keys present when
// it is (re)built (with room for the range to double), keys beyond it in an
// overflow list that becomes the next table once the front reaches the
// end.  A slot's keys sit unordered in 14-key chunks until the front
// reaches it; then they are sorted (pairs cancel) into the front run.  Keys
// at or below the run's last key are merged into it, a step's keys at once.
// With diameter ranks in the top bits (the sphere's chain) a slot is about
// one rank, so each key is moved once and sorted once, where the radix heap
// refiles it level by level.
template <class K> struct SlotHeap {
    static constexpr int CK = 14;
    struct Chunk {
        uint32_t next, cnt;
        K k[CK];
    };
    std::vector<Chunk> pool;
    uint32_t free_head = 0;       // 1-based chunk index, 0: none
    std::vector<uint32_t> head;   // newest chunk of each slot, 1-based
    std::vector<uint64_t> occ;    // bit per non-empty slot
    std::vector<uint64_t> occ2;   // bit per non-zero occ word
    uint32_t ns = 0;              // slots
    K base = 0;
    int s = 0;
    uint32_t cur = 0;             // slots below cur are empty
    bool laid = false;
    std::vector<K> over;          // keys beyond the table
    std::vector<K> run;           // front run: run[rh..] ascending
    size_t rh = 0;
    size_t nslot = 0;             // keys in slots
    std::vector<K> batch, run2, tmp;

    static int bitlen(K x)
    {
        if (sizeof(K) > 8) {
            const uint64_t hi = (uint64_t)(x >> 32 >> 32);
            if (hi)
                return 128 - __builtin_clzll(hi);
        }
        const uint64_t lo = (uint64_t)x;
        return lo ? 64 - __builtin_clzll(lo) : 0;
    }
    uint32_t new_chunk()
    {
        if (free_head) {
            const uint32_t c = free_head;
            free_head = pool[c - 1].next;
            return c;
        }
        pool.emplace_back();
        return (uint32_t)pool.size();
    }
    void mark(uint32_t i)
    {
        occ[i >> 6] |= 1ull << (i & 63);
        occ2[i >> 12] |= 1ull << ((i >> 6) & 63);
    }
    void unmark(uint32_t i)
    {
        occ[i >> 6] &= ~(1ull << (i & 63));
        if (!occ[i >> 6])
            occ2[i >> 12] &= ~(1ull << ((i >> 6) & 63));
    }
    void put_slot(uint32_t i, K k)
    {
        uint32_t c = head[i];
        if (!c || pool[c - 1].cnt == CK) {
            const uint32_t nc = new_chunk();
            pool[nc - 1].next = c;
            pool[nc - 1].cnt = 0;
            head[i] = nc;
            if (!c)
                mark(i);
            c = nc;
        }
        Chunk &ch = pool[c - 1];
        ch.k[ch.cnt++] = k;
        ++nslot;
    }
    bool run_empty() const { return rh == run.size(); }
    // Z/2 add of one key at or below the run's end.
    void toggle(K k)
    {
        K *f = run.data() + rh, *e = run.data() + run.size();
        K *at = std::lower_bound(f, e, k);
        if (at != e && *at == k) {
            if (at == f) {
                ++rh;
            } else {
                std::move(at + 1, e, at);
                run.pop_back();
            }
            return;
        }
        if (rh > 0 && at - f < e - at) {
            std::move(f, at, f - 1);
            --rh;
            *(at - 1) = k;
        } else {
            run.insert(run.begin() + (at - run.data()), k);
        }
    }
    // A key above the run's end (or the run empty).
    void put(K k)
    {
        if (!laid) {
            over.push_back(k);
            return;
        }
        if (k < base) {  // below the table: the run holds the smallest keys
            if (run_empty()) {
                run.clear();
                rh = 0;
                run.push_back(k);
            } else {
                toggle(k);
            }
            return;
        }
        const K off = (K)(k - base) >> s;
        if (off >= (K)ns) {
            over.push_back(k);
            return;
        }
        const uint32_t i = (uint32_t)off;
        if (i < cur)
            cur = i;
        put_slot(i, k);
    }
    void push(const K *e, size_t len)
    {
        if (run_empty()) {
            for (size_t i = 0; i < len; ++i)
                put(e[i]);
            return;
        }
        const K rb = run.back();
        batch.clear();
        for (size_t i = 0; i < len; ++i) {
            if (e[i] <= rb)
                batch.push_back(e[i]);
            else
                put(e[i]);
        }
        if (batch.size() <= 4) {
            for (K k : batch)
                toggle(k);
            return;
        }
        std::sort(batch.begin(), batch.end());
        // Z/2 merge of the run and the batch
        run2.clear();
        size_t a = rh, b = 0;
        const size_t ae = run.size(), be = batch.size();
        while (a < ae && b < be) {
            const K x = run[a], y = batch[b];
            if (x < y) {
                run2.push_back(x);
                ++a;
                continue;
            }
            size_t q = b + 1;
            while (q < be && batch[q] == y)
                ++q;
            const bool odd = (q - b) & 1;
            if (y < x) {
                if (odd)
                    run2.push_back(y);
            } else {
                if (!odd)
                    run2.push_back(x);
                ++a;
            }
            b = q;
        }
        run2.insert(run2.end(), run.begin() + (ptrdiff_t)a, run.end());
        while (b < be) {
            const K y = batch[b];
            size_t q = b + 1;
            while (q < be && batch[q] == y)
                ++q;
            if ((q - b) & 1)
                run2.push_back(y);
            b = q;
        }
        run.swap(run2);
        rh = 0;
    }
    // Lays a table over the overflow keys (every slot empty).
    void rebuild()
    {
        K m = over[0], M = over[0];
        for (K k : over) {
            m = k < m ? k : m;
            M = k > M ? k : M;
        }
        int sb = 8;  // log2 of the slots: about twice the keys, 256 to 2^17
        while (sb < 17 && ((size_t)1 << sb) < 2 * over.size())
            ++sb;
        if (ns != (1u << sb)) {
            ns = 1u << sb;
            head.assign(ns, 0);
            occ.assign(ns / 64, 0);
            occ2.assign((ns / 64 + 63) / 64, 0);
        }
        base = m;
        laid = true;
        const int bl = bitlen((K)(M - m));
        s = bl > sb - 1 ? bl - (sb - 1) : 0;  // the range fills half the table
        cur = 0;
        tmp.swap(over);
        over.clear();
        for (K k : tmp)
            put(k);
        tmp.clear();
    }
    // First occupied slot at or above cur, or ns.
    uint32_t next_slot() const
    {
        const uint32_t nw = ns / 64;
        uint32_t w = cur >> 6;
        if (w >= nw)
            return ns;
        const uint64_t m = occ[w] & (~0ull << (cur & 63));
        if (m)
            return (w << 6) | (uint32_t)__builtin_ctzll(m);
        ++w;
        if (w >= nw)
            return ns;
        uint32_t w2 = w >> 6;
        uint64_t m2 = occ2[w2] & (~0ull << (w & 63));
        while (!m2) {
            if (++w2 >= (uint32_t)occ2.size())
                return ns;
            m2 = occ2[w2];
        }
        w = (w2 << 6) | (uint32_t)__builtin_ctzll(m2);
        return (w << 6) | (uint32_t)__builtin_ctzll(occ[w]);
    }
    // Slot i's keys into out (appended); the slot becomes empty.
    void take_slot(uint32_t i, std::vector<K> &out)
    {
        for (uint32_t c = head[i]; c;) {
            Chunk &ch = pool[c - 1];
            out.insert(out.end(), ch.k, ch.k + ch.cnt);
            nslot -= ch.cnt;
            const uint32_t nx = ch.next;
            ch.next = free_head;
            free_head = c;
            c = nx;
        }
        head[i] = 0;
        unmark(i);
    }
    bool low(K &out)
    {
        while (true) {
            if (!run_empty()) {
                out = run[rh];
                return true;
            }
            if (!laid) {
                if (over.empty())
                    return false;
                rebuild();
                continue;
            }
            const uint32_t i = next_slot();
            if (i == ns) {
                if (over.empty())
                    return false;
                rebuild();
                continue;
            }
            cur = i;
            tmp.clear();
            take_slot(i, tmp);
            std::sort(tmp.begin(), tmp.end());
            run.clear();
            rh = 0;
            for (size_t j = 0; j < tmp.size();) {
                size_t e = j + 1;
                while (e < tmp.size() && tmp[e] == tmp[j])
                    ++e;
                if ((e - j) & 1)
                    run.push_back(tmp[j]);
                j = e;
            }
        }
    }
    size_t ahead(K *out, size_t w, size_t bmax) const
    {
        size_t c = 0;
        for (size_t j = rh + 1; j < run.size() && c < w; ++j)
            out[c++] = run[j];
        if (c < w && laid) {
            const uint32_t i = next_slot();
            if (i < ns) {
                size_t cnt = 0;
                for (uint32_t ch = head[i]; ch; ch = pool[ch - 1].next)
                    cnt += pool[ch - 1].cnt;
                if (cnt <= bmax)
                    for (uint32_t ch = head[i]; ch; ch = pool[ch - 1].next)
                        for (uint32_t q = 0; q < pool[ch - 1].cnt; ++q)
                            out[c++] = pool[ch - 1].k[q];
            }
        }
        return c;
    }
    template <class F> void for_each(F f) const
    {
        for (size_t j = rh; j < run.size(); ++j)
            f(run[j]);
        for (uint32_t i = 0; i < ns; ++i)
            for (uint32_t ch = head[i]; ch; ch = pool[ch - 1].next)
                for (uint32_t q = 0; q < pool[ch - 1].cnt; ++q)
                    f(pool[ch - 1].k[q]);
        for (K k : over)
            f(k);
    }
    size_t size() const { return run.size() - rh + nslot + over.size(); }
};

// The ordered store of a long column: the bucket queue above, or with
// RPP_SLOT_HEAP=0 the radix heap (on the 4096-point sphere's chain the
// queue's lows take 9.7 ms against the radix heap's 21.8).
template <class K> struct FrontHeap {
    static bool slots_wanted()
    {
        static const bool v = [] {
            const char *e = getenv("RPP_SLOT_HEAP");
            return !e || atoi(e) != 0;
        }();
        return v;
    }
    std::unique_ptr<RadixHeap<K>> r;
    std::unique_ptr<SlotHeap<K>> q;
    explicit FrontHeap(K last)
    {
        if (slots_wanted()) {
            q.reset(new SlotHeap<K>());
        } else {
            r.reset(new RadixHeap<K>());
            r->last = last;
        }
    }
    void push(const K *e, size_t len) { r ? r->push(e, len) : q->push(e, len); }
    void merge(const FrontHeap &o)
    {
        if (r && o.r) {
            r->merge(*o.r);
            return;
        }
        std::vector<K> all;
        all.reserve(o.size());
        o.for_each([&](K k) { all.push_back(k); });
        if (!all.empty())
            push(all.data(), all.size());
    }
    bool low(K &out) { return r ? r->low(out) : q->low(out); }
    size_t size() const { return r ? r->size() : q->size(); }
    size_t ahead(K *out, size_t w, size_t bmax) const
    {
        return r ? r->ahead(out, w, bmax) : q->ahead(out, w, bmax);
    }
    template <class F> void for_each(F f) const
    {
        if (r)
            r->for_each(f);
        else
            q->for_each(f);
    }
};

// Working column = Z/2 sum of several coboundaries.  Each added coboundary
// is its own stream; a min-heap over the streams' current fronts yields the
// sum's entries oldest-first.  Only the entries that reach the front are
// ever ordered, which is what finding the low needs.  A column that has
// taken many additions (an essential class is a long chain of them, each
// key eventually reaching the front) moves every remaining key into a
// radix heap instead: the 4-ary heap over thousands of streams costs a
// cache miss per level per key, the radix heap appends.
template <class K> class Column {
public:
    DepthPolicy *policy = nullptr;  // shared by the columns of one reduction
    const KeyCodec *codec = nullptr;  // key layout of that reduction
    // RPP_RADIX_STREAMS set: every column goes radix at that many streams,
    // whatever share of its keys has been taken (tests)
    static bool radix_forced()
    {
        static const bool v = getenv("RPP_RADIX_STREAMS") != nullptr;
        return v;
    }
    static size_t radix_at()
    {
        static const size_t v = [] {
            const char *e = getenv("RPP_RADIX_STREAMS");
            const long x = e ? atol(e) : 512;
            return x > 0 ? (size_t)x : ~(size_t)0;  // <= 0: never
        }();
        return v;
    }
    // Adds the coboundary in e[0..len) (arena storage) as a new stream; its
    // first `ties` keys are already in ascending order.
    void push_stream(K *e, size_t len, size_t ties)
    {
        if (len == 0)
            return;
        if (rh) {
            rh->push(e, len);
            return;
        }
        streams.emplace_back();
        Stream<K> &st = streams.back();
        st.e = e;
        st.len = (uint32_t)len;
        st.prepare(policy && policy->hot(), (uint32_t)ties);
        if (policy)
            policy->streams.fetch_add(1, std::memory_order_relaxed);
        top_push(st.front(), (uint32_t)(streams.size() - 1));
        maybe_radix();
    }
    // Add another column's current contents: its streams hold exactly its
    // Z/2 sum (cancelled pairs were removed together).  The remaining keys
    // are copied, since both columns reorder their streams as they go.
    void add(const Column &o, Arena &arena)
    {
        if (o.rh && !rh)
            to_radix();  // a stream holds distinct keys; the other's buckets
                         // may still hold pairs that have not cancelled
        if (rh) {
            if (o.rh) {
                rh->merge(*o.rh);
                return;
            }
            for (const Stream<K> &src : o.streams)
                if (!src.empty())
                    rh->push(src.e + src.pos, src.len - src.pos);
            return;
        }
        for (const Stream<K> &src : o.streams) {
            if (src.empty())
                continue;
            const size_t rem = src.len - src.pos;
            K *e = arena.reserve<K>(rem);
            memcpy(e, src.e + src.pos, rem * sizeof(K));
            arena.commit<K>(rem);
            streams.emplace_back();
            Stream<K> &dst = streams.back();
            dst.e = e;
            dst.len = (uint32_t)rem;
            dst.pos = 0;
            dst.sorted = src.sorted - src.pos;
            dst.chunk = src.chunk;
            top_push(dst.front(), (uint32_t)(streams.size() - 1));
        }
        maybe_radix();
    }
    // Low of the sum over Z/2: keys present in an even number of streams
    // cancel.  In the min-heap every copy of the minimum lies in a subtree
    // containing the root, so a second copy exists iff a child of the root
    // holds it; pairs are dropped until the minimum is unique.
    bool low(Entry &out)
    {
        if (rh) {
            K k;
            if (!rh->low(k))
                return false;
            out = unpack_key<K>(*codec, k);
            return true;
        }
        while (!hk.empty()) {
            const K e = hk[0];
            const size_t m = hk.size();
            const size_t e4 = m < 5 ? m : 5;
            bool dup = false;
            for (size_t j = 1; j < e4; ++j)
                dup |= hk[j] == e;
            if (!dup) {
                out = unpack_key<K>(*codec, e);
                return true;
            }
            advance_root();  // the other copy becomes the root
            advance_root();
        }
        return false;
    }

    // Keys still held (what adding this column copies), and the length of
    // its first stream (its own coboundary), 0 once it went radix.
    size_t remaining() const
    {
        if (rh)
            return rh->size();
        size_t r = 0;
        for (const Stream<K> &st : streams)
            r += st.len - st.pos;
        return r;
    }
    size_t first_len() const { return rh || streams.empty() ? 0 : streams[0].len; }
    bool radix() const { return (bool)rh; }
    // Radix columns: keys just above the low (RadixHeap::ahead); 0 otherwise.
    size_t ahead(K *out, size_t w, size_t bmax) const { return rh ? rh->ahead(out, w, bmax) : 0; }

private:
    // At radix_at() streams, and each doubling after: go radix when an
    // eighth of the keys added so far have already reached the front (the
    // sphere's essential chain: a fifth at 512 streams, and in the end all
    // of them), not when the streams are long and mostly untouched (dense
    // coboundaries and edges' coboundaries, 1-4% taken).
    void maybe_radix()
    {
        if (streams.size() < next_check)
            return;
        next_check = streams.size() >= (~(size_t)0 >> 1) ? ~(size_t)0 : 2 * streams.size();
        uint64_t taken = 0, total = 0;
        for (const Stream<K> &st : streams) {
            taken += st.pos;
            total += st.len;
        }
        if (radix_forced() || 8 * taken >= total)
            to_radix();
    }
    // Every remaining key of every stream into a radix heap based at the
    // current minimum (each stream's unordered rest lies above its ordered
    // prefix, so the heap root is the smallest key present).
    void to_radix()
    {
        rh.reset(new FrontHeap<K>(hk.empty() ? K(0) : hk[0]));
        for (const Stream<K> &st : streams)
            if (!st.empty())
                rh->push(st.e + st.pos, st.len - st.pos);
        streams.clear();
        streams.shrink_to_fit();
        hk.clear();
        hk.shrink_to_fit();
        hs.clear();
        hs.shrink_to_fit();
    }
    // 4-ary min-heap, keys and stream ids in separate arrays: half the
    // levels of a binary heap, a node's four child keys share a cache line,
    // and the smallest child is picked without branches.
    void sift_down(size_t i)
    {
        const K x = hk[i];
        const uint32_t xs = hs[i];
        const size_t m = hk.size();
        while (true) {
            const size_t c = 4 * i + 1;
            if (c >= m)
                break;
            size_t best = c;
            K bk = hk[c];
            const size_t e = c + 4 < m ? c + 4 : m;
            for (size_t j = c + 1; j < e; ++j) {
                const K v = hk[j];
                const bool lt = v < bk;
                bk = lt ? v : bk;
                best = lt ? j : best;
            }
            if (!(bk < x))
                break;
            hk[i] = bk;
            hs[i] = hs[best];
            i = best;
        }
        hk[i] = x;
        hs[i] = xs;
    }
    void top_push(K k, uint32_t s)
    {
        hk.push_back(k);
        hs.push_back(s);
        size_t i = hk.size() - 1;
        while (i > 0) {
            const size_t par = (i - 1) / 4;
            if (!(k < hk[par]))
                break;
            hk[i] = hk[par];
            hs[i] = hs[par];
            i = par;
        }
        hk[i] = k;
        hs[i] = s;
    }
    // Consume the root's entry from its stream and restore the heap.
    void advance_root()
    {
        Stream<K> &st = streams[hs[0]];
        st.pop();
        if (st.pos == Stream<K>::SINGLES && policy)
            policy->deep.fetch_add(1, std::memory_order_relaxed);
        if (!st.empty()) {
            hk[0] = st.front();
        } else {
            hk[0] = hk.back();
            hs[0] = hs.back();
            hk.pop_back();
            hs.pop_back();
            if (hk.empty())
                return;
        }
        sift_down(0);
    }
    std::vector<Stream<K>> streams;
    std::vector<K> hk;
    std::vector<uint32_t> hs;
    std::unique_ptr<FrontHeap<K>> rh;  // set once the column goes radix
    size_t next_check = radix_at();    // stream count of the next radix check
};

// ---------------------------------------------------------------------------
// AVX-512 variants (chosen at run time when the CPU has F, VL, BW and VBMI2)
// ---------------------------------------------------------------------------

// Bit reversal of a byte (lane order of an 8-lane mask).
static const struct RevTable {
    uint8_t t[256];
    RevTable()
    {
        for (int x = 0; x < 256; ++x) {
            int r = 0;
            for (int b = 0; b < 8; ++b)
                r |= ((x >> b) & 1) << (7 - b);
            t[x] = (uint8_t)r;
        }
    }
} REV8;

// Dense coboundary with 32-bit cofacet indices (u64 keys): 16 candidate
// vertices per step -- row maxima, the threshold test, the packed keys --
// and register compresses of the cofacets that pass (the memory form of
// compress is slow on some cores).  The vertices w run downward (each gap
// between sigma's vertices from its top, the gaps from the top), so the
// cofacets whose diameter is d itself -- sigma's own -- come out in
// ascending key order (for a fixed diameter the key falls as w rises);
// they go to out[0..ties), the others (larger diameters, unordered) to gt
// and then behind them.  out and gt need 16 slots of slack.
__attribute__((target("avx512f,avx512vl,avx512bw,avx512vbmi2"))) static size_t
cob_dense_u64_avx512(const float *const *rows, int nv, const int *v, uint64_t sigma, float d,
                     float thr, const uint64_t *binom, int n, uint64_t *out, uint64_t *gt,
                     size_t *ties)
{
    size_t neq = 0, ngt = 0;
    uint64_t above = 0, below = sigma;
    int hi = n;
    const __m512 vd = _mm512_set1_ps(d), vthr = _mm512_set1_ps(thr);
    const __m512i vM = _mm512_set1_epi64((long long)0xffffffffull);
    const __m512i rev = _mm512_set_epi64(0, 1, 2, 3, 4, 5, 6, 7);
    for (int idx = 0; idx <= nv; ++idx) {
        const int lo = idx < nv ? v[idx] : -1;
        const int j = nv - idx;  // vertices of sigma below w
        const uint64_t *Cj = binom + (int64_t)(j + 1) * (n + 1);
        const __m512i vbase = _mm512_set1_epi64((long long)(above + below));
        for (int top = hi - 1; top > lo; top -= 16) {
            const int w0 = top - 15 > lo + 1 ? top - 15 : lo + 1;  // lowest w of the step
            const int cnt = top - w0 + 1;
            const __mmask16 lm = cnt >= 16 ? (__mmask16)0xffff : (__mmask16)((1u << cnt) - 1u);
            __m512 mx = _mm512_maskz_loadu_ps(lm, rows[0] + w0);
            for (int i = 1; i < nv; ++i)
                mx = _mm512_max_ps(mx, _mm512_maskz_loadu_ps(lm, rows[i] + w0));
            const __mmask16 in = _mm512_mask_cmp_ps_mask(lm, mx, vthr, _CMP_LE_OQ);
            const __mmask16 eq = _mm512_mask_cmp_ps_mask(in, mx, vd, _CMP_LE_OQ);
            const __mmask16 up = in & (__mmask16)~eq;
            const __m512i ndb = _mm512_castps_si512(_mm512_max_ps(mx, vd));
            const __m512i c0 =
                _mm512_add_epi64(vbase, _mm512_maskz_loadu_epi64((__mmask8)lm, Cj + w0));
            const __m512i c1 =
                _mm512_add_epi64(vbase, _mm512_maskz_loadu_epi64((__mmask8)(lm >> 8), Cj + w0 + 8));
            const __m512i d0 = _mm512_cvtepu32_epi64(_mm512_castsi512_si256(ndb));
            const __m512i d1 = _mm512_cvtepu32_epi64(_mm512_extracti64x4_epi64(ndb, 1));
            const __m512i k0 = _mm512_or_si512(_mm512_slli_epi64(d0, 32), _mm512_sub_epi64(vM, c0));
            const __m512i k1 = _mm512_or_si512(_mm512_slli_epi64(d1, 32), _mm512_sub_epi64(vM, c1));
            // ties in descending w: upper half first, each half lane-reversed
            const __mmask8 e1 = (__mmask8)REV8.t[(uint8_t)(eq >> 8)];
            const __mmask8 e0 = (__mmask8)REV8.t[(uint8_t)eq];
            _mm512_storeu_si512(out + neq,
                                _mm512_maskz_compress_epi64(e1, _mm512_permutexvar_epi64(rev, k1)));
            neq += (size_t)__builtin_popcount((unsigned)e1);
            _mm512_storeu_si512(out + neq,
                                _mm512_maskz_compress_epi64(e0, _mm512_permutexvar_epi64(rev, k0)));
            neq += (size_t)__builtin_popcount((unsigned)e0);
            const __mmask8 u0 = (__mmask8)up, u1 = (__mmask8)(up >> 8);
            _mm512_storeu_si512(gt + ngt, _mm512_maskz_compress_epi64(u0, k0));
            ngt += (size_t)__builtin_popcount((unsigned)u0);
            _mm512_storeu_si512(gt + ngt, _mm512_maskz_compress_epi64(u1, k1));
            ngt += (size_t)__builtin_popcount((unsigned)u1);
        }
        if (idx < nv) {
            const int r = nv - 1 - idx;  // rank of v[idx] from the bottom
            below -= binom[(int64_t)(r + 1) * (n + 1) + lo];
            above += binom[(int64_t)(r + 2) * (n + 1) + lo];
        }
        hi = lo;
    }
    memcpy(out + neq, gt, ngt * sizeof(uint64_t));
    *ties = neq;
    return neq + ngt;
}

struct Ctx {
    const ResidualProblem &P;
    int n, p;
    mutable Arena arena;  // this thread's stream storage
    KeyCodec kc;          // key layout
    Ctx(const ResidualProblem &pp, BlockSink *sink, const KeyCodec &codec)
        : P(pp), n(pp.n), p(pp.p), arena(sink), kc(codec)
    {
    }

    uint64_t C(int v, int k) const { return P.binom[(int64_t)k * (n + 1) + v]; }
    float D(int a, int b) const
    {
        if (!P.nbd)
            return P.dsq[(int64_t)a * n + b];
        if (a == b)
            return 0.0f;
        const int64_t k = (int64_t)a * P.words + (b >> 6);
        return P.nbd[P.npre[k] + (uint32_t)__builtin_popcountll(P.bits[k] &
                                                                 ((1ull << (b & 63)) - 1))];
    }

    // vertices of a simplex with q+1 vertices, decreasing
    // Vertex v[pos] is the largest v < (the previous one) with C(v, k) <= c,
    // k = q + 1 - pos.  Started from the real root of v^k / k! = c (exact
    // for k <= 2 up to rounding) and stepped to the exact answer on the
    // binomial table, so the guess's accuracy only affects the steps taken.
    void decode(uint64_t c, int q, int *v) const
    {
        int hi = n;
        for (int pos = 0; pos <= q; ++pos) {
            const int k = q + 1 - pos;
            const int lo = k - 1;
            double x;
            if (k == 1)
                x = (double)c;
            else if (k == 2)
                x = 0.5 * (1.0 + std::sqrt(1.0 + 8.0 * (double)c));
            else if (k == 3)
                x = std::cbrt(6.0 * (double)c) + 1.0;
            else
                x = std::pow((double)c * factorial(k), 1.0 / k) + 0.5 * (k - 1);
            int g = x >= (double)(hi - 1) ? hi - 1 : (x <= (double)lo ? lo : (int)x);
            while (g > lo && C(g, k) > c)
                --g;
            while (g + 1 < hi && C(g + 1, k) <= c)
                ++g;
            v[pos] = g;
            c -= C(g, k);
            hi = g;
        }
    }
    static double factorial(int k)
    {
        double f = 1.0;
        for (int i = 2; i <= k; ++i)
            f *= i;
        return f;
    }

    // cidx of sigma + {w} (w not in sigma, v decreasing)
    uint64_t insert_index(const int *v, int w) const
    {
        uint64_t c = 0;
        int r = 0;
        bool placed = false;
        for (int i = p; i >= 0; --i) {
            if (!placed && w < v[i]) {
                c += C(w, r + 1);
                ++r;
                placed = true;
            }
            c += C(v[i], r + 1);
            ++r;
        }
        if (!placed)
            c += C(w, r + 1);
        return c;
    }

    // Sparse coboundary from the neighbour bitsets and packed neighbour rows
    // (sigma's NV vertices ascending in u): the common neighbours w are
    // listed first, word by word without a branch per neighbour (up to four
    // per word, the rarer rest in a loop), then each gets its diameter and
    // key in a loop of known length.  w ascends, so the cofacets of sigma's
    // own diameter come out in descending key order and are reversed; the
    // others follow them.  Returns the count; out needs n + 16 slots.
    template <class K, int NV>
    size_t cob_packed(const int *u, float d, const uint64_t *base, K *out, size_t &ties) const
    {
        const int W = P.words;
        const uint64_t *bv[NV];
        const uint32_t *pre[NV];
        for (int i = 0; i < NV; ++i) {
            bv[i] = P.bits + (int64_t)u[i] * W;
            pre[i] = P.npre + (int64_t)u[i] * W;
        }
        int *ws = w_scratch();
        int cnt = 0;
        for (int wd = 0; wd < W; ++wd) {
            uint64_t m = bv[0][wd];
            for (int i = 1; i < NV; ++i)
                m &= bv[i][wd];
            const int w0 = wd << 6;
            for (int t = 0; t < 4; ++t) {
                ws[cnt] = w0 + (m ? __builtin_ctzll(m) : 0);
                cnt += m ? 1 : 0;
                m &= m - 1;
            }
            while (m) {
                ws[cnt++] = w0 + __builtin_ctzll(m);
                m &= m - 1;
            }
        }
        K *gt = gt_scratch<K>();
        size_t neq = 0, ngt = 0;
        int k = 0;  // vertices of sigma below w
        for (int t = 0; t < cnt; ++t) {
            const int w = ws[t];
            while (k < NV && u[k] < w)
                ++k;
            const int wd = w >> 6;
            const uint64_t below = (1ull << (w & 63)) - 1;
            float nd = d;
            for (int i = 0; i < NV; ++i) {
                const float e = P.nbd[pre[i][wd] + (uint32_t)__builtin_popcountll(bv[i][wd] & below)];
                nd = e > nd ? e : nd;
            }
            const K key = pack_key<K>(kc, nd, base[k] + C(w, k + 1));
            out[neq] = key;
            gt[ngt] = key;
            const bool tie = !(nd > d);
            neq += tie ? 1 : 0;
            ngt += tie ? 0 : 1;
        }
        std::reverse(out, out + neq);
        memcpy(out + neq, gt, ngt * sizeof(K));
        ties = neq;
        return neq + ngt;
    }
    // Scratch for the common neighbours of one coboundary, n + 64 ints.
    int *w_scratch() const
    {
        thread_local std::vector<int> buf;
        if (buf.size() < (size_t)n + 64)
            buf.resize((size_t)n + 64);
        return buf.data();
    }

    // Adds sigma's coboundary to col as a new stream.
    template <class K> void add_coboundary(Column<K> &col, uint64_t sigma, float d) const
    {
        K *e;
        size_t ties = 0;
        const size_t len = coboundary<K>(sigma, d, e, ties);
        col.push_stream(e, len, ties);
    }

    // Every cofacet of sigma with diameter <= threshold, appended to out as
    // packed keys.
    // Scratch for the cofacets above sigma's diameter (reordered behind the
    // ties), n + 16 keys.
    template <class K> K *gt_scratch() const
    {
        thread_local std::vector<u128> buf;
        const size_t need = ((size_t)n + 16) * sizeof(K) / sizeof(u128) + 1;
        if (buf.size() < need)
            buf.resize(need);
        return reinterpret_cast<K *>(buf.data());
    }

    // Writes sigma's coboundary into this thread's arena; returns its length.
    // The first `ties` keys are the cofacets of sigma's own diameter, in
    // ascending order; the rest are larger and unordered.
    template <class K> size_t coboundary(uint64_t sigma, float d, K *&out, size_t &ties) const
    {
        int v[8];
        decode(sigma, p, v);
        if (P.bits) {
            // common neighbours only: every new edge is within the threshold.
            // w runs upward; with sigma's vertices ascending u_0 < ... < u_p
            // and k of them below w, cidx(sigma + {w}) = base[k] + C(w, k+1),
            // where base[k] = sum_{i<k} C(u_i, i+1) + sum_{i>=k} C(u_i, i+2).
            const int nv = p + 1;
            int u[8];
            for (int i = 0; i < nv; ++i)
                u[i] = v[p - i];
            uint64_t base[9];
            for (int k = 0; k <= nv; ++k) {
                uint64_t b = 0;
                for (int i = 0; i < nv; ++i)
                    b += i < k ? C(u[i], i + 1) : C(u[i], i + 2);
                base[k] = b;
            }
            if (P.nbd && nv >= 2 && nv <= 4) {
                out = arena.reserve<K>((size_t)n + 16);
                size_t cnt = 0;
                switch (nv) {
                case 2: cnt = cob_packed<K, 2>(u, d, base, out, ties); break;
                case 3: cnt = cob_packed<K, 3>(u, d, base, out, ties); break;
                default: cnt = cob_packed<K, 4>(u, d, base, out, ties); break;
                }
                arena.commit<K>(cnt);
                return cnt;
            }
            const float *rows[8];
            for (int i = 0; i < nv; ++i)
                rows[i] = P.nbd ? nullptr : P.dsq + (int64_t)v[i] * n;
            const uint64_t *brow[8];  // C(., k+1) for each gap k
            for (int k = 0; k <= nv; ++k)
                brow[k] = P.binom + (int64_t)(k + 1) * (n + 1);
            const uint64_t *bv[8];
            for (int i = 0; i < nv; ++i)
                bv[i] = P.bits + (int64_t)v[i] * P.words;
            // room for every other vertex; the arena keeps only what is used
            out = arena.reserve<K>((size_t)n + 16);
            K *gt = gt_scratch<K>();
            size_t neq = 0, ngt = 0;
            int k = nv;  // vertices of sigma below w; w runs downward
            for (int wd = P.words - 1; wd >= 0; --wd) {
                uint64_t m = bv[0][wd];
                for (int i = 1; i < nv; ++i)
                    m &= bv[i][wd];
                // packed rows: each vertex's distances of this word's
                // neighbours start at its prefix position
                const float *nrow[8];
                if (P.nbd && m)
                    for (int i = 0; i < nv; ++i)
                        nrow[i] = P.nbd + P.npre[(int64_t)v[i] * P.words + wd];
                while (m) {
                    const int b = 63 - __builtin_clzll(m);
                    m &= ~(1ull << b);
                    const int w = wd * 64 + b;
                    while (k > 0 && u[k - 1] > w)
                        --k;
                    float nd = d;
                    if (P.nbd) {
                        const uint64_t below = (1ull << b) - 1;
                        for (int i = 0; i < nv; ++i) {
                            const float e = nrow[i][__builtin_popcountll(bv[i][wd] & below)];
                            nd = e > nd ? e : nd;
                        }
                    } else {
                        for (int i = 0; i < nv; ++i) {
                            const float e = rows[i][w];
                            nd = e > nd ? e : nd;
                        }
                    }
                    const K key = pack_key<K>(kc, nd, base[k] + brow[k][w]);
                    out[neq] = key;
                    gt[ngt] = key;
                    const bool tie = !(nd > d);
                    neq += tie ? 1 : 0;
                    ngt += tie ? 0 : 1;
                }
            }
            memcpy(out + neq, gt, ngt * sizeof(K));
            ties = neq;
            const size_t cnt = neq + ngt;
            arena.commit<K>(cnt);
            return cnt;
        }
        const float *rows[8];
        for (int i = 0; i <= p; ++i)
            rows[i] = P.dsq + (int64_t)v[i] * n;
        out = arena.reserve<K>((size_t)n + 16);  // 16 slots of slack for vector stores
        K *gt = gt_scratch<K>();
        size_t cnt;
        if (std::is_same<K, uint64_t>::value && HAVE_AVX512 && !kc.rank && kc.shift == 32) {
            cnt = cob_dense_u64_avx512(rows, p + 1, v, sigma, d, P.thr, P.binom, n,
                                       reinterpret_cast<uint64_t *>(out),
                                       reinterpret_cast<uint64_t *>(gt), &ties);
        } else {
            switch (p) {
            case 1: cnt = cob_dense<K, 2>(rows, v, sigma, d, out, gt, ties); break;
            case 2: cnt = cob_dense<K, 3>(rows, v, sigma, d, out, gt, ties); break;
            case 3: cnt = cob_dense<K, 4>(rows, v, sigma, d, out, gt, ties); break;
            default: cnt = cob_dense<K, 0>(rows, v, sigma, d, out, gt, ties); break;
            }
        }
        arena.commit<K>(cnt);
        return cnt;
    }

    // Dense coboundary: cidx of sigma + {w} = above + C(w, j+1) + below,
    // where the vertices of sigma above w move up one rank.  Between two
    // consecutive vertices of sigma, j, above and below are constant, so w
    // runs over each gap in a tight loop that writes every cofacet and
    // advances an output only for those within the threshold: w runs
    // downward, so the cofacets of sigma's own diameter reach out[0..ties)
    // in ascending key order; the others go to gt, then behind them.
    template <class K, int NV>
    size_t cob_dense(const float *const *rows, const int *v, uint64_t sigma, float d, K *out,
                     K *gt, size_t &ties) const
    {
        const int nv = NV ? NV : p + 1;
        const float thr = P.thr;
        size_t neq = 0, ngt = 0;
        uint64_t above = 0, below = sigma;
        int hi = n;
        for (int idx = 0; idx <= nv; ++idx) {
            const int lo = idx < nv ? v[idx] : -1;
            const int j = nv - idx;  // vertices of sigma below w
            const uint64_t *Cj = P.binom + (int64_t)(j + 1) * (n + 1);
            const uint64_t base = above + below;
            for (int w = hi - 1; w > lo; --w) {
                float mx = rows[0][w];
                for (int i = 1; i < nv; ++i) {
                    const float e = rows[i][w];
                    mx = e > mx ? e : mx;
                }
                const float nd = mx > d ? mx : d;
                const K key = pack_key<K>(kc, nd, base + Cj[w]);
                out[neq] = key;
                gt[ngt] = key;
                neq += (mx <= d) ? 1 : 0;
                ngt += (mx > d && mx <= thr) ? 1 : 0;
            }
            if (idx < nv) {
                const int r = nv - 1 - idx;  // rank of v[idx] from the bottom
                below -= C(lo, r + 1);
                above += C(lo, r + 2);
            }
            hi = lo;
        }
        memcpy(out + neq, gt, ngt * sizeof(K));
        ties = neq;
        return neq + ngt;
    }

    // Implicit second layer: if row tau (diameter dt) is the pivot of an
    // apparent column, return that column.  The column can only be tau's
    // youngest facet: among the facets of full diameter dt, the one of
    // smallest cidx, i.e. tau minus its largest vertex u whose removal keeps
    // the diameter.  (sigma*, tau) is apparent iff tau is sigma*'s oldest
    // cofacet: no w > u outside tau has d(w, s) <= dt for all s in sigma*.
    bool apparent_partner(uint64_t tau, float dt, uint64_t *sigma_out) const
    {
        int t[9];
        decode(tau, p + 1, t);
        int ui = -1;
        for (int i = 0; i <= p + 1 && ui < 0; ++i) {
            float fd = 0.0f;
            for (int a = 0; a <= p + 1; ++a) {
                if (a == i)
                    continue;
                for (int b = a + 1; b <= p + 1; ++b)
                    if (b != i) {
                        const float e = D(t[a], t[b]);
                        fd = e > fd ? e : fd;
                    }
            }
            if (fd == dt)
                ui = i;
        }
        if (ui < 0)
            return false;
        const int u = t[ui];
        int s[8], q = 0;
        for (int i = 0; i <= p + 1; ++i)
            if (i != ui)
                s[q++] = t[i];
        if (P.bits) {
            // candidates: common neighbours of sigma* above u
            for (int k = P.words - 1; k >= 0 && k * 64 + 63 > u; --k) {
                uint64_t m = ~0ull;
                for (int i = 0; i <= p; ++i)
                    m &= P.bits[(int64_t)s[i] * P.words + k];
                if (!m)
                    continue;
                // packed rows: this word's distances of each vertex
                const float *nrow[8];
                uint64_t nb[8];
                if (P.nbd)
                    for (int i = 0; i <= p; ++i) {
                        const int64_t x = (int64_t)s[i] * P.words + k;
                        nrow[i] = P.nbd + P.npre[x];
                        nb[i] = P.bits[x];
                    }
                for (; m; m &= m - 1) {
                    const int b = __builtin_ctzll(m);
                    const int w = k * 64 + b;
                    if (w <= u)
                        continue;
                    bool all = true;
                    if (P.nbd) {
                        const uint64_t below = (1ull << b) - 1;
                        for (int i = 0; i <= p && all; ++i)
                            all = nrow[i][__builtin_popcountll(nb[i] & below)] <= dt;
                    } else {
                        for (int i = 0; i <= p && all; ++i)
                            all = P.dsq[(int64_t)s[i] * n + w] <= dt;
                    }
                    if (all)
                        return false;
                }
            }
            uint64_t c = 0;
            for (int i = 0; i <= p; ++i)
                c += C(s[i], p + 1 - i);
            *sigma_out = c;
            return true;
        }
        int nxt = 0;  // next vertex of tau at or below w (tau is decreasing)
        for (int w = n - 1; w > u; --w) {
            if (nxt <= p + 1 && t[nxt] == w) {
                ++nxt;
                continue;
            }
            bool all = true;
            for (int i = 0; i <= p && all; ++i)
                all = P.dsq[(int64_t)s[i] * n + w] <= dt;
            if (all)
                return false;
        }
        uint64_t c = 0;
        for (int i = 0; i <= p; ++i)
            c += C(s[i], p + 1 - i);
        *sigma_out = c;
        return true;
    }
};

// ---------------------------------------------------------------------------
// A small persistent worker pool, shared by every caller in the process.
// ---------------------------------------------------------------------------
// A job is a function that claims its work items dynamically (an atomic
// counter) and returns once none is left, so any number of threads may run
// it at once, and a thread that joins after the last item was claimed just
// returns.  Several callers (the serving slots, the exact phase of one
// dimension next to the speculative phase of the next) may run jobs at the
// same time: each idle worker joins the open job with the fewest threads, so
// the workers are shared out instead of going to whoever came first.
class Pool {
public:
    static Pool &get()
    {
        static Pool pool;
        return pool;
    }
    int size() const { return (int)workers_.size() + 1; }
    // Runs fn(tid) on the calling thread (tid 0) and on the workers that
    // join, and returns when every thread that entered fn has left it.
    void run(const std::function<void(int)> &fn)
    {
        if (workers_.empty()) {
            fn(0);
            return;
        }
        Job job;
        job.fn = &fn;
        {
            std::lock_guard<std::mutex> lk(mu_);
            open_.push_back(&job);
        }
        cv_.notify_all();
        fn(0);
        std::unique_lock<std::mutex> lk(mu_);
        close_locked(&job);
        done_.wait(lk, [&] { return job.active == 0; });
    }

private:
    struct Job {
        const std::function<void(int)> *fn = nullptr;
        int active = 0;  // threads inside fn, the caller excluded
    };

public:
    // A job the caller does not take part in: launch() offers fn(tid) to the
    // workers (those idle join), join() closes it and waits until every
    // thread that entered fn has left it.
    class Async {
        friend class Pool;
        Job job;
        std::function<void(int)> fn;
    };
    void launch(Async &a, std::function<void(int)> fn)
    {
        a.fn = std::move(fn);
        a.job.fn = &a.fn;
        if (workers_.empty())
            return;
        {
            std::lock_guard<std::mutex> lk(mu_);
            open_.push_back(&a.job);
        }
        cv_.notify_all();
    }
    void join(Async &a)
    {
        std::unique_lock<std::mutex> lk(mu_);
        close_locked(&a.job);
        done_.wait(lk, [&] { return a.job.active == 0; });
    }

private:
    // Threads: the CPUs this process may use (affinity mask, and the
    // cgroup CPU quota when one is set), less one for the thread that
    // enqueues GPU work while the pool is busy, at most 16.
    static int usable_cpus()
    {
        int n = (int)std::thread::hardware_concurrency();
        cpu_set_t set;
        if (sched_getaffinity(0, sizeof(set), &set) == 0)
            n = std::min(n > 0 ? n : CPU_COUNT(&set), CPU_COUNT(&set));
        if (FILE *f = fopen("/sys/fs/cgroup/cpu.max", "r")) {
            char quota[32] = {0};
            long period = 0;
            if (fscanf(f, "%31s %ld", quota, &period) == 2 && strcmp(quota, "max") != 0 &&
                period > 0) {
                const long q = atol(quota);
                if (q > 0)
                    n = std::min(n, (int)std::max(1L, q / period));
            }
            fclose(f);
        } else if (FILE *fq = fopen("/sys/fs/cgroup/cpu/cpu.cfs_quota_us", "r")) {
            long q = -1, period = 0;
            if (fscanf(fq, "%ld", &q) != 1)
                q = -1;
            fclose(fq);
            if (FILE *fp = fopen("/sys/fs/cgroup/cpu/cpu.cfs_period_us", "r")) {
                if (fscanf(fp, "%ld", &period) != 1)
                    period = 0;
                fclose(fp);
            }
            if (q > 0 && period > 0)
                n = std::min(n, (int)std::max(1L, q / period));
        }
        return std::max(1, n);
    }
    Pool()
    {
        int n = std::min(usable_cpus() - 1, 16);
        if (const char *e = getenv("RPP_HOST_THREADS"))
            n = atoi(e);
        n = std::max(1, std::min(n, 64));
        for (int t = 1; t < n; ++t)
            workers_.emplace_back([this, t] { loop(t); });
    }
    ~Pool()
    {
        {
            std::lock_guard<std::mutex> lk(mu_);
            stop_ = true;
        }
        cv_.notify_all();
        for (auto &w : workers_)
            w.join();
    }
    // A job whose items are all claimed takes no new threads.
    void close_locked(Job *j)
    {
        auto it = std::find(open_.begin(), open_.end(), j);
        if (it != open_.end())
            open_.erase(it);
    }
    void loop(int tid)
    {
        std::unique_lock<std::mutex> lk(mu_);
        while (true) {
            cv_.wait(lk, [&] { return stop_ || !open_.empty(); });
            if (stop_)
                return;
            Job *j = open_[0];
            for (Job *o : open_)
                if (o->active < j->active)
                    j = o;
            ++j->active;
            lk.unlock();
            (*j->fn)(tid);
            lk.lock();
            // fn returned: every item is claimed, so nobody else should join
            close_locked(j);
            if (--j->active == 0)
                done_.notify_all();
        }
    }
    std::vector<std::thread> workers_;
    std::mutex mu_;
    std::condition_variable cv_, done_;
    std::vector<Job *> open_;
    bool stop_ = false;
};

// Look-ahead for one long column, a chain of additions whose every step
// waits on the previous one's low (the essential class of a sphere: ~19,000
// additions, almost all of them apparent partners).  Such a column's next
// lows are usually among the keys just above its current low, so helper
// threads take those keys as they appear, find their apparent partners and
// generate the partners' coboundaries ahead of the column's thread, which
// uses a result when its low has one and otherwise computes as before.
// Both sides compute the same pure function of the key, so the additions
// are the ones the column would make alone.  64-bit keys only.
//
// Requests: a ring of keys written by the column's thread only; a helper
// that falls behind skips the oldest (a skipped key is computed by the
// column's thread if it becomes a low).  Results: direct-mapped slots under
// a sequence lock (odd while a helper writes one), every field a relaxed
// atomic; the reader copies a slot and keeps it only if the sequence number
// did not move meanwhile.
struct ChainAssist {
    static constexpr size_t RING = 256;
    static constexpr size_t NSLOT = 64;
    static constexpr size_t CAP = 256;  // longest coboundary handed over
    static constexpr uint64_t NOT_APPARENT = ~0ull;
    struct alignas(64) Slot {
        std::atomic<uint32_t> seq{0};
        std::atomic<uint64_t> tau{~0ull};
        std::atomic<uint64_t> sigma{0};
        std::atomic<uint32_t> len{0}, ties{0};
        std::atomic<uint64_t> keys[CAP];
    };
    // written by the column's thread (one store of head per step)
    alignas(64) std::atomic<uint64_t> ring[RING];
    alignas(64) std::atomic<uint64_t> head{0};
    // written by the helpers, on lines of their own
    alignas(64) std::atomic<uint64_t> claim{0};
    std::atomic<uint64_t> finished{0};  // requests answered or skipped
    std::atomic<int> helping{0};         // helpers inside help()
    alignas(64) std::atomic<bool> stop{false};
    std::unique_ptr<Slot[]> slots{new Slot[NSLOT]};
    uint64_t asked[256];  // the column thread's recent requests

    ChainAssist()
    {
        for (auto &r : ring)
            r.store(0, std::memory_order_relaxed);
        for (auto &a : asked)
            a = ~0ull;
    }
    static size_t slot_of(uint64_t tau) { return (size_t)((tau * 0x9E3779B97F4A7C15ull) >> 58); }

    // Column thread: ask for keys k[0..m) (each skipped when asked
    // recently).
    void publish(const uint64_t *k, size_t m)
    {
        const uint64_t h0 = head.load(std::memory_order_relaxed);
        uint64_t h = h0;
        for (size_t i = 0; i < m; ++i) {
            const size_t a = (size_t)((k[i] * 0xC2B2AE3D27D4EB4Full) >> 56);
            if (asked[a] == k[i])
                continue;
            asked[a] = k[i];
            ring[h++ % RING].store(k[i], std::memory_order_relaxed);
        }
        if (h != h0)
            head.store(h, std::memory_order_release);
    }
    // Column thread: start bringing in tau's slot (its header and first
    // keys), read a little later by take().
    void prefetch(uint64_t tau) const
    {
        const char *p = reinterpret_cast<const char *>(&slots[slot_of(tau)]);
        for (int i = 0; i < 10; ++i)
            _mm_prefetch(p + 64 * i, _MM_HINT_T0);
    }
    // Column thread: the result for cofacet tau, if a helper has one:
    // sigma (NOT_APPARENT when tau has no apparent partner) and its
    // coboundary in buf[0..len), the first `ties` keys ascending.
    bool take(uint64_t tau, uint64_t &sigma, uint64_t *buf, size_t &len, size_t &ties) const
    {
        const Slot &s = slots[slot_of(tau)];
        const uint32_t s1 = s.seq.load(std::memory_order_acquire);
        if ((s1 & 1) || s1 == 0 || s.tau.load(std::memory_order_relaxed) != tau)
            return false;
        sigma = s.sigma.load(std::memory_order_relaxed);
        len = s.len.load(std::memory_order_relaxed);
        ties = s.ties.load(std::memory_order_relaxed);
        if (len > CAP || ties > len)
            return false;
        for (size_t i = 0; i < len; ++i)
            buf[i] = s.keys[i].load(std::memory_order_relaxed);
        std::atomic_thread_fence(std::memory_order_acquire);
        return s.seq.load(std::memory_order_relaxed) == s1;
    }
    // Helper thread, until stop: compute(k, tau, sigma, e, len, ties) for
    // each requested key; false from it means nothing to hand over.
    template <class F> void help(F compute)
    {
        helping.fetch_add(1, std::memory_order_relaxed);
        while (!stop.load(std::memory_order_acquire)) {
            uint64_t c = claim.load(std::memory_order_relaxed);
            const uint64_t h = head.load(std::memory_order_acquire);
            if (c >= h) {
                _mm_pause();
                continue;
            }
            if (h - c > RING / 2) {  // far behind: only recent keys matter
                if (claim.compare_exchange_weak(c, h - RING / 4, std::memory_order_relaxed))
                    finished.fetch_add(h - RING / 4 - c, std::memory_order_release);
                continue;
            }
            if (!claim.compare_exchange_weak(c, c + 1, std::memory_order_relaxed))
                continue;
            answer(ring[c % RING].load(std::memory_order_relaxed), compute);
            finished.fetch_add(1, std::memory_order_release);
        }
    }
    template <class F> void answer(uint64_t k, F &compute)
    {
        uint64_t tau = 0, sigma = NOT_APPARENT;
        const uint64_t *e = nullptr;
        size_t len = 0, ties = 0;
        if (!compute(k, tau, sigma, e, len, ties) || len > CAP)
            return;
        Slot &s = slots[slot_of(tau)];
        uint32_t q = s.seq.load(std::memory_order_relaxed);
        if ((q & 1) || !s.seq.compare_exchange_strong(q, q + 1, std::memory_order_relaxed))
            return;  // another helper is writing this slot
        std::atomic_thread_fence(std::memory_order_release);
        s.tau.store(tau, std::memory_order_relaxed);
        s.sigma.store(sigma, std::memory_order_relaxed);
        s.len.store((uint32_t)len, std::memory_order_relaxed);
        s.ties.store((uint32_t)ties, std::memory_order_relaxed);
        for (size_t i = 0; i < len; ++i)
            s.keys[i].store(e[i], std::memory_order_relaxed);
        s.seq.store(q + 2, std::memory_order_release);
    }
    // Tests: let the helpers answer every request so far (none when no
    // helper has joined; bounded).
    void settle(int64_t spins) const
    {
        while (helping.load(std::memory_order_relaxed) > 0 &&
               finished.load(std::memory_order_acquire) < head.load(std::memory_order_relaxed) &&
               spins-- > 0)
            _mm_pause();
    }
    // Already answered (a slot holds tau): the helper skips it.
    bool has(uint64_t tau) const
    {
        const Slot &s = slots[slot_of(tau)];
        return !(s.seq.load(std::memory_order_acquire) & 1) &&
               s.tau.load(std::memory_order_relaxed) == tau;
    }
};

// Helper threads a long column's look-ahead may take: RPP_CHAIN_HELPERS
// (0: none), default 2.
int chain_helpers()
{
    static const int v = [] {
        const char *e = getenv("RPP_CHAIN_HELPERS");
        const int x = e ? atoi(e) : 2;
        return std::max(0, std::min(x, 8));
    }();
    return v;
}
// Tests: RPP_TEST_CHAIN_SETTLE=1 has a column wait (boundedly) after each
// request for the helpers' answers, so that handed-over coboundaries are
// used even on small inputs.
bool chain_test_settle()
{
    static const bool v = [] {
        const char *e = getenv("RPP_TEST_CHAIN_SETTLE");
        return e && atoi(e) != 0;
    }();
    return v;
}
// Additions a column makes in one call before it takes helpers (once it is
// a radix column): RPP_CHAIN_AFTER (tests), default 128.
int64_t chain_assist_after()
{
    static const int64_t v = [] {
        const char *e = getenv("RPP_CHAIN_AFTER");
        const long x = e ? atol(e) : 128;
        return (int64_t)std::max(0L, x);
    }();
    return v;
}

}  // namespace

void parallel_for(int64_t n, const std::function<void(int64_t)> &fn)
{
    std::atomic<int64_t> next{0};
    Pool::get().run([&](int) {
        for (int64_t i = next.fetch_add(1); i < n; i = next.fetch_add(1))
            fn(i);
    });
}

// Two phases, exact:
//  A (parallel over columns): reduce each column against the apparent
//    pivots only -- they are fixed before the reduction starts -- until its
//    low is not an apparent pivot (or the column is zero).
//  B (sequential, column order): the true reduction performs exactly the
//    same additions up to that point, because a row is the pivot of at most
//    one column, so apparent rows are never host pivots.  If the phase-A low
//    is not a pivot of an earlier host column, the column is final;
//    otherwise the reduction resumes from the phase-A state with the full
//    pivot store.
namespace {

// One dimension's reduction, split so that the speculative phase can run
// before the previous dimension's pivots (the clearing set) are known: the
// constructor runs phase A, finish() phase B.
template <class K> class SpecImpl final : public ResidualSpec {
public:
    SpecImpl(const ResidualProblem &p, const KeyCodec &kc)
        : codec(kc), P(p), ncols(p.ncols), spec_low(p.ncols), spec_nz(p.ncols, 0), spec_adds(p.ncols, 0),
          spec_cut(p.ncols, 0), state(p.ncols)
    {
        policy.prior = p.p == 1;
        phase_a();
    }
    void finish(const uint8_t *drop, ResidualResult &R) override
    {
        struct Known final : DropGate {
            const uint8_t *d;
            bool ready() override { return true; }
            const uint8_t *wait() override { return d; }
        } gate;
        gate.d = drop;
        R.lookups_apparent = looks_a;
        phase_b(gate, 0, R);
    }
    void finish_gated(DropGate &gate, int64_t cap, ResidualResult &R) override
    {
        R.lookups_apparent = looks_a;
        phase_b(gate, cap, R);
    }

private:
    bool apparent_lookup(const Ctx &X, uint64_t tau, float dt, uint64_t *other) const
    {
        if (P.app_tau) {
            const uint64_t *b = P.app_tau, *e = P.app_tau + P.napp;
            const uint64_t *f = std::lower_bound(b, e, tau);
            if (f == e || *f != tau)
                return false;
            *other = P.app_sigma[f - b];
            return true;
        }
        return X.apparent_partner(tau, dt, other);
    }
    float diam_of_key(int64_t j) const
    {
        return __builtin_bit_cast(float, (uint32_t)~(uint32_t)P.col_key[j]);
    }

    void phase_a()
    {
        // ---- phase A ----------------------------------------------------------
        Pool &pool = Pool::get();
        const int workers = P.parallel ? pool.size() : 1;
        std::atomic<int64_t> next{0};
        std::atomic<int64_t> look_app{0};
        const int64_t chunk = std::max<int64_t>(1, std::min<int64_t>(16, ncols / (8 * workers)));
        const int64_t budget = P.spec_budget;
        auto phase_a = [&](int) {
            Ctx X(P, &sink, codec);
            int64_t looks = 0;
            while (true) {
                const int64_t j0 = next.fetch_add(chunk);
                if (j0 >= ncols)
                    break;
                const int64_t j1 = std::min(ncols, j0 + chunk);
                for (int64_t j = j0; j < j1; ++j) {
                    Entry lo{P.col_low_diam[j], P.col_low[j]};
                    if (lo.cidx == ~0ull)
                        continue;  // empty coboundary
                    uint64_t other;
                    ++looks;
                    if (!apparent_lookup(X, lo.cidx, lo.diam, &other)) {
                        spec_low[j] = lo;
                        spec_nz[j] = 1;
                        continue;
                    }
                    std::unique_ptr<Column<K>> col(new Column<K>());
                    col->policy = &policy;
                    col->codec = &codec;
                    X.add_coboundary(*col, P.col_cidx[j], diam_of_key(j));
                    bool nz;
                    int64_t adds = 0;
                    bool cut = false;
                    while (true) {
                        // Algorithm 2: add the ORIGINAL column of the pivot's owner
                        // (an apparent column has the diameter of its tau)
                        X.add_coboundary(*col, other, lo.diam);
                        ++adds;
                        nz = col->low(lo);
                        if (!nz)
                            break;
                        ++looks;
                        if (!apparent_lookup(X, lo.cidx, lo.diam, &other))
                            break;
                        if (budget > 0 && adds >= budget) {
                            cut = true;  // low still apparent: phase B goes on
                            break;
                        }
                    }
                    spec_low[j] = lo;
                    spec_nz[j] = nz ? 1 : 0;
                    spec_adds[j] = adds;
                    spec_cut[j] = cut ? 1 : 0;
                    state[j] = std::move(col);
                }
            }
            look_app += looks;
        };
        if (P.parallel)
            pool.run(phase_a);
        else
            phase_a(0);
        looks_a = look_app.load();
    }

    void phase_b(DropGate &gate, int64_t cap, ResidualResult &R)
    {
        // ---- phase B ----------------------------------------------------------
        // Columns become final in column order (the frontier).  A column is
        // final once every earlier column is final and its low is not the pivot
        // of one of them.  A column whose low IS a final pivot makes exactly the
        // addition the sequential algorithm makes at that point (pivots never
        // change once final), so such columns -- anywhere past the frontier --
        // are advanced together on the worker pool, each until its low is
        // neither a final pivot nor apparent.  A waiting column is woken when
        // its low becomes a final pivot.
        //
        // A finished column that needed additions keeps its heap state: its
        // streams hold its reduced column R_k, which a later column adds in one
        // step (R_j += R_k) instead of replaying k's reduction from the original
        // column.  The copied entries are a subset of what the replay would
        // regenerate, so this is never more work.
        //
        // Columns that clearing removes (pivots of the previous dimension, not
        // known when the speculative phase ran) take no part: no pair, no
        // class.  Until the gate says which they are, every column is reduced
        // as usual (a dropped one would end at zero), zero columns wait to be
        // classified, and a column past `cap` additions parks until then.
        Pool &pool = Pool::get();
        const uint8_t *drop = nullptr;
        bool known = false;
        std::vector<uint8_t> parked(ncols, 0);
        std::vector<int64_t> parked_list, zero_open;
        FlatMap pivots((size_t)ncols);  // tau -> index in R.sigma
        std::vector<std::unique_ptr<Column<K>>> reduced;  // by index in R.sigma
        reduced.reserve((size_t)ncols);
        FlatMap whead((size_t)ncols);  // low -> last waiting column
        std::vector<int64_t> wnext(ncols, -1);
        std::vector<uint8_t> pending(ncols, 0);
        std::vector<int64_t> work;
        auto wait_on = [&](int64_t j) {
            auto r = whead.emplace(spec_low[j].cidx, j);
            if (!r.second) {
                wnext[j] = *r.first;
                *r.first = j;
            } else {
                wnext[j] = -1;
            }
        };
        for (int64_t j = 0; j < ncols; ++j) {
            if (!spec_nz[j])
                continue;
            if (spec_cut[j]) {
                pending[j] = 1;  // resumes in the first round
                work.push_back(j);
            } else {
                wait_on(j);
            }
        }

        auto essential = [&](int64_t j) {
            R.additions += spec_adds[j];
            R.ess_sigma.push_back(P.col_cidx[j]);
            R.ess_birth.push_back(diam_of_key(j));
        };
        auto finalize = [&](int64_t j) {
            if (drop && drop[j])
                return;
            const uint64_t sigma = P.col_cidx[j];
            const float d = diam_of_key(j);
            if (!spec_nz[j]) {
                if (known)
                    essential(j);
                else
                    zero_open.push_back(j);  // an essential class unless dropped
                return;
            }
            // nonzero: not a dropped column, whatever the gate will say
            R.additions += spec_adds[j];
            const Entry lo = spec_low[j];
            if (spec_adds[j] == 0)
                ++R.emergent;
            pivots.emplace(lo.cidx, (int64_t)R.sigma.size());
            R.sigma.push_back(sigma);
            R.tau.push_back(lo.cidx);
            R.birth.push_back(d);
            R.death.push_back(lo.diam);
            // oblivious: nothing is kept, a later column adds D_k instead
            reduced.push_back(spec_adds[j] && !P.oblivious ? std::move(state[j]) : nullptr);
            state[j].reset();
            if (const Column<K> *rk = reduced.back().get()) {
                // R_k holding many more keys than D_k: a later column adds
                // D_k and reduces it again lazily rather than copying R_k
                const size_t d0 = rk->first_len();
                if (P.keep_ratio > 0.0 && d0 > 0 &&
                    (double)rk->remaining() > P.keep_ratio * (double)d0)
                    reduced.back().reset();
            }
            const int64_t *it = whead.find(lo.cidx);
            if (!it)
                return;
            for (int64_t k = *it; k >= 0; k = wnext[k])
                if (k != j && spec_nz[k] && spec_low[k].cidx == lo.cidx && !pending[k]) {
                    pending[k] = 1;
                    work.push_back(k);
                }
            whead.erase(lo.cidx);
        };

        // The dropped columns are known: drop them, classify the open zero
        // columns, and resume the parked ones.
        // RPP_TRACE: when the gate opened, the slices run before it, and the
        // longest round of the exact phase
        static const bool trace = [] {
            const char *e = getenv("RPP_TRACE");
            return e && atoi(e) != 0;
        }();
        const auto t0 = std::chrono::steady_clock::now();
        auto ms_since = [&t0]() {
            return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0)
                .count();
        };
        int64_t nslices = 0, nrounds = 0, longest_size = 0;
        double longest_ms = 0.0, slice_ms = 0.0;
        std::mutex trace_mu;
        int64_t trace_adds = 0;  // the call with the most additions, and its times
        double trace_tm[4] = {0, 0, 0, 0};
        auto learn = [&]() {
            const double w0 = trace ? ms_since() : 0.0;
            drop = gate.wait();
            if (trace)
                fprintf(stderr,
                        "rpp trace:   p=%d exact phase: gate open at %.3f ms (waited %.3f ms, "
                        "%lld slices of parked columns before it, %.3f ms)\n",
                        P.p, ms_since(), ms_since() - w0, (long long)nslices, slice_ms);
            known = true;
            if (drop)
                for (int64_t j = 0; j < ncols; ++j)
                    if (drop[j])
                        spec_nz[j] = 0;  // never woken, never finalized
            for (int64_t j : zero_open)
                if (!(drop && drop[j]))
                    essential(j);
            zero_open.clear();
            for (int64_t j : parked_list) {
                parked[j] = 0;
                if (!(drop && drop[j])) {
                    pending[j] = 1;
                    work.push_back(j);
                }
            }
            parked_list.clear();
        };
        if (gate.ready())
            learn();

        // Advance column j from a low that is a final pivot (read-only use of
        // the pivot store and the finished columns; safe to run concurrently).
        std::atomic<int64_t> look_hash{0}, look_app_b{0};
        bool open = !known;  // read by advance(); set before each round
        int64_t cap_now = cap;  // the additions a column may reach while open
        std::vector<int64_t> slice_cap((size_t)ncols, 0);  // a sliced column's own cap
        std::atomic<int64_t> n_handed{0}, n_assisted{0};  // RPP_TRACE counts
        // Look-ahead helpers for a long column (64-bit keys): at most
        // chain_helpers() idle workers, once a call has made ASSIST_AFTER
        // additions on a radix column.
        const int64_t ASSIST_AFTER = chain_assist_after();
        const int helpers =
            sizeof(K) == 8 && P.parallel ? std::min(chain_helpers(), pool.size() - 1) : 0;
        struct Assisted {  // stops and joins the helpers on every way out
            Pool &pool;
            std::unique_ptr<ChainAssist> as;
            Pool::Async job;
            std::vector<uint64_t> buf;  // a handed-over coboundary
            explicit Assisted(Pool &p) : pool(p), as(new ChainAssist()), buf(ChainAssist::CAP) {}
            ~Assisted()
            {
                as->stop.store(true, std::memory_order_release);
                pool.join(job);
            }
        };
        auto start_assist = [&](std::unique_ptr<Assisted> &A) {
            A.reset(new Assisted(pool));
            ChainAssist *as = A->as.get();
            auto joined = std::make_shared<std::atomic<int>>(0);
            pool.launch(A->job, [this, as, joined, helpers, &pivots](int) {
                if (joined->fetch_add(1) >= helpers)
                    return;
                Ctx Xh(P, &sink, codec);
                as->help([&](uint64_t k, uint64_t &tau, uint64_t &sigma, const uint64_t *&e,
                             size_t &len, size_t &ties) {
                    const Entry t = unpack_key<K>(codec, (K)k);
                    tau = t.cidx;
                    if (as->has(tau) || pivots.find(tau))
                        return false;  // answered, or a host pivot
                    uint64_t other = 0;
                    if (!apparent_lookup(Xh, t.cidx, t.diam, &other)) {
                        sigma = ChainAssist::NOT_APPARENT;
                        return true;
                    }
                    K *out = nullptr;
                    size_t tl = 0;
                    len = Xh.coboundary<K>(other, t.diam, out, tl);
                    Xh.arena.uncommit<K>(len);  // copied out before the next one
                    sigma = other;
                    ties = tl;
                    e = reinterpret_cast<const uint64_t *>(out);
                    return true;
                });
            });
        };
        auto advance = [&](Ctx &Xc, int64_t j) {
            if (drop && drop[j])
                return;  // dropped after it was queued
            std::unique_ptr<Column<K>> &col = state[j];
            if (!col) {
                col.reset(new Column<K>());
                col->policy = &policy;
                col->codec = &codec;
                Xc.add_coboundary(*col, P.col_cidx[j], diam_of_key(j));
            }
            Entry lo = spec_low[j];
            int64_t adds = 0, lh = 0, la = 0;
            bool nz = true;
            // RPP_TRACE: where the longest call's time goes
            double tm[4] = {0, 0, 0, 0};  // pivot adds, apparent lookups, coboundaries, lows
            auto tick = [](std::chrono::steady_clock::time_point &t) {
                const auto u = std::chrono::steady_clock::now();
                const double d = std::chrono::duration<double, std::milli>(u - t).count();
                t = u;
                return d;
            };
            std::chrono::steady_clock::time_point tt;
            if (trace)
                tt = std::chrono::steady_clock::now();
            std::unique_ptr<Assisted> A;  // declared after col: joined before col may go
            ChainAssist *as = nullptr;
            while (true) {
                if (!as && adds >= ASSIST_AFTER && helpers > 0 && col->radix()) {
                    start_assist(A);
                    as = A->as.get();
                    ++n_assisted;
                }
                const int64_t capj = slice_cap[j] ? slice_cap[j] : cap_now;
                if (open && capj > 0 && spec_adds[j] + adds >= capj) {
                    parked[j] = 1;  // resumes once the dropped columns are known
                    break;
                }
                // the owner of the low: a final host column, else an
                // apparent column, else the column stops here
                const int64_t *f = pivots.find(lo.cidx);
                if (f) {
                    ++lh;
                    const int64_t k = *f;
                    if (reduced[k])
                        col->add(*reduced[k], Xc.arena);
                    else
                        Xc.add_coboundary(*col, R.sigma[k], R.birth[k]);
                    if (trace)
                        tm[0] += tick(tt);
                } else {
                    uint64_t other = 0;
                    ++la;
                    size_t alen = 0, aties = 0;
                    bool app, handed = false;
                    if (as && as->take(lo.cidx, other, A->buf.data(), alen, aties)) {
                        handed = true;
                        ++n_handed;
                        app = other != ChainAssist::NOT_APPARENT;
                    } else {
                        app = apparent_lookup(Xc, lo.cidx, lo.diam, &other);
                    }
                    if (trace)
                        tm[1] += tick(tt);
                    if (!app)
                        break;
                    if (handed)  // a radix column copies the keys in
                        col->push_stream(reinterpret_cast<K *>(A->buf.data()), alen, aties);
                    else
                        Xc.add_coboundary(*col, other, lo.diam);  // diameter of its tau
                    if (trace)
                        tm[2] += tick(tt);
                }
                ++adds;
                nz = col->low(lo);
                if (trace)
                    tm[3] += tick(tt);
                if (!nz)
                    break;
                if (as) {  // ask for the keys just above the new low
                    as->prefetch(lo.cidx);
                    K ah[8 + 16];
                    const size_t m = col->ahead(ah, 8, 16);
                    uint64_t ak[8 + 16];
                    for (size_t i = 0; i < m; ++i)
                        ak[i] = (uint64_t)ah[i];
                    as->publish(ak, m);
                    if (chain_test_settle())
                        as->settle(1000000);
                }
            }
            if (trace) {
                std::lock_guard<std::mutex> lk(trace_mu);
                if (adds > trace_adds) {
                    trace_adds = adds;
                    for (int q = 0; q < 4; ++q)
                        trace_tm[q] = tm[q];
                }
            }
            spec_low[j] = lo;
            spec_nz[j] = nz ? 1 : 0;
            spec_adds[j] += adds;
            look_hash += lh;
            look_app_b += la;
        };

        Ctx X(P, &sink, codec);
        int64_t frontier = 0;
        std::vector<int64_t> round;
        while (frontier < ncols) {
            if (!known && gate.ready())
                learn();
            while (frontier < ncols && !pending[frontier] && !parked[frontier])
                finalize(frontier++);
            if (frontier == ncols)
                break;
            if (work.empty()) {
                // the frontier waits on a parked column: only the gate helps
                if (known)
                    throw std::logic_error("residual reduction: frontier stalled");
                if (!parked_list.empty() && P.park_slice > 0 && !gate.ready()) {
                    // Nothing can move until the dropped columns are known.
                    // Instead of waiting idle, take every parked column a
                    // slice of additions further, in parallel (a column's
                    // work is lost only if the gate then drops it; the long
                    // chain the frontier will wait on is among them), and
                    // look at the gate again.
                    round.assign(parked_list.begin(), parked_list.end());
                    parked_list.clear();
                    for (int64_t j : round) {
                        parked[j] = 0;
                        slice_cap[j] = spec_adds[j] + P.park_slice;
                    }
                    open = true;
                    const double s0 = trace ? ms_since() : 0.0;
                    if (round.size() == 1 || !P.parallel) {
                        for (int64_t j : round)
                            advance(X, j);
                    } else {
                        std::atomic<int64_t> nx{0};
                        pool.run([&](int) {
                            Ctx Xw(P, &sink, codec);
                            for (int64_t i = nx.fetch_add(1); i < (int64_t)round.size();
                                 i = nx.fetch_add(1))
                                advance(Xw, round[i]);
                        });
                    }
                    if (trace)
                        slice_ms += ms_since() - s0;
                    nslices += (int64_t)round.size();
                    for (int64_t j : round) {
                        slice_cap[j] = 0;
                        if (parked[j])
                            parked_list.push_back(j);
                        else if (spec_nz[j] && !(drop && drop[j]))
                            wait_on(j);
                    }
                    continue;
                }
                learn();
                continue;
            }
            open = !known;
            round.swap(work);
            work.clear();
            const double r0 = trace ? ms_since() : 0.0;
            if (round.size() == 1 || !P.parallel) {
                for (int64_t j : round)
                    advance(X, j);
            } else {
                std::atomic<int64_t> nx{0};
                pool.run([&](int) {
                    Ctx Xw(P, &sink, codec);
                    for (int64_t i = nx.fetch_add(1); i < (int64_t)round.size(); i = nx.fetch_add(1))
                        advance(Xw, round[i]);
                });
            }
            ++nrounds;
            if (trace && ms_since() - r0 > longest_ms) {
                longest_ms = ms_since() - r0;
                longest_size = (int64_t)round.size();
            }
            for (int64_t j : round) {
                pending[j] = 0;
                if (parked[j])
                    parked_list.push_back(j);
                else if (spec_nz[j] && !(drop && drop[j]))
                    wait_on(j);
            }
        }
        if (!known)
            learn();  // classifies the zero columns still open
        if (trace)
            fprintf(stderr,
                    "rpp trace:   p=%d exact phase: %lld rounds, longest %.3f ms (%lld columns), "
                    "done at %.3f ms; longest column call %lld additions: pivot adds %.3f ms, "
                    "apparent lookups %.3f ms, coboundaries %.3f ms, lows %.3f ms; look-ahead: %lld columns, %lld handed over\n",
                    P.p, (long long)nrounds, longest_ms, (long long)longest_size, ms_since(),
                    (long long)trace_adds, trace_tm[0], trace_tm[1], trace_tm[2], trace_tm[3],
                    (long long)n_assisted.load(), (long long)n_handed.load());
        R.lookups_hash += look_hash.load();
        R.lookups_apparent += look_app_b.load();
    }

    BlockSink sink;  // stream storage of every column below; freed last
    DepthPolicy policy;
    const KeyCodec codec;
    const ResidualProblem P;
    const int64_t ncols;
    std::vector<Entry> spec_low;
    std::vector<uint8_t> spec_nz;
    std::vector<int64_t> spec_adds;
    std::vector<uint8_t> spec_cut;  // phase A stopped at its budget, low apparent
    std::vector<std::unique_ptr<Column<K>>> state;
    int64_t looks_a = 0;
};

}  // namespace

std::unique_ptr<ResidualSpec> residual_speculate(const ResidualProblem &P)
{
    // largest cofacet index + 1 = C(n, p+2)
    const uint64_t ncof = P.binom[(int64_t)(P.p + 2) * (P.n + 1) + P.n];
    // tests: RPP_WIDE_KEYS=1 takes the 128-bit keys even where 64 suffice,
    // RPP_RANK_KEYS=1 the rank-coded ones whenever diameters are ranks
    const char *wide_env = getenv("RPP_WIDE_KEYS"), *rank_env = getenv("RPP_RANK_KEYS");
    const bool wide = wide_env && atoi(wide_env) != 0;
    const bool rank_keys = rank_env && atoi(rank_env) != 0;
    if (ncof <= (1ull << 32) && !wide && !(rank_keys && P.rank_bits > 0))
        return std::unique_ptr<ResidualSpec>(
            new SpecImpl<uint64_t>(P, default_codec<uint64_t>()));
    int cbits = 0;  // bits of the largest cofacet index, ncof - 1
    while (cbits < 64 && ((ncof - 1) >> cbits) != 0)
        ++cbits;
    if (P.rank_bits > 0 && P.rank_bits <= 24 && P.rank_bits + cbits <= 64 && !wide) {
        KeyCodec kc;
        kc.rank = true;
        kc.shift = cbits;
        kc.mask = cbits == 64 ? ~0ull : (1ull << cbits) - 1;
        return std::unique_ptr<ResidualSpec>(new SpecImpl<uint64_t>(P, kc));
    }
    return std::unique_ptr<ResidualSpec>(new SpecImpl<u128>(P, default_codec<u128>()));
}

void residual_reduce(const ResidualProblem &P, ResidualResult &R)
{
    residual_speculate(P)->finish(nullptr, R);
}

}  // namespace rpp
