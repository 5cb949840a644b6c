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

#include <algorithm>
#include <atomic>
#include <type_traits>
#include <condition_variable>
#include <functional>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>

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
template <class K> inline K pack(float d, uint64_t c)
{
    return ((K)__builtin_bit_cast(uint32_t, d) << KeyFmt<K>::S) | (K)(KeyFmt<K>::M - c);
}
template <class K> inline Entry unpack(K k)
{
    return Entry{__builtin_bit_cast(float, (uint32_t)(k >> KeyFmt<K>::S)),
                 KeyFmt<K>::M - (uint64_t)(k & (K)KeyFmt<K>::M)};
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

// One added coboundary, consumed oldest-first.  Only a sorted prefix is
// kept: the oldest `chunk` remaining keys are selected (linear on average)
// and sorted; when they run out the next, twice as large, chunk is
// selected.  A column's low usually lies a few dozen entries into each
// stream, so most keys are never ordered, and pops read memory in order.
// Allocator whose construct() default-initialises: resizing a stream's
// storage before the coboundary is written into it does not zero it.
template <class T> struct NoInit : std::allocator<T> {
    template <class U> struct rebind {
        using other = NoInit<U>;
    };
    NoInit() = default;
    template <class U> NoInit(const NoInit<U> &) noexcept {}
    template <class U> void construct(U *p) noexcept { ::new ((void *)p) U; }
    template <class U, class... A> void construct(U *p, A &&...a)
    {
        ::new ((void *)p) U(std::forward<A>(a)...);
    }
};
template <class K> using KeyVec = std::vector<K, NoInit<K>>;

template <class K> struct Stream {
    KeyVec<K> e;
    uint32_t pos = 0, sorted = 0, chunk = 32;
    bool empty() const { return pos >= e.size(); }
    K front() const { return e[pos]; }
    void prepare()
    {
        pos = sorted = 0;
        chunk = 32;
        refill();
    }
    void refill()
    {
        const size_t rem = e.size() - pos;
        if (rem == 0)
            return;
        const size_t c = std::min<size_t>(rem, chunk);
        if (c < rem)
            select_smallest(e.data() + pos, rem, c);
        std::sort(e.begin() + pos, e.begin() + pos + c);
        sorted = pos + (uint32_t)c;
        chunk = chunk < (1u << 30) ? chunk * 2 : chunk;
    }
    void pop()
    {
        if (++pos == sorted)
            refill();
    }
};

// Working column = Z/2 sum of several coboundaries.  Each added coboundary
// is its own stream; a min-heap over the streams' current fronts yields the
// sum's entries oldest-first.  Only the entries that reach the front are
// ever ordered, which is what finding the low needs.
template <class K> class Column {
public:
    // Storage for the next coboundary: fill it, then commit().
    KeyVec<K> &next_stream()
    {
        if (nstreams == streams.size())
            streams.emplace_back();
        KeyVec<K> &v = streams[nstreams].e;
        v.clear();
        return v;
    }
    void commit()
    {
        Stream<K> &st = streams[nstreams];
        if (st.e.empty())
            return;
        st.prepare();
        top_push(st.front(), (uint32_t)nstreams);
        ++nstreams;
    }
    // Add another column's current contents: its streams hold exactly its
    // Z/2 sum (cancelled pairs were removed together).
    void add(const Column &o)
    {
        for (size_t k = 0; k < o.nstreams; ++k) {
            const Stream<K> &src = o.streams[k];
            if (src.empty())
                continue;
            if (nstreams == streams.size())
                streams.emplace_back();
            Stream<K> &dst = streams[nstreams];
            dst.e.assign(src.e.begin() + src.pos, src.e.end());
            dst.pos = 0;
            dst.sorted = src.sorted - src.pos;
            dst.chunk = src.chunk;
            top_push(dst.front(), (uint32_t)nstreams);
            ++nstreams;
        }
    }
    // Low of the sum over Z/2: keys present in an even number of streams
    // cancel.  In the min-heap every copy of the minimum lies in a subtree
    // containing the root, so a second copy exists iff a child of the root
    // holds it; pairs are dropped until the minimum is unique.
    bool low(Entry &out)
    {
        while (!hk.empty()) {
            const K e = hk[0];
            const size_t m = hk.size();
            const size_t e4 = m < 5 ? m : 5;
            bool dup = false;
            for (size_t j = 1; j < e4; ++j)
                dup |= hk[j] == e;
            if (!dup) {
                out = unpack<K>(e);
                return true;
            }
            advance_root();  // the other copy becomes the root
            advance_root();
        }
        return false;
    }

private:
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
    size_t nstreams = 0;
    std::vector<K> hk;
    std::vector<uint32_t> hs;
};

// ---------------------------------------------------------------------------
// AVX-512 variants (chosen at run time when the CPU has F, VL, BW and VBMI2)
// ---------------------------------------------------------------------------
static bool cpu_has_avx512()
{
    static const bool ok = __builtin_cpu_supports("avx512f") &&
                           __builtin_cpu_supports("avx512vl") &&
                           __builtin_cpu_supports("avx512bw") &&
                           __builtin_cpu_supports("avx512vbmi2");
    return ok;
}

// Dense coboundary with 32-bit cofacet indices (u64 keys): 16 candidate
// vertices per step -- row maxima, the threshold test, the packed keys --
// and a compress of the cofacets that pass (out needs 16 slots of slack).  Same set of keys as the
// scalar loop; the order within a stream does not matter.
__attribute__((target("avx512f,avx512vl,avx512bw,avx512vbmi2"))) static size_t
cob_dense_u64_avx512(const float *const *rows, int nv, const int *v, uint64_t sigma, float d,
                     float thr, const uint64_t *binom, int n, uint64_t *out)
{
    size_t cnt = 0;
    uint64_t above = 0, below = sigma;
    int hi = n;
    const __m512 vd = _mm512_set1_ps(d), vthr = _mm512_set1_ps(thr);
    const __m512i vM = _mm512_set1_epi64((long long)0xffffffffull);
    for (int idx = 0; idx <= nv; ++idx) {
        const int lo = idx < nv ? v[idx] : -1;
        const int j = nv - idx;  // vertices of sigma below w
        const uint64_t *Cj = binom + (int64_t)(j + 1) * (n + 1);
        const __m512i vbase = _mm512_set1_epi64((long long)(above + below));
        for (int w0 = lo + 1; w0 < hi; w0 += 16) {
            const int rem = hi - w0;
            const __mmask16 lm = rem >= 16 ? (__mmask16)0xffff : (__mmask16)((1u << rem) - 1u);
            __m512 mx = _mm512_maskz_loadu_ps(lm, rows[0] + w0);
            for (int i = 1; i < nv; ++i)
                mx = _mm512_max_ps(mx, _mm512_maskz_loadu_ps(lm, rows[i] + w0));
            const __mmask16 ok = _mm512_mask_cmp_ps_mask(lm, mx, vthr, _CMP_LE_OQ);
            const __m512i ndb = _mm512_castps_si512(_mm512_max_ps(mx, vd));
            const __m512i c0 =
                _mm512_add_epi64(vbase, _mm512_maskz_loadu_epi64((__mmask8)lm, Cj + w0));
            const __m512i c1 =
                _mm512_add_epi64(vbase, _mm512_maskz_loadu_epi64((__mmask8)(lm >> 8), Cj + w0 + 8));
            const __m512i d0 = _mm512_cvtepu32_epi64(_mm512_castsi512_si256(ndb));
            const __m512i d1 = _mm512_cvtepu32_epi64(_mm512_extracti64x4_epi64(ndb, 1));
            const __m512i k0 = _mm512_or_si512(_mm512_slli_epi64(d0, 32), _mm512_sub_epi64(vM, c0));
            const __m512i k1 = _mm512_or_si512(_mm512_slli_epi64(d1, 32), _mm512_sub_epi64(vM, c1));
            // compress in registers, then full stores (the memory form of
            // compress is slow on some cores); out has 16 slots of slack
            const __mmask8 ok0 = (__mmask8)ok, ok1 = (__mmask8)(ok >> 8);
            _mm512_storeu_si512(out + cnt, _mm512_maskz_compress_epi64(ok0, k0));
            cnt += (size_t)__builtin_popcount(ok0);
            _mm512_storeu_si512(out + cnt, _mm512_maskz_compress_epi64(ok1, k1));
            cnt += (size_t)__builtin_popcount(ok1);
        }
        if (idx < nv) {
            const int r = nv - 1 - idx;  // rank of v[idx] from the bottom
            below -= binom[(int64_t)(r + 1) * (n + 1) + lo];
            above += binom[(int64_t)(r + 2) * (n + 1) + lo];
        }
        hi = lo;
    }
    return cnt;
}

struct Ctx {
    const ResidualProblem &P;
    int n, p;
    explicit Ctx(const ResidualProblem &pp) : P(pp), n(pp.n), p(pp.p) {}

    uint64_t C(int v, int k) const { return P.binom[(int64_t)k * (n + 1) + v]; }
    float D(int a, int b) const { return P.dsq[(int64_t)a * n + b]; }

    // vertices of a simplex with q+1 vertices, decreasing
    void decode(uint64_t c, int q, int *v) const
    {
        int hi = n;
        for (int pos = 0; pos <= q; ++pos) {
            const int k = q + 1 - pos;
            int lo = k - 1, h = hi - 1;
            while (lo < h) {
                int mid = (lo + h + 1) >> 1;
                if (C(mid, k) <= c)
                    lo = mid;
                else
                    h = mid - 1;
            }
            v[pos] = lo;
            c -= C(lo, k);
            hi = lo;
        }
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

    // Adds sigma's coboundary to col as a new stream.
    template <class K> void add_coboundary(Column<K> &col, uint64_t sigma, float d) const
    {
        coboundary(sigma, d, col.next_stream());
        col.commit();
    }

    // Every cofacet of sigma with diameter <= threshold, appended to out as
    // packed keys.
    template <class K> void coboundary(uint64_t sigma, float d, KeyVec<K> &out) const
    {
        int v[8];
        decode(sigma, p, v);
        if (P.bits) {
            // common neighbours only: every new edge is within the threshold;
            // count them first so the stream is sized exactly
            size_t cnt = 0;
            for (int k = 0; k < P.words; ++k) {
                uint64_t m = ~0ull;
                for (int i = 0; i <= p; ++i)
                    m &= P.bits[(int64_t)v[i] * P.words + k];
                cnt += (size_t)__builtin_popcountll(m);
            }
            out.resize(cnt);
            K *o = out.data();
            for (int k = 0; k < P.words; ++k) {
                uint64_t m = ~0ull;
                for (int i = 0; i <= p; ++i)
                    m &= P.bits[(int64_t)v[i] * P.words + k];
                for (; m; m &= m - 1) {
                    const int w = k * 64 + __builtin_ctzll(m);
                    float nd = d;
                    for (int i = 0; i <= p; ++i) {
                        const float e = D(v[i], w);
                        nd = e > nd ? e : nd;
                    }
                    *o++ = pack<K>(nd, insert_index(v, w));
                }
            }
            return;
        }
        const float *rows[8];
        for (int i = 0; i <= p; ++i)
            rows[i] = P.dsq + (int64_t)v[i] * n;
        out.resize((size_t)n + 16);
        size_t cnt;
        if (std::is_same<K, uint64_t>::value && cpu_has_avx512()) {
            cnt = cob_dense_u64_avx512(rows, p + 1, v, sigma, d, P.thr, P.binom, n,
                                       reinterpret_cast<uint64_t *>(out.data()));
            out.resize(cnt);
            return;
        }
        switch (p) {
        case 1: cnt = cob_dense<K, 2>(rows, v, sigma, d, out.data()); break;
        case 2: cnt = cob_dense<K, 3>(rows, v, sigma, d, out.data()); break;
        case 3: cnt = cob_dense<K, 4>(rows, v, sigma, d, out.data()); break;
        default: cnt = cob_dense<K, 0>(rows, v, sigma, d, out.data()); break;
        }
        out.resize(cnt);
    }

    // Dense coboundary: cidx of sigma + {w} = above + C(w, j+1) + below,
    // where the vertices of sigma above w move up one rank.  Between two
    // consecutive vertices of sigma, j, above and below are constant, so w
    // runs over each gap in a tight loop that writes every cofacet and
    // advances the output only for those within the threshold.
    template <class K, int NV>
    size_t cob_dense(const float *const *rows, const int *v, uint64_t sigma, float d, K *out) const
    {
        const int nv = NV ? NV : p + 1;
        const float thr = P.thr;
        size_t cnt = 0;
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
                out[cnt] = pack<K>(nd, base + Cj[w]);
                cnt += (mx <= thr) ? 1 : 0;
            }
            if (idx < nv) {
                const int r = nv - 1 - idx;  // rank of v[idx] from the bottom
                below -= C(lo, r + 1);
                above += C(lo, r + 2);
            }
            hi = lo;
        }
        return cnt;
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
                for (; m; m &= m - 1) {
                    const int w = k * 64 + __builtin_ctzll(m);
                    if (w <= u)
                        continue;
                    bool all = true;
                    for (int i = 0; i <= p && all; ++i)
                        all = P.dsq[(int64_t)s[i] * n + w] <= dt;
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
    Pool()
    {
        unsigned hw = std::thread::hardware_concurrency();
        int n = (int)(hw ? hw : 1);
        if (const char *e = getenv("RPP_HOST_THREADS"))
            n = atoi(e);
        n = std::max(1, std::min(n, 16));
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
    explicit SpecImpl(const ResidualProblem &p)
        : P(p), ncols(p.ncols), spec_low(p.ncols), spec_nz(p.ncols, 0), spec_adds(p.ncols, 0),
          spec_cut(p.ncols, 0), state(p.ncols)
    {
        phase_a();
    }
    void finish(const uint8_t *drop, ResidualResult &R) override
    {
        R.lookups_apparent = looks_a;
        phase_b(drop, R);
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
            Ctx X(P);
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

    void phase_b(const uint8_t *drop, ResidualResult &R)
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
        Pool &pool = Pool::get();
        // columns that clearing removes (pivots of the previous dimension, not
        // known when the speculative phase ran) take no part: no pair, no class
        if (drop)
            for (int64_t j = 0; j < ncols; ++j)
                if (drop[j])
                    spec_nz[j] = 0;
        std::unordered_map<uint64_t, int64_t> pivots;  // tau -> index in R.sigma
        pivots.reserve((size_t)ncols * 2 + 16);
        std::vector<std::unique_ptr<Column<K>>> reduced;  // by index in R.sigma
        reduced.reserve((size_t)ncols);
        std::unordered_map<uint64_t, int64_t> whead;  // low -> last waiting column
        whead.reserve((size_t)ncols * 2 + 16);
        std::vector<int64_t> wnext(ncols, -1);
        std::vector<uint8_t> pending(ncols, 0);
        std::vector<int64_t> work;
        auto wait_on = [&](int64_t j) {
            auto r = whead.emplace(spec_low[j].cidx, j);
            if (!r.second) {
                wnext[j] = r.first->second;
                r.first->second = j;
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

        auto finalize = [&](int64_t j) {
            if (drop && drop[j])
                return;
            const uint64_t sigma = P.col_cidx[j];
            const float d = diam_of_key(j);
            R.additions += spec_adds[j];
            if (!spec_nz[j]) {
                R.ess_sigma.push_back(sigma);
                R.ess_birth.push_back(d);
                return;
            }
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
            auto it = whead.find(lo.cidx);
            if (it == whead.end())
                return;
            for (int64_t k = it->second; k >= 0; k = wnext[k])
                if (k != j && spec_nz[k] && spec_low[k].cidx == lo.cidx && !pending[k]) {
                    pending[k] = 1;
                    work.push_back(k);
                }
            whead.erase(it);
        };

        // Advance column j from a low that is a final pivot (read-only use of
        // the pivot store and the finished columns; safe to run concurrently).
        std::atomic<int64_t> look_hash{0}, look_app_b{0};
        auto advance = [&](Ctx &Xc, int64_t j) {
            std::unique_ptr<Column<K>> &col = state[j];
            if (!col) {
                col.reset(new Column<K>());
                Xc.add_coboundary(*col, P.col_cidx[j], diam_of_key(j));
            }
            Entry lo = spec_low[j];
            int64_t adds = 0, lh = 0, la = 0;
            bool nz = true;
            while (true) {
                // the owner of the low: a final host column, else an
                // apparent column, else the column stops here
                auto f = pivots.find(lo.cidx);
                if (f != pivots.end()) {
                    ++lh;
                    const int64_t k = f->second;
                    if (reduced[k])
                        col->add(*reduced[k]);
                    else
                        Xc.add_coboundary(*col, R.sigma[k], R.birth[k]);
                } else {
                    uint64_t other = 0;
                    ++la;
                    if (!apparent_lookup(Xc, lo.cidx, lo.diam, &other))
                        break;
                    Xc.add_coboundary(*col, other, lo.diam);  // diameter of its tau
                }
                ++adds;
                nz = col->low(lo);
                if (!nz)
                    break;
            }
            spec_low[j] = lo;
            spec_nz[j] = nz ? 1 : 0;
            spec_adds[j] += adds;
            look_hash += lh;
            look_app_b += la;
        };

        Ctx X(P);
        int64_t frontier = 0;
        std::vector<int64_t> round;
        while (frontier < ncols) {
            while (frontier < ncols && !pending[frontier])
                finalize(frontier++);
            if (frontier == ncols)
                break;
            round.swap(work);
            work.clear();
            if (round.size() == 1 || !P.parallel) {
                for (int64_t j : round)
                    advance(X, j);
            } else {
                std::atomic<int64_t> nx{0};
                pool.run([&](int) {
                    Ctx Xw(P);
                    for (int64_t i = nx.fetch_add(1); i < (int64_t)round.size(); i = nx.fetch_add(1))
                        advance(Xw, round[i]);
                });
            }
            for (int64_t j : round) {
                pending[j] = 0;
                if (spec_nz[j])
                    wait_on(j);
            }
        }
        R.lookups_hash += look_hash.load();
        R.lookups_apparent += look_app_b.load();
    }

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
    if (ncof <= (1ull << 32))
        return std::unique_ptr<ResidualSpec>(new SpecImpl<uint64_t>(P));
    return std::unique_ptr<ResidualSpec>(new SpecImpl<u128>(P));
}

void residual_reduce(const ResidualProblem &P, ResidualResult &R)
{
    residual_speculate(P)->finish(nullptr, R);
}

}  // namespace rpp
