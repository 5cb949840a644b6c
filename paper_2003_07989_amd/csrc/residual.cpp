// residual.cpp -- host reduction of the columns the GPU could not pair.
//
// Paper, "Reduction Matrix vs. Oblivious Matrix Reduction" (Algorithm 2)
// and "Core System Optimizations" (two-layer pair store).  Columns arrive in
// coboundary order together with their lows (oldest cofacets), computed on
// the GPU.  A column whose low is not yet a pivot is paired at once, with no
// coboundary built (its unreduced column is already reduced).  Otherwise its
// coboundary is regenerated from the distance matrix (implicit matrix
// reduction) into a binary heap ordered oldest-first, so the heap top is the
// column's low; Z/2 addition pushes the other column's entries, and equal
// entries cancel in pairs when the low is taken.
#include "residual.h"

#include <algorithm>
#include <atomic>
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

// Max-heap comparator whose top is the OLDEST entry (smallest diameter,
// then largest cidx): a < b means a is younger than b.
struct YoungerFirst {
    bool operator()(const Entry &a, const Entry &b) const
    {
        if (a.diam != b.diam)
            return a.diam > b.diam;
        return a.cidx < b.cidx;
    }
};

// Working column = Z/2 sum of several coboundaries.  Each added coboundary
// is kept as its own small heap (a "stream", built in linear time); a heap
// over the streams' current tops yields the sum's entries oldest-first.
// Only the entries that reach the top are ever ordered, which is what
// finding the low needs.
class Column {
public:
    void clear()
    {
        nstreams = 0;
        top.clear();
    }
    void add(const std::vector<Entry> &batch)
    {
        if (batch.empty())
            return;
        if (nstreams == streams.size())
            streams.emplace_back();
        std::vector<Entry> &h = streams[nstreams];
        h.assign(batch.begin(), batch.end());
        std::make_heap(h.begin(), h.end(), YoungerFirst());
        top_push(h.front(), (uint32_t)nstreams);
        ++nstreams;
    }
    // Add another column's current contents: its streams hold exactly its
    // Z/2 sum (cancelled pairs were removed together), each a valid heap.
    void add(const Column &o)
    {
        for (size_t k = 0; k < o.nstreams; ++k) {
            const std::vector<Entry> &src = o.streams[k];
            if (src.empty())
                continue;
            if (nstreams == streams.size())
                streams.emplace_back();
            streams[nstreams].assign(src.begin(), src.end());
            top_push(streams[nstreams].front(), (uint32_t)nstreams);
            ++nstreams;
        }
    }
    // Low of the sum over Z/2: entries present in an even number of
    // streams cancel; the surviving low stays in its stream.
    bool low(Entry &out)
    {
        while (!top.empty()) {
            const Entry e = top.front().e;
            hits.clear();
            while (!top.empty() && top.front().e.cidx == e.cidx) {
                hits.push_back(top.front().s);
                top_pop();
            }
            const size_t keep = (hits.size() & 1) ? 1 : 0;
            for (size_t i = 0; i < hits.size(); ++i) {
                const uint32_t k = hits[i];
                if (i < keep) {
                    top_push(e, k);  // the surviving copy stays put
                    continue;
                }
                std::vector<Entry> &h = streams[k];
                std::pop_heap(h.begin(), h.end(), YoungerFirst());
                h.pop_back();
                if (!h.empty())
                    top_push(h.front(), k);
            }
            if (keep) {
                out = e;
                return true;
            }
        }
        return false;
    }

private:
    struct Top {
        Entry e;
        uint32_t s;
    };
    struct TopYounger {
        bool operator()(const Top &a, const Top &b) const { return YoungerFirst()(a.e, b.e); }
    };
    void top_push(const Entry &e, uint32_t k)
    {
        top.push_back(Top{e, k});
        std::push_heap(top.begin(), top.end(), TopYounger());
    }
    void top_pop()
    {
        std::pop_heap(top.begin(), top.end(), TopYounger());
        top.pop_back();
    }
    std::vector<std::vector<Entry>> streams;
    size_t nstreams = 0;
    std::vector<Top> top;
    std::vector<uint32_t> hits;
};

struct Ctx {
    const ResidualProblem &P;
    int n, p;
    std::vector<Entry> scratch;
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

    // Every cofacet of sigma with diameter <= threshold.
    const std::vector<Entry> &coboundary(uint64_t sigma, float d)
    {
        scratch.clear();
        int v[8];
        decode(sigma, p, v);
        if (P.bits) {
            // common neighbours only: every new edge is within the threshold
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
                    scratch.push_back(Entry{nd, insert_index(v, w)});
                }
            }
            return scratch;
        }
        const float *rows[8];
        for (int i = 0; i <= p; ++i)
            rows[i] = P.dsq + (int64_t)v[i] * n;
        // cidx of sigma + {w}: vertices above w move up one rank.  Scan w
        // downward, keeping the two partial sums of the CNS formula.
        uint64_t above = 0;       // sum over v_i > w of C(v_i, rank+2)
        uint64_t below = sigma;   // sum over v_i < w of C(v_i, rank+1)
        int j = p + 1;            // number of sigma's vertices below w
        int nxt = 0;              // index (in v) of the next vertex at or below w
        for (int w = n - 1; w >= 0; --w) {
            if (nxt <= p && v[nxt] == w) {
                const int r = p - nxt;  // rank from the bottom
                below -= C(w, r + 1);
                above += C(w, r + 2);
                --j;
                ++nxt;
                continue;
            }
            float nd = d;
            bool ok = true;
            for (int i = 0; i <= p; ++i) {
                const float e = rows[i][w];
                if (!(e <= P.thr)) {
                    ok = false;
                    break;
                }
                nd = e > nd ? e : nd;
            }
            if (ok)
                scratch.push_back(Entry{nd, above + C(w, j + 1) + below});
        }
        return scratch;
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
// A small persistent worker pool for the speculative phase.
// ---------------------------------------------------------------------------
class Pool {
public:
    static Pool &get()
    {
        static Pool pool;
        return pool;
    }
    int size() const { return (int)workers_.size() + 1; }
    // Runs fn(tid) on every worker and on the calling thread (tid 0), and
    // returns when all have finished.  One caller at a time uses the
    // workers; a concurrent caller runs fn(0) alone on its own thread.
    void run(const std::function<void(int)> &fn)
    {
        std::unique_lock<std::mutex> owner(run_mu_, std::try_to_lock);
        if (workers_.empty() || !owner.owns_lock()) {
            fn(0);
            return;
        }
        {
            std::unique_lock<std::mutex> lk(mu_);
            job_ = &fn;
            pending_ = (int)workers_.size();
            ++epoch_;
        }
        cv_.notify_all();
        fn(0);
        std::unique_lock<std::mutex> lk(mu_);
        done_.wait(lk, [&] { return pending_ == 0; });
        job_ = nullptr;
    }

private:
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
            std::unique_lock<std::mutex> lk(mu_);
            stop_ = true;
            ++epoch_;
        }
        cv_.notify_all();
        for (auto &w : workers_)
            w.join();
    }
    void loop(int tid)
    {
        uint64_t seen = 0;
        while (true) {
            const std::function<void(int)> *job;
            {
                std::unique_lock<std::mutex> lk(mu_);
                cv_.wait(lk, [&] { return stop_ || epoch_ != seen; });
                if (stop_)
                    return;
                seen = epoch_;
                job = job_;
            }
            (*job)(tid);
            std::unique_lock<std::mutex> lk(mu_);
            if (--pending_ == 0)
                done_.notify_one();
        }
    }
    std::vector<std::thread> workers_;
    std::mutex run_mu_;
    std::mutex mu_;
    std::condition_variable cv_, done_;
    const std::function<void(int)> *job_ = nullptr;
    int pending_ = 0;
    uint64_t epoch_ = 0;
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
void residual_reduce(const ResidualProblem &P, ResidualResult &R)
{
    const int64_t ncols = P.ncols;
    std::vector<Entry> spec_low(ncols);
    std::vector<uint8_t> spec_nz(ncols, 0);
    std::vector<int64_t> spec_adds(ncols, 0);
    std::vector<std::unique_ptr<Column>> state(ncols);

    auto apparent_lookup = [&](const Ctx &X, uint64_t tau, float dt, uint64_t *other) -> bool {
        if (P.app_tau) {
            const uint64_t *b = P.app_tau, *e = P.app_tau + P.napp;
            const uint64_t *f = std::lower_bound(b, e, tau);
            if (f == e || *f != tau)
                return false;
            *other = P.app_sigma[f - b];
            return true;
        }
        return X.apparent_partner(tau, dt, other);
    };
    auto diam_of_key = [&](int64_t j) {
        return __builtin_bit_cast(float, (uint32_t)~(uint32_t)P.col_key[j]);
    };

    // ---- phase A ----------------------------------------------------------
    Pool &pool = Pool::get();
    const int workers = P.parallel ? pool.size() : 1;
    std::atomic<int64_t> next{0};
    std::atomic<int64_t> look_app{0};
    const int64_t chunk = std::max<int64_t>(1, std::min<int64_t>(16, ncols / (8 * workers)));
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
                std::unique_ptr<Column> col(new Column());
                col->add(X.coboundary(P.col_cidx[j], diam_of_key(j)));
                bool nz;
                int64_t adds = 0;
                while (true) {
                    // Algorithm 2: add the ORIGINAL column of the pivot's owner
                    // (an apparent column has the diameter of its tau)
                    col->add(X.coboundary(other, lo.diam));
                    ++adds;
                    nz = col->low(lo);
                    if (!nz)
                        break;
                    ++looks;
                    if (!apparent_lookup(X, lo.cidx, lo.diam, &other))
                        break;
                }
                spec_low[j] = lo;
                spec_nz[j] = nz ? 1 : 0;
                spec_adds[j] = adds;
                state[j] = std::move(col);
            }
        }
        look_app += looks;
    };
    if (P.parallel)
        pool.run(phase_a);
    else
        phase_a(0);
    R.lookups_apparent = look_app.load();

    // ---- phase B ----------------------------------------------------------
    // A finished column that needed additions keeps its heap state: its
    // streams hold its reduced column R_k, which a later column adds in one
    // step (the standard algorithm's R_j += R_k) instead of replaying k's
    // reduction from the original column.  The copied entries are a subset
    // of what the replay would regenerate, so this is never more work.
    Ctx X(P);
    std::unordered_map<uint64_t, int64_t> pivots;  // tau -> index in R.sigma
    pivots.reserve((size_t)ncols * 2 + 16);
    std::vector<std::unique_ptr<Column>> reduced;  // by index in R.sigma
    reduced.reserve((size_t)ncols);
    for (int64_t j = 0; j < ncols; ++j) {
        const uint64_t sigma = P.col_cidx[j];
        const float d = diam_of_key(j);
        int64_t adds = spec_adds[j];
        bool nz = spec_nz[j] != 0;
        Entry lo = spec_low[j];
        std::unique_ptr<Column> col = std::move(state[j]);
        if (nz) {
            auto it = pivots.find(lo.cidx);
            if (it != pivots.end()) {
                ++R.lookups_hash;
                if (!col) {
                    col.reset(new Column());
                    col->add(X.coboundary(sigma, d));
                }
                // owner of the current low: host column k, or apparent column
                int64_t k = it->second;
                bool host = true;
                uint64_t other = 0;
                while (true) {
                    if (!host)
                        col->add(X.coboundary(other, lo.diam));  // diameter of its tau
                    else if (reduced[k])
                        col->add(*reduced[k]);
                    else
                        col->add(X.coboundary(R.sigma[k], R.birth[k]));
                    ++adds;
                    nz = col->low(lo);
                    if (!nz)
                        break;
                    auto f = pivots.find(lo.cidx);
                    if (f != pivots.end()) {
                        ++R.lookups_hash;
                        k = f->second;
                        host = true;
                        continue;
                    }
                    ++R.lookups_apparent;
                    if (!apparent_lookup(X, lo.cidx, lo.diam, &other))
                        break;
                    host = false;
                }
            }
        }
        R.additions += adds;
        if (nz) {
            if (adds == 0)
                ++R.emergent;
            pivots.emplace(lo.cidx, (int64_t)R.sigma.size());
            R.sigma.push_back(sigma);
            R.tau.push_back(lo.cidx);
            R.birth.push_back(d);
            R.death.push_back(lo.diam);
            reduced.push_back(adds ? std::move(col) : nullptr);
        } else {
            R.ess_sigma.push_back(sigma);
            R.ess_birth.push_back(d);
        }
    }
}

}  // namespace rpp
