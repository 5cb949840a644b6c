// residual.cpp -- host reduction of the columns the GPU could not pair.
//
// Paper, "Reduction Matrix vs. Oblivious Matrix Reduction" (Algorithm 2)
// and "Core System Optimizations" (two-layer pair store).  Each column's
// coboundary is regenerated from the distance matrix (implicit matrix
// reduction) into a binary heap ordered oldest-first, so the heap top is
// the column's low.  Z/2 addition pushes the other column's entries; equal
// entries cancel in pairs when the low is taken.
#include "residual.h"

#include <algorithm>
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

class Column {
public:
    std::vector<Entry> heap;
    void clear() { heap.clear(); }
    void push(const Entry &e)
    {
        heap.push_back(e);
        std::push_heap(heap.begin(), heap.end(), YoungerFirst());
    }
    Entry pop()
    {
        std::pop_heap(heap.begin(), heap.end(), YoungerFirst());
        Entry e = heap.back();
        heap.pop_back();
        return e;
    }
    // Low of the column over Z/2: drop entries that occur an even number of
    // times at the top; leave the surviving low in the heap.
    bool low(Entry &out)
    {
        while (!heap.empty()) {
            Entry e = pop();
            int cnt = 1;
            while (!heap.empty() && heap.front().cidx == e.cidx) {
                pop();
                ++cnt;
            }
            if (cnt & 1) {
                push(e);
                out = e;
                return true;
            }
        }
        return false;
    }
};

struct Ctx {
    const ResidualProblem &P;
    int n, p;
    explicit Ctx(const ResidualProblem &pp) : P(pp), n(pp.n), p(pp.p) {}

    uint64_t C(int v, int k) const { return P.binom[(int64_t)k * (n + 1) + v]; }
    float D(int a, int b) const { return P.dsq[(int64_t)a * n + b]; }

    void decode(uint64_t c, int *v) const
    {
        int hi = n;
        for (int pos = 0; pos <= p; ++pos) {
            const int k = p + 1 - pos;
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

    // Push every cofacet of sigma with diameter <= threshold.
    void push_coboundary(uint64_t sigma, float d, Column &col) const
    {
        int v[8];
        decode(sigma, v);
        // cidx of sigma + {w}: vertices above w move up one rank.  Scan w
        // downward, keeping the two partial sums of the CNS formula.
        uint64_t above = 0;  // sum over v_i > w of C(v_i, rank+2)
        uint64_t below = sigma;  // sum over v_i < w of C(v_i, rank+1)
        int j = p + 1;       // number of sigma's vertices below w
        int nxt = 0;         // index (in v) of the next vertex at or below w
        for (int w = n - 1; w >= 0; --w) {
            if (nxt <= p && v[nxt] == w) {
                // w is a vertex of sigma: move it from "below" to "above"
                const int r = p - nxt;  // its rank from the bottom
                below -= C(w, r + 1);
                above += C(w, r + 2);
                --j;
                ++nxt;
                continue;
            }
            float nd = d;
            bool ok = true;
            for (int i = 0; i <= p; ++i) {
                const float e = D(w, v[i]);
                if (!(e <= P.thr)) {
                    ok = false;
                    break;
                }
                nd = e > nd ? e : nd;
            }
            if (!ok)
                continue;
            col.push(Entry{nd, above + C(w, j + 1) + below});
        }
    }
};

}  // namespace

void residual_reduce(const ResidualProblem &P, ResidualResult &R)
{
    Ctx X(P);
    std::unordered_map<uint64_t, int64_t> pivots;  // tau -> index in R.sigma
    pivots.reserve((size_t)P.ncols * 2 + 16);
    Column col;
    for (int64_t j = 0; j < P.ncols; ++j) {
        const uint64_t sigma = P.col_cidx[j];
        const float d = __builtin_bit_cast(float, (uint32_t)~(uint32_t)P.col_key[j]);
        col.clear();
        X.push_coboundary(sigma, d, col);
        Entry lo;
        bool nonzero = col.low(lo);
        while (nonzero) {
            // first layer: pairs found by this reduction
            auto it = pivots.find(lo.cidx);
            uint64_t other;
            float odiam;
            if (it != pivots.end()) {
                ++R.lookups_hash;
                other = R.sigma[it->second];
                odiam = R.birth[it->second];
            } else {
                // second layer: apparent pairs, sorted by tau
                const uint64_t *b = P.app_tau, *e = P.app_tau + P.napp;
                const uint64_t *f = std::lower_bound(b, e, lo.cidx);
                ++R.lookups_apparent;
                if (f == e || *f != lo.cidx)
                    break;  // low is free: (sigma, low) is a new pair
                other = P.app_sigma[f - b];
                odiam = lo.diam;  // an apparent column has the diameter of its tau
            }
            // Algorithm 2: add the ORIGINAL column of the pivot's owner
            X.push_coboundary(other, odiam, col);
            ++R.additions;
            nonzero = col.low(lo);
        }
        if (nonzero) {
            pivots.emplace(lo.cidx, (int64_t)R.sigma.size());
            R.sigma.push_back(sigma);
            R.tau.push_back(lo.cidx);
            R.birth.push_back(d);
            R.death.push_back(lo.diam);
        } else {
            R.ess_sigma.push_back(sigma);
            R.ess_birth.push_back(d);
        }
    }
}

}  // namespace rpp
