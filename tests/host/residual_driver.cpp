// Test driver for the host residual reduction (csrc/residual.cpp) on the
// CPU: it builds, by brute force, what the GPU stages hand to the host --
// the columns of each dimension with their clearing, the apparent pairs
// (apparent pairs lemma), the non-apparent columns in coboundary order
// (diameter desc, cidx asc) and their lows -- then reduces them with one of
// three schedules and prints every pair and essential class:
//   mode 0  residual_reduce, clearing by all pivots of the previous dimension
//   mode 1  the same with a speculative budget of 2 additions per column
//   mode 2  the overlapped schedule: clearing by the previous dimension's
//           apparent pivots only, its host pivots dropped at finish()
// Usage: residual_driver <file of n*(n-1)/2 float32> n maxdim thr mode
// Output lines: "P dim sigma tau" and "E dim sigma".
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <unordered_set>
#include <vector>

#include "../../paper_2003_07989_amd/csrc/residual.h"

using namespace rpp;

static int N;
static std::vector<uint64_t> B;   // C(v, k) at k * (N + 1) + v
static std::vector<float> Dsq;    // N x N

static uint64_t C(int v, int k) { return B[(size_t)k * (N + 1) + v]; }
static float D(int a, int b) { return Dsq[(size_t)a * N + b]; }

static void vertices(uint64_t c, int q, int *v)  // decreasing
{
    int hi = N;
    for (int pos = 0; pos <= q; ++pos) {
        const int k = q + 1 - pos;
        int x = k - 1;
        while (x + 1 < hi && C(x + 1, k) <= c)
            ++x;
        v[pos] = x;
        c -= C(x, k);
        hi = x;
    }
}

static uint64_t index_of(const int *v, int q)
{
    uint64_t c = 0;
    for (int i = 0; i <= q; ++i)
        c += C(v[i], q + 1 - i);
    return c;
}

static float diameter(const int *v, int q)
{
    float d = 0.0f;
    for (int a = 0; a <= q; ++a)
        for (int b = a + 1; b <= q; ++b)
            d = std::max(d, D(v[a], v[b]));
    return d;
}

// sigma + {w}, vertices decreasing
static int insert(const int *v, int q, int w, int *t)
{
    int k = 0;
    bool placed = false;
    for (int i = 0; i <= q; ++i) {
        if (!placed && w > v[i]) {
            t[k++] = w;
            placed = true;
        }
        t[k++] = v[i];
    }
    if (!placed)
        t[k++] = w;
    return k;
}

// Older in the filtration: smaller diameter, then larger cidx.
static bool older(float da, uint64_t ca, float db, uint64_t cb)
{
    return da != db ? da < db : ca > cb;
}

int main(int argc, char **argv)
{
    if (argc != 6)
        return 2;
    N = atoi(argv[2]);
    const int maxdim = atoi(argv[3]);
    float thr = (float)atof(argv[4]);
    // mode & 32: rank-coded diameters (below);
    // mode & 16: cofacets through neighbour bitsets (the sparse path);
    // mode & 3: schedule (0 plain, 1 speculative budget, 2 overlapped,
    // 3 overlapped with the dropped columns known late: columns park past
    // 2 additions, or with mode & 8 never, so dropped columns end at zero
    // before the gate opens);
    // mode & 4: oblivious additions; mode & 64 (with 16): packed rows
    const int mode = atoi(argv[5]);
    const int sched = mode & 3;
    const int n = N;
    const size_t m = (size_t)n * (n - 1) / 2;
    std::vector<float> dc(m);
    FILE *f = fopen(argv[1], "rb");
    if (!f || fread(dc.data(), 4, m, f) != m)
        return 3;
    fclose(f);
    Dsq.assign((size_t)n * n, 0.0f);
    for (int i = 1; i < n; ++i)
        for (int j = 0; j < i; ++j)
            Dsq[(size_t)i * n + j] = Dsq[(size_t)j * n + i] = dc[(size_t)i * (i - 1) / 2 + j];
    // Rank-coded diameters: every distance within the threshold becomes the
    // rank of its length among the distinct ones (as a float), larger ones a
    // rank above them all, and the threshold the top rank.  Every
    // comparison keeps its outcome, so pairs and classes must not change.
    int rank_bits = 0;
    if (mode & 32) {
        std::vector<float> vals;
        for (int i = 1; i < n; ++i)
            for (int j = 0; j < i; ++j)
                if (Dsq[(size_t)i * n + j] <= thr)
                    vals.push_back(Dsq[(size_t)i * n + j]);
        std::sort(vals.begin(), vals.end());
        vals.erase(std::unique(vals.begin(), vals.end()), vals.end());
        const float above = (float)vals.size();
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                float &x = Dsq[(size_t)i * n + j];
                if (i == j)
                    x = 0.0f;
                else if (x <= thr)
                    x = (float)(std::lower_bound(vals.begin(), vals.end(), x) - vals.begin());
                else
                    x = above;
            }
        thr = vals.empty() ? 0.0f : (float)(vals.size() - 1);
        while ((1u << rank_bits) <= vals.size())
            ++rank_bits;
    }
    const int K = maxdim + 2;
    B.assign((size_t)(K + 1) * (n + 1), 0);
    for (int k = 0; k <= K; ++k)
        for (int v = 0; v <= n; ++v)
            B[(size_t)k * (n + 1) + v] =
                k == 0 ? 1 : (v == 0 ? 0 : C(v - 1, k - 1) + C(v - 1, k));

    // dimension 0 by Kruskal (edges in filtration order): the MST edges
    // are dimension 1's clearing set
    std::unordered_set<uint64_t> clear;
    {
        std::vector<std::pair<float, uint64_t>> e;
        for (uint64_t c = 0; c < m; ++c) {
            int v[2];
            vertices(c, 1, v);
            if (D(v[0], v[1]) <= thr)
                e.push_back({D(v[0], v[1]), c});
        }
        std::sort(e.begin(), e.end(), [](const auto &a, const auto &b) {
            return older(a.first, a.second, b.first, b.second);
        });
        std::vector<int> par(n);
        for (int i = 0; i < n; ++i)
            par[i] = i;
        auto root = [&](int x) {
            while (par[x] != x)
                x = par[x] = par[par[x]];
            return x;
        };
        for (auto &x : e) {
            int v[2];
            vertices(x.second, 1, v);
            const int a = root(v[0]), b = root(v[1]);
            if (a != b) {
                par[std::max(a, b)] = std::min(a, b);
                clear.insert(x.second);
            }
        }
    }

    std::vector<uint64_t> prev_host;  // host pivots of the previous dimension
    for (int p = 1; p <= maxdim; ++p) {
        // columns: p-simplices within the threshold, not cleared
        std::vector<float> cd;
        std::vector<uint64_t> cc;
        for (uint64_t c = 0; c < C(n, p + 1); ++c) {
            int v[8];
            vertices(c, p, v);
            const float d = diameter(v, p);
            if (d <= thr && !clear.count(c)) {
                cd.push_back(d);
                cc.push_back(c);
            }
        }
        // apparent pairs: the oldest cofacet tau of sigma has the same
        // diameter and sigma is tau's youngest facet
        std::vector<uint64_t> app_tau(cc.size(), ~0ull);
        for (size_t i = 0; i < cc.size(); ++i) {
            int v[8], t[9], fv[8];
            vertices(cc[i], p, v);
            bool have = false;
            float bd = 0.0f;
            uint64_t bc = 0;
            for (int w = 0; w < n; ++w) {
                bool in = false;
                for (int a = 0; a <= p; ++a)
                    in |= v[a] == w;
                if (in)
                    continue;
                insert(v, p, w, t);
                const float d = diameter(t, p + 1);
                const uint64_t c = index_of(t, p + 1);
                if (d <= thr && (!have || older(d, c, bd, bc))) {
                    have = true;
                    bd = d;
                    bc = c;
                }
            }
            if (!have || bd != cd[i])
                continue;
            vertices(bc, p + 1, t);
            float yd = -1.0f;
            uint64_t yc = 0;
            for (int drop = 0; drop <= p + 1; ++drop) {
                int k = 0;
                for (int a = 0; a <= p + 1; ++a)
                    if (a != drop)
                        fv[k++] = t[a];
                const float d = diameter(fv, p);
                const uint64_t c = index_of(fv, p);
                if (yd < 0.0f || older(yd, yc, d, c)) {
                    yd = d;
                    yc = c;
                }
            }
            if (yc == cc[i])
                app_tau[i] = bc;
        }
        // non-apparent columns in coboundary order, with their lows
        std::vector<size_t> na;
        for (size_t i = 0; i < cc.size(); ++i)
            if (app_tau[i] == ~0ull)
                na.push_back(i);
        std::stable_sort(na.begin(), na.end(), [&](size_t a, size_t b) { return cd[a] > cd[b]; });
        std::vector<uint64_t> key, cid, low;
        std::vector<float> lowd;
        for (size_t i : na) {
            uint32_t bits;
            memcpy(&bits, &cd[i], 4);
            key.push_back((uint64_t)(uint32_t)~bits);
            cid.push_back(cc[i]);
            int v[8], t[9];
            vertices(cc[i], p, v);
            bool have = false;
            float bd = 0.0f;
            uint64_t bc = 0;
            for (int w = 0; w < n; ++w) {
                bool in = false;
                for (int a = 0; a <= p; ++a)
                    in |= v[a] == w;
                if (in)
                    continue;
                insert(v, p, w, t);
                const float d = diameter(t, p + 1);
                const uint64_t c = index_of(t, p + 1);
                if (d <= thr && (!have || older(d, c, bd, bc))) {
                    have = true;
                    bd = d;
                    bc = c;
                }
            }
            low.push_back(have ? bc : ~0ull);
            lowd.push_back(have ? bd : INFINITY);
        }
        int64_t napp = 0;
        for (size_t i = 0; i < cc.size(); ++i)
            napp += app_tau[i] != ~0ull;
        ResidualProblem P;
        P.n = n;
        P.p = p;
        P.thr = thr;
        P.dsq = Dsq.data();
        P.binom = B.data();
        P.ncols = (int64_t)cid.size();
        P.col_key = key.data();
        P.col_cidx = cid.data();
        P.col_low = low.data();
        P.col_low_diam = lowd.data();
        P.napp = napp;
        P.rank_bits = rank_bits;
        // mode & 16: cofacets from neighbour bitsets (the sparse path);
        // mode & 64 as well: distances from packed neighbour rows only (the
        // square matrix is withheld)
        std::vector<uint64_t> bits;
        std::vector<uint32_t> npre;
        std::vector<float> nbd;
        if (mode & 16) {
            const int words = (n + 63) / 64;
            bits.assign((size_t)n * words, 0);
            for (int a = 0; a < n; ++a)
                for (int b = 0; b < n; ++b)
                    if (a != b && D(a, b) <= thr)
                        bits[(size_t)a * words + b / 64] |= 1ull << (b % 64);
            P.bits = bits.data();
            P.words = words;
            if (mode & 64) {
                npre.assign((size_t)n * words, 0);
                uint32_t run = 0;
                for (size_t k = 0; k < (size_t)n * words; ++k) {
                    npre[k] = run;
                    run += (uint32_t)__builtin_popcountll(bits[k]);
                }
                for (int a = 0; a < n; ++a)
                    for (int b = 0; b < n; ++b)
                        if (a != b && D(a, b) <= thr)
                            nbd.push_back(D(a, b));
                P.npre = npre.data();
                P.nbd = nbd.data();
                P.dsq = nullptr;
            }
        }
        P.spec_budget = sched >= 1 ? 2 : 0;
        P.oblivious = (mode & 4) != 0;
        // RPP_TEST_PARK_SLICE: additions per slice of a parked column while
        // the gate is closed (0: parked columns wait idle)
        if (const char *e = getenv("RPP_TEST_PARK_SLICE"))
            P.park_slice = atoll(e);
        // RPP_TEST_KEEP_RATIO: add D_k for kept R_k holding more than this
        // many times D_k's keys (0: always R_k)
        if (const char *e = getenv("RPP_TEST_KEEP_RATIO"))
            P.keep_ratio = atof(e);
        ResidualResult R;
        if (sched >= 2) {
            std::unordered_set<uint64_t> ph(prev_host.begin(), prev_host.end());
            std::vector<uint8_t> drop(cid.size(), 0);
            for (size_t j = 0; j < cid.size(); ++j)
                drop[j] = ph.count(cid[j]) ? 1 : 0;
            if (sched == 2) {
                residual_speculate(P)->finish(drop.data(), R);
            } else {
                // the dropped columns become known only after a few polls:
                // the reduction runs open, parks columns past 2 additions,
                // and classifies its zero columns late
                // (RPP_TEST_GATE_POLLS of them, default 5)
                struct Late final : DropGate {
                    const uint8_t *d;
                    int polls = 0, after = 5;
                    bool ready() override { return ++polls > after; }
                    const uint8_t *wait() override { return d; }
                } gate;
                gate.d = drop.data();
                if (const char *e = getenv("RPP_TEST_GATE_POLLS"))
                    gate.after = atoi(e);
                residual_speculate(P)->finish_gated(gate, (mode & 8) ? 1000000 : 2, R);
            }
        } else {
            residual_reduce(P, R);
        }
        for (size_t i = 0; i < cc.size(); ++i)
            if (app_tau[i] != ~0ull)
                printf("P %d %llu %llu\n", p, (unsigned long long)cc[i],
                       (unsigned long long)app_tau[i]);
        for (size_t i = 0; i < R.sigma.size(); ++i)
            printf("P %d %llu %llu\n", p, (unsigned long long)R.sigma[i],
                   (unsigned long long)R.tau[i]);
        for (uint64_t e : R.ess_sigma)
            printf("E %d %llu\n", p, (unsigned long long)e);
        printf("A %d %lld\n", p, (long long)R.additions);
        // next clearing set: apparent pivots always; host pivots unless the
        // overlapped schedule drops them instead
        clear.clear();
        for (size_t i = 0; i < cc.size(); ++i)
            if (app_tau[i] != ~0ull)
                clear.insert(app_tau[i]);
        if (sched < 2)
            for (uint64_t t : R.tau)
                clear.insert(t);
        prev_host = R.tau;
    }
    return 0;
}
