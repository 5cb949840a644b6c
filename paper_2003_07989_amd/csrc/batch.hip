// batch.hip -- many clouds of one shape through the hot path together.
//
// B clouds of n points (same maxdim) are packed cloud after cloud.  Every
// GPU stage is ONE launch over all clouds (cloud = blockIdx.y, or one
// workgroup per cloud for Kruskal) with buffers sized by capacity and the
// per-cloud counts kept in device memory, so a dimension's whole GPU chain
// has a fixed shape: it is captured once into a hipGraph per (shape, tuned
// parameters) and replayed for every later batch of that shape.  After the
// chain, the non-apparent columns of all clouds are packed on the device
// and copied back in one transfer; the per-cloud host reductions run in
// parallel on the worker pool.  The lane-group size of the apparent kernel
// is chosen per (n, p) by timing the candidates on the first batch
// (optionally persisted in the JSON file named by RPP_TUNE_CACHE), with
// the rounds per wave and the workgroup size.
#include "host_common.h"
#include "kernels.h"
#include "pipeline.h"
#include "residual.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <map>
#include <memory>
#include <mutex>
#include <tuple>

namespace rpp {

// ---------------------------------------------------------------------------
// small batch-only kernels
// ---------------------------------------------------------------------------
__global__ void k_copy_u64(const uint64_t *__restrict__ a, uint64_t *__restrict__ b, int64_t m)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m)
        b[i] = a[i];
}

__global__ void k_fill_u64(uint64_t *__restrict__ a, int64_t m, uint64_t v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m)
        a[i] = v;
}

// out[c] = a[c * sa] - b[c * sb]
__global__ void k_sub_counts(const uint64_t *__restrict__ a, int64_t sa,
                             const uint64_t *__restrict__ b, int64_t sb, uint64_t *__restrict__ out,
                             int nb)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < nb)
        out[c] = a[(int64_t)c * sa] - b[(int64_t)c * sb];
}

// Gather each cloud's first count[c] entries (arrays strided by cap) to
// packed positions off[c] .. off[c] + count[c].
__global__ void k_pack(const uint64_t *__restrict__ key, const uint64_t *__restrict__ cidx,
                       const uint64_t *__restrict__ low, const float *__restrict__ lowd,
                       const uint64_t *__restrict__ count, const uint64_t *__restrict__ off,
                       int64_t cap, uint64_t *__restrict__ pkey, uint64_t *__restrict__ pcidx,
                       uint64_t *__restrict__ plow, float *__restrict__ plowd)
{
    const int64_t c = blockIdx.y;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)count[c])
        return;
    const int64_t src = c * cap + i, dst = (int64_t)off[c] + i;
    pkey[dst] = key[src];
    pcidx[dst] = cidx[src];
    plow[dst] = low[src];
    plowd[dst] = lowd[src];
}

// bits[cloud[i] * stride + t/32] |= bit of t, t = idx[i]
__global__ void k_mark_bits_cloud(const uint64_t *__restrict__ idx,
                                  const int32_t *__restrict__ cloud, int64_t m,
                                  uint32_t *__restrict__ bits, int64_t stride)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) {
        const uint64_t t = idx[i];
        atomicOr(&bits[(int64_t)cloud[i] * stride + (int64_t)(t >> 5)], 1u << (t & 31));
    }
}

static unsigned blocks_for(int64_t m)
{
    return (unsigned)((m + 255) / 256);
}

// ---------------------------------------------------------------------------
// autotuner cache: (n, p) -> launch configuration of the apparent kernel,
// one code: G + 100 R + 10000 B, with G lanes per column, R rounds of
// 64/G columns per wave (0: chosen from the column count) and B wavefronts
// per workgroup (0: four, i.e. 256 threads)
// ---------------------------------------------------------------------------
struct AppCfg {
    int group, rounds, block;
};
static AppCfg app_cfg(int code)
{
    const int b = (code / 10000) % 10;
    return {code % 100, (code / 100) % 100, b ? b * 64 : 256};
}
static std::mutex g_tune_mu;
static std::map<std::pair<int, int>, int> g_tune;
static bool g_tune_loaded = false;

static void tune_load_locked()
{
    if (g_tune_loaded)
        return;
    g_tune_loaded = true;
    const char *path = getenv("RPP_TUNE_CACHE");
    if (!path)
        return;
    FILE *f = fopen(path, "r");
    if (!f)
        return;
    // format: {"n:p": code, ...} (code as app_cfg reads it)
    int n, p, g;
    int ch;
    while ((ch = fgetc(f)) != EOF) {
        if (ch == '"' && fscanf(f, "%d:%d\": %d", &n, &p, &g) == 3)
            g_tune[{n, p}] = g;
    }
    fclose(f);
}

static void tune_store_locked()
{
    const char *path = getenv("RPP_TUNE_CACHE");
    if (!path)
        return;
    FILE *f = fopen(path, "w");
    if (!f)
        return;
    fputc('{', f);
    bool first = true;
    for (auto &kv : g_tune) {
        fprintf(f, "%s\"%d:%d\": %d", first ? "" : ", ", kv.first.first, kv.first.second,
                kv.second);
        first = false;
    }
    fputs("}\n", f);
    fclose(f);
}

int tuned_group(int n, int p)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_load_locked();
    auto it = g_tune.find({n, p});
    return it == g_tune.end() ? 0 : it->second;
}

// ---------------------------------------------------------------------------
// batch workspace and captured graphs, per shape
// ---------------------------------------------------------------------------
struct BatchWs {
    std::mutex mu;
    int n = 0, maxdim = 0, nb = 0;
    DevBuf dcond, dsq, rowmax, bad, radius, thr_req, thr;
    DevBuf nv;                             // each cloud's own number of points (bucket)
    DevBuf binom;
    DevBuf stats;                          // 2 u64 per cloud per stage
    DevBuf tcount, toff, scan;             // compaction
    DevBuf tcount2, toff2;                 // partition
    DevBuf cdiam, ccidx, tau;
    DevBuf ekey, eval, ekey2, eval2;
    DevBuf akey, aval, akey2, aval2;
    DevBuf nkey, nval, nkey2, nval2, nna;
    DevBuf lowc, lowd;
    DevBuf mst, bits[2];                   // clearing bitmaps: dim p reads bits[p & 1]
    int na_where = 0;                      // sorted non-apparent columns in nkey (0) or nkey2
    DevBuf deaths, dedges, counters, ufs;
    DevBuf rscratch;
    DevBuf poff, pkey, pcidx, plow, plowd;  // packed non-apparent columns
    DevBuf hidx, hcloud;                   // host pivots for the next clearing set
    HostBuf h_dsq;                         // pinned host copies of the square matrices
    std::vector<uint64_t> binom_host;
    std::map<std::tuple<int, int>, hipGraphExec_t> graphs;  // (p, group) -> graph
    // The batch runs on its own stream (the caller's may be the null stream,
    // which cannot be captured), ordered after the caller's stream.
    hipStream_t own = nullptr;
    hipEvent_t ready = nullptr;
    int in_use = 0;          // callers holding it (guarded by g_bws_mu)
    uint64_t last_use = 0;   // for least-recently-used eviction
    ~BatchWs()
    {
        for (auto &kv : graphs)
            (void)hipGraphExecDestroy(kv.second);
        if (ready)
            (void)hipEventDestroy(ready);
        if (own)
            (void)hipStreamDestroy(own);
    }
};

static std::mutex g_bws_mu;
static std::map<std::tuple<int, int, int, int>, BatchWs *> g_bws;

// At most this many batch workspaces are cached per device; beyond it the
// least recently used idle one is freed (a stream of many shapes would
// otherwise keep every shape's capacity-sized arenas).
constexpr size_t BATCH_CACHE_ENTRIES = 4;
static uint64_t g_bws_clock = 0;

// The workspace for a shape, marked in use until batch_ws_release.
static BatchWs *batch_ws_acquire(int n, int maxdim, int nb)
{
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::vector<BatchWs *> victims;
    BatchWs *w;
    {
        std::lock_guard<std::mutex> lk(g_bws_mu);
        BatchWs *&slot = g_bws[{dev, n, maxdim, nb}];
        if (!slot) {
            slot = new BatchWs();
            slot->n = n;
            slot->maxdim = maxdim;
            slot->nb = nb;
        }
        w = slot;
        ++w->in_use;
        w->last_use = ++g_bws_clock;
        while (true) {
            size_t count = 0;
            auto lru = g_bws.end();
            for (auto it = g_bws.begin(); it != g_bws.end(); ++it) {
                if (std::get<0>(it->first) != dev)
                    continue;
                ++count;
                if (it->second->in_use == 0 &&
                    (lru == g_bws.end() || it->second->last_use < lru->second->last_use))
                    lru = it;
            }
            if (count <= BATCH_CACHE_ENTRIES || lru == g_bws.end())
                break;
            victims.push_back(lru->second);
            g_bws.erase(lru);
        }
    }
    for (BatchWs *v : victims)
        delete v;  // idle and unreachable: frees its buffers, graphs and stream
    return w;
}

static void batch_ws_release(BatchWs *w)
{
    std::lock_guard<std::mutex> lk(g_bws_mu);
    --w->in_use;
}

// Sizes of one dimension's stage.
struct DimShape {
    int p;
    int64_t cap;        // C(n, p+1): per-cloud capacity
    int64_t tiles;      // compaction tiles per cloud
    int64_t words;      // u32 words of this dimension's clearing bitmap
    int64_t next_words; // u32 words of the next dimension's bitmap (0 at the top)
};

static DimShape dim_shape(int n, int p, int maxdim)
{
    DimShape d;
    d.p = p;
    d.cap = (int64_t)binom_sat(n, p + 1);
    d.tiles = compact_tiles(d.cap);
    d.words = d.cap / 32 + 1;
    d.next_words = p < maxdim ? (int64_t)binom_sat(n, p + 2) / 32 + 1 : 0;
    return d;
}

// Allocate every buffer at its capacity (once per shape).
static int batch_alloc(BatchWs &W, std::string &err)
{
    const int n = W.n, nb = W.nb;
    const int64_t E = (int64_t)n * (n - 1) / 2;
    int64_t cap = E;
    for (int p = 2; p <= W.maxdim; ++p)
        cap = std::max<int64_t>(cap, (int64_t)binom_sat(n, p + 1));
    const int64_t tiles = compact_tiles(cap);
    const int64_t words = cap / 32 + 1;
    int64_t nwords = 0;
    for (int p = 1; p < W.maxdim; ++p)
        nwords = std::max<int64_t>(nwords, (int64_t)binom_sat(n, p + 2) / 32 + 1);
    const size_t B = (size_t)nb;
    ALLOC_TRY(W.dcond, B * E * 4 + 4);
    ALLOC_TRY(W.nv, B * 4);
    ALLOC_TRY(W.dsq, B * n * n * 4);
    ALLOC_TRY(W.rowmax, B * n * 4);
    ALLOC_TRY(W.bad, B * 4);
    ALLOC_TRY(W.radius, B * 4);
    ALLOC_TRY(W.thr_req, B * 4);
    ALLOC_TRY(W.thr, B * 4);
    ALLOC_TRY(W.stats, B * 2 * 8 * (W.maxdim + 1));
    ALLOC_TRY(W.tcount, B * (tiles + 1) * 4);
    ALLOC_TRY(W.toff, B * (tiles + 2) * 8);
    ALLOC_TRY(W.tcount2, B * (tiles + 1) * 4);
    ALLOC_TRY(W.toff2, B * (tiles + 2) * 8);
    ALLOC_TRY(W.scan, B * scan_scratch_words(tiles) * 8);
    ALLOC_TRY(W.cdiam, B * cap * 4);
    ALLOC_TRY(W.ccidx, B * cap * 8);
    ALLOC_TRY(W.tau, B * cap * 8);
    ALLOC_TRY(W.ekey, B * E * 8);
    ALLOC_TRY(W.eval, B * E * 8);
    ALLOC_TRY(W.ekey2, B * E * 8);
    ALLOC_TRY(W.eval2, B * E * 8);
    ALLOC_TRY(W.akey, B * cap * 8);
    ALLOC_TRY(W.aval, B * cap * 8);
    ALLOC_TRY(W.nkey, B * cap * 8);
    ALLOC_TRY(W.nval, B * cap * 8);
    ALLOC_TRY(W.nkey2, B * cap * 8);
    ALLOC_TRY(W.nval2, B * cap * 8);
    ALLOC_TRY(W.nna, B * 8);
    ALLOC_TRY(W.lowc, B * cap * 8);
    ALLOC_TRY(W.lowd, B * cap * 4);
    ALLOC_TRY(W.mst, B * (E / 32 + 1) * 4);
    ALLOC_TRY(W.bits[0], B * std::max<int64_t>(words, nwords) * 4 + 4);
    ALLOC_TRY(W.bits[1], B * std::max<int64_t>(words, nwords) * 4 + 4);
    ALLOC_TRY(W.deaths, B * n * 4);
    ALLOC_TRY(W.dedges, B * n * 8);
    ALLOC_TRY(W.counters, B * 2 * 4);
    ALLOC_TRY(W.ufs, B * 2 * n * 4);
    ALLOC_TRY(W.rscratch, (size_t)radix_scratch_words(cap, nb) * 8);
    ALLOC_TRY(W.poff, (B + 1) * 8);
    HIP_TRY(hipStreamCreateWithFlags(&W.own, hipStreamNonBlocking));
    HIP_TRY(hipEventCreateWithFlags(&W.ready, hipEventDisableTiming));
    W.binom_host = binomial_table(n, W.maxdim + 2);
    ALLOC_TRY(W.binom, W.binom_host.size() * 8);
    HIP_TRY(hipMemcpy(W.binom.p, W.binom_host.data(), W.binom_host.size() * 8,
                      hipMemcpyHostToDevice));
    return RPP_OK;
}

// The apparent kernel of dimension p over the batch's kept columns, with the
// launch configuration `code` (see app_cfg).
static void launch_apparent(BatchWs &W, const DimShape &D, const Batch &bk, int code,
                            hipStream_t s)
{
    const AppCfg ac = app_cfg(code);
    launch_apparent_b(W.cdiam.as<float>(), W.ccidx.as<uint64_t>(), D.cap, W.dsq.as<float>(), W.n,
                      D.p, W.binom.as<uint64_t>(), ac.group, W.tau.as<uint64_t>(), bk, W.nb, s,
                      ac.rounds, ac.block);
}

// The GPU chain of dimension p (and, for p == 1, the staging and H0 stages
// in front of it).  Fixed shape: suitable for graph capture.  No memset.
static void enqueue_dim(BatchWs &W, const DimShape &D, int group, uint32_t flags, hipStream_t s)
{
    const int n = W.n, nb = W.nb, p = D.p;
    const int64_t E = (int64_t)n * (n - 1) / 2;
    const uint64_t *binom = W.binom.as<uint64_t>();
    unsigned long long *stats = W.stats.as<unsigned long long>() + (size_t)2 * nb * p;
    if (p == 1) {
        hipLaunchKernelGGL(k_fill_u64, dim3(blocks_for(nb)), dim3(256), 0, s,
                           reinterpret_cast<uint64_t *>(W.bad.p), (int64_t)(nb + 1) / 2, 0ull);
        // bucket padding: the edges of each cloud's padding vertices at +inf
        launch_pad_dcond_b(W.dcond.as<float>(), n, nb, W.nv.as<int32_t>(), s);
        launch_stage_b(W.dcond.as<float>(), n, nb, W.dsq.as<float>(), W.rowmax.as<float>(),
                       W.bad.as<uint32_t>(), s, W.nv.as<int32_t>());
        launch_radius_b(W.rowmax.as<float>(), n, nb, W.thr_req.as<float>(),
                        (flags & RPP_NO_ENCLOSING_RADIUS) ? 1 : 0, W.radius.as<float>(),
                        W.thr.as<float>(), s, W.nv.as<int32_t>());
        // H0: edges <= thr per cloud, sorted, Kruskal (one workgroup each)
        unsigned long long *st0 = W.stats.as<unsigned long long>();
        hipLaunchKernelGGL(k_fill_u64, dim3(blocks_for(2 * nb)), dim3(256), 0, s,
                           reinterpret_cast<uint64_t *>(st0), (int64_t)2 * nb, 0ull);
        EnumArgs ea{W.dcond.as<float>(), n, 1, 0.0f, binom, nullptr, (uint64_t)E};
        ea.thr_dev = W.thr.as<float>();
        ea.out_stride = E;
        ea.nbatch = nb;
        const int64_t t1 = compact_tiles(E);
        launch_enum_count(ea, W.tcount.as<uint32_t>(), st0, s);
        launch_exclusive_scan_b(W.tcount.as<uint32_t>(), t1, nb, W.toff.as<uint64_t>(),
                                W.scan.as<uint64_t>(), s);
        launch_enum_scatter(ea, W.toff.as<uint64_t>(), W.cdiam.as<float>(), W.ccidx.as<uint64_t>(),
                            s);
        Batch be{W.toff.as<uint64_t>() + t1, t1 + 1, E, W.nv.as<int32_t>()};
        launch_desc_keys(W.cdiam.as<float>(), E, W.ekey.as<uint64_t>(), s, be, nb);
        hipLaunchKernelGGL(k_copy_u64, dim3(blocks_for((int64_t)nb * E)), dim3(256), 0, s,
                           W.ccidx.as<uint64_t>(), W.eval.as<uint64_t>(), (int64_t)nb * E);
        const int w = radix_sort_pairs_b(W.ekey.as<uint64_t>(), W.eval.as<uint64_t>(),
                                         W.ekey2.as<uint64_t>(), W.eval2.as<uint64_t>(), E, 32,
                                         W.rscratch.as<uint64_t>(), s, be, nb);
        const uint64_t *sk = w ? W.ekey2.as<uint64_t>() : W.ekey.as<uint64_t>();
        const uint64_t *sv = w ? W.eval2.as<uint64_t>() : W.eval.as<uint64_t>();
        const int64_t mw = E / 32 + 1;
        launch_fill_u32(W.mst.as<uint32_t>(), (int64_t)nb * mw, 0u, s);
        launch_kruskal(sk, sv, E, n, W.mst.as<uint32_t>(), W.deaths.as<float>(),
                       W.dedges.as<uint64_t>(), W.counters.as<int>(), W.ufs.as<int>(), s, be, nb,
                       mw);
    }
    // ---- dimension p: enumerate, apparent test, partition, sort, lows ----
    hipLaunchKernelGGL(k_fill_u64, dim3(blocks_for(2 * nb)), dim3(256), 0, s,
                       reinterpret_cast<uint64_t *>(stats), (int64_t)2 * nb, 0ull);
    const uint32_t *clear = (p == 1) ? W.mst.as<uint32_t>() : W.bits[p & 1].as<uint32_t>();
    uint32_t *next = W.bits[(p + 1) & 1].as<uint32_t>();
    EnumArgs ea{W.dcond.as<float>(), n, p, 0.0f, binom, clear, (uint64_t)D.cap};
    ea.thr_dev = W.thr.as<float>();
    ea.clear_stride = (p == 1) ? E / 32 + 1 : D.words;
    ea.out_stride = D.cap;
    ea.nbatch = nb;
    launch_enum_count(ea, W.tcount.as<uint32_t>(), stats, s);
    launch_exclusive_scan_b(W.tcount.as<uint32_t>(), D.tiles, nb, W.toff.as<uint64_t>(),
                            W.scan.as<uint64_t>(), s);
    launch_enum_scatter(ea, W.toff.as<uint64_t>(), W.cdiam.as<float>(), W.ccidx.as<uint64_t>(), s);
    Batch bk{W.toff.as<uint64_t>() + D.tiles, D.tiles + 1, D.cap, W.nv.as<int32_t>()};  // kept per cloud
    launch_apparent(W, D, bk, group, s);
    launch_partition_count(W.tau.as<uint64_t>(), D.cap, W.tcount2.as<uint32_t>(), s, bk, nb);
    launch_exclusive_scan_b(W.tcount2.as<uint32_t>(), D.tiles, nb, W.toff2.as<uint64_t>(),
                            W.scan.as<uint64_t>(), s);
    launch_partition_scatter(W.tau.as<uint64_t>(), W.cdiam.as<float>(), W.ccidx.as<uint64_t>(),
                             D.cap, W.toff2.as<uint64_t>(), W.akey.as<uint64_t>(),
                             W.aval.as<uint64_t>(), W.nkey.as<uint64_t>(), W.nval.as<uint64_t>(),
                             s, bk, nb);
    Batch ba{W.toff2.as<uint64_t>() + D.tiles, D.tiles + 1, D.cap};  // apparent per cloud
    hipLaunchKernelGGL(k_sub_counts, dim3(blocks_for(nb)), dim3(256), 0, s,
                       W.toff.as<uint64_t>() + D.tiles, D.tiles + 1,
                       W.toff2.as<uint64_t>() + D.tiles, D.tiles + 1, W.nna.as<uint64_t>(), nb);
    Batch bn{W.nna.as<uint64_t>(), 1, D.cap};  // non-apparent per cloud
    if (D.next_words) {
        launch_fill_u32(next, (int64_t)nb * D.next_words, 0u, s);
        launch_mark_bits(W.akey.as<uint64_t>(), D.cap, next, s, ba, nb, D.next_words);
    }
    const int wn = radix_sort_pairs_b(W.nkey.as<uint64_t>(), W.nval.as<uint64_t>(),
                                      W.nkey2.as<uint64_t>(), W.nval2.as<uint64_t>(), D.cap, 32,
                                      W.rscratch.as<uint64_t>(), s, bn, nb);
    W.na_where = wn;
    const uint64_t *nk = wn ? W.nkey2.as<uint64_t>() : W.nkey.as<uint64_t>();
    const uint64_t *nv = wn ? W.nval2.as<uint64_t>() : W.nval.as<uint64_t>();
    launch_lows(nk, nv, D.cap, W.dsq.as<float>(), n, p, 0.0f, binom, W.lowc.as<uint64_t>(),
                W.lowd.as<float>(), s, bn, nb, W.thr.as<float>());
}

// Where the last enqueued chain left the sorted non-apparent columns (the
// number of sort passes is fixed by the shape, so the same for replays).
static void sorted_na(BatchWs &W, const uint64_t **nk, const uint64_t **nv)
{
    *nk = W.na_where ? W.nkey2.as<uint64_t>() : W.nkey.as<uint64_t>();
    *nv = W.na_where ? W.nval2.as<uint64_t>() : W.nval.as<uint64_t>();
}

static int launch_dim(BatchWs &W, const DimShape &D, int group, uint32_t flags, bool use_graph,
                      hipStream_t s, std::string &err)
{
    if (!use_graph) {
        enqueue_dim(W, D, group, flags, s);
        HIP_TRY(hipGetLastError());
        return RPP_OK;
    }
    auto key = std::make_tuple(D.p, group * 2 + ((flags & RPP_NO_ENCLOSING_RADIUS) ? 1 : 0));
    auto it = W.graphs.find(key);
    if (it == W.graphs.end()) {
        hipGraph_t g;
        HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        enqueue_dim(W, D, group, flags, s);
        HIP_TRY(hipStreamEndCapture(s, &g));
        hipGraphExec_t ex;
        hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        HIP_TRY(e);
        it = W.graphs.emplace(key, ex).first;
    }
    HIP_TRY(hipGraphLaunch(it->second, s));
    return RPP_OK;
}

// Tune the apparent kernel's launch on the current batch: after one run of
// the dimension's chain (its kept columns in place), time the kernel alone
// (eager, once to warm and once timed; it only rewrites tau) for every lane
// count G in {4, 8, 16, 32}, rounds per wave R in {chosen from the column
// count, 1, 2, 4, 8} (R <= G) and workgroup size in {64, 128, 256}, and keep
// the fastest for (n, p).
static int autotune(BatchWs &W, const DimShape &D, uint32_t flags, hipStream_t s, int *best,
                    std::string &err)
{
    enqueue_dim(W, D, 8, flags, s);
    HIP_TRY(hipGetLastError());
    Batch bk{W.toff.as<uint64_t>() + D.tiles, D.tiles + 1, D.cap, W.nv.as<int32_t>()};
    float best_ms = 1e30f;
    *best = 8;
    for (int g : {4, 8, 16, 32})
        for (int r : {0, 1, 2, 4, 8}) {
            if (r > g)
                continue;
            for (int bw : {4, 1, 2}) {  // wavefronts per workgroup (4: code 0)
                const int code = g + 100 * r + (bw == 4 ? 0 : 10000 * bw);
                GpuTimer t(s);
                launch_apparent(W, D, bk, code, s);  // warm
                t.start();
                launch_apparent(W, D, bk, code, s);
                t.stop();
                HIP_TRY(hipGetLastError());
                const float ms = t.ms();
                if (ms < best_ms) {
                    best_ms = ms;
                    *best = code;
                }
            }
        }
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[{W.n, D.p}] = *best;
    tune_store_locked();
    return RPP_OK;
}

int run_batch(const BatchArgs &a, std::vector<RunOut> &outs, std::string &err)
{
    const int nb = a.count, n = a.n, maxdim = a.maxdim;
    outs.assign(nb, RunOut());
    for (auto &o : outs)
        o.dims.assign(maxdim + 1, DimOut());
    if (nb == 0)
        return RPP_OK;
    if (n < 2 || maxdim < 1) {
        // nothing batched to gain: run one by one
        for (int c = 0; c < nb; ++c) {
            RunArgs r;
            hipStream_t s = a.stream;
            r.dcond_dev = a.dist_dev[c];
            r.n = a.nv ? a.nv[c] : n;
            r.maxdim = maxdim;
            r.threshold = a.threshold[c];
            r.flags = a.flags | RPP_FORCE_DENSE;
            r.stream = s;
            int rc = run_pipeline(r, outs[c], err);
            if (rc)
                return rc;
        }
        return RPP_OK;
    }
    BatchWs *Wp = batch_ws_acquire(n, maxdim, nb);
    struct Release {
        BatchWs *w;
        ~Release() { batch_ws_release(w); }
    } release{Wp};
    BatchWs &W = *Wp;
    std::lock_guard<std::mutex> lk(W.mu);
    if (!W.dcond.p) {
        int rc = batch_alloc(W, err);
        if (rc)
            return rc;
    }
    hipStream_t s = W.own;
    HIP_TRY(hipEventRecord(W.ready, a.stream));
    HIP_TRY(hipStreamWaitEvent(s, W.ready, 0));
    const int64_t E = (int64_t)n * (n - 1) / 2;
    // each cloud's own size (bucket padding beyond it)
    std::vector<int32_t> nvh((size_t)nb);
    for (int c = 0; c < nb; ++c)
        nvh[c] = a.nv ? a.nv[c] : n;
    // inputs: pack the clouds (a cloud's condensed matrix is a prefix of its
    // padded one); requested thresholds; sizes
    for (int c = 0; c < nb; ++c) {
        const int64_t Ec = (int64_t)nvh[c] * (nvh[c] - 1) / 2;
        if (Ec > 0)
            HIP_TRY(hipMemcpyAsync(W.dcond.as<float>() + (size_t)c * E, a.dist_dev[c],
                                   (size_t)Ec * 4, hipMemcpyDeviceToDevice, s));
    }
    HIP_TRY(hipMemcpyAsync(W.thr_req.p, a.threshold, (size_t)nb * 4, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(W.nv.p, nvh.data(), (size_t)nb * 4, hipMemcpyHostToDevice, s));

    // host copies for the reductions (pinned, kept with the batch workspace)
    if (maxdim >= 1 && !W.h_dsq.ensure((size_t)nb * n * n * 4)) {
        err = "hipHostMalloc of the host distance copies failed";
        return RPP_E_NOMEM;
    }
    const float *h_dsq_all = W.h_dsq.as<float>();
    for (int p = 1; p <= maxdim; ++p) {
        const DimShape D = dim_shape(n, p, maxdim);
        int group = a.group > 0 ? a.group : tuned_group(n, p);
        if (group <= 0) {
            if (a.tune) {
                int rc = (p == 1) ? launch_dim(W, D, 8, a.flags, false, s, err) : RPP_OK;
                if (rc)
                    return rc;
                rc = autotune(W, D, a.flags, s, &group, err);
                if (rc)
                    return rc;
            } else {
                group = 8;
            }
        }
        GpuTimer tg(s);
        tg.start();
        int rc = launch_dim(W, D, group, a.flags, a.use_graph, s, err);
        if (rc)
            return rc;
        tg.stop();
        // per-cloud counts
        std::vector<uint64_t> toff((size_t)nb * (D.tiles + 2)), toff2((size_t)nb * (D.tiles + 2));
        std::vector<uint64_t> nna(nb), st((size_t)2 * nb);
        HIP_TRY(hipMemcpyAsync(toff.data(), W.toff.p, (size_t)nb * (D.tiles + 1) * 8,
                               hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(toff2.data(), W.toff2.p, (size_t)nb * (D.tiles + 1) * 8,
                               hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(nna.data(), W.nna.p, (size_t)nb * 8, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(st.data(), W.stats.as<uint64_t>() + (size_t)2 * nb * p,
                               (size_t)2 * nb * 8, hipMemcpyDeviceToHost, s));
        std::vector<int> hc((size_t)2 * nb);
        std::vector<uint32_t> bad(nb);
        std::vector<float> radius(nb), thr(nb), deaths;
        std::vector<uint64_t> dedges;
        if (p == 1) {
            HIP_TRY(hipMemcpyAsync(hc.data(), W.counters.p, (size_t)2 * nb * 4,
                                   hipMemcpyDeviceToHost, s));
            HIP_TRY(hipMemcpyAsync(bad.data(), W.bad.p, (size_t)nb * 4, hipMemcpyDeviceToHost, s));
            HIP_TRY(hipMemcpyAsync(radius.data(), W.radius.p, (size_t)nb * 4,
                                   hipMemcpyDeviceToHost, s));
            HIP_TRY(hipMemcpyAsync(thr.data(), W.thr.p, (size_t)nb * 4, hipMemcpyDeviceToHost, s));
            deaths.resize((size_t)nb * n);
            dedges.resize((size_t)nb * n);
            HIP_TRY(hipMemcpyAsync(deaths.data(), W.deaths.p, deaths.size() * 4,
                                   hipMemcpyDeviceToHost, s));
            HIP_TRY(hipMemcpyAsync(dedges.data(), W.dedges.p, dedges.size() * 8,
                                   hipMemcpyDeviceToHost, s));
            HIP_TRY(hipMemcpyAsync(W.h_dsq.p, W.dsq.p, (size_t)nb * n * n * 4,
                                   hipMemcpyDeviceToHost, s));
        }
        HIP_TRY(stream_wait(s));
        const float gpu_ms = tg.ms();
        if (p == 1) {
            for (int c = 0; c < nb; ++c)
                if (bad[c]) {
                    err = "distance matrix " + std::to_string(c) +
                          " holds a NaN, infinite or negative entry";
                    return RPP_E_DATA;
                }
            for (int c = 0; c < nb; ++c) {
                RunOut &o = outs[c];
                o.radius = radius[c];
                o.thr_used = thr[c];
                DimOut &d0 = o.dims[0];
                const int nd = hc[2 * c], merges = hc[2 * c + 1];
                d0.death.assign(deaths.begin() + (size_t)c * n, deaths.begin() + (size_t)c * n + nd);
                d0.death_edge.assign(dedges.begin() + (size_t)c * n,
                                     dedges.begin() + (size_t)c * n + nd);
                d0.birth.assign(nd, 0.0f);
                d0.birth_edge.assign(nd, UINT64_MAX);
                const int nc = nvh[c];  // padding vertices are components of their own
                for (int i = 0; i < nc - merges; ++i) {
                    d0.birth.push_back(0.0f);
                    d0.death.push_back(INFINITY);
                    d0.birth_edge.push_back(UINT64_MAX);
                    d0.death_edge.push_back(UINT64_MAX);
                }
                d0.st.n_candidates = nc;
                d0.st.n_simplices = nc;
                d0.st.n_kept = nc;
                d0.st.n_host_pairs = merges;
                d0.st.n_essential = nc - merges;
                d0.st.n_bars = (int64_t)d0.birth.size();
            }
        }
        // pack the non-apparent columns of all clouds, copy back once
        std::vector<uint64_t> off(nb + 1, 0);
        for (int c = 0; c < nb; ++c)
            off[c + 1] = off[c] + nna[c];
        const int64_t tot = (int64_t)off[nb];
        ALLOC_TRY(W.pkey, (size_t)(tot + 1) * 8);
        ALLOC_TRY(W.pcidx, (size_t)(tot + 1) * 8);
        ALLOC_TRY(W.plow, (size_t)(tot + 1) * 8);
        ALLOC_TRY(W.plowd, (size_t)(tot + 1) * 4);
        std::vector<uint64_t> hk(tot + 1), hv(tot + 1), hl(tot + 1);
        std::vector<float> hld(tot + 1);
        if (tot) {
            uint64_t maxc = *std::max_element(nna.begin(), nna.end());
            HIP_TRY(hipMemcpyAsync(W.poff.p, off.data(), (size_t)(nb + 1) * 8,
                                   hipMemcpyHostToDevice, s));
            const uint64_t *nk, *nv;
            sorted_na(W, &nk, &nv);
            hipLaunchKernelGGL(k_pack, dim3(blocks_for((int64_t)maxc), nb), dim3(256), 0, s, nk, nv,
                               W.lowc.as<uint64_t>(), W.lowd.as<float>(), W.nna.as<uint64_t>(),
                               W.poff.as<uint64_t>(), D.cap, W.pkey.as<uint64_t>(),
                               W.pcidx.as<uint64_t>(), W.plow.as<uint64_t>(),
                               W.plowd.as<float>());
            HIP_TRY(hipMemcpyAsync(hk.data(), W.pkey.p, (size_t)tot * 8, hipMemcpyDeviceToHost, s));
            HIP_TRY(hipMemcpyAsync(hv.data(), W.pcidx.p, (size_t)tot * 8, hipMemcpyDeviceToHost, s));
            HIP_TRY(hipMemcpyAsync(hl.data(), W.plow.p, (size_t)tot * 8, hipMemcpyDeviceToHost, s));
            HIP_TRY(hipMemcpyAsync(hld.data(), W.plowd.p, (size_t)tot * 4, hipMemcpyDeviceToHost, s));
            HIP_TRY(stream_wait(s));
        }
        // per-cloud host reductions, in parallel over clouds
        std::vector<ResidualResult> RR(nb);
        auto h0 = std::chrono::steady_clock::now();
        const double kr = keep_ratio();
        parallel_for(nb, [&](int64_t c) {
            ResidualProblem P;
            P.n = n;
            P.p = p;
            P.thr = outs[c].thr_used;
            P.dsq = h_dsq_all + (size_t)c * n * n;
            P.binom = W.binom_host.data();
            P.ncols = (int64_t)nna[c];
            P.col_key = hk.data() + off[c];
            P.col_cidx = hv.data() + off[c];
            P.col_low = hl.data() + off[c];
            P.col_low_diam = hld.data() + off[c];
            P.parallel = false;
            P.oblivious = (a.flags & RPP_OBLIVIOUS_REDUCTION) != 0;
            P.keep_ratio = kr;
            residual_reduce(P, RR[c]);
        });
        auto h1 = std::chrono::steady_clock::now();
        const float host_ms = std::chrono::duration<float, std::milli>(h1 - h0).count();
        // results, and the next dimension's clearing set
        std::vector<uint64_t> hidx;
        std::vector<int32_t> hcl;
        for (int c = 0; c < nb; ++c) {
            DimOut &Dd = outs[c].dims[p];
            const ResidualResult &R = RR[c];
            const float *dsq = h_dsq_all + (size_t)c * n * n;
            for (size_t i = 0; i < R.sigma.size(); ++i)
                if (R.death[i] > R.birth[i]) {
                    Dd.birth.push_back(R.birth[i]);
                    Dd.death.push_back(R.death[i]);
                    Dd.birth_edge.push_back(critical_edge(dsq, n, W.binom_host.data(), R.sigma[i], p));
                    Dd.death_edge.push_back(critical_edge(dsq, n, W.binom_host.data(), R.tau[i], p + 1));
                }
            for (size_t i = 0; i < R.ess_sigma.size(); ++i) {
                Dd.birth.push_back(R.ess_birth[i]);
                Dd.death.push_back(INFINITY);
                Dd.birth_edge.push_back(critical_edge(dsq, n, W.binom_host.data(), R.ess_sigma[i], p));
                Dd.death_edge.push_back(UINT64_MAX);
            }
            const int64_t kept = (int64_t)toff[(size_t)c * (D.tiles + 1) + D.tiles];
            const int64_t napp = (int64_t)toff2[(size_t)c * (D.tiles + 1) + D.tiles];
            // candidates with a padding vertex were all thresholded (+inf)
            const int64_t own = (int64_t)binom_sat(nvh[c], p + 1);
            Dd.st.n_candidates = own;
            Dd.st.n_thresholded = (int64_t)st[2 * c] - (D.cap - own);
            Dd.st.n_cleared = (int64_t)st[2 * c + 1];
            Dd.st.n_simplices = own - Dd.st.n_thresholded;
            Dd.st.n_kept = kept;
            Dd.st.apparent_group = app_cfg(group).group;
            Dd.st.n_apparent = napp;
            Dd.st.n_nonapparent = kept - napp;
            Dd.st.n_host_pairs = (int64_t)R.sigma.size();
            Dd.st.n_essential = (int64_t)R.ess_sigma.size();
            Dd.st.n_bars = (int64_t)Dd.birth.size();
            Dd.st.n_column_adds = R.additions;
            Dd.st.ms_gpu = gpu_ms / nb;
            Dd.st.ms_host = host_ms / nb;
            if (p < maxdim)
                for (uint64_t t : R.tau) {
                    hidx.push_back(t);
                    hcl.push_back(c);
                }
        }
        if (p < maxdim) {
            if (!hidx.empty()) {
                ALLOC_TRY(W.hidx, hidx.size() * 8);
                ALLOC_TRY(W.hcloud, hcl.size() * 4);
                HIP_TRY(hipMemcpyAsync(W.hidx.p, hidx.data(), hidx.size() * 8,
                                       hipMemcpyHostToDevice, s));
                HIP_TRY(hipMemcpyAsync(W.hcloud.p, hcl.data(), hcl.size() * 4,
                                       hipMemcpyHostToDevice, s));
                hipLaunchKernelGGL(k_mark_bits_cloud, dim3(blocks_for((int64_t)hidx.size())),
                                   dim3(256), 0, s, W.hidx.as<uint64_t>(),
                                   W.hcloud.as<int32_t>(), (int64_t)hidx.size(),
                                   W.bits[(p + 1) & 1].as<uint32_t>(), D.next_words);
            }
        }
    }
    HIP_TRY(stream_wait(s));
    return RPP_OK;
}

}  // namespace rpp
