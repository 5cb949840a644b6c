// pipeline.hip -- one point cloud through the Vietoris-Rips hot path.
//
// Stage order per cloud (paper, overview of GPU-accelerated computation,
// with H0 moved to the GPU):
//   a1  square matrix + enclosing radius             (k_stage, k_min)
//   a2  H0: edges <= threshold, radix sort, union-find (k_enum_*, sort, k_kruskal)
//   for p = 1..maxdim:
//   a3+a4 enumerate p-simplices in cidx order, threshold, clearing
//   a5  apparent-pair test on every kept column
//   a6  partition; sort non-apparent columns by (diameter desc, cidx asc)
//       and apparent pairs by tau
//   a7  host reduction of the non-apparent columns; clearing bitmap of
//       dimension p+1 from all dimension-p pivots
#include "host_common.h"
#include "kernels.h"
#include "pipeline.h"
#include "residual.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <map>
#include <mutex>
#include <thread>

namespace rpp {

// ---------------------------------------------------------------------------
// binomials
// ---------------------------------------------------------------------------
std::vector<uint64_t> binomial_table(int n, int kmax)
{
    std::vector<uint64_t> t((size_t)(kmax + 1) * (n + 1));
    for (int v = 0; v <= n; ++v)
        for (int k = 0; k <= kmax; ++k) {
            uint64_t val;
            if (k == 0)
                val = 1;
            else if (v == 0)
                val = 0;
            else {
                uint64_t a = t[(size_t)(k - 1) * (n + 1) + v - 1];
                uint64_t b = t[(size_t)k * (n + 1) + v - 1];
                val = (a > UINT64_MAX - b) ? UINT64_MAX : a + b;
            }
            t[(size_t)k * (n + 1) + v] = val;
        }
    return t;
}

uint64_t binom_sat(int n, int k)
{
    if (k < 0 || k > n)
        return 0;
    std::vector<uint64_t> t = binomial_table(n, k);
    return t[(size_t)k * (n + 1) + n];
}

// ---------------------------------------------------------------------------
// device workspace: grow-only buffers cached per device
// ---------------------------------------------------------------------------
struct Workspace {
    Workspace();
    DevPool pool;                    // where the device buffers come from
    std::mutex mu;
    DevBuf dsq, rowmax, scal, binom;
    DevBuf ekey, eval, ekey2, eval2;  // edges for H0
    DevBuf mst, deaths, dedges, ufs;
    DevBuf tcount, toff, scan;
    DevBuf lookback;                 // one-pass enumeration: tile flags + ticket
    DevBuf skd[2], skc[2];           // sparse path: all simplices <= thr, previous dim
    DevBuf ndeg, noff, nbw, nbd;     // sparse path: packed neighbour rows
    DevBuf hnbd;                     // sparse path: the host's packed rows (rank-coded)
    DevBuf rflags, rexcl, rmat, rvals;  // sparse path: rank-coded diameters
    DevBuf bits;                     // sparse path: neighbour bitsets
    DevBuf clr, clr2, clrv, clrv2;   // sparse path: sorted cleared cidx
    DevBuf cpos;                     // sparse path: cleared entries below each prefix
    DevBuf cdiam, ccidx, tau;
    DevBuf akey, aval, akey2, aval2;  // apparent pairs
    DevBuf nkey, nval, nkey2, nval2;  // non-apparent columns
    DevBuf clear, next, hostpiv;
    DevBuf lowc, lowd;               // lows of the non-apparent columns
    DevBuf gedges, gvals;            // backward: gradient terms
    DevBuf rscratch, scancnt;
    DevBuf dsqp;                     // row-padded square matrix (vector apparent kernel)
    bool dsqp_ready = false;         // dsqp holds this call's matrix
    DevBuf cvtx;                     // packed vertex tuples of the kept columns
    bool cvtx_ok = false;            // cvtx matches cdiam / ccidx
    // host hand-off of one dimension; two sets, since the reduction of
    // dimension p still reads its set while dimension p+1 fills the other
    HostBuf h_app_tau[2], h_app_sigma[2], h_na_key[2], h_na_cidx[2], h_low[2], h_lowd[2];
    HostBuf h_small;
    HostBuf h_dsq, h_bits;           // pinned host copies for the residual reduction
    HostBuf h_nbd;                   // sparse path: packed rows for the host
    std::vector<uint32_t> h_npre;    // and their per-word positions
    int binom_n = -1, binom_k = -1;
    std::vector<uint64_t> binom_host;
};

// Every device buffer of a workspace, in one list (pool wiring, swaps,
// accounting).
static std::vector<DevBuf *> device_buffers(Workspace &w)
{
    return {&w.dsq,     &w.rowmax,  &w.scal,    &w.binom,  &w.ekey,   &w.eval,    &w.ekey2,
            &w.eval2,   &w.mst,     &w.deaths,  &w.dedges, &w.ufs,    &w.tcount,  &w.toff,
            &w.scan,    &w.lookback, &w.ndeg,    &w.noff,    &w.skd[0], &w.skd[1], &w.skc[0],  &w.skc[1],
            &w.nbw,     &w.nbd,     &w.hnbd,    &w.rflags,  &w.rexcl,  &w.rmat,   &w.rvals,   &w.bits,
            &w.clr,     &w.clr2,    &w.clrv,    &w.clrv2,  &w.cdiam,  &w.ccidx,   &w.tau,
            &w.akey,    &w.aval,    &w.akey2,   &w.aval2,  &w.nkey,   &w.nval,    &w.nkey2,
            &w.nval2,   &w.clear,   &w.next,    &w.hostpiv, &w.lowc,  &w.lowd,    &w.gedges,
            &w.gvals,   &w.rscratch, &w.scancnt, &w.dsqp,  &w.cvtx,   &w.cpos};
}

Workspace::Workspace()
{
    for (DevBuf *b : device_buffers(*this))
        b->pool = &pool;
}

// The largest size each device buffer can take in one call of run_pipeline
// on n points and dimensions 0..maxdim, whatever the distances, the
// threshold and the path (dense or sparse): every count is bounded by the
// number of candidates, C(n, p+1) for a p-simplex.  Written into the
// buffers' hints (arena plan); rpp_workspace_bytes is their sum.
static void plan_limits(Workspace &w, int n, int maxdim)
{
    for (DevBuf *b : device_buffers(w))
        b->hint = 0;
    if (n < 2)
        return;
    const int m = std::max(1, maxdim);
    const uint64_t E = binom_sat(n, 2);
    // C(n, k) is not monotone in k (it falls past k = n/2): take maxima
    auto cmax_k = [&](int k0, int k1) {
        uint64_t c = 0;
        for (int k = k0; k <= k1; ++k)
            c = std::max(c, binom_sat(n, k));
        return c;
    };
    const uint64_t cmax = cmax_k(2, m + 1);   // most p-simplices, p = 1..maxdim
    const uint64_t cpre = cmax_k(2, m);       // p-simplices, p < maxdim (skeleton, prefixes)
    const uint64_t cnext = cmax_k(3, m + 1);  // bitmap of the next dimension's clearing set
    const uint64_t tiles = (uint64_t)compact_tiles((int64_t)cmax);
    const uint64_t scan_n = std::max(std::max(tiles, cpre), E);
    const int words = (n + 63) / 64;
    const size_t pitch = (size_t)((n + 3) & ~3);
    const size_t nn = (size_t)n;
    w.dsq.hint = nn * nn * 4;
    w.rowmax.hint = nn * 4;
    w.scal.hint = 256;
    w.binom.hint = (size_t)(maxdim + 3) * (nn + 1) * 8;
    w.ekey.hint = w.eval.hint = w.ekey2.hint = w.eval2.hint = (E + 1) * 8;
    w.mst.hint = (E / 32 + 2) * 4;
    w.deaths.hint = nn * 4;
    w.dedges.hint = nn * 8;
    w.ufs.hint = 2 * nn * 4 + 64;
    w.tcount.hint = (std::max(tiles, cpre) + 1) * 4;
    w.toff.hint = (std::max(tiles, cpre) + 2) * 8;
    w.scan.hint = (size_t)scan_scratch_words((int64_t)scan_n) * 8;
    w.lookback.hint = (std::max(tiles, (uint64_t)compact_tiles((int64_t)E)) + 2) * 8;
    w.cdiam.hint = (cmax + 1) * 4;
    w.ccidx.hint = w.cvtx.hint = (cmax + 1) * 8;
    w.tau.hint = w.akey.hint = w.aval.hint = w.akey2.hint = w.aval2.hint = (cmax + 1) * 8;
    w.nkey.hint = w.nval.hint = w.nkey2.hint = w.nval2.hint = (cmax + 1) * 8;
    w.lowc.hint = (cmax + 1) * 8;
    w.lowd.hint = (cmax + 1) * 4;
    w.rscratch.hint = (size_t)radix_scratch_words((int64_t)cmax) * 8;
    w.scancnt.hint = (size_t)SCAN_COUNTERS * 8;
    w.dsqp.hint = nn * pitch * 4;
    w.next.hint = w.clear.hint = (cnext / 32 + 2) * 4;
    if (maxdim >= 1) {  // sparse path
        w.skd[0].hint = w.skd[1].hint = (cpre + 1) * 4;
        w.skc[0].hint = w.skc[1].hint = (cpre + 1) * 8;
        w.ndeg.hint = (nn + 1) * 4;
        w.noff.hint = (nn + 2) * 8;
        w.nbw.hint = nn * (size_t)words * 16;
        w.nbd.hint = w.hnbd.hint = (2 * E + 1) * 4;
        w.rflags.hint = (E + 1) * 4;
        w.rexcl.hint = (E + 2) * 8;
        w.rmat.hint = nn * nn * 4;
        w.rvals.hint = (E + 1) * 4;
        w.bits.hint = nn * (size_t)words * 8;
        w.clr.hint = w.clr2.hint = w.clrv.hint = w.clrv2.hint = (cpre + 1) * 8;
        w.cpos.hint = (cpre + 1) * 8;
    }
}

// Device bytes every call on n points needs before its data are seen: the
// square matrix and H0 (staging, edge enumeration, edge keys and sort,
// union-find).
size_t workspace_floor_bytes(int n, int maxdim)
{
    if (n < 2)
        return 0;
    const uint64_t E = binom_sat(n, 2);
    const int64_t tiles = compact_tiles((int64_t)E);
    size_t b = (size_t)n * n * 4 + (size_t)n * 4 + 256 + (size_t)(maxdim + 3) * (n + 1) * 8;
    b += (size_t)(tiles + 1) * 4 + (size_t)(tiles + 2) * 8 + (size_t)scan_scratch_words(tiles) * 8;
    b += (size_t)(E + 1) * (4 + 8) + (size_t)(E + 1) * 8 * 4;
    b += (size_t)radix_scratch_words((int64_t)E) * 8 + (size_t)(E / 32 + 2) * 4;
    b += (size_t)n * (4 + 8 + 8) + 64;
    return b;
}

static std::mutex g_ws_mu;
static std::map<int, Workspace *> g_ws;

static Workspace &workspace_for_current_device()
{
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> lk(g_ws_mu);
    Workspace *&w = g_ws[dev];
    if (!w)
        w = new Workspace();
    return *w;
}

void *workspace_new()
{
    return new Workspace();
}

void workspace_delete(void *w)
{
    delete static_cast<Workspace *>(w);
}

size_t workspace_allocated(void *wp)
{
    Workspace &w = *static_cast<Workspace *>(wp);
    size_t t = 0;
    for (const DevBuf *b : device_buffers(w))
        t += b->owned ? b->cap : 0;
    return t;
}

void workspace_trim(void *wp)
{
    Workspace &w = *static_cast<Workspace *>(wp);
    std::lock_guard<std::mutex> lk(w.mu);
    for (DevBuf *b : device_buffers(w))
        b->release();
    w.binom_n = w.binom_k = -1;
    w.dsqp_ready = false;
    w.cvtx_ok = false;
}

void workspace_set_limit(void *wp, size_t limit)
{
    Workspace &w = *static_cast<Workspace *>(wp);
    std::lock_guard<std::mutex> lk(w.mu);
    w.pool.limit = limit;
}

size_t workspace_bytes(int n, int maxdim)
{
    if (n < 2)
        return 4096;
    Workspace w;
    plan_limits(w, n, maxdim);
    size_t b = 0;
    for (const DevBuf *x : device_buffers(w))
        if (x->hint)
            b += grow_capacity(0, x->hint);  // each at most one 64 KiB round-up
    return b;
}

// For the length of one call, the workspace's device buffers come from a
// caller-provided arena: its own buffers are set aside (and put back
// afterwards), and each buffer's hint is its planned maximum for the call.
struct ArenaScope {
    Workspace &w;
    std::vector<DevBuf> kept;
    int binom_n, binom_k;
    ArenaScope(Workspace &ws, void *base, size_t bytes, int n, int maxdim)
        : w(ws), binom_n(ws.binom_n), binom_k(ws.binom_k)
    {
        for (DevBuf *b : device_buffers(w)) {
            kept.push_back(std::move(*b));
            b->pool = &w.pool;
        }
        w.pool.arena = static_cast<char *>(base);
        w.pool.arena_size = bytes;
        w.pool.arena_top = 0;
        w.binom_n = w.binom_k = -1;
        plan_limits(w, n, maxdim);
    }
    ~ArenaScope()
    {
        size_t i = 0;
        for (DevBuf *b : device_buffers(w)) {
            b->release();  // arena memory: forgotten, not freed
            *b = std::move(kept[i++]);
            b->hint = 0;
        }
        w.pool.arena = nullptr;
        w.pool.arena_size = w.pool.arena_top = 0;
        w.binom_n = binom_n;
        w.binom_k = binom_k;
        w.dsqp_ready = false;
        w.cvtx_ok = false;
    }
};

bool fault_injected(const char *stage, int n)
{
    const char *e = getenv("RPP_FAULT_INJECT");
    if (!e || !*e)
        return false;
    const char *colon = strchr(e, ':');
    const size_t len = colon ? (size_t)(colon - e) : strlen(e);
    if (strlen(stage) != len || strncmp(e, stage, len) != 0)
        return false;
    return !colon || atoi(colon + 1) == n;
}

#define FAULT_POINT(stage)                                                         \
    do {                                                                           \
        if (fault_injected(stage, n)) {                                            \
            err = std::string("fault injected at stage '") + stage + "' (RPP_FAULT_INJECT)"; \
            return RPP_E_DEVICE;                                                   \
        }                                                                          \
    } while (0)

#define CANCEL_POINT()                                                             \
    do {                                                                           \
        if (a.cancel && a.cancel->load(std::memory_order_relaxed)) {               \
            err = "request cancelled";                                             \
            return RPP_E_CANCELLED;                                                \
        }                                                                          \
    } while (0)

// Largest output allocation (bytes) that the dense enumeration makes for every
// candidate before counting them: 1 GiB, or RPP_ENUM_UPFRONT_MAX_BYTES (the
// tests set 0 to run every input through the path that reads the kept count
// back between the count and scatter passes).
static size_t upfront_limit()
{
    const char *e = getenv("RPP_ENUM_UPFRONT_MAX_BYTES");
    return e ? (size_t)strtoull(e, nullptr, 10) : ((size_t)1 << 30);
}

// Waits for the work queued on s by polling an event for up to 2 ms (most
// waits in a call are for a few hundred microseconds of kernels), then in
// the runtime's blocking wait.  The blocking wait alone left, about once in
// 60 calls, a 6-7 ms gap between two stages of a dimension: the thread woke
// that late after the GPU had finished (torus, 124 calls with the polling:
// none).  RPP_SPIN_SYNC=0: the blocking wait only; =2: poll without limit.
hipError_t stream_wait(hipStream_t s)
{
    static const int mode = [] {
        const char *e = getenv("RPP_SPIN_SYNC");
        return e ? atoi(e) : 1;
    }();
    if (mode == 0)
        return hipStreamSynchronize(s);
    thread_local hipEvent_t ev = nullptr;
    thread_local int ev_dev = -1;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return e;
    if (!ev || ev_dev != dev) {
        e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e != hipSuccess)
            return e;
        ev_dev = dev;
    }
    e = hipEventRecord(ev, s);
    if (e != hipSuccess)
        return e;
    const auto t0 = std::chrono::steady_clock::now();
    unsigned polls = 0;
    while ((e = hipEventQuery(ev)) == hipErrorNotReady) {
        __builtin_ia32_pause();
        if (mode == 1 && (++polls & 255u) == 0 &&
            std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(2))
            return hipStreamSynchronize(s);
    }
    return e;
}

// Stable compaction of the p-simplices (dense enumeration) into ws.cdiam /
// ws.ccidx; returns the kept count through *kept and the counters.
// ncleared: the number of set bits of ea.clear, all of them candidates
// within the threshold (pivots of earlier pairs), when the caller knows it:
// the thresholded count is then the remainder and the kernel counts
// nothing; -1: the kernel counts both.
static int enumerate_dense(Workspace &ws, const EnumArgs &ea, hipStream_t s, int64_t *kept,
                           uint64_t *nthr, uint64_t *nclr, std::string &err,
                           GpuTimer *tm = nullptr, int64_t ncleared = -1)
{
    if (ea.p >= 2 && ea.n > 65535) {
        // the enumeration walks address the condensed matrix with 32-bit
        // offsets (and C(n, 3) candidates would not fit in any case)
        err = "dense enumeration of p >= 2 needs n <= 65535";
        return RPP_E_RANGE;
    }
    const int64_t tiles = compact_tiles((int64_t)ea.ncand);
    ALLOC_TRY(ws.tcount, (size_t)(tiles + 1) * 4);
    ALLOC_TRY(ws.toff, (size_t)(tiles + 2) * 8);
    ALLOC_TRY(ws.scan, (size_t)scan_scratch_words(tiles) * 8);
    ALLOC_TRY(ws.h_small, 256);
    unsigned long long *stats = ws.scal.as<unsigned long long>() + 2;
    HIP_TRY(hipMemsetAsync(stats, 0, 2 * sizeof(unsigned long long), s));
    // the vertex tuples too, which the two-phase apparent kernel reads
    // instead of decoding every column (the walk has them at hand)
    ws.cvtx_ok = (ea.p == 2 || ea.p == 3) && ea.n <= 65536;
    // Outputs sized for every candidate when that takes at most 1 GiB: the
    // count, scan and scatter passes then run back to back and the kept
    // count is read once, after them; larger inputs read it between the
    // passes and size the outputs exactly.
    const size_t per = 4 + 8 + (ws.cvtx_ok ? 8 : 0);
    const bool upfront = (ea.ncand + 1) * per <= upfront_limit();
    if (upfront) {
        ALLOC_TRY(ws.cdiam, (size_t)(ea.ncand + 1) * 4);
        ALLOC_TRY(ws.ccidx, (size_t)(ea.ncand + 1) * 8);
        if (ws.cvtx_ok)
            ALLOC_TRY(ws.cvtx, (size_t)(ea.ncand + 1) * 8);
    }
    uint64_t *h = ws.h_small.as<uint64_t>();
    auto read_counts = [&]() -> int {
        HIP_TRY(hipMemcpyAsync(h, ws.toff.as<uint64_t>() + tiles, 8, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(h + 1, stats, 16, hipMemcpyDeviceToHost, s));
        HIP_TRY(stream_wait(s));
        *kept = tiles ? (int64_t)h[0] : 0;
        *nthr = h[1];
        *nclr = h[2];
        if (ncleared >= 0) {
            *nclr = (uint64_t)ncleared;
            *nthr = ea.ncand - (uint64_t)*kept - (uint64_t)ncleared;
        }
        return RPP_OK;
    };
    // RPP_ENUM_ONE_PASS=1: one pass (decoupled look-back) when the outputs
    // are sized up front and the thresholded / cleared counts come from the
    // clearing set's size.  Not the default: the look-back's round trips
    // between thousands of concurrent tiles cost more than the count pass
    // and the scan they replace (torus dimension 2: 112 against 91 us per
    // stage; sphere dimension 1: 63 against 44).
    const char *op = getenv("RPP_ENUM_ONE_PASS");
    if (upfront && ncleared >= 0 && ea.nbatch <= 1 && op && atoi(op) != 0) {
        ALLOC_TRY(ws.lookback, (size_t)(tiles + 2) * 8);
        if (tm)
            tm->start();
        launch_enum_onepass(ea, ws.lookback.as<unsigned long long>(),
                            ws.toff.as<uint64_t>() + tiles, ws.cdiam.as<float>(),
                            ws.ccidx.as<uint64_t>(), s,
                            ws.cvtx_ok ? ws.cvtx.as<uint64_t>() : nullptr);
        if (tm)
            tm->stop();
        if (tiles == 0) {
            *kept = 0;
            *nthr = 0;
            *nclr = (uint64_t)ncleared;
            return RPP_OK;
        }
        return read_counts();
    }
    if (tm)
        tm->start();
    launch_enum_count(ea, ws.tcount.as<uint32_t>(), ncleared >= 0 ? nullptr : stats, s);
    launch_exclusive_scan(ws.tcount.as<uint32_t>(), tiles, ws.toff.as<uint64_t>(),
                          ws.scan.as<uint64_t>(), s);
    if (!upfront) {
        int rc = read_counts();
        if (rc)
            return rc;
        ALLOC_TRY(ws.cdiam, (size_t)(*kept + 1) * 4);
        ALLOC_TRY(ws.ccidx, (size_t)(*kept + 1) * 8);
        if (ws.cvtx_ok)
            ALLOC_TRY(ws.cvtx, (size_t)(*kept + 1) * 8);
    }
    launch_enum_scatter(ea, ws.toff.as<uint64_t>(), ws.cdiam.as<float>(),
                        ws.ccidx.as<uint64_t>(), s, ws.cvtx_ok ? ws.cvtx.as<uint64_t>() : nullptr);
    if (tm)
        tm->stop();
    if (upfront)
        return read_counts();
    return RPP_OK;
}

// Sparse enumeration of the p-simplices (p >= 2) from the (p-1)-simplices in
// ws.skd/skc[cur]: every p-simplex <= threshold, in cidx order, into
// ws.skd/skc[1-cur] when want_all (the next dimension's prefixes), and in the
// same pass the kept columns -- those not in the sorted clearing set --
// still in cidx order, into ws.cdiam/ccidx.
static int enumerate_sparse(Workspace &ws, const ExtArgs &ea, const uint64_t *clear,
                            int64_t nclear, bool want_all, int cur, hipStream_t s,
                            int64_t *kept, int64_t *all, std::string &err, GpuTimer *tm,
                            int fused_group = 0, unsigned long long *scan_count = nullptr)
{
    ws.cvtx_ok = false;
    const int64_t np = ea.npre_count;
    ALLOC_TRY(ws.tcount, (size_t)(np + 1) * 4);
    ALLOC_TRY(ws.toff, (size_t)(np + 2) * 8);
    ALLOC_TRY(ws.scan, (size_t)scan_scratch_words(np) * 8);
    if (tm)
        tm->start();
    launch_ext_count(ea, ws.tcount.as<uint32_t>(), s);
    launch_exclusive_scan(ws.tcount.as<uint32_t>(), np, ws.toff.as<uint64_t>(),
                          ws.scan.as<uint64_t>(), s);
    uint64_t *h = ws.h_small.as<uint64_t>();
    HIP_TRY(hipMemcpyAsync(h, ws.toff.as<uint64_t>() + np, 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(stream_wait(s));
    const int64_t nall = np ? (int64_t)h[0] : 0;
    *all = nall;
    if (nclear > nall) {
        err = "clearing set larger than the simplices it clears";
        return RPP_E_DEVICE;
    }
    *kept = nall - nclear;  // the clearing set is a subset of the extensions
    if (want_all) {
        ALLOC_TRY(ws.skd[1 - cur], (size_t)(nall + 1) * 4);
        ALLOC_TRY(ws.skc[1 - cur], (size_t)(nall + 1) * 8);
    }
    ALLOC_TRY(ws.cdiam, (size_t)(*kept + 1) * 4);
    ALLOC_TRY(ws.ccidx, (size_t)(*kept + 1) * 8);
    // each prefix's place in the clearing set, found beforehand by one
    // thread per prefix; RPP_NO_CLEAR_POS=1: each scatter wave searches the
    // clearing set itself at its start instead
    const char *ncp = getenv("RPP_NO_CLEAR_POS");
    int64_t *cpos = nullptr;
    if (nclear > 0 && !(ncp && atoi(ncp) != 0)) {
        ALLOC_TRY(ws.cpos, (size_t)(np + 1) * 8);
        cpos = ws.cpos.as<int64_t>();
        launch_clear_pos(ea, clear, nclear, cpos, s);
    }
    if (fused_group > 0) {
        // the apparent test runs in the scatter pass: tau of every kept column
        ALLOC_TRY(ws.tau, (size_t)(*kept + 1) * 8);
        launch_ext_scatter_apparent(ea, fused_group, ws.toff.as<uint64_t>(),
                                    want_all ? ws.skd[1 - cur].as<float>() : nullptr,
                                    want_all ? ws.skc[1 - cur].as<uint64_t>() : nullptr, clear,
                                    nclear, ws.cdiam.as<float>(), ws.ccidx.as<uint64_t>(),
                                    (uint64_t)*kept, ws.tau.as<uint64_t>(), scan_count, s, cpos);
        if (tm)
            tm->stop();
        return RPP_OK;
    }
    const bool vtx = ea.p <= 3 && ea.n <= 65536;  // vertex tuples for the apparent test
    if (vtx)
        ALLOC_TRY(ws.cvtx, (size_t)(*kept + 1) * 8);
    launch_ext_scatter(ea, ws.toff.as<uint64_t>(),
                       want_all ? ws.skd[1 - cur].as<float>() : nullptr,
                       want_all ? ws.skc[1 - cur].as<uint64_t>() : nullptr, clear, nclear,
                       ws.cdiam.as<float>(), ws.ccidx.as<uint64_t>(), (uint64_t)*kept,
                       vtx ? ws.cvtx.as<uint64_t>() : nullptr, s, cpos);
    ws.cvtx_ok = vtx;
    if (tm)
        tm->stop();
    return RPP_OK;
}

// Apparent test + partition of ws.cdiam/ccidx (ncols columns).  Results in
// ws.akey/aval (tau, sigma), ws.nkey/nval (~bits(diam), cidx).
static int apparent_and_partition(Workspace &ws, int64_t ncols, int n, int p, int group,
                                  hipStream_t s, int64_t *napp, std::string &err,
                                  GpuTimer *t_app = nullptr, GpuTimer *t_part = nullptr,
                                  int64_t *scanned = nullptr, int words = 0,
                                  GpuTimer *t_pre = nullptr, bool tau_ready = false)
{
    const int64_t tiles = compact_tiles(ncols);
    ALLOC_TRY(ws.tau, (size_t)(ncols + 1) * 8);
    ALLOC_TRY(ws.akey, (size_t)(ncols + 1) * 8);
    ALLOC_TRY(ws.aval, (size_t)(ncols + 1) * 8);
    ALLOC_TRY(ws.akey2, (size_t)(ncols + 1) * 8);
    ALLOC_TRY(ws.aval2, (size_t)(ncols + 1) * 8);
    ALLOC_TRY(ws.nkey, (size_t)(ncols + 1) * 8);
    ALLOC_TRY(ws.nval, (size_t)(ncols + 1) * 8);
    ALLOC_TRY(ws.nkey2, (size_t)(ncols + 1) * 8);
    ALLOC_TRY(ws.nval2, (size_t)(ncols + 1) * 8);
    ALLOC_TRY(ws.tcount, (size_t)(tiles + 1) * 4);
    ALLOC_TRY(ws.toff, (size_t)(tiles + 2) * 8);
    ALLOC_TRY(ws.scan, (size_t)scan_scratch_words(tiles) * 8);
    unsigned long long *sc = nullptr;
    if (scanned) {
        // (a fused enumeration already counted into it)
        ALLOC_TRY(ws.scancnt, (size_t)SCAN_COUNTERS * 8);
        sc = ws.scancnt.as<unsigned long long>();
        if (!tau_ready)
            HIP_TRY(hipMemsetAsync(sc, 0, (size_t)SCAN_COUNTERS * 8, s));
    }
    if (t_pre) {
        ws.cvtx_ok = false;  // the columns are reordered below; cvtx is not
        // The paper's order: every kept column sorted by (diameter desc,
        // cidx asc) before the apparent test, so the partition leaves the
        // non-apparent columns in coboundary order.  The columns are in cidx
        // order, so a stable sort on the complemented diameter suffices.
        t_pre->start();
        ALLOC_TRY(ws.rscratch, (size_t)radix_scratch_words(ncols) * 8);
        launch_desc_keys(ws.cdiam.as<float>(), ncols, ws.nkey.as<uint64_t>(), s);
        if (ncols)
            HIP_TRY(hipMemcpyAsync(ws.nval.p, ws.ccidx.p, (size_t)ncols * 8,
                                   hipMemcpyDeviceToDevice, s));
        const int w = radix_sort_pairs(ws.nkey.as<uint64_t>(), ws.nval.as<uint64_t>(),
                                       ws.nkey2.as<uint64_t>(), ws.nval2.as<uint64_t>(), ncols,
                                       32, ws.rscratch.as<uint64_t>(), s);
        const DevBuf &k = w ? ws.nkey2 : ws.nkey;
        const DevBuf &v = w ? ws.nval2 : ws.nval;
        launch_diam_from_keys(k.as<uint64_t>(), ncols, ws.cdiam.as<float>(), s);
        if (ncols)
            HIP_TRY(hipMemcpyAsync(ws.ccidx.p, v.p, (size_t)ncols * 8, hipMemcpyDeviceToDevice, s));
        t_pre->stop();
    }
    if (t_app)
        t_app->start();
    if (tau_ready)
        ;  // the enumeration ran the test
    else if (words > 0)
        launch_apparent_sparse(ws.cdiam.as<float>(), ws.ccidx.as<uint64_t>(), ncols, n, p, words,
                               ws.nbw.as<uint4>(), ws.nbd.as<float>(), ws.binom.as<uint64_t>(),
                               group, ws.tau.as<uint64_t>(), sc, s,
                               ws.cvtx_ok ? ws.cvtx.as<uint64_t>() : nullptr);
    else if (group >= 20000) {
        const int pitch = (n + 3) & ~3;
        if (!ws.dsqp_ready) {
            ALLOC_TRY(ws.dsqp, (size_t)n * pitch * 4);
            launch_pad_rows(ws.dsq.as<float>(), n, pitch, ws.dsqp.as<float>(), s);
            ws.dsqp_ready = true;
        }
        launch_apparent_vec(ws.cdiam.as<float>(), ws.ccidx.as<uint64_t>(), ncols,
                            ws.dsqp.as<float>(), pitch, n, p, ws.binom.as<uint64_t>(), group,
                            ws.tau.as<uint64_t>(), sc, s,
                            ws.cvtx_ok ? ws.cvtx.as<uint64_t>() : nullptr);
    } else
        launch_apparent(ws.cdiam.as<float>(), ws.ccidx.as<uint64_t>(), ncols,
                        ws.dsq.as<float>(), n, p, ws.binom.as<uint64_t>(), group,
                        ws.tau.as<uint64_t>(), sc, s);
    if (t_app)
        t_app->stop();
    if (t_part)
        t_part->start();
    launch_partition_count(ws.tau.as<uint64_t>(), ncols, ws.tcount.as<uint32_t>(), s);
    launch_exclusive_scan(ws.tcount.as<uint32_t>(), tiles, ws.toff.as<uint64_t>(),
                          ws.scan.as<uint64_t>(), s);
    launch_partition_scatter(ws.tau.as<uint64_t>(), ws.cdiam.as<float>(),
                             ws.ccidx.as<uint64_t>(), ncols, ws.toff.as<uint64_t>(),
                             ws.akey.as<uint64_t>(), ws.aval.as<uint64_t>(),
                             ws.nkey.as<uint64_t>(), ws.nval.as<uint64_t>(), s);
    if (t_part)
        t_part->stop();
    uint64_t *h = ws.h_small.as<uint64_t>();
    HIP_TRY(hipMemcpyAsync(h, ws.toff.as<uint64_t>() + tiles, 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(stream_wait(s));
    *napp = ncols > 0 ? (int64_t)h[0] : 0;
    if (scanned) {
        std::vector<unsigned long long> c(SCAN_COUNTERS);
        HIP_TRY(hipMemcpy(c.data(), sc, (size_t)SCAN_COUNTERS * 8, hipMemcpyDeviceToHost));
        int64_t tot = 0;
        for (unsigned long long x : c)
            tot += (int64_t)x;
        *scanned = tot;
    }
    return RPP_OK;
}

// Additions per column in the speculative phase before it defers the column
// to the exact phase (which then drops it, if the previous dimension's host
// pivots clear it).
constexpr int64_t SPEC_BUDGET = 16;
// Additions a column may make in the exact phase while the previous
// dimension's host pivots (the columns to drop) are still unknown
// (RPP_OPEN_CAP overrides it).
constexpr int64_t OPEN_CAP = 64;
static int64_t open_cap()
{
    const char *e = getenv("RPP_OPEN_CAP");
    return e ? std::max<int64_t>(1, atoll(e)) : OPEN_CAP;
}
// Reduction-matrix form: a kept R_k with more than this many times the
// keys of its own coboundary is added as D_k (RPP_KEEP_RATIO; 0: never).
constexpr double KEEP_RATIO = 0.0;
double keep_ratio()
{
    const char *e = getenv("RPP_KEEP_RATIO");
    return e ? std::max(0.0, atof(e)) : KEEP_RATIO;
}
// Additions per slice of a parked column while the gate is closed and the
// frontier waits on it (RPP_PARK_SLICE overrides it; 0: it waits idle).
// Off: on the torus the slices go to columns the gate then drops and slow
// the previous dimension's reduction beside them (9.0 against 9.4 ms per
// step); on the sphere they change nothing measurable.
constexpr int64_t PARK_SLICE = 0;
static int64_t park_slice()
{
    const char *e = getenv("RPP_PARK_SLICE");
    return e ? std::max<int64_t>(0, atoll(e)) : PARK_SLICE;
}

// 100 K + G selects the two-phase kernel (K candidates per lane alone,
// then G lanes per column still open), 10000 + that its form with the open
// columns pooled per workgroup, 20000 + 100 NB + G the pooled form reading
// its first NB blocks of four candidates as 16-byte vectors (from a
// row-padded copy of the matrix): for short mean scans.
constexpr int TWO_PHASE = 20008;

static int default_group(int p)
{
    return p == 1 ? 16 : TWO_PHASE;
}

// Lanes per column for the dense apparent kernel, from the mean scan length
// s of the oldest-cofacet search: a step tests `group` candidates, so the
// group should cover about one mean scan.  Large inputs measure s on a
// probe of 16384 columns; small ones use the per-dimension default (edges
// of point clouds scan ~10-15 candidates, higher simplices ~4, where most
// columns stop within 4 and the two-phase kernel takes them).
static int group_for_scan(double sbar)
{
    return sbar <= 6 ? TWO_PHASE : sbar <= 12 ? 8 : sbar <= 40 ? 16 : sbar <= 96 ? 32 : 64;
}

static int choose_group(Workspace &ws, int64_t ncols, int n, int p, hipStream_t s, int *group,
                        std::string &err)
{
    const int64_t probe = 16384;
    *group = default_group(p);
    if (ncols < 4 * probe)
        return RPP_OK;
    ALLOC_TRY(ws.tau, (size_t)(ncols + 1) * 8);
    ALLOC_TRY(ws.scancnt, (size_t)SCAN_COUNTERS * 8);
    unsigned long long *sc = ws.scancnt.as<unsigned long long>();
    HIP_TRY(hipMemsetAsync(sc, 0, (size_t)SCAN_COUNTERS * 8, s));
    launch_apparent(ws.cdiam.as<float>(), ws.ccidx.as<uint64_t>(), probe, ws.dsq.as<float>(), n, p,
                    ws.binom.as<uint64_t>(), 8, ws.tau.as<uint64_t>(), sc, s);
    std::vector<unsigned long long> c(SCAN_COUNTERS);
    HIP_TRY(hipMemcpyAsync(c.data(), sc, (size_t)SCAN_COUNTERS * 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(stream_wait(s));
    double tot = 0;
    for (unsigned long long x : c)
        tot += (double)x;
    *group = group_for_scan(tot / (double)probe);
    return RPP_OK;
}

int run_pipeline(const RunArgs &a, RunOut &out, std::string &err)
{
    const int n = a.n, maxdim = a.maxdim;
    hipStream_t s = a.stream;
    out.dims.assign(maxdim + 1, DimOut());
    if (n == 1) {
        out.thr_used = a.threshold;
        out.radius = 0.0f;
        out.dims[0].birth.push_back(0.0f);
        out.dims[0].death.push_back(INFINITY);
        out.dims[0].st.n_simplices = 1;
        out.dims[0].st.n_kept = 1;
        out.dims[0].st.n_essential = 1;
        out.dims[0].st.n_bars = 1;
        return RPP_OK;
    }
    Workspace &ws = a.workspace ? *static_cast<Workspace *>(a.workspace)
                                : workspace_for_current_device();
    std::lock_guard<std::mutex> lk(ws.mu);
    // A caller-provided arena replaces the workspace's buffers for this
    // call; a device limit caps the workspace's own buffers (an idle cache
    // holding more is emptied first).  Either way the stream is drained
    // before the call returns, on success or error, so no kernel still uses
    // the memory afterwards.
    struct Drain {
        hipStream_t s;
        ~Drain() { (void)hipStreamSynchronize(s); }
    };
    struct LimitScope {
        Workspace &w;
        size_t saved;
        LimitScope(Workspace &ws_, size_t lim) : w(ws_), saved(ws_.pool.limit)
        {
            if (lim == SIZE_MAX)
                return;
            if (w.pool.held > lim) {
                for (DevBuf *b : device_buffers(w))
                    b->release();
                w.binom_n = w.binom_k = -1;
            }
            w.pool.limit = lim;
        }
        ~LimitScope() { w.pool.limit = saved; }
    };
    LimitScope limit_scope(ws, a.arena ? SIZE_MAX : a.device_limit);
    std::unique_ptr<ArenaScope> arena;
    if (a.arena)
        arena.reset(new ArenaScope(ws, a.arena, a.arena_bytes, n, maxdim));
    Drain drain{s};
    ws.pool.exhausted = false;
    FAULT_POINT("stage");

    const uint64_t E = (uint64_t)n * (n - 1) / 2;
    ALLOC_TRY(ws.dsq, (size_t)n * n * 4);
    ALLOC_TRY(ws.rowmax, (size_t)n * 4);
    ALLOC_TRY(ws.scal, 256);
    ALLOC_TRY(ws.h_small, 256);

    // ---------------- a1: staging --------------------------------------
    GpuTimer t0(s);
    t0.start();
    uint32_t *bad = ws.scal.as<uint32_t>();
    float *radius = ws.scal.as<float>() + 1;
    HIP_TRY(hipMemsetAsync(bad, 0, 4, s));
    launch_stage(a.dcond_dev, n, ws.dsq.as<float>(), ws.rowmax.as<float>(), bad, s);
    ws.dsqp_ready = false;
    launch_min(ws.rowmax.as<float>(), n, radius, s);
    uint32_t *hs = ws.h_small.as<uint32_t>();
    HIP_TRY(hipMemcpyAsync(hs, ws.scal.p, 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(stream_wait(s));
    if (hs[0]) {
        err = "distance matrix holds a NaN, infinite or negative entry";
        return RPP_E_DATA;
    }
    float R;
    memcpy(&R, hs + 1, 4);
    out.radius = R;
    float thr = a.threshold;
    if (isinf(thr) && !(a.flags & RPP_NO_ENCLOSING_RADIUS))
        thr = R;
    out.thr_used = thr;

    const int kmax = maxdim + 2;
    if (ws.binom_n != n || ws.binom_k < kmax) {
        ws.binom_host = binomial_table(n, kmax);
        ALLOC_TRY(ws.binom, ws.binom_host.size() * 8);
        HIP_TRY(hipMemcpyAsync(ws.binom.p, ws.binom_host.data(), ws.binom_host.size() * 8,
                               hipMemcpyHostToDevice, s));
        ws.binom_n = n;
        ws.binom_k = kmax;
    }
    const int bstride = n + 1;
    (void)bstride;

    // The host's view of the distances for the residual reduction, set
    // once the path is chosen: the square matrix (dense path), or packed
    // neighbour rows (sparse path; with rank-coded diameters, of the ranks).
    const float *h_dsq = nullptr;
    HostDist hdist;
    hdist.n = n;

    // ---------------- a2: H0 ---------------------------------------------
    FAULT_POINT("h0");
    CANCEL_POINT();
    int64_t nedges = 0;
    int64_t mst_edges = 0;  // spanning-forest edges: the p = 1 clearing set
    const uint64_t *h0_keys = nullptr, *h0_cidx = nullptr;  // edges <= thr, diameter desc
    {
        EnumArgs ea{a.dcond_dev, n, 1, thr, ws.binom.as<uint64_t>(), nullptr, E};
        uint64_t nthr = 0, nclr = 0;
        int rc = enumerate_dense(ws, ea, s, &nedges, &nthr, &nclr, err, nullptr, 0);
        if (rc)
            return rc;
        ALLOC_TRY(ws.ekey, (size_t)(nedges + 1) * 8);
        ALLOC_TRY(ws.eval, (size_t)(nedges + 1) * 8);
        ALLOC_TRY(ws.ekey2, (size_t)(nedges + 1) * 8);
        ALLOC_TRY(ws.eval2, (size_t)(nedges + 1) * 8);
        ALLOC_TRY(ws.rscratch, (size_t)radix_scratch_words(nedges) * 8);
        ALLOC_TRY(ws.mst, (size_t)(E / 32 + 2) * 4);
        ALLOC_TRY(ws.deaths, (size_t)n * 4);
        ALLOC_TRY(ws.dedges, (size_t)n * 8);
        ALLOC_TRY(ws.ufs, (size_t)2 * n * 4 + 64);
        launch_desc_keys(ws.cdiam.as<float>(), nedges, ws.ekey.as<uint64_t>(), s);
        HIP_TRY(hipMemcpyAsync(ws.eval.p, ws.ccidx.p, (size_t)nedges * 8,
                               hipMemcpyDeviceToDevice, s));
        int where = radix_sort_pairs(ws.ekey.as<uint64_t>(), ws.eval.as<uint64_t>(),
                                     ws.ekey2.as<uint64_t>(), ws.eval2.as<uint64_t>(), nedges,
                                     32, ws.rscratch.as<uint64_t>(), s);
        const uint64_t *sk = where ? ws.ekey2.as<uint64_t>() : ws.ekey.as<uint64_t>();
        const uint64_t *sv = where ? ws.eval2.as<uint64_t>() : ws.eval.as<uint64_t>();
        h0_keys = sk;
        h0_cidx = sv;
        launch_fill_u32(ws.mst.as<uint32_t>(), (int64_t)(E / 32 + 1), 0u, s);
        int *counters = ws.scal.as<int>() + 8;
        launch_kruskal(sk, sv, nedges, n, ws.mst.as<uint32_t>(), ws.deaths.as<float>(),
                       ws.dedges.as<uint64_t>(), counters, ws.ufs.as<int>(), s);
        int hc[2];
        HIP_TRY(hipMemcpyAsync(hc, counters, 8, hipMemcpyDeviceToHost, s));
        HIP_TRY(stream_wait(s));
        mst_edges = hc[1];
        DimOut &d0 = out.dims[0];
        d0.death.resize(hc[0]);
        d0.death_edge.resize(hc[0]);
        if (hc[0]) {
            HIP_TRY(hipMemcpy(d0.death.data(), ws.deaths.p, (size_t)hc[0] * 4,
                              hipMemcpyDeviceToHost));
            HIP_TRY(hipMemcpy(d0.death_edge.data(), ws.dedges.p, (size_t)hc[0] * 8,
                              hipMemcpyDeviceToHost));
        }
        d0.birth.assign(hc[0], 0.0f);
        d0.birth_edge.assign(hc[0], UINT64_MAX);
        const int ncomp = n - hc[1];
        for (int i = 0; i < ncomp; ++i) {
            d0.birth.push_back(0.0f);
            d0.death.push_back(INFINITY);
            d0.birth_edge.push_back(UINT64_MAX);
            d0.death_edge.push_back(UINT64_MAX);
        }
        d0.st.n_candidates = n;
        d0.st.n_simplices = n;
        d0.st.n_kept = n;
        d0.st.n_host_pairs = hc[1];
        d0.st.n_essential = ncomp;
        d0.st.n_bars = (int64_t)d0.birth.size();
        t0.stop();
        d0.st.ms_gpu = t0.ms();
        if (a.flags & RPP_WANT_PAIRS) {
            // dimension-0 pairs: the edge (tau) of every spanning-forest
            // merge; the vertex side is not tracked (sigma = UINT64_MAX)
            std::vector<uint32_t> bits((size_t)(E / 32 + 1));
            HIP_TRY(hipMemcpy(bits.data(), ws.mst.p, bits.size() * 4, hipMemcpyDeviceToHost));
            for (uint64_t c = 0; c < E; ++c)
                if ((bits[c >> 5] >> (c & 31)) & 1u) {
                    d0.pair_sigma.push_back(UINT64_MAX);
                    d0.pair_tau.push_back(c);
                }
        }
    }

    // ---------------- path choice --------------------------------------------
    const bool sparse = maxdim >= 1 && ((a.flags & RPP_FORCE_SPARSE) ||
                                        (!(a.flags & RPP_FORCE_DENSE) &&
                                         (double)nedges < 0.25 * (double)E));
    const int words = (n + 63) / 64;
    const uint64_t *h_bits = nullptr;
    int cur = 0;
    int64_t nskel = 0;
    if (sparse) {
        // all edges <= thr, in cidx order, are the prefixes of dimension 2
        ALLOC_TRY(ws.skd[0], (size_t)(nedges + 1) * 4);
        ALLOC_TRY(ws.skc[0], (size_t)(nedges + 1) * 8);
        if (nedges) {
            HIP_TRY(hipMemcpyAsync(ws.skd[0].p, ws.cdiam.p, (size_t)nedges * 4,
                                   hipMemcpyDeviceToDevice, s));
            HIP_TRY(hipMemcpyAsync(ws.skc[0].p, ws.ccidx.p, (size_t)nedges * 8,
                                   hipMemcpyDeviceToDevice, s));
        }
        nskel = nedges;
        ALLOC_TRY(ws.bits, (size_t)n * words * 8);
        launch_nbr_bits(ws.dsq.as<float>(), n, thr, ws.bits.as<uint64_t>(), words, s);
        // packed neighbour rows: the 2 * nedges distances under the threshold
        ALLOC_TRY(ws.ndeg, (size_t)(n + 1) * 4);
        ALLOC_TRY(ws.noff, (size_t)(n + 2) * 8);
        ALLOC_TRY(ws.nbw, (size_t)n * words * 16);
        ALLOC_TRY(ws.nbd, (size_t)(2 * nedges + 1) * 4);
        ALLOC_TRY(ws.scan, (size_t)scan_scratch_words(n) * 8);
        launch_nbr_degree(ws.bits.as<uint64_t>(), n, words, ws.ndeg.as<uint32_t>(), s);
        launch_exclusive_scan(ws.ndeg.as<uint32_t>(), n, ws.noff.as<uint64_t>(),
                              ws.scan.as<uint64_t>(), s);
        launch_nbr_pack(ws.dsq.as<float>(), ws.bits.as<uint64_t>(), n, words,
                        ws.noff.as<uint64_t>(), ws.nbw.as<uint4>(), ws.nbd.as<float>(),
                        (uint64_t)(2 * nedges), s);
        if (!ws.h_bits.ensure((size_t)n * words * 8)) {
            err = "hipHostMalloc of the host bitset copy failed";
            return RPP_E_NOMEM;
        }
        h_bits = ws.h_bits.as<uint64_t>();
        HIP_TRY(hipMemcpyAsync(ws.h_bits.p, ws.bits.p, (size_t)n * words * 8,
                               hipMemcpyDeviceToHost, s));
    }

    // Rank-coded diameters for the host reduction (sparse path): where a
    // dimension's cofacet indices pass 2^32, the host keys hold the rank of
    // the diameter among the distinct edge lengths under the threshold
    // instead of its bit pattern, and fit 64 bits instead of 128.  The host
    // then sees every distance as its rank: a matrix of ranks replaces its
    // copy of the distances, and column and low diameters are recoded.
    bool ranks = false;
    int64_t nranks = 0;
    std::vector<float> rank_vals;
    if (sparse && nedges > 0 && nedges < (1 << 24)) {
        // (RPP_RANK_CODING=1 takes this path whenever it can: tests)
        const char *force = getenv("RPP_RANK_CODING");
        bool wide = force && atoi(force) != 0;
        for (int q = 1; q <= maxdim; ++q)
            wide = wide || binom_sat(n, q + 2) > (1ull << 32);
        if (wide) {
            ALLOC_TRY(ws.rflags, (size_t)(nedges + 1) * 4);
            ALLOC_TRY(ws.rexcl, (size_t)(nedges + 2) * 8);
            ALLOC_TRY(ws.scan, (size_t)scan_scratch_words(nedges) * 8);
            launch_rank_flags(h0_keys, nedges, ws.rflags.as<uint32_t>(), s);
            launch_exclusive_scan(ws.rflags.as<uint32_t>(), nedges, ws.rexcl.as<uint64_t>(),
                                  ws.scan.as<uint64_t>(), s);
            uint64_t *hs = ws.h_small.as<uint64_t>();
            HIP_TRY(hipMemcpyAsync(hs, ws.rexcl.as<uint64_t>() + nedges, 8,
                                   hipMemcpyDeviceToHost, s));
            HIP_TRY(stream_wait(s));
            nranks = (int64_t)hs[0];
            ALLOC_TRY(ws.rmat, (size_t)n * n * 4);
            ALLOC_TRY(ws.rvals, (size_t)(nranks + 1) * 4);
            launch_rank_matrix(h0_keys, h0_cidx, ws.rflags.as<uint32_t>(),
                               ws.rexcl.as<uint64_t>(), nedges, n, (float)nranks,
                               ws.rmat.as<float>(), ws.rvals.as<float>(), s);
            rank_vals.resize((size_t)nranks);
            HIP_TRY(hipMemcpyAsync(rank_vals.data(), ws.rvals.p, (size_t)nranks * 4,
                                   hipMemcpyDeviceToHost, s));
            HIP_TRY(stream_wait(s));
            ranks = true;
        }
    }
    // Host distances.  Sparse path: packed rows, 2E values (2.7 MB on the
    // 4096-point sphere instead of a 67 MB matrix), which the host's caches
    // hold; RPP_HOST_MATRIX=1 sends the square matrix instead (comparison).
    const char *hm_env = getenv("RPP_HOST_MATRIX");
    const bool host_packed = sparse && !(hm_env && atoi(hm_env) != 0);
    if (maxdim >= 1 && host_packed) {
        const float *src = ws.nbd.as<float>();
        if (ranks) {  // the same rows over the rank matrix
            ALLOC_TRY(ws.hnbd, (size_t)(2 * nedges + 1) * 4);
            launch_nbr_pack(ws.rmat.as<float>(), ws.bits.as<uint64_t>(), n, words,
                            ws.noff.as<uint64_t>(), ws.nbw.as<uint4>(), ws.hnbd.as<float>(),
                            (uint64_t)(2 * nedges), s);
            src = ws.hnbd.as<float>();
        }
        if (!ws.h_nbd.ensure((size_t)(2 * nedges + 1) * 4)) {
            err = "hipHostMalloc of the host neighbour rows failed";
            return RPP_E_NOMEM;
        }
        if (nedges)
            HIP_TRY(hipMemcpyAsync(ws.h_nbd.p, src, (size_t)(2 * nedges) * 4,
                                   hipMemcpyDeviceToHost, s));
        HIP_TRY(stream_wait(s));  // the bitsets too, for the positions
        ws.h_npre.resize((size_t)n * words);
        packed_row_prefix(h_bits, n, words, ws.h_npre.data());
        hdist.bits = h_bits;
        hdist.npre = ws.h_npre.data();
        hdist.nbd = ws.h_nbd.as<float>();
        hdist.words = words;
    } else if (maxdim >= 1) {
        if (!ws.h_dsq.ensure((size_t)n * n * 4)) {
            err = "hipHostMalloc of the host distance copy failed";
            return RPP_E_NOMEM;
        }
        h_dsq = ws.h_dsq.as<float>();
        HIP_TRY(hipMemcpyAsync(ws.h_dsq.p, ranks ? ws.rmat.p : ws.dsq.p, (size_t)n * n * 4,
                               hipMemcpyDeviceToHost, s));
        hdist.dsq = h_dsq;
    }
    int rank_bits = 0;
    while (ranks && ((uint64_t)1 << rank_bits) <= (uint64_t)nranks)
        ++rank_bits;
    // a diameter seen by the host reduction, back as a length
    auto length_of = [&](float x) -> float {
        return (ranks && x < (float)nranks) ? rank_vals[(size_t)x] : x;
    };

    // ---------------- dimensions 1..maxdim --------------------------------
    // Host reduction of each dimension: the speculative phase, then the
    // exact phase on a host thread that overlaps the next dimension's GPU
    // stages and speculative phase.
    struct HostDim {
        ResidualProblem P;
        std::unique_ptr<ResidualSpec> spec;
        std::vector<uint8_t> drop;  // columns the previous dimension's host pivots clear
        int64_t ndrop = 0;
        ResidualResult RR;
        std::thread th;
        bool failed = false;
        bool collected = false;     // results moved into the output
        std::mutex mu;              // guards done
        std::condition_variable cv;
        bool done = false;          // exact phase over (RR final)
        float ms_spec = 0.0f, ms_exact = 0.0f;
        double t_exact_start = 0.0, t_exact_end = 0.0;  // ms since the call began
        int64_t napp = 0;
        const uint64_t *app_tau = nullptr, *app_sigma = nullptr;
    };
    std::vector<HostDim> hd((size_t)maxdim + 1);
    // RPP_TRACE=1: per-dimension timings of the schedule on stderr
    const char *trace_env = getenv("RPP_TRACE");
    const bool trace = trace_env && atoi(trace_env) != 0;
    const auto t_call = std::chrono::steady_clock::now();
    auto since = [&](std::chrono::steady_clock::time_point t) {
        return std::chrono::duration<double, std::milli>(t - t_call).count();
    };
    struct JoinAll {
        std::vector<HostDim> &h;
        ~JoinAll()
        {
            for (HostDim &x : h)
                if (x.th.joinable())
                    x.th.join();
        }
    } join_all{hd};
    const bool want_pairs_all = (a.flags & RPP_WANT_PAIRS) != 0;
    auto finish_dim = [&](int q) -> int {
        HostDim &H = hd[(size_t)q];
        if (H.collected)
            return RPP_OK;
        H.collected = true;
        if (H.th.joinable())
            H.th.join();
        if (H.failed) {
            err = "host allocation failed in the residual reduction";
            return RPP_E_NOMEM;
        }
        DimOut &Dq = out.dims[q];
        const ResidualResult &RR = H.RR;
        Dq.st.ms_host = H.ms_spec + H.ms_exact;
        if (trace)
            fprintf(stderr,
                    "rpp trace: dim %d gpu %.3f ms (enumerate %.3f, apparent %.3f, partition "
                    "%.3f, sort %.3f) | speculative %.3f ms | exact %.3f ms "
                    "(from %.3f to %.3f ms) | joined at %.3f ms | %lld columns, %lld dropped\n",
                    q, Dq.st.ms_gpu, Dq.st.ms_enumerate, Dq.st.ms_apparent, Dq.st.ms_partition,
                    Dq.st.ms_sort, H.ms_spec, H.ms_exact, H.t_exact_start, H.t_exact_end,
                    since(std::chrono::steady_clock::now()), (long long)H.P.ncols,
                    (long long)H.ndrop);
        for (size_t i = 0; i < RR.sigma.size(); ++i)
            if (RR.death[i] > RR.birth[i]) {
                Dq.birth.push_back(length_of(RR.birth[i]));
                Dq.death.push_back(length_of(RR.death[i]));
                Dq.birth_edge.push_back(critical_edge(hdist, ws.binom_host.data(),
                                                      RR.sigma[i], q));
                Dq.death_edge.push_back(critical_edge(hdist, ws.binom_host.data(),
                                                      RR.tau[i], q + 1));
            }
        for (size_t i = 0; i < RR.ess_sigma.size(); ++i) {
            Dq.birth.push_back(length_of(RR.ess_birth[i]));
            Dq.death.push_back(INFINITY);
            Dq.birth_edge.push_back(critical_edge(hdist, ws.binom_host.data(),
                                                  RR.ess_sigma[i], q));
            Dq.death_edge.push_back(UINT64_MAX);
        }
        // the dropped columns count as cleared, as if the previous
        // dimension's host pivots had been in the device clearing set
        Dq.st.n_cleared += H.ndrop;
        Dq.st.n_kept -= H.ndrop;
        Dq.st.n_nonapparent -= H.ndrop;
        Dq.st.n_host_pairs = (int64_t)RR.sigma.size();
        Dq.st.n_essential = (int64_t)RR.ess_sigma.size();
        Dq.st.n_bars = (int64_t)Dq.birth.size();
        Dq.st.n_column_adds = RR.additions;
        if (want_pairs_all) {
            Dq.pair_sigma.assign(H.app_sigma, H.app_sigma + H.napp);
            Dq.pair_tau.assign(H.app_tau, H.app_tau + H.napp);
            Dq.pair_sigma.insert(Dq.pair_sigma.end(), RR.sigma.begin(), RR.sigma.end());
            Dq.pair_tau.insert(Dq.pair_tau.end(), RR.tau.begin(), RR.tau.end());
        }
        return RPP_OK;
    };

    // clearing set of the current dimension: p = 1 uses the MST bitmap;
    // later dimensions a bitmap (dense) or a sorted cidx array (sparse) of
    // the previous dimension's apparent pivots
    const uint32_t *clear_bits = ws.mst.as<uint32_t>();
    int64_t clear_count = mst_edges;  // set bits of clear_bits
    int64_t nclear_sorted = 0;
    const uint64_t *clear_sorted = nullptr;
    for (int p = 1; p <= maxdim; ++p) {
        DimOut &D = out.dims[p];
        GpuTimer tg(s), t_enum(s), t_app(s), t_part(s), t_sort(s);
        tg.start();
        int64_t ncols = 0, ncand = 0;
        uint64_t nthr = 0, nclr = 0;
        bool fused = false;  // the apparent test ran inside the enumeration
        int rc;
        FAULT_POINT("enumerate");
        CANCEL_POINT();
        if (!sparse || p == 1) {
            const uint64_t nc = binom_sat(n, p + 1);
            EnumArgs ea{a.dcond_dev, n, p, thr, ws.binom.as<uint64_t>(), clear_bits, nc};
            rc = enumerate_dense(ws, ea, s, &ncols, &nthr, &nclr, err, &t_enum, clear_count);
            ncand = (int64_t)nc;
        } else {
            ExtArgs xa{n, p, words, ws.nbw.as<uint4>(), ws.nbd.as<float>(),
                       ws.binom.as<uint64_t>(), ws.skd[cur].as<float>(),
                       ws.skc[cur].as<uint64_t>(), nskel};
            int64_t nall = 0;
            // RPP_SPARSE_FUSED=1: the apparent test fused into the scatter
            // pass (two-phase forms, columns in cidx order).  Not the
            // default: with one wave per prefix about half the lanes idle
            // in the test, and the standalone kernel after the scatter is
            // faster (sphere dimension 2: 0.50 + 0.43 ms apart, 1.23 fused)
            const int sg = sparse_group(a.apparent_group);
            const char *fu = getenv("RPP_SPARSE_FUSED");
            fused = sg >= 100 && !(a.flags & RPP_SORT_FIRST) && fu && atoi(fu) != 0;
            unsigned long long *sc = nullptr;
            if (fused && a.count_scans) {
                ALLOC_TRY(ws.scancnt, (size_t)SCAN_COUNTERS * 8);
                sc = ws.scancnt.as<unsigned long long>();
                HIP_TRY(hipMemsetAsync(sc, 0, (size_t)SCAN_COUNTERS * 8, s));
            }
            rc = enumerate_sparse(ws, xa, clear_sorted, nclear_sorted, p < maxdim, cur, s,
                                  &ncols, &nall, err, &t_enum, fused ? sg : 0, sc);
            ncand = nall;
            nclr = (uint64_t)(nall - ncols);
            if (p < maxdim) {
                cur = 1 - cur;
                nskel = nall;
            }
        }
        if (rc)
            return rc;
        int64_t napp = 0, scanned = 0;
        int group = a.apparent_group;
        if (group <= 0 && !sparse) {
            rc = choose_group(ws, ncols, n, p, s, &group, err);
            if (rc)
                return rc;
        }
        const bool sort_first = (a.flags & RPP_SORT_FIRST) != 0;
        GpuTimer t_pre(s);
        FAULT_POINT("apparent");
        rc = apparent_and_partition(ws, ncols, n, p, group, s, &napp, err, &t_app, &t_part,
                                    a.count_scans ? &scanned : nullptr, sparse ? words : 0,
                                    sort_first ? &t_pre : nullptr, fused);
        if (rc)
            return rc;
        t_sort.start();
        const int64_t nna = ncols - napp;

        // next dimension's clearing bitmap (dense): this dimension's apparent
        // taus (its host taus are dropped on the host instead)
        if (p < maxdim && !sparse) {
            const uint64_t nnext = binom_sat(n, p + 2);
            ALLOC_TRY(ws.next, (size_t)(nnext / 32 + 2) * 4);
            launch_fill_u32(ws.next.as<uint32_t>(), (int64_t)(nnext / 32 + 1), 0u, s);
            launch_mark_bits(ws.akey.as<uint64_t>(), napp, ws.next.as<uint32_t>(), s);
        }
        // a6: sort the non-apparent columns into coboundary order (the
        // partition kept them in cidx order, so a stable sort on the
        // descending-diameter key yields diameter desc, cidx asc)
        const bool sorted_store = (a.flags & RPP_SORTED_PAIR_STORE) != 0;
        const bool want_pairs = (a.flags & RPP_WANT_PAIRS) != 0;
        ALLOC_TRY(ws.rscratch,
                  (size_t)radix_scratch_words(sorted_store ? std::max(napp, nna) : nna) * 8);
        // (already in coboundary order when every column was sorted first)
        int wn = sort_first ? 0
                            : radix_sort_pairs(ws.nkey.as<uint64_t>(), ws.nval.as<uint64_t>(),
                                               ws.nkey2.as<uint64_t>(), ws.nval2.as<uint64_t>(),
                                               nna, 32, ws.rscratch.as<uint64_t>(), s);
        const uint64_t *d_nk = wn ? ws.nkey2.as<uint64_t>() : ws.nkey.as<uint64_t>();
        const uint64_t *d_nv = wn ? ws.nval2.as<uint64_t>() : ws.nval.as<uint64_t>();
        const uint64_t *d_at = ws.akey.as<uint64_t>();
        const uint64_t *d_as = ws.aval.as<uint64_t>();
        if (sorted_store) {
            const int tau_bits = bit_length(binom_sat(n, p + 2));
            int wa = radix_sort_pairs(ws.akey.as<uint64_t>(), ws.aval.as<uint64_t>(),
                                      ws.akey2.as<uint64_t>(), ws.aval2.as<uint64_t>(), napp,
                                      tau_bits, ws.rscratch.as<uint64_t>(), s);
            d_at = wa ? ws.akey2.as<uint64_t>() : ws.akey.as<uint64_t>();
            d_as = wa ? ws.aval2.as<uint64_t>() : ws.aval.as<uint64_t>();
        }
        t_sort.stop();
        // a7: lows of the non-apparent columns for the host reduction
        ALLOC_TRY(ws.lowc, (size_t)(nna + 1) * 8);
        ALLOC_TRY(ws.lowd, (size_t)(nna + 1) * 4);
        if (sparse)
            launch_lows_sparse(d_nk, d_nv, nna, ws.nbw.as<uint4>(), ws.nbd.as<float>(), n, p, words,
                               ws.binom.as<uint64_t>(), ws.lowc.as<uint64_t>(),
                               ws.lowd.as<float>(), s);
        else
            launch_lows(d_nk, d_nv, nna, ws.dsq.as<float>(), n, p, thr, ws.binom.as<uint64_t>(),
                        ws.lowc.as<uint64_t>(), ws.lowd.as<float>(), s);
        // device -> host handoff (the set of this dimension's parity)
        const int hb = p & 1;
        // dimension p-2 used these host buffers: its exact phase must be over
        if (p >= 3) {
            int rc2 = finish_dim(p - 2);
            if (rc2)
                return rc2;
        }
        ALLOC_TRY(ws.h_na_key[hb], (size_t)(nna + 1) * 8);
        ALLOC_TRY(ws.h_na_cidx[hb], (size_t)(nna + 1) * 8);
        ALLOC_TRY(ws.h_low[hb], (size_t)(nna + 1) * 8);
        ALLOC_TRY(ws.h_lowd[hb], (size_t)(nna + 1) * 4);
        if (ranks)
            launch_recode_ranks(const_cast<uint64_t *>(d_nk), ws.lowd.as<float>(), nna,
                                ws.rvals.as<float>(), nranks, s);
        if (nna) {
            HIP_TRY(hipMemcpyAsync(ws.h_na_key[hb].p, d_nk, (size_t)nna * 8,
                                   hipMemcpyDeviceToHost, s));
            HIP_TRY(hipMemcpyAsync(ws.h_na_cidx[hb].p, d_nv, (size_t)nna * 8,
                                   hipMemcpyDeviceToHost, s));
            HIP_TRY(hipMemcpyAsync(ws.h_low[hb].p, ws.lowc.p, (size_t)nna * 8,
                                   hipMemcpyDeviceToHost, s));
            HIP_TRY(hipMemcpyAsync(ws.h_lowd[hb].p, ws.lowd.p, (size_t)nna * 4,
                                   hipMemcpyDeviceToHost, s));
        }
        ALLOC_TRY(ws.h_app_tau[hb], (size_t)(napp + 1) * 8);
        ALLOC_TRY(ws.h_app_sigma[hb], (size_t)(napp + 1) * 8);
        if ((sorted_store || want_pairs) && napp) {
            HIP_TRY(hipMemcpyAsync(ws.h_app_tau[hb].p, d_at, (size_t)napp * 8,
                                   hipMemcpyDeviceToHost, s));
            HIP_TRY(hipMemcpyAsync(ws.h_app_sigma[hb].p, d_as, (size_t)napp * 8,
                                   hipMemcpyDeviceToHost, s));
        }
        // next dimension's clearing set on the device: this dimension's
        // apparent pivots.  Its host pivots are not known yet; the columns
        // they would clear are dropped from the next reduction instead.
        if (p < maxdim) {
            if (!sparse) {
                std::swap(ws.clear, ws.next);
                clear_bits = ws.clear.as<uint32_t>();
                clear_count = napp;
            } else {
                ALLOC_TRY(ws.clr, (size_t)(napp + 1) * 8);
                ALLOC_TRY(ws.clr2, (size_t)(napp + 1) * 8);
                ALLOC_TRY(ws.clrv, (size_t)(napp + 1) * 8);
                ALLOC_TRY(ws.clrv2, (size_t)(napp + 1) * 8);
                ALLOC_TRY(ws.rscratch, (size_t)radix_scratch_words(napp) * 8);
                if (napp)
                    HIP_TRY(hipMemcpyAsync(ws.clr.p, d_at, (size_t)napp * 8,
                                           hipMemcpyDeviceToDevice, s));
                int wc = radix_sort_pairs(ws.clr.as<uint64_t>(), ws.clrv.as<uint64_t>(),
                                          ws.clr2.as<uint64_t>(), ws.clrv2.as<uint64_t>(), napp,
                                          bit_length(binom_sat(n, p + 2)),
                                          ws.rscratch.as<uint64_t>(), s);
                clear_sorted = wc ? ws.clr2.as<uint64_t>() : ws.clr.as<uint64_t>();
                nclear_sorted = napp;
            }
        }
        tg.stop();
        HIP_TRY(stream_wait(s));
        D.st.ms_gpu = tg.ms();
        D.st.ms_enumerate = t_enum.ms();
        D.st.ms_apparent = t_app.ms();
        D.st.ms_partition = t_part.ms();
        D.st.ms_sort = t_sort.ms() + (sort_first ? t_pre.ms() : 0.0f);
        D.st.n_scanned = scanned;
        D.st.n_candidates = ncand;
        D.st.n_thresholded = (int64_t)nthr;
        D.st.n_cleared = (int64_t)nclr;
        D.st.n_simplices = ncand - (int64_t)nthr;
        D.st.n_kept = ncols;
        // negative: the sparse kernel, with that many lanes per column
        // (fused into the enumeration: -(1000 + the two-phase code))
        D.st.apparent_group = sparse ? -(sparse_group(group) + (fused ? 1000 : 0)) : group;
        D.st.n_apparent = napp;
        D.st.n_nonapparent = nna;

        FAULT_POINT("host");
        CANCEL_POINT();
        // a7: host residual reduction.  The speculative phase runs now; the
        // exact phase needs the previous dimension's host pivots (its
        // clearing set) and runs on a host thread while the next dimension's
        // GPU stages proceed.
        HostDim &H = hd[p];
        H.P.n = n;
        H.P.p = p;
        H.P.thr = thr;
        H.P.dsq = h_dsq;
        H.P.npre = hdist.npre;
        H.P.nbd = hdist.nbd;
        H.P.binom = ws.binom_host.data();
        H.P.bits = sparse ? h_bits : nullptr;
        H.P.words = sparse ? words : 0;
        H.P.ncols = nna;
        H.P.col_key = ws.h_na_key[hb].as<uint64_t>();
        H.P.col_cidx = ws.h_na_cidx[hb].as<uint64_t>();
        H.P.col_low = ws.h_low[hb].as<uint64_t>();
        H.P.col_low_diam = ws.h_lowd[hb].as<float>();
        H.P.napp = napp;
        H.P.app_tau = sorted_store ? ws.h_app_tau[hb].as<uint64_t>() : nullptr;
        H.P.app_sigma = sorted_store ? ws.h_app_sigma[hb].as<uint64_t>() : nullptr;
        H.P.spec_budget = SPEC_BUDGET;
        H.P.park_slice = park_slice();
        if (ranks) {
            H.P.rank_bits = rank_bits;
            H.P.thr = (float)(nranks - 1);
        }
        H.P.oblivious = (a.flags & RPP_OBLIVIOUS_REDUCTION) != 0;
        H.P.keep_ratio = keep_ratio();
        H.napp = napp;
        H.app_tau = ws.h_app_tau[hb].as<uint64_t>();
        H.app_sigma = ws.h_app_sigma[hb].as<uint64_t>();
        {
            auto a0 = std::chrono::steady_clock::now();
            try {
                H.spec = residual_speculate(H.P);
            } catch (const std::bad_alloc &) {
                err = "host allocation failed in the residual reduction";
                return RPP_E_NOMEM;
            }
            const auto a1 = std::chrono::steady_clock::now();
            H.ms_spec = std::chrono::duration<float, std::milli>(a1 - a0).count();
            if (trace)
                fprintf(stderr, "rpp trace: dim %d hand-off at %.3f ms, speculative done at %.3f ms\n",
                        p, since(a0), since(a1));
        }
        // The exact phase starts at once.  The previous dimension's host
        // pivots -- this dimension's dropped columns -- are still being found
        // on its own thread; the gate waits for them when they are needed.
        HostDim *prevp = p > 1 ? &hd[(size_t)p - 1] : nullptr;
        const int64_t cap = open_cap();
        H.th = std::thread([&H, prevp, cap, &since, trace] {
            struct PrevGate final : DropGate {
                HostDim &prev, &cur;
                bool have = false;
                PrevGate(HostDim &pr, HostDim &c) : prev(pr), cur(c) {}
                bool ready() override
                {
                    std::lock_guard<std::mutex> lk(prev.mu);
                    return prev.done;
                }
                const uint8_t *wait() override
                {
                    if (!have) {
                        {
                            std::unique_lock<std::mutex> lk(prev.mu);
                            prev.cv.wait(lk, [&] { return prev.done; });
                        }
                        have = true;
                        const std::vector<uint64_t> &tau = prev.RR.tau;
                        const int64_t m = cur.P.ncols;
                        if (!prev.failed && !tau.empty() && m) {
                            cur.drop.assign((size_t)m, 0);
                            std::vector<uint64_t> sp(tau);
                            std::sort(sp.begin(), sp.end());
                            for (int64_t j = 0; j < m; ++j)
                                if (std::binary_search(sp.begin(), sp.end(), cur.P.col_cidx[j])) {
                                    cur.drop[(size_t)j] = 1;
                                    ++cur.ndrop;
                                }
                        }
                    }
                    return cur.drop.empty() ? nullptr : cur.drop.data();
                }
            };
            auto b0 = std::chrono::steady_clock::now();
            H.t_exact_start = since(b0);
            try {
                if (prevp) {
                    PrevGate gate(*prevp, H);
                    H.spec->finish_gated(gate, cap, H.RR);
                } else {
                    H.spec->finish(nullptr, H.RR);
                }
            } catch (const std::exception &) {
                H.failed = true;
            }
            const auto f0 = std::chrono::steady_clock::now();
            H.spec.reset();
            const auto b1 = std::chrono::steady_clock::now();
            if (trace)
                fprintf(stderr, "rpp trace:   p=%d exact phase state freed in %.3f ms\n", H.P.p,
                        std::chrono::duration<float, std::milli>(b1 - f0).count());
            H.ms_exact = std::chrono::duration<float, std::milli>(b1 - b0).count();
            H.t_exact_end = since(b1);
            {
                std::lock_guard<std::mutex> lk(H.mu);
                H.done = true;
            }
            H.cv.notify_all();
        });
    }
    for (int q = 1; q <= maxdim; ++q) {
        int rc2 = finish_dim(q);
        if (rc2)
            return rc2;
    }
    if (trace)
        fprintf(stderr, "rpp trace: n %d maxdim %d done at %.3f ms\n", n, maxdim,
                since(std::chrono::steady_clock::now()));
    HIP_TRY(stream_wait(s));
    return RPP_OK;
}

int run_pdist(const float *pts, int n, int d, float *dist, hipStream_t s, std::string &err)
{
    launch_pdist(pts, n, d, dist, s);
    HIP_TRY(hipGetLastError());
    HIP_TRY(stream_wait(s));
    return RPP_OK;
}

int run_backward(const float *pts, int n, int d, const std::vector<uint64_t> &edges,
                 const std::vector<float> &g, float *grad, hipStream_t s, std::string &err)
{
    Workspace &ws = workspace_for_current_device();
    std::lock_guard<std::mutex> lk(ws.mu);
    const int64_t m = (int64_t)edges.size();
    ALLOC_TRY(ws.gedges, (size_t)(m + 1) * 8);
    ALLOC_TRY(ws.gvals, (size_t)(m + 1) * 4);
    if (m) {
        HIP_TRY(hipMemcpyAsync(ws.gedges.p, edges.data(), (size_t)m * 8, hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(ws.gvals.p, g.data(), (size_t)m * 4, hipMemcpyHostToDevice, s));
    }
    launch_edge_grad(pts, n, d, ws.gedges.as<uint64_t>(), ws.gvals.as<float>(), m, grad, s);
    HIP_TRY(hipGetLastError());
    HIP_TRY(stream_wait(s));
    return RPP_OK;
}

int run_apparent_only(const float *dcond_dev, int n, int p, float threshold, hipStream_t s,
                      bool copy_pairs, bool count_scans, std::vector<uint64_t> &sigma,
                      std::vector<uint64_t> &tau, int64_t &ncols, int64_t &napp,
                      rpp_dim_stats *st, std::string &err)
{
    Workspace &ws = workspace_for_current_device();
    std::lock_guard<std::mutex> lk(ws.mu);
    GpuTimer t_all(s), t_enum(s), t_app(s), t_part(s);
    t_all.start();
    ALLOC_TRY(ws.dsq, (size_t)n * n * 4);
    ALLOC_TRY(ws.rowmax, (size_t)n * 4);
    ALLOC_TRY(ws.scal, 256);
    ALLOC_TRY(ws.h_small, 256);
    uint32_t *bad = ws.scal.as<uint32_t>();
    HIP_TRY(hipMemsetAsync(bad, 0, 4, s));
    launch_stage(dcond_dev, n, ws.dsq.as<float>(), ws.rowmax.as<float>(), bad, s);
    ws.dsqp_ready = false;
    uint32_t hb = 0;
    HIP_TRY(hipMemcpyAsync(&hb, bad, 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(stream_wait(s));
    if (hb) {
        err = "distance matrix holds a NaN, infinite or negative entry";
        return RPP_E_DATA;
    }
    const int kmax = p + 2;
    if (ws.binom_n != n || ws.binom_k < kmax) {
        ws.binom_host = binomial_table(n, kmax);
        ALLOC_TRY(ws.binom, ws.binom_host.size() * 8);
        HIP_TRY(hipMemcpyAsync(ws.binom.p, ws.binom_host.data(), ws.binom_host.size() * 8,
                               hipMemcpyHostToDevice, s));
        ws.binom_n = n;
        ws.binom_k = kmax;
    }
    const uint64_t ncand = binom_sat(n, p + 1);
    EnumArgs ea{dcond_dev, n, p, threshold, ws.binom.as<uint64_t>(), nullptr, ncand};
    uint64_t nthr = 0, nclr = 0;
    int rc = enumerate_dense(ws, ea, s, &ncols, &nthr, &nclr, err, &t_enum, 0);
    if (rc)
        return rc;
    // lanes per column from the mean scan length (random edge orders scan
    // hundreds of candidates per column, point clouds a few)
    int group = 8;
    const char *ge = getenv("RPP_APPARENT_GROUP");  // tests: a fixed kernel form
    if (ge && atoi(ge) > 0) {
        group = atoi(ge);
    } else {
        rc = choose_group(ws, ncols, n, p, s, &group, err);
        if (rc)
            return rc;
    }
    int64_t scanned = 0;
    rc = apparent_and_partition(ws, ncols, n, p, group, s, &napp, err, &t_app, &t_part,
                                count_scans ? &scanned : nullptr);
    if (rc)
        return rc;
    t_all.stop();
    if (copy_pairs) {
        sigma.resize(napp);
        tau.resize(napp);
        if (napp) {
            HIP_TRY(hipMemcpyAsync(sigma.data(), ws.aval.p, (size_t)napp * 8,
                                   hipMemcpyDeviceToHost, s));
            HIP_TRY(hipMemcpyAsync(tau.data(), ws.akey.p, (size_t)napp * 8,
                                   hipMemcpyDeviceToHost, s));
        }
    }
    HIP_TRY(stream_wait(s));
    if (st) {
        memset(st, 0, sizeof(*st));
        st->n_candidates = (int64_t)ncand;
        st->n_simplices = (int64_t)ncand - (int64_t)nthr;
        st->n_thresholded = (int64_t)nthr;
        st->n_kept = ncols;
        st->n_apparent = napp;
        st->n_nonapparent = ncols - napp;
        st->n_scanned = count_scans ? scanned : 0;
        st->ms_enumerate = t_enum.ms();
        st->ms_apparent = t_app.ms();
        st->ms_partition = t_part.ms();
        st->ms_gpu = t_all.ms();
        st->apparent_group = group;
    }
    return RPP_OK;
}

}  // namespace rpp
