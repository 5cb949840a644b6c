// capi.cpp -- the extern "C" boundary declared in include/rpp.h.
//
// Validates arguments, moves host input to the device when needed, runs the
// pipeline and turns its output into a library-owned rpp_result with
// canonically sorted bars.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/rpp.h"
#include "pipeline.h"

namespace {

// The last error's text, per thread, in a fixed buffer: setting it never
// allocates (the allocation-free entry point reports through it too).
thread_local char g_last_error[512];

void set_error_text(const char *msg, size_t len)
{
    if (len >= sizeof(g_last_error))
        len = sizeof(g_last_error) - 1;
    memcpy(g_last_error, msg, len);
    g_last_error[len] = 0;
}

int fail(int code, const std::string &msg)
{
    set_error_text(msg.data(), msg.size());
    return code;
}

// Argument checks common to every entry point.
int check_args(int32_t n, int32_t maxdim, float threshold, rpp_result **out)
{
    if (!out)
        return fail(RPP_E_INVAL, "out is NULL");
    *out = nullptr;
    if (n < 1)
        return fail(RPP_E_INVAL, "n must be >= 1");
    if (maxdim < 0 || maxdim > RPP_MAX_DIM)
        return fail(RPP_E_INVAL, "maxdim must be in 0..RPP_MAX_DIM");
    if (isnan(threshold) || threshold < 0.0f)
        return fail(RPP_E_INVAL, "threshold must be >= 0 or +inf");
    if (n > 1 && rpp::binom_sat(n, std::min<int>(n, maxdim + 2)) >= (uint64_t)INT64_MAX)
        return fail(RPP_E_RANGE, "C(n, maxdim+2) exceeds the 63-bit index range");
    if ((int64_t)n * n > (int64_t)1 << 31)
        return fail(RPP_E_RANGE, "n too large for the dense distance matrix");
    return RPP_OK;
}

// RPP_DEVICE_BUDGET_BYTES: cap on the device bytes the library's own cache
// may hold during a call (SIZE_MAX when unset).
size_t device_budget()
{
    const char *e = getenv("RPP_DEVICE_BUDGET_BYTES");
    if (!e || !*e)
        return SIZE_MAX;
    return (size_t)strtoull(e, nullptr, 10);
}

// Up-front device-memory check of a call on n points (before any device
// work): a caller workspace below the floor, or a budget below the floor
// plus `extra` bytes of the call's own (the host entry point's input copy).
int check_device_memory(int32_t n, int32_t maxdim, const void *ws, size_t ws_bytes,
                        size_t extra)
{
    if (!ws && ws_bytes)
        return fail(RPP_E_INVAL, "workspace_bytes > 0 with a NULL workspace_dev");
    const size_t floor = rpp::workspace_floor_bytes(n, maxdim);
    if (ws && ws_bytes < floor)
        return fail(RPP_E_NOMEM, "caller workspace of " + std::to_string(ws_bytes) +
                                     " bytes is below the " + std::to_string(floor) +
                                     " bytes that staging and H0 need for n = " +
                                     std::to_string(n));
    const size_t budget = device_budget();
    if (!ws && budget != SIZE_MAX && floor + extra > budget)
        return fail(RPP_E_NOMEM, "RPP_DEVICE_BUDGET_BYTES=" + std::to_string(budget) +
                                     " is below the " + std::to_string(floor + extra) +
                                     " device bytes that staging and H0 need for n = " +
                                     std::to_string(n));
    return RPP_OK;
}

template <typename T>
T *dup(const std::vector<T> &v)
{
    T *p = static_cast<T *>(malloc(std::max<size_t>(1, v.size()) * sizeof(T)));
    if (p && !v.empty())
        memcpy(p, v.data(), v.size() * sizeof(T));
    return p;
}

int build_result(const rpp::RunOut &ro, int n, int maxdim, uint32_t flags, rpp_result **out)
{
    rpp_result *r = static_cast<rpp_result *>(calloc(1, sizeof(rpp_result)));
    if (!r)
        return fail(RPP_E_NOMEM, "result allocation failed");
    r->maxdim = maxdim;
    r->n = n;
    r->threshold_used = ro.thr_used;
    r->enclosing_radius = ro.radius;
    r->dims = static_cast<rpp_bars *>(calloc(maxdim + 1, sizeof(rpp_bars)));
    r->stats = static_cast<rpp_dim_stats *>(calloc(maxdim + 1, sizeof(rpp_dim_stats)));
    if (flags & RPP_WANT_PAIRS)
        r->pairs = static_cast<rpp_pairs *>(calloc(maxdim + 1, sizeof(rpp_pairs)));
    if (!r->dims || !r->stats || ((flags & RPP_WANT_PAIRS) && !r->pairs)) {
        rpp_result_free(r);
        return fail(RPP_E_NOMEM, "result allocation failed");
    }
    for (int p = 0; p <= maxdim; ++p) {
        const rpp::DimOut &D = ro.dims[p];
        // canonical order: birth, then death (+inf last); zeros as +0.0
        std::vector<size_t> idx(D.birth.size());
        std::iota(idx.begin(), idx.end(), 0);
        std::sort(idx.begin(), idx.end(), [&](size_t x, size_t y) {
            if (D.birth[x] != D.birth[y])
                return D.birth[x] < D.birth[y];
            return D.death[x] < D.death[y];
        });
        std::vector<float> b(idx.size()), d(idx.size());
        std::vector<uint64_t> be(idx.size()), de(idx.size());
        const bool crit = (flags & RPP_WANT_CRITICAL_EDGES) && D.birth_edge.size() == idx.size();
        for (size_t i = 0; i < idx.size(); ++i) {
            b[i] = D.birth[idx[i]] + 0.0f;
            d[i] = D.death[idx[i]] + 0.0f;
            if (crit) {
                be[i] = D.birth_edge[idx[i]];
                de[i] = D.death_edge[idx[i]];
            }
        }
        r->dims[p].dim = p;
        r->dims[p].count = (int64_t)b.size();
        r->dims[p].birth = dup(b);
        r->dims[p].death = dup(d);
        if (flags & RPP_WANT_CRITICAL_EDGES) {
            if (!crit)
                be.assign(idx.size(), UINT64_MAX), de.assign(idx.size(), UINT64_MAX);
            r->dims[p].birth_edge = dup(be);
            r->dims[p].death_edge = dup(de);
        }
        r->stats[p] = D.st;
        if (!r->dims[p].birth || !r->dims[p].death ||
            ((flags & RPP_WANT_CRITICAL_EDGES) &&
             (!r->dims[p].birth_edge || !r->dims[p].death_edge))) {
            rpp_result_free(r);
            return fail(RPP_E_NOMEM, "result allocation failed");
        }
        if (r->pairs) {
            r->pairs[p].dim = p;
            r->pairs[p].count = (int64_t)D.pair_sigma.size();
            r->pairs[p].sigma = dup(D.pair_sigma);
            r->pairs[p].tau = dup(D.pair_tau);
            if (!r->pairs[p].sigma || !r->pairs[p].tau) {
                rpp_result_free(r);
                return fail(RPP_E_NOMEM, "result allocation failed");
            }
        }
    }
    *out = r;
    return RPP_OK;
}

}  // namespace

namespace rpp {
int build_result_public(const RunOut &ro, int n, int maxdim, uint32_t flags, rpp_result **out)
{
    return build_result(ro, n, maxdim, flags, out);
}
void set_last_error(const std::string &msg)
{
    set_error_text(msg.data(), msg.size());
}
void set_last_error_text(const char *msg)
{
    set_error_text(msg, strlen(msg));
}
}  // namespace rpp

namespace {

// rpp_barcodes_device with `held_elsewhere` device bytes of the caller's
// counted against the budget (the host entry point's input copy).
int barcodes_device(const float *dist_dev, int32_t n, int32_t maxdim, float threshold,
                    void *workspace_dev, size_t workspace_bytes, void *hip_stream,
                    uint32_t flags, rpp_result **out, size_t held_elsewhere)
{
    int rc = check_args(n, maxdim, threshold, out);
    if (rc)
        return rc;
    if (n > 1 && !dist_dev)
        return fail(RPP_E_INVAL, "dist_dev is NULL");
    rc = check_device_memory(n, maxdim, workspace_dev, workspace_bytes, held_elsewhere);
    if (rc)
        return rc;
    try {
        rpp::RunArgs a;
        a.arena = workspace_dev;
        a.arena_bytes = workspace_dev ? workspace_bytes : 0;
        const size_t budget = device_budget();
        a.device_limit = budget == SIZE_MAX ? SIZE_MAX : budget - held_elsewhere;
        a.dcond_dev = dist_dev;
        a.n = n;
        a.maxdim = maxdim;
        a.threshold = threshold;
        a.flags = flags;
        a.stream = static_cast<hipStream_t>(hip_stream);
        const char *g = getenv("RPP_APPARENT_GROUP");
        a.apparent_group = g ? atoi(g) : 0;
        const char *cs = getenv("RPP_COUNT_SCANS");
        a.count_scans = cs && atoi(cs) != 0;
        rpp::RunOut ro;
        std::string err;
        rc = rpp::run_pipeline(a, ro, err);
        if (rc)
            return fail(rc, err);
        return build_result(ro, n, maxdim, flags, out);
    } catch (const std::bad_alloc &) {
        return fail(RPP_E_NOMEM, "host allocation failed");
    }
}

}  // namespace

extern "C" {

int rpp_barcodes_device(const float *dist_dev, int32_t n, int32_t maxdim, float threshold,
                        void *workspace_dev, size_t workspace_bytes, void *hip_stream,
                        uint32_t flags, rpp_result **out)
{
    return barcodes_device(dist_dev, n, maxdim, threshold, workspace_dev, workspace_bytes,
                           hip_stream, flags, out, 0);
}

int rpp_barcodes_batch(int32_t count, const rpp_request *reqs, void *hip_stream, uint32_t flags,
                       rpp_result **outs)
{
    if (count < 0 || (count > 0 && (!reqs || !outs)))
        return fail(RPP_E_INVAL, "bad batch arguments");
    for (int32_t i = 0; i < count; ++i)
        outs[i] = nullptr;
    if (flags & RPP_WANT_PAIRS)
        return fail(RPP_E_INVAL, "pair lists are not available for batches");
    for (int32_t i = 0; i < count; ++i) {
        rpp_result *dummy = nullptr;
        int rc = check_args(reqs[i].n, reqs[i].maxdim, reqs[i].threshold, &dummy);
        if (rc)
            return rc;
        if (reqs[i].n > 1 && !reqs[i].dist_dev)
            return fail(RPP_E_INVAL, "dist_dev is NULL");
    }
    try {
        // Shape groups, in first-appearance order.  A group is a shape
        // bucket: n rounded up to a multiple of 64 (each cloud padded with
        // vertices at infinite distance), with one maxdim.  Padding needs a
        // finite threshold: a request with threshold +inf and
        // RPP_NO_ENCLOSING_RADIUS, and any request with RPP_BATCH_EXACT_SHAPES,
        // keeps its exact n.
        const bool radius = !(flags & RPP_NO_ENCLOSING_RADIUS);
        auto bucket_of = [&](const rpp_request &r) {
            const bool pad = !(flags & RPP_BATCH_EXACT_SHAPES) && r.n >= 2 && r.maxdim >= 1 &&
                             (radius || !isinf(r.threshold));
            return pad ? (r.n + 63) / 64 * 64 : -r.n;  // negative: exact
        };
        std::vector<std::pair<std::pair<int, int>, std::vector<int>>> groups;
        for (int32_t i = 0; i < count; ++i) {
            std::pair<int, int> key{bucket_of(reqs[i]), reqs[i].maxdim};
            auto it = std::find_if(groups.begin(), groups.end(),
                                   [&](const auto &g) { return g.first == key; });
            if (it == groups.end())
                groups.push_back({key, {i}});
            else
                it->second.push_back(i);
        }
        std::vector<rpp::RunOut> all(count);
        for (auto &g : groups) {
            // A group of one cloud, or of clouds whose top dimension has more
            // than 2^22 candidate columns each (the batch sizes its buffers
            // by that capacity per cloud, e.g. 17 GB at n = 1024, maxdim 2),
            // runs cloud by cloud through the single-cloud pipeline.
            const int nb_pts = std::abs(g.first.first);
            if (g.second.size() == 1 || nb_pts < 2 || g.first.second < 1 ||
                rpp::binom_sat(nb_pts, g.first.second + 1) > (1ull << 22)) {
                for (int i : g.second) {
                    rpp::RunArgs r;
                    r.dcond_dev = reqs[i].dist_dev;
                    r.n = reqs[i].n;
                    r.maxdim = reqs[i].maxdim;
                    r.threshold = reqs[i].threshold;
                    r.flags = flags & ~(RPP_BATCH_NO_GRAPH | RPP_BATCH_AUTOTUNE |
                                        RPP_BATCH_EXACT_SHAPES);
                    r.stream = static_cast<hipStream_t>(hip_stream);
                    std::string err;
                    int rc = rpp::run_pipeline(r, all[i], err);
                    if (rc)
                        return fail(rc, err);
                }
                continue;
            }
            std::vector<const float *> ptrs;
            std::vector<float> thr;
            std::vector<int> nv;
            for (int i : g.second) {
                ptrs.push_back(reqs[i].dist_dev);
                thr.push_back(reqs[i].threshold);
                nv.push_back(reqs[i].n);
            }
            rpp::BatchArgs a;
            a.count = (int)g.second.size();
            a.n = std::abs(g.first.first);
            a.nv = nv.data();
            a.maxdim = g.first.second;
            a.dist_dev = ptrs.data();
            a.threshold = thr.data();
            a.flags = flags;
            a.stream = static_cast<hipStream_t>(hip_stream);
            a.use_graph = !(flags & RPP_BATCH_NO_GRAPH);
            a.tune = (flags & RPP_BATCH_AUTOTUNE) != 0;
            const char *gs = getenv("RPP_APPARENT_GROUP");
            a.group = gs ? atoi(gs) : 0;
            std::vector<rpp::RunOut> outs;
            std::string err;
            int rc = rpp::run_batch(a, outs, err);
            if (rc)
                return fail(rc, err);
            for (size_t k = 0; k < g.second.size(); ++k)
                all[g.second[k]] = std::move(outs[k]);
        }
        for (int32_t i = 0; i < count; ++i) {
            int rc = build_result(all[i], reqs[i].n, reqs[i].maxdim, flags, &outs[i]);
            if (rc) {
                for (int32_t j = 0; j < i; ++j) {
                    rpp_result_free(outs[j]);
                    outs[j] = nullptr;
                }
                return rc;
            }
        }
        return RPP_OK;
    } catch (const std::bad_alloc &) {
        return fail(RPP_E_NOMEM, "host allocation failed");
    }
}

int rpp_barcodes(const float *dist, int32_t n, int32_t maxdim, float threshold,
                 rpp_result **out)
{
    int rc = check_args(n, maxdim, threshold, out);
    if (rc)
        return rc;
    if (n > 1 && !dist)
        return fail(RPP_E_INVAL, "dist is NULL");
    const size_t m = (size_t)n * (n - 1) / 2;
    for (size_t i = 0; i < m; ++i)
        if (!(dist[i] >= 0.0f) || isinf(dist[i]))
            return fail(RPP_E_DATA, "distance matrix holds a NaN, infinite or negative entry");
    rc = check_device_memory(n, maxdim, nullptr, 0, m * sizeof(float));
    if (rc)
        return rc;
    float *d = nullptr;
    if (m) {
        hipError_t e = hipMalloc(&d, m * sizeof(float));
        if (e != hipSuccess)
            return fail(RPP_E_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
        e = hipMemcpy(d, dist, m * sizeof(float), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            (void)hipFree(d);
            return fail(RPP_E_DEVICE, std::string("hipMemcpy: ") + hipGetErrorString(e));
        }
    }
    rc = barcodes_device(d, n, maxdim, threshold, nullptr, 0, nullptr, 0, out, m * sizeof(float));
    if (d)
        (void)hipFree(d);
    return rc;
}

size_t rpp_workspace_bytes(int32_t n, int32_t maxdim, float threshold)
{
    (void)threshold;
    if (n < 1 || maxdim < 0 || maxdim > RPP_MAX_DIM)
        return 0;
    return rpp::workspace_bytes(n, maxdim);
}

int rpp_apparent_pairs(const float *dist_dev, int32_t n, int32_t p, float threshold,
                       void *hip_stream, uint64_t *sigma_out, uint64_t *tau_out, int64_t cap,
                       int64_t *count, int64_t *n_columns, rpp_dim_stats *stats)
{
    if (!count || !n_columns)
        return fail(RPP_E_INVAL, "count / n_columns is NULL");
    if (n < 2 || p < 1 || p > RPP_MAX_DIM)
        return fail(RPP_E_INVAL, "need n >= 2 and 1 <= p <= RPP_MAX_DIM");
    if (!dist_dev)
        return fail(RPP_E_INVAL, "dist_dev is NULL");
    if (isnan(threshold) || threshold < 0.0f)
        return fail(RPP_E_INVAL, "threshold must be >= 0 or +inf");
    if (cap > 0 && (!sigma_out || !tau_out))
        return fail(RPP_E_INVAL, "output arrays are NULL");
    if (rpp::binom_sat(n, std::min<int>(n, p + 2)) >= (uint64_t)INT64_MAX)
        return fail(RPP_E_RANGE, "C(n, p+2) exceeds the 63-bit index range");
    try {
        std::vector<uint64_t> s, t;
        int64_t ncols = 0, napp = 0;
        std::string err;
        const char *cs = getenv("RPP_COUNT_SCANS");
        const bool count_scans = stats && cs && atoi(cs) != 0;
        int rc = rpp::run_apparent_only(dist_dev, n, p, threshold,
                                        static_cast<hipStream_t>(hip_stream), cap > 0,
                                        count_scans, s, t, ncols, napp, stats, err);
        if (rc)
            return fail(rc, err);
        *count = napp;
        *n_columns = ncols;
        const int64_t k = std::min<int64_t>(cap, (int64_t)s.size());
        if (k > 0) {
            memcpy(sigma_out, s.data(), (size_t)k * 8);
            memcpy(tau_out, t.data(), (size_t)k * 8);
        }
        return RPP_OK;
    } catch (const std::bad_alloc &) {
        return fail(RPP_E_NOMEM, "host allocation failed");
    }
}

int rpp_pdist_device(const float *points_dev, int32_t n, int32_t d, float *dist_dev,
                     void *hip_stream)
{
    if (n < 1 || d < 1)
        return fail(RPP_E_INVAL, "need n >= 1 and d >= 1");
    if (n > 1 && (!points_dev || !dist_dev))
        return fail(RPP_E_INVAL, "null device pointer");
    if ((int64_t)n * n > (int64_t)1 << 31)
        return fail(RPP_E_RANGE, "n too large");
    std::string err;
    int rc = rpp::run_pdist(points_dev, n, d, dist_dev, static_cast<hipStream_t>(hip_stream), err);
    return rc ? fail(rc, err) : RPP_OK;
}

int rpp_backward(const float *points_dev, int32_t n, int32_t d, int64_t nbars,
                 const uint64_t *birth_edge, const uint64_t *death_edge,
                 const float *grad_birth, const float *grad_death, float *grad_points_dev,
                 void *hip_stream)
{
    if (n < 1 || d < 1 || nbars < 0)
        return fail(RPP_E_INVAL, "need n >= 1, d >= 1, nbars >= 0");
    if (!points_dev || !grad_points_dev)
        return fail(RPP_E_INVAL, "null device pointer");
    if (nbars > 0 && (!birth_edge || !death_edge))
        return fail(RPP_E_INVAL, "edge arrays are NULL");
    const uint64_t E = (uint64_t)n * (n - 1) / 2;
    try {
        std::vector<uint64_t> edges;
        std::vector<float> g;
        edges.reserve((size_t)nbars * 2);
        g.reserve((size_t)nbars * 2);
        for (int64_t i = 0; i < nbars; ++i) {
            const float gb = grad_birth ? grad_birth[i] : 0.0f;
            const float gd = grad_death ? grad_death[i] : 0.0f;
            if (birth_edge[i] != UINT64_MAX && gb != 0.0f) {
                if (birth_edge[i] >= E)
                    return fail(RPP_E_INVAL, "birth edge index out of range");
                edges.push_back(birth_edge[i]);
                g.push_back(gb);
            }
            if (death_edge[i] != UINT64_MAX && gd != 0.0f) {
                if (death_edge[i] >= E)
                    return fail(RPP_E_INVAL, "death edge index out of range");
                edges.push_back(death_edge[i]);
                g.push_back(gd);
            }
        }
        std::string err;
        int rc = rpp::run_backward(points_dev, n, d, edges, g, grad_points_dev,
                                   static_cast<hipStream_t>(hip_stream), err);
        return rc ? fail(rc, err) : RPP_OK;
    } catch (const std::bad_alloc &) {
        return fail(RPP_E_NOMEM, "host allocation failed");
    }
}

void rpp_result_free(rpp_result *r)
{
    if (!r)
        return;
    if (r->dims)
        for (int p = 0; p <= r->maxdim; ++p) {
            free(r->dims[p].birth);
            free(r->dims[p].death);
            free(r->dims[p].birth_edge);
            free(r->dims[p].death_edge);
        }
    if (r->pairs)
        for (int p = 0; p <= r->maxdim; ++p) {
            free(r->pairs[p].sigma);
            free(r->pairs[p].tau);
        }
    free(r->dims);
    free(r->stats);
    free(r->pairs);
    free(r);
}

const char *rpp_strerror(int code)
{
    switch (code) {
    case RPP_OK: return "success";
    case RPP_E_INVAL: return "invalid argument";
    case RPP_E_DATA: return "invalid distance entry (NaN, infinite or negative)";
    case RPP_E_RANGE: return "problem size outside the supported index range";
    case RPP_E_NOMEM: return "out of memory";
    case RPP_E_DEVICE: return "HIP runtime error";
    case RPP_E_CANCELLED: return "request cancelled";
    default: return "unknown error";
    }
}

const char *rpp_last_error(void)
{
    return g_last_error;
}

const char *rpp_version(void)
{
    return "rpp-mi355x 0.1 (gfx950)";
}

}  // extern "C"
