// pipeline.h -- host orchestration of one point cloud through the hot path.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>
#include <string>
#include <vector>

#include "../../include/rpp.h"

namespace rpp {

// Per-dimension output gathered by the pipeline before it becomes an
// rpp_result.
struct DimOut {
    std::vector<float> birth, death;     // bars, not yet sorted
    std::vector<uint64_t> birth_edge, death_edge;  // critical edges (same order)
    std::vector<uint64_t> pair_sigma, pair_tau;  // only with RPP_WANT_PAIRS
    rpp_dim_stats st{};
};

struct RunOut {
    float thr_used = 0.0f;
    float radius = 0.0f;
    std::vector<DimOut> dims;
};

struct RunArgs {
    const float *dcond_dev = nullptr;  // device condensed matrix
    int n = 0;
    int maxdim = 0;
    float threshold = 0.0f;
    uint32_t flags = 0;
    hipStream_t stream = nullptr;
    int apparent_group = 0;            // lanes per column, 0 = default
    bool count_scans = false;          // tally cofacet candidates per column
    void *workspace = nullptr;         // explicit workspace (workspace_new), or the device's
    void *arena = nullptr;             // caller device memory for every device buffer, or null
    size_t arena_bytes = 0;
    size_t device_limit = SIZE_MAX;    // most device bytes the call's own buffers may hold
    const std::atomic<bool> *cancel = nullptr;  // set: stop at the next stage boundary
};

// Device workspaces for concurrent callers (one per serving slot).
void *workspace_new();
void workspace_delete(void *w);
size_t workspace_allocated(void *w);   // device bytes the workspace holds
void workspace_trim(void *w);          // free every device buffer of an idle workspace
void workspace_set_limit(void *w, size_t limit);  // cap on the bytes it may hold

// Device bytes every call on n points needs whatever its data (staging and
// H0); a caller workspace or a device budget below it cannot work.
size_t workspace_floor_bytes(int n, int maxdim);

// RPP_FAULT_INJECT=<stage>[:<n>]: true when the call on n points should fail
// at `stage` (tests of the error paths; stages: stage, h0, enumerate,
// apparent, host).
bool fault_injected(const char *stage, int n);

// Returns an RPP_* code; on error `err` holds a message.
int run_pipeline(const RunArgs &a, RunOut &out, std::string &err);

// Several clouds with the same maxdim, processed together at one size n: a
// shape bucket pads each cloud's points to n with vertices at infinite
// distance (finite thresholds only), which no simplex within the threshold
// contains, so each cloud's pairs and bars are its own.
struct BatchArgs {
    int count = 0;
    int n = 0;                                // the group's (padded) number of points
    const int *nv = nullptr;                  // count clouds' own sizes (<= n), or null: all n
    int maxdim = 0;
    const float *const *dist_dev = nullptr;  // count device pointers
    const float *threshold = nullptr;         // count requested thresholds (host)
    uint32_t flags = 0;
    hipStream_t stream = nullptr;
    bool use_graph = true;                    // capture / replay the GPU chain
    bool tune = false;                        // time lane-group sizes when untuned
    int group = 0;                            // fixed lane-group size, 0 = tuned / default
};
int run_batch(const BatchArgs &a, std::vector<RunOut> &outs, std::string &err);

// Apparent pairs of dimension (p, p+1) over all p-simplices <= threshold.
// copy_pairs: fetch the pairs to sigma / tau; count_scans: tally the cofacet
// candidates the scans examine; st (may be null): counts and GPU stage times.
int run_apparent_only(const float *dcond_dev, int n, int p, float threshold, hipStream_t s,
                      bool copy_pairs, bool count_scans, std::vector<uint64_t> &sigma,
                      std::vector<uint64_t> &tau, int64_t &ncols, int64_t &napp,
                      rpp_dim_stats *st, std::string &err);

int run_pdist(const float *pts, int n, int d, float *dist, hipStream_t s, std::string &err);
// edges[i] / g[i]: gradient terms (edge cidx or UINT64_MAX, dL/dlength)
int run_backward(const float *pts, int n, int d, const std::vector<uint64_t> &edges,
                 const std::vector<float> &g, float *grad, hipStream_t s, std::string &err);

// Exact binomial table C(v,k), k = 0..kmax, v = 0..n (saturating at
// UINT64_MAX).
std::vector<uint64_t> binomial_table(int n, int kmax);

// C(n, k) with saturation.
uint64_t binom_sat(int n, int k);

size_t workspace_bytes(int n, int maxdim);
// ResidualProblem::keep_ratio for every host reduction (RPP_KEEP_RATIO).
double keep_ratio();
// Waits for the work queued on s: polls an event for up to 2 ms, then the
// runtime's blocking wait (RPP_SPIN_SYNC=0: the blocking wait only).
hipError_t stream_wait(hipStream_t s);

}  // namespace rpp
