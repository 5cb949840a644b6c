// residual.h -- host-side reduction of the non-apparent columns.
#pragma once

#include <stdint.h>

#include <functional>
#include <memory>
#include <vector>

namespace rpp {

// One dimension's leftover coboundary matrix, everything in host memory.
struct ResidualProblem {
    int n = 0;
    int p = 0;                         // column dimension, >= 1
    float thr = 0.0f;                  // inclusive threshold
    const float *dsq = nullptr;        // n x n distances, zero diagonal
    const uint64_t *binom = nullptr;   // C(v,k) at [k * (n+1) + v], k <= p+2
    // optional neighbour bitsets (bit u of row v: u != v, d(u,v) <= thr);
    // when given, cofacets are found among common neighbours only
    const uint64_t *bits = nullptr;
    int words = 0;
    // optional packed neighbour rows (with bits): npre[v*words + k] is the
    // position in nbd of v's first neighbour in word k, nbd the neighbours'
    // distances row after row; when given, dsq is never read (a few MB
    // instead of n^2 floats: cache-resident where the matrix is not)
    const uint32_t *npre = nullptr;
    const float *nbd = nullptr;
    // non-apparent columns in coboundary order (diameter desc, cidx asc);
    // key = ~bits(diameter) in the low 32 bits
    int64_t ncols = 0;
    const uint64_t *col_key = nullptr;
    const uint64_t *col_cidx = nullptr;
    // low (oldest cofacet) of each unreduced column, ~0 when empty, and its
    // diameter (computed on the GPU)
    const uint64_t *col_low = nullptr;
    const float *col_low_diam = nullptr;
    // second layer of the pivot store.  Sorted mode: apparent pairs (tau,
    // sigma) sorted by tau.  Implicit mode (app_tau == nullptr): a row tau is
    // an apparent pivot iff tau is the oldest cofacet of its youngest facet,
    // which is recomputed from the distance matrix on demand.
    int64_t napp = 0;
    const uint64_t *app_tau = nullptr;
    const uint64_t *app_sigma = nullptr;
    // run the speculative phase on the shared worker pool (false: on the
    // calling thread only, e.g. when the caller already runs in parallel)
    bool parallel = true;
    // at most this many additions per column in the speculative phase
    // (0: no limit); a column cut off there resumes in the exact phase
    int64_t spec_budget = 0;
    // finish_gated: while the gate is closed and every other column waits
    // on it, the parked column nearest the frontier goes on this many
    // additions at a time instead of idling (0: parked columns wait)
    int64_t park_slice = 0;
    // How a column adds a host pivot column k (paper, "Reduction Matrix vs.
    // Oblivious Matrix Reduction").  false: k's reduced column R_k, kept from
    // k's own reduction as the streams of the coboundaries it summed (the
    // reduction-matrix technique: V_k's coboundaries, duplicates cancelling).
    // true: only k's unreduced coboundary D_k, with nothing kept after a
    // column is final (oblivious reduction, Algorithm 2).  The paper's lemma
    // on oblivious reduction makes the pairs and classes identical; the
    // oblivious form needs less memory and may need more additions.
    bool oblivious = false;
    // > 0, with the reduction-matrix form: a kept R_k whose remaining keys
    // exceed keep_ratio times the length of its own coboundary D_k is added
    // as D_k instead (the same result by the paper's lemma on oblivious
    // reduction, chosen per addition by its cost); 0: always R_k
    double keep_ratio = 0.0;
    // > 0: every diameter in this problem -- dsq, col_key, col_low_diam,
    // thr -- is an integer rank below 2^rank_bits (<= 24) held as a float
    // (ranks of the distinct edge lengths, ascending), so keys can pack the
    // rank and the cofacet index into 64 bits where the diameter's bit
    // pattern and the index would need 128.  The results carry ranks too.
    int rank_bits = 0;
};

struct ResidualResult {
    std::vector<uint64_t> sigma, tau;  // pairs found by the reduction
    std::vector<float> birth, death;
    std::vector<uint64_t> ess_sigma;   // columns reduced to zero
    std::vector<float> ess_birth;
    int64_t additions = 0;
    int64_t emergent = 0;              // columns paired without any addition
    int64_t lookups_hash = 0, lookups_apparent = 0;
};

// Column reduction (paper, Algorithm 1, with the additions chosen by
// ResidualProblem::oblivious) of every column, in order, with the two-layer
// pivot store: the pivots found here in a hash map first, then the apparent
// pairs.
void residual_reduce(const ResidualProblem &P, ResidualResult &R);

// The same reduction in two steps.  residual_speculate runs the parallel
// speculative phase (reduction against the apparent pivots only) and may run
// before the previous dimension's pivots are known; finish() completes the
// exact reduction, skipping every column j with drop[j] != 0 (columns the
// clearing lemma removes, which would reduce to zero: no pair, no essential
// class).  The problem's arrays must stay valid until finish() returns.
// When the dropped columns of finish() become known.  ready() must not
// block; wait() blocks until they are known and returns them (drop[j] != 0:
// column j is dropped; nullptr: none is).
struct DropGate {
    virtual ~DropGate() = default;
    virtual bool ready() = 0;
    virtual const uint8_t *wait() = 0;
};
class ResidualSpec {
public:
    virtual ~ResidualSpec() = default;
    virtual void finish(const uint8_t *drop, ResidualResult &R) = 0;
    // The same, started before the dropped columns are known.  A column
    // whose fate is open is still reduced -- a dropped column reduces to
    // zero (the clearing lemma), so a column that ends nonzero is not
    // dropped and its pair is final, and a zero column waits for the gate to
    // tell an essential class from a dropped column -- but one that needs
    // more than `cap` additions before the gate opens waits for it, so that
    // little work is spent on columns that turn out to be dropped.
    virtual void finish_gated(DropGate &gate, int64_t cap, ResidualResult &R) = 0;
};
std::unique_ptr<ResidualSpec> residual_speculate(const ResidualProblem &P);

// Runs fn(i) for i in [0, n) on the shared worker pool (dynamic schedule);
// fn must not itself use the pool.
void parallel_for(int64_t n, const std::function<void(int64_t)> &fn);

}  // namespace rpp
