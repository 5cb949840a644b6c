/*
 * rpp.h -- C ABI of the MI355X Vietoris-Rips persistence library.
 *
 * The library computes Vietoris-Rips persistence barcodes of a finite metric
 * space given by its distance matrix, as described in "GPU-Accelerated
 * Computation of Vietoris-Rips Persistence Barcodes" (arXiv 2003.07989).
 * The data-parallel stages run as HIP kernels on one AMD Instinct MI355X
 * (gfx950): distance staging and the enclosing radius, H0 by edge sort and
 * union-find, enumeration of p-simplices in combinatorial-number-system
 * order with the threshold and clearing filter, the apparent-pair test, the
 * partition of columns and the key sorts.  The residual reduction of the
 * non-apparent columns over Z/2 runs on host threads.
 *
 * Conventions shared by every entry point
 * ----------------------------------------
 * Distance matrix.  The condensed LOWER triangle, n*(n-1)/2 IEEE-754 binary32
 * values in edge combinatorial-index order: entry i*(i-1)/2 + j holds d(i,j)
 * for i > j (paper, Background: D[i,i] = 0 is implied; the experiments read
 * a lower-triangular matrix).  Entries must be finite and >= 0; -0.0 is read
 * as 0.  The triangle inequality is not required.
 *
 * Threshold.  Inclusive: a simplex is in the complex iff its diameter (its
 * largest pairwise distance) is <= threshold (paper, definition of Rips_t).
 * +INFINITY means no threshold; the library then truncates at the enclosing
 * radius R = min_x max_y d(x,y), which leaves every nonzero interval
 * unchanged (paper, proposition on the enclosing radius), unless
 * RPP_NO_ENCLOSING_RADIUS is given.  NaN or a negative threshold is an error.
 *
 * Result.  Dimensions 0..maxdim.  Each bar is [birth, death) with birth and
 * death equal to entries of the distance matrix (or 0 for H0 births);
 * zero-length intervals (birth == death) are omitted; essential classes have
 * death = +INFINITY.  Bars of a dimension are sorted by birth, then death,
 * +INFINITY last; zeros are written as +0.0.  Results are allocated by the
 * library and released with rpp_result_free.
 *
 * Simplices are identified by their combinatorial index (paper, section on
 * the combinatorial number system): the simplex with vertices
 * v_p > ... > v_0 has cidx = C(v_p, p+1) + ... + C(v_0, 1).
 *
 * Errors.  Every function returning int returns RPP_OK (0) or a negative
 * RPP_E_* code; on error *out is left NULL and rpp_last_error() describes
 * the failure (thread-local text).  Test hook: the environment variable
 * RPP_FAULT_INJECT=<stage>[:<n>] makes every call (or every call on n
 * points) fail with RPP_E_DEVICE at that stage boundary, stage one of
 * stage, h0, enumerate, apparent, host; nothing else changes.
 */
#ifndef RPP_H
#define RPP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RPP_MAX_DIM 4

enum {
    RPP_OK = 0,
    RPP_E_INVAL = -1,  /* null pointer, n < 1, maxdim outside 0..RPP_MAX_DIM, bad threshold */
    RPP_E_DATA = -2,   /* NaN, infinite or negative distance entry */
    RPP_E_RANGE = -3,  /* C(n, maxdim+2) does not fit the index type, or n too large */
    RPP_E_NOMEM = -4,  /* host or device allocation failed, or workspace too small */
    RPP_E_DEVICE = -5, /* HIP runtime error */
    RPP_E_CANCELLED = -6, /* serving request cancelled (rpp_server_cancel) */
};

/* flags for rpp_barcodes_device */
#define RPP_NO_ENCLOSING_RADIUS 0x1u /* use the threshold as given, even if +inf */
#define RPP_WANT_PAIRS 0x2u          /* also return every persistence pair */
/* Keep the apparent pairs as an array sorted by tau, copied to the host and
 * binary-searched by the host reduction (the paper's two-layer store).
 * Default: the host decides whether a row is an apparent pivot by
 * recomputing the apparent-pair condition from the distance matrix, so the
 * apparent pairs are neither sorted nor copied.  Results are identical. */
#define RPP_SORTED_PAIR_STORE 0x4u
/* Enumeration path.  Dense: every C(n, p+1) combinatorial index is examined
 * in order.  Sparse: p-simplices are grown from the (p-1)-simplices under
 * the threshold through neighbour bitsets (paper, sparse 1-skeletons).  By
 * default the sparse path is taken when under a quarter of the edges are
 * within the threshold.  Results are identical. */
#define RPP_FORCE_SPARSE 0x8u
#define RPP_FORCE_DENSE 0x10u
/* Fill rpp_bars.birth_edge / death_edge with each bar's critical edges. */
#define RPP_WANT_CRITICAL_EDGES 0x20u
/* rpp_barcodes_batch: launch each stage eagerly instead of replaying the
 * captured graph (results identical). */
#define RPP_BATCH_NO_GRAPH 0x40u
/* rpp_barcodes_batch: when no tuned parameters exist for a shape, time the
 * candidates on this batch first (results identical). */
#define RPP_BATCH_AUTOTUNE 0x80u
/* Host reduction of the non-apparent columns: when a column's low is the
 * pivot of an earlier host-reduced column k, add k's unreduced coboundary
 * D_k (paper, oblivious matrix reduction, Algorithm 2; nothing is kept once a
 * column is final) instead of its reduced column R_k, kept from k's own
 * reduction (the paper's reduction-matrix technique; the default).  Results
 * are identical (the paper's lemma on oblivious reduction); the oblivious
 * form uses less host memory and may need many more additions. */
#define RPP_OBLIVIOUS_REDUCTION 0x100u
/* The paper's stage order: sort every kept column by (diameter desc, cidx
 * asc) before the apparent-pair test, instead of sorting only the
 * non-apparent columns after it (the default; apparent-ness does not depend
 * on column order, so the results are identical).  Kept for comparison; the
 * sort then runs over every column (stats.ms_sort includes it). */
#define RPP_SORT_FIRST 0x200u
/* rpp_barcodes_batch: group requests by their exact n instead of by shape
 * bucket (n rounded up to a multiple of 64).  Kept for comparison. */
#define RPP_BATCH_EXACT_SHAPES 0x400u

/* Per-dimension counters (paper, tables of apparent pairs and of the
 * clearing / threshold accounting).  For p >= 1:
 *   n_candidates = n_thresholded + n_cleared + n_kept          (dense path)
 *   n_kept       = n_apparent + n_nonapparent
 *   n_simplices  = p-simplices with diameter <= threshold
 * For p = 0, n_kept = n and n_apparent = n_nonapparent = 0. */
typedef struct {
    int64_t n_candidates;   /* simplices examined by the filter */
    int64_t n_simplices;    /* p-simplices with diameter <= threshold */
    int64_t n_thresholded;  /* removed by the threshold */
    int64_t n_cleared;      /* removed by the clearing lemma */
    int64_t n_kept;         /* columns of the dimension-p coboundary matrix */
    int64_t n_apparent;     /* apparent pairs (sigma, tau) found on the GPU */
    int64_t n_nonapparent;  /* columns handed to the host reduction */
    int64_t n_host_pairs;   /* pairs found by the host reduction */
    int64_t n_essential;    /* essential classes */
    int64_t n_bars;         /* reported intervals, essential included */
    int64_t n_column_adds;  /* column additions done by the host reduction */
    int64_t n_scanned;      /* cofacet candidates examined by the apparent test
                               (sum over columns; only when the environment
                               variable RPP_COUNT_SCANS=1, else 0) */
    float ms_gpu;           /* device time of the dimension's GPU stages */
    float ms_host;          /* host reduction wall time */
    float ms_enumerate;     /* device time: enumeration + filter + compaction */
    float ms_apparent;      /* device time: apparent-pair kernel */
    float ms_partition;     /* device time: partition */
    float ms_sort;          /* device time: key sorts and clearing bitmap */
    int32_t apparent_group; /* lanes that test one column in the apparent
                               kernel; negative when it was the sparse kernel
                               (candidates from neighbour bitsets); 100 K + G
                               for the two-phase dense kernel (each lane alone
                               on the top K candidates of its column, then G
                               lanes per column still open), 10000 + 100 K + G
                               for its form that pools the open columns of a
                               workgroup, 20000 + 100 NB + G for the pooled
                               form reading its first NB blocks of 4
                               candidates as 16-byte vectors (NB = 0: 2) */
} rpp_dim_stats;

typedef struct {
    int32_t dim;
    int64_t count;
    float *birth;
    float *death;
    /* Only with RPP_WANT_CRITICAL_EDGES (else NULL): the edge, as a
     * combinatorial index, whose length is the bar's birth / death value:
     * the longest edge of the birth / death simplex, the one of largest
     * cidx among equally long edges.  UINT64_MAX where there is none (H0
     * births, essential deaths). */
    uint64_t *birth_edge;
    uint64_t *death_edge;
} rpp_bars;

/* Only filled with RPP_WANT_PAIRS: every persistence pair (sigma, tau) of
 * dimension dim (zero-length pairs included), sigma a dim-simplex and tau a
 * (dim+1)-simplex, as combinatorial indices.  For dim 0 tau is the edge of
 * each spanning-forest merge and sigma is UINT64_MAX (the vertex side is not
 * tracked).  Order: unspecified. */
typedef struct {
    int32_t dim;
    int64_t count;
    uint64_t *sigma;
    uint64_t *tau;
} rpp_pairs;

typedef struct {
    int32_t maxdim;
    int32_t n;
    float threshold_used;   /* threshold after enclosing-radius truncation */
    float enclosing_radius;
    rpp_bars *dims;         /* maxdim + 1 entries */
    rpp_dim_stats *stats;   /* maxdim + 1 entries */
    rpp_pairs *pairs;       /* maxdim + 1 entries, or NULL */
} rpp_result;

/* Barcodes of a host-resident distance matrix.
 *   dist      condensed lower triangle (host memory, read only, n*(n-1)/2
 *             floats; may be NULL when n == 1)
 *   n         number of points, >= 1
 *   maxdim    highest homology dimension, 0..RPP_MAX_DIM
 *   threshold inclusive diameter threshold, or +INFINITY
 *   out       receives a library-allocated result
 * Uses device 0's current HIP device and its null stream. */
int rpp_barcodes(const float *dist, int32_t n, int32_t maxdim, float threshold,
                 rpp_result **out);

/* As rpp_barcodes, for a distance matrix already resident in device memory
 * (HBM).  Work is issued on hip_stream (a hipStream_t, NULL = null stream)
 * of the current device; the call returns after the result is complete and
 * every kernel it launched has finished.  flags: RPP_*.
 *
 * Device memory.  workspace_dev / workspace_bytes: caller-owned device
 * memory (any alignment is accepted; 256-byte alignment is best) from which
 * EVERY device buffer of the call is carved; the library allocates no device
 * memory of its own for the call and keeps no pointer into the workspace
 * after it returns.  The caller keeps ownership and must not touch the
 * memory during the call.  A workspace of at least rpp_workspace_bytes(n,
 * maxdim, threshold) never runs out.  A smaller one is used as far as it
 * goes (a threshold usually leaves most of that bound unused): the call
 * fails with RPP_E_NOMEM, *out left NULL, as soon as a buffer no longer fits,
 * and up front, before any device work, when workspace_bytes is below what
 * staging and H0 need for n points.  workspace_bytes > 0 with a NULL
 * workspace_dev is RPP_E_INVAL.
 * NULL / 0: the library uses its own grow-only per-device cache; the
 * environment variable RPP_DEVICE_BUDGET_BYTES then caps the device bytes
 * that cache may hold during the call (RPP_E_NOMEM when a buffer would pass
 * it; up front, before any device work, when staging and H0 alone would). */
int rpp_barcodes_device(const float *dist_dev, int32_t n, int32_t maxdim, float threshold,
                        void *workspace_dev, size_t workspace_bytes, void *hip_stream,
                        uint32_t flags, rpp_result **out);

/* One cloud of a batch: a device-resident condensed matrix (as for
 * rpp_barcodes_device), its size, highest dimension and threshold. */
typedef struct {
    const float *dist_dev;
    int32_t n;
    int32_t maxdim;
    float threshold;
} rpp_request;

/* Barcodes of count clouds at once.  Requests with the same maxdim whose n
 * round up to the same multiple of 64 form a shape bucket: each cloud is
 * padded to that size with points at infinite distance (no simplex within
 * the threshold contains one, so every cloud's bars and pairs are its own;
 * the kernels read each cloud's own size from device memory), each stage
 * runs as one launch over the whole bucket, the GPU stages of a dimension
 * are captured once per bucket as a hipGraph and replayed for any mix of
 * sizes in it, and the host reductions of the clouds run in parallel.
 * Padding needs a finite threshold, so a request with threshold +INFINITY
 * under RPP_NO_ENCLOSING_RADIUS groups by its exact n, as every request
 * does under RPP_BATCH_EXACT_SHAPES.  A group of one cloud, or one whose
 * clouds have more than 2^22 candidate simplices in the top dimension (the
 * batch sizes its buffers by that count per cloud), runs cloud by cloud
 * through the single-cloud pipeline of rpp_barcodes_device.  Bars and
 * critical edges are identical to rpp_barcodes_device on each cloud.
 * outs: count pointers, each set to a library-allocated result (free each
 * with rpp_result_free); on error every out is NULL.  flags: RPP_* (pair
 * lists are not supported here). */
int rpp_barcodes_batch(int32_t count, const rpp_request *reqs, void *hip_stream, uint32_t flags,
                       rpp_result **outs);

/* Upper bound of the device workspace that rpp_barcodes_device needs for a
 * matrix of n points, dimensions 0..maxdim, whatever the distances and the
 * threshold (0 on invalid arguments): the sum over the call's device buffers
 * of their largest possible size, every count taken at its combinatorial
 * maximum C(n, p+1).  Also the footprint bound of the serving admission. */
size_t rpp_workspace_bytes(int32_t n, int32_t maxdim, float threshold);

/* Apparent pairs of dimension (p, p+1) over EVERY p-simplex with diameter
 * <= threshold (no clearing, no truncation at the enclosing radius), by the
 * apparent pairs lemma, on the GPU (paper, algorithm for finding apparent
 * pairs; the dimension-1 apparent fraction of its random-order experiments).
 * dist_dev is a device condensed matrix.  Writes at most cap pairs
 * (sigma_cidx, tau_cidx) in increasing sigma order into host arrays
 * sigma_out / tau_out (either may be NULL when cap == 0; with cap == 0 the
 * pairs are only counted and never leave the device) and stores the number
 * of apparent pairs in *count and the number of p-simplices examined in
 * *n_columns.  stats (may be NULL) receives the counts, the GPU stage times
 * and the lanes per column; n_scanned is filled when the environment
 * variable RPP_COUNT_SCANS=1. */
int rpp_apparent_pairs(const float *dist_dev, int32_t n, int32_t p, float threshold,
                       void *hip_stream, uint64_t *sigma_out, uint64_t *tau_out,
                       int64_t cap, int64_t *count, int64_t *n_columns,
                       rpp_dim_stats *stats);

/* Condensed FP32 distance matrix of n points in R^d.  points_dev: n x d
 * FP32 coordinates, row-major, device memory; dist_dev: n*(n-1)/2 floats,
 * device memory, written in edge-cidx order.  Each distance is the square
 * root of the sum of squared coordinate differences, accumulated in FP64 in
 * coordinate order and rounded once to FP32 (the inputs' own recipe).
 * Work is issued on hip_stream; the call returns after it completes. */
int rpp_pdist_device(const float *points_dev, int32_t n, int32_t d, float *dist_dev,
                     void *hip_stream);

/* Gradient of a loss on the bars with respect to the point coordinates,
 * through the bars' critical edges (a bar's birth and death values are the
 * lengths of those edges, and d|x_u - x_v| / dx_u = (x_u - x_v)/|x_u - x_v|).
 *   points_dev        n x d FP32 coordinates (device, row-major)
 *   nbars             number of bars
 *   birth_edge, death_edge   host arrays of nbars edge cidx (UINT64_MAX:
 *                     no edge, no contribution), e.g. from a result made
 *                     with RPP_WANT_CRITICAL_EDGES
 *   grad_birth, grad_death   host arrays of nbars FP32 values dL/dbirth,
 *                     dL/ddeath (may be NULL for all-zero)
 *   grad_points_dev   n x d FP32 output (device), overwritten
 * Each coordinate's gradient is summed in bar order (deterministic).  Edges
 * of zero length contribute nothing.  Returns after completion. */
int rpp_backward(const float *points_dev, int32_t n, int32_t d, int64_t nbars,
                 const uint64_t *birth_edge, const uint64_t *death_edge,
                 const float *grad_birth, const float *grad_death, float *grad_points_dev,
                 void *hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * computation as rpp_backward, with the same arguments and bitwise the same
 * result, but the bar arrays are staged in a fixed device array of the
 * library (RPP_NOALLOC_MAX_BARS bars, 24 bytes each: 6 MiB, held on every
 * GPU the library runs on until the process ends) instead of library-
 * allocated device memory; the call makes no device or host allocation.
 * The caller still provides points_dev and grad_points_dev.
 * nbars > RPP_NOALLOC_MAX_BARS is RPP_E_RANGE, before any device work.
 * Every call on one GPU shares that GPU's array: calls that overlap on the
 * same GPU (from several threads or streams) race and must be serialised
 * by the caller.  Returns after completion, so consecutive calls are safe. */
#define RPP_NOALLOC_MAX_BARS 262144
int rpp_backward_noalloc(const float *points_dev, int32_t n, int32_t d, int64_t nbars,
                         const uint64_t *birth_edge, const uint64_t *death_edge,
                         const float *grad_birth, const float *grad_death,
                         float *grad_points_dev, void *hip_stream);

/* ---- serving -------------------------------------------------------------
 * A server runs requests on `slots` concurrent slots, each with its own HIP
 * stream and device workspace, so the GPU stages of different requests
 * overlap and each request's filtration and clearing state stay in HBM until
 * it finishes.  A request is admitted as soon as a slot is free and its
 * footprint bound (rpp_workspace_bytes + its input) fits hbm_budget_bytes
 * next to the requests in flight (a request larger than the whole budget is
 * admitted alone); the queue is scanned in arrival order.  All functions
 * are thread-safe. */
typedef struct rpp_server rpp_server;

typedef struct {
    int32_t slots;
    size_t budget_bytes;
    size_t in_flight_bytes;         /* sum of footprint bounds now running */
    size_t peak_in_flight_bytes;
    size_t peak_allocated_bytes;    /* device memory held by the slots */
    int32_t peak_concurrency;       /* most requests running at once */
    int64_t admitted, completed, queued;
} rpp_server_info;

/* slots: 1..64; hbm_budget_bytes: 0 = three quarters of the free device
 * memory.  Uses the current device. */
int rpp_server_create(int32_t slots, size_t hbm_budget_bytes, rpp_server **out);
/* Queue a request; dist is a host condensed matrix, copied before return.
 * flags: as rpp_barcodes_device (RPP_WANT_PAIRS is ignored).  *ticket
 * identifies the request for rpp_server_wait. */
int rpp_server_submit(rpp_server *s, const float *dist, int32_t n, int32_t maxdim,
                      float threshold, uint32_t flags, uint64_t *ticket);
/* Block until the request is done; *out receives its result (free with
 * rpp_result_free).  latency_ms: submission to completion; queue_ms:
 * submission to admission (either may be NULL).  Returns the request's own
 * error code if it failed.  Each ticket can be waited for once. */
int rpp_server_wait(rpp_server *s, uint64_t ticket, rpp_result **out, double *latency_ms,
                    double *queue_ms);
/* Cancel a request.  A queued request never runs; a running one stops at
 * its next stage boundary (its GPU work so far completes).  Its
 * rpp_server_wait then returns RPP_E_CANCELLED.  Returns RPP_OK, or
 * RPP_E_INVAL for an unknown, already finished or already waited ticket. */
int rpp_server_cancel(rpp_server *s, uint64_t ticket);
int rpp_server_stats(rpp_server *s, rpp_server_info *st);
/* Finishes the queued requests, then releases everything. */
void rpp_server_destroy(rpp_server *s);

void rpp_result_free(rpp_result *r);

/* Static text for an RPP_E_* code. */
const char *rpp_strerror(int code);

/* Text describing the last error raised on the calling thread. */
const char *rpp_last_error(void);

/* Library version string. */
const char *rpp_version(void);

#ifdef __cplusplus
}
#endif

#endif /* RPP_H */
