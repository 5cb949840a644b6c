// kernels.h -- host-side launchers of the gfx950 kernels (kernels.hip).
//
// Every launcher enqueues work on `stream` and returns immediately; sizes
// that the host needs afterwards are left in device memory for the caller
// to copy back.  Pointers are device pointers unless stated otherwise.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace rpp {

// Batched launches process several clouds at once: cloud c is blockIdx.y
// (blockIdx.x for one-workgroup-per-cloud kernels), its arrays start
// c * stride elements in, and its element count is count[c * cstride] when
// count is set (device memory), else the launch's own count.  The default
// describes a single cloud.
// A shape bucket packs clouds of different sizes at one padded size n:
// nv (device memory, or null) holds each cloud's own number of points; its
// vertices nv[c] .. n-1 are padding, at infinite distance from everything.
struct Batch {
    const uint64_t *count = nullptr;
    int64_t cstride = 0;
    int64_t stride = 0;
    const int32_t *nv = nullptr;
};
#ifdef __HIPCC__
__device__ __forceinline__ int64_t batch_count(const Batch &b, int64_t c, int64_t fallback)
{
    return b.count ? (int64_t)b.count[c * b.cstride] : fallback;
}
__device__ __forceinline__ int batch_nv(const Batch &b, int64_t c, int n)
{
    return b.nv ? b.nv[c] : n;
}
#endif

// ---- a1: staging -------------------------------------------------------
// Square n x n copy (zero diagonal, -0 folded to +0), per-row maxima, and a
// validity flag (bit 0 set when an entry is NaN, infinite or negative).
void launch_stage(const float *dcond, int n, float *dsq, float *rowmax, uint32_t *bad,
                  hipStream_t s);
// out[0] = min over rows of rowmax (the enclosing radius).
void launch_min(const float *x, int n, float *out, hipStream_t s);
// Batched staging of nb clouds of n points (inputs and outputs packed cloud
// after cloud), and per-cloud radius / threshold used.
// nv (device, or null): each cloud's own number of points in a shape bucket
// of padded size n; entries of padding vertices must already hold +inf in
// dcond (launch_pad_dcond_b) and are neither validated nor counted in the
// row maxima or the radius.
void launch_stage_b(const float *dcond, int n, int nb, float *dsq, float *rowmax, uint32_t *bad,
                    hipStream_t s, const int32_t *nv = nullptr);
void launch_radius_b(const float *rowmax, int n, int nb, const float *req, int no_radius,
                     float *radius, float *thr, hipStream_t s, const int32_t *nv = nullptr);
// Per cloud of a bucket: condensed entries nv(nv-1)/2 .. n(n-1)/2 - 1 (the
// padding vertices' edges) set to +inf.
void launch_pad_dcond_b(float *dcond, int n, int nb, const int32_t *nv, hipStream_t s);

// ---- device-wide helpers --------------------------------------------------
void launch_fill_u32(uint32_t *p, int64_t count, uint32_t value, hipStream_t s);
// Exclusive scan of u32 counts into u64 offsets; out has len+1 entries and
// out[len] is the total.  scratch must hold scan_scratch_words(len) u64.
int64_t scan_scratch_words(int64_t len);
void launch_exclusive_scan(const uint32_t *in, int64_t len, uint64_t *out, uint64_t *scratch,
                           hipStream_t s);
// Batched: nbatch independent scans of len entries each, in cloud after
// cloud (out: len+1 per cloud; scratch: scan_scratch_words(len) per cloud).
void launch_exclusive_scan_b(const uint32_t *in, int64_t len, int nbatch, uint64_t *out,
                             uint64_t *scratch, hipStream_t s);

// ---- a3 + a4: enumeration with threshold and clearing --------------------
constexpr int64_t COMPACT_TILE = 4096;  // candidates per workgroup
inline int64_t compact_tiles(int64_t count) { return (count + COMPACT_TILE - 1) / COMPACT_TILE; }

struct EnumArgs {
    const float *dcond;        // condensed distances (edge cidx order)
    int n;
    int p;                     // simplex dimension, 1..4
    float thr;                 // inclusive threshold
    const uint64_t *binom;     // C(v,k) table, stride n+1
    const uint32_t *clear;     // clearing bitmap over C(n,p+1) cidx, or null
    uint64_t ncand;            // C(n, p+1)
    // batched launches (nbatch clouds of n points, packed one after the
    // other): per-cloud thresholds, bitmap stride (u32 words) and output
    // stride (elements); tile counts / offsets are laid out per cloud
    const float *thr_dev = nullptr;
    int64_t clear_stride = 0;
    int64_t out_stride = 0;
    int nbatch = 1;
};
// Pass 1: kept count per tile; stats[0] += thresholded, stats[1] += cleared
// (per cloud), unless stats is null.
void launch_enum_count(const EnumArgs &a, uint32_t *tile_counts,
                       unsigned long long *stats, hipStream_t s);
// Pass 2: write kept simplices (diameter, cidx) in increasing cidx order.
// out_vtx (p = 2 or 3, n <= 65536, or null): each kept simplex's vertices
// v_0 > ... > v_p packed 16 bits each, v_i at bit 16 i.
void launch_enum_scatter(const EnumArgs &a, const uint64_t *tile_offsets, float *out_diam,
                         uint64_t *out_cidx, hipStream_t s, uint64_t *out_vtx = nullptr);

// One pass for a single cloud whose outputs hold every candidate: the kept
// simplices as launch_enum_scatter writes them, each tile's offset found by
// a decoupled look-back over the tiles before it (no count pass, no scan).
// status: tiles + 1 words of scratch (cleared here); *total (device) gets
// the kept count.  Statistics are not counted.
void launch_enum_onepass(const EnumArgs &a, unsigned long long *status, uint64_t *total,
                         float *out_diam, uint64_t *out_cidx, hipStream_t s,
                         uint64_t *out_vtx = nullptr);

// ---- a5: apparent-pair test -----------------------------------------------
// tau_out[i] = cidx of the apparent partner of column i, or ~0 when the
// column is not apparent.  group = lanes cooperating on one column.  When
// scan_count is not null (SCAN_COUNTERS u64 slots, zeroed by the caller)
// the number of cofacet candidates each column examines in decreasing
// vertex order, up to and including the first equal-diameter cofacet (all
// n-p-1 when there is none), is added to it.
constexpr int SCAN_COUNTERS = 1024;
void launch_apparent(const float *col_diam, const uint64_t *col_cidx, int64_t ncols,
                     const float *dsq, int n, int p, const uint64_t *binom, int group,
                     uint64_t *tau_out, unsigned long long *scan_count, hipStream_t s);
// Row-padded copy of the n x n matrix: out[r * pitch + c] = dsq[r * n + c]
// for c < n, pitch a multiple of 4 (16-byte aligned rows), 0 in the pad.
void launch_pad_rows(const float *dsq, int n, int pitch, float *out, hipStream_t s);
// The two-phase apparent test with vector reads of the first candidates
// over the row-padded matrix (group = 20000 + 100 NB + G: NB aligned blocks
// of 4 candidates, NB in {2, 3, 4}, 0 meaning 2; G = 16 only with 2 blocks,
// else 8); the same output as launch_apparent.
// col_vtx (or null): the columns' packed vertex tuples, as launch_enum_scatter
// writes them, read instead of decoding col_cidx.
void launch_apparent_vec(const float *col_diam, const uint64_t *col_cidx, int64_t ncols,
                         const float *dsqp, int pitch, int n, int p, const uint64_t *binom,
                         int group, uint64_t *tau_out, unsigned long long *scan_count,
                         hipStream_t s, const uint64_t *col_vtx = nullptr);
// Batched: cap = per-cloud capacity (grid size); dsq packed n*n per cloud.
// rounds (0: from the column count) and block (64, 128 or 256 threads per
// workgroup) as the autotuner picks them.
void launch_apparent_b(const float *col_diam, const uint64_t *col_cidx, int64_t cap,
                       const float *dsq, int n, int p, const uint64_t *binom, int group,
                       uint64_t *tau_out, Batch bt, int nbatch, hipStream_t s, int rounds = 0,
                       int block = 256);

// ---- a6: partition --------------------------------------------------------
// Pass 1: apparent columns per tile.
void launch_partition_count(const uint64_t *tau, int64_t ncols, uint32_t *tile_counts,
                            hipStream_t s, Batch bt = Batch(), int nbatch = 1);
// Pass 2: apparent -> (tau, sigma) pairs; non-apparent -> (key, cidx) with
// key = ~bits(diameter), both in increasing column (cidx) order.
void launch_partition_scatter(const uint64_t *tau, const float *col_diam,
                              const uint64_t *col_cidx, int64_t ncols,
                              const uint64_t *tile_offsets, uint64_t *app_tau,
                              uint64_t *app_sigma, uint64_t *na_key, uint64_t *na_cidx,
                              hipStream_t s, Batch bt = Batch(), int nbatch = 1);
// key[i] = ~bits(diam[i]) (descending-diameter radix key).
void launch_diam_from_keys(const uint64_t *keys, int64_t count, float *diam, hipStream_t s);
// Rank-coded diameters (host reduction of the sparse path): flags of the
// edges (sorted by diameter descending) that start a new length; after an
// exclusive scan of the flags (excl, m + 1 entries), the n x n matrix of
// ranks as floats (`above` beyond the threshold, 0 on the diagonal) and the
// table vals[rank] of the distinct lengths, ascending.
void launch_rank_flags(const uint64_t *keys, int64_t m, uint32_t *flags, hipStream_t s);
void launch_rank_matrix(const uint64_t *keys, const uint64_t *cidx, const uint32_t *flags,
                        const uint64_t *excl, int64_t m, int n, float above, float *rk,
                        float *vals, hipStream_t s);
// Recodes column keys (~bits(diameter)) and low diameters as ranks.
void launch_recode_ranks(uint64_t *keys, float *lowd, int64_t m, const float *vals, int64_t R,
                         hipStream_t s);
void launch_desc_keys(const float *diam, int64_t count, uint64_t *keys, hipStream_t s,
                      Batch bt = Batch(), int nbatch = 1);

// ---- a7: host handoff -------------------------------------------------------
// For every non-apparent column (key = ~bits(diameter), cidx): its oldest
// cofacet inside the threshold, i.e. the low of the unreduced coboundary
// column (smallest diameter, then largest cidx), or ~0 when the coboundary
// is empty.  One wave per column.
void launch_lows(const uint64_t *na_key, const uint64_t *na_cidx, int64_t ncols,
                 const float *dsq, int n, int p, float thr, const uint64_t *binom,
                 uint64_t *low_out, float *low_diam_out, hipStream_t s, Batch bt = Batch(),
                 int nbatch = 1, const float *thr_dev = nullptr);

// ---- sparse path (a threshold that keeps few edges) -------------------------
// Neighbour bitsets: bit b of bits[v * words + k] is set iff u = 64k + b is a
// vertex, u != v and d(u, v) <= thr.
void launch_nbr_bits(const float *dsq, int n, float thr, uint64_t *bits, int words,
                     hipStream_t s);

// Packed neighbour rows (sparse path).  nbd lists every vertex's neighbours'
// distances (d <= thr, the vertex itself excluded), row after row, the
// neighbours of a row in ascending order.  nbw[v*words + k] is a 16-byte
// record (x, y: bitset word k of v's row, low and high halves; z: position
// in nbd of v's first neighbour in that word; w: 0), read with one load, so
// a neighbour u = 64k + b of v has d(v, u) = nbd[z + popcount(word &
// (2^b - 1))].  The rows hold the 2E distances of the E edges under the
// threshold: a few MB that stay in L2 where the square matrix (n^2 floats)
// does not.
void launch_nbr_degree(const uint64_t *bits, int n, int words, uint32_t *deg, hipStream_t s);
// row_off: exclusive scan of the degrees (n + 1 entries); cap: entries nbd
// holds (2E; writes past it are dropped)
void launch_nbr_pack(const float *dsq, const uint64_t *bits, int n, int words,
                     const uint64_t *row_off, uint4 *nbw, float *nbd, uint64_t cap,
                     hipStream_t s);

// p-simplices <= thr as one-vertex extensions of the (p-1)-simplices <= thr
// (paper, enumeration of cofacets for sparse 1-skeletons): prefix
// (v_p > ... > v_1) extends by every common neighbour v_0 < v_1.  Listing
// prefixes in cidx order and v_0 upward yields the p-simplices in cidx order.
// Distances come from the packed neighbour rows.
struct ExtArgs {
    int n;
    int p;                           // dimension of the produced simplices, >= 2
    int words;
    const uint4 *nbw;                // packed neighbour rows
    const float *nbd;
    const uint64_t *binom;
    const float *pre_diam;           // (p-1)-simplices <= thr, cidx order
    const uint64_t *pre_cidx;
    int64_t npre_count;              // number of prefixes
};
// Pass 1: per prefix, the number of extensions.
void launch_ext_count(const ExtArgs &a, uint32_t *cnt_all, hipStream_t s);
// Pass 2, with the clearing filter (the paper's clearing lemma) fused in:
// every extension is written to all_diam/all_cidx at the scanned offsets
// off_all (skipped when all_diam is null), and those not in `clear` -- the
// sorted cidx of the previous dimension's pivot rows, a subset of the
// extensions -- to kept_diam/kept_cidx, in cidx order.  A prefix's kept
// entries start at off_all[prefix] minus the number of clear entries below
// the prefix's first extension, which one wave-wide search of `clear`
// finds; the kept total is (number of extensions) - nclear, and kept_cap
// (that total) bounds the kept writes.  kept_vtx (may be null; used for
// p <= 3 and n <= 65536): the kept columns' vertex tuples, 16 bits per
// vertex from the largest.
void launch_ext_scatter(const ExtArgs &a, const uint64_t *off_all, float *all_diam,
                        uint64_t *all_cidx, const uint64_t *clear, int64_t nclear,
                        float *kept_diam, uint64_t *kept_cidx, uint64_t kept_cap,
                        uint64_t *kept_vtx, hipStream_t s,
                        const int64_t *cpos = nullptr);
// The scatter pass with the apparent-pair test of every kept extension fused
// in (two-phase form; group = 100 K + G as for launch_apparent_sparse):
// tau_out[kept position] = its apparent partner or NONE; scan_count as for
// launch_apparent.  No vertex tuples are written.
void launch_ext_scatter_apparent(const ExtArgs &a, int group, const uint64_t *off_all,
                                 float *all_diam, uint64_t *all_cidx, const uint64_t *clear,
                                 int64_t nclear, float *kept_diam, uint64_t *kept_cidx,
                                 uint64_t kept_cap, uint64_t *tau_out,
                                 unsigned long long *scan_count, hipStream_t s,
                                 const int64_t *cpos = nullptr);
// cpos[pre] = entries of the sorted clearing set below prefix pre's first
// extension (what the fused scatter otherwise searches for itself).
void launch_clear_pos(const ExtArgs &a, const uint64_t *clear, int64_t nclear, int64_t *cpos,
                      hipStream_t s);
// Apparent test and lows for the sparse path: candidates are the common
// neighbours of the column's vertices, scanned from the top.  group = G in
// {4, 8, 16}: G words per step by as many lanes per column; group = 100 K +
// G (K in {1, 2, 4}, G in {4, 8}): the two-phase form, each lane alone on
// its column's top K words first, then G lanes per column still open.
// Anything else means the default, 404.
int sparse_group(int group);
void launch_apparent_sparse(const float *col_diam, const uint64_t *col_cidx, int64_t ncols,
                            int n, int p, int words, const uint4 *nbw, const float *nbd,
                            const uint64_t *binom, int group, uint64_t *tau_out,
                            unsigned long long *scan_count, hipStream_t s,
                            const uint64_t *col_vtx = nullptr);
void launch_lows_sparse(const uint64_t *na_key, const uint64_t *na_cidx, int64_t ncols,
                        const uint4 *nbw, const float *nbd, int n, int p, int words,
                        const uint64_t *binom, uint64_t *low_out, float *low_diam_out,
                        hipStream_t s);

// ---- a7: clearing bitmap ---------------------------------------------------
void launch_mark_bits(const uint64_t *idx, int64_t count, uint32_t *bits, hipStream_t s,
                      Batch bt = Batch(), int nbatch = 1, int64_t bits_stride = 0);

// ---- a2: H0 by union-find ---------------------------------------------------
// Edges sorted in coboundary order (diameter descending, cidx ascending);
// processed from the back, i.e. in filtration order.  Sets the MST bit of
// each spanning-forest edge, writes the nonzero death diameters to deaths
// (and the edge to death_edges[i]), counters[0] = #deaths, counters[1] =
// #merges.  uf_scratch: 2n ints, used when the union-find arrays do not fit
// in LDS.
void launch_kruskal(const uint64_t *edge_key, const uint64_t *edge_cidx, int64_t nedges, int n,
                    uint32_t *mst_bits, float *deaths, uint64_t *death_edges, int *counters,
                    int *uf_scratch, hipStream_t s, Batch bt = Batch(), int nbatch = 1,
                    int64_t mst_stride = 0);

// ---- distances and gradients ---------------------------------------------
// Condensed FP32 distances of n points in R^d (row-major FP32 coordinates):
// squared differences summed in FP64 in coordinate order, FP64 square root,
// one rounding to FP32.  No contraction into fused multiply-adds.
void launch_pdist(const float *pts, int n, int d, float *dist, hipStream_t s);
// grad[u*d + k] = sum over terms t (in order) touching u of
//   g_t * (x_u - x_v)_k / |x_u - x_v|   (u, v the endpoints of edge e_t),
// zero-length edges contributing nothing.  One thread per coordinate.
void launch_edge_grad(const float *pts, int n, int d, const uint64_t *edges, const float *g,
                      int64_t nterms, float *grad, hipStream_t s);

// ---- a6: LDS radix sort -------------------------------------------------
// Stable LSD radix sort of (key, value) pairs on key bits [0, bits).  The
// sorted data end up in either the input or the alternate buffers; the
// return value is 0 when they are in (keys, vals), 1 when in (keys_alt,
// vals_alt).  scratch must hold radix_scratch_words(count) u64.
int64_t radix_scratch_words(int64_t count, int nbatch = 1);
int radix_sort_pairs(uint64_t *keys, uint64_t *vals, uint64_t *keys_alt, uint64_t *vals_alt,
                     int64_t count, int bits, uint64_t *scratch, hipStream_t s);
// Batched: count = per-cloud capacity (stride), per-cloud counts in bt.
int radix_sort_pairs_b(uint64_t *keys, uint64_t *vals, uint64_t *keys_alt, uint64_t *vals_alt,
                       int64_t count, int bits, uint64_t *scratch, hipStream_t s, Batch bt,
                       int nbatch);

}  // namespace rpp
