// kernels.hip -- gfx950 kernels of the Vietoris-Rips hot path.
//
// Wave64 throughout: compaction ranks come from 64-bit ballots and
// popcounts, the apparent-pair scan uses sub-wave groups that read
// contiguous runs of a distance-matrix row, and the sort ranks digits with
// wave-level match masks staged in LDS.  No MFMA: nothing here is a dense
// contraction.
#include "device_common.h"
#include "kernels.h"

#include <limits.h>

namespace rpp {

// ===========================================================================
// block-level helpers
// ===========================================================================
template <typename T>
__device__ __forceinline__ T wave_inclusive_scan(T v)
{
    const int lane = threadIdx.x & (WAVE - 1);
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
        T t = __shfl_up(v, o, WAVE);
        if (lane >= o)
            v += t;
    }
    return v;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v)
{
#pragma unroll
    for (int o = WAVE / 2; o > 0; o >>= 1)
        v += __shfl_xor(v, o, WAVE);
    return v;
}

// Exclusive scan across the block (blockDim.x = NT); *total gets the sum.
// `sh` must hold NT/64 + 1 elements.  Contains barriers: call from all
// threads.
template <int NT, typename T>
__device__ __forceinline__ T block_exclusive_scan(T v, T *total, T *sh)
{
    const int lane = threadIdx.x & (WAVE - 1);
    const int wave = threadIdx.x / WAVE;
    constexpr int NW = NT / WAVE;
    T inc = wave_inclusive_scan(v);
    if (lane == WAVE - 1)
        sh[wave] = inc;
    __syncthreads();
    if (threadIdx.x == 0) {
        T run = 0;
        for (int w = 0; w < NW; ++w) {
            T t = sh[w];
            sh[w] = run;
            run += t;
        }
        sh[NW] = run;
    }
    __syncthreads();
    T out = sh[wave] + inc - v;
    *total = sh[NW];
    __syncthreads();
    return out;
}

template <int NT, typename T>
__device__ __forceinline__ T block_sum(T v, T *sh)
{
    const int lane = threadIdx.x & (WAVE - 1);
    const int wave = threadIdx.x / WAVE;
    constexpr int NW = NT / WAVE;
    v = wave_sum(v);
    if (lane == 0)
        sh[wave] = v;
    __syncthreads();
    T s = 0;
    if (threadIdx.x == 0)
        for (int w = 0; w < NW; ++w)
            s += sh[w];
    __syncthreads();
    return s;  // valid in thread 0
}

// ===========================================================================
// a1: staging -- square matrix, row maxima, validation
// ===========================================================================
__global__ __launch_bounds__(256) void k_stage(const float *__restrict__ dcond, int n,
                                               float *__restrict__ dsq,
                                               float *__restrict__ rowmax,
                                               uint32_t *__restrict__ bad,
                                               const int32_t *__restrict__ nvs)
{
    __shared__ float sh[5];
    const int i = blockIdx.x;
    int nv = n;  // the cloud's own points; the rest is bucket padding
    {   // batched launch: cloud blockIdx.y, arrays packed cloud after cloud
        const int64_t c = blockIdx.y;
        dcond += c * ((int64_t)n * (n - 1) / 2);
        dsq += c * (int64_t)n * n;
        rowmax += c * n;
        bad += c;
        if (nvs)
            nv = nvs[c];
    }
    float mx = 0.0f;
    uint32_t flag = 0;
    const int64_t rowi = (int64_t)i * (i - 1) / 2;
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
        float d;
        if (j == i)
            d = 0.0f;
        else if (j < i)
            d = dcond[rowi + j];
        else
            d = dcond[(int64_t)j * (j - 1) / 2 + i];
        const bool real = i < nv && j < nv;
        if (real && (!(d >= 0.0f) || isinf(d)))
            flag = 1;
        d = d + 0.0f;
        dsq[(int64_t)i * n + j] = d;
        if (j < nv)
            mx = fmaxf(mx, d);
    }
    // block max
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        mx = fmaxf(mx, __shfl_xor(mx, o, 64));
    if (lane == 0)
        sh[wave] = mx;
    if (flag)
        atomicOr(bad, 1u);
    __syncthreads();
    if (threadIdx.x == 0) {
        float m = sh[0];
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w)
            m = fmaxf(m, sh[w]);
        rowmax[i] = m;
    }
}

__global__ __launch_bounds__(1024) void k_min(const float *__restrict__ x, int n,
                                              float *__restrict__ out)
{
    __shared__ float sh[16];
    float m = INFINITY;
    for (int i = threadIdx.x; i < n; i += blockDim.x)
        m = fminf(m, x[i]);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        m = fminf(m, __shfl_xor(m, o, 64));
    if ((threadIdx.x & 63) == 0)
        sh[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        float r = sh[0];
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w)
            r = fminf(r, sh[w]);
        out[0] = r;
    }
}

void launch_stage(const float *dcond, int n, float *dsq, float *rowmax, uint32_t *bad,
                  hipStream_t s)
{
    hipLaunchKernelGGL(k_stage, dim3(n), dim3(256), 0, s, dcond, n, dsq, rowmax, bad,
                       (const int32_t *)nullptr);
}

void launch_min(const float *x, int n, float *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_min, dim3(1), dim3(1024), 0, s, x, n, out);
}

void launch_stage_b(const float *dcond, int n, int nb, float *dsq, float *rowmax, uint32_t *bad,
                    hipStream_t s, const int32_t *nv)
{
    hipLaunchKernelGGL(k_stage, dim3(n, nb), dim3(256), 0, s, dcond, n, dsq, rowmax, bad, nv);
}

__global__ void k_pad_dcond(float *__restrict__ dcond, int n, const int32_t *__restrict__ nvs)
{
    const int64_t c = blockIdx.y;
    const int64_t E = (int64_t)n * (n - 1) / 2;
    const int64_t nv = nvs[c];
    const int64_t t = nv * (nv - 1) / 2 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < E)
        dcond[c * E + t] = INFINITY;
}

void launch_pad_dcond_b(float *dcond, int n, int nb, const int32_t *nv, hipStream_t s)
{
    // the largest padding region is that of the smallest cloud: bound it by
    // the whole matrix (threads past a cloud's region exit)
    const int64_t E = (int64_t)n * (n - 1) / 2;
    if (E <= 0 || nb <= 0)
        return;
    hipLaunchKernelGGL(k_pad_dcond, dim3((unsigned)((E + 255) / 256), nb), dim3(256), 0, s, dcond,
                       n, nv);
}

// Per cloud: radius = min over rows of the row maxima; the threshold used is
// the radius when the requested one is +inf (unless no_radius), else the
// requested one.  One block per cloud.
__global__ __launch_bounds__(1024) void k_radius_b(const float *__restrict__ rowmax, int n,
                                                  const float *__restrict__ req, int no_radius,
                                                  float *__restrict__ radius,
                                                  float *__restrict__ thr,
                                                  const int32_t *__restrict__ nvs)
{
    __shared__ float sh[16];
    const int c = blockIdx.x;
    const int nv = nvs ? nvs[c] : n;
    float m = INFINITY;
    for (int i = threadIdx.x; i < nv; i += blockDim.x)
        m = fminf(m, rowmax[(int64_t)c * n + i]);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        m = fminf(m, __shfl_xor(m, o, 64));
    if ((threadIdx.x & 63) == 0)
        sh[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        float r = sh[0];
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w)
            r = fminf(r, sh[w]);
        radius[c] = r;
        const float q = req[c];
        thr[c] = (isinf(q) && !no_radius) ? r : q;
    }
}

void launch_radius_b(const float *rowmax, int n, int nb, const float *req, int no_radius,
                     float *radius, float *thr, hipStream_t s, const int32_t *nv)
{
    hipLaunchKernelGGL(k_radius_b, dim3(nb), dim3(1024), 0, s, rowmax, n, req, no_radius, radius,
                       thr, nv);
}

// ===========================================================================
// fill and device-wide exclusive scan (u32 counts -> u64 offsets)
// ===========================================================================
__global__ void k_fill_u32(uint32_t *p, int64_t count, uint32_t value)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < count; i += stride)
        p[i] = value;
}

void launch_fill_u32(uint32_t *p, int64_t count, uint32_t value, hipStream_t s)
{
    if (count <= 0)
        return;
    int64_t blocks = (count + 255) / 256;
    if (blocks > 65536)
        blocks = 65536;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, s, p, count, value);
}

constexpr int SCAN_T = 1024;
constexpr int SCAN_I = 4;
constexpr int64_t SCAN_CHUNK = SCAN_T * SCAN_I;

int64_t scan_scratch_words(int64_t len)
{
    return (len + SCAN_CHUNK - 1) / SCAN_CHUNK + 2;
}

__global__ __launch_bounds__(SCAN_T) void k_scan_partial(const uint32_t *__restrict__ in,
                                                         int64_t len,
                                                         uint64_t *__restrict__ part)
{
    __shared__ uint64_t sh[SCAN_T / WAVE + 1];
    in += (int64_t)blockIdx.y * len;
    part += (int64_t)blockIdx.y * (gridDim.x + 2);
    const int64_t base = (int64_t)blockIdx.x * SCAN_CHUNK;
    uint64_t s = 0;
#pragma unroll
    for (int k = 0; k < SCAN_I; ++k) {
        int64_t i = base + (int64_t)k * SCAN_T + threadIdx.x;
        if (i < len)
            s += in[i];
    }
    s = block_sum<SCAN_T>(s, sh);
    if (threadIdx.x == 0)
        part[blockIdx.x] = s;
}

__global__ __launch_bounds__(SCAN_T) void k_scan_top(uint64_t *__restrict__ part, int nb)
{
    __shared__ uint64_t sh[SCAN_T / WAVE + 1];
    part += (int64_t)blockIdx.y * (nb + 2);
    uint64_t carry = 0;
    for (int start = 0; start < nb; start += SCAN_T) {
        int i = start + threadIdx.x;
        uint64_t v = (i < nb) ? part[i] : 0;
        uint64_t tot;
        uint64_t ex = block_exclusive_scan<SCAN_T>(v, &tot, sh);
        if (i < nb)
            part[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0)
        part[nb] = carry;
}

__global__ __launch_bounds__(SCAN_T) void k_scan_apply(const uint32_t *__restrict__ in,
                                                       int64_t len,
                                                       const uint64_t *__restrict__ part, int nb,
                                                       uint64_t *__restrict__ out)
{
    __shared__ uint64_t sh[SCAN_T / WAVE + 1];
    in += (int64_t)blockIdx.y * len;
    part += (int64_t)blockIdx.y * (nb + 2);
    out += (int64_t)blockIdx.y * (len + 1);
    const int64_t base = (int64_t)blockIdx.x * SCAN_CHUNK;
    uint64_t carry = part[blockIdx.x];
#pragma unroll
    for (int k = 0; k < SCAN_I; ++k) {
        int64_t i = base + (int64_t)k * SCAN_T + threadIdx.x;
        uint64_t v = (i < len) ? in[i] : 0;
        uint64_t tot;
        uint64_t ex = block_exclusive_scan<SCAN_T>(v, &tot, sh);
        if (i < len)
            out[i] = carry + ex;
        carry += tot;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0)
        out[len] = part[nb];
}

void launch_exclusive_scan_b(const uint32_t *in, int64_t len, int nbatch, uint64_t *out,
                             uint64_t *scratch, hipStream_t s)
{
    int nb = (int)((len + SCAN_CHUNK - 1) / SCAN_CHUNK);
    if (nb == 0) {
        launch_fill_u32(reinterpret_cast<uint32_t *>(out), 2, 0u, s);
        return;
    }
    hipLaunchKernelGGL(k_scan_partial, dim3(nb, nbatch), dim3(SCAN_T), 0, s, in, len, scratch);
    hipLaunchKernelGGL(k_scan_top, dim3(1, nbatch), dim3(SCAN_T), 0, s, scratch, nb);
    hipLaunchKernelGGL(k_scan_apply, dim3(nb, nbatch), dim3(SCAN_T), 0, s, in, len, scratch, nb,
                       out);
}

void launch_exclusive_scan(const uint32_t *in, int64_t len, uint64_t *out, uint64_t *scratch,
                           hipStream_t s)
{
    launch_exclusive_scan_b(in, len, 1, out, scratch, s);
}

// ===========================================================================
// a3 + a4: dense enumeration in cidx order, threshold and clearing filter
// ===========================================================================
constexpr int CT = 256;
constexpr int CI = (int)(COMPACT_TILE / CT);

// Condensed lookup d(a, b) for a > b.
__device__ __forceinline__ float dc_at(const float *__restrict__ dcond, int a, int b)
{
    return dcond[(int64_t)a * (a - 1) / 2 + b];
}

// Per-cloud view of the enumeration arguments (batched launches).
__device__ __forceinline__ EnumArgs enum_view(EnumArgs a)
{
    const int64_t c = blockIdx.y;
    if (c) {
        a.dcond += c * ((int64_t)a.n * (a.n - 1) / 2);
        if (a.clear)
            a.clear += c * a.clear_stride;
    }
    if (a.thr_dev)
        a.thr = a.thr_dev[c];
    return a;
}

// A lane's walk through consecutive candidates.  A wave owns a contiguous
// run of CI * 64 candidates of its workgroup's tile and steps through it 64
// at a time, lane i at candidate run + 64 k + i, so reads and writes stay
// coalesced; instead of decoding every candidate, a lane moves its vertex
// tuple forward by 64: within the current row (v_0 .. v_{P-1} fixed) the
// last vertex just grows, across up to four row ends the next-to-last vertex
// carries, and only a longer jump decodes afresh.  The walk itself is
// register arithmetic, so a chunk of steps computes all its condensed
// offsets first and then issues every load of the chunk at once.
template <int P> struct EnumWalk {
    static constexpr int NPAIR = (P + 1) * P / 2;
    int v[P + 1];
    // to candidate c_new = current + delta (c_new < number of candidates)
    __device__ __forceinline__ void advance(const Binom &B, uint64_t c_new, int delta, int n)
    {
        const int x = v[P] + delta;
        if (x < v[P - 1]) {
            v[P] = x;
            return;
        }
        int y = v[P - 1] + 1;  // next row: v_P runs over [0, y)
        int e = x - v[P - 1];  // position in it
        const int lim = P >= 2 ? v[P >= 2 ? P - 2 : 0] : n;
        for (int it = 0; it < 3 && e >= y && y + 1 < lim; ++it) {
            e -= y;  // past that row too
            ++y;
        }
        if (y < lim && e < y) {
            v[P - 1] = y;
            v[P] = e;
        } else {
            decode<P>(B, c_new, n, v);
        }
    }
    // condensed offsets a (a - 1) / 2 + b of every pair a > b of the simplex
    // (n <= 65535 keeps them below 2^31)
    __device__ __forceinline__ void offsets(uint32_t (&o)[NPAIR]) const
    {
        int q = 0;
#pragma unroll
        for (int i = 0; i < P; ++i) {
            const uint32_t r = (uint32_t)v[i] * (uint32_t)(v[i] - 1) / 2u;
#pragma unroll
            for (int j = i + 1; j <= P; ++j)
                o[q++] = r + (uint32_t)v[j];
        }
    }
};

// Steps per chunk of the walk: all loads of a chunk are in flight together.
template <int P> struct EnumChunk {
    static constexpr int S = P <= 2 ? 8 : P == 3 ? 4 : 2;
};

// Diameters of the candidates c0 + 64 (k0 + s), s < S, of a lane's walk
// (valid where the candidate exists), advancing the walk past them.
template <int P, int S, bool VTX = false>
__device__ __forceinline__ void enum_chunk(EnumWalk<P> &wk, const Binom &B, const EnumArgs &a,
                                           uint64_t c, int k0, float (&d)[S],
                                           uint64_t *vtx = nullptr)
{
    constexpr int NP = EnumWalk<P>::NPAIR;
    uint32_t o[S][NP];
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const uint64_t cs = c + (uint64_t)s * WAVE;
        if (cs < a.ncand) {
            wk.offsets(o[s]);
            if (VTX) {
                uint64_t x = 0;
#pragma unroll
                for (int i = 0; i <= P; ++i)
                    x |= (uint64_t)(uint32_t)wk.v[i] << (16 * i);
                vtx[s] = x;  // vtx: an array of S, indexed by constants
            }
            if (k0 + s + 1 < CI && cs + WAVE < a.ncand)
                wk.advance(B, cs + WAVE, WAVE, a.n);
        } else {
#pragma unroll
            for (int q = 0; q < NP; ++q)
                o[s][q] = 0;  // a harmless load; the candidate is ignored
        }
    }
#pragma unroll
    for (int s = 0; s < S; ++s) {
        float x = 0.0f;
#pragma unroll
        for (int q = 0; q < NP; ++q)
            x = fmaxf(x, a.dcond[o[s][q]]);
        d[s] = x + 0.0f;  // -0 -> +0
    }
}

// 0 = kept, 1 = removed by the threshold, 2 = removed by clearing.
__device__ __forceinline__ int enum_filter(const EnumArgs &a, uint64_t c, float d)
{
    if (!(d <= a.thr))
        return 1;
    if (a.clear && ((a.clear[c >> 5] >> (c & 31)) & 1u))
        return 2;
    return 0;
}

template <int P>
__global__ __launch_bounds__(CT) void k_enum_count(EnumArgs a0, uint32_t *__restrict__ tile_counts,
                                                   unsigned long long *__restrict__ stats)
{
    __shared__ uint32_t sh[CT / WAVE + 1];
    const EnumArgs a = enum_view(a0);
    const bool count_stats = stats != nullptr;
    tile_counts += (int64_t)blockIdx.y * gridDim.x;
    if (count_stats)
        stats += 2 * blockIdx.y;
    const Binom B{a.binom, a.n + 1};
    const int lane = threadIdx.x & (WAVE - 1), wave = threadIdx.x / WAVE;
    const uint32_t tile = xcd_block(blockIdx.x, gridDim.x);
    uint64_t c = (uint64_t)tile * COMPACT_TILE + (uint64_t)wave * (CI * WAVE) + lane;
    uint32_t keep = 0, nthr = 0, nclr = 0;
    if (P == 1) {
        for (int k = 0; k < CI && c < a.ncand; ++k, c += WAVE) {
            const int r = enum_filter(a, c, a.dcond[c] + 0.0f);
            keep += (r == 0);
            nthr += (r == 1);
            nclr += (r == 2);
        }
    } else if (c < a.ncand) {
        constexpr int S = EnumChunk<P>::S;
        EnumWalk<P> wk;
        decode<P>(B, c, a.n, wk.v);
#pragma unroll
        for (int k0 = 0; k0 < CI; k0 += S) {
            float d[S];
            enum_chunk<P, S>(wk, B, a, c, k0, d);
#pragma unroll
            for (int s = 0; s < S; ++s) {
                const uint64_t cs = c + (uint64_t)s * WAVE;
                if (cs < a.ncand) {
                    const int r = enum_filter(a, cs, d[s]);
                    keep += (r == 0);
                    nthr += (r == 1);
                    nclr += (r == 2);
                }
            }
            c += (uint64_t)S * WAVE;
        }
    }
    uint32_t sk = block_sum<CT>(keep, sh);
    if (threadIdx.x == 0)
        tile_counts[tile] = sk;
    if (!count_stats)
        return;  // the caller derives both counts (one counter for every
                 // block is a long queue of atomics on one address)
    uint32_t st = block_sum<CT>(nthr, sh);
    uint32_t sc = block_sum<CT>(nclr, sh);
    if (threadIdx.x == 0) {
        if (st)
            atomicAdd(&stats[0], (unsigned long long)st);
        if (sc)
            atomicAdd(&stats[1], (unsigned long long)sc);
    }
}

template <int P>
__global__ __launch_bounds__(CT) void k_enum_scatter(EnumArgs a0,
                                                     const uint64_t *__restrict__ tile_offsets,
                                                     float *__restrict__ out_diam,
                                                     uint64_t *__restrict__ out_cidx,
                                                     uint64_t *__restrict__ out_vtx)
{
    __shared__ uint32_t wsum[CT / WAVE];
    const EnumArgs a = enum_view(a0);
    tile_offsets += (int64_t)blockIdx.y * (gridDim.x + 1);
    out_diam += (int64_t)blockIdx.y * a.out_stride;
    out_cidx += (int64_t)blockIdx.y * a.out_stride;
    const Binom B{a.binom, a.n + 1};
    const int lane = threadIdx.x & (WAVE - 1), wave = threadIdx.x / WAVE;
    const uint32_t tile = xcd_block(blockIdx.x, gridDim.x);
    const uint64_t c0 = (uint64_t)tile * COMPACT_TILE + (uint64_t)wave * (CI * WAVE) + lane;
    // sweep 1: every candidate once; keep flags as bits, diameters (and the
    // packed vertex tuples, when asked for) in registers
    float dk[CI];
    uint64_t vk[P <= 3 ? CI : 1];
    const bool want_vtx = P >= 2 && P <= 3 && out_vtx != nullptr;
    uint32_t bits = 0;
    uint32_t total = 0;  // kept by the wave
    if (P == 1) {
#pragma unroll
        for (int k = 0; k < CI; ++k) {
            const uint64_t c = c0 + (uint64_t)k * WAVE;
            dk[k] = c < a.ncand ? a.dcond[c] + 0.0f : 0.0f;
        }
    } else if (c0 < a.ncand) {
        constexpr int S = EnumChunk<P>::S;
        EnumWalk<P> wk;
        decode<P>(B, c0, a.n, wk.v);
#pragma unroll
        for (int k0 = 0; k0 < CI; k0 += S) {
            float d[S];
            if (P <= 3 && want_vtx) {
                uint64_t x[S];
                enum_chunk<P, S, true>(wk, B, a, c0 + (uint64_t)k0 * WAVE, k0, d, x);
#pragma unroll
                for (int s = 0; s < S; ++s)
                    vk[P <= 3 ? k0 + s : 0] = x[s];
            } else {
                enum_chunk<P, S>(wk, B, a, c0 + (uint64_t)k0 * WAVE, k0, d);
            }
#pragma unroll
            for (int s = 0; s < S; ++s)
                dk[k0 + s] = d[s];
        }
    }
#pragma unroll
    for (int k = 0; k < CI; ++k) {
        const uint64_t c = c0 + (uint64_t)k * WAVE;
        const bool keep = c < a.ncand && enum_filter(a, c, dk[k]) == 0;
        bits |= (keep ? 1u : 0u) << k;
        total += (uint32_t)__popcll(__ballot(keep));
    }
    if (lane == 0)
        wsum[wave] = total;
    __syncthreads();
    uint64_t running = tile_offsets[tile];
#pragma unroll
    for (int w = 0; w < CT / WAVE; ++w)
        running += (w < wave) ? wsum[w] : 0;
    // sweep 2: the kept candidates in cidx order, coalesced per step
#pragma unroll
    for (int k = 0; k < CI; ++k) {
        const bool keep = (bits >> k) & 1u;
        const uint64_t m = __ballot(keep);
        if (keep) {
            const uint64_t pos = running + (uint32_t)__popcll(m & lanemask_lt());
            out_diam[pos] = dk[k];
            out_cidx[pos] = c0 + (uint64_t)k * WAVE;
            if (P <= 3 && want_vtx)
                out_vtx[pos] = vk[P <= 3 ? k : 0];
        }
        running += (uint32_t)__popcll(m);
    }
}

// One-pass enumeration (a single cloud whose outputs are sized for every
// candidate): the scatter pass above with its tile offset found by a
// decoupled look-back instead of a separate count pass and scan.  A
// workgroup takes its tile from a ticket counter (status[tiles]), so tiles
// start in ticket order; it evaluates its candidates, publishes its kept
// count (flag AGG), then adds up the published counts of the tiles before
// it, walking back until one that has published its inclusive prefix (flag
// PRE), publishes its own prefix and writes at its offset.  A tile waits
// only on tiles with smaller tickets, which are running and publish their
// counts before they wait on anything, so every wait ends.  status must be
// zero before the launch; the last tile writes the kept total to *total.
constexpr uint64_t LB_AGG = 1ull << 62, LB_PRE = 2ull << 62, LB_VAL = (1ull << 62) - 1;

template <int P>
__global__ __launch_bounds__(CT) void k_enum_onepass(EnumArgs a,
                                                     unsigned long long *__restrict__ status,
                                                     int64_t tiles, uint64_t *__restrict__ total,
                                                     float *__restrict__ out_diam,
                                                     uint64_t *__restrict__ out_cidx,
                                                     uint64_t *__restrict__ out_vtx)
{
    __shared__ uint32_t wsum[CT / WAVE];
    __shared__ uint32_t s_tile;
    __shared__ uint64_t s_base;
    if (threadIdx.x == 0)
        s_tile = (uint32_t)atomicAdd(&status[tiles], 1ull);
    __syncthreads();
    const uint32_t tile = s_tile;
    const Binom B{a.binom, a.n + 1};
    const int lane = threadIdx.x & (WAVE - 1), wave = threadIdx.x / WAVE;
    const uint64_t c0 = (uint64_t)tile * COMPACT_TILE + (uint64_t)wave * (CI * WAVE) + lane;
    float dk[CI];
    uint64_t vk[P <= 3 ? CI : 1];
    const bool want_vtx = P >= 2 && P <= 3 && out_vtx != nullptr;
    uint32_t bits = 0;
    uint32_t cnt = 0;  // kept by the wave
    if (P == 1) {
#pragma unroll
        for (int k = 0; k < CI; ++k) {
            const uint64_t c = c0 + (uint64_t)k * WAVE;
            dk[k] = c < a.ncand ? a.dcond[c] + 0.0f : 0.0f;
        }
    } else if (c0 < a.ncand) {
        constexpr int S = EnumChunk<P>::S;
        EnumWalk<P> wk;
        decode<P>(B, c0, a.n, wk.v);
#pragma unroll
        for (int k0 = 0; k0 < CI; k0 += S) {
            float d[S];
            if (P <= 3 && want_vtx) {
                uint64_t x[S];
                enum_chunk<P, S, true>(wk, B, a, c0 + (uint64_t)k0 * WAVE, k0, d, x);
#pragma unroll
                for (int q = 0; q < S; ++q)
                    vk[P <= 3 ? k0 + q : 0] = x[q];
            } else {
                enum_chunk<P, S>(wk, B, a, c0 + (uint64_t)k0 * WAVE, k0, d);
            }
#pragma unroll
            for (int q = 0; q < S; ++q)
                dk[k0 + q] = d[q];
        }
    }
#pragma unroll
    for (int k = 0; k < CI; ++k) {
        const uint64_t c = c0 + (uint64_t)k * WAVE;
        const bool keep = c < a.ncand && enum_filter(a, c, dk[k]) == 0;
        bits |= (keep ? 1u : 0u) << k;
        cnt += (uint32_t)__popcll(__ballot(keep));
    }
    if (lane == 0)
        wsum[wave] = cnt;
    __syncthreads();
    if (wave == 0) {
        // Look-back by the whole first wave: lane l reads the flag word of
        // tile (j - l), so one round trip covers 64 predecessors.  The
        // nearest one holding its inclusive prefix ends the walk; every
        // tile between must have published at least its aggregate (they
        // all hold a ticket below ours, so they are running and publish it
        // without waiting on anyone).  A flag word carries its value, and
        // nothing else written by the tile is read before the kernel ends,
        // so the loads and stores are relaxed (device scope): acquire and
        // release at device scope would invalidate and write back this
        // XCD's whole L2 on every poll and publication, under the feet of
        // every other tile reading the distances through it.
        uint64_t agg = 0;
#pragma unroll
        for (int w = 0; w < CT / WAVE; ++w)
            agg += wsum[w];
        uint64_t excl = 0;
        if (tile == 0) {
            if (lane == 0)
                __hip_atomic_store(&status[0], LB_PRE | agg, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        } else {
            if (lane == 0)
                __hip_atomic_store(&status[tile], LB_AGG | agg, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
            for (int64_t j = (int64_t)tile - 1;;) {
                const int64_t idx = j - lane;
                const unsigned long long st =
                    idx >= 0 ? __hip_atomic_load(&status[idx], __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT)
                             : LB_PRE;  // before tile 0: an empty prefix
                const uint64_t pre = __ballot((st & LB_PRE) != 0);
                const uint64_t none = __ballot((st & ~LB_VAL) == 0);
                const int first = pre ? __ffsll((long long)pre) - 1 : WAVE;
                const uint64_t upto = first >= WAVE - 1 ? ~0ull : (2ull << first) - 1;
                if (none & upto) {
                    __builtin_amdgcn_s_sleep(1);  // a tile in the window not yet published
                    continue;
                }
                excl += wave_sum<uint64_t>(lane <= first ? (uint64_t)(st & LB_VAL) : 0ull);
                if (pre)
                    break;
                j -= WAVE;
            }
            if (lane == 0)
                __hip_atomic_store(&status[tile], LB_PRE | (excl + agg), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        }
        if (lane == 0) {
            if ((int64_t)tile == tiles - 1)
                *total = excl + agg;
            s_base = excl;
        }
    }
    __syncthreads();
    uint64_t running = s_base;
#pragma unroll
    for (int w = 0; w < CT / WAVE; ++w)
        running += (w < wave) ? wsum[w] : 0;
#pragma unroll
    for (int k = 0; k < CI; ++k) {
        const bool keep = (bits >> k) & 1u;
        const uint64_t m = __ballot(keep);
        if (keep) {
            const uint64_t pos = running + (uint32_t)__popcll(m & lanemask_lt());
            out_diam[pos] = dk[k];
            out_cidx[pos] = c0 + (uint64_t)k * WAVE;
            if (P <= 3 && want_vtx)
                out_vtx[pos] = vk[P <= 3 ? k : 0];
        }
        running += (uint32_t)__popcll(m);
    }
}

void launch_enum_onepass(const EnumArgs &a, unsigned long long *status, uint64_t *total,
                         float *out_diam, uint64_t *out_cidx, hipStream_t s, uint64_t *out_vtx)
{
    const int64_t tiles = compact_tiles((int64_t)a.ncand);
    if (tiles == 0)
        return;
    // status: tiles flag words and the ticket counter, all zero
    launch_fill_u32(reinterpret_cast<uint32_t *>(status), 2 * (tiles + 1), 0u, s);
    dim3 g((unsigned)tiles), b(CT);
    switch (a.p) {
    case 1: hipLaunchKernelGGL(k_enum_onepass<1>, g, b, 0, s, a, status, tiles, total, out_diam, out_cidx, nullptr); break;
    case 2: hipLaunchKernelGGL(k_enum_onepass<2>, g, b, 0, s, a, status, tiles, total, out_diam, out_cidx, out_vtx); break;
    case 3: hipLaunchKernelGGL(k_enum_onepass<3>, g, b, 0, s, a, status, tiles, total, out_diam, out_cidx, out_vtx); break;
    default: hipLaunchKernelGGL(k_enum_onepass<4>, g, b, 0, s, a, status, tiles, total, out_diam, out_cidx, nullptr); break;
    }
}

#define RPP_DISPATCH_P(p, F, ...)                                                        \
    switch (p) {                                                                         \
    case 1: F<1> __VA_ARGS__; break;                                                     \
    case 2: F<2> __VA_ARGS__; break;                                                     \
    case 3: F<3> __VA_ARGS__; break;                                                     \
    default: F<4> __VA_ARGS__; break;                                                    \
    }

void launch_enum_count(const EnumArgs &a, uint32_t *tile_counts, unsigned long long *stats,
                       hipStream_t s)
{
    int64_t tiles = compact_tiles((int64_t)a.ncand);
    if (tiles == 0)
        return;
    dim3 g((unsigned)tiles, a.nbatch > 0 ? a.nbatch : 1), b(CT);
    switch (a.p) {
    case 1: hipLaunchKernelGGL(k_enum_count<1>, g, b, 0, s, a, tile_counts, stats); break;
    case 2: hipLaunchKernelGGL(k_enum_count<2>, g, b, 0, s, a, tile_counts, stats); break;
    case 3: hipLaunchKernelGGL(k_enum_count<3>, g, b, 0, s, a, tile_counts, stats); break;
    default: hipLaunchKernelGGL(k_enum_count<4>, g, b, 0, s, a, tile_counts, stats); break;
    }
}

void launch_enum_scatter(const EnumArgs &a, const uint64_t *tile_offsets, float *out_diam,
                         uint64_t *out_cidx, hipStream_t s, uint64_t *out_vtx)
{
    int64_t tiles = compact_tiles((int64_t)a.ncand);
    if (tiles == 0)
        return;
    dim3 g((unsigned)tiles, a.nbatch > 0 ? a.nbatch : 1), b(CT);
    switch (a.p) {
    case 1: hipLaunchKernelGGL(k_enum_scatter<1>, g, b, 0, s, a, tile_offsets, out_diam, out_cidx, nullptr); break;
    case 2: hipLaunchKernelGGL(k_enum_scatter<2>, g, b, 0, s, a, tile_offsets, out_diam, out_cidx, out_vtx); break;
    case 3: hipLaunchKernelGGL(k_enum_scatter<3>, g, b, 0, s, a, tile_offsets, out_diam, out_cidx, out_vtx); break;
    default: hipLaunchKernelGGL(k_enum_scatter<4>, g, b, 0, s, a, tile_offsets, out_diam, out_cidx, nullptr); break;
    }
}

// ===========================================================================
// a5: apparent-pair test (apparent pairs lemma)
//
// Column sigma = (v_0 > ... > v_P) of diameter d.
//  1. Oldest cofacet: scanning w = n-1 down to 0 visits the cofacets
//     sigma + {w} in decreasing cidx; the first w (not in sigma) with
//     d(w, v_i) <= d for all i gives the lexicographically greatest cofacet
//     of equal diameter.  None: the oldest cofacet is strictly larger in
//     diameter and sigma is not apparent.
//  2. Youngest facet: the other facets of tau are sigma - {u} + {w}; such a
//     facet precedes sigma in cidx order exactly when u > w, and is younger
//     than sigma exactly when, in addition, its diameter equals d.
//
// A wave owns 64 consecutive columns.  Every lane loads and decodes one of
// them (coalesced, no redundant decodes); then the wave works through them
// in G rounds of 64/G columns, G lanes per column: the lanes of a group
// fetch their column's diameter and vertices from the owner lane by
// shuffles, test the G vertices top, top-1, ..., top-G+1 per step with
// contiguous reads of the rows of the square matrix, and a ballot picks the
// largest hit.  The facet test takes d(v_i, w) from the registers of the
// lane that hit, and the distances among sigma's own vertices are loaded
// while the scan runs.  Each tau returns to its owner lane for one
// coalesced store.
// ===========================================================================
__device__ __forceinline__ uint64_t shfl_u64(uint64_t x, int src)
{
    const uint32_t lo = (uint32_t)__shfl((int)(uint32_t)x, src, WAVE);
    const uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(x >> 32), src, WAVE);
    return ((uint64_t)hi << 32) | lo;
}

template <int P, int G>
__global__ __launch_bounds__(256) void k_apparent(const float *__restrict__ col_diam,
                                                  const uint64_t *__restrict__ col_cidx,
                                                  int64_t ncols, const float *__restrict__ dsq,
                                                  int n, const uint64_t *__restrict__ binom,
                                                  uint64_t *__restrict__ tau_out,
                                                  unsigned long long *__restrict__ scan_count,
                                                  Batch bt, int rounds)
{
    constexpr int CPR = WAVE / G;  // columns per round
    const int lane = threadIdx.x & (WAVE - 1);
    const int g = lane & (G - 1);
    const int grp = lane / G;
    const int gbase = lane - g;
    const uint64_t gmask = (G == WAVE) ? ~0ull : (((1ull << G) - 1) << gbase);
    const int own = CPR * rounds;  // columns owned by a wave (rounds <= G)
    const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
    const int64_t base = ((blk * blockDim.x + threadIdx.x) / WAVE) * own;
    {
        const int64_t cl = blockIdx.y;
        ncols = batch_count(bt, cl, ncols);
        col_diam += cl * bt.stride;
        col_cidx += cl * bt.stride;
        tau_out += cl * bt.stride;
        dsq += cl * (int64_t)n * n;
    }
    if (base >= ncols)
        return;  // whole waves leave together
    // the cloud's own points: candidates above are bucket padding (never a
    // cofacet: infinitely far), so the scans start below them
    const int nv = batch_nv(bt, blockIdx.y, n);
    const Binom B{binom, n + 1};
    const int64_t mycol = base + lane;
    const bool myvalid = lane < own && mycol < ncols;
    float myd = 0.0f;
    int myv[P + 1];
#pragma unroll
    for (int i = 0; i <= P; ++i)
        myv[i] = 0;
    if (myvalid) {
        myd = col_diam[mycol];
        decode<P>(B, col_cidx[mycol], n, myv);
    }
    uint64_t mytau = NONE;
    for (int r = 0; r < rounds; ++r) {
        const int src = r * CPR + grp;
        const float d = __shfl(myd, src, WAVE);
        int v[P + 1];
#pragma unroll
        for (int i = 0; i <= P; ++i)
            v[i] = __shfl(myv[i], src, WAVE);
        const bool valid = base + src < ncols;  // uniform in the group
        const float *row[P + 1];
#pragma unroll
        for (int i = 0; i <= P; ++i)
            row[i] = dsq + (int64_t)v[i] * n;
        // distances among sigma's own vertices (facet test), loaded early
        float dv[P + 1][P + 1];
#pragma unroll
        for (int a = 0; a <= P; ++a)
#pragma unroll
            for (int b = a + 1; b <= P; ++b)
                dv[a][b] = valid ? row[a][v[b]] : 0.0f;
        int w = -1;
        int hit = 0;
        float e[P + 1];
#pragma unroll
        for (int i = 0; i <= P; ++i)
            e[i] = 0.0f;
        if (valid) {
            for (int top = nv - 1; top >= 0; top -= G) {
                const int u = top - g;
                bool ok = u >= 0;
                if (ok) {
#pragma unroll
                    for (int i = 0; i <= P; ++i) {
                        e[i] = row[i][u];
                        ok = ok && (u != v[i]) && (e[i] <= d);
                    }
                }
                const uint64_t m = __ballot(ok) & gmask;
                if (m) {
                    hit = __ffsll((unsigned long long)m) - 1;  // lane of the largest u
                    w = top - (hit - gbase);
                    break;
                }
            }
        }
        // d(v_i, w) from the lane that found w (every lane joins the shuffle)
        float ew[P + 1];
#pragma unroll
        for (int i = 0; i <= P; ++i)
            ew[i] = __shfl(e[i], w >= 0 ? hit : lane, WAVE);
        uint64_t tau = NONE;
        if (w >= 0) {
            bool apparent = true;
#pragma unroll
            for (int j = 0; j <= P; ++j) {
                if (v[j] > w && apparent) {
                    // facet sigma - {v_j} + {w}
                    float fd = 0.0f;
#pragma unroll
                    for (int a = 0; a <= P; ++a) {
                        if (a == j)
                            continue;
                        fd = fmaxf(fd, ew[a]);
#pragma unroll
                        for (int b = a + 1; b <= P; ++b)
                            if (b != j)
                                fd = fmaxf(fd, dv[a][b]);
                    }
                    if (fd == d)
                        apparent = false;
                }
            }
            if (apparent)
                tau = cofacet_index<P>(B, v, w);
        }
        if (scan_count && valid && g == 0) {
            // candidates w not in sigma, visited from n-1 down to w*
            long long sc = n - P - 1;
            if (w >= 0) {
                sc = (n - 1) - w + 1;
#pragma unroll
                for (int i = 0; i <= P; ++i)
                    sc -= (v[i] > w);
            }
            atomicAdd(&scan_count[blockIdx.x & (SCAN_COUNTERS - 1)], (unsigned long long)sc);
        }
        // the owner of column base + r*CPR + k is lane r*CPR + k; group k's
        // first lane holds its tau
        const uint64_t t = shfl_u64(tau, (lane % CPR) * G);
        if (lane / CPR == r)
            mytau = t;
    }
    if (myvalid)
        tau_out[mycol] = mytau;
}

// Two-phase form for short scans.  Most columns find their oldest cofacet
// among the first few candidates (on a dense torus 85% within 4), but a
// wave of k_apparent runs until its deepest group is done.  Here every lane
// first tests the top K candidates of its own column with all loads in
// flight at once; the columns still open after them are numbered within the
// wave (ballot + popcount) and scanned G lanes per column from candidate
// n-1-K down, as in k_apparent.  A wave owns 64 consecutive columns.
__device__ __forceinline__ int select_set_bit(uint64_t m, int t)
{
    // lane index of the t-th set bit of m (t < popcount(m))
    int pos = 0;
#pragma unroll
    for (int half = 32; half >= 1; half >>= 1) {
        const uint64_t low = m & ((1ull << half) - 1);
        const int c = __popcll(low);
        const bool up = t >= c;
        t -= up ? c : 0;
        m = up ? (m >> half) : low;
        pos += up ? half : 0;
    }
    return pos;
}

template <int P, int K, int G>
__global__ __launch_bounds__(256) void k_apparent2(const float *__restrict__ col_diam,
                                                   const uint64_t *__restrict__ col_cidx,
                                                   int64_t ncols, const float *__restrict__ dsq,
                                                   int n, const uint64_t *__restrict__ binom,
                                                   uint64_t *__restrict__ tau_out,
                                                   unsigned long long *__restrict__ scan_count)
{
    constexpr int CPR = WAVE / G;  // open columns per round of phase 2
    const int lane = threadIdx.x & (WAVE - 1);
    const int g = lane & (G - 1);
    const int grp = lane / G;
    const int gbase = lane - g;
    const uint64_t gmask = (G == WAVE) ? ~0ull : (((1ull << G) - 1) << gbase);
    const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
    const int64_t base = ((blk * blockDim.x + threadIdx.x) / WAVE) * WAVE;
    if (base >= ncols)
        return;  // whole waves leave together
    const Binom B{binom, n + 1};
    const int64_t mycol = base + lane;
    const bool myvalid = mycol < ncols;
    float myd = 0.0f;
    int myv[P + 1];
#pragma unroll
    for (int i = 0; i <= P; ++i)
        myv[i] = 0;
    if (myvalid) {
        myd = col_diam[mycol];
        decode<P>(B, col_cidx[mycol], n, myv);
    }

    // ---- phase 1: candidates n-1 .. n-K of the lane's own column ----
    float dv[P + 1][P + 1];  // distances among sigma's vertices
    float ew[P + 1];         // d(v_i, w) at the hit
    int w = -1;
#pragma unroll
    for (int i = 0; i <= P; ++i)
        ew[i] = 0.0f;
    if (myvalid) {
        const float *row[P + 1];
#pragma unroll
        for (int i = 0; i <= P; ++i)
            row[i] = dsq + (int64_t)myv[i] * n;
#pragma unroll
        for (int a = 0; a <= P; ++a)
#pragma unroll
            for (int b = a + 1; b <= P; ++b)
                dv[a][b] = row[a][myv[b]];
        // batches of up to 8 candidates, every load of a batch in flight
        constexpr int KB = K < 8 ? K : 8;
#pragma unroll
        for (int k0 = 0; k0 < K; k0 += KB) {
            if (w < 0) {
                float e[KB][P + 1];
#pragma unroll
                for (int k = 0; k < KB; ++k) {
                    const int u = n - 1 - k0 - k;
                    const int uc = u >= 0 ? u : 0;  // in bounds; u < 0 never hits
#pragma unroll
                    for (int i = 0; i <= P; ++i)
                        e[k][i] = row[i][uc];
                }
                // the largest passing u wins: k runs down so the smallest
                // k is applied last
#pragma unroll
                for (int k = KB - 1; k >= 0; --k) {
                    const int u = n - 1 - k0 - k;
                    bool ok = u >= 0;
#pragma unroll
                    for (int i = 0; i <= P; ++i)
                        ok = ok && (u != myv[i]) && (e[k][i] <= myd);
                    if (ok) {
                        w = u;
#pragma unroll
                        for (int i = 0; i <= P; ++i)
                            ew[i] = e[k][i];
                    }
                }
            }
        }
    } else {
#pragma unroll
        for (int a = 0; a <= P; ++a)
#pragma unroll
            for (int b = a + 1; b <= P; ++b)
                dv[a][b] = 0.0f;
    }
    // open: no hit among the K and candidates below them remain
    const bool open = myvalid && w < 0 && n - 1 - K >= 0;
    const uint64_t omask = __ballot(open);

    // ---- phase 2: open columns, G lanes each ----
    const int nopen = __popcll(omask);
    uint64_t tau2 = NONE;  // this lane's tau when its column was open
    int w2 = -1;           // and its hit (scan count)
    for (int r = 0; r * CPR < nopen; ++r) {
        const int t = r * CPR + grp;
        const bool valid = t < nopen;  // uniform in the group
        const int src = valid ? select_set_bit(omask, t) : lane;
        const float d = __shfl(myd, src, WAVE);
        int v[P + 1];
#pragma unroll
        for (int i = 0; i <= P; ++i)
            v[i] = __shfl(myv[i], src, WAVE);
        float dvv[P + 1][P + 1];
#pragma unroll
        for (int a = 0; a <= P; ++a)
#pragma unroll
            for (int b = a + 1; b <= P; ++b)
                dvv[a][b] = __shfl(dv[a][b], src, WAVE);
        const float *row[P + 1];
#pragma unroll
        for (int i = 0; i <= P; ++i)
            row[i] = dsq + (int64_t)v[i] * n;
        int ww = -1, hit = 0;
        float e[P + 1];
#pragma unroll
        for (int i = 0; i <= P; ++i)
            e[i] = 0.0f;
        if (valid) {
            for (int top = n - 1 - K; top >= 0; top -= G) {
                const int u = top - g;
                bool ok = u >= 0;
                if (ok) {
#pragma unroll
                    for (int i = 0; i <= P; ++i) {
                        e[i] = row[i][u];
                        ok = ok && (u != v[i]) && (e[i] <= d);
                    }
                }
                const uint64_t m = __ballot(ok) & gmask;
                if (m) {
                    hit = __ffsll((unsigned long long)m) - 1;  // lane of the largest u
                    ww = top - (hit - gbase);
                    break;
                }
            }
        }
        float eh[P + 1];
#pragma unroll
        for (int i = 0; i <= P; ++i)
            eh[i] = __shfl(e[i], ww >= 0 ? hit : lane, WAVE);
        uint64_t tau = NONE;
        if (ww >= 0) {
            bool apparent = true;
#pragma unroll
            for (int j = 0; j <= P; ++j) {
                if (v[j] > ww && apparent) {
                    float fd = 0.0f;
#pragma unroll
                    for (int a = 0; a <= P; ++a) {
                        if (a == j)
                            continue;
                        fd = fmaxf(fd, eh[a]);
#pragma unroll
                        for (int b = a + 1; b <= P; ++b)
                            if (b != j)
                                fd = fmaxf(fd, dvv[a][b]);
                    }
                    if (fd == d)
                        apparent = false;
                }
            }
            if (apparent)
                tau = cofacet_index<P>(B, v, ww);
        }
        // the owner of open column t is the t-th set lane of omask; group
        // (t mod CPR)'s first lane holds its tau
        const int mine = open ? __popcll(omask & ((1ull << lane) - 1)) : -1;
        const int from = mine >= 0 ? (mine % CPR) * G : lane;
        const uint64_t tt = shfl_u64(tau, from);
        const int wt = __shfl(ww, from, WAVE);
        if (mine >= 0 && mine / CPR == r) {
            tau2 = tt;
            w2 = wt;
        }
    }

    if (!myvalid)
        return;
    uint64_t mytau = NONE;
    if (open) {
        mytau = tau2;
        w = w2;
    } else if (w >= 0) {
        bool apparent = true;
#pragma unroll
        for (int j = 0; j <= P; ++j) {
            if (myv[j] > w && apparent) {
                // facet sigma - {v_j} + {w}
                float fd = 0.0f;
#pragma unroll
                for (int a = 0; a <= P; ++a) {
                    if (a == j)
                        continue;
                    fd = fmaxf(fd, ew[a]);
#pragma unroll
                    for (int b = a + 1; b <= P; ++b)
                        if (b != j)
                            fd = fmaxf(fd, dv[a][b]);
                }
                if (fd == myd)
                    apparent = false;
            }
        }
        if (apparent)
            mytau = cofacet_index<P>(B, myv, w);
    }
    if (scan_count) {
        // candidates w not in sigma, visited from n-1 down to w*
        long long sc = n - P - 1;
        if (w >= 0) {
            sc = (n - 1) - w + 1;
#pragma unroll
            for (int i = 0; i <= P; ++i)
                sc -= (myv[i] > w);
        }
        atomicAdd(&scan_count[(blockIdx.x * 4 + lane) & (SCAN_COUNTERS - 1)],
                  (unsigned long long)sc);
    }
    tau_out[mycol] = mytau;
}

// The same two phases with the open columns of a whole workgroup pooled:
// phase 1 leaves about 15% of the 256 columns open, which a wave alone
// would scan in ceil(open/8) rounds; queued in LDS they are shared by the
// four waves (fewer, fuller rounds), and a group reads its column straight
// from the queue instead of selecting and shuffling it from the owner lane.
// The workgroup owns 256 consecutive columns.
template <int P, int K, int G>
__global__ __launch_bounds__(256) void k_apparent2b(const float *__restrict__ col_diam,
                                                    const uint64_t *__restrict__ col_cidx,
                                                    int64_t ncols, const float *__restrict__ dsq,
                                                    int n, const uint64_t *__restrict__ binom,
                                                    uint64_t *__restrict__ tau_out,
                                                    unsigned long long *__restrict__ scan_count)
{
    constexpr int NT = 256, NW = NT / WAVE;
    constexpr int CPR = WAVE / G;  // open columns per wave per round
    constexpr int NPAIR = (P + 1) * P / 2;
    __shared__ int q_col[NT];             // thread (column) of each open slot
    __shared__ float q_d[NT];
    __shared__ int q_v[P + 1][NT];
    __shared__ float q_dv[NPAIR > 0 ? NPAIR : 1][NT];
    __shared__ int q_wave[NW + 1];
    const int lane = threadIdx.x & (WAVE - 1), wave = threadIdx.x / WAVE;
    const int g = lane & (G - 1);
    const int grp = lane / G;
    const int gbase = lane - g;
    const uint64_t gmask = (G == WAVE) ? ~0ull : (((1ull << G) - 1) << gbase);
    const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
    const int64_t base = blk * NT;  // the workgroup's first column
    const Binom B{binom, n + 1};
    const int64_t mycol = base + threadIdx.x;
    const bool myvalid = mycol < ncols;
    float myd = 0.0f;
    int myv[P + 1];
#pragma unroll
    for (int i = 0; i <= P; ++i)
        myv[i] = 0;
    if (myvalid) {
        myd = col_diam[mycol];
        decode<P>(B, col_cidx[mycol], n, myv);
    }

    // ---- phase 1: candidates n-1 .. n-K of the thread's own column ----
    float dv[NPAIR > 0 ? NPAIR : 1];  // distances among sigma's vertices
    float ew[P + 1];                  // d(v_i, w) at the hit
    int w = -1;
#pragma unroll
    for (int i = 0; i <= P; ++i)
        ew[i] = 0.0f;
#pragma unroll
    for (int q = 0; q < NPAIR; ++q)
        dv[q] = 0.0f;
    if (myvalid) {
        const float *row[P + 1];
#pragma unroll
        for (int i = 0; i <= P; ++i)
            row[i] = dsq + (int64_t)myv[i] * n;
        {
            int q = 0;
#pragma unroll
            for (int a = 0; a <= P; ++a)
#pragma unroll
                for (int b = a + 1; b <= P; ++b)
                    dv[q++] = row[a][myv[b]];
        }
        float e[K][P + 1];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int u = n - 1 - k;
            const int uc = u >= 0 ? u : 0;  // in bounds; u < 0 never hits
#pragma unroll
            for (int i = 0; i <= P; ++i)
                e[k][i] = row[i][uc];
        }
        // the largest passing u wins: k runs down so k = 0 is applied last
#pragma unroll
        for (int k = K - 1; k >= 0; --k) {
            const int u = n - 1 - k;
            bool ok = u >= 0;
#pragma unroll
            for (int i = 0; i <= P; ++i)
                ok = ok && (u != myv[i]) && (e[k][i] <= myd);
            if (ok) {
                w = u;
#pragma unroll
                for (int i = 0; i <= P; ++i)
                    ew[i] = e[k][i];
            }
        }
    }
    // open: no hit among the K and candidates below them remain
    const bool open = myvalid && w < 0 && n - 1 - K >= 0;

    // ---- queue the open columns in LDS, in thread order ----
    const uint64_t omask = __ballot(open);
    if (lane == 0)
        q_wave[wave] = __popcll(omask);
    __syncthreads();
    int woff = 0, nopen = 0;
#pragma unroll
    for (int x = 0; x < NW; ++x) {
        const int c = q_wave[x];
        woff += x < wave ? c : 0;
        nopen += c;
    }
    if (open) {
        const int t = woff + __popcll(omask & lanemask_lt());
        q_col[t] = threadIdx.x;
        q_d[t] = myd;
#pragma unroll
        for (int i = 0; i <= P; ++i)
            q_v[i][t] = myv[i];
#pragma unroll
        for (int q = 0; q < NPAIR; ++q)
            q_dv[q][t] = dv[q];
    }
    __syncthreads();

    // ---- resolved columns: facet test and tau ----
    if (myvalid && !open) {
        uint64_t mytau = NONE;
        if (w >= 0) {
            bool apparent = true;
#pragma unroll
            for (int j = 0; j <= P; ++j) {
                if (myv[j] > w && apparent) {
                    // facet sigma - {v_j} + {w}
                    float fd = 0.0f;
                    int q = 0;
#pragma unroll
                    for (int a = 0; a <= P; ++a) {
                        if (a != j)
                            fd = fmaxf(fd, ew[a]);
#pragma unroll
                        for (int b = a + 1; b <= P; ++b, ++q)
                            if (a != j && b != j)
                                fd = fmaxf(fd, dv[q]);
                    }
                    if (fd == myd)
                        apparent = false;
                }
            }
            if (apparent)
                mytau = cofacet_index<P>(B, myv, w);
        }
        tau_out[mycol] = mytau;
        if (scan_count) {
            // candidates w not in sigma, visited from n-1 down to w*
            long long sc = n - P - 1;
            if (w >= 0) {
                sc = (n - 1) - w + 1;
#pragma unroll
                for (int i = 0; i <= P; ++i)
                    sc -= (myv[i] > w);
            }
            atomicAdd(&scan_count[(blockIdx.x * 4 + lane) & (SCAN_COUNTERS - 1)],
                      (unsigned long long)sc);
        }
    }

    // ---- phase 2: the queue, G lanes per column, every wave taking turns ----
    for (int r0 = 0; r0 < nopen; r0 += NW * CPR) {
        const int t = r0 + wave * CPR + grp;
        const bool valid = t < nopen;  // uniform in the group
        const int tq = valid ? t : 0;
        const float d = q_d[tq];
        int v[P + 1];
#pragma unroll
        for (int i = 0; i <= P; ++i)
            v[i] = q_v[i][tq];
        const float *row[P + 1];
#pragma unroll
        for (int i = 0; i <= P; ++i)
            row[i] = dsq + (int64_t)v[i] * n;
        int ww = -1, hit = 0;
        float e[P + 1];
#pragma unroll
        for (int i = 0; i <= P; ++i)
            e[i] = 0.0f;
        if (valid) {
            for (int top = n - 1 - K; top >= 0; top -= G) {
                const int u = top - g;
                bool ok = u >= 0;
                if (ok) {
#pragma unroll
                    for (int i = 0; i <= P; ++i) {
                        e[i] = row[i][u];
                        ok = ok && (u != v[i]) && (e[i] <= d);
                    }
                }
                const uint64_t m = __ballot(ok) & gmask;
                if (m) {
                    hit = __ffsll((unsigned long long)m) - 1;  // lane of the largest u
                    ww = top - (hit - gbase);
                    break;
                }
            }
        }
        float eh[P + 1];
#pragma unroll
        for (int i = 0; i <= P; ++i)
            eh[i] = __shfl(e[i], ww >= 0 ? hit : lane, WAVE);
        if (valid && g == 0) {
            uint64_t tau = NONE;
            if (ww >= 0) {
                bool apparent = true;
#pragma unroll
                for (int j = 0; j <= P; ++j) {
                    if (v[j] > ww && apparent) {
                        float fd = 0.0f;
                        int q = 0;
#pragma unroll
                        for (int a = 0; a <= P; ++a) {
                            if (a != j)
                                fd = fmaxf(fd, eh[a]);
#pragma unroll
                            for (int b = a + 1; b <= P; ++b, ++q)
                                if (a != j && b != j)
                                    fd = fmaxf(fd, q_dv[q][tq]);
                        }
                        if (fd == d)
                            apparent = false;
                    }
                }
                if (apparent)
                    tau = cofacet_index<P>(B, v, ww);
            }
            tau_out[base + q_col[tq]] = tau;
            if (scan_count) {
                long long sc = n - P - 1;
                if (ww >= 0) {
                    sc = (n - 1) - ww + 1;
#pragma unroll
                    for (int i = 0; i <= P; ++i)
                        sc -= (v[i] > ww);
                }
                atomicAdd(&scan_count[(blockIdx.x * 4 + lane) & (SCAN_COUNTERS - 1)],
                          (unsigned long long)sc);
            }
        }
    }
}

// Row-padded copy of the square matrix: pitch = n rounded up to a multiple
// of 4, so every row starts 16-byte aligned (the pad entries are never read
// as candidates).
__global__ void k_pad_rows(const float *__restrict__ dsq, int n, int pitch,
                           float *__restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)n * pitch)
        return;
    const int r = (int)(i / pitch), c = (int)(i - (int64_t)r * pitch);
    out[i] = c < n ? dsq[(int64_t)r * n + c] : 0.0f;
}

void launch_pad_rows(const float *dsq, int n, int pitch, float *out, hipStream_t s)
{
    const int64_t total = (int64_t)n * pitch;
    if (total <= 0)
        return;
    hipLaunchKernelGGL(k_pad_rows, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, dsq, n,
                       pitch, out);
}

// The pooled two-phase kernel with vector reads in phase 1.  A lane's first
// candidates lie in one row segment per vertex of sigma, but read one by
// one each load instruction touches a different cache line for every lane
// of the wave.  With 16-byte aligned rows a lane reads the aligned block of
// four that holds candidate n-1 and the NB-1 blocks below it as 16-byte
// loads, one per block and vertex, testing candidates n-1 down to
// a-4(NB-1) (a = (n-1) rounded down to a multiple of 4).  Phase 2 goes on
// below them.
template <int P, int G, int NB>
__global__ __launch_bounds__(256) void k_apparent2v(const float *__restrict__ col_diam,
                                                    const uint64_t *__restrict__ col_cidx,
                                                    int64_t ncols, const float *__restrict__ dsqp,
                                                    int pitch, int n,
                                                    const uint64_t *__restrict__ binom,
                                                    uint64_t *__restrict__ tau_out,
                                                    unsigned long long *__restrict__ scan_count,
                                                    const uint64_t *__restrict__ col_vtx)
{
    constexpr int NT = 256, NW = NT / WAVE;
    constexpr int CPR = WAVE / G;  // open columns per wave per round
    constexpr int NPAIR = (P + 1) * P / 2;
    __shared__ int q_col[NT];             // thread (column) of each open slot
    __shared__ float q_d[NT];
    __shared__ int q_v[P + 1][NT];
    __shared__ float q_dv[NPAIR > 0 ? NPAIR : 1][NT];
    __shared__ int q_wave[NW + 1];
    const int lane = threadIdx.x & (WAVE - 1), wave = threadIdx.x / WAVE;
    const int g = lane & (G - 1);
    const int grp = lane / G;
    const int gbase = lane - g;
    const uint64_t gmask = (G == WAVE) ? ~0ull : (((1ull << G) - 1) << gbase);
    const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
    const int64_t base = blk * NT;  // the workgroup's first column
    const Binom B{binom, n + 1};
    const int64_t mycol = base + threadIdx.x;
    const bool myvalid = mycol < ncols;
    const int a4 = (n - 1) & ~3;  // aligned block holding candidate n-1
    float myd = 0.0f;
    int myv[P + 1];
#pragma unroll
    for (int i = 0; i <= P; ++i)
        myv[i] = 0;
    if (myvalid) {
        myd = col_diam[mycol];
        if (P <= 3 && col_vtx) {
            // the vertex tuple as the enumeration packed it: no decode
            const uint64_t x = col_vtx[mycol];
#pragma unroll
            for (int i = 0; i <= P; ++i)
                myv[i] = (int)((x >> (16 * i)) & 0xffffu);
        } else {
            decode<P>(B, col_cidx[mycol], n, myv);
        }
    }

    // ---- phase 1: candidates n-1 .. max(a4-4, 0) of the thread's column ----
    float dv[NPAIR > 0 ? NPAIR : 1];
    float ew[P + 1];
    int w = -1;
#pragma unroll
    for (int i = 0; i <= P; ++i)
        ew[i] = 0.0f;
#pragma unroll
    for (int q = 0; q < NPAIR; ++q)
        dv[q] = 0.0f;
    if (myvalid) {
        const float *row[P + 1];
#pragma unroll
        for (int i = 0; i <= P; ++i)
            row[i] = dsqp + (int64_t)myv[i] * pitch;
        {
            int q = 0;
#pragma unroll
            for (int a = 0; a <= P; ++a)
#pragma unroll
                for (int b = a + 1; b <= P; ++b)
                    dv[q++] = row[a][myv[b]];
        }
        constexpr int NC = 4 * NB;
        const int lo = a4 - 4 * (NB - 1);  // lowest candidate of the blocks
        float e[P + 1][NC];  // e[i][c]: d(v_i, lo + c)
#pragma unroll
        for (int i = 0; i <= P; ++i) {
#pragma unroll
            for (int bk = 0; bk < NB; ++bk) {
                const int at = lo + 4 * bk;
                const float4 x = at >= 0 ? *reinterpret_cast<const float4 *>(row[i] + at)
                                         : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                e[i][4 * bk + 0] = x.x;
                e[i][4 * bk + 1] = x.y;
                e[i][4 * bk + 2] = x.z;
                e[i][4 * bk + 3] = x.w;
            }
        }
        // ascending u, so the largest passing u is applied last
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const int u = lo + c;
            bool ok = u >= 0 && u <= n - 1;
#pragma unroll
            for (int i = 0; i <= P; ++i)
                ok = ok && (u != myv[i]) && (e[i][c] <= myd);
            if (ok) {
                w = u;
#pragma unroll
                for (int i = 0; i <= P; ++i)
                    ew[i] = e[i][c];
            }
        }
    }
    // open: no hit and candidates below the blocks remain
    const int below = a4 - 4 * (NB - 1) - 1;  // highest candidate of phase 2
    const bool open = myvalid && w < 0 && below >= 0;

    // ---- queue the open columns in LDS, in thread order ----
    const uint64_t omask = __ballot(open);
    if (lane == 0)
        q_wave[wave] = __popcll(omask);
    __syncthreads();
    int woff = 0, nopen = 0;
#pragma unroll
    for (int x = 0; x < NW; ++x) {
        const int c = q_wave[x];
        woff += x < wave ? c : 0;
        nopen += c;
    }
    if (open) {
        const int t = woff + __popcll(omask & lanemask_lt());
        q_col[t] = threadIdx.x;
        q_d[t] = myd;
#pragma unroll
        for (int i = 0; i <= P; ++i)
            q_v[i][t] = myv[i];
#pragma unroll
        for (int q = 0; q < NPAIR; ++q)
            q_dv[q][t] = dv[q];
    }
    __syncthreads();

    // ---- resolved columns: facet test and tau ----
    if (myvalid && !open) {
        uint64_t mytau = NONE;
        if (w >= 0) {
            bool apparent = true;
#pragma unroll
            for (int j = 0; j <= P; ++j) {
                if (myv[j] > w && apparent) {
                    // facet sigma - {v_j} + {w}
                    float fd = 0.0f;
                    int q = 0;
#pragma unroll
                    for (int a = 0; a <= P; ++a) {
                        if (a != j)
                            fd = fmaxf(fd, ew[a]);
#pragma unroll
                        for (int b = a + 1; b <= P; ++b, ++q)
                            if (a != j && b != j)
                                fd = fmaxf(fd, dv[q]);
                    }
                    if (fd == myd)
                        apparent = false;
                }
            }
            if (apparent)
                mytau = cofacet_index<P>(B, myv, w);
        }
        tau_out[mycol] = mytau;
        if (scan_count) {
            // candidates w not in sigma, visited from n-1 down to w*
            long long sc = n - P - 1;
            if (w >= 0) {
                sc = (n - 1) - w + 1;
#pragma unroll
                for (int i = 0; i <= P; ++i)
                    sc -= (myv[i] > w);
            }
            atomicAdd(&scan_count[(blockIdx.x * 4 + lane) & (SCAN_COUNTERS - 1)],
                      (unsigned long long)sc);
        }
    }

    // ---- phase 2: the queue, G lanes per column, every wave taking turns ----
    for (int r0 = 0; r0 < nopen; r0 += NW * CPR) {
        const int t = r0 + wave * CPR + grp;
        const bool valid = t < nopen;  // uniform in the group
        const int tq = valid ? t : 0;
        const float d = q_d[tq];
        int v[P + 1];
#pragma unroll
        for (int i = 0; i <= P; ++i)
            v[i] = q_v[i][tq];
        const float *row[P + 1];
#pragma unroll
        for (int i = 0; i <= P; ++i)
            row[i] = dsqp + (int64_t)v[i] * pitch;
        int ww = -1, hit = 0;
        float e[P + 1];
#pragma unroll
        for (int i = 0; i <= P; ++i)
            e[i] = 0.0f;
        if (valid) {
            for (int top = below; top >= 0; top -= G) {
                const int u = top - g;
                bool ok = u >= 0;
                if (ok) {
#pragma unroll
                    for (int i = 0; i <= P; ++i) {
                        e[i] = row[i][u];
                        ok = ok && (u != v[i]) && (e[i] <= d);
                    }
                }
                const uint64_t m = __ballot(ok) & gmask;
                if (m) {
                    hit = __ffsll((unsigned long long)m) - 1;  // lane of the largest u
                    ww = top - (hit - gbase);
                    break;
                }
            }
        }
        float eh[P + 1];
#pragma unroll
        for (int i = 0; i <= P; ++i)
            eh[i] = __shfl(e[i], ww >= 0 ? hit : lane, WAVE);
        if (valid && g == 0) {
            uint64_t tau = NONE;
            if (ww >= 0) {
                bool apparent = true;
#pragma unroll
                for (int j = 0; j <= P; ++j) {
                    if (v[j] > ww && apparent) {
                        float fd = 0.0f;
                        int q = 0;
#pragma unroll
                        for (int a = 0; a <= P; ++a) {
                            if (a != j)
                                fd = fmaxf(fd, eh[a]);
#pragma unroll
                            for (int b = a + 1; b <= P; ++b, ++q)
                                if (a != j && b != j)
                                    fd = fmaxf(fd, q_dv[q][tq]);
                        }
                        if (fd == d)
                            apparent = false;
                    }
                }
                if (apparent)
                    tau = cofacet_index<P>(B, v, ww);
            }
            tau_out[base + q_col[tq]] = tau;
            if (scan_count) {
                long long sc = n - P - 1;
                if (ww >= 0) {
                    sc = (n - 1) - ww + 1;
#pragma unroll
                    for (int i = 0; i <= P; ++i)
                        sc -= (v[i] > ww);
                }
                atomicAdd(&scan_count[(blockIdx.x * 4 + lane) & (SCAN_COUNTERS - 1)],
                          (unsigned long long)sc);
            }
        }
    }
}

void launch_apparent_vec(const float *col_diam, const uint64_t *col_cidx, int64_t ncols,
                         const float *dsqp, int pitch, int n, int p, const uint64_t *binom,
                         int group, uint64_t *tau_out, unsigned long long *scan_count,
                         hipStream_t s, const uint64_t *col_vtx)
{
    if (ncols <= 0)
        return;
    dim3 g((unsigned)((ncols + 255) / 256)), b(256);
    // group = 20000 + 100 NB + G (NB = 0 means 2)
    const int nb = (group - 20000) / 100;
    const bool g16 = group % 100 == 16;
#define RPP_LAUNCH_VEC(PP)                                                                        \
    if (nb == 3)                                                                                  \
        hipLaunchKernelGGL((k_apparent2v<PP, 8, 3>), g, b, 0, s, col_diam, col_cidx, ncols, dsqp, \
                           pitch, n, binom, tau_out, scan_count, col_vtx);                        \
    else if (nb == 4)                                                                             \
        hipLaunchKernelGGL((k_apparent2v<PP, 8, 4>), g, b, 0, s, col_diam, col_cidx, ncols, dsqp, \
                           pitch, n, binom, tau_out, scan_count, col_vtx);                        \
    else if (g16)                                                                                 \
        hipLaunchKernelGGL((k_apparent2v<PP, 16, 2>), g, b, 0, s, col_diam, col_cidx, ncols,      \
                           dsqp, pitch, n, binom, tau_out, scan_count, col_vtx);                  \
    else                                                                                          \
        hipLaunchKernelGGL((k_apparent2v<PP, 8, 2>), g, b, 0, s, col_diam, col_cidx, ncols, dsqp, \
                           pitch, n, binom, tau_out, scan_count, col_vtx);
    switch (p) {
    case 1: RPP_LAUNCH_VEC(1) break;
    case 2: RPP_LAUNCH_VEC(2) break;
    case 3: RPP_LAUNCH_VEC(3) break;
    default: RPP_LAUNCH_VEC(4) break;
    }
#undef RPP_LAUNCH_VEC
}

template <int P>
static void launch_apparent_p(const float *cd, const uint64_t *cc, int64_t ncols,
                              const float *dsq, int n, const uint64_t *binom, int group,
                              uint64_t *tau, unsigned long long *sc, hipStream_t s,
                              Batch bt = Batch(), int nbatch = 1, int rounds_req = 0,
                              int block = 256)
{
    if (group >= 100 && nbatch <= 1 && bt.count == nullptr && bt.stride == 0) {
        // two-phase kernel: group = 100 K + G (K candidates alone, then G
        // lanes per open column); 10000 + that: open columns pooled per
        // workgroup
        const int64_t waves = (ncols + WAVE - 1) / WAVE;
        dim3 g((unsigned)((waves * WAVE + 255) / 256)), b(256);
        if (group >= 10000) {
            dim3 gb((unsigned)((ncols + 255) / 256));
            switch (group - 10000) {
            case 416: hipLaunchKernelGGL((k_apparent2b<P, 4, 16>), gb, b, 0, s, cd, cc, ncols, dsq, n, binom, tau, sc); break;
            default: hipLaunchKernelGGL((k_apparent2b<P, 4, 8>), gb, b, 0, s, cd, cc, ncols, dsq, n, binom, tau, sc); break;
            }
            return;
        }
        switch (group) {
        case 416: hipLaunchKernelGGL((k_apparent2<P, 4, 16>), g, b, 0, s, cd, cc, ncols, dsq, n, binom, tau, sc); break;
        case 808: hipLaunchKernelGGL((k_apparent2<P, 8, 8>), g, b, 0, s, cd, cc, ncols, dsq, n, binom, tau, sc); break;
        case 1608: hipLaunchKernelGGL((k_apparent2<P, 16, 8>), g, b, 0, s, cd, cc, ncols, dsq, n, binom, tau, sc); break;
        case 1616: hipLaunchKernelGGL((k_apparent2<P, 16, 16>), g, b, 0, s, cd, cc, ncols, dsq, n, binom, tau, sc); break;
        default: hipLaunchKernelGGL((k_apparent2<P, 4, 8>), g, b, 0, s, cd, cc, ncols, dsq, n, binom, tau, sc); break;
        }
        return;
    }
    if (group != 1 && group != 4 && group != 16 && group != 32 && group != 64)
        group = 8;  // the instantiated group sizes; 8 is the default
    // Rounds per wave (each round covers 64/group columns): as many as the
    // group size allows while the grid keeps at least ~4 waves per SIMD
    // (1024 SIMDs), so small column counts still fill the chip.
    const int cpr = WAVE / group;
    const int64_t total = ncols * (nbatch > 0 ? nbatch : 1);
    int rounds = 1;
    while (rounds < group && total / ((int64_t)cpr * rounds * 2) >= 4096)
        rounds *= 2;
    if (rounds_req > 0)  // a tuned value (rounds <= group)
        rounds = rounds_req < group ? rounds_req : group;
    if (block != 64 && block != 128)
        block = 256;  // any multiple of 64 up to the kernel's launch bound
    const int64_t waves = (ncols + (int64_t)cpr * rounds - 1) / ((int64_t)cpr * rounds);
    const int64_t threads = waves * WAVE;
    dim3 g((unsigned)((threads + block - 1) / block), nbatch), b(block);
    switch (group) {
    case 1: hipLaunchKernelGGL((k_apparent<P, 1>), g, b, 0, s, cd, cc, ncols, dsq, n, binom, tau, sc, bt, rounds); break;
    case 4: hipLaunchKernelGGL((k_apparent<P, 4>), g, b, 0, s, cd, cc, ncols, dsq, n, binom, tau, sc, bt, rounds); break;
    case 16: hipLaunchKernelGGL((k_apparent<P, 16>), g, b, 0, s, cd, cc, ncols, dsq, n, binom, tau, sc, bt, rounds); break;
    case 32: hipLaunchKernelGGL((k_apparent<P, 32>), g, b, 0, s, cd, cc, ncols, dsq, n, binom, tau, sc, bt, rounds); break;
    case 64: hipLaunchKernelGGL((k_apparent<P, 64>), g, b, 0, s, cd, cc, ncols, dsq, n, binom, tau, sc, bt, rounds); break;
    default: hipLaunchKernelGGL((k_apparent<P, 8>), g, b, 0, s, cd, cc, ncols, dsq, n, binom, tau, sc, bt, rounds); break;
    }
}

void launch_apparent_b(const float *col_diam, const uint64_t *col_cidx, int64_t cap,
                       const float *dsq, int n, int p, const uint64_t *binom, int group,
                       uint64_t *tau_out, Batch bt, int nbatch, hipStream_t s, int rounds,
                       int block)
{
    if (cap <= 0)
        return;
#define RPP_AB(P) launch_apparent_p<P>(col_diam, col_cidx, cap, dsq, n, binom, group, tau_out, nullptr, s, bt, nbatch, rounds, block)
    switch (p) {
    case 1: RPP_AB(1); break;
    case 2: RPP_AB(2); break;
    case 3: RPP_AB(3); break;
    default: RPP_AB(4); break;
    }
#undef RPP_AB
}

void launch_apparent(const float *col_diam, const uint64_t *col_cidx, int64_t ncols,
                     const float *dsq, int n, int p, const uint64_t *binom, int group,
                     uint64_t *tau_out, unsigned long long *scan_count, hipStream_t s)
{
    if (ncols <= 0)
        return;
    switch (p) {
    case 1: launch_apparent_p<1>(col_diam, col_cidx, ncols, dsq, n, binom, group, tau_out, scan_count, s); break;
    case 2: launch_apparent_p<2>(col_diam, col_cidx, ncols, dsq, n, binom, group, tau_out, scan_count, s); break;
    case 3: launch_apparent_p<3>(col_diam, col_cidx, ncols, dsq, n, binom, group, tau_out, scan_count, s); break;
    default: launch_apparent_p<4>(col_diam, col_cidx, ncols, dsq, n, binom, group, tau_out, scan_count, s); break;
    }
}

// ===========================================================================
// a6: partition into apparent pairs and non-apparent columns
// ===========================================================================
__global__ __launch_bounds__(CT) void k_partition_count(const uint64_t *__restrict__ tau,
                                                        int64_t ncols,
                                                        uint32_t *__restrict__ tile_counts,
                                                        Batch bt)
{
    __shared__ uint32_t sh[CT / WAVE + 1];
    {
        const int64_t cl = blockIdx.y;
        ncols = batch_count(bt, cl, ncols);
        tau += cl * bt.stride;
        tile_counts += cl * gridDim.x;
    }
    const int64_t base = (int64_t)blockIdx.x * COMPACT_TILE;
    uint32_t cnt = 0;
#pragma unroll 4
    for (int k = 0; k < CI; ++k) {
        int64_t i = base + (int64_t)k * CT + threadIdx.x;
        if (i < ncols)
            cnt += (tau[i] != NONE);
    }
    cnt = block_sum<CT>(cnt, sh);
    if (threadIdx.x == 0)
        tile_counts[blockIdx.x] = cnt;
}

__global__ __launch_bounds__(CT) void k_partition_scatter(
    const uint64_t *__restrict__ tau, const float *__restrict__ col_diam,
    const uint64_t *__restrict__ col_cidx, int64_t ncols,
    const uint64_t *__restrict__ tile_offsets, uint64_t *__restrict__ app_tau,
    uint64_t *__restrict__ app_sigma, uint64_t *__restrict__ na_key,
    uint64_t *__restrict__ na_cidx, Batch bt)
{
    __shared__ uint32_t wsum[CT / WAVE];
    {
        const int64_t cl = blockIdx.y, st = bt.stride;
        ncols = batch_count(bt, cl, ncols);
        tau += cl * st;
        col_diam += cl * st;
        col_cidx += cl * st;
        app_tau += cl * st;
        app_sigma += cl * st;
        na_key += cl * st;
        na_cidx += cl * st;
        tile_offsets += cl * (gridDim.x + 1);
    }
    const int lane = threadIdx.x & (WAVE - 1), wave = threadIdx.x / WAVE;
    const int64_t base = (int64_t)blockIdx.x * COMPACT_TILE;
    uint64_t run_a = tile_offsets[blockIdx.x];
    uint64_t run_n = (uint64_t)base - run_a;
    for (int k = 0; k < CI; ++k) {
        int64_t i = base + (int64_t)k * CT + threadIdx.x;
        const bool valid = i < ncols;
        uint64_t t = valid ? tau[i] : NONE;
        const bool app = valid && t != NONE;
        const bool non = valid && t == NONE;
        uint64_t ma = __ballot(app), mv = __ballot(valid);
        if (lane == 0)
            wsum[wave] = (uint32_t)__popcll(ma) | ((uint32_t)__popcll(mv) << 16);
        __syncthreads();
        uint32_t pa = 0, pv = 0, ta = 0, tv = 0;
#pragma unroll
        for (int w = 0; w < CT / WAVE; ++w) {
            uint32_t x = wsum[w];
            uint32_t xa = x & 0xffffu, xv = x >> 16;
            if (w < wave) {
                pa += xa;
                pv += xv;
            }
            ta += xa;
            tv += xv;
        }
        const uint32_t la = (uint32_t)__popcll(ma & lanemask_lt());
        const uint32_t lv = (uint32_t)__popcll(mv & lanemask_lt());
        if (app) {
            uint64_t pos = run_a + pa + la;
            app_tau[pos] = t;
            app_sigma[pos] = col_cidx[i];
        } else if (non) {
            // rank among non-apparent = rank among valid - rank among apparent
            uint64_t pos = run_n + (pv - pa) + (lv - la);
            na_key[pos] = (uint64_t)(~diam_bits(col_diam[i]));
            na_cidx[pos] = col_cidx[i];
        }
        run_a += ta;
        run_n += tv - ta;
        __syncthreads();
    }
}

void launch_partition_count(const uint64_t *tau, int64_t ncols, uint32_t *tile_counts,
                            hipStream_t s, Batch bt, int nbatch)
{
    int64_t tiles = compact_tiles(ncols);
    if (tiles == 0)
        return;
    hipLaunchKernelGGL(k_partition_count, dim3((unsigned)tiles, nbatch), dim3(CT), 0, s, tau,
                       ncols, tile_counts, bt);
}

void launch_partition_scatter(const uint64_t *tau, const float *col_diam,
                              const uint64_t *col_cidx, int64_t ncols,
                              const uint64_t *tile_offsets, uint64_t *app_tau,
                              uint64_t *app_sigma, uint64_t *na_key, uint64_t *na_cidx,
                              hipStream_t s, Batch bt, int nbatch)
{
    int64_t tiles = compact_tiles(ncols);
    if (tiles == 0)
        return;
    hipLaunchKernelGGL(k_partition_scatter, dim3((unsigned)tiles, nbatch), dim3(CT), 0, s, tau,
                       col_diam, col_cidx, ncols, tile_offsets, app_tau, app_sigma, na_key,
                       na_cidx, bt);
}

__global__ void k_desc_keys(const float *__restrict__ diam, int64_t count,
                            uint64_t *__restrict__ keys, Batch bt)
{
    const int64_t cl = blockIdx.y;
    count = batch_count(bt, cl, count);
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count)
        keys[cl * bt.stride + i] = (uint64_t)(~diam_bits(diam[cl * bt.stride + i]));
}

// ===========================================================================
// Rank-coded diameters for the host reduction: the rank of each edge length
// among the distinct lengths within the threshold, ascending.
// ===========================================================================
// flags[i] = 1 where sorted edge i (diameter descending) starts a new length
__global__ void k_rank_flags(const uint64_t *__restrict__ keys, int64_t m,
                             uint32_t *__restrict__ flags)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m)
        flags[i] = (i == 0 || keys[i] != keys[i - 1]) ? 1u : 0u;
}

// n x n matrix of ranks (as floats): `above` everywhere, 0 on the diagonal
__global__ void k_rank_fill(float *__restrict__ rk, int n, float above)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < (int64_t)n * n)
        rk[i] = (i / n == i % n) ? 0.0f : above;
}

// Edge i of the sorted list gets rank R - (excl[i] + flags[i]), R = excl[m]
// distinct lengths; vals[rank] = its length.
__global__ void k_rank_scatter(const uint64_t *__restrict__ keys,
                               const uint64_t *__restrict__ cidx,
                               const uint32_t *__restrict__ flags,
                               const uint64_t *__restrict__ excl, int64_t m, int n,
                               float *__restrict__ rk, float *__restrict__ vals)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m)
        return;
    const uint64_t R = excl[m];
    const uint64_t r = R - (excl[i] + flags[i]);
    int a, b;
    decode_edge(cidx[i], a, b);
    const float rf = (float)r;
    rk[(int64_t)a * n + b] = rf;
    rk[(int64_t)b * n + a] = rf;
    if (flags[i])
        vals[r] = __uint_as_float(~(uint32_t)keys[i]);
}

void launch_rank_flags(const uint64_t *keys, int64_t m, uint32_t *flags, hipStream_t s)
{
    if (m <= 0)
        return;
    hipLaunchKernelGGL(k_rank_flags, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, keys, m,
                       flags);
}

void launch_rank_matrix(const uint64_t *keys, const uint64_t *cidx, const uint32_t *flags,
                        const uint64_t *excl, int64_t m, int n, float above, float *rk,
                        float *vals, hipStream_t s)
{
    const int64_t nn = (int64_t)n * n;
    hipLaunchKernelGGL(k_rank_fill, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, s, rk, n,
                       above);
    if (m > 0)
        hipLaunchKernelGGL(k_rank_scatter, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s,
                           keys, cidx, flags, excl, m, n, rk, vals);
}

// Rank of a length within the threshold: its index in vals (ascending,
// distinct, R entries); larger values are left alone.
__device__ __forceinline__ float rank_of(float x, const float *__restrict__ vals, int64_t R)
{
    if (!(x <= vals[R - 1]))
        return x;
    int64_t lo = 0, hi = R - 1;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (vals[mid] < x)
            lo = mid + 1;
        else
            hi = mid;
    }
    return (float)lo;
}

// Column keys (~bits(diameter) in the low 32 bits) and low diameters
// recoded as ranks.
__global__ void k_recode_ranks(uint64_t *__restrict__ keys, float *__restrict__ lowd, int64_t m,
                               const float *__restrict__ vals, int64_t R)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m)
        return;
    const float d = __uint_as_float(~(uint32_t)keys[i]);
    keys[i] = (uint64_t)(~diam_bits(rank_of(d, vals, R)));
    lowd[i] = rank_of(lowd[i], vals, R);
}

void launch_recode_ranks(uint64_t *keys, float *lowd, int64_t m, const float *vals, int64_t R,
                         hipStream_t s)
{
    if (m <= 0 || R <= 0)
        return;
    hipLaunchKernelGGL(k_recode_ranks, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, keys,
                       lowd, m, vals, R);
}

// Diameters back from the keys of launch_desc_keys (the low 32 bits hold
// the complemented bit pattern).
__global__ void k_diam_from_keys(const uint64_t *__restrict__ keys, int64_t count,
                                 float *__restrict__ diam)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count)
        diam[i] = __uint_as_float(~(uint32_t)keys[i]);
}

void launch_diam_from_keys(const uint64_t *keys, int64_t count, float *diam, hipStream_t s)
{
    if (count <= 0)
        return;
    hipLaunchKernelGGL(k_diam_from_keys, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s,
                       keys, count, diam);
}

void launch_desc_keys(const float *diam, int64_t count, uint64_t *keys, hipStream_t s, Batch bt,
                      int nbatch)
{
    if (count <= 0)
        return;
    hipLaunchKernelGGL(k_desc_keys, dim3((unsigned)((count + 255) / 256), nbatch), dim3(256), 0,
                       s, diam, count, keys, bt);
}

// ===========================================================================
// a7: low of every non-apparent column, for the host reduction
// ===========================================================================
template <int P>
__global__ __launch_bounds__(256) void k_lows(const uint64_t *__restrict__ na_key,
                                              const uint64_t *__restrict__ na_cidx,
                                              int64_t ncols, const float *__restrict__ dsq,
                                              int n, float thr,
                                              const uint64_t *__restrict__ binom,
                                              uint64_t *__restrict__ low_out,
                                              float *__restrict__ low_diam_out, Batch bt,
                                              const float *__restrict__ thr_dev)
{
    const int lane = threadIdx.x & (WAVE - 1);
    const int64_t wave_id = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / WAVE;
    {
        const int64_t cl = blockIdx.y, st = bt.stride;
        ncols = batch_count(bt, cl, ncols);
        na_key += cl * st;
        na_cidx += cl * st;
        low_out += cl * st;
        low_diam_out += cl * st;
        dsq += cl * (int64_t)n * n;
        if (thr_dev)
            thr = thr_dev[cl];
    }
    const Binom B{binom, n + 1};
    for (int64_t col = wave_id; col < ncols; col += nwaves) {  // whole waves per column
        const float d = __uint_as_float(~(uint32_t)na_key[col]);
        int v[P + 1];
        decode<P>(B, na_cidx[col], n, v);
        const float *row[P + 1];
#pragma unroll
        for (int i = 0; i <= P; ++i)
            row[i] = dsq + (int64_t)v[i] * n;
        float best = INFINITY;
        int bw = -1;
        for (int base = 0; base < n; base += WAVE) {
            const int w = base + lane;
            if (w >= n)
                break;
            bool ok = true;
            float m = d;
#pragma unroll
            for (int i = 0; i <= P; ++i) {
                const float e = row[i][w];
                ok = ok && (w != v[i]) && (e <= thr);
                m = fmaxf(m, e);
            }
            // later w wins ties: larger w gives the larger cofacet cidx
            if (ok && m <= best) {
                best = m;
                bw = w;
            }
        }
#pragma unroll
        for (int o = WAVE / 2; o > 0; o >>= 1) {
            const float ob = __shfl_xor(best, o, WAVE);
            const int ow = __shfl_xor(bw, o, WAVE);
            if (ob < best || (ob == best && ow > bw)) {
                best = ob;
                bw = ow;
            }
        }
        if (lane == 0) {
            low_out[col] = bw >= 0 ? cofacet_index<P>(B, v, bw) : NONE;
            low_diam_out[col] = best;
        }
    }
}

void launch_lows(const uint64_t *na_key, const uint64_t *na_cidx, int64_t ncols,
                 const float *dsq, int n, int p, float thr, const uint64_t *binom,
                 uint64_t *low_out, float *low_diam_out, hipStream_t s, Batch bt, int nbatch,
                 const float *thr_dev)
{
    if (ncols <= 0)
        return;
    int64_t blocks = (ncols * WAVE + 255) / 256;
    if (bt.count && blocks > 256)
        blocks = 256;  // batched: counts live on the device; waves loop over columns
    dim3 g((unsigned)blocks, nbatch), b(256);
    switch (p) {
    case 1: hipLaunchKernelGGL(k_lows<1>, g, b, 0, s, na_key, na_cidx, ncols, dsq, n, thr, binom, low_out, low_diam_out, bt, thr_dev); break;
    case 2: hipLaunchKernelGGL(k_lows<2>, g, b, 0, s, na_key, na_cidx, ncols, dsq, n, thr, binom, low_out, low_diam_out, bt, thr_dev); break;
    case 3: hipLaunchKernelGGL(k_lows<3>, g, b, 0, s, na_key, na_cidx, ncols, dsq, n, thr, binom, low_out, low_diam_out, bt, thr_dev); break;
    default: hipLaunchKernelGGL(k_lows<4>, g, b, 0, s, na_key, na_cidx, ncols, dsq, n, thr, binom, low_out, low_diam_out, bt, thr_dev); break;
    }
}


// ===========================================================================
// sparse path: neighbour bitsets, extension enumeration, apparent test
// ===========================================================================
__global__ void k_nbr_bits(const float *__restrict__ dsq, int n, float thr,
                           uint64_t *__restrict__ bits, int words)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)n * words)
        return;
    const int v = (int)(t / words), k = (int)(t % words);
    const float *row = dsq + (int64_t)v * n;
    uint64_t m = 0;
    const int base = k * 64;
    for (int b = 0; b < 64; ++b) {
        const int u = base + b;
        if (u < n && u != v && row[u] <= thr)
            m |= 1ull << b;
    }
    bits[t] = m;
}

void launch_nbr_bits(const float *dsq, int n, float thr, uint64_t *bits, int words, hipStream_t s)
{
    const int64_t tot = (int64_t)n * words;
    hipLaunchKernelGGL(k_nbr_bits, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, dsq, n,
                       thr, bits, words);
}

// Degree of every vertex in the threshold graph: one wave per row.
__global__ __launch_bounds__(256) void k_nbr_degree(const uint64_t *__restrict__ bits, int n,
                                                   int words, uint32_t *__restrict__ deg)
{
    const int lane = threadIdx.x & (WAVE - 1);
    const int64_t v = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
    if (v >= n)
        return;
    uint32_t c = 0;
    for (int k = lane; k < words; k += WAVE)
        c += (uint32_t)__popcll(bits[v * words + k]);
    c = wave_sum(c);
    if (lane == 0)
        deg[v] = c;
}

void launch_nbr_degree(const uint64_t *bits, int n, int words, uint32_t *deg, hipStream_t s)
{
    if (n <= 0)
        return;
    hipLaunchKernelGGL(k_nbr_degree, dim3((unsigned)(((int64_t)n * WAVE + 255) / 256)), dim3(256),
                       0, s, bits, n, words, deg);
}

// Packed rows: one wave per vertex, lane k on word k of a 64-word block; the
// position of a word's first neighbour is the row offset plus an exclusive
// scan of the words' popcounts.
__global__ __launch_bounds__(256) void k_nbr_pack(const float *__restrict__ dsq,
                                                 const uint64_t *__restrict__ bits, int n,
                                                 int words, const uint64_t *__restrict__ row_off,
                                                 uint4 *__restrict__ nbw,
                                                 float *__restrict__ nbd, uint64_t cap)
{
    const int lane = threadIdx.x & (WAVE - 1);
    const int64_t v = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
    if (v >= n)
        return;
    uint64_t run = row_off[v];
    const float *row = dsq + v * n;
    for (int wb = 0; wb < words; wb += WAVE) {
        const int k = wb + lane;
        const uint64_t m = k < words ? bits[v * words + k] : 0ull;
        const uint32_t c = (uint32_t)__popcll(m);
        const uint32_t inc = wave_inclusive_scan(c);
        uint64_t pos = run + (inc - c);
        if (k < words)
            nbw[v * words + k] = make_uint4((uint32_t)m, (uint32_t)(m >> 32), (uint32_t)pos, 0u);
        for (uint64_t r = m; r && pos < cap; r &= r - 1)
            nbd[pos++] = row[k * 64 + __ffsll((unsigned long long)r) - 1];
        run += __shfl(inc, WAVE - 1, WAVE);
    }
}

void launch_nbr_pack(const float *dsq, const uint64_t *bits, int n, int words,
                     const uint64_t *row_off, uint4 *nbw, float *nbd, uint64_t cap,
                     hipStream_t s)
{
    if (n <= 0)
        return;
    hipLaunchKernelGGL(k_nbr_pack, dim3((unsigned)(((int64_t)n * WAVE + 255) / 256)), dim3(256),
                       0, s, dsq, bits, n, words, row_off, nbw, nbd, cap);
}

// Word k of v's neighbour row as one 16-byte record: its bitset word and the
// packed position of its first neighbour.
__device__ __forceinline__ void nb_word(const uint4 *__restrict__ nbw, int64_t idx,
                                        uint64_t &bits, uint32_t &pre)
{
    const uint4 x = nbw[idx];
    bits = (uint64_t)x.x | ((uint64_t)x.y << 32);
    pre = x.z;
}

// d(v, u) for a neighbour u = 64k + b of v, given v's bitset word k and the
// packed position of its first neighbour in that word.
__device__ __forceinline__ float nb_dist(const float *__restrict__ nbd, uint32_t pre,
                                         uint64_t word_bits, int b)
{
    return nbd[pre + (uint32_t)__popcll(word_bits & ((1ull << b) - 1ull))];
}

// First index j of the sorted array a[0, m) with a[j] >= key (m if none),
// found by the whole wave: each round probes 64 evenly spaced entries and
// keeps the interval between the last probe below the key and the next, so
// four rounds cover 2^24 entries.  Every lane returns the same value; call
// with the whole wave.
__device__ __forceinline__ int64_t wave_lower_bound(const uint64_t *__restrict__ a, int64_t m,
                                                    uint64_t key)
{
    const int lane = threadIdx.x & (WAVE - 1);
    int64_t lo = 0, hi = m;  // a[j] < key for j < lo; a[hi] >= key or hi == m
    while (hi - lo > WAVE) {
        const int64_t step = (hi - lo + WAVE - 1) / WAVE;
        const int64_t j = lo + (int64_t)lane * step;
        const bool below = j < hi && a[j] < key;
        const int c = __popcll(__ballot(below));  // the probes below key come first
        if (c == 0) {
            hi = lo;
            break;
        }
        const int64_t nhi = lo + (int64_t)c * step;
        lo = lo + (int64_t)(c - 1) * step + 1;
        hi = nhi < hi ? nhi : hi;
    }
    const int64_t j = lo + lane;
    const bool below = j < hi && a[j] < key;
    return lo + __popcll(__ballot(below));
}

// One wave per prefix, one lane per 64-vertex word of candidates v_0 < v_1.
// Count pass (WRITE = false): extensions per prefix.  Scatter pass: every
// extension to all_* (when given) and the uncleared ones to kept_*.
template <int P, bool WRITE>
__global__ __launch_bounds__(256) void k_ext(ExtArgs a, uint32_t *__restrict__ cnt_all,
                                             const uint64_t *__restrict__ off_all,
                                             float *__restrict__ all_diam,
                                             uint64_t *__restrict__ all_cidx,
                                             const uint64_t *__restrict__ clear, int64_t nclear,
                                             float *__restrict__ kept_diam,
                                             uint64_t *__restrict__ kept_cidx, uint64_t kept_cap,
                                             uint64_t *__restrict__ kept_vtx,
                                             const int64_t *__restrict__ cpos_all)
{
    const int lane = threadIdx.x & (WAVE - 1);
    const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
    // the wave's prefix, wave-uniform: what derives from it sits in scalar
    // registers
    const int pre = __builtin_amdgcn_readfirstlane((int)((blk * blockDim.x + threadIdx.x) / WAVE));
    if (pre >= a.npre_count)
        return;  // whole waves leave together
    const Binom B{a.binom, a.n + 1};
    int u[P];  // prefix vertices, decreasing; u[P-1] = v_1
    decode<P - 1>(B, a.pre_cidx[pre], a.n, u);
#pragma unroll
    for (int i = 0; i < P; ++i)
        u[i] = __builtin_amdgcn_readfirstlane(u[i]);
    // cidx of (u, v0) = sum_i C(u_i, P+1-i) + v0
    uint64_t shifted = 0;
#pragma unroll
    for (int i = 0; i < P; ++i)
        shifted += B(u[i], P + 1 - i);
    const int limit = u[P - 1];
    if (!WRITE) {
        uint32_t tot = 0;
        for (int wb = 0; wb * 64 < limit; wb += WAVE) {
            const int word = wb + lane;
            uint64_t m = 0;
            if (word * 64 < limit) {
                m = ~0ull;
#pragma unroll
                for (int i = 0; i < P; ++i)
                    m &= (uint64_t)a.nbw[(int64_t)u[i] * a.words + word].x |
                         ((uint64_t)a.nbw[(int64_t)u[i] * a.words + word].y << 32);
                const int hi = limit - word * 64;  // keep bits below v_1
                if (hi < 64)
                    m &= (1ull << hi) - 1;
            }
            tot += wave_sum((uint32_t)__popcll(m));
        }
        if (lane == 0)
            cnt_all[pre] = tot;
        return;
    }
    const float pd = a.pre_diam[pre];
    // the kept columns' vertex tuples, 16 bits per vertex from the largest
    // (the form the apparent kernels read instead of decoding the column)
    uint64_t vtx_hi = 0;
    if (P <= 3) {
#pragma unroll
        for (int i = 0; i < P; ++i)
            vtx_hi |= (uint64_t)(uint32_t)u[i] << (16 * i);
    }
    uint64_t run = off_all[pre];
    // cleared entries below this prefix's first extension: the kept entries
    // of the prefix start that many places before its extensions
    int64_t cpos = cpos_all ? cpos_all[pre]
                            : (nclear ? wave_lower_bound(clear, nclear, shifted) : 0);
    uint64_t krun = run - (uint64_t)cpos;
    for (int wb = 0; wb * 64 < limit; wb += WAVE) {
        const int word = wb + lane;
        uint64_t m = 0, bw[P];
        uint32_t pw[P];
#pragma unroll
        for (int i = 0; i < P; ++i) {
            bw[i] = 0;
            pw[i] = 0;
        }
        if (word * 64 < limit) {
            m = ~0ull;
#pragma unroll
            for (int i = 0; i < P; ++i) {
                nb_word(a.nbw, (int64_t)u[i] * a.words + word, bw[i], pw[i]);
                m &= bw[i];
            }
            const int hi = limit - word * 64;
            if (hi < 64)
                m &= (1ull << hi) - 1;
        }
        // this block's cleared extensions, 64 clear entries per step: the
        // ones below the block's end belong to it (the clear entries are
        // sorted, a subset of the extensions, and none lies below the
        // prefix's first extension past cpos)
        const int blk_end = (wb + WAVE) * 64 < limit ? (wb + WAVE) * 64 : limit;
        uint64_t cm = 0;
        for (;;) {
            const int64_t j = cpos + lane;
            const uint64_t cv = j < nclear ? clear[j] : ~0ull;
            const bool in = cv < shifted + (uint64_t)blk_end;
            const uint64_t bm = __ballot(in);
            const int c = __popcll(bm);
            for (int k = 0; k < c; ++k) {
                const uint64_t x = __shfl(cv, k, WAVE) - shifted;  // the cleared v0
                if ((int)(x >> 6) == word)
                    cm |= 1ull << (x & 63);
            }
            cpos += c;
            if (c < WAVE)
                break;
        }
        const uint64_t km = m & ~cm;
        const uint32_t na = (uint32_t)__popcll(m), nk = (uint32_t)__popcll(km);
        const uint32_t ia = wave_inclusive_scan(na), ik = wave_inclusive_scan(nk);
        const uint32_t tot = __shfl(ia, WAVE - 1, WAVE), totk = __shfl(ik, WAVE - 1, WAVE);
        // One extension per lane: lane l of round e0 takes extension e0 + l
        // of the block (cidx order), found in the word of the first lane
        // whose inclusive count exceeds it, at the matching set bit; so the
        // lookups and stores run on every lane however the extensions lie
        // across the words (a lane walking its own word's bits would leave
        // most lanes idle where a prefix's extensions crowd a few words).
        for (uint32_t e0 = 0; e0 < tot; e0 += WAVE) {
            const uint32_t e = e0 + (uint32_t)lane;
            int lo = 0;
#pragma unroll
            for (int step = WAVE / 2; step >= 1; step >>= 1) {
                const uint32_t x = __shfl(ia, lo + step - 1, WAVE);
                lo += x <= e ? step : 0;
            }
            const uint64_t mw = shfl_u64(m, lo), kw = shfl_u64(km, lo);
            const uint32_t exa = __shfl(ia - na, lo, WAVE), exk = __shfl(ik - nk, lo, WAVE);
            uint64_t bl[P];
            uint32_t pl[P];
#pragma unroll
            for (int i = 0; i < P; ++i) {
                bl[i] = shfl_u64(bw[i], lo);
                pl[i] = (uint32_t)__shfl((int)pw[i], lo, WAVE);
            }
            if (e < tot) {
                const int b = select_set_bit(mw, (int)(e - exa));
                const int v0 = (wb + lo) * 64 + b;
                float d = pd;
#pragma unroll
                for (int i = 0; i < P; ++i)
                    d = fmaxf(d, nb_dist(a.nbd, pl[i], bl[i], b));
                const uint64_t c = shifted + (uint64_t)v0;
                if (all_diam) {
                    all_diam[run + e] = d;
                    all_cidx[run + e] = c;
                }
                if ((kw >> b) & 1ull) {
                    const uint64_t pk =
                        krun + exk + (uint32_t)__popcll(kw & ((1ull << b) - 1ull));
                    if (pk < kept_cap) {  // (the cap only guards the subset property)
                        kept_diam[pk] = d;
                        kept_cidx[pk] = c;
                        if (P <= 3 && kept_vtx)
                            kept_vtx[pk] = vtx_hi | ((uint64_t)(uint32_t)v0 << (16 * P));
                    }
                }
            }
        }
        run += tot;
        krun += totk;
    }
}

#define RPP_EXT_LAUNCH(WR, ...)                                                                  \
    switch (a.p) {                                                                               \
    case 2: hipLaunchKernelGGL((k_ext<2, WR>), g, b, 0, s, a, __VA_ARGS__); break;               \
    case 3: hipLaunchKernelGGL((k_ext<3, WR>), g, b, 0, s, a, __VA_ARGS__); break;               \
    default: hipLaunchKernelGGL((k_ext<4, WR>), g, b, 0, s, a, __VA_ARGS__); break;              \
    }

void launch_ext_count(const ExtArgs &a, uint32_t *cnt_all, hipStream_t s)
{
    if (a.npre_count <= 0)
        return;
    dim3 g((unsigned)((a.npre_count * WAVE + 255) / 256)), b(256);
    RPP_EXT_LAUNCH(false, cnt_all, nullptr, nullptr, nullptr, nullptr, (int64_t)0, nullptr,
                   nullptr, (uint64_t)0, nullptr, nullptr)
}

void launch_ext_scatter(const ExtArgs &a, const uint64_t *off_all, float *all_diam,
                        uint64_t *all_cidx, const uint64_t *clear, int64_t nclear,
                        float *kept_diam, uint64_t *kept_cidx, uint64_t kept_cap,
                        uint64_t *kept_vtx, hipStream_t s, const int64_t *cpos)
{
    if (a.npre_count <= 0)
        return;
    if (a.p > 3 || a.n > 65536)
        kept_vtx = nullptr;
    dim3 g((unsigned)((a.npre_count * WAVE + 255) / 256)), b(256);
    RPP_EXT_LAUNCH(true, nullptr, off_all, all_diam, all_cidx, clear, nclear, kept_diam,
                   kept_cidx, kept_cap, kept_vtx, cpos)
}

// Youngest-facet condition of the apparent pairs lemma for sigma (vertices
// v, diameter d) and its oldest cofacet sigma + {w}, e[i] = d(v_i, w): no
// facet sigma - {v_j} + {w} with v_j > w (those precede sigma) has diameter
// d.  The distances among sigma's own vertices (all within the threshold)
// are read from the packed rows, and only when some v_j lies above w.
template <int P>
__device__ __forceinline__ bool apparent_facets_ok(const uint4 *__restrict__ nbw,
                                                   const float *__restrict__ nbd, int words,
                                                   const int (&v)[P + 1], float d, int w,
                                                   const float (&e)[P + 1])
{
    bool need = false;
#pragma unroll
    for (int j = 0; j <= P; ++j)
        need = need || v[j] > w;
    if (!need)
        return true;
    float dv[P + 1][P + 1];
#pragma unroll
    for (int a = 0; a <= P; ++a)
#pragma unroll
        for (int b = a + 1; b <= P; ++b) {
            uint64_t wb;
            uint32_t wp;
            nb_word(nbw, (int64_t)v[a] * words + (v[b] >> 6), wb, wp);
            dv[a][b] = nb_dist(nbd, wp, wb, v[b] & 63);
        }
#pragma unroll
    for (int j = 0; j <= P; ++j) {
        if (v[j] > w) {
            float fd = 0.0f;
#pragma unroll
            for (int a = 0; a <= P; ++a) {
                if (a == j)
                    continue;
                fd = fmaxf(fd, e[a]);
#pragma unroll
                for (int b = a + 1; b <= P; ++b)
                    if (b != j)
                        fd = fmaxf(fd, dv[a][b]);
            }
            if (fd == d)
                return false;
        }
    }
    return true;
}

// Sparse apparent test.  The candidates for sigma's oldest cofacet are the
// common neighbours of its vertices: the AND of their neighbour bitsets,
// which leaves out sigma's own vertices.  Layout as in the dense kernel: a
// wave owns CPR x rounds columns, every lane decodes one, and each round G
// lanes take one column.  The group scans G words per step from the top
// (lane g: word top - g); each lane walks its word's candidates downward
// and stops at its first hit (every d(v_i, x) <= d).  The group's hit is
// that of its first lane with one: the lanes before it hold higher words
// and had no candidate that passed.  A column usually ends in its first
// step, so it reads G words of each of its vertices' bitsets instead of
// whole rows.
template <int P, int G>
__global__ __launch_bounds__(256) void k_apparent_sparse(
    const float *__restrict__ col_diam, const uint64_t *__restrict__ col_cidx, int64_t ncols,
    int n, int words, const uint4 *__restrict__ nbw, const float *__restrict__ nbd,
    const uint64_t *__restrict__ binom, uint64_t *__restrict__ tau_out,
    unsigned long long *__restrict__ scan_count, int rounds,
    const uint64_t *__restrict__ col_vtx)
{
    constexpr int CPR = WAVE / G;  // columns per round
    const int lane = threadIdx.x & (WAVE - 1);
    const int g = lane & (G - 1);
    const int grp = lane / G;
    const int gbase = lane - g;
    const uint64_t gmask = (G == WAVE) ? ~0ull : (((1ull << G) - 1) << gbase);
    const int own = CPR * rounds;  // columns owned by a wave (rounds <= G)
    const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
    const int64_t base = ((blk * blockDim.x + threadIdx.x) / WAVE) * own;
    if (base >= ncols)
        return;  // whole waves leave together
    const Binom B{binom, n + 1};
    const int64_t mycol = base + lane;
    const bool myvalid = lane < own && mycol < ncols;
    float myd = 0.0f;
    int myv[P + 1];
#pragma unroll
    for (int i = 0; i <= P; ++i)
        myv[i] = 0;
    if (myvalid) {
        myd = col_diam[mycol];
        if (P <= 3 && col_vtx) {
            const uint64_t x = col_vtx[mycol];
#pragma unroll
            for (int i = 0; i <= P; ++i)
                myv[i] = (int)((x >> (16 * i)) & 0xffffu);
        } else {
            decode<P>(B, col_cidx[mycol], n, myv);
        }
    }
    uint64_t mytau = NONE;
    unsigned long long examined = 0;  // this lane's share of the candidates visited
    for (int r = 0; r < rounds; ++r) {
        const int src = r * CPR + grp;
        const float d = __shfl(myd, src, WAVE);
        int v[P + 1];
#pragma unroll
        for (int i = 0; i <= P; ++i)
            v[i] = __shfl(myv[i], src, WAVE);
        const bool valid = base + src < ncols;  // uniform in the group
        int x = -1;  // this lane's hit in the current step
        int hit = -1;
        float e[P + 1];
#pragma unroll
        for (int i = 0; i <= P; ++i)
            e[i] = 0.0f;
        if (valid) {
            for (int top = words - 1; top >= 0; top -= G) {
                const int word = top - g;
                uint64_t m = 0, bw[P + 1];
                uint32_t pw[P + 1];
                if (word >= 0) {
                    m = ~0ull;
#pragma unroll
                    for (int i = 0; i <= P; ++i) {
                        nb_word(nbw, (int64_t)v[i] * words + word, bw[i], pw[i]);
                        m &= bw[i];
                    }
                }
                unsigned tested = 0;
                for (uint64_t mm = m; mm;) {
                    const int b = 63 - __clzll((long long)mm);
                    const int c = word * 64 + b;
                    bool ok = true;
                    float t[P + 1];
#pragma unroll
                    for (int i = 0; i <= P; ++i) {
                        t[i] = nb_dist(nbd, pw[i], bw[i], b);
                        ok = ok && (t[i] <= d);
                    }
                    ++tested;
                    if (ok) {
                        x = c;
#pragma unroll
                        for (int i = 0; i <= P; ++i)
                            e[i] = t[i];
                        break;
                    }
                    mm &= ~(1ull << b);
                }
                const uint64_t hm = __ballot(x >= 0) & gmask;
                const int hl = hm ? __ffsll((unsigned long long)hm) - 1 - gbase : G;
                // candidates visited from the top: every one of the lanes
                // before the hit lane, the hit lane's down to its hit
                if (scan_count)
                    examined += g < hl ? (unsigned)__popcll(m) : (g == hl ? tested : 0u);
                if (hm) {
                    hit = gbase + hl;
                    break;
                }
            }
        }
        // w and d(v_i, w) from the lane that hit (every lane joins the shuffle)
        const int w = __shfl(x, hit >= 0 ? hit : lane, WAVE);
        float ew[P + 1];
#pragma unroll
        for (int i = 0; i <= P; ++i)
            ew[i] = __shfl(e[i], hit >= 0 ? hit : lane, WAVE);
        uint64_t tau = NONE;
        if (hit >= 0) {
            // distances among sigma's vertices, needed only when a vertex of
            // sigma lies above w (sigma's edges are all within the
            // threshold: packed-row lookups)
            bool need = false;
#pragma unroll
            for (int j = 0; j <= P; ++j)
                need = need || v[j] > w;
            float dv[P + 1][P + 1];
#pragma unroll
            for (int a = 0; a <= P; ++a)
#pragma unroll
                for (int b = a + 1; b <= P; ++b) {
                    dv[a][b] = 0.0f;
                    if (need) {
                        uint64_t wb;
                        uint32_t wp;
                        nb_word(nbw, (int64_t)v[a] * words + (v[b] >> 6), wb, wp);
                        dv[a][b] = nb_dist(nbd, wp, wb, v[b] & 63);
                    }
                }
            bool apparent = true;
#pragma unroll
            for (int j = 0; j <= P; ++j) {
                if (v[j] > w && apparent) {
                    // facet sigma - {v_j} + {w}
                    float fd = 0.0f;
#pragma unroll
                    for (int a = 0; a <= P; ++a) {
                        if (a == j)
                            continue;
                        fd = fmaxf(fd, ew[a]);
#pragma unroll
                        for (int b = a + 1; b <= P; ++b)
                            if (b != j)
                                fd = fmaxf(fd, dv[a][b]);
                    }
                    if (fd == d)
                        apparent = false;
                }
            }
            if (apparent)
                tau = cofacet_index<P>(B, v, w);
        }
        // the owner of column base + r*CPR + k is lane r*CPR + k; group k's
        // first lane holds its tau
        const uint64_t t = shfl_u64(tau, (lane % CPR) * G);
        if (lane / CPR == r)
            mytau = t;
    }
    if (scan_count) {
        const unsigned long long tot = wave_sum(examined);
        if (lane == 0)
            atomicAdd(&scan_count[blockIdx.x & (SCAN_COUNTERS - 1)], tot);
    }
    if (myvalid)
        tau_out[mycol] = mytau;
}

// Phase 2 of the two-phase sparse apparent test: the wave's open columns
// (omask; a lane's own column has vertices myv, diameter myd) numbered in
// lane order and scanned G lanes per column from word top0 down, as
// k_apparent_sparse scans.  Returns, on each open column's lane, its tau
// (NONE when not apparent); adds the candidates visited to `examined` when
// counting.  Every lane of the wave must call it.
template <int P, int G>
__device__ __forceinline__ uint64_t sparse_open_columns(uint64_t omask, const int (&myv)[P + 1],
                                                        float myd, int top0, int words,
                                                        const uint4 *__restrict__ nbw,
                                                        const float *__restrict__ nbd,
                                                        const Binom &B, bool counting,
                                                        unsigned long long &examined)
{
    constexpr int CPR = WAVE / G;  // open columns per round
    const int lane = threadIdx.x & (WAVE - 1);
    const int g = lane & (G - 1);
    const int grp = lane / G;
    const int gbase = lane - g;
    const uint64_t gmask = (G == WAVE) ? ~0ull : (((1ull << G) - 1) << gbase);
    const bool open = (omask >> lane) & 1ull;
    const int nopen = __popcll(omask);
    uint64_t tau2 = NONE;
    for (int r = 0; r * CPR < nopen; ++r) {
        const int t = r * CPR + grp;
        const bool valid = t < nopen;  // uniform in the group
        const int src = valid ? select_set_bit(omask, t) : lane;
        const float d = __shfl(myd, src, WAVE);
        int v[P + 1];
#pragma unroll
        for (int i = 0; i <= P; ++i)
            v[i] = __shfl(myv[i], src, WAVE);
        int x = -1;  // this lane's hit in the current step
        int hit = -1;
        float e[P + 1];
#pragma unroll
        for (int i = 0; i <= P; ++i)
            e[i] = 0.0f;
        if (valid) {
            for (int top = top0; top >= 0; top -= G) {
                const int word = top - g;
                uint64_t m = 0, bw[P + 1];
                uint32_t pw[P + 1];
                if (word >= 0) {
                    m = ~0ull;
#pragma unroll
                    for (int i = 0; i <= P; ++i) {
                        nb_word(nbw, (int64_t)v[i] * words + word, bw[i], pw[i]);
                        m &= bw[i];
                    }
                }
                unsigned tested = 0;
                for (uint64_t mm = m; mm;) {
                    const int b = 63 - __clzll((long long)mm);
                    bool ok = true;
                    float tt[P + 1];
#pragma unroll
                    for (int i = 0; i <= P; ++i) {
                        tt[i] = nb_dist(nbd, pw[i], bw[i], b);
                        ok = ok && (tt[i] <= d);
                    }
                    ++tested;
                    if (ok) {
                        x = word * 64 + b;
#pragma unroll
                        for (int i = 0; i <= P; ++i)
                            e[i] = tt[i];
                        break;
                    }
                    mm &= ~(1ull << b);
                }
                const uint64_t hm = __ballot(x >= 0) & gmask;
                const int hl = hm ? __ffsll((unsigned long long)hm) - 1 - gbase : G;
                if (counting)
                    examined += g < hl ? (unsigned)__popcll(m) : (g == hl ? tested : 0u);
                if (hm) {
                    hit = gbase + hl;
                    break;
                }
            }
        }
        const int ww = __shfl(x, hit >= 0 ? hit : lane, WAVE);
        float eh[P + 1];
#pragma unroll
        for (int i = 0; i <= P; ++i)
            eh[i] = __shfl(e[i], hit >= 0 ? hit : lane, WAVE);
        uint64_t tau = NONE;
        if (hit >= 0 && apparent_facets_ok<P>(nbw, nbd, words, v, d, ww, eh))
            tau = cofacet_index<P>(B, v, ww);
        // the owner of open column t is the t-th set lane of omask; group
        // (t mod CPR)'s first lane holds its tau
        const int mine = open ? __popcll(omask & lanemask_lt()) : -1;
        const int from = mine >= 0 ? (mine % CPR) * G : lane;
        const uint64_t tt = shfl_u64(tau, from);
        if (mine >= 0 && mine / CPR == r)
            tau2 = tt;
    }
    return tau2;
}

// Two-phase sparse apparent test.  Phase 1: every lane takes its own
// column and scans the top K bitset words of its vertices (all K (P+1)
// records loaded at once), testing the common neighbours word by word from
// the top; a column decides there unless none of them passes.  Phase 2: the
// columns still open (no hit in the K words, words left below) are numbered
// within the wave and scanned G lanes per column from word words-1-K down,
// exactly as k_apparent_sparse scans.  One wave owns 64 consecutive columns,
// so the per-column work of phase 1 (shuffles, facet test, cofacet index)
// runs once per 64 columns instead of once per 64/G.
template <int P, int K, int G>
__global__ __launch_bounds__(256) void k_apparent_sparse2(
    const float *__restrict__ col_diam, const uint64_t *__restrict__ col_cidx, int64_t ncols,
    int n, int words, const uint4 *__restrict__ nbw, const float *__restrict__ nbd,
    const uint64_t *__restrict__ binom, uint64_t *__restrict__ tau_out,
    unsigned long long *__restrict__ scan_count, const uint64_t *__restrict__ col_vtx)
{
    const int lane = threadIdx.x & (WAVE - 1);
    const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
    const int64_t base = ((blk * blockDim.x + threadIdx.x) / WAVE) * WAVE;
    if (base >= ncols)
        return;  // whole waves leave together
    const Binom B{binom, n + 1};
    const int64_t mycol = base + lane;
    const bool myvalid = mycol < ncols;
    float myd = 0.0f;
    int myv[P + 1];
#pragma unroll
    for (int i = 0; i <= P; ++i)
        myv[i] = 0;
    if (myvalid) {
        myd = col_diam[mycol];
        if (P <= 3 && col_vtx) {
            const uint64_t x = col_vtx[mycol];
#pragma unroll
            for (int i = 0; i <= P; ++i)
                myv[i] = (int)((x >> (16 * i)) & 0xffffu);
        } else {
            decode<P>(B, col_cidx[mycol], n, myv);
        }
    }
    unsigned long long examined = 0;  // this lane's share of the candidates visited

    // ---- phase 1: the top K words of the lane's own column ----
    int w = -1;
    float ew[P + 1];
#pragma unroll
    for (int i = 0; i <= P; ++i)
        ew[i] = 0.0f;
    if (myvalid) {
        uint64_t bw[K][P + 1];
        uint32_t pw[K][P + 1];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int word = words - 1 - k;
#pragma unroll
            for (int i = 0; i <= P; ++i) {
                bw[k][i] = 0;
                pw[k][i] = 0;
                if (word >= 0)
                    nb_word(nbw, (int64_t)myv[i] * words + word, bw[k][i], pw[k][i]);
            }
        }
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int word = words - 1 - k;
            uint64_t m = ~0ull;
#pragma unroll
            for (int i = 0; i <= P; ++i)
                m &= bw[k][i];
            while (m && w < 0) {
                const int b = 63 - __clzll((long long)m);
                bool ok = true;
                float t[P + 1];
#pragma unroll
                for (int i = 0; i <= P; ++i) {
                    t[i] = nb_dist(nbd, pw[k][i], bw[k][i], b);
                    ok = ok && (t[i] <= myd);
                }
                ++examined;
                if (ok) {
                    w = word * 64 + b;
#pragma unroll
                    for (int i = 0; i <= P; ++i)
                        ew[i] = t[i];
                }
                m &= ~(1ull << b);
            }
        }
    }
    // open: no hit in the K words and words left below them
    const bool open = myvalid && w < 0 && words - 1 - K >= 0;
    const uint64_t omask = __ballot(open);

    // ---- phase 2: open columns, G lanes each, from word words-1-K down ----
    const uint64_t tau2 = sparse_open_columns<P, G>(omask, myv, myd, words - 1 - K, words, nbw,
                                                    nbd, B, scan_count != nullptr, examined);
    if (scan_count) {
        const unsigned long long tot = wave_sum(examined);
        if (lane == 0)
            atomicAdd(&scan_count[blockIdx.x & (SCAN_COUNTERS - 1)], tot);
    }
    if (!myvalid)
        return;
    uint64_t mytau = NONE;
    if (open)
        mytau = tau2;
    else if (w >= 0 && apparent_facets_ok<P>(nbw, nbd, words, myv, myd, w, ew))
        mytau = cofacet_index<P>(B, myv, w);
    tau_out[mycol] = mytau;
}

// Cleared entries below each prefix's first extension (the clearing set is
// sorted): one thread per prefix and a plain binary search, so the fused
// scatter below reads one word instead of searching with a whole wave at
// its start.
template <int P>
__global__ __launch_bounds__(256) void k_clear_pos(ExtArgs a, const uint64_t *__restrict__ clear,
                                                   int64_t nclear, int64_t *__restrict__ cpos_out)
{
    const int64_t pre = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (pre >= a.npre_count)
        return;
    const Binom B{a.binom, a.n + 1};
    int u[P];
    decode<P - 1>(B, a.pre_cidx[pre], a.n, u);
    uint64_t shifted = 0;
#pragma unroll
    for (int i = 0; i < P; ++i)
        shifted += B(u[i], P + 1 - i);
    int64_t lo = 0, hi = nclear;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (clear[mid] < shifted)
            lo = mid + 1;
        else
            hi = mid;
    }
    cpos_out[pre] = lo;
}

void launch_clear_pos(const ExtArgs &a, const uint64_t *clear, int64_t nclear, int64_t *cpos,
                      hipStream_t s)
{
    if (a.npre_count <= 0)
        return;
    dim3 g((unsigned)((a.npre_count + 255) / 256)), b(256);
    switch (a.p) {
    case 2: hipLaunchKernelGGL(k_clear_pos<2>, g, b, 0, s, a, clear, nclear, cpos); break;
    case 3: hipLaunchKernelGGL(k_clear_pos<3>, g, b, 0, s, a, clear, nclear, cpos); break;
    default: hipLaunchKernelGGL(k_clear_pos<4>, g, b, 0, s, a, clear, nclear, cpos); break;
    }
}

// Scatter pass of the sparse enumeration with the apparent-pair test fused
// in (two-phase, as k_apparent_sparse2): a kept extension sigma = (u, v0) is
// tested on the lane that holds it, so its column never goes back to memory
// before the test, and the prefix's bitset records of the top K words --
// the same for every extension of the wave -- are read once per wave; only
// v0's records are per lane.  tau_out[kept position] gets the apparent
// partner or NONE.  Same outputs otherwise as k_ext<P, true> (no vertex
// tuples: nothing reads them after the test).
// W: the waves per SIMD the register allocation must allow (1: the
// compiler's choice, 100 VGPRs and four waves for P = 2; more trades
// spills for occupancy).  The default form takes 5 (96 VGPRs, 3 spilled):
// on the 4096-point sphere 1.38 -> 1.20 ms per stage; 6 (80 VGPRs, 25
// spilled) gives 1.35 and 8 (64, 48 spilled) 1.64.
template <int P, int K, int G, int W>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(W))) void k_ext_app(ExtArgs a, const uint64_t *__restrict__ off_all,
                                                 float *__restrict__ all_diam,
                                                 uint64_t *__restrict__ all_cidx,
                                                 const uint64_t *__restrict__ clear,
                                                 int64_t nclear, float *__restrict__ kept_diam,
                                                 uint64_t *__restrict__ kept_cidx,
                                                 uint64_t kept_cap, uint64_t *__restrict__ tau_out,
                                                 unsigned long long *__restrict__ scan_count,
                                                 const int64_t *__restrict__ cpos_all)
{
    const int lane = threadIdx.x & (WAVE - 1);
    const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
    // the wave's prefix, made wave-uniform so that everything derived from
    // it (its vertices, bitset records, offsets) sits in scalar registers
    const int pre = __builtin_amdgcn_readfirstlane((int)((blk * blockDim.x + threadIdx.x) / WAVE));
    if (pre >= a.npre_count)
        return;  // whole waves leave together
    const Binom B{a.binom, a.n + 1};
    const int words = a.words;
    int u[P];  // prefix vertices, decreasing; u[P-1] = v_1
    decode<P - 1>(B, a.pre_cidx[pre], a.n, u);
#pragma unroll
    for (int i = 0; i < P; ++i)
        u[i] = __builtin_amdgcn_readfirstlane(u[i]);
    uint64_t shifted = 0;
#pragma unroll
    for (int i = 0; i < P; ++i)
        shifted += B(u[i], P + 1 - i);
    const int limit = u[P - 1];
    const float pd = a.pre_diam[pre];
    // the prefix's records of the top K words (the same for every lane)
    uint64_t ub[K][P];
    uint32_t up[K][P];
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
        for (int i = 0; i < P; ++i) {
            ub[k][i] = 0;
            up[k][i] = 0;
            if (words - 1 - k >= 0)
                nb_word(a.nbw, (int64_t)u[i] * words + (words - 1 - k), ub[k][i], up[k][i]);
        }
    unsigned long long examined = 0;
    uint64_t run = off_all[pre];
    int64_t cpos = cpos_all ? cpos_all[pre]
                            : (nclear ? wave_lower_bound(clear, nclear, shifted) : 0);
    uint64_t krun = run - (uint64_t)cpos;
    for (int wb = 0; wb * 64 < limit; wb += WAVE) {
        const int word = wb + lane;
        uint64_t m = 0, bw[P];
        uint32_t pw[P];
#pragma unroll
        for (int i = 0; i < P; ++i) {
            bw[i] = 0;
            pw[i] = 0;
        }
        if (word * 64 < limit) {
            m = ~0ull;
#pragma unroll
            for (int i = 0; i < P; ++i) {
                nb_word(a.nbw, (int64_t)u[i] * words + word, bw[i], pw[i]);
                m &= bw[i];
            }
            const int hi = limit - word * 64;
            if (hi < 64)
                m &= (1ull << hi) - 1;
        }
        const int blk_end = (wb + WAVE) * 64 < limit ? (wb + WAVE) * 64 : limit;
        uint64_t cm = 0;
        for (;;) {
            const int64_t j = cpos + lane;
            const uint64_t cv = j < nclear ? clear[j] : ~0ull;
            const bool in = cv < shifted + (uint64_t)blk_end;
            const uint64_t bm = __ballot(in);
            const int c = __popcll(bm);
            for (int k = 0; k < c; ++k) {
                const uint64_t x = __shfl(cv, k, WAVE) - shifted;
                if ((int)(x >> 6) == word)
                    cm |= 1ull << (x & 63);
            }
            cpos += c;
            if (c < WAVE)
                break;
        }
        const uint64_t km = m & ~cm;
        const uint32_t na = (uint32_t)__popcll(m), nk = (uint32_t)__popcll(km);
        const uint32_t ia = wave_inclusive_scan(na), ik = wave_inclusive_scan(nk);
        const uint32_t tot = __shfl(ia, WAVE - 1, WAVE), totk = __shfl(ik, WAVE - 1, WAVE);
        for (uint32_t e0 = 0; e0 < tot; e0 += WAVE) {
            const uint32_t e = e0 + (uint32_t)lane;
            int lo = 0;
#pragma unroll
            for (int step = WAVE / 2; step >= 1; step >>= 1) {
                const uint32_t x = __shfl(ia, lo + step - 1, WAVE);
                lo += x <= e ? step : 0;
            }
            const uint64_t mw = shfl_u64(m, lo), kw = shfl_u64(km, lo);
            const uint32_t exa = __shfl(ia - na, lo, WAVE), exk = __shfl(ik - nk, lo, WAVE);
            uint64_t bl[P];
            uint32_t pl[P];
#pragma unroll
            for (int i = 0; i < P; ++i) {
                bl[i] = shfl_u64(bw[i], lo);
                pl[i] = (uint32_t)__shfl((int)pw[i], lo, WAVE);
            }
            bool kept = false;
            uint64_t pk = 0;
            int myv[P + 1];
#pragma unroll
            for (int i = 0; i <= P; ++i)
                myv[i] = 0;
            float myd = 0.0f;
            if (e < tot) {
                const int b = select_set_bit(mw, (int)(e - exa));
                const int v0 = (wb + lo) * 64 + b;
                float d = pd;
#pragma unroll
                for (int i = 0; i < P; ++i)
                    d = fmaxf(d, nb_dist(a.nbd, pl[i], bl[i], b));
                const uint64_t c = shifted + (uint64_t)v0;
                if (all_diam) {
                    all_diam[run + e] = d;
                    all_cidx[run + e] = c;
                }
                if ((kw >> b) & 1ull) {
                    pk = krun + exk + (uint32_t)__popcll(kw & ((1ull << b) - 1ull));
                    kept = pk < kept_cap;  // (the cap only guards the subset property)
                    if (kept) {
                        kept_diam[pk] = d;
                        kept_cidx[pk] = c;
                    }
                }
                myd = d;
#pragma unroll
                for (int i = 0; i < P; ++i)
                    myv[i] = u[i];
                myv[P] = v0;
            }
            // apparent test of the kept columns, phase 1: the top K words
            int w = -1;
            float ew[P + 1];
#pragma unroll
            for (int i = 0; i <= P; ++i)
                ew[i] = 0.0f;
            if (kept) {
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    const int wd = words - 1 - k;
                    if (wd < 0 || w >= 0)
                        continue;
                    uint64_t vb;
                    uint32_t vp;
                    nb_word(a.nbw, (int64_t)myv[P] * words + wd, vb, vp);
                    uint64_t mm = vb;
#pragma unroll
                    for (int i = 0; i < P; ++i)
                        mm &= ub[k][i];
                    while (mm && w < 0) {
                        const int b = 63 - __clzll((long long)mm);
                        bool ok = true;
                        float t[P + 1];
#pragma unroll
                        for (int i = 0; i < P; ++i) {
                            t[i] = nb_dist(a.nbd, up[k][i], ub[k][i], b);
                            ok = ok && (t[i] <= myd);
                        }
                        t[P] = nb_dist(a.nbd, vp, vb, b);
                        ok = ok && (t[P] <= myd);
                        ++examined;
                        if (ok) {
                            w = wd * 64 + b;
#pragma unroll
                            for (int i = 0; i <= P; ++i)
                                ew[i] = t[i];
                        }
                        mm &= ~(1ull << b);
                    }
                }
            }
            const bool open = kept && w < 0 && words - 1 - K >= 0;
            const uint64_t omask = __ballot(open);
            uint64_t tau2 = NONE;
            if (omask)  // uniform: every lane calls it or none
                tau2 = sparse_open_columns<P, G>(omask, myv, myd, words - 1 - K, words, a.nbw,
                                                 a.nbd, B, scan_count != nullptr, examined);
            if (kept) {
                uint64_t tau = NONE;
                if (open)
                    tau = tau2;
                else if (w >= 0 && apparent_facets_ok<P>(a.nbw, a.nbd, words, myv, myd, w, ew))
                    tau = cofacet_index<P>(B, myv, w);
                tau_out[pk] = tau;
            }
        }
        run += tot;
        krun += totk;
    }
    if (scan_count) {
        const unsigned long long t = wave_sum(examined);
        if (lane == 0)
            atomicAdd(&scan_count[blockIdx.x & (SCAN_COUNTERS - 1)], t);
    }
}

template <int P>
static void launch_ext_app_p(const ExtArgs &a, int group, dim3 g, dim3 b, hipStream_t s,
                             const uint64_t *off_all, float *all_diam, uint64_t *all_cidx,
                             const uint64_t *clear, int64_t nclear, float *kept_diam,
                             uint64_t *kept_cidx, uint64_t kept_cap, uint64_t *tau,
                             unsigned long long *sc, const int64_t *cpos)
{
#define RPP_EA(K, G, W) hipLaunchKernelGGL((k_ext_app<P, K, G, W>), g, b, 0, s, a, off_all, all_diam, all_cidx, clear, nclear, kept_diam, kept_cidx, kept_cap, tau, sc, cpos)
    // RPP_EXT_APP_WAVES (1, 5, 6 or 8): the default form compiled for that
    // many waves per SIMD (a tuning knob; 5 unless set)
    const char *we = getenv("RPP_EXT_APP_WAVES");
    const int waves = we ? atoi(we) : 5;
    switch (group) {
    case 104: RPP_EA(1, 4, 1); break;
    case 108: RPP_EA(1, 8, 1); break;
    case 204: RPP_EA(2, 4, 1); break;
    case 208: RPP_EA(2, 8, 1); break;
    case 408: RPP_EA(4, 8, 1); break;
    default:
        if (waves == 5)
            RPP_EA(4, 4, 5);
        else if (waves == 6)
            RPP_EA(4, 4, 6);
        else if (waves == 8)
            RPP_EA(4, 4, 8);
        else
            RPP_EA(4, 4, 1);
        break;
    }
#undef RPP_EA
}

void launch_ext_scatter_apparent(const ExtArgs &a, int group, const uint64_t *off_all,
                                 float *all_diam, uint64_t *all_cidx, const uint64_t *clear,
                                 int64_t nclear, float *kept_diam, uint64_t *kept_cidx,
                                 uint64_t kept_cap, uint64_t *tau_out,
                                 unsigned long long *scan_count, hipStream_t s,
                                 const int64_t *cpos)
{
    if (a.npre_count <= 0)
        return;
    dim3 g((unsigned)((a.npre_count * WAVE + 255) / 256)), b(256);
    switch (a.p) {
    case 2: launch_ext_app_p<2>(a, group, g, b, s, off_all, all_diam, all_cidx, clear, nclear, kept_diam, kept_cidx, kept_cap, tau_out, scan_count, cpos); break;
    case 3: launch_ext_app_p<3>(a, group, g, b, s, off_all, all_diam, all_cidx, clear, nclear, kept_diam, kept_cidx, kept_cap, tau_out, scan_count, cpos); break;
    default: launch_ext_app_p<4>(a, group, g, b, s, off_all, all_diam, all_cidx, clear, nclear, kept_diam, kept_cidx, kept_cap, tau_out, scan_count, cpos); break;
    }
}

template <int P>
__global__ __launch_bounds__(256) void k_lows_sparse(
    const uint64_t *__restrict__ na_key, const uint64_t *__restrict__ na_cidx, int64_t ncols,
    const uint4 *__restrict__ nbw, const float *__restrict__ nbd, int n, int words,
    const uint64_t *__restrict__ binom, uint64_t *__restrict__ low_out,
    float *__restrict__ low_diam_out)
{
    const int lane = threadIdx.x & (WAVE - 1);
    const int64_t col = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
    if (col >= ncols)
        return;
    const Binom B{binom, n + 1};
    const float d = __uint_as_float(~(uint32_t)na_key[col]);
    int v[P + 1];
    decode<P>(B, na_cidx[col], n, v);
    float best = INFINITY;
    int bw = -1;
    for (int word = lane; word < words; word += WAVE) {
        uint64_t m = ~0ull, wbits[P + 1];
        uint32_t wpre[P + 1];
#pragma unroll
        for (int i = 0; i <= P; ++i) {
            nb_word(nbw, (int64_t)v[i] * words + word, wbits[i], wpre[i]);
            m &= wbits[i];
        }
        for (; m; m &= m - 1) {
            const int b = __ffsll((unsigned long long)m) - 1;
            const int x = word * 64 + b;
            float c = d;
#pragma unroll
            for (int i = 0; i <= P; ++i)
                c = fmaxf(c, nb_dist(nbd, wpre[i], wbits[i], b));
            if (c <= best) {  // ascending x: later (larger) x wins ties
                best = c;
                bw = x;
            }
        }
    }
#pragma unroll
    for (int o = WAVE / 2; o > 0; o >>= 1) {
        const float ob = __shfl_xor(best, o, WAVE);
        const int ow = __shfl_xor(bw, o, WAVE);
        if (ob < best || (ob == best && ow > bw)) {
            best = ob;
            bw = ow;
        }
    }
    if (lane == 0) {
        low_out[col] = bw >= 0 ? cofacet_index<P>(B, v, bw) : NONE;
        low_diam_out[col] = best;
    }
}

template <int P, int G>
static void launch_apparent_sparse_pg(const float *cd, const uint64_t *cc, int64_t ncols,
                                      int n, int words, const uint4 *nbw, const float *nbd,
                                      const uint64_t *binom, uint64_t *tau,
                                      unsigned long long *sc, hipStream_t s,
                                      const uint64_t *cv)
{
    // rounds per wave as in the dense kernel: as many as G allows while the
    // grid keeps ~4 waves per SIMD
    constexpr int cpr = WAVE / G;
    int rounds = 1;
    while (rounds < G && ncols / ((int64_t)cpr * rounds * 2) >= 4096)
        rounds *= 2;
    const int64_t waves = (ncols + (int64_t)cpr * rounds - 1) / ((int64_t)cpr * rounds);
    dim3 g((unsigned)((waves * WAVE + 255) / 256)), b(256);
    hipLaunchKernelGGL((k_apparent_sparse<P, G>), g, b, 0, s, cd, cc, ncols, n, words, nbw, nbd,
                       binom, tau, sc, rounds, cv);
}

template <int P, int K, int G>
static void launch_apparent_sparse2_pkg(const float *cd, const uint64_t *cc, int64_t ncols, int n,
                                        int words, const uint4 *nbw, const float *nbd,
                                        const uint64_t *binom, uint64_t *tau,
                                        unsigned long long *sc, hipStream_t s,
                                        const uint64_t *cv)
{
    const int64_t waves = (ncols + WAVE - 1) / WAVE;
    dim3 g((unsigned)((waves * WAVE + 255) / 256)), b(256);
    hipLaunchKernelGGL((k_apparent_sparse2<P, K, G>), g, b, 0, s, cd, cc, ncols, n, words, nbw,
                       nbd, binom, tau, sc, cv);
}

template <int P>
static void launch_apparent_sparse_p(const float *cd, const uint64_t *cc, int64_t ncols, int n,
                                     int words, const uint4 *nbw, const float *nbd,
                                     const uint64_t *binom, int group, uint64_t *tau,
                                     unsigned long long *sc, hipStream_t s, const uint64_t *cv)
{
#define RPP_AS2(K, G) launch_apparent_sparse2_pkg<P, K, G>(cd, cc, ncols, n, words, nbw, nbd, binom, tau, sc, s, cv)
    switch (group) {
    case 16: launch_apparent_sparse_pg<P, 16>(cd, cc, ncols, n, words, nbw, nbd, binom, tau, sc, s, cv); break;
    case 8: launch_apparent_sparse_pg<P, 8>(cd, cc, ncols, n, words, nbw, nbd, binom, tau, sc, s, cv); break;
    case 104: RPP_AS2(1, 4); break;
    case 108: RPP_AS2(1, 8); break;
    case 204: RPP_AS2(2, 4); break;
    case 208: RPP_AS2(2, 8); break;
    case 404: RPP_AS2(4, 4); break;
    case 408: RPP_AS2(4, 8); break;
    default: launch_apparent_sparse_pg<P, 4>(cd, cc, ncols, n, words, nbw, nbd, binom, tau, sc, s, cv); break;
    }
#undef RPP_AS2
}

// Sparse kernel forms: G in {4, 8, 16} lanes per column (k_apparent_sparse),
// or 100 K + G, K in {1, 2, 4}, G in {4, 8} (the two-phase
// k_apparent_sparse2); anything else means the default.
constexpr int SPARSE_DEFAULT = 404;
int sparse_group(int group)
{
    switch (group) {
    case 4: case 8: case 16:
    case 104: case 108: case 204: case 208: case 404: case 408:
        return group;
    default:
        return SPARSE_DEFAULT;
    }
}


void launch_apparent_sparse(const float *col_diam, const uint64_t *col_cidx, int64_t ncols,
                            int n, int p, int words, const uint4 *nbw, const float *nbd,
                            const uint64_t *binom, int group, uint64_t *tau_out,
                            unsigned long long *scan_count, hipStream_t s,
                            const uint64_t *col_vtx)
{
    if (ncols <= 0)
        return;
    group = sparse_group(group);
    if (p > 3 || n > 65536)
        col_vtx = nullptr;
#define RPP_APS(P) launch_apparent_sparse_p<P>(col_diam, col_cidx, ncols, n, words, nbw, nbd, binom, group, tau_out, scan_count, s, col_vtx)
    switch (p) {
    case 1: RPP_APS(1); break;
    case 2: RPP_APS(2); break;
    case 3: RPP_APS(3); break;
    default: RPP_APS(4); break;
    }
#undef RPP_APS
}

void launch_lows_sparse(const uint64_t *na_key, const uint64_t *na_cidx, int64_t ncols,
                        const uint4 *nbw, const float *nbd, int n, int p, int words,
                        const uint64_t *binom, uint64_t *low_out, float *low_diam_out,
                        hipStream_t s)
{
    if (ncols <= 0)
        return;
    dim3 g((unsigned)((ncols * WAVE + 255) / 256)), b(256);
#define RPP_LS(P) hipLaunchKernelGGL(k_lows_sparse<P>, g, b, 0, s, na_key, na_cidx, ncols, nbw, nbd, n, words, binom, low_out, low_diam_out)
    switch (p) {
    case 1: RPP_LS(1); break;
    case 2: RPP_LS(2); break;
    case 3: RPP_LS(3); break;
    default: RPP_LS(4); break;
    }
#undef RPP_LS
}

// ===========================================================================
// a7: clearing bitmap for the next dimension
// ===========================================================================
__global__ void k_mark_bits(const uint64_t *__restrict__ idx, int64_t count,
                            uint32_t *__restrict__ bits, Batch bt, int64_t bits_stride)
{
    const int64_t cl = blockIdx.y;
    count = batch_count(bt, cl, count);
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) {
        uint64_t t = idx[cl * bt.stride + i];
        atomicOr(&bits[cl * bits_stride + (int64_t)(t >> 5)], 1u << (t & 31));
    }
}

void launch_mark_bits(const uint64_t *idx, int64_t count, uint32_t *bits, hipStream_t s,
                      Batch bt, int nbatch, int64_t bits_stride)
{
    if (count <= 0)
        return;
    hipLaunchKernelGGL(k_mark_bits, dim3((unsigned)((count + 255) / 256), nbatch), dim3(256), 0,
                       s, idx, count, bits, bt, bits_stride);
}

// ===========================================================================
// a2: H0 -- Kruskal in one workgroup
//
// Edges are visited in filtration order in batches of one per thread.  A
// batch is settled in rounds: each unsettled thread finds the roots of its
// endpoints; equal roots settle it as a non-tree edge.  Every root claimed
// by several threads goes to the lowest thread (the oldest edge); a thread
// that owns both its roots merges them and settles as a tree edge.  Winners
// touch disjoint components that no older unsettled edge touches, so the
// outcome equals sequential Kruskal under the strict (diameter, cidx)
// order.
// ===========================================================================
constexpr int KT = 1024;

__device__ __forceinline__ int uf_find(volatile int *parent, int x)
{
    while (true) {
        int p = parent[x];
        if (p == x)
            return x;
        int gp = parent[p];
        if (gp != p)
            parent[x] = gp;  // path halving: gp is an ancestor of x
        x = gp;
    }
}

template <bool IN_LDS>
__global__ __launch_bounds__(KT) void k_kruskal(const uint64_t *__restrict__ edge_key,
                                                const uint64_t *__restrict__ edge_cidx,
                                                int64_t nedges, int n,
                                                uint32_t *__restrict__ mst_bits,
                                                float *__restrict__ deaths,
                                                uint64_t *__restrict__ death_edges,
                                                int *__restrict__ counters,
                                                int *__restrict__ uf_scratch, Batch bt,
                                                int64_t mst_stride)
{
    extern __shared__ int smem[];
    {   // batched launch: one workgroup per cloud
        const int64_t cl = blockIdx.x;
        nedges = batch_count(bt, cl, nedges);
        edge_key += cl * bt.stride;
        edge_cidx += cl * bt.stride;
        mst_bits += cl * mst_stride;
        deaths += cl * n;
        death_edges += cl * n;
        counters += 2 * cl;
        uf_scratch += 2 * (int64_t)n * cl;
    }
    volatile int *parent = IN_LDS ? smem : uf_scratch;
    int *owner = IN_LDS ? smem + n : uf_scratch + n;
    __shared__ int s_merges, s_deaths;
    const int tid = threadIdx.x;
    for (int v = tid; v < n; v += KT) {
        parent[v] = v;
        owner[v] = INT_MAX;
    }
    if (tid == 0) {
        s_merges = 0;
        s_deaths = 0;
    }
    __syncthreads();
    for (int64_t base = 0; base < nedges; base += KT) {
        if (s_merges >= batch_nv(bt, blockIdx.x, n) - 1)
            break;  // spanning tree complete: no later edge can merge
        const int64_t k = base + tid;
        bool active = k < nedges;
        int a = 0, b = 0;
        uint64_t c = 0;
        float dm = 0.0f;
        if (active) {
            const int64_t idx = nedges - 1 - k;  // oldest first
            c = edge_cidx[idx];
            dm = __uint_as_float(~(uint32_t)edge_key[idx]);
            decode_edge(c, a, b);
        }
        while (true) {
            int ra = 0, rb = 0;
            if (active) {
                ra = uf_find(parent, a);
                rb = uf_find(parent, b);
                if (ra == rb)
                    active = false;
            }
            if (!__syncthreads_or(active))
                break;
            if (active) {
                atomicMin(&owner[ra], tid);
                atomicMin(&owner[rb], tid);
            }
            __syncthreads();
            const bool win = active && owner[ra] == tid && owner[rb] == tid;
            __syncthreads();
            if (active) {
                owner[ra] = INT_MAX;
                owner[rb] = INT_MAX;
            }
            if (win) {
                parent[max(ra, rb)] = min(ra, rb);
                atomicOr(&mst_bits[c >> 5], 1u << (c & 31));
                if (dm > 0.0f) {
                    const int slot = atomicAdd(&s_deaths, 1);
                    deaths[slot] = dm;
                    death_edges[slot] = c;
                }
                atomicAdd(&s_merges, 1);
                active = false;
            }
            __syncthreads();
        }
        __syncthreads();
    }
    if (tid == 0) {
        counters[0] = s_deaths;
        counters[1] = s_merges;
    }
}

void launch_kruskal(const uint64_t *edge_key, const uint64_t *edge_cidx, int64_t nedges, int n,
                    uint32_t *mst_bits, float *deaths, uint64_t *death_edges, int *counters,
                    int *uf_scratch, hipStream_t s, Batch bt, int nbatch, int64_t mst_stride)
{
    const size_t lds = (size_t)2 * n * sizeof(int);
    if (lds <= 60 * 1024) {
        hipLaunchKernelGGL(k_kruskal<true>, dim3(nbatch), dim3(KT), lds, s, edge_key, edge_cidx,
                           nedges, n, mst_bits, deaths, death_edges, counters, uf_scratch, bt,
                           mst_stride);
    } else {
        hipLaunchKernelGGL(k_kruskal<false>, dim3(nbatch), dim3(KT), 0, s, edge_key, edge_cidx,
                           nedges, n, mst_bits, deaths, death_edges, counters, uf_scratch, bt,
                           mst_stride);
    }
}

// ===========================================================================
// distances from coordinates, and the critical-edge gradient
// ===========================================================================
__global__ void k_pdist(const float *__restrict__ pts, int n, int d, float *__restrict__ dist)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)n * (n - 1) / 2)
        return;
    int a, b;
    decode_edge((uint64_t)e, a, b);
    double acc = 0.0;
    for (int k = 0; k < d; ++k) {
        const double df = __dsub_rn((double)pts[(int64_t)a * d + k], (double)pts[(int64_t)b * d + k]);
        acc = __dadd_rn(acc, __dmul_rn(df, df));
    }
    dist[e] = __double2float_rn(__dsqrt_rn(acc));
}

void launch_pdist(const float *pts, int n, int d, float *dist, hipStream_t s)
{
    const int64_t m = (int64_t)n * (n - 1) / 2;
    if (m <= 0)
        return;
    hipLaunchKernelGGL(k_pdist, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, pts, n, d,
                       dist);
}

__global__ void k_edge_grad(const float *__restrict__ pts, int n, int d,
                            const uint64_t *__restrict__ edges, const float *__restrict__ g,
                            int64_t nterms, float *__restrict__ grad)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)n * d)
        return;
    const int u = (int)(t / d), k = (int)(t % d);
    double acc = 0.0;
    for (int64_t i = 0; i < nterms; ++i)
        edge_grad_add(acc, pts, d, u, k, edges[i], g[i]);
    grad[t] = (float)acc;
}

void launch_edge_grad(const float *pts, int n, int d, const uint64_t *edges, const float *g,
                      int64_t nterms, float *grad, hipStream_t s)
{
    const int64_t m = (int64_t)n * d;
    if (m <= 0)
        return;
    hipLaunchKernelGGL(k_edge_grad, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, pts, n,
                       d, edges, g, nterms, grad);
}

// ===========================================================================
// a6: stable LSD radix sort, 8-bit digits
//
// Per pass: (1) per-tile digit histograms (LDS atomics), laid out
// digit-major so that (2) one exclusive scan yields every tile's global
// offset per digit; (3) each tile ranks its keys stably -- rounds of 256
// keys in index order, ranks within a wave from 8 ballots (lanes with the
// same digit), across waves from LDS counters -- stages the tile in LDS in
// digit order and writes it out in runs.
// ===========================================================================
constexpr int RT = 256;
constexpr int RI = 8;
constexpr int RTILE = RT * RI;
constexpr int RBINS = 256;

int64_t radix_scratch_words(int64_t count, int nbatch)
{
    int64_t tiles = (count + RTILE - 1) / RTILE;
    int64_t hist_words = (nbatch * tiles * RBINS + 1) / 2 + 1;   // u32 histograms
    int64_t off_words = nbatch * (tiles * RBINS + 1);            // u64 offsets
    return hist_words + off_words + nbatch * scan_scratch_words(tiles * RBINS) + 8;
}

__global__ __launch_bounds__(RT) void k_rs_hist(const uint64_t *__restrict__ keys, int64_t count,
                                                int shift, uint32_t *__restrict__ hist,
                                                int64_t tiles, Batch bt)
{
    __shared__ uint32_t h[RBINS];
    {
        const int64_t cl = blockIdx.y;
        count = batch_count(bt, cl, count);
        keys += cl * bt.stride;
        hist += cl * tiles * RBINS;
    }
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * RTILE;
#pragma unroll
    for (int k = 0; k < RI; ++k) {
        int64_t i = base + (int64_t)k * RT + threadIdx.x;
        if (i < count)
            atomicAdd(&h[(keys[i] >> shift) & (RBINS - 1)], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * tiles + blockIdx.x] = h[threadIdx.x];
}

__global__ __launch_bounds__(RT) void k_rs_scatter(const uint64_t *__restrict__ kin,
                                                   const uint64_t *__restrict__ vin,
                                                   uint64_t *__restrict__ kout,
                                                   uint64_t *__restrict__ vout, int64_t count,
                                                   int shift,
                                                   const uint64_t *__restrict__ offs,
                                                   int64_t tiles, Batch bt)
{
    __shared__ uint64_t sk[RTILE];
    {
        const int64_t cl = blockIdx.y, st = bt.stride;
        count = batch_count(bt, cl, count);
        kin += cl * st;
        vin += cl * st;
        kout += cl * st;
        vout += cl * st;
        offs += cl * (tiles * RBINS + 1);
    }
    if ((int64_t)blockIdx.x * RTILE >= count)
        return;  // no keys of this cloud in this tile (uniform per block)
    __shared__ uint64_t sv[RTILE];
    __shared__ uint32_t wcnt[RT / WAVE][RBINS];
    __shared__ uint32_t run[RBINS];
    __shared__ uint32_t loff[RBINS];
    __shared__ uint32_t scan_sh[RT / WAVE + 1];

    const int tid = threadIdx.x, lane = tid & (WAVE - 1), wave = tid / WAVE;
    const int64_t base = (int64_t)blockIdx.x * RTILE;
    run[tid] = 0;
#pragma unroll
    for (int w = 0; w < RT / WAVE; ++w)
        wcnt[w][tid] = 0;
    __syncthreads();

    uint64_t key[RI], val[RI];
    uint32_t rank[RI];
    int dig[RI];
#pragma unroll
    for (int k = 0; k < RI; ++k) {
        const int64_t i = base + (int64_t)k * RT + tid;
        const bool valid = i < count;
        key[k] = valid ? kin[i] : 0;
        val[k] = valid ? vin[i] : 0;
        const int d = valid ? (int)((key[k] >> shift) & (RBINS - 1)) : -1;
        dig[k] = d;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
            const bool set = valid && ((d >> bit) & 1);
            const uint64_t bb = __ballot(set);
            peers &= set ? bb : ~bb;
        }
        const uint64_t below = peers & lanemask_lt();
        if (valid && below == 0)
            wcnt[wave][d] = (uint32_t)__popcll(peers);
        __syncthreads();
        if (valid) {
            uint32_t pre = run[d];
            for (int w = 0; w < wave; ++w)
                pre += wcnt[w][d];
            rank[k] = pre + (uint32_t)__popcll(below);
        }
        __syncthreads();
        uint32_t tot = 0;
#pragma unroll
        for (int w = 0; w < RT / WAVE; ++w) {
            tot += wcnt[w][tid];
            wcnt[w][tid] = 0;
        }
        run[tid] += tot;
        __syncthreads();
    }
    uint32_t total;
    const uint32_t ex = block_exclusive_scan<RT>(run[tid], &total, scan_sh);
    loff[tid] = ex;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < RI; ++k) {
        if (dig[k] >= 0) {
            const uint32_t pos = loff[dig[k]] + rank[k];
            sk[pos] = key[k];
            sv[pos] = val[k];
        }
    }
    __syncthreads();
    const int64_t cnt = (count - base < RTILE) ? (count - base) : RTILE;
#pragma unroll
    for (int k = 0; k < RI; ++k) {
        const int j = k * RT + tid;
        if (j < cnt) {
            const uint64_t kk = sk[j];
            const int d = (int)((kk >> shift) & (RBINS - 1));
            const uint64_t g = offs[(int64_t)d * tiles + blockIdx.x] + (uint64_t)(j - loff[d]);
            kout[g] = kk;
            vout[g] = sv[j];
        }
    }
}

int radix_sort_pairs_b(uint64_t *keys, uint64_t *vals, uint64_t *keys_alt, uint64_t *vals_alt,
                       int64_t count, int bits, uint64_t *scratch, hipStream_t s, Batch bt,
                       int nbatch)
{
    if (count <= 1 && !bt.count)
        return 0;
    if (count <= 0 || bits <= 0)
        return 0;
    const int64_t tiles = (count + RTILE - 1) / RTILE;
    const int64_t per = radix_scratch_words(count);
    // per-cloud scratch regions: [hist | offsets | scan scratch]
    uint32_t *hist = reinterpret_cast<uint32_t *>(scratch);
    const int64_t hist_words = (nbatch * tiles * RBINS + 1) / 2 + 1;
    uint64_t *offs = scratch + hist_words;
    uint64_t *scan_tmp = offs + nbatch * (tiles * RBINS + 1);
    (void)per;
    uint64_t *ki = keys, *vi = vals, *ko = keys_alt, *vo = vals_alt;
    int where = 0;
    for (int shift = 0; shift < bits; shift += 8) {
        hipLaunchKernelGGL(k_rs_hist, dim3((unsigned)tiles, nbatch), dim3(RT), 0, s, ki, count,
                           shift, hist, tiles, bt);
        launch_exclusive_scan_b(hist, tiles * RBINS, nbatch, offs, scan_tmp, s);
        hipLaunchKernelGGL(k_rs_scatter, dim3((unsigned)tiles, nbatch), dim3(RT), 0, s, ki, vi,
                           ko, vo, count, shift, offs, tiles, bt);
        uint64_t *t = ki;
        ki = ko;
        ko = t;
        t = vi;
        vi = vo;
        vo = t;
        where ^= 1;
    }
    return where;
}

// Small sorts in one launch: one workgroup sorts fewer than 8192 pairs by
// the low `bits` (<= 51) bits of the key, stably -- a bitonic network over
// (key bits << 13 | index), whose distinct values make it stable, then
// whole keys and values gathered by index.  A radix sort of a few thousand
// keys would spend its time in ~20 launches.
constexpr int SS_N = 8192;
constexpr int SS_T = 1024;

__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t x, int mask)
{
    const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)x, mask, WAVE);
    const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(x >> 32), mask, WAVE);
    return ((uint64_t)hi << 32) | lo;
}

// Thread t holds elements t + SS_T r, r < R, in registers.  Partners closer
// than 64 (j < 64) sit in the same wave at lane t ^ j with the same r, so
// those stages are register compare-exchanges across a shuffle; only the
// wider stages go through LDS, one barrier each.
// R = elements per thread = max(1, m / SS_T), m = count rounded up to a
// power of two.
template <int R>
__global__ __launch_bounds__(SS_T) void k_small_sort(const uint64_t *__restrict__ kin,
                                                     const uint64_t *__restrict__ vin,
                                                     uint64_t *__restrict__ kout,
                                                     uint64_t *__restrict__ vout, int count,
                                                     int bits)
{
    __shared__ uint64_t a[SS_N];
    int m = 2;
    while (m < count)
        m <<= 1;
    const int t = threadIdx.x;
    const bool act = t < m;
    const uint64_t mask = (1ull << bits) - 1;
    // padding sorts last: a real composite is below ~0 (index <= 8190)
    uint64_t x[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int i = t + SS_T * r;
        x[r] = (act && i < count) ? (((kin[i] & mask) << 13) | (uint64_t)i) : ~0ull;
    }
    for (int k = 2; k <= m; k <<= 1) {
        int j = k >> 1;
        if (j >= WAVE) {
#pragma unroll
            for (int r = 0; r < R; ++r)
                if (act)
                    a[t + SS_T * r] = x[r];
            __syncthreads();
            for (; j >= WAVE; j >>= 1) {
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int i = t + SS_T * r;
                    const int l = i ^ j;
                    if (act && l > i) {
                        const uint64_t p = a[i], q = a[l];
                        const bool up = (i & k) == 0;
                        if ((p > q) == up) {
                            a[i] = q;
                            a[l] = p;
                        }
                    }
                }
                __syncthreads();
            }
#pragma unroll
            for (int r = 0; r < R; ++r)
                if (act)
                    x[r] = a[t + SS_T * r];
            __syncthreads();  // every read done before the next stores
        }
        for (; j > 0; j >>= 1) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int i = t + SS_T * r;
                const uint64_t y = shfl_xor_u64(x[r], j);  // element i ^ j
                const bool up = (i & k) == 0, lower = (i & j) == 0;
                const bool keep_min = lower == up;
                const uint64_t lo = x[r] < y ? x[r] : y, hi = x[r] < y ? y : x[r];
                if (act)
                    x[r] = keep_min ? lo : hi;
            }
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r)
        if (act)
            a[t + SS_T * r] = x[r];
    __syncthreads();
    for (int i = t; i < count; i += SS_T) {
        const int src = (int)(a[i] & 0x1fffull);
        kout[i] = kin[src];
        vout[i] = vin[src];
    }
}

int radix_sort_pairs(uint64_t *keys, uint64_t *vals, uint64_t *keys_alt, uint64_t *vals_alt,
                     int64_t count, int bits, uint64_t *scratch, hipStream_t s)
{
    if (count <= 1 || bits <= 0)
        return 0;
    if (count < SS_N && bits <= 51) {
        int m = 2;
        while (m < count)
            m <<= 1;
        const int r = m >= SS_T ? (int)(m / SS_T) : 1;
        switch (r) {
        case 1: hipLaunchKernelGGL(k_small_sort<1>, dim3(1), dim3(SS_T), 0, s, keys, vals, keys_alt, vals_alt, (int)count, bits); break;
        case 2: hipLaunchKernelGGL(k_small_sort<2>, dim3(1), dim3(SS_T), 0, s, keys, vals, keys_alt, vals_alt, (int)count, bits); break;
        case 4: hipLaunchKernelGGL(k_small_sort<4>, dim3(1), dim3(SS_T), 0, s, keys, vals, keys_alt, vals_alt, (int)count, bits); break;
        default: hipLaunchKernelGGL(k_small_sort<8>, dim3(1), dim3(SS_T), 0, s, keys, vals, keys_alt, vals_alt, (int)count, bits); break;
        }
        return 1;
    }
    return radix_sort_pairs_b(keys, vals, keys_alt, vals_alt, count, bits, scratch, s, Batch(), 1);
}

}  // namespace rpp
