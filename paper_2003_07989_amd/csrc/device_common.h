// device_common.h -- index arithmetic shared by the gfx950 kernels.
//
// Simplices are named by their combinatorial index (paper, section on the
// combinatorial number system): vertices v_p > ... > v_0 map to
// cidx = C(v_p, p+1) + ... + C(v_0, 1).  Ordering simplices by cidx is the
// colexicographic order on increasing vertex tuples.
//
// Binomial coefficients come from a table binom[k * stride + v] = C(v, k),
// k = 0..kmax, v = 0..n, built once per point count on the host (paper:
// cofacets are generated from the distance matrix and a small binomial
// coefficient table).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rpp {

constexpr uint64_t NONE = ~0ull;
constexpr int WAVE = 64;

struct Binom {
    const uint64_t *__restrict__ t;
    int stride;  // n + 1
    __device__ __forceinline__ uint64_t operator()(int v, int k) const
    {
        return t[(int64_t)k * stride + v];
    }
};

// Largest v in [k-1, hi) with C(v, k) <= c.  C(k-1, k) = 0 <= c always.
// For k <= 4 a closed-form root of C(v, k) = c gives a guess within a step
// or two of the answer (C(v,2) ~ v(v-1)/2, C(v,3) ~ (v-1)^3/6,
// C(v,4) ~ (v-1.5)^4/24); table comparisons then step to the exact value,
// so a decode costs a couple of independent loads instead of a dependent
// binary search.  Larger k use the binary search.
__device__ __forceinline__ int top_vertex(const Binom &B, uint64_t c, int k, int hi)
{
    if (k == 1)
        return (int)c;
    if (k <= 4) {
        // Guess from C(x, k) ~ x^k / k!, in single precision with the
        // hardware square root, log2 and exp2: a guess a few units off only
        // costs a step of the exact correction below.
        const float cf = (float)c;
        float g;
        if (k == 2)
            g = 0.5f * (1.0f + __builtin_sqrtf(1.0f + 8.0f * cf));
        else if (k == 3)
            g = __builtin_amdgcn_exp2f(__builtin_amdgcn_logf(6.0f * cf) * (1.0f / 3.0f)) + 1.0f;
        else
            g = __builtin_sqrtf(__builtin_sqrtf(24.0f * cf)) + 1.5f;
        int x = (int)fminf(g, (float)(hi - 1));
        x = x < k - 1 ? k - 1 : x;
        while (x > k - 1 && B(x, k) > c)
            --x;
        while (x + 1 < hi && B(x + 1, k) <= c)
            ++x;
        return x;
    }
    int lo = k - 1, h = hi - 1;
    while (lo < h) {
        int mid = (lo + h + 1) >> 1;
        if (B(mid, k) <= c)
            lo = mid;
        else
            h = mid - 1;
    }
    return lo;
}

// Vertices of a p-simplex in decreasing order: v[0] > v[1] > ... > v[P].
template <int P>
__device__ __forceinline__ void decode(const Binom &B, uint64_t c, int n, int (&v)[P + 1])
{
    int hi = n;
#pragma unroll
    for (int pos = 0; pos <= P; ++pos) {
        const int k = P + 1 - pos;
        int x = top_vertex(B, c, k, hi);
        v[pos] = x;
        c -= B(x, k);
        hi = x;
    }
}

// Edge (a > b) from its index c = C(a,2) + b, without the table.
__device__ __forceinline__ void decode_edge(uint64_t c, int &a, int &b)
{
    int x = (int)(0.5f * (1.0f + __builtin_sqrtf(1.0f + 8.0f * (float)c)));
    while ((uint64_t)x * (x - 1) / 2 > c)
        --x;
    while ((uint64_t)(x + 1) * x / 2 <= c)
        ++x;
    a = x;
    b = (int)(c - (uint64_t)x * (x - 1) / 2);
}

// One gradient term of the backward pass: an edge e of length |x_a - x_b|
// with dL/dlength = gval adds gval * (x_u[k] - x_o[k]) / |x_u - x_o| to
// coordinate k of its endpoint u (o the other endpoint), accumulated in FP64.
// Edges not touching u, the "no edge" index and zero-length edges add
// nothing.
__device__ __forceinline__ void edge_grad_add(double &acc, const float *__restrict__ pts, int d,
                                              int u, int k, uint64_t e, float gval)
{
    if (e == NONE)
        return;
    int a, b;
    decode_edge(e, a, b);
    if (a != u && b != u)
        return;
    const int o = (a == u) ? b : a;
    double len2 = 0.0;
    for (int q = 0; q < d; ++q) {
        const double df = (double)pts[(int64_t)u * d + q] - (double)pts[(int64_t)o * d + q];
        len2 += df * df;
    }
    if (len2 > 0.0)
        acc += (double)gval * ((double)pts[(int64_t)u * d + k] - (double)pts[(int64_t)o * d + k]) /
               sqrt(len2);
}

// cidx of sigma + {w} where sigma = v[0] > ... > v[P] and w is not in sigma:
// with j = #{i : v_i < w}, cidx = sum_{v_i < w} C(v_i, rank+1) + C(w, j+1)
// + sum_{v_i > w} C(v_i, rank+2) (ranks counted from the bottom).
template <int P>
__device__ __forceinline__ uint64_t cofacet_index(const Binom &B, const int (&v)[P + 1], int w)
{
    uint64_t c = 0;
    int r = 0;
    bool placed = false;
#pragma unroll
    for (int i = P; i >= 0; --i) {
        if (!placed && w < v[i]) {
            c += B(w, r + 1);
            ++r;
            placed = true;
        }
        c += B(v[i], r + 1);
        ++r;
    }
    if (!placed)
        c += B(w, r + 1);
    return c;
}

// Distance through the square matrix (row-major, n x n, zero diagonal).
__device__ __forceinline__ float dsq_at(const float *__restrict__ dsq, int n, int a, int b)
{
    return dsq[(int64_t)a * n + b];
}

// Bit pattern of a non-negative float, -0.0 folded to +0.0: monotone in the
// value, so unsigned comparison of the patterns orders the diameters.
__device__ __forceinline__ uint32_t diam_bits(float d)
{
    return __float_as_uint(d + 0.0f);
}

// Workgroups are dispatched to the chip's 8 XCDs round-robin, and each XCD
// has its own L2.  Renumbering block b of nb so that every XCD gets one
// contiguous range of the logical grid keeps neighbouring tiles -- which
// read the same distance rows -- in one L2.  A bijection on [0, nb): XCD x
// gets q + 1 blocks when x < r, q otherwise (nb = 8q + r).
__device__ __forceinline__ uint32_t xcd_block(uint32_t b, uint32_t nb)
{
    constexpr uint32_t X = 8;
    const uint32_t q = nb / X, r = nb % X;
    const uint32_t x = b % X, i = b / X;
    return x < r ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

__device__ __forceinline__ uint64_t lanemask_lt()
{
    const int lane = threadIdx.x & (WAVE - 1);
    return (lane == 0) ? 0ull : (~0ull >> (WAVE - lane));
}

}  // namespace rpp
