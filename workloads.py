"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module only *draws* inputs.  It holds none of the persistence method's
arithmetic: it produces point clouds and the FP32 distance matrices computed
from them, in the layout both the HIP library and the oracle accept.

Layout of a distance matrix handed to either side: the condensed lower
triangle in edge combinatorial-index order, ``D[i*(i-1)/2 + j] = d(i, j)`` for
``i > j`` (the lower-triangular input form the paper's experiments use, and
exactly the CNS order of edges, ``cidx(i, j) = C(i, 2) + j``).

Bit-reproducibility across machines.  Stored expected values are produced on
one machine and checked on another, so every floating-point step here uses
only IEEE-754 basic operations (``+ - * / sqrt``), which are correctly rounded
everywhere.  Library transcendental functions (numpy's ``sin``/``cos``/``log``)
may dispatch to CPU-specific vector code that differs in the last bit, so the
few transcendental values needed (sine, cosine, logarithm, exponential) are
computed by the short polynomial routines below, evaluated in a fixed order.
Random numbers come from numpy's PCG64, whose integer stream and
``random()`` doubles are platform independent.  Coordinates and distances are
computed in FP64 and rounded once to FP32 (round-to-nearest-even).
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "condensed_from_points",
    "square_from_condensed",
    "uniform_square_points",
    "noisy_torus_points",
    "noisy_sphere_points",
    "noisy_circle_points",
    "mixture_request",
    "serving_stream",
    "unit_square_example",
    "cycle_graph_metric",
    "all_equal_metric",
    "reverse_lex_metric",
    "random_permutation_metric",
    "greedy_assignment_order",
    "greedy_assignment_metric",
    "random_integer_metric",
    "duplicate_points_cloud",
    "signed_zero_metric",
    "collinear_integer_metric",
    "WORKLOADS",
]

# --------------------------------------------------------------------------
# Deterministic elementary functions (basic IEEE operations only)
# --------------------------------------------------------------------------
_PI = 3.141592653589793
_TWO_PI = 6.283185307179586
# pi/2 split so that k*_PIO2_HI is exact for the small k used here
_PIO2_HI = 1.5707963267341256
_PIO2_LO = 6.077100506506192e-11
_LN2_HI = 0.6931471803691238
_LN2_LO = 1.9082149292705877e-10


def _poly(x, coeffs):
    """Horner evaluation, highest coefficient first, fixed order."""
    acc = np.full_like(x, coeffs[0])
    for c in coeffs[1:]:
        acc = acc * x + c
    return acc


# Taylor coefficients of sin(r)/r and cos(r) in r^2, highest first.
_SIN_C = [
    -1.0 / 1307674368000.0,   # -r^14/15!
    1.0 / 6227020800.0,       #  r^12/13!
    -1.0 / 39916800.0,        # -r^10/11!
    1.0 / 362880.0,           #  r^8/9!
    -1.0 / 5040.0,            # -r^6/7!
    1.0 / 120.0,              #  r^4/5!
    -1.0 / 6.0,               # -r^2/3!
    1.0,
]
_COS_C = [
    1.0 / 20922789888000.0,   #  r^16/16!
    -1.0 / 87178291200.0,     # -r^14/14!
    1.0 / 479001600.0,        #  r^12/12!
    -1.0 / 3628800.0,         # -r^10/10!
    1.0 / 40320.0,            #  r^8/8!
    -1.0 / 720.0,             # -r^6/6!
    1.0 / 24.0,               #  r^4/4!
    -0.5,                     # -r^2/2!
    1.0,
]


def det_sincos(x):
    """(sin x, cos x) for float64 arrays with |x| < 1e6, error ~1e-16.

    Method: Cody-Waite argument reduction by pi/2 with a two-part constant
    (x - k*hi - k*lo, exact for the small k used here), then the Taylor
    polynomials of sin and cos on |r| <= pi/4 and the quadrant swap."""
    x = np.asarray(x, dtype=np.float64)
    k = np.floor(x / _PIO2_HI + 0.5)
    r = (x - k * _PIO2_HI) - k * _PIO2_LO          # |r| <= pi/4 (+tiny)
    r2 = r * r
    s = r * _poly(r2, _SIN_C)
    c = _poly(r2, _COS_C)
    q = np.mod(k, 4.0)
    sin_x = np.where(q == 0, s, np.where(q == 1, c, np.where(q == 2, -s, -c)))
    cos_x = np.where(q == 0, c, np.where(q == 1, -s, np.where(q == 2, -c, s)))
    return sin_x, cos_x


def det_log(u):
    """Natural logarithm of positive float64 arrays, error ~1e-16.

    Method: u = m * 2^e with m in [sqrt(1/2), sqrt(2)); ln m = 2 atanh(s),
    s = (m - 1)/(m + 1), by its odd power series; e * ln 2 is added with a
    two-part (Cody-Waite) constant."""
    u = np.asarray(u, dtype=np.float64)
    m, e = np.frexp(u)                      # u = m * 2^e, m in [0.5, 1)
    e = e.astype(np.float64)
    small = m < 0.7071067811865476
    m = np.where(small, m * 2.0, m)
    e = np.where(small, e - 1.0, e)
    s = (m - 1.0) / (m + 1.0)                # |s| <= 0.1716
    s2 = s * s
    # 2*atanh(s) = 2*(s + s^3/3 + s^5/5 + ...), 12 terms
    coeffs = [1.0 / (2 * k + 1) for k in range(11, -1, -1)]
    lnm = 2.0 * s * _poly(s2, coeffs)
    return (e * _LN2_HI + lnm) + e * _LN2_LO


def det_exp(x):
    """exp of float64 arrays with |x| < 700, error ~1e-15 relative.

    Method: x = k ln 2 + r with a two-part (Cody-Waite) ln 2, |r| <= ln2/2;
    the Taylor polynomial of exp(r), scaled by 2^k."""
    x = np.asarray(x, dtype=np.float64)
    k = np.floor(x / (_LN2_HI + _LN2_LO) + 0.5)
    r = (x - k * _LN2_HI) - k * _LN2_LO     # |r| <= ln2/2
    coeffs = [1.0 / float(np.prod(np.arange(1, j + 1))) for j in range(17, -1, -1)]
    return np.ldexp(_poly(r, coeffs), k.astype(np.int64))


def det_normal(rng: np.random.Generator, size) -> np.ndarray:
    """Standard normals by the Box-Muller transform on PCG64 uniforms."""
    size = int(np.prod(size)) if not np.isscalar(size) else int(size)
    half = (size + 1) // 2
    u1 = 1.0 - rng.random(half)              # (0, 1]
    u2 = rng.random(half)
    rad = np.sqrt(-2.0 * det_log(u1))
    s, c = det_sincos(_TWO_PI * u2)
    z = np.empty(2 * half, dtype=np.float64)
    z[0::2] = rad * c
    z[1::2] = rad * s
    return z[:size]


# --------------------------------------------------------------------------
# Distance matrices
# --------------------------------------------------------------------------
def condensed_from_points(x: np.ndarray) -> np.ndarray:
    """FP32 condensed lower triangle of Euclidean distances.

    ``x`` is (n, d); it is promoted to float64, squared differences are summed
    coordinate by coordinate in a fixed order, the square root is taken in
    float64, and the result is rounded once to float32.
    """
    x = np.ascontiguousarray(x, dtype=np.float64)
    n = x.shape[0]
    out = np.empty(n * (n - 1) // 2, dtype=np.float32)
    for i in range(1, n):
        diff = x[:i] - x[i]
        acc = diff[:, 0] * diff[:, 0]
        for k in range(1, x.shape[1]):
            acc = acc + diff[:, k] * diff[:, k]
        out[i * (i - 1) // 2: i * (i - 1) // 2 + i] = np.sqrt(acc).astype(np.float32)
    return out


def square_from_condensed(dc: np.ndarray, n: int) -> np.ndarray:
    """Symmetric n x n float32 matrix with a +0 diagonal."""
    sq = np.zeros((n, n), dtype=np.float32)
    if n > 1:
        ii, jj = np.tril_indices(n, -1)
        # np.tril_indices enumerates row-major (i ascending, j ascending),
        # which is exactly condensed (edge cidx) order.
        sq[ii, jj] = dc
        sq[jj, ii] = dc
    return sq


# --------------------------------------------------------------------------
# Point clouds shaped like the paper's workloads
# --------------------------------------------------------------------------
def uniform_square_points(n: int = 32, seed: int = 1001) -> np.ndarray:
    """n points i.i.d. uniform in [0,1]^2."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.random((n, 2))


def noisy_torus_points(n: int = 400, seed: int = 1002, R: float = 2.0,
                       r: float = 1.0, sigma: float = 0.05) -> np.ndarray:
    """Torus in R^3 (major radius R, minor radius r), both angles uniform in
    [0, 2pi) (not area-uniform), plus i.i.d. N(0, sigma^2 I_3) noise."""
    rng = np.random.Generator(np.random.PCG64(seed))
    theta = _TWO_PI * rng.random(n)
    phi = _TWO_PI * rng.random(n)
    st, ct = det_sincos(theta)
    sp, cp = det_sincos(phi)
    ring = R + r * ct
    x = np.stack([ring * cp, ring * sp, r * st], axis=1)
    return x + sigma * det_normal(rng, (n, 3)).reshape(n, 3)


def noisy_sphere_points(n: int = 4096, seed: int = 1003,
                        sigma: float = 0.01) -> np.ndarray:
    """Uniform on the unit sphere S^2 (normalised Gaussians) plus
    i.i.d. N(0, sigma^2 I_3) noise."""
    rng = np.random.Generator(np.random.PCG64(seed))
    g = det_normal(rng, (n, 3)).reshape(n, 3)
    nrm = np.sqrt((g[:, 0] * g[:, 0] + g[:, 1] * g[:, 1]) + g[:, 2] * g[:, 2])
    x = g / nrm[:, None]
    return x + sigma * det_normal(rng, (n, 3)).reshape(n, 3)


def noisy_circle_points(n: int = 512, seed: int = 0,
                        sigma: float = 0.1) -> np.ndarray:
    """Unit circle in the xy-plane of R^3, angle uniform, plus
    N(0, sigma^2 I_3) noise; returned as FP32 coordinates."""
    rng = np.random.Generator(np.random.PCG64(seed))
    theta = _TWO_PI * rng.random(n)
    s, c = det_sincos(theta)
    x = np.stack([c, s, np.zeros(n)], axis=1)
    x = x + sigma * det_normal(rng, (n, 3)).reshape(n, 3)
    return x.astype(np.float32)


def noisy_circle_batch(count: int = 64, n: int = 512, seed: int = 1005):
    """``count`` noisy circles of ``n`` points each (FP32 coordinates) and
    their condensed FP32 distance matrices (computed from the FP32
    coordinates in FP64)."""
    pts = [noisy_circle_points(n, seed=seed * 1000 + i) for i in range(count)]
    dists = [condensed_from_points(p) for p in pts]
    return pts, dists


def mixture_request(i: int, base_seed: int = 1004) -> dict:
    """One serving request: a Gaussian-mixture point cloud.

    n is log-uniform in [64, 1024]; ambient dimension d uniform in {2..8};
    K uniform in {3..8} equally weighted isotropic components with centres
    uniform in [0,1]^d and per-component standard deviation uniform in
    [0.02, 0.1]; maxdim uniform in {1, 2}; the threshold is the enclosing
    radius of the request's own distance matrix (passed as +inf, which the
    library replaces by that radius)."""
    rng = np.random.Generator(np.random.PCG64([base_seed, i]))
    lo, hi = det_log(np.array([64.0]))[0], det_log(np.array([1024.0]))[0]
    n = int(np.floor(det_exp(np.array([lo + (hi - lo) * rng.random()]))[0] + 0.5))
    n = min(max(n, 64), 1024)
    d = int(rng.integers(2, 9))
    K = int(rng.integers(3, 9))
    centres = rng.random((K, d))
    sig = 0.02 + 0.08 * rng.random(K)
    comp = rng.integers(0, K, size=n)
    z = det_normal(rng, (n, d)).reshape(n, d)
    x = centres[comp] + sig[comp][:, None] * z
    maxdim = int(rng.integers(1, 3))
    return {"n": n, "d": d, "K": K, "maxdim": maxdim, "points": x,
            "dist": condensed_from_points(x), "threshold": float("inf")}


def serving_stream(count: int = 512, rate_per_s: float = 100.0,
                   base_seed: int = 1004) -> list:
    """``count`` requests with Poisson arrivals at ``rate_per_s``."""
    rng = np.random.Generator(np.random.PCG64([base_seed, 1 << 20]))
    gaps = -det_log(1.0 - rng.random(count)) / rate_per_s
    arrivals = np.cumsum(gaps)
    out = []
    for i in range(count):
        req = mixture_request(i, base_seed)
        req["arrival_s"] = float(arrivals[i])
        out.append(req)
    return out


# --------------------------------------------------------------------------
# Small exact constructions (worked examples and closed cases)
# --------------------------------------------------------------------------
def unit_square_example() -> np.ndarray:
    """The four corners of the unit square (the paper's introductory
    example): sides 1, diagonals sqrt(2) rounded to FP32."""
    x = np.array([[0.0, 0.0], [1.0, 0.0], [1.0, 1.0], [0.0, 1.0]])
    return condensed_from_points(x)


def cycle_graph_metric(n: int) -> np.ndarray:
    """Integer shortest-path metric of the cycle graph C_n, exact in FP32."""
    out = np.empty(n * (n - 1) // 2, dtype=np.float32)
    k = 0
    for i in range(1, n):
        for j in range(i):
            g = i - j
            out[k] = float(min(g, n - g))
            k += 1
    return out


def all_equal_metric(n: int, value: float = 1.0) -> np.ndarray:
    return np.full(n * (n - 1) // 2, value, dtype=np.float32)


def reverse_lex_metric(n: int) -> np.ndarray:
    """Edge with combinatorial index i gets distance N - i (N = C(n,2)):
    distances strictly decrease along edge-index order."""
    N = n * (n - 1) // 2
    return (N - np.arange(N, dtype=np.float64)).astype(np.float32)


def random_permutation_metric(n: int, seed: int) -> np.ndarray:
    """A uniformly random permutation of the ranks 1..C(n,2) placed in the
    lower triangle, encoded as distinct FP32 values that preserve the order
    (bit pattern 0x3F800000 + rank: every such float is exact, so ties
    cannot arise from rounding)."""
    N = n * (n - 1) // 2
    rng = np.random.Generator(np.random.PCG64(seed))
    ranks = rng.permutation(N).astype(np.uint32) + np.uint32(1)
    return (np.uint32(0x3F800000) + ranks).view(np.float32)


def greedy_assignment_order(n: int):
    """The paper's greedy deterministic distance assignment on the full
    2-skeleton of n points (its random apparent-pair construction with the
    edge choice made greedy): while triangles remain, take the edge with
    the most remaining triangles (ties: the larger cidx), give it the next
    smaller diameter, and remove every triangle that contains it.  Edges
    left when no triangle remains get the smallest diameters, in decreasing
    cidx order.  Returns (edges in decreasing-diameter order, number of
    picks made while triangles remained)."""
    import heapq
    E = n * (n - 1) // 2
    ends = [(a, b) for a in range(n) for b in range(a)]   # cidx order

    def edge(a, b):
        return a * (a - 1) // 2 + b

    def tri(a, b, c):
        return a * (a - 1) * (a - 2) // 6 + b * (b - 1) // 2 + c

    alive = np.ones(max(n * (n - 1) * (n - 2) // 6, 1), dtype=bool)
    remaining = n * (n - 1) * (n - 2) // 6
    count = [n - 2] * E
    picked = [False] * E
    heap = [(-(n - 2), -e) for e in range(E)]
    heapq.heapify(heap)
    order = []
    while remaining > 0:
        c, ne = heapq.heappop(heap)
        e = -ne
        if picked[e] or -c != count[e]:
            continue  # stale entry
        picked[e] = True
        order.append(e)
        a, b = ends[e]
        for w in range(n):
            if w == a or w == b:
                continue
            x = sorted((a, b, w), reverse=True)
            t = tri(*x)
            if not alive[t]:
                continue
            alive[t] = False
            remaining -= 1
            for f in (edge(x[0], x[1]), edge(x[0], x[2]), edge(x[1], x[2])):
                if f != e and not picked[f]:
                    count[f] -= 1
                    heapq.heappush(heap, (-count[f], -f))
    picks = len(order)
    order += [e for e in range(E - 1, -1, -1) if not picked[e]]
    return order, picks


def greedy_assignment_metric(n: int) -> np.ndarray:
    """Distance matrix of the greedy assignment (distinct FP32 values that
    preserve its order: the first edge taken is the longest)."""
    order, _ = greedy_assignment_order(n)
    E = len(order)
    ranks = np.empty(E, dtype=np.uint32)
    ranks[np.asarray(order, dtype=np.int64)] = np.arange(E, 0, -1, dtype=np.uint32)
    return (np.uint32(0x3F800000) + ranks).view(np.float32)


def random_integer_metric(n: int, seed: int, vmax: int = 4) -> np.ndarray:
    """Tie-heavy matrices: i.i.d. integers in [1, vmax] (not necessarily a
    metric; the method only reads edge lengths)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.integers(1, vmax + 1, size=n * (n - 1) // 2).astype(np.float32)


def duplicate_points_cloud(n: int, seed: int, ndup: int) -> np.ndarray:
    """n points i.i.d. uniform in [0,1]^2 of which ndup are exact copies of
    earlier points (coincident points: zero distances off the diagonal),
    the copies spread over the index range."""
    rng = np.random.Generator(np.random.PCG64(seed))
    x = rng.random((n, 2))
    for i in rng.choice(np.arange(1, n), size=min(ndup, n - 1), replace=False):
        x[i] = x[int(rng.integers(0, i))]
    return x


def signed_zero_metric(n: int, seed: int, vmax: int = 3, zero_frac: float = 0.15) -> np.ndarray:
    """Tie-heavy integer matrix (entries in [1, vmax]) in which about
    zero_frac of the entries are zero, half of them written as -0.0 and half
    as +0.0 (both are the distance 0)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    m = n * (n - 1) // 2
    d = rng.integers(1, vmax + 1, size=m).astype(np.float32)
    z = rng.random(m) < zero_frac
    neg = rng.random(m) < 0.5
    d[z & neg] = np.float32(-0.0)
    d[z & ~neg] = np.float32(0.0)
    return d


def collinear_integer_metric(k: int) -> np.ndarray:
    """The k+1 points 0, 1, ..., k on a line: d(i, j) = |i - j| (exact)."""
    n = k + 1
    out = np.empty(n * (n - 1) // 2, dtype=np.float32)
    idx = 0
    for i in range(1, n):
        for j in range(i):
            out[idx] = float(i - j)
            idx += 1
    return out


def _dist(points_fn, *a, **k):
    return condensed_from_points(points_fn(*a, **k))


# Named workloads: (name, n, maxdim, threshold, builder)
WORKLOADS = {
    "square32": dict(n=32, maxdim=1, threshold=float("inf"),
                     build=lambda: _dist(uniform_square_points, 32, 1001)),
    "torus400": dict(n=400, maxdim=2, threshold=float("inf"),
                     build=lambda: _dist(noisy_torus_points, 400, 1002)),
    "sphere4096": dict(n=4096, maxdim=2, threshold=0.4,
                       build=lambda: _dist(noisy_sphere_points, 4096, 1003)),
    # request 448 of the serving stream: 703 points of a 5-dimensional
    # Gaussian mixture, dims 0-2, threshold at its enclosing radius (its
    # C(703,3) = 57.7M triangle candidates take more than 1 GiB of outputs,
    # so the dense enumeration counts them before sizing its outputs)
    "mixture448": dict(n=703, maxdim=2, threshold=float("inf"), golden_threshold="radius",
                       build=lambda: mixture_request(448)["dist"]),
    # the same cloud and threshold, one dimension higher (C(4096,5) ~ 9.5e15
    # cofacet indices)
    "sphere4096d3": dict(n=4096, maxdim=3, threshold=0.4,
                         build=lambda: _dist(noisy_sphere_points, 4096, 1003)),
}
