"""Brute-force homology checkers used to pin the oracle.

Nothing here reduces a filtration.  Betti numbers of each Rips complex are
computed from first principles: list every simplex of diameter <= t, build
the mod-2 boundary matrices and take ranks by Gaussian elimination
(beta_p = dim C_p - rank d_p - rank d_{p+1}).
"""
from __future__ import annotations

import itertools

import numpy as np


def square(dc: np.ndarray, n: int) -> np.ndarray:
    sq = np.zeros((n, n), dtype=np.float64)
    k = 0
    for i in range(1, n):
        for j in range(i):
            sq[i, j] = sq[j, i] = float(dc[k])
            k += 1
    return sq


def rips_simplices(sq: np.ndarray, t: float, maxdim: int) -> list:
    """simplices[p] = list of sorted vertex tuples with diameter <= t."""
    n = sq.shape[0]
    out = [[(v,) for v in range(n)]]
    for p in range(1, maxdim + 1):
        lvl = []
        for s in out[-1]:
            for v in range(s[-1] + 1, n):
                if all(sq[v, u] <= t for u in s):
                    lvl.append(s + (v,))
        out.append(lvl)
    return out


def gf2_rank(vectors: list) -> int:
    """Rank over Z/2 of integer bit-vectors."""
    pivots = {}
    rank = 0
    for v in vectors:
        while v:
            h = v.bit_length() - 1
            if h in pivots:
                v ^= pivots[h]
            else:
                pivots[h] = v
                rank += 1
                break
    return rank


def betti(sq: np.ndarray, t: float, maxdim: int) -> list:
    """Betti numbers beta_0..beta_maxdim of Rips_t over Z/2."""
    simp = rips_simplices(sq, t, maxdim + 1)
    index = [{s: i for i, s in enumerate(lvl)} for lvl in simp]
    ranks = [0] * (maxdim + 2)   # ranks[p] = rank of boundary C_p -> C_{p-1}
    for p in range(1, maxdim + 2):
        cols = []
        for s in simp[p]:
            v = 0
            for drop in range(len(s)):
                f = s[:drop] + s[drop + 1:]
                v |= 1 << index[p - 1][f]
            cols.append(v)
        ranks[p] = gf2_rank(cols)
    return [len(simp[p]) - ranks[p] - ranks[p + 1] for p in range(maxdim + 1)]


def alive(bars, t: float) -> int:
    b, d = bars
    return int(np.sum((b <= t) & (t < d)))


def check_bars_against_betti(dc: np.ndarray, n: int, maxdim: int, bars: list,
                             threshold: float = np.inf) -> None:
    """For every distinct scale t <= threshold (and just below each), the
    number of bars alive at t equals beta_p(Rips_t)."""
    sq = square(dc, n)
    vals = sorted(set(float(x) for x in dc if float(x) <= threshold) | {0.0})
    probes = []
    for v in vals:
        probes.append(v)
        below = np.nextafter(np.float32(v), np.float32(-1))
        if below >= 0:
            probes.append(float(below))
    for t in probes:
        bt = betti(sq, t, maxdim)
        for p in range(maxdim + 1):
            got = alive(bars[p], t)
            assert got == bt[p], (t, p, got, bt[p])


def kruskal_free_mst_weights(dc: np.ndarray, n: int, threshold: float = np.inf):
    """MST edge weights of the threshold graph via scipy (an independent
    minimum-spanning-forest routine), and its number of components."""
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import connected_components, minimum_spanning_tree
    ii, jj = np.tril_indices(n, -1)
    w = dc.astype(np.float64)
    keep = w <= threshold
    # scipy treats explicit zeros as absent edges; shift weights by +1 so
    # zero-length edges survive, then undo the shift.
    g = csr_matrix((w[keep] + 1.0, (ii[keep], jj[keep])), shape=(n, n))
    mst = minimum_spanning_tree(g)
    weights = np.sort(mst.data - 1.0)
    ncomp = connected_components(g, directed=False)[0]
    return weights.astype(np.float32), ncomp


def apparent_by_brute_force(dc: np.ndarray, n: int, p: int, threshold: float = np.inf):
    """Apparent pairs by the definition, straight from vertex tuples: sort
    every simplex of dimensions p and p+1 in the simplex-wise filtration
    order, then pair sigma with its oldest cofacet tau when sigma is tau's
    youngest facet.  Returns a set of (sigma_vertices, tau_vertices)."""
    sq = square(dc, n)
    simp = rips_simplices(sq, threshold, p + 1)

    def diam(s):
        return max((sq[a, b] for a, b in itertools.combinations(s, 2)), default=0.0)

    def colex_key(s):
        # combinatorial number system order == colexicographic order on
        # increasing tuples == lexicographic order on decreasing tuples
        return tuple(sorted(s, reverse=True))

    def filt_key(s):
        # diameter ascending, dimension ascending, cidx descending
        ck = colex_key(s)
        return (diam(s), len(s), tuple(-v for v in ck))

    pos = {s: i for i, s in enumerate(sorted(simp[p] + simp[p + 1], key=filt_key))}
    out = set()
    for s in simp[p]:
        cof = [t for t in simp[p + 1] if set(s) <= set(t)]
        if not cof:
            continue
        tau = min(cof, key=lambda t: pos[t])
        facets = [tuple(x for x in tau if x != v) for v in tau]
        young = max(facets, key=lambda f: pos[f])
        if young == s:
            out.add((s, tau))
    return out


def cidx(vertices, binom=None) -> int:
    """Combinatorial index sum_i C(v_i, i+1) of a vertex set."""
    from math import comb
    vs = sorted(vertices)
    return sum(comb(v, i + 1) for i, v in enumerate(vs))
