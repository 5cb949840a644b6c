"""Pins of the CPU oracle against facts that do not come from the oracle.

Each test checks the oracle against something the paper or plain
mathematics fixes: the paper's worked example, closed forms, brute-force
homology, a library minimum spanning tree, counting identities, the
enclosing-radius proposition and the apparent-pair bounds theorem.
"""
import math
import os

import numpy as np
import pytest

import brute
import oracle
import workloads as w

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _bars_equal(a, b):
    for (b1, d1), (b2, d2) in zip(a, b):
        assert np.array_equal(b1.view(np.uint32), b2.view(np.uint32))
        assert np.array_equal(d1.view(np.uint32), d2.view(np.uint32))


def test_unit_square_worked_example():
    """Paper, Background (Rips filtration figure): H1 = [1, sqrt 2)."""
    rows = [l.split() for l in open(os.path.join(GOLDEN, "unit_square.txt"))
            if l.strip() and not l.startswith("#")]
    bars = oracle.barcodes(w.unit_square_example(), 4, 1)
    for p in range(2):
        exp = [(np.float32(r[1]), np.float32(np.inf if r[2] == "inf" else r[2]))
               for r in rows if int(r[0]) == p]
        got = list(zip(bars[p][0].tolist(), bars[p][1].tolist()))
        assert got == [(float(a), float(b)) for a, b in exp]


@pytest.mark.parametrize("n", [5, 6, 7, 8, 9, 10, 12])
def test_cycle_graph_h1_closed_form(n):
    """Integer geodesic metric of C_n: one H1 bar [1, ceil(n/3))."""
    bars = oracle.barcodes(w.cycle_graph_metric(n), n, 1)
    b, d = bars[1]
    assert b.tolist() == [1.0]
    assert d.tolist() == [float(math.ceil(n / 3))]
    # H0: n-1 bars [0,1) and one essential bar
    assert bars[0][1].tolist() == [1.0] * (n - 1) + [np.inf]


@pytest.mark.parametrize("n", [6, 9, 12])
def test_cycle_graph_h2_closed_form(n):
    """For 3 | n: n/3 - 1 bars [n/3, n/3 + 1) in H2."""
    bars = oracle.barcodes(w.cycle_graph_metric(n), n, 2)
    k = n // 3
    assert list(zip(bars[2][0].tolist(), bars[2][1].tolist())) == [(k, k + 1)] * (k - 1)


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("thr", [np.inf, 0.25])
def test_h0_equals_minimum_spanning_tree(seed, thr):
    """H0 deaths = MST edge weights; #essential = #components (scipy)."""
    pts = w.uniform_square_points(40, seed=seed)
    dc = w.condensed_from_points(pts)
    bars = oracle.barcodes(dc, 40, 0, thr)
    weights, ncomp = brute.kruskal_free_mst_weights(dc, 40, thr)
    b, d = bars[0]
    assert np.all(b == 0)
    fin = d[np.isfinite(d)]
    assert np.array_equal(np.sort(fin), weights[weights > 0])
    assert int(np.sum(~np.isfinite(d))) == ncomp


def test_h0_duplicate_points_give_no_zero_length_bars():
    pts = np.array([[0, 0], [0, 0], [1, 0], [1, 0], [3, 0]], dtype=np.float64)
    dc = w.condensed_from_points(pts)
    bars = oracle.barcodes(dc, 5, 1)
    assert bars[0][1].tolist() == [1.0, 2.0, np.inf]


@pytest.mark.parametrize("case", range(12))
def test_bars_match_brute_force_betti_numbers(case):
    """#bars alive at t == beta_p(Rips_t) by GF(2) ranks, every scale t."""
    n = 6 + case % 3
    if case % 2 == 0:
        dc = w.random_integer_metric(n, seed=100 + case, vmax=3 + case % 4)
    else:
        dc = w.condensed_from_points(w.uniform_square_points(n, seed=200 + case))
    thr = np.inf if case % 4 < 2 else float(np.quantile(dc, 0.7))
    maxdim = 2 if n > 6 else 3
    bars = oracle.barcodes(dc, n, maxdim, thr)
    brute.check_bars_against_betti(dc, n, maxdim, bars, thr)


@pytest.mark.parametrize("case", range(6))
def test_zero_distance_bars_match_brute_force_betti_numbers(case):
    """Coincident points and explicit -0.0 / +0.0 entries: the bars still
    give beta_p(Rips_t) at every scale, no bar has zero length, and every
    reported value is written as +0.0, never -0.0."""
    n = 6 + case % 3
    if case % 2 == 0:
        dc = w.signed_zero_metric(n, seed=300 + case, vmax=3)
        assert np.any(np.signbit(dc) & (dc == 0))
    else:
        dc = w.condensed_from_points(w.duplicate_points_cloud(n, 310 + case, 2))
    assert np.any(dc == 0)
    thr = np.inf if case < 4 else 1.5
    maxdim = 2 if n > 6 else 3
    bars = oracle.barcodes(dc, n, maxdim, thr)
    brute.check_bars_against_betti(dc, n, maxdim, bars, thr)
    for b, d in bars:
        assert np.all(d > b)
        assert not np.any(np.signbit(b)) and not np.any(np.signbit(d))


@pytest.mark.parametrize("seed", range(4))
def test_pair_count_identity(seed):
    """n_p = P_p + E_p + P_{p-1}; full Rips: P_p = C(n-1, p+1), E_p = 0 for
    p >= 1 and E_0 = 1 (Pascal's rule on the full simplex)."""
    n = 14
    dc = w.random_integer_metric(n, seed=seed, vmax=5) if seed % 2 else \
        w.condensed_from_points(w.uniform_square_points(n, seed=seed))
    red = oracle.reduce(dc, n, 3)
    bars = oracle.bars_from_pairs(red)
    prev = 0
    for p, r in enumerate(red):
        ess = int(np.sum(~np.isfinite(bars[p][1])))
        assert r["n_simplices"] == math.comb(n, p + 1)
        assert len(r["sigma"]) == math.comb(n - 1, p + 1)
        assert ess == (1 if p == 0 else 0)
        assert r["n_simplices"] == len(r["sigma"]) + ess + prev
        prev = len(r["sigma"])


@pytest.mark.parametrize("seed", range(3))
def test_pair_count_identity_thresholded(seed):
    n = 16
    dc = w.condensed_from_points(w.uniform_square_points(n, seed=50 + seed))
    thr = float(np.quantile(dc, 0.4))
    red = oracle.reduce(dc, n, 2, thr)
    bars = oracle.bars_from_pairs(red)
    prev = 0
    for p, r in enumerate(red):
        ess = int(np.sum(~np.isfinite(bars[p][1])))
        assert r["n_simplices"] == len(r["sigma"]) + ess + prev
        prev = len(r["sigma"])


def test_clearing_lemma():
    """Every tau of a dimension-(p-1) pair is a zero column in dimension p."""
    n = 12
    dc = w.condensed_from_points(w.uniform_square_points(n, seed=7))
    red = oracle.reduce(dc, n, 2)
    for p in (1, 2):
        assert np.all(np.isin(red[p - 1]["tau"], red[p]["zero_sigma"]))


def test_enclosing_radius_closed_forms():
    """R = min_x max_y d(x, y) on inputs where it is known in closed form,
    chosen so that the usual slips (the global maximum, the smallest entry,
    the maximum of the row minima) give other values:
      - the unit square's corners: every corner's farthest point is the
        opposite corner, R = fl32(sqrt 2);
      - the cycle-graph metric on C_n: every vertex's farthest vertex is
        floor(n/2) steps away, R = floor(n/2);
      - the points 0..k on a line: the middle point sees both ends,
        R = ceil(k/2), while the global maximum is k;
      - one point: R = 0; two points: R = their distance."""
    assert oracle.enclosing_radius(w.unit_square_example(), 4) == np.float32(math.sqrt(2.0))
    for n in range(3, 14):
        assert oracle.enclosing_radius(w.cycle_graph_metric(n), n) == n // 2, n
    for k in range(1, 12):
        assert oracle.enclosing_radius(w.collinear_integer_metric(k), k + 1) == (k + 1) // 2, k
    assert oracle.enclosing_radius(np.zeros(0, np.float32), 1) == 0.0
    assert oracle.enclosing_radius(np.array([2.5], np.float32), 2) == 2.5
    # a star: the centre (vertex 0) is at distance 1 from every leaf, leaves
    # are 2 apart; R = 1 although most rows have maximum 2
    n = 7
    star = np.array([1.0 if j == 0 else 2.0 for i in range(1, n) for j in range(i)], np.float32)
    assert oracle.enclosing_radius(star, n) == 1.0


@pytest.mark.parametrize("seed", range(4))
def test_enclosing_radius_does_not_change_bars(seed):
    """Proposition (enclosing radius): truncating at R keeps every nonzero
    interval; bars at thr=R and thr=inf are bitwise identical."""
    n = 18
    dc = w.condensed_from_points(w.uniform_square_points(n, seed=seed))
    R = oracle.enclosing_radius(dc, n)
    _bars_equal(oracle.barcodes(dc, n, 2, R), oracle.barcodes(dc, n, 2, np.inf))


# ---------------------------- apparent pairs -----------------------------

@pytest.mark.parametrize("case", range(10))
def test_apparent_definition_matches_brute_force(case):
    n = 6 + case % 3
    p = 1 + case % 2
    dc = w.random_integer_metric(n, seed=300 + case, vmax=2 + case % 3)
    thr = np.inf if case < 6 else float(np.quantile(dc, 0.6))
    s, t = oracle.apparent_pairs(dc, n, p, thr)
    got = set(zip(s.tolist(), t.tolist()))
    exp = {(brute.cidx(a), brute.cidx(b)) for a, b in
           brute.apparent_by_brute_force(dc, n, p, thr)}
    assert got == exp


@pytest.mark.parametrize("p", [1, 2, 3])
@pytest.mark.parametrize("n", [5, 6, 8])
def test_theorem1_upper_bound_all_equal(n, p):
    """All diameters equal: exactly C(n-1, p+1) apparent p-simplices."""
    s, _ = oracle.apparent_pairs(w.all_equal_metric(n), n, p)
    assert len(s) == math.comb(n - 1, p + 1)


@pytest.mark.parametrize("n", [3, 4, 5, 6, 7, 8, 9])
def test_theorem1_upper_bound_distinct_diameters(n):
    """Edge cidx i gets distance N - i: still C(n-1, 2) apparent edges
    (n = 5: 6 of 10); the recurrence T(n) = T(n-1) + n - 2, T(3) = 1."""
    s, _ = oracle.apparent_pairs(w.reverse_lex_metric(n), n, 1)
    assert len(s) == math.comb(n - 1, 2)
    if n > 3:
        prev, _ = oracle.apparent_pairs(w.reverse_lex_metric(n - 1), n - 1, 1)
        assert len(s) == len(prev) + n - 2


@pytest.mark.parametrize("p", [1, 2, 3])
@pytest.mark.parametrize("seed", range(3))
def test_theorem1_lower_bound_single_simplex(p, seed):
    """n = p+2 points with distinct distances: exactly one apparent pair
    among the p+2 facets of the single (p+1)-simplex."""
    n = p + 2
    dc = w.random_permutation_metric(n, seed=seed)
    s, t = oracle.apparent_pairs(dc, n, p)
    assert len(s) == 1
    assert int(t[0]) == 0  # the only (p+1)-simplex has cidx 0


@pytest.mark.parametrize("seed", range(4))
def test_apparent_pairs_are_persistence_pairs(seed):
    """Apparent pairs are pivots of the standard reduction; the apparent
    rate respects Theorem 1's bounds; apparent edges avoid the MST."""
    n = 14
    dc = w.condensed_from_points(w.uniform_square_points(n, seed=seed))
    red = oracle.reduce(dc, n, 2)
    for p in (1, 2):
        s, t = oracle.apparent_pairs(dc, n, p)
        pairs = set(zip(red[p]["sigma"].tolist(), red[p]["tau"].tolist()))
        assert set(zip(s.tolist(), t.tolist())) <= pairs
        frac = len(s) / math.comb(n, p + 1)
        assert 1.0 / (p + 2) <= frac <= (n - p - 1) / n
    # GMST lemma: the longest edge of an apparent edge column is the edge
    # itself, and it is never a minimum-spanning-tree edge
    s, _ = oracle.apparent_pairs(dc, n, 1)
    mst_edges = set(red[0]["tau"].tolist())
    assert not (set(s.tolist()) & mst_edges)


@pytest.mark.parametrize("case", range(8))
def test_clearing_mode_matches_plain_reduction(case):
    """The oracle's clearing mode (used only where the plain reduction cannot
    finish) gives the same pairs and bitwise the same bars as the plain
    standard reduction (paper, clearing lemma)."""
    n = 16 + 4 * (case % 4)
    if case % 2:
        dc = w.random_integer_metric(n, seed=400 + case, vmax=6)
    else:
        dc = w.condensed_from_points(w.noisy_torus_points(n, seed=500 + case))
    thr = np.inf if case < 4 else float(np.quantile(dc, 0.5))
    plain = oracle.reduce(dc, n, 2, thr)
    clear = oracle.reduce(dc, n, 2, thr, clearing=True)
    for p in range(3):
        a = set(zip(plain[p]["sigma"].tolist(), plain[p]["tau"].tolist()))
        b = set(zip(clear[p]["sigma"].tolist(), clear[p]["tau"].tolist()))
        assert a == b
        if p > 0:
            assert clear[p]["n_cleared"] == len(plain[p - 1]["tau"])
    _bars_equal(oracle.bars_from_pairs(plain), oracle.bars_from_pairs(clear))


@pytest.mark.parametrize("case", range(6))
def test_clearing_mode_matches_plain_reduction_maxdim3(case):
    """The clearing mode against the plain reduction through dimension 3,
    where clearing removes columns in three dimensions (dimension 3's
    cleared columns are the taus of dimension 2, themselves found on
    columns that survived dimension 1's clearing)."""
    n = 10 + case % 3
    if case % 3 == 0:
        dc = w.random_integer_metric(n, seed=420 + case, vmax=4)
    elif case % 3 == 1:
        dc = w.condensed_from_points(w.noisy_torus_points(n, seed=520 + case))
    else:
        dc = w.signed_zero_metric(n, seed=620 + case, vmax=4)
    thr = np.inf if case < 3 else float(np.quantile(dc, 0.6))
    plain = oracle.reduce(dc, n, 3, thr)
    clear = oracle.reduce(dc, n, 3, thr, clearing=True)
    for p in range(4):
        a = set(zip(plain[p]["sigma"].tolist(), plain[p]["tau"].tolist()))
        b = set(zip(clear[p]["sigma"].tolist(), clear[p]["tau"].tolist()))
        assert a == b, p
        if p > 0:
            assert clear[p]["n_cleared"] == len(plain[p - 1]["tau"])
    assert clear[3]["n_cleared"] > 0
    _bars_equal(oracle.bars_from_pairs(plain), oracle.bars_from_pairs(clear))


# ---------------------------------------------------------------------------
# Greedy deterministic distance assignment (the paper's greedy variant of its
# random apparent-pair construction): every edge it takes while triangles
# remain forms an apparent pair with its oldest remaining cofacet, so the
# apparent-pair test must find exactly that many pairs; the fraction stays
# above the lower bound 1/(p+2) = 1/3 and near 1/2.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n", [4, 7, 12, 20, 33])
def test_greedy_assignment_apparent_count_is_its_pick_count(n):
    order, picks = w.greedy_assignment_order(n)
    d = w.greedy_assignment_metric(n)
    s, t = oracle.apparent_pairs(d, n, 1)
    assert len(s) == picks
    assert len(s) / (n * (n - 1) / 2) >= 1.0 / 3.0
    # the pairs are exactly the picked edges
    assert set(s.tolist()) == set(order[:picks])


def test_greedy_assignment_fraction_near_one_half():
    n = 60
    d = w.greedy_assignment_metric(n)
    s, _ = oracle.apparent_pairs(d, n, 1)
    frac = len(s) / (n * (n - 1) / 2)
    assert 0.4 <= frac <= 0.6, frac
