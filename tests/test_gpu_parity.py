"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Barcodes are compared bit for bit: every birth and death is an entry of the
FP32 distance matrix, never the result of arithmetic, so the tolerance is
zero.  Persistence pairs are compared as exact sets of combinatorial
indices.  The apparent-pair kernel is also compared with the literal
definition, and with the exact counts of the paper's Theorem 1
constructions.
"""
import hashlib
import math
import os

import numpy as np
import pytest

import oracle
import workloads as w

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def rpp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2003_07989_amd as m
    m.load()
    return m


def assert_bars_equal(got, exp, label=""):
    assert len(got) == len(exp), label
    for p, ((gb, gd), (eb, ed)) in enumerate(zip(got, exp)):
        ok = (len(gb) == len(eb) and np.array_equal(gb.view(np.uint32), eb.view(np.uint32))
              and np.array_equal(gd.view(np.uint32), ed.view(np.uint32)))
        if not ok:
            msg = "%s dim %d: %d bars vs oracle %d\n gpu %s\n ora %s" % (
                label, p, len(gb), len(eb), list(zip(gb[:8], gd[:8])), list(zip(eb[:8], ed[:8])))
            raise AssertionError(msg)


def _cases():
    c = []
    for n in (5, 8, 12, 20, 33):
        c.append(("square%d" % n, w.condensed_from_points(w.uniform_square_points(n, 10 + n)),
                  n, 3 if n <= 12 else 2, math.inf))
    for n in (48, 64):
        c.append(("square%d" % n, w.condensed_from_points(w.uniform_square_points(n, 10 + n)),
                  n, 2, math.inf))
    for n in (30, 60):
        c.append(("torus%d" % n, w.condensed_from_points(w.noisy_torus_points(n, 20 + n)),
                  n, 2, math.inf))
    for n, vmax in ((8, 2), (16, 3), (30, 5), (45, 4)):
        c.append(("int%d_%d" % (n, vmax), w.random_integer_metric(n, 30 + n, vmax), n,
                  3 if n <= 16 else 2, math.inf))
    c.append(("equal20", w.all_equal_metric(20), 20, 3, math.inf))
    c.append(("revlex40", w.reverse_lex_metric(40), 40, 2, math.inf))
    for n in (9, 12, 30):
        c.append(("cycle%d" % n, w.cycle_graph_metric(n), n, 2, math.inf))
    c.append(("perm50", w.random_permutation_metric(50, 5), 50, 2, math.inf))
    # thresholded cases
    for n, q in ((25, 0.3), (40, 0.5), (64, 0.25)):
        d = w.condensed_from_points(w.uniform_square_points(n, 40 + n))
        c.append(("square%d_q%g" % (n, q), d, n, 2, float(np.quantile(d, q))))
    d = w.random_integer_metric(30, 77, 6)
    c.append(("int30_thr3", d, 30, 2, 3.0))
    d = w.condensed_from_points(w.uniform_square_points(40, 91))
    c.append(("square40_R", d, 40, 2, oracle.enclosing_radius(d, 40)))
    return c


CASES = _cases()


def _oracle_bars(d, n, maxdim, thr):
    return oracle.barcodes(d, n, maxdim, thr, clearing=n > 33)


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_barcodes_match_oracle(rpp, case):
    name, d, n, maxdim, thr = case
    print("case", name, n, maxdim, thr, flush=True)
    got = rpp.barcodes(d, maxdim, thr)
    assert_bars_equal(got.bars, _oracle_bars(d, n, maxdim, thr), name)


@pytest.mark.parametrize("case", CASES[:14], ids=[c[0] for c in CASES[:14]])
def test_pairs_match_oracle(rpp, case):
    """Apparent pairs (GPU) plus host pairs == the oracle's pivots, as exact
    (sigma, tau) sets, with the threshold as given (no radius truncation)."""
    name, d, n, maxdim, thr = case
    print("case", name, flush=True)
    got = rpp.barcodes(d, maxdim, thr, flags=rpp.RPP_WANT_PAIRS | rpp.RPP_NO_ENCLOSING_RADIUS)
    red = oracle.reduce(d, n, maxdim, thr, clearing=n > 33)
    assert set(got.pairs[0][1].tolist()) == set(red[0]["tau"].tolist())
    for p in range(1, maxdim + 1):
        gs = set(zip(got.pairs[p][0].tolist(), got.pairs[p][1].tolist()))
        es = set(zip(red[p]["sigma"].tolist(), red[p]["tau"].tolist()))
        assert gs == es, (name, p, len(gs), len(es))


@pytest.mark.parametrize("case", CASES[:10], ids=[c[0] for c in CASES[:10]])
def test_stats_accounting(rpp, case):
    """Filter accounting (candidates = thresholded + cleared + kept), the
    partition (kept = apparent + non-apparent) and the pair identity
    n_p = P_p + E_p + P_{p-1}."""
    name, d, n, maxdim, thr = case
    got = rpp.barcodes(d, maxdim, thr, flags=rpp.RPP_NO_ENCLOSING_RADIUS)
    prev_pairs = 0
    for p, st in enumerate(got.stats):
        if p >= 1:
            assert st["n_candidates"] == st["n_thresholded"] + st["n_cleared"] + st["n_kept"]
            assert st["n_kept"] == st["n_apparent"] + st["n_nonapparent"]
            assert st["n_cleared"] == prev_pairs
            assert st["n_simplices"] == oracle.count_simplices(d, n, p, thr)
        pairs = st["n_apparent"] + st["n_host_pairs"]
        assert st["n_simplices"] == pairs + st["n_essential"] + prev_pairs
        prev_pairs = pairs


@pytest.mark.parametrize("p", [1, 2, 3])
@pytest.mark.parametrize("case", range(6))
def test_apparent_kernel_matches_definition(rpp, p, case):
    n = (7, 10, 14, 18, 12, 16)[case]
    if case % 2:
        d = w.random_integer_metric(n, 600 + case, 2 + case % 3)
    else:
        d = w.condensed_from_points(w.uniform_square_points(n, 700 + case))
    thr = math.inf if case < 4 else float(np.quantile(d, 0.6))
    s, t, ncols = rpp.apparent_pairs(d, p, thr)
    es, et = oracle.apparent_pairs(d, n, p, thr)
    assert ncols == oracle.count_simplices(d, n, p, thr)
    assert set(zip(s.tolist(), t.tolist())) == set(zip(es.tolist(), et.tolist()))


TWO_PHASE_CASES = [
    # (name, n, p): shallow scans (torus, square), ties (integer metric),
    # deep scans (random orders), and n at or below the K candidates
    ("torus60", 60, 2), ("square50", 50, 3), ("int40", 40, 3), ("int45", 45, 2),
    ("perm80", 80, 1), ("perm30", 30, 2), ("tiny3", 3, 1), ("tiny4", 4, 2),
    ("tiny5", 5, 1), ("tiny9", 9, 3),
    # n = 3 mod 4 (with the cases above, every residue of n mod 4: the
    # vector form's aligned top block holds 4, 1, 2 or 3 real candidates)
    ("torus63", 63, 2), ("perm43", 43, 2), ("tiny7", 7, 2),
]


def _two_phase_metric(name, n):
    if name.startswith("torus"):
        return w.condensed_from_points(w.noisy_torus_points(n, 5))
    if name.startswith("square") or name.startswith("tiny"):
        return w.condensed_from_points(w.uniform_square_points(n, 31 + n))
    if name.startswith("int"):
        return w.random_integer_metric(n, 611 + n, 3)
    return w.random_permutation_metric(n, 12 + n)


@pytest.mark.parametrize("group", [408, 416, 808, 1608, 1616, 10408, 10416, 20008, 20016,
                                   20308, 20408])
@pytest.mark.parametrize("case", TWO_PHASE_CASES, ids=[c[0] for c in TWO_PHASE_CASES])
def test_two_phase_apparent_kernel_matches_oracle(rpp, monkeypatch, group, case):
    """The two-phase apparent kernel (each lane alone on the top K
    candidates of its column, then G lanes per column still open): pairs
    equal the oracle's, with and without a threshold, over several waves and
    a ragged last one, and the scan tally equals the single-phase kernel's."""
    name, n, p = case
    d = _two_phase_metric(name, n)
    for thr in (math.inf, float(np.quantile(d, 0.7))):
        monkeypatch.setenv("RPP_APPARENT_GROUP", str(group))
        s, t, ncols = rpp.apparent_pairs(d, p, thr)
        es, et = oracle.apparent_pairs(d, n, p, thr)
        assert ncols == oracle.count_simplices(d, n, p, thr)
        assert set(zip(s.tolist(), t.tolist())) == set(zip(es.tolist(), et.tolist())), thr
    monkeypatch.setenv("RPP_COUNT_SCANS", "1")
    _, _, st2 = rpp.apparent_count(d, p)
    monkeypatch.setenv("RPP_APPARENT_GROUP", "8")
    _, _, st1 = rpp.apparent_count(d, p)
    assert st2["apparent_group"] == group and st1["apparent_group"] == 8
    assert st2["n_scanned"] == st1["n_scanned"]


@pytest.mark.parametrize("n,p", [(60, 1), (60, 2), (30, 3), (400, 1), (100, 2)])
def test_theorem1_upper_bound_all_equal_on_gpu(rpp, n, p):
    s, _, ncols = rpp.apparent_pairs(w.all_equal_metric(n), p)
    assert ncols == math.comb(n, p + 1)
    assert len(s) == math.comb(n - 1, p + 1)


@pytest.mark.parametrize("n", [5, 50, 300, 1000])
def test_theorem1_distinct_diameters_on_gpu(rpp, n):
    s, _, _ = rpp.apparent_pairs(w.reverse_lex_metric(n), 1)
    assert len(s) == math.comb(n - 1, 2)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_theorem1_lower_bound_on_gpu(rpp, p):
    s, t, _ = rpp.apparent_pairs(w.random_permutation_metric(p + 2, 3), p)
    assert len(s) == 1 and int(t[0]) == 0


def test_group_sizes_agree(rpp, monkeypatch):
    d = w.condensed_from_points(w.noisy_torus_points(80, 5))
    ref = None
    for g in (1, 4, 8, 16, 32, 64, 408, 416, 808, 1608, 1616, 10408, 10416, 20008, 20016,
              20308, 20408):
        monkeypatch.setenv("RPP_APPARENT_GROUP", str(g))
        r = rpp.barcodes(d, 2, flags=rpp.RPP_WANT_PAIRS)
        key = [set(zip(a.tolist(), b.tolist())) for a, b in r.pairs[1:]]
        if ref is None:
            ref = key
        assert key == ref, g


def test_repeat_runs_are_bitwise_identical(rpp):
    d = w.condensed_from_points(w.noisy_torus_points(120, 9))
    a = rpp.barcodes(d, 2)
    b = rpp.barcodes(d, 2)
    assert_bars_equal(a.bars, b.bars)


def test_host_entry_point_matches_device_entry_point(rpp):
    d = w.condensed_from_points(w.uniform_square_points(50, 3))
    assert_bars_equal(rpp.barcodes_host(d, 2).bars, rpp.barcodes(d, 2).bars)


def test_device_validation_rejects_bad_entries(rpp):
    d = w.condensed_from_points(w.uniform_square_points(20, 3))
    d[17] = np.nan
    with pytest.raises(rpp.RppError) as e:
        rpp.barcodes(d, 1)
    assert e.value.code == -2


def test_enclosing_radius_reported(rpp):
    d = w.condensed_from_points(w.uniform_square_points(40, 8))
    r = rpp.barcodes(d, 1)
    assert r.enclosing_radius == np.float32(oracle.enclosing_radius(d, 40))
    assert r.threshold_used == r.enclosing_radius


def test_uniform_square_32_matches_oracle(rpp):
    """32 points i.i.d. uniform in [0,1]^2, dims 0-1, no threshold."""
    cfg = w.WORKLOADS["square32"]
    d = cfg["build"]()
    got = rpp.barcodes(d, cfg["maxdim"], cfg["threshold"])
    assert_bars_equal(got.bars, oracle.barcodes(d, 32, 1), "square32")


def test_torus400_matches_stored_oracle(rpp):
    """400-point noisy torus, dims 0-2, no threshold: against the oracle's
    barcodes stored by tests/golden/make_golden.py."""
    head, exp = _golden("torus400")
    cfg = w.WORKLOADS["torus400"]
    d = cfg["build"]()
    import hashlib
    assert hashlib.sha256(d.tobytes()).hexdigest() == head["sha256"], "input generator drifted"
    got = rpp.barcodes(d, cfg["maxdim"], cfg["threshold"])
    assert_bars_equal(got.bars, exp, "torus400")
    for p in range(1, 3):
        st = got.stats[p]
        assert st["n_apparent"] + st["n_host_pairs"] > 0


@pytest.mark.parametrize("case", CASES[::3], ids=[c[0] for c in CASES[::3]])
def test_sorted_pair_store_mode_matches_oracle(rpp, case):
    """The paper's two-layer store (apparent pairs sorted by tau, binary
    searched on the host) gives the same bars and pairs as the default."""
    name, d, n, maxdim, thr = case
    got = rpp.barcodes(d, maxdim, thr, flags=rpp.RPP_SORTED_PAIR_STORE)
    assert_bars_equal(got.bars, _oracle_bars(d, n, maxdim, thr), name)
    f = rpp.RPP_WANT_PAIRS | rpp.RPP_NO_ENCLOSING_RADIUS
    a = rpp.barcodes(d, maxdim, thr, flags=f)
    b = rpp.barcodes(d, maxdim, thr, flags=f | rpp.RPP_SORTED_PAIR_STORE)
    for p in range(1, maxdim + 1):
        assert set(zip(*map(list, a.pairs[p]))) == set(zip(*map(list, b.pairs[p])))


def test_torus400_sorted_pair_store(rpp):
    head, exp = _golden("torus400")
    d = w.WORKLOADS["torus400"]["build"]()
    got = rpp.barcodes(d, 2, flags=rpp.RPP_SORTED_PAIR_STORE)
    assert_bars_equal(got.bars, exp, "torus400 sorted store")


@pytest.mark.parametrize("case", CASES[1::3], ids=[c[0] for c in CASES[1::3]])
def test_oblivious_reduction_matches_oracle(rpp, case):
    """Adding a host pivot's unreduced coboundary (oblivious reduction)
    instead of its reduced column gives the same bars and pairs (the
    paper's lemma on oblivious reduction)."""
    name, d, n, maxdim, thr = case
    got = rpp.barcodes(d, maxdim, thr, flags=rpp.RPP_OBLIVIOUS_REDUCTION)
    assert_bars_equal(got.bars, _oracle_bars(d, n, maxdim, thr), name)
    f = rpp.RPP_WANT_PAIRS | rpp.RPP_NO_ENCLOSING_RADIUS
    a = rpp.barcodes(d, maxdim, thr, flags=f)
    b = rpp.barcodes(d, maxdim, thr, flags=f | rpp.RPP_OBLIVIOUS_REDUCTION)
    for p in range(1, maxdim + 1):
        assert set(zip(*map(list, a.pairs[p]))) == set(zip(*map(list, b.pairs[p])))


def test_torus400_oblivious_reduction(rpp):
    head, exp = _golden("torus400")
    d = w.WORKLOADS["torus400"]["build"]()
    got = rpp.barcodes(d, 2, flags=rpp.RPP_OBLIVIOUS_REDUCTION)
    assert_bars_equal(got.bars, exp, "torus400 oblivious")


@pytest.mark.parametrize("case", CASES[2::3], ids=[c[0] for c in CASES[2::3]])
def test_sort_first_order_matches_oracle(rpp, case):
    """The paper's stage order (every kept column sorted before the
    apparent test) gives the same bars and pairs as sorting only the
    non-apparent columns after it."""
    name, d, n, maxdim, thr = case
    got = rpp.barcodes(d, maxdim, thr, flags=rpp.RPP_SORT_FIRST)
    assert_bars_equal(got.bars, _oracle_bars(d, n, maxdim, thr), name)
    f = rpp.RPP_WANT_PAIRS | rpp.RPP_NO_ENCLOSING_RADIUS
    a = rpp.barcodes(d, maxdim, thr, flags=f)
    b = rpp.barcodes(d, maxdim, thr, flags=f | rpp.RPP_SORT_FIRST)
    for p in range(1, maxdim + 1):
        assert set(zip(*map(list, a.pairs[p]))) == set(zip(*map(list, b.pairs[p])))
        assert a.stats[p]["n_apparent"] == b.stats[p]["n_apparent"]


def test_torus400_sort_first(rpp):
    head, exp = _golden("torus400")
    d = w.WORKLOADS["torus400"]["build"]()
    got = rpp.barcodes(d, 2, flags=rpp.RPP_SORT_FIRST)
    assert_bars_equal(got.bars, exp, "torus400 sort first")
    got = rpp.barcodes(d, 2, flags=rpp.RPP_SORT_FIRST | rpp.RPP_FORCE_SPARSE)
    assert_bars_equal(got.bars, exp, "torus400 sort first, sparse path")


SPARSE_CASES = [c for c in CASES if not math.isinf(c[4])] + CASES[:8]


@pytest.mark.parametrize("case", SPARSE_CASES, ids=["sp_" + c[0] for c in SPARSE_CASES])
def test_sparse_path_matches_oracle(rpp, case):
    """Neighbour-bitset enumeration (forced) gives the oracle's bars and
    pairs."""
    name, d, n, maxdim, thr = case
    print("case", name, flush=True)
    got = rpp.barcodes(d, maxdim, thr, flags=rpp.RPP_FORCE_SPARSE)
    assert_bars_equal(got.bars, _oracle_bars(d, n, maxdim, thr), name)
    f = rpp.RPP_FORCE_SPARSE | rpp.RPP_WANT_PAIRS | rpp.RPP_NO_ENCLOSING_RADIUS
    g = rpp.barcodes(d, maxdim, thr, flags=f)
    red = oracle.reduce(d, n, maxdim, thr, clearing=n > 33)
    for p in range(1, maxdim + 1):
        gs = set(zip(g.pairs[p][0].tolist(), g.pairs[p][1].tolist()))
        es = set(zip(red[p]["sigma"].tolist(), red[p]["tau"].tolist()))
        assert gs == es, (name, p)
        st = g.stats[p]
        assert st["n_kept"] == st["n_apparent"] + st["n_nonapparent"]
        assert st["n_simplices"] == oracle.count_simplices(d, n, p, thr)


@pytest.mark.parametrize("case", SPARSE_CASES[1::3], ids=["hm_" + c[0] for c in SPARSE_CASES[1::3]])
def test_host_packed_rows_match_host_matrix(rpp, monkeypatch, case):
    """The sparse path's host reduction reading packed neighbour rows (the
    default) and reading the square matrix (RPP_HOST_MATRIX=1): the same
    bars, critical edges and pairs, with and without rank coding."""
    name, d, n, maxdim, thr = case
    f = rpp.RPP_FORCE_SPARSE | rpp.RPP_WANT_PAIRS | rpp.RPP_WANT_CRITICAL_EDGES
    for rank in ("0", "1"):
        monkeypatch.setenv("RPP_RANK_CODING", rank)
        monkeypatch.delenv("RPP_HOST_MATRIX", raising=False)
        a = rpp.barcodes(d, maxdim, thr, flags=f)
        monkeypatch.setenv("RPP_HOST_MATRIX", "1")
        b = rpp.barcodes(d, maxdim, thr, flags=f)
        assert_bars_equal(a.bars, b.bars, name)
        for p in range(maxdim + 1):
            assert np.array_equal(a.edges[p][0], b.edges[p][0]), (name, rank, p)
            assert np.array_equal(a.edges[p][1], b.edges[p][1]), (name, rank, p)
        for p in range(1, maxdim + 1):
            assert set(zip(*map(list, a.pairs[p]))) == set(zip(*map(list, b.pairs[p])))


SPARSE_GROUPS = [4, 8, 16, 104, 108, 204, 208, 404, 408]


@pytest.mark.parametrize("case", SPARSE_CASES[::3], ids=["spg_" + c[0] for c in SPARSE_CASES[::3]])
def test_sparse_apparent_kernel_forms_match_oracle(rpp, monkeypatch, case):
    """Every sparse apparent-kernel form (G lanes per column; two-phase with
    the top K words per lane first) gives the oracle's pairs, and the same
    scan tally."""
    name, d, n, maxdim, thr = case
    red = oracle.reduce(d, n, maxdim, thr, clearing=n > 33)
    f = rpp.RPP_FORCE_SPARSE | rpp.RPP_WANT_PAIRS | rpp.RPP_NO_ENCLOSING_RADIUS
    scans = None
    monkeypatch.setenv("RPP_COUNT_SCANS", "1")
    for grp in SPARSE_GROUPS:
        for unfused in ("0", "1"):
            if unfused == "0" and grp < 100:
                continue  # the single-phase forms always run apart
            monkeypatch.setenv("RPP_APPARENT_GROUP", str(grp))
            monkeypatch.setenv("RPP_SPARSE_FUSED", "0" if unfused == "1" else "1")
            g = rpp.barcodes(d, maxdim, thr, flags=f)
            for p in range(1, maxdim + 1):
                gs = set(zip(g.pairs[p][0].tolist(), g.pairs[p][1].tolist()))
                es = set(zip(red[p]["sigma"].tolist(), red[p]["tau"].tolist()))
                assert gs == es, (name, grp, unfused, p)
                # two-phase forms above dimension 1 run inside the enumeration
                fused = grp >= 100 and p >= 2 and unfused == "0"
                assert g.stats[p]["apparent_group"] == -(grp + (1000 if fused else 0))
            sc = [g.stats[p]["n_scanned"] for p in range(1, maxdim + 1)]
            if scans is None:
                scans = sc
            assert sc == scans, (name, grp, unfused)


@pytest.mark.parametrize("waves,search", [("1", "0"), ("6", "0"), ("8", "0"), ("5", "1")])
def test_fused_sparse_kernel_occupancy_forms_match_oracle(rpp, monkeypatch, waves, search):
    """The fused sparse enumeration + apparent kernel compiled for 1 (the
    compiler's choice), 6 or 8 waves per SIMD instead of the default 5
    (registers spilled to reach them), and with each wave
    searching the clearing set itself instead of reading its precomputed
    position: the oracle's pairs and the default form's scan tally."""
    f = rpp.RPP_FORCE_SPARSE | rpp.RPP_WANT_PAIRS | rpp.RPP_NO_ENCLOSING_RADIUS
    monkeypatch.setenv("RPP_COUNT_SCANS", "1")
    monkeypatch.setenv("RPP_SPARSE_FUSED", "1")
    monkeypatch.delenv("RPP_APPARENT_GROUP", raising=False)
    for name, d, n, maxdim, thr in SPARSE_CASES[::3]:
        red = oracle.reduce(d, n, maxdim, thr, clearing=n > 33)
        monkeypatch.delenv("RPP_EXT_APP_WAVES", raising=False)
        monkeypatch.delenv("RPP_NO_CLEAR_POS", raising=False)
        base = rpp.barcodes(d, maxdim, thr, flags=f)
        monkeypatch.setenv("RPP_EXT_APP_WAVES", waves)
        monkeypatch.setenv("RPP_NO_CLEAR_POS", search)
        g = rpp.barcodes(d, maxdim, thr, flags=f)
        for p in range(1, maxdim + 1):
            gs = set(zip(g.pairs[p][0].tolist(), g.pairs[p][1].tolist()))
            es = set(zip(red[p]["sigma"].tolist(), red[p]["tau"].tolist()))
            assert gs == es, (name, waves, p)
            assert g.stats[p]["n_scanned"] == base.stats[p]["n_scanned"], (name, waves, p)


@pytest.mark.parametrize("search", ["0", "1"])
def test_sparse_scatter_clearing_positions_match_oracle(rpp, monkeypatch, search):
    """The sparse extension scatter with each prefix's place in the clearing
    set read from the precomputed positions (default) or searched by the
    wave itself (RPP_NO_CLEAR_POS=1): the oracle's pairs, and the same kept
    and cleared counts."""
    f = rpp.RPP_FORCE_SPARSE | rpp.RPP_WANT_PAIRS | rpp.RPP_NO_ENCLOSING_RADIUS
    monkeypatch.delenv("RPP_SPARSE_FUSED", raising=False)
    for name, d, n, maxdim, thr in SPARSE_CASES:
        red = oracle.reduce(d, n, maxdim, thr, clearing=n > 33)
        monkeypatch.setenv("RPP_NO_CLEAR_POS", search)
        g = rpp.barcodes(d, maxdim, thr, flags=f)
        monkeypatch.setenv("RPP_NO_CLEAR_POS", "1" if search == "0" else "0")
        h = rpp.barcodes(d, maxdim, thr, flags=f)
        for p in range(1, maxdim + 1):
            gs = set(zip(g.pairs[p][0].tolist(), g.pairs[p][1].tolist()))
            es = set(zip(red[p]["sigma"].tolist(), red[p]["tau"].tolist()))
            assert gs == es, (name, search, p)
            for k in ("n_kept", "n_cleared", "n_candidates"):
                assert g.stats[p][k] == h.stats[p][k], (name, search, p, k)


@pytest.mark.parametrize("case", SPARSE_CASES[::2], ids=["rk_" + c[0] for c in SPARSE_CASES[::2]])
def test_rank_coded_host_keys_match_oracle(rpp, case, monkeypatch):
    """Sparse path with the host reduction on rank-coded diameters and
    64-bit rank keys (taken by default only where cofacet indices pass
    2^32, forced here on small inputs): the oracle's bars and pairs."""
    name, d, n, maxdim, thr = case
    monkeypatch.setenv("RPP_RANK_CODING", "1")
    monkeypatch.setenv("RPP_RANK_KEYS", "1")
    got = rpp.barcodes(d, maxdim, thr, flags=rpp.RPP_FORCE_SPARSE)
    assert_bars_equal(got.bars, _oracle_bars(d, n, maxdim, thr), name)
    f = rpp.RPP_FORCE_SPARSE | rpp.RPP_WANT_PAIRS | rpp.RPP_NO_ENCLOSING_RADIUS
    g = rpp.barcodes(d, maxdim, thr, flags=f | rpp.RPP_WANT_CRITICAL_EDGES)
    red = oracle.reduce(d, n, maxdim, thr, clearing=n > 33)
    for p in range(1, maxdim + 1):
        gs = set(zip(g.pairs[p][0].tolist(), g.pairs[p][1].tolist()))
        es = set(zip(red[p]["sigma"].tolist(), red[p]["tau"].tolist()))
        assert gs == es, (name, p)


def test_sparse_and_dense_paths_agree_on_maxdim3(rpp):
    d = w.condensed_from_points(w.noisy_torus_points(60, 77))
    thr = float(np.quantile(d, 0.2))
    a = rpp.barcodes(d, 3, thr, flags=rpp.RPP_FORCE_DENSE)
    b = rpp.barcodes(d, 3, thr, flags=rpp.RPP_FORCE_SPARSE)
    assert_bars_equal(a.bars, b.bars, "dense vs sparse")
    assert_bars_equal(a.bars, oracle.barcodes(d, 60, 3, thr, clearing=True), "vs oracle")


def _golden_module():
    import importlib.util
    spec = importlib.util.spec_from_file_location("make_golden",
                                                  os.path.join(GOLDEN, "make_golden.py"))
    mg = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mg)
    return mg


def _golden(name):
    return _golden_module().read(os.path.join(GOLDEN, name + ".bars.txt"))


def test_sphere4096_matches_stored_oracle(rpp):
    """4096 points on the unit sphere + noise 0.01, dims 0-2, threshold 0.4
    (sparse path): against the oracle's stored barcodes."""
    import hashlib
    head, exp = _golden("sphere4096")
    cfg = w.WORKLOADS["sphere4096"]
    d = cfg["build"]()
    assert hashlib.sha256(d.tobytes()).hexdigest() == head["sha256"], "input generator drifted"
    got = rpp.barcodes(d, cfg["maxdim"], cfg["threshold"])
    assert_bars_equal(got.bars, exp, "sphere4096")
    for p in range(3):
        assert got.stats[p]["n_simplices"] == head["dims"][p]["simplices"]
        assert got.stats[p]["n_apparent"] + got.stats[p]["n_host_pairs"] == head["dims"][p]["pairs"]


def test_sphere4096_dim3_matches_stored_oracle(rpp):
    """The same sphere with dimension 3 (2.1e8 tetrahedra under the
    threshold, cofacet indices beyond 2^32): against the oracle's stored
    barcodes and per-dimension simplex and pair counts."""
    import hashlib
    head, exp = _golden("sphere4096d3")
    cfg = w.WORKLOADS["sphere4096d3"]
    d = cfg["build"]()
    assert hashlib.sha256(d.tobytes()).hexdigest() == head["sha256"], "input generator drifted"
    print("case sphere4096d3", flush=True)
    got = rpp.barcodes(d, cfg["maxdim"], cfg["threshold"])
    assert_bars_equal(got.bars, exp, "sphere4096d3")
    for p in range(4):
        assert got.stats[p]["n_simplices"] == head["dims"][p]["simplices"]
        assert got.stats[p]["n_apparent"] + got.stats[p]["n_host_pairs"] == head["dims"][p]["pairs"]


# ---------------------------------------------------------------------------
# Dimension-1 apparent fraction of random orders (the paper's random
# distance-matrix experiments): every C(n0,2) edge, no threshold.
# ---------------------------------------------------------------------------
def test_apparent_count_matches_pairs_and_oracle(rpp):
    d = w.random_permutation_metric(60, 11)
    s, t, ncols = rpp.apparent_pairs(d, 1)
    k, ncols2, st = rpp.apparent_count(d, 1)
    es, et = oracle.apparent_pairs(d, 60, 1)
    assert k == len(s) == len(es) and ncols == ncols2 == 60 * 59 // 2
    assert np.array_equal(s, es) and np.array_equal(t, et)
    assert st["n_kept"] == ncols and st["n_apparent"] == k
    assert st["apparent_group"] >= 1


def test_random_order_1500_matches_oracle_with_adaptive_lanes(rpp):
    """1.1e6 edges, large enough for the lanes-per-column probe: the pairs
    equal the oracle's (stored by tests/golden/make_golden.py as a count and
    a SHA-256 of the pair arrays), whatever group size the probe picked."""
    mg = _golden_module()
    g = mg.read_perm(os.path.join(GOLDEN, "perm1500.apparent.txt"))
    n0 = g["n0"]
    d = w.random_permutation_metric(n0, g["seed"])
    assert hashlib.sha256(d.tobytes()).hexdigest() == g["input_sha256"]
    s, t, ncols = rpp.apparent_pairs(d, 1)
    assert ncols == g["edges"]
    assert len(s) == g["pairs"]
    assert mg.pair_digest(s, t) == g["pairs_sha256"]
    _, _, st = rpp.apparent_count(d, 1)
    assert st["apparent_group"] in (8, 16, 32, 64)


def test_random_order_apparent_fraction_10000(rpp):
    """The paper reports an average dimension-1 apparent fraction of
    0.991127743 at 10000 points (random orders of the C(n0,2) edge lengths,
    averaged over samples, with very low variance); one sample must land
    within 1e-3 of it and below the upper bound (n0-2)/n0 of Theorem 1."""
    n0 = 10000
    d = w.random_permutation_metric(n0, 1006)
    k, ncols, _ = rpp.apparent_count(d, 1)
    frac = k / ncols
    assert ncols == n0 * (n0 - 1) // 2
    assert frac <= (n0 - 2) / n0
    assert abs(frac - 0.991127743) < 1e-3, frac


def test_greedy_assignment_pairs_are_its_picks(rpp):
    """Greedy deterministic distance assignment (an adversarial input, about
    half the edges apparent): the GPU's apparent pairs are exactly the edges
    the construction took while triangles remained."""
    n = 150
    order, picks = w.greedy_assignment_order(n)
    d = w.greedy_assignment_metric(n)
    s, t, ncols = rpp.apparent_pairs(d, 1)
    assert ncols == n * (n - 1) // 2
    assert len(s) == picks
    assert set(s.tolist()) == set(order[:picks])
    assert picks / ncols >= 1.0 / 3.0
