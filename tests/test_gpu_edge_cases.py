"""Parity of the HIP path with the oracle on the branches and inputs that the
main parity cases do not reach.

- The dense enumeration's second output path: outputs for every candidate
  are allocated before counting when that takes at most 1 GiB; larger
  inputs (a serving request of ~700 points at dimension 2, H0 past ~13,400
  points) count first, read the kept count back and size the outputs
  exactly.  RPP_ENUM_UPFRONT_MAX_BYTES=0 sends every input down that path.
- Zero distances: coincident points, and entries written as -0.0 and +0.0,
  on the dense and the sparse path, with and without a threshold and with
  rank-coded host keys.
- A serving request at its real size (703 points, dimensions 0-2, threshold
  at its enclosing radius) against the oracle's stored barcodes, through
  the default path, the server and the read-back branch.

Barcodes are compared bit for bit, persistence pairs as exact sets.
"""
import hashlib
import math
import os

import numpy as np
import pytest

import oracle
import workloads as w
from test_gpu_parity import CASES, GOLDEN, _golden, _golden_module, _oracle_bars, \
    assert_bars_equal

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rpp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2003_07989_amd as m
    m.load()
    return m


# ---------------------------------------------------------------------------
# the dense enumeration's count-then-size path
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("case", CASES, ids=["rb_" + c[0] for c in CASES])
def test_readback_branch_matches_oracle(rpp, monkeypatch, case):
    name, d, n, maxdim, thr = case
    print("case", name, flush=True)
    monkeypatch.setenv("RPP_ENUM_UPFRONT_MAX_BYTES", "0")
    got = rpp.barcodes(d, maxdim, thr, flags=rpp.RPP_FORCE_DENSE)
    assert_bars_equal(got.bars, _oracle_bars(d, n, maxdim, thr), name)
    f = rpp.RPP_FORCE_DENSE | rpp.RPP_WANT_PAIRS | rpp.RPP_NO_ENCLOSING_RADIUS
    g = rpp.barcodes(d, maxdim, thr, flags=f)
    red = oracle.reduce(d, n, maxdim, thr, clearing=n > 33)
    for p in range(1, maxdim + 1):
        gs = set(zip(g.pairs[p][0].tolist(), g.pairs[p][1].tolist()))
        es = set(zip(red[p]["sigma"].tolist(), red[p]["tau"].tolist()))
        assert gs == es, (name, p)
        st = g.stats[p]
        assert st["n_candidates"] == st["n_thresholded"] + st["n_cleared"] + st["n_kept"]


def test_readback_branch_torus400(rpp, monkeypatch):
    head, exp = _golden("torus400")
    d = w.WORKLOADS["torus400"]["build"]()
    monkeypatch.setenv("RPP_ENUM_UPFRONT_MAX_BYTES", "0")
    got = rpp.barcodes(d, 2)
    assert_bars_equal(got.bars, exp, "torus400, read-back branch")


@pytest.mark.parametrize("n,p", [(60, 1), (60, 2), (30, 3), (400, 1)])
def test_readback_branch_theorem1_counts(rpp, monkeypatch, n, p):
    monkeypatch.setenv("RPP_ENUM_UPFRONT_MAX_BYTES", "0")
    s, _, ncols = rpp.apparent_pairs(w.all_equal_metric(n), p)
    assert ncols == math.comb(n, p + 1)
    assert len(s) == math.comb(n - 1, p + 1)
    s, _, _ = rpp.apparent_pairs(w.reverse_lex_metric(n), 1)
    assert len(s) == math.comb(n - 1, 2)


def test_readback_branch_random_order_1500(rpp, monkeypatch):
    mg = _golden_module()
    g = mg.read_perm(os.path.join(GOLDEN, "perm1500.apparent.txt"))
    d = w.random_permutation_metric(g["n0"], g["seed"])
    monkeypatch.setenv("RPP_ENUM_UPFRONT_MAX_BYTES", "0")
    s, t, ncols = rpp.apparent_pairs(d, 1)
    assert ncols == g["edges"] and len(s) == g["pairs"]
    assert mg.pair_digest(s, t) == g["pairs_sha256"]


# ---------------------------------------------------------------------------
# one pass (decoupled look-back) against count + scan + scatter
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("case", CASES[::2], ids=["op_" + c[0] for c in CASES[::2]])
def test_one_pass_enumeration_matches_two_passes(rpp, monkeypatch, case):
    """The one-pass dense enumeration (RPP_ENUM_ONE_PASS=1, taken when
    outputs are sized up front) and the count + scan + scatter passes: the
    same pairs and every per-dimension count; bars equal the oracle's."""
    name, d, n, maxdim, thr = case
    f = rpp.RPP_FORCE_DENSE | rpp.RPP_WANT_PAIRS | rpp.RPP_NO_ENCLOSING_RADIUS
    monkeypatch.setenv("RPP_ENUM_ONE_PASS", "1")
    a = rpp.barcodes(d, maxdim, thr, flags=f)
    monkeypatch.delenv("RPP_ENUM_ONE_PASS", raising=False)
    b = rpp.barcodes(d, maxdim, thr, flags=f)
    assert_bars_equal(a.bars, _oracle_bars(d, n, maxdim, thr), name)
    for p in range(1, maxdim + 1):
        assert set(zip(*map(list, a.pairs[p]))) == set(zip(*map(list, b.pairs[p]))), (name, p)
        for k in ("n_candidates", "n_thresholded", "n_cleared", "n_kept", "n_apparent"):
            assert a.stats[p][k] == b.stats[p][k], (name, p, k)


def test_one_pass_enumeration_torus400_and_theorem1(rpp, monkeypatch):
    monkeypatch.setenv("RPP_ENUM_ONE_PASS", "1")
    head, exp = _golden("torus400")
    got = rpp.barcodes(w.WORKLOADS["torus400"]["build"](), 2)
    assert_bars_equal(got.bars, exp, "torus400, one pass")
    for n, p in ((60, 2), (400, 1), (30, 3)):
        s, _, ncols = rpp.apparent_pairs(w.all_equal_metric(n), p)
        assert ncols == math.comb(n, p + 1)
        assert len(s) == math.comb(n - 1, p + 1)


# ---------------------------------------------------------------------------
# zero distances
# ---------------------------------------------------------------------------
def _zero_cases():
    c = []
    for n, seed, ndup in ((24, 3, 4), (40, 5, 8)):
        d = w.condensed_from_points(w.duplicate_points_cloud(n, seed, ndup))
        c.append(("dup%d" % n, d, n, 2))
    c.append(("dup12", w.condensed_from_points(w.duplicate_points_cloud(12, 9, 3)), 12, 3))
    for n, seed in ((16, 21), (30, 22)):
        c.append(("zeros%d" % n, w.signed_zero_metric(n, seed, vmax=3), n, 3 if n <= 16 else 2))
    c.append(("zeros45", w.signed_zero_metric(45, 23, vmax=5, zero_frac=0.05), 45, 2))
    # a cluster of 6 copies of one point among distinct ones
    x = w.uniform_square_points(30, 24)
    x[10:16] = x[3]
    c.append(("cluster30", w.condensed_from_points(x), 30, 2))
    return c


ZERO_CASES = _zero_cases()


@pytest.mark.parametrize("mode", ["dense", "sparse", "sparse_ranks"])
@pytest.mark.parametrize("thr_q", [None, 0.5])
@pytest.mark.parametrize("case", ZERO_CASES, ids=[c[0] for c in ZERO_CASES])
def test_zero_distances_match_oracle(rpp, monkeypatch, case, thr_q, mode):
    name, d, n, maxdim = case
    assert np.any(d == 0)
    thr = math.inf if thr_q is None else float(np.quantile(d, thr_q))
    print("case", name, thr, mode, flush=True)
    flags = rpp.RPP_FORCE_DENSE if mode == "dense" else rpp.RPP_FORCE_SPARSE
    if mode == "sparse_ranks":
        monkeypatch.setenv("RPP_RANK_CODING", "1")
        monkeypatch.setenv("RPP_RANK_KEYS", "1")
    got = rpp.barcodes(d, maxdim, thr, flags=flags)
    assert_bars_equal(got.bars, _oracle_bars(d, n, maxdim, thr), name)
    for b, dd in got.bars:
        assert np.all(dd > b) and not np.any(np.signbit(b)) and not np.any(np.signbit(dd))
    g = rpp.barcodes(d, maxdim, thr,
                     flags=flags | rpp.RPP_WANT_PAIRS | rpp.RPP_NO_ENCLOSING_RADIUS)
    red = oracle.reduce(d, n, maxdim, thr, clearing=n > 33)
    assert set(g.pairs[0][1].tolist()) == set(red[0]["tau"].tolist())
    for p in range(1, maxdim + 1):
        gs = set(zip(g.pairs[p][0].tolist(), g.pairs[p][1].tolist()))
        es = set(zip(red[p]["sigma"].tolist(), red[p]["tau"].tolist()))
        assert gs == es, (name, p)


@pytest.mark.parametrize("group", [8, 16, 64, 408, 10408, 20008, 20016, 20408])
@pytest.mark.parametrize("p", [1, 2, 3])
@pytest.mark.parametrize("case", ZERO_CASES[:5], ids=[c[0] for c in ZERO_CASES[:5]])
def test_zero_distances_apparent_kernels_match_definition(rpp, monkeypatch, case, p, group):
    """Every dense apparent-kernel form on zero diameters (equal-diameter
    cofacets and facets at 0)."""
    name, d, n, _ = case
    monkeypatch.setenv("RPP_APPARENT_GROUP", str(group))
    for thr in (math.inf, float(np.quantile(d, 0.6))):
        s, t, ncols = rpp.apparent_pairs(d, p, thr)
        es, et = oracle.apparent_pairs(d, n, p, thr)
        assert ncols == oracle.count_simplices(d, n, p, thr)
        assert set(zip(s.tolist(), t.tolist())) == set(zip(es.tolist(), et.tolist())), thr


def test_duplicate_points_h0(rpp):
    """Coincident points merge at 0, which is not reported: n - #copies
    finite H0 bars plus one essential, and every finite bar positive."""
    x = w.duplicate_points_cloud(50, 11, 7)
    d = w.condensed_from_points(x)
    distinct = len({tuple(r) for r in x.tolist()})
    got = rpp.barcodes(d, 1)
    b, dd = got.bars[0]
    assert int(np.sum(np.isinf(dd))) == 1
    assert len(b) == distinct
    assert np.all(dd[np.isfinite(dd)] > 0)


# ---------------------------------------------------------------------------
# a serving request at its real size
# ---------------------------------------------------------------------------
def _mixture448():
    head, exp = _golden("mixture448")
    cfg = w.WORKLOADS["mixture448"]
    d = cfg["build"]()
    assert hashlib.sha256(d.tobytes()).hexdigest() == head["sha256"], "input generator drifted"
    return head, exp, d


def test_mixture448_matches_stored_oracle(rpp):
    """703 points, dims 0-2, no threshold (the library truncates at the
    enclosing radius, the stored answer was computed there): 57.7M triangle
    candidates, past the 1 GiB up-front limit, so the default path counts
    before sizing its outputs."""
    head, exp, d = _mixture448()
    print("case mixture448", flush=True)
    got = rpp.barcodes(d, 2)
    assert got.threshold_used == np.float32(head["threshold"])
    assert_bars_equal(got.bars, exp, "mixture448")
    for p in range(3):
        assert got.stats[p]["n_simplices"] == head["dims"][p]["simplices"]
        assert got.stats[p]["n_apparent"] + got.stats[p]["n_host_pairs"] == \
            head["dims"][p]["pairs"]
    assert got.stats[2]["n_candidates"] * 20 > (1 << 30)


def test_mixture448_served(rpp):
    head, exp, d = _mixture448()
    with rpp.Server(slots=2) as srv:
        small = w.mixture_request(1)
        t0 = srv.submit(small["dist"], small["maxdim"])
        t1 = srv.submit(d, 2)
        got, _, _ = srv.wait(t1)
        srv.wait(t0)
    assert_bars_equal(got.bars, exp, "mixture448 served")


def test_mixture448_upfront_branch(rpp, monkeypatch):
    """The same request with the up-front limit raised past its outputs."""
    head, exp, d = _mixture448()
    monkeypatch.setenv("RPP_ENUM_UPFRONT_MAX_BYTES", str(4 << 30))
    got = rpp.barcodes(d, 2)
    assert_bars_equal(got.bars, exp, "mixture448, up-front outputs")
