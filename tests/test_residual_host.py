"""Host residual reduction (csrc/residual.cpp) on the CPU, through a test
driver that builds the GPU stages' hand-off by brute force: every schedule
-- plain, with a speculative budget, the overlapped one that drops the
previous dimension's host pivots instead of clearing them, and the same with
those pivots known only after the reduction has started -- gives the
oracle's persistence pairs and essential classes exactly, with either way of
adding a host pivot column: its reduced column (reduction-matrix technique)
or its unreduced coboundary (oblivious reduction, the paper's lemma on
oblivious reduction)."""
import os
import subprocess
import tempfile

import numpy as np
import pytest

import oracle
import workloads as w

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.fixture(scope="module")
def driver():
    out = os.path.join(tempfile.mkdtemp(prefix="rpp_resdrv_"), "residual_driver")
    cmd = ["g++", "-O2", "-std=c++17", "-pthread", "-o", out,
           os.path.join(HERE, "host", "residual_driver.cpp"),
           os.path.join(ROOT, "paper_2003_07989_amd", "csrc", "residual.cpp")]
    subprocess.run(cmd, check=True)
    return out


def _run(driver, d, n, maxdim, thr, mode, with_additions=False, env=None):
    with tempfile.NamedTemporaryFile(suffix=".f32", delete=False) as f:
        np.ascontiguousarray(d, dtype=np.float32).tofile(f)
        path = f.name
    try:
        r = subprocess.run([driver, path, str(n), str(maxdim), repr(float(thr)), str(mode)],
                           check=True, capture_output=True, text=True,
                           env=dict(os.environ, **(env or {})))
    finally:
        os.unlink(path)
    pairs = {p: set() for p in range(1, maxdim + 1)}
    ess = {p: set() for p in range(1, maxdim + 1)}
    adds = {}
    for line in r.stdout.splitlines():
        t = line.split()
        if t[0] == "P":
            pairs[int(t[1])].add((int(t[2]), int(t[3])))
        elif t[0] == "E":
            ess[int(t[1])].add(int(t[2]))
        else:
            adds[int(t[1])] = int(t[2])
    if with_additions:
        return pairs, ess, adds
    return pairs, ess


def _expected(d, n, maxdim, thr):
    red = oracle.reduce(d, n, maxdim, thr, clearing=True)
    pairs = {p: set(zip(red[p]["sigma"].tolist(), red[p]["tau"].tolist()))
             for p in range(1, maxdim + 1)}
    ess = {p: set(red[p]["zero_sigma"].tolist()) for p in range(1, maxdim + 1)}
    return pairs, ess


CASES = [
    ("torus40", lambda: w.condensed_from_points(w.noisy_torus_points(40, 31)), 40, 2, np.inf),
    ("circle48", lambda: w.condensed_from_points(w.noisy_circle_points(48, seed=5)), 48, 1,
     np.inf),
    ("perm24", lambda: w.random_permutation_metric(24, 8), 24, 2, np.inf),
    ("ties22", lambda: w.random_integer_metric(22, 9, vmax=3), 22, 2, np.inf),
    ("square30_thr", lambda: w.condensed_from_points(w.uniform_square_points(30, 4)), 30, 2,
     0.35),
]


@pytest.mark.parametrize("name,build,n,maxdim,thr", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("mode", [0, 1, 2, 3, 11, 4, 6, 7, 16, 19, 80, 83],
                         ids=["plain", "budget", "overlap", "late-drops", "late-drops-nocap",
                              "oblivious", "overlap-oblivious", "late-drops-oblivious",
                              "bitsets", "bitsets-late-drops", "packed", "packed-late-drops"])
def test_schedules_match_oracle(driver, name, build, n, maxdim, thr, mode):
    d = build()
    if np.isinf(thr):
        thr = oracle.enclosing_radius(d, n)  # the library's truncation; bars unchanged
    got_p, got_e = _run(driver, d, n, maxdim, thr, mode)
    exp_p, exp_e = _expected(d, n, maxdim, thr)
    for p in range(1, maxdim + 1):
        assert got_p[p] == exp_p[p], (name, mode, p)
        assert got_e[p] == exp_e[p], (name, mode, p)


def test_oblivious_additions_differ_where_host_pivots_are_reduced(driver):
    """The two ways of adding a host pivot column differ in work, not in the
    result: on an input whose host pivot columns needed additions of their
    own, the oblivious form (D_k) makes more additions than adding the kept
    reduced columns (R_k), and the pairs are the same."""
    d = w.random_permutation_metric(40, 3)
    thr = oracle.enclosing_radius(d, 40)
    rm_p, rm_e, rm_a = _run(driver, d, 40, 2, thr, 0, with_additions=True)
    ob_p, ob_e, ob_a = _run(driver, d, 40, 2, thr, 4, with_additions=True)
    assert rm_p == ob_p and rm_e == ob_e
    assert sum(ob_a.values()) > sum(rm_a.values()), (ob_a, rm_a)


@pytest.mark.parametrize("mode", [0, 3, 16, 19], ids=["plain", "late-drops", "bitsets",
                                                      "bitsets-late-drops"])
def test_wide_keys_match_oracle(driver, mode):
    """The 128-bit key path (cofacet indices past 2^32, as on the 4096-point
    sphere), forced on small inputs: the same pairs and classes."""
    for name, build, n, maxdim, thr in CASES:
        d = build()
        if np.isinf(thr):
            thr = oracle.enclosing_radius(d, n)
        got_p, got_e = _run(driver, d, n, maxdim, thr, mode, env={"RPP_WIDE_KEYS": "1"})
        exp_p, exp_e = _expected(d, n, maxdim, thr)
        for p in range(1, maxdim + 1):
            assert got_p[p] == exp_p[p], (name, mode, p)
            assert got_e[p] == exp_e[p], (name, mode, p)


@pytest.mark.parametrize("mode", [32, 35, 48, 51, 115], ids=["ranks", "ranks-late-drops",
                                                           "ranks-bitsets",
                                                           "ranks-bitsets-late-drops",
                                                           "ranks-packed-late-drops"])
def test_rank_coded_keys_match_oracle(driver, mode):
    """Diameters replaced by the ranks of the distinct edge lengths, and
    keys that pack the rank above a cofacet-index field only as wide as the
    largest index (the layout that gives 64-bit keys where indices pass
    2^32): the same pairs and classes."""
    for name, build, n, maxdim, thr in CASES:
        d = build()
        if np.isinf(thr):
            thr = oracle.enclosing_radius(d, n)
        got_p, got_e = _run(driver, d, n, maxdim, thr, mode, env={"RPP_RANK_KEYS": "1"})
        exp_p, exp_e = _expected(d, n, maxdim, thr)
        for p in range(1, maxdim + 1):
            assert got_p[p] == exp_p[p], (name, mode, p)
            assert got_e[p] == exp_e[p], (name, mode, p)


@pytest.mark.parametrize("heap", ["1", "0"], ids=["slot-queue", "radix-heap"])
@pytest.mark.parametrize("streams", [1, 3])
@pytest.mark.parametrize("mode,env", [(0, None), (3, None), (4, None), (7, None), (83, None),
                                      (3, {"RPP_WIDE_KEYS": "1"}),
                                      (115, {"RPP_RANK_KEYS": "1"})],
                         ids=["plain", "late-drops", "oblivious", "late-drops-oblivious",
                              "packed-late-drops", "wide-keys", "ranks-packed-late-drops"])
def test_radix_columns_match_oracle(driver, mode, env, streams, heap):
    """Columns that switch from the stream heap to a bucket structure (the
    slot queue over the keys' top bits, or the radix heap) after `streams`
    added coboundaries (normally only long chains such as an essential
    class's do): with every column switching at once or after a few
    additions, on every key layout, and with the oblivious form (whose
    unreduced additions can lie below the column's low: below the table, or
    re-basing the buckets), the same pairs and classes."""
    for name, build, n, maxdim, thr in CASES:
        d = build()
        if np.isinf(thr):
            thr = oracle.enclosing_radius(d, n)
        e = dict(env or {}, RPP_RADIX_STREAMS=str(streams), RPP_SLOT_HEAP=heap)
        got_p, got_e = _run(driver, d, n, maxdim, thr, mode, env=e)
        exp_p, exp_e = _expected(d, n, maxdim, thr)
        for p in range(1, maxdim + 1):
            assert got_p[p] == exp_p[p], (name, mode, streams, heap, p)
            assert got_e[p] == exp_e[p], (name, mode, streams, heap, p)


@pytest.mark.parametrize("slice_,polls", [(0, 5), (1, 5), (1, 100000), (3, 100000),
                                          (256, 100000)])
@pytest.mark.parametrize("mode", [3, 7, 19, 83], ids=["late-drops", "late-drops-oblivious",
                                                      "bitsets-late-drops",
                                                      "packed-late-drops"])
def test_parked_slices_match_oracle(driver, mode, slice_, polls):
    """While the dropped columns are unknown and every other column waits
    on them, the parked column nearest the frontier goes on `slice_`
    additions at a time (0: parked columns wait idle); with the gate opening
    after a few polls or only once nothing else can run, the same pairs and
    classes -- a column the gate then drops ends as no pair and no class,
    whatever its slices did."""
    for name, build, n, maxdim, thr in CASES:
        d = build()
        if np.isinf(thr):
            thr = oracle.enclosing_radius(d, n)
        e = {"RPP_TEST_PARK_SLICE": str(slice_), "RPP_TEST_GATE_POLLS": str(polls)}
        got_p, got_e = _run(driver, d, n, maxdim, thr, mode, env=e)
        exp_p, exp_e = _expected(d, n, maxdim, thr)
        for p in range(1, maxdim + 1):
            assert got_p[p] == exp_p[p], (name, mode, slice_, polls, p)
            assert got_e[p] == exp_e[p], (name, mode, slice_, polls, p)


@pytest.mark.parametrize("ratio", ["0.01", "1", "4"])
@pytest.mark.parametrize("mode", [0, 3, 19, 83], ids=["plain", "late-drops", "bitsets-late-drops",
                                                      "packed-late-drops"])
def test_keep_ratio_matches_oracle(driver, mode, ratio):
    """The reduction-matrix form choosing per pivot column between its kept
    R_k and its coboundary D_k (D_k when R_k holds more than `ratio` times
    D_k's keys; 0.01 takes D_k almost always, a mixed choice in between):
    the same pairs and classes as the oracle, whatever the mix."""
    for name, build, n, maxdim, thr in CASES:
        d = build()
        if np.isinf(thr):
            thr = oracle.enclosing_radius(d, n)
        got_p, got_e = _run(driver, d, n, maxdim, thr, mode, env={"RPP_TEST_KEEP_RATIO": ratio})
        exp_p, exp_e = _expected(d, n, maxdim, thr)
        for p in range(1, maxdim + 1):
            assert got_p[p] == exp_p[p], (name, mode, ratio, p)
            assert got_e[p] == exp_e[p], (name, mode, ratio, p)


# Look-ahead helpers on every radix column from its first addition; with
# RPP_TEST_CHAIN_SETTLE the column waits for the helpers' answers, so that it
# takes handed-over coboundaries even on small inputs.
_LOOKAHEAD = {"RPP_RADIX_STREAMS": "1", "RPP_CHAIN_AFTER": "0"}
# the void of a 120-point sphere survives radius 1.0: an essential class
# whose column is a chain of apparent additions, as on the large sphere
SPHERE = ("sphere120_thr", lambda: w.condensed_from_points(w.noisy_sphere_points(120, seed=7)),
          120, 2, 1.0)


@pytest.mark.parametrize("settle", ["0", "1"], ids=["racing", "settled"])
@pytest.mark.parametrize("helpers", ["1", "3"])
@pytest.mark.parametrize("mode,env", [(0, None), (3, None), (7, None), (11, None), (15, None),
                                      (19, None), (83, None), (91, None),
                                      (123, {"RPP_RANK_KEYS": "1"})],
                         ids=["plain", "late-drops", "late-drops-oblivious", "never-parked",
                              "never-parked-oblivious", "bitsets-late-drops",
                              "packed-late-drops", "packed-never-parked",
                              "ranks-packed-never-parked"])
def test_chain_lookahead_matches_oracle(driver, mode, env, helpers, settle):
    """Helper threads that look ahead of a long column (its next lows'
    apparent partners and their coboundaries, handed over when the column
    reaches them): the oracle's pairs and classes, and the same number of
    additions per dimension as without helpers (a handed-over coboundary is
    the one the column would have generated)."""
    for name, build, n, maxdim, thr in CASES + [SPHERE]:
        d = build()
        if np.isinf(thr):
            thr = oracle.enclosing_radius(d, n)
        e = dict(env or {}, RPP_TEST_CHAIN_SETTLE=settle, **_LOOKAHEAD)
        got_p, got_e, got_a = _run(driver, d, n, maxdim, thr, mode, with_additions=True,
                                   env=dict(e, RPP_CHAIN_HELPERS=helpers))
        _, _, alone_a = _run(driver, d, n, maxdim, thr, mode, with_additions=True,
                             env=dict(e, RPP_CHAIN_HELPERS="0"))
        exp_p, exp_e = _expected(d, n, maxdim, thr)
        for p in range(1, maxdim + 1):
            assert got_p[p] == exp_p[p], (name, mode, helpers, p)
            assert got_e[p] == exp_e[p], (name, mode, helpers, p)
        assert got_a == alone_a, (name, mode, helpers)


def test_chain_lookahead_hands_over(driver):
    """The settled look-ahead on the sphere's essential chain does hand
    coboundaries over (what the tests above then check is the hand-over
    path, not only the column's own)."""
    name, build, n, maxdim, thr = SPHERE
    with tempfile.NamedTemporaryFile(suffix=".f32", delete=False) as f:
        np.ascontiguousarray(build(), dtype=np.float32).tofile(f)
        path = f.name
    try:
        r = subprocess.run([driver, path, str(n), str(maxdim), repr(float(thr)), "91"],
                           check=True, capture_output=True, text=True,
                           env=dict(os.environ, RPP_TRACE="1", RPP_CHAIN_HELPERS="2",
                                    RPP_TEST_CHAIN_SETTLE="1", **_LOOKAHEAD))
    finally:
        os.unlink(path)
    handed = [int(line.split("look-ahead:")[1].split(",")[1].split()[0])
              for line in r.stderr.splitlines() if "look-ahead:" in line]
    assert handed and max(handed) > 100, r.stderr[-2000:]


@pytest.fixture(scope="module")
def tsan_driver():
    """The driver and reduction built with ThreadSanitizer (host code)."""
    out = os.path.join(tempfile.mkdtemp(prefix="rpp_resdrv_tsan_"), "residual_driver")
    cmd = ["g++", "-O1", "-g", "-std=c++17", "-pthread", "-fsanitize=thread", "-o", out,
           os.path.join(HERE, "host", "residual_driver.cpp"),
           os.path.join(ROOT, "paper_2003_07989_amd", "csrc", "residual.cpp")]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        pytest.skip("no thread sanitizer runtime: " + r.stderr[-300:])
    return out


@pytest.mark.parametrize("mode,env", [(11, dict(_LOOKAHEAD, RPP_CHAIN_HELPERS="3",
                                                RPP_TEST_CHAIN_SETTLE="1")),
                                      (91, dict(_LOOKAHEAD, RPP_CHAIN_HELPERS="3",
                                                RPP_TEST_CHAIN_SETTLE="1")),
                                      (91, dict(_LOOKAHEAD, RPP_CHAIN_HELPERS="3")),
                                      (3, None),
                                      (3, {"RPP_TEST_PARK_SLICE": "1",
                                           "RPP_TEST_GATE_POLLS": "100000"})],
                         ids=["lookahead-settled", "lookahead-packed-settled",
                              "lookahead-packed-racing", "late-drops", "park-slices"])
def test_host_reduction_is_race_free(tsan_driver, mode, env):
    """The threaded schedules (worker pool, overlapped gate, look-ahead
    helpers with their sequence-locked hand-over) under ThreadSanitizer: no
    report, and the oracle's pairs."""
    cases = (SPHERE,) if env else (CASES[0], CASES[4])
    for name, build, n, maxdim, thr in cases:
        d = build()
        if np.isinf(thr):
            thr = oracle.enclosing_radius(d, n)
        e = dict(env or {}, TSAN_OPTIONS="halt_on_error=1:abort_on_error=1")
        got_p, got_e = _run(tsan_driver, d, n, maxdim, thr, mode, env=e)
        exp_p, exp_e = _expected(d, n, maxdim, thr)
        for p in range(1, maxdim + 1):
            assert got_p[p] == exp_p[p], (name, mode, p)
            assert got_e[p] == exp_e[p], (name, mode, p)


@pytest.fixture(scope="module")
def sanitized_driver():
    """The same driver and reduction built with AddressSanitizer and
    UndefinedBehaviorSanitizer (host code only; any report aborts)."""
    out = os.path.join(tempfile.mkdtemp(prefix="rpp_resdrv_asan_"), "residual_driver")
    cmd = ["g++", "-O1", "-g", "-std=c++17", "-pthread", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-o", out,
           os.path.join(HERE, "host", "residual_driver.cpp"),
           os.path.join(ROOT, "paper_2003_07989_amd", "csrc", "residual.cpp")]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        pytest.skip("no sanitizer runtime: " + r.stderr[-300:])
    return out


@pytest.mark.parametrize("mode,env", [(0, None), (3, None), (19, None), (7, None),
                                      (51, {"RPP_RANK_KEYS": "1"}),
                                      (115, {"RPP_RANK_KEYS": "1"}),
                                      (3, {"RPP_WIDE_KEYS": "1"}),
                                      (7, {"RPP_RADIX_STREAMS": "2"}),
                                      (3, {"RPP_TEST_PARK_SLICE": "1",
                                           "RPP_TEST_GATE_POLLS": "100000"}),
                                      (3, {"RPP_RADIX_STREAMS": "2", "RPP_WIDE_KEYS": "1"}),
                                      (91, dict(_LOOKAHEAD, RPP_CHAIN_HELPERS="3",
                                                RPP_TEST_CHAIN_SETTLE="1")),
                                      (7, {"RPP_RADIX_STREAMS": "2", "RPP_SLOT_HEAP": "0"}),
                                      (3, {"RPP_RADIX_STREAMS": "2", "RPP_WIDE_KEYS": "1",
                                           "RPP_SLOT_HEAP": "0"})],
                         ids=["plain", "late-drops", "bitsets-late-drops",
                              "late-drops-oblivious", "ranks-bitsets-late-drops",
                              "ranks-packed-late-drops", "wide-keys", "radix-oblivious",
                              "park-slices", "radix-wide-keys", "lookahead",
                              "radix-heap-oblivious", "radix-heap-wide-keys"])
def test_host_reduction_is_sanitizer_clean(sanitized_driver, mode, env):
    """Every schedule and key layout of the host reduction under ASan and
    UBSan, on a dense and a thresholded input: no report, and the oracle's
    pairs."""
    for name, build, n, maxdim, thr in (CASES[0], CASES[4]):
        d = build()
        if np.isinf(thr):
            thr = oracle.enclosing_radius(d, n)
        e = dict(env or {}, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
                 UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
        got_p, got_e = _run(sanitized_driver, d, n, maxdim, thr, mode, env=e)
        exp_p, exp_e = _expected(d, n, maxdim, thr)
        for p in range(1, maxdim + 1):
            assert got_p[p] == exp_p[p], (name, mode, p)
            assert got_e[p] == exp_e[p], (name, mode, p)
