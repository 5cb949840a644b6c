"""Batched execution (rpp_barcodes_batch): every cloud's result equals the
single-cloud path and the oracle, with and without graph replay."""
import math

import numpy as np
import pytest

import oracle
import workloads as w

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rpp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2003_07989_amd as m
    m.load()
    return m


def _same(a, b, label=""):
    for p, ((b1, d1), (b2, d2)) in enumerate(zip(a.bars, b.bars)):
        assert np.array_equal(b1.view(np.uint32), b2.view(np.uint32)), (label, p)
        assert np.array_equal(d1.view(np.uint32), d2.view(np.uint32)), (label, p)
    if a.edges is not None and b.edges is not None:
        for p, ((e1, f1), (e2, f2)) in enumerate(zip(a.edges, b.edges)):
            assert np.array_equal(e1, e2) and np.array_equal(f1, f2), (label, p)


def _dev(d):
    import torch
    return torch.from_numpy(np.ascontiguousarray(d, dtype=np.float32)).cuda()


def _mixed():
    clouds = []
    for i, n in enumerate((40, 40, 40, 25, 25, 64, 40)):
        d = w.condensed_from_points(w.noisy_torus_points(n, 1300 + i))
        maxdim = 2 if n <= 40 else 1
        thr = math.inf if i % 3 else float(np.quantile(d, 0.5))
        clouds.append((d, n, maxdim, thr))
    return clouds


@pytest.mark.parametrize("flags_name", ["graph", "eager"])
def test_mixed_batch_matches_single_and_oracle(rpp, flags_name):
    flags = rpp.RPP_WANT_CRITICAL_EDGES
    if flags_name == "eager":
        flags |= rpp.RPP_BATCH_NO_GRAPH
    clouds = _mixed()
    dev = [_dev(d) for d, _, _, _ in clouds]
    out = rpp.barcodes_batch(dev, [c[2] for c in clouds], [c[3] for c in clouds], flags=flags)
    for i, ((d, n, maxdim, thr), r) in enumerate(zip(clouds, out)):
        single = rpp.barcodes_device(dev[i], maxdim, thr,
                                     flags=rpp.RPP_WANT_CRITICAL_EDGES | rpp.RPP_FORCE_DENSE)
        _same(r, single, "cloud %d" % i)
        exp = oracle.barcodes(d, n, maxdim, thr, clearing=True)
        for p in range(maxdim + 1):
            assert np.array_equal(r.bars[p][0].view(np.uint32), exp[p][0].view(np.uint32))
            assert np.array_equal(r.bars[p][1].view(np.uint32), exp[p][1].view(np.uint32))


def test_graph_replays_match_eager(rpp):
    """Replay the captured graph several times, with unrelated eager work and
    synchronisations in between; every replay equals the eager batch."""
    import torch
    clouds = [w.condensed_from_points(w.noisy_circle_points(96, seed=40 + i)) for i in range(12)]
    dev = [_dev(d) for d in clouds]
    ref = rpp.barcodes_batch(dev, 1, flags=rpp.RPP_BATCH_NO_GRAPH)
    other = _dev(w.condensed_from_points(w.uniform_square_points(30, 9)))
    for rep in range(4):
        got = rpp.barcodes_batch(dev, 1)
        rpp.barcodes_device(other, 1)   # eager work between replays
        torch.cuda.synchronize()
        for i in range(len(dev)):
            _same(got[i], ref[i], "replay %d cloud %d" % (rep, i))


def test_batch_of_circles_512(rpp):
    """64 noisy circles of 512 points (FP32 coordinates), dims 0-1."""
    pts, dists = w.noisy_circle_batch(64, 512)
    dev = [_dev(d) for d in dists]
    out = rpp.barcodes_batch(dev, 1, flags=rpp.RPP_WANT_CRITICAL_EDGES)
    for i in range(0, 64, 9):
        single = rpp.barcodes_device(dev[i], 1, flags=rpp.RPP_WANT_CRITICAL_EDGES)
        _same(out[i], single, "circle %d" % i)
    # one cloud against the oracle
    exp = oracle.barcodes(dists[5], 512, 1, clearing=True)
    for p in range(2):
        assert np.array_equal(out[5].bars[p][0].view(np.uint32), exp[p][0].view(np.uint32))
        assert np.array_equal(out[5].bars[p][1].view(np.uint32), exp[p][1].view(np.uint32))


def test_autotuned_batch_matches(rpp):
    clouds = [w.condensed_from_points(w.noisy_torus_points(72, 70 + i)) for i in range(5)]
    dev = [_dev(d) for d in clouds]
    a = rpp.barcodes_batch(dev, 2, flags=rpp.RPP_BATCH_AUTOTUNE)
    b = rpp.barcodes_batch(dev, 2, flags=rpp.RPP_BATCH_NO_GRAPH)
    for i in range(len(dev)):
        _same(a[i], b[i], "tuned %d" % i)
        _same(a[i], rpp.barcodes_device(dev[i], 2), "single %d" % i)


def test_batch_rejects_bad_entries(rpp):
    d = w.condensed_from_points(w.uniform_square_points(20, 1))
    bad = d.copy()
    bad[3] = -1.0
    with pytest.raises(rpp.RppError) as e:
        rpp.barcodes_batch([_dev(d), _dev(bad)], 1)
    assert e.value.code == -2


def test_many_shapes_evict_and_recreate_workspaces(rpp):
    """More distinct batch shapes than the workspace cache holds, then the
    first shape again (its workspace was evicted and is rebuilt): every
    result still equals the single-cloud path."""
    shapes = [20, 21, 22, 23, 24, 25, 26, 20]
    for k, n in enumerate(shapes):
        clouds = [w.condensed_from_points(w.noisy_torus_points(n, 900 + 10 * k + i))
                  for i in range(2)]
        dev = [_dev(d) for d in clouds]
        out = rpp.barcodes_batch(dev, 2, flags=rpp.RPP_BATCH_EXACT_SHAPES)
        for i in range(2):
            _same(out[i], rpp.barcodes_device(dev[i], 2, flags=rpp.RPP_FORCE_DENSE),
                  "shape %d cloud %d" % (n, i))


_ALL_COUNTS = ("n_candidates", "n_simplices", "n_thresholded", "n_cleared", "n_kept",
               "n_apparent", "n_nonapparent", "n_essential", "n_bars")
# counts that do not depend on the schedule (the single-cloud path clears by
# the apparent pivots on the device and drops the host pivots' columns later)
_PATH_FREE = ("n_candidates", "n_simplices", "n_thresholded", "n_essential", "n_bars")


def _stats_equal(a, b, label, keys=_ALL_COUNTS):
    for p in range(len(a.stats)):
        for k in keys:
            assert a.stats[p][k] == b.stats[p][k], (label, p, k)


@pytest.mark.parametrize("maxdim", [1, 2])
def test_shape_bucket_mixed_sizes_match_single_and_oracle(rpp, maxdim):
    """Clouds of 65..128 points share the 128-point bucket (padding vertices
    at infinite distance): bars, critical edges and every per-dimension count
    equal the single-cloud path, and the bars equal the oracle's."""
    sizes = (65, 128, 97, 70, 111, 66) if maxdim == 1 else (65, 90, 77)
    clouds = [w.condensed_from_points(w.noisy_torus_points(n, 4200 + n)) for n in sizes]
    thr = [math.inf, float(np.quantile(clouds[1], 0.3))] + [math.inf] * (len(sizes) - 2)
    dev = [_dev(d) for d in clouds]
    flags = rpp.RPP_WANT_CRITICAL_EDGES
    out = rpp.barcodes_batch(dev, maxdim, thr, flags=flags)
    for i, n in enumerate(sizes):
        single = rpp.barcodes_device(dev[i], maxdim, thr[i], flags=flags | rpp.RPP_FORCE_DENSE)
        _same(out[i], single, "n=%d" % n)
        _stats_equal(out[i], single, "n=%d" % n, _PATH_FREE)
    exact = rpp.barcodes_batch(dev, maxdim, thr, flags=flags | rpp.RPP_BATCH_EXACT_SHAPES)
    for i, n in enumerate(sizes):
        _stats_equal(out[i], exact[i], "n=%d" % n)
    for i in (0, 2):
        exp = oracle.barcodes(clouds[i], sizes[i], maxdim, thr[i], clearing=True)
        for p in range(maxdim + 1):
            assert np.array_equal(out[i].bars[p][0].view(np.uint32), exp[p][0].view(np.uint32))
            assert np.array_equal(out[i].bars[p][1].view(np.uint32), exp[p][1].view(np.uint32))


def test_shape_bucket_replays_with_new_sizes(rpp):
    """The bucket's captured graph replays for a different mix of sizes (the
    sizes live in device memory): each replay equals the exact-shape path."""
    for rep, sizes in enumerate([(129, 150, 192), (180, 131, 160), (192, 192, 129)]):
        clouds = [w.condensed_from_points(w.noisy_circle_points(n, seed=500 + 7 * rep + n))
                  for n in sizes]
        dev = [_dev(d) for d in clouds]
        got = rpp.barcodes_batch(dev, 1)
        ref = rpp.barcodes_batch(dev, 1, flags=rpp.RPP_BATCH_EXACT_SHAPES)
        for i in range(len(sizes)):
            _same(got[i], ref[i], "replay %d n=%d" % (rep, sizes[i]))
            _stats_equal(got[i], ref[i], "replay %d n=%d" % (rep, sizes[i]))


def test_no_radius_infinite_threshold_keeps_exact_shape(rpp):
    """Threshold +inf without the enclosing radius cannot be padded (padding
    edges would be within it): such requests run at their exact size and
    still match the single-cloud path."""
    clouds = [w.condensed_from_points(w.noisy_torus_points(n, 77 + n)) for n in (30, 41)]
    dev = [_dev(d) for d in clouds]
    out = rpp.barcodes_batch(dev, 1, flags=rpp.RPP_NO_ENCLOSING_RADIUS)
    for i in range(2):
        _same(out[i], rpp.barcodes_device(dev[i], 1, flags=rpp.RPP_NO_ENCLOSING_RADIUS |
                                          rpp.RPP_FORCE_DENSE), "cloud %d" % i)


_TUNE_CHILD = r"""
import hashlib, sys
import numpy as np, torch
sys.path.insert(0, sys.argv[1])
import paper_2003_07989_amd as m
import workloads as w
m.load()
dev = [torch.from_numpy(np.ascontiguousarray(
           w.condensed_from_points(w.noisy_torus_points(72, 90 + i)), dtype=np.float32)).cuda()
       for i in range(3)]
flags = m.RPP_BATCH_AUTOTUNE if sys.argv[2] == "tune" else 0
out = m.barcodes_batch(dev, 2, flags=flags)
h = hashlib.sha256()
for r in out:
    for b, d in r.bars:
        h.update(b.view(np.uint32).tobytes()); h.update(d.view(np.uint32).tobytes())
print("digest", h.hexdigest())
"""


def test_tune_cache_persists_across_processes(rpp, tmp_path):
    """RPP_TUNE_CACHE: a process that autotunes writes the chosen launch
    configuration per (n, dimension) to the file; a second process reads it
    back and runs the batch with it; both give the same barcodes."""
    import json
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    cache = tmp_path / "tune.json"
    env = dict(os.environ, RPP_TUNE_CACHE=str(cache))

    def child(mode):
        r = subprocess.run([sys.executable, "-c", _TUNE_CHILD, root, mode], env=env,
                           capture_output=True, text=True, timeout=300)
        assert r.returncode == 0, r.stderr[-2000:]
        return [l for l in r.stdout.splitlines() if l.startswith("digest")][-1]

    first = child("tune")
    table = json.loads(cache.read_text())
    # 72 points share the 128-point shape bucket; one entry per dimension
    assert {"128:1", "128:2"} <= set(table), table
    for code in table.values():
        assert isinstance(code, int) and 0 < code % 100 <= 64, table
    stamp = os.stat(cache).st_mtime_ns
    # asked to tune again, the second process finds both entries and
    # tunes nothing (a tuning run rewrites the file)
    second = child("tune")
    assert first == second
    assert os.stat(cache).st_mtime_ns == stamp
    assert json.loads(cache.read_text()) == table
    assert child("plain") == first
