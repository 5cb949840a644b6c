"""rpp_backward_noalloc (bars staged in the library's fixed device array)
against rpp_backward (library-allocated staging) through the C ABI: the
gradients must be bitwise equal, on two calls in a row, the second with a
smaller input, so that whatever the first call left in the shared array
cannot leak into the second."""
import numpy as np
import pytest

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


def _terms(rpp, x, seed):
    """Critical edges of every bar of dims 0-1 and random bar gradients
    (some zero), as the autograd path would pass them."""
    import torch
    dist = rpp.pdist_device(torch.from_numpy(np.ascontiguousarray(x)).cuda())
    r = rpp.barcodes_device(dist, 1, flags=rpp.RPP_WANT_CRITICAL_EDGES)
    be = np.concatenate([r.edges[p][0] for p in range(2)])
    de = np.concatenate([r.edges[p][1] for p in range(2)])
    rng = np.random.Generator(np.random.PCG64(seed))
    gb = rng.standard_normal(be.size).astype(np.float32)
    gd = rng.standard_normal(de.size).astype(np.float32)
    gb[rng.random(be.size) < 0.2] = 0.0
    gd[rng.random(de.size) < 0.2] = 0.0
    return be, de, gb, gd


def _check_pair(rpp, x, seed):
    import torch
    pts = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    be, de, gb, gd = _terms(rpp, x, seed)
    assert be.size > 0
    ref = rpp.backward_points(pts, be, de, gb, gd).cpu().numpy()
    out = torch.full_like(pts, float("nan"))
    got = rpp.backward_points(pts, be, de, gb, gd, out=out, noalloc=True).cpu().numpy()
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))
    assert np.any(ref != 0.0)
    return be.size


def test_noalloc_backward_matches_allocating_entry_point_twice():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2003_07989_amd as rpp
    rpp.load()
    big = _check_pair(rpp, w.noisy_circle_points(512, seed=41), 1)
    small = _check_pair(rpp, w.noisy_circle_points(64, seed=42), 2)
    assert small < big


def test_noalloc_backward_without_death_gradients(rpp):
    import torch
    x = w.noisy_circle_points(200, seed=43)
    pts = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    be, de, gb, _ = _terms(rpp, x, 3)
    zero = np.zeros_like(gb)
    ref = rpp.backward_points(pts, be, de, gb, zero).cpu().numpy()
    got = rpp.backward_points(pts, be, de, gb, zero, noalloc=True).cpu().numpy()
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))
