"""Serving with continuous admission: each result equals the same request
alone; admission respects the HBM budget; requests overlap on the device."""
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


def _requests(k, nmax=400):
    out = []
    i = 0
    while len(out) < k:
        r = w.mixture_request(i)
        i += 1
        if r["n"] <= nmax:
            out.append(r)
    return out


def test_served_results_equal_results_alone(rpp):
    reqs = _requests(12)
    alone = [rpp.barcodes(r["dist"], r["maxdim"], r["threshold"]) for r in reqs]
    with rpp.Server(slots=4) as srv:
        tickets = [srv.submit(r["dist"], r["maxdim"], r["threshold"]) for r in reqs]
        for k, t in enumerate(tickets):
            got, lat, q = srv.wait(t)
            assert lat >= q >= 0.0
            _same(got, alone[k], "request %d" % k)
        st = srv.stats()
    assert st["completed"] == len(reqs)
    assert st["peak_concurrency"] >= 1


def test_served_matches_oracle_small(rpp):
    reqs = _requests(3, nmax=90)
    with rpp.Server(slots=2) as srv:
        ts = [srv.submit(r["dist"], r["maxdim"], r["threshold"]) for r in reqs]
        for r, t in zip(reqs, ts):
            got, _, _ = srv.wait(t)
            exp = oracle.barcodes(r["dist"], r["n"], r["maxdim"], math.inf, clearing=True)
            for p in range(r["maxdim"] + 1):
                assert np.array_equal(got.bars[p][0].view(np.uint32), exp[p][0].view(np.uint32))
                assert np.array_equal(got.bars[p][1].view(np.uint32), exp[p][1].view(np.uint32))


def test_admission_respects_budget(rpp):
    reqs = _requests(10)
    needs = [rpp.workspace_bytes(r["n"], r["maxdim"]) + 4 * r["dist"].size for r in reqs]
    budget = int(max(needs) * 1.2)
    with rpp.Server(slots=4, hbm_budget_bytes=budget) as srv:
        ts = [srv.submit(r["dist"], r["maxdim"], r["threshold"]) for r in reqs]
        for t in ts:
            srv.wait(t)
        st = srv.stats()
    assert st["peak_in_flight_bytes"] <= budget
    assert st["completed"] == len(reqs)


def test_oversized_request_runs_alone(rpp):
    reqs = _requests(3)
    with rpp.Server(slots=3, hbm_budget_bytes=1024) as srv:
        ts = [srv.submit(r["dist"], r["maxdim"], r["threshold"]) for r in reqs]
        for t in ts:
            srv.wait(t)
        st = srv.stats()
    assert st["peak_concurrency"] == 1


def test_requests_overlap_on_the_device(rpp):
    reqs = [w.mixture_request(i) for i in range(40) if w.mixture_request(i)["n"] <= 300][:16]
    with rpp.Server(slots=4) as srv:
        ts = [srv.submit(r["dist"], r["maxdim"], r["threshold"]) for r in reqs]
        for t in ts:
            srv.wait(t)
        st = srv.stats()
    assert st["peak_concurrency"] >= 2


def test_bad_request_is_rejected_at_submission(rpp):
    d = w.condensed_from_points(w.uniform_square_points(10, 1))
    d[0] = np.nan
    with rpp.Server(slots=1) as srv:
        with pytest.raises(rpp.RppError):
            srv.submit(d, 1)
        good = w.condensed_from_points(w.uniform_square_points(10, 2))
        r, _, _ = srv.wait(srv.submit(good, 1))
        assert len(r.bars[0][0]) == 10
