"""The device-memory and error-handling side of the C ABI on the GPU.

- A caller-provided workspace (torch-allocated, filled with garbage first):
  results equal the oracle's bit for bit; too small a workspace returns
  RPP_E_NOMEM (up front, or when a buffer no longer fits) and leaves the
  library usable; a workspace far below the dense bound still serves a
  thresholded sparse input.
- RPP_DEVICE_BUDGET_BYTES on the library's own cache.
- RPP_FAULT_INJECT at every stage boundary, alone and inside a server (only
  the targeted request fails).
- Server cancellation, and admission that counts what idle slots retain.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as w
from test_gpu_parity import CASES, _golden, _oracle_bars, assert_bars_equal

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rpp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2003_07989_amd as m
    m.load()
    return m


def _garbage_workspace(nbytes, seed=0):
    import torch
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    ws.random_(0, 256, generator=g)
    return ws


WS_CASES = CASES[::2]


@pytest.mark.parametrize("sparse", [False, True])
@pytest.mark.parametrize("case", WS_CASES, ids=["ws_" + c[0] for c in WS_CASES])
def test_caller_workspace_matches_oracle(rpp, case, sparse):
    import torch
    name, d, n, maxdim, thr = case
    print("case", name, sparse, flush=True)
    nbytes = rpp.workspace_bytes(n, maxdim, thr)
    ws = _garbage_workspace(nbytes, seed=n)
    dist = torch.from_numpy(d).cuda()
    flags = rpp.RPP_FORCE_SPARSE if sparse else 0
    got = rpp.barcodes_device(dist, maxdim, thr, flags=flags, workspace=ws)
    assert_bars_equal(got.bars, _oracle_bars(d, n, maxdim, thr), name)
    # and again on the same (now dirty) workspace
    again = rpp.barcodes_device(dist, maxdim, thr, flags=flags, workspace=ws)
    assert_bars_equal(again.bars, got.bars, name + " (second call)")


def test_caller_workspace_torus400(rpp):
    import torch
    head, exp = _golden("torus400")
    d = w.WORKLOADS["torus400"]["build"]()
    ws = _garbage_workspace(rpp.workspace_bytes(400, 2), seed=400)
    got = rpp.barcodes_device(torch.from_numpy(d).cuda(), 2, workspace=ws)
    assert_bars_equal(got.bars, exp, "torus400 in a caller workspace")


def test_caller_workspace_below_the_bound_serves_a_sparse_input(rpp):
    """The 4096-point sphere at threshold 0.4: the dense bound is about a
    terabyte, 6 GiB of caller memory is enough for the data."""
    import torch
    head, exp = _golden("sphere4096")
    cfg = w.WORKLOADS["sphere4096"]
    d = cfg["build"]()
    assert rpp.workspace_bytes(4096, 2, 0.4) > (1 << 40)
    ws = _garbage_workspace(6 << 30, seed=4096)
    got = rpp.barcodes_device(torch.from_numpy(d).cuda(), 2, 0.4, workspace=ws)
    assert_bars_equal(got.bars, exp, "sphere4096 in a 6 GiB workspace")


def test_too_small_workspace_returns_nomem_and_the_library_recovers(rpp):
    import torch
    d = w.condensed_from_points(w.noisy_torus_points(120, 3))
    dist = torch.from_numpy(d).cuda()
    with pytest.raises(rpp.RppError) as e:
        rpp.barcodes_device(dist, 2, workspace=_garbage_workspace(4096))
    assert e.value.code == -4 and "below" in str(e.value)
    # enough for staging and H0, not for dimension 2's columns
    with pytest.raises(rpp.RppError) as e:
        rpp.barcodes_device(dist, 2, workspace=_garbage_workspace(1 << 20))
    assert e.value.code == -4 and "workspace too small" in str(e.value)
    exp = oracle.barcodes(d, 120, 2, math.inf, clearing=True)
    assert_bars_equal(rpp.barcodes_device(dist, 2).bars, exp, "after NOMEM, own cache")
    ws = _garbage_workspace(rpp.workspace_bytes(120, 2))
    assert_bars_equal(rpp.barcodes_device(dist, 2, workspace=ws).bars, exp,
                      "after NOMEM, caller workspace")


def test_device_budget(rpp, monkeypatch):
    d = w.condensed_from_points(w.noisy_torus_points(150, 4))
    exp = oracle.barcodes(d, 150, 2, math.inf, clearing=True)
    monkeypatch.setenv("RPP_DEVICE_BUDGET_BYTES", str(rpp.workspace_bytes(150, 2)))
    assert_bars_equal(rpp.barcodes(d, 2).bars, exp, "within the budget")
    monkeypatch.setenv("RPP_DEVICE_BUDGET_BYTES", str(2 << 20))
    with pytest.raises(rpp.RppError) as e:
        rpp.barcodes(d, 2)
    assert e.value.code == -4 and "limit" in str(e.value)
    monkeypatch.setenv("RPP_DEVICE_BUDGET_BYTES", "1000")
    with pytest.raises(rpp.RppError) as e:
        rpp.barcodes(d, 2)
    assert e.value.code == -4 and "RPP_DEVICE_BUDGET_BYTES" in str(e.value)
    monkeypatch.delenv("RPP_DEVICE_BUDGET_BYTES")
    assert_bars_equal(rpp.barcodes(d, 2).bars, exp, "budget lifted")


@pytest.mark.parametrize("stage", ["stage", "h0", "enumerate", "apparent", "host"])
def test_fault_injection_fails_cleanly(rpp, monkeypatch, stage):
    d = w.condensed_from_points(w.uniform_square_points(40, 77))
    exp = oracle.barcodes(d, 40, 2, math.inf, clearing=True)
    monkeypatch.setenv("RPP_FAULT_INJECT", stage)
    with pytest.raises(rpp.RppError) as e:
        rpp.barcodes(d, 2)
    assert e.value.code == -5 and stage in str(e.value)
    monkeypatch.setenv("RPP_FAULT_INJECT", "%s:41" % stage)  # another n: no effect
    assert_bars_equal(rpp.barcodes(d, 2).bars, exp, stage)
    monkeypatch.delenv("RPP_FAULT_INJECT")
    assert_bars_equal(rpp.barcodes(d, 2).bars, exp, stage)


def _requests(k, nmax=300):
    out, seen, i = [], set(), 0
    while len(out) < k:
        r = w.mixture_request(i)
        i += 1
        if r["n"] <= nmax and r["n"] not in seen:
            seen.add(r["n"])
            out.append(r)
    return out


def test_server_fault_is_per_request(rpp, monkeypatch):
    reqs = _requests(8)
    alone = [rpp.barcodes(r["dist"], r["maxdim"]) for r in reqs]
    victim = reqs[3]["n"]
    monkeypatch.setenv("RPP_FAULT_INJECT", "apparent:%d" % victim)
    with rpp.Server(slots=3) as srv:
        ts = [srv.submit(r["dist"], r["maxdim"]) for r in reqs]
        for k, t in enumerate(ts):
            if reqs[k]["n"] == victim:
                with pytest.raises(rpp.RppError) as e:
                    srv.wait(t)
                assert e.value.code == -5
            else:
                got, _, _ = srv.wait(t)
                assert_bars_equal(got.bars, alone[k].bars, "request %d" % k)
        st = srv.stats()
    assert st["completed"] == len(reqs)


def test_server_cancel(rpp):
    # three requests of 500+ points at dimension 2 (tens of milliseconds
    # each) ahead of the ones cancelled while they wait on the single slot
    heavy = [r for r in (w.mixture_request(i) for i in range(120))
             if r["n"] >= 500 and r["maxdim"] == 2][:3]
    reqs = heavy + _requests(7)
    with rpp.Server(slots=1) as srv:
        ts = [srv.submit(r["dist"], r["maxdim"]) for r in reqs]
        srv.cancel(ts[-1])
        srv.cancel(ts[-2])
        for k, t in enumerate(ts[:-2]):
            got, _, _ = srv.wait(t)
            assert len(got.bars[0][0]) >= 1
        for t in ts[-2:]:
            with pytest.raises(rpp.RppError) as e:
                srv.wait(t)
            assert e.value.code == -6
        with pytest.raises(rpp.RppError):
            srv.cancel(ts[0])    # already waited for
        # the server keeps serving
        got, _, _ = srv.wait(srv.submit(reqs[0]["dist"], reqs[0]["maxdim"]))
        assert_bars_equal(got.bars, rpp.barcodes(reqs[0]["dist"], reqs[0]["maxdim"]).bars)


def test_admission_counts_retained_memory(rpp):
    """A tight budget, one large request and then small ones on four slots:
    the device memory the slots hold (retained buffers included) never
    passes the budget, and every result equals the request alone."""
    big = next(r for r in (w.mixture_request(i) for i in range(200))
               if 500 <= r["n"] <= 650 and r["maxdim"] == 2)
    small = _requests(10, nmax=200)
    reqs = [big] + small
    needs = [rpp.workspace_bytes(r["n"], r["maxdim"]) + 4 * r["dist"].size for r in reqs]
    budget = int(max(needs) * 1.1)
    alone = [rpp.barcodes(r["dist"], r["maxdim"]) for r in reqs]
    with rpp.Server(slots=4, hbm_budget_bytes=budget) as srv:
        for rnd in range(2):
            ts = [srv.submit(r["dist"], r["maxdim"]) for r in reqs]
            for k, t in enumerate(ts):
                got, _, _ = srv.wait(t)
                assert_bars_equal(got.bars, alone[k].bars, "round %d request %d" % (rnd, k))
        st = srv.stats()
    assert st["peak_allocated_bytes"] <= budget, st
    assert st["peak_in_flight_bytes"] <= budget, st
