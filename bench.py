"""Benchmark: simplices/s through filtration + apparent-pair test (and the
rest of the hot path) on one MI355X.

A step is one call of rpp_barcodes_device on a distance matrix already
resident in HBM: staging, H0, and for every dimension p >= 1 enumeration
with threshold and clearing, the apparent-pair test, the partition and key
sorts, the host reduction of the non-apparent columns and the clearing set
of the next dimension.  value = simplices per second of whole-step time,
where simplices = the p-simplices (p = 1..maxdim) of the Rips complex with
diameter up to the workload's threshold (all C(n, p+1) when the workload has
no threshold; the library's own truncation at the enclosing radius is an
optimisation and does not change the count).

Default (no --workload): the headline line is the 4096-point sphere at
threshold 0.4, dims 0-2 (the largest single-GPU configuration), with the
other four configurations measured in the same process under "configs":
square32 (latency per barcode), torus400 (simplices/s), serving512
(barcodes/s and p50/p99, served vs batched vs plain) and circles64x512
(batched vs plain forward, backward, finite-difference check).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
--workload runs one workload on its own line: sphere4096, torus400, square32,
circles64x512, serving512, perm20000 (dimension-1 apparent test over all
edges of a random edge order on 20000 points), greedy200 (the same test on
the greedy deterministic distance assignment), sphere4096d3, mixture448.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E


def algorithmic_bytes_enumerate(st: dict, p: int) -> float:
    """Filter stage: 4*C(p+1,2) distance bytes + 1/8 clearing bit per
    candidate, 12 bytes (diameter + index) per kept simplex."""
    return st["n_candidates"] * (4.0 * math.comb(p + 1, 2) + 0.125) + 12.0 * st["n_kept"]


def algorithmic_bytes_apparent(st: dict, p: int) -> float:
    """Apparent test: 12 bytes of column key in, 8 bytes of result out, and
    4*(p+1) distance bytes per cofacet candidate examined."""
    return st["n_kept"] * 20.0 + 4.0 * (p + 1) * st["n_scanned"]


def apparent_kernel_name(p, g):
    """The apparent kernel a dimension ran, from its apparent_group stat:
    negative for the sparse kernels (-(100 K + G) for the two-phase one),
    100 K + G for the two-phase kernel,
    10000 + 100 K + G for its workgroup-pooled form, 20000 + 100 NB + G
    for the pooled form with vector reads of its first NB blocks of four
    candidates (NB = 0 meaning 2)."""
    if g < 0:
        if -g >= 1000:  # fused into the sparse enumeration's scatter pass
            return "k_ext_app<%d,%d,%d>" % (p, (-g - 1000) // 100, (-g - 1000) % 100)
        if -g >= 100:
            return "k_apparent_sparse2<%d,%d,%d>" % (p, -g // 100, -g % 100)
        return "k_apparent_sparse<%d,%d>" % (p, -g)
    if g >= 20000:
        nb = (g - 20000) // 100
        return "k_apparent2v<%d,%d,%d>" % (p, 16 if g % 100 == 16 and nb in (0, 2) else 8,
                                            nb if nb in (3, 4) else 2)
    if g >= 10000:
        return "k_apparent2b<%d,%d,%d>" % (p, (g - 10000) // 100, g % 100)
    if g >= 100:
        return "k_apparent2<%d,%d,%d>" % (p, g // 100, g % 100)
    return "k_apparent<%d,%d>" % (p, g)


KERNEL_SOURCES = ("kernels.hip", "kernels.h", "device_common.h")


def kernel_sources_sha256() -> str:
    """SHA-256 over the device kernels' sources, in KERNEL_SOURCES order:
    the profiles' counters hold for the code with this hash only."""
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2003_07989_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def _counter_summary(workload: str, kernel: str) -> dict:
    """The committed rocprofv3 counter summary of `kernel` on `workload`
    (profiles/counters_<workload>.txt) as a dict, or {} when there is none,
    it names another kernel, or the kernel sources changed since."""
    path = os.path.join(ROOT, "profiles", "counters_%s.txt" % workload)
    if not os.path.exists(path):
        return {}
    kv = {}
    for line in open(path):
        if line.startswith("#") or ":" not in line:
            continue
        k, v = line.split(":", 1)
        kv[k.strip()] = v.strip()
    if kv.get("kernel_sources_sha256") != kernel_sources_sha256() or \
            kv.get("kernel", "").replace(" ", "") != kernel.replace(" ", ""):
        return {}
    return kv


def measured_traffic(workload: str, kernel: str):
    """HBM bytes per launch of `kernel` from the rocprofv3 FETCH_SIZE /
    WRITE_SIZE summary committed under profiles/, scaled by a copy kernel
    of known size; None when there is none or the kernel source changed
    since the counters were taken."""
    try:
        return float(_counter_summary(workload, kernel)["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def measured_l2_hit(workload: str, kernel: str):
    """L2 (TCC) hit rate of `kernel` from the same summary, or None."""
    try:
        return float(_counter_summary(workload, kernel)["l2_hit_rate"])
    except (KeyError, ValueError):
        return None


def host_info() -> dict:
    """Host cores this process may use, the machine's CPU count and model."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0)),
            "cpu_model": model}


def host_threads() -> int:
    """Threads for the oracle baselines: the cores this process may use,
    at most 16 (the host share of one GPU on the MI355X boxes)."""
    return max(1, min(16, len(os.sched_getaffinity(0))))


def cpu_baseline_sphere(m: int = 2048) -> dict:
    """The oracle on the host cores: one random subset of m of the 4096
    sphere points per thread (each subset its own seeded draw), threshold
    0.4, dims 0-2, clearing mode, one thread per subset, all subsets at
    once; simplices/s = the subsets' p-simplices (p = 1, 2) over the wall
    time.  Denser subsets cost more per simplex, so the full-size oracle is
    slower per simplex than this sample."""
    import threading
    import numpy as np
    import oracle
    import workloads
    oracle.build()
    cores = host_threads()
    pts = workloads.noisy_sphere_points(4096, 1003)
    subsets = []
    for k in range(cores):
        rng = np.random.Generator(np.random.PCG64([1003, k]))
        idx = np.sort(rng.choice(4096, size=m, replace=False))
        subsets.append(workloads.condensed_from_points(pts[idx]))
    counts = [0] * cores

    def run(k):
        red = oracle.reduce(subsets[k], m, 2, 0.4, threads=1, clearing=True)
        counts[k] = red[1]["n_simplices"] + red[2]["n_simplices"]
    ths = [threading.Thread(target=run, args=(k,)) for k in range(cores)]
    t0 = time.perf_counter()
    for t in ths:
        t.start()
    for t in ths:
        t.join()
    el = time.perf_counter() - t0
    out = {"value": round(sum(counts) / el, 1), "unit": "simplices/s", "cores": cores,
           "kind": "oracle", "seconds": round(el, 3),
           "sample": "%d random subsets of %d of the 4096 sphere points (one per thread, run "
                     "together), threshold 0.4, dims 0-2, oracle clearing mode; %d simplices "
                     "in total" % (cores, m, sum(counts))}
    out.update(host_info())
    return out


def cpu_baseline(name: str) -> dict:
    """The CPU oracle timed on a bounded sample of the same workload."""
    import numpy as np
    import oracle
    import workloads
    if name == "sphere4096":
        return cpu_baseline_sphere()
    if name == "torus400":
        m = 300
        pts = workloads.noisy_torus_points(400, 1002)[:m]
        d = workloads.condensed_from_points(pts)
        maxdim, thr = 2, math.inf
        sample = ("first %d of the 400 torus points, dims 0-2, no threshold "
                  "(oracle clearing mode, single thread)" % m)
    elif name == "square32":
        m = 32
        d = workloads.WORKLOADS["square32"]["build"]()
        maxdim, thr = 1, math.inf
        sample = "the full 32-point cloud, dims 0-1, repeated"
    else:
        raise SystemExit("no CPU sample defined for " + name)
    oracle.build()
    reps, t0 = 0, time.perf_counter()
    while True:
        oracle.reduce(d, m, maxdim, thr, threads=1, clearing=True)
        reps += 1
        el = time.perf_counter() - t0
        if el > 5.0 or name != "square32":
            break
    simplices = sum(math.comb(m, p + 1) for p in range(1, maxdim + 1)) * reps
    out = {"value": simplices / el, "unit": "simplices/s", "cores": 1, "kind": "oracle",
           "sample": sample, "seconds": round(el, 3)}
    out.update(host_info())
    return out


def _pct(x, q):
    import numpy as np
    return float(np.percentile(np.asarray(x), q)) if len(x) else None


def bench_circles(args):
    """64 noisy circles of 512 points, dims 0-1: forward barcodes/s one cloud
    per call vs one batched call, the backward pass of the total finite H1
    persistence, and an FP64 central-difference check of the gradient."""
    import numpy as np
    import torch
    import paper_2003_07989_amd as rpp
    import workloads
    torch.cuda.set_device(0)
    rpp.load()
    pts, dists = workloads.noisy_circle_batch(64, 512)
    P = [torch.from_numpy(p).cuda() for p in pts]
    D = [torch.from_numpy(d).cuda() for d in dists]
    flags = rpp.RPP_WANT_CRITICAL_EDGES
    if args.oblivious:
        flags |= rpp.RPP_OBLIVIOUS_REDUCTION
    for _ in range(args.warmup):
        rpp.barcodes_batch(D, 1, flags=flags)
        for d in D[:4]:
            rpp.barcodes_device(d, 1, flags=flags)
    torch.cuda.synchronize()
    reps = max(1, args.steps // 5)
    t0 = time.perf_counter()
    for _ in range(reps):
        plain = [rpp.barcodes_device(d, 1, flags=flags) for d in D]
    torch.cuda.synchronize()
    t_plain = (time.perf_counter() - t0) / reps
    t0 = time.perf_counter()
    for _ in range(reps):
        batched = rpp.barcodes_batch(D, 1, flags=flags)
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t0) / reps
    for a, b in zip(plain, batched):
        for p in range(2):
            assert np.array_equal(a.bars[p][0].view(np.uint32), b.bars[p][0].view(np.uint32))
            assert np.array_equal(a.bars[p][1].view(np.uint32), b.bars[p][1].view(np.uint32))
    # backward of loss = sum over finite H1 bars of (death - birth), per cloud
    terms = []
    for r in batched:
        be, de = r.edges[1]
        fin = np.isfinite(r.bars[1][1])
        terms.append((be, de, np.where(fin, -1.0, 0.0).astype(np.float32),
                      np.where(fin, 1.0, 0.0).astype(np.float32)))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        grads = [rpp.backward_points(P[i], *terms[i]) for i in range(64)]
    torch.cuda.synchronize()
    t_bwd = (time.perf_counter() - t0) / reps
    print("circles: forward and backward timed; finite-difference check", file=sys.stderr,
          flush=True)
    rng_c = None
    if args.fd_clouds:
        a0, a1 = (int(x) for x in args.fd_clouds.split(":"))
        rng_c = (a0, a1)
    fd = _fd_check(rpp, pts, batched, grads, full=args.fd_full, clouds=rng_c)
    out = {
        "metric": "barcodes/sec forward, batched vs plain (64 noisy circles x 512 points, dims 0-1)",
        "value": round(64 / t_batch, 2), "unit": "barcodes/s", "n_gpus": 1,
        "steps": reps, "warmup": args.warmup, "ms_per_step": round(t_batch * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic", "config": {"workload": "circles64x512", "clouds": 64, "n": 512,
                                        "maxdim": 1},
        "plain_barcodes_per_s": round(64 / t_plain, 2),
        "batched_speedup": round(t_plain / t_batch, 3),
        "ms_forward_plain_64": round(t_plain * 1e3, 3),
        "ms_forward_batched_64": round(t_batch * 1e3, 3),
        "ms_backward_64": round(t_bwd * 1e3, 3),
        "plain_stage_ms_mean": {k: [round(sum(r.stats[p][k] for r in plain) / 64, 4)
                                    for p in range(2)] for k in ("ms_gpu", "ms_host")},
        "fd_check": fd,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_clouds(dists, 512)
    return out


def _edge_vertices(e):
    """Endpoints (a, b), a > b, of the edge with combinatorial index e = C(a,2) + b."""
    a = int((1 + math.isqrt(1 + 8 * e)) // 2)
    while a * (a - 1) // 2 > e:
        a -= 1
    return (a, e - a * (a - 1) // 2)


def _finite_h1_terms(res):
    import numpy as np
    be, de = res.edges[1]
    fin = np.isfinite(res.bars[1][1])
    return sorted(zip(be[fin].tolist(), de[fin].tolist()))


def _fd_check(rpp, pts, batched, grads, full=False, h=1e-4, chunk=32, clouds=None):
    """Central differences in FP64 of the loss evaluated with the pairing of
    the unperturbed cloud; a coordinate whose +-h perturbation changes that
    pairing (a near-tie) is skipped and counted.  Perturbed clouds go through
    the batched path, 2*chunk clouds per launch.  Default sample: every
    coordinate of every vertex on a critical edge plus 8 other vertices, for
    8 of the 64 clouds; full=True checks all 64 x 512 x 3 coordinates."""
    import numpy as np
    import torch
    rng = np.random.Generator(np.random.PCG64(7))
    checked = skipped = bad = 0
    worst = 0.0
    cloud_ids = range(64) if full else range(0, 64, 8)
    if clouds is not None:
        cloud_ids = range(clouds[0], clouds[1])
    for ci in cloud_ids:
        x = pts[ci].astype(np.float64)
        n = x.shape[0]
        base = _finite_h1_terms(batched[ci])
        ends = np.array([[*_edge_vertices(ed), *_edge_vertices(eb)] for eb, ed in base],
                        dtype=np.int64).reshape(-1, 4)
        g = grads[ci].cpu().numpy()
        if full:
            verts = list(range(n))
        else:
            touched = sorted(set(ends.ravel().tolist()))
            others = [v for v in range(n) if v not in set(touched)]
            verts = touched + sorted(rng.choice(others, size=min(8, len(others)),
                                                replace=False).tolist())
        coords = [(i, k) for i in verts for k in range(x.shape[1])]

        def loss64(xx):
            dd = np.sqrt(np.sum((xx[ends[:, 0]] - xx[ends[:, 1]]) ** 2, axis=1))
            db = np.sqrt(np.sum((xx[ends[:, 2]] - xx[ends[:, 3]]) ** 2, axis=1))
            return float(np.sum(dd) - np.sum(db))

        for c0 in range(0, len(coords), chunk):
            cs = coords[c0:c0 + chunk]
            xs = []
            for i, k in cs:
                for sg in (1.0, -1.0):
                    xx = x.copy()
                    xx[i, k] += sg * h
                    xs.append(xx)
            dev = [rpp.pdist_device(torch.from_numpy(xx.astype(np.float32)).cuda()) for xx in xs]
            res = rpp.barcodes_batch(dev, 1, flags=rpp.RPP_WANT_CRITICAL_EDGES)
            for j, (i, k) in enumerate(cs):
                if _finite_h1_terms(res[2 * j]) != base or _finite_h1_terms(res[2 * j + 1]) != base:
                    skipped += 1
                    continue
                fd = (loss64(xs[2 * j]) - loss64(xs[2 * j + 1])) / (2 * h)
                err = abs(float(g[i, k]) - fd)
                checked += 1
                worst = max(worst, err / (1e-4 + 1e-3 * abs(fd)))
                bad += err > 1e-4 + 1e-3 * abs(fd)
        print("fd check: cloud %d done (%d coordinates checked, %d skipped, %d failures so far)"
              % (ci, checked, skipped, bad), file=sys.stderr, flush=True)
    return {"clouds": len(cloud_ids), "coords_checked": checked,
            "coords_skipped_near_ties": skipped, "failures": int(bad),
            "worst_err_over_tol": round(worst, 4), "h": h, "tol": "abs 1e-4 + rel 1e-3",
            "sample": "all coordinates" if full else
                      "vertices on critical edges + 8 others, every 8th cloud"}


def cpu_baseline_clouds(dists, n):
    """The oracle on one circle per host thread in parallel (threshold =
    enclosing radius, clearing mode): barcodes/s over the host cores."""
    import threading
    import oracle
    oracle.build()
    cores = host_threads()
    sample = dists[:cores]
    t0 = time.perf_counter()
    ths = [threading.Thread(target=lambda d=d: oracle.barcodes(
        d, n, 1, oracle.enclosing_radius(d, n), threads=1, clearing=True)) for d in sample]
    for t in ths:
        t.start()
    for t in ths:
        t.join()
    el = time.perf_counter() - t0
    return {"value": round(len(sample) / el, 4), "unit": "barcodes/s", "cores": cores,
            "kind": "oracle", "seconds": round(el, 3),
            "sample": "%d of the 64 circles, one per thread, threshold = enclosing radius"
                      % len(sample)}


def bench_serving(args):
    """512 Gaussian-mixture requests (n log-uniform in [64, 1024], d in 2..8,
    maxdim 1 or 2, threshold = enclosing radius) arriving as a Poisson
    process at rate lam = f x the measured plain serial capacity (f = 0.8 by
    default, --rates for a sweep); barcodes/s and p50/p99 latency (finish -
    arrival) for plain serial processing, static batches of 8, and the
    continuous-admission server."""
    import threading
    import numpy as np
    import torch
    import paper_2003_07989_amd as rpp
    import workloads
    torch.cuda.set_device(0)
    rpp.load()
    count = args.requests
    # arrivals at rate 1 scale to any rate lam as t / lam
    reqs = workloads.serving_stream(count, rate_per_s=1.0)
    for r in reqs[:3]:
        rpp.barcodes(r["dist"], r["maxdim"])
    t0 = time.perf_counter()
    for r in reqs:
        rpp.barcodes(r["dist"], r["maxdim"])
    torch.cuda.synchronize()
    serial_s = time.perf_counter() - t0
    capacity = count / serial_s
    print("serving: plain capacity %.1f barcodes/s" % capacity, file=sys.stderr, flush=True)

    def plain_mode(arrivals):
        lat, t0 = [], time.perf_counter()
        for r, a in zip(reqs, arrivals):
            now = time.perf_counter() - t0
            if now < a:
                time.sleep(a - now)
            rpp.barcodes(r["dist"], r["maxdim"])
            lat.append(time.perf_counter() - t0 - a)
        return lat, time.perf_counter() - t0, {}

    def batched_mode(arrivals, size=8):
        lat, t0 = [], time.perf_counter()
        for b in range(0, count, size):
            idx = list(range(b, min(count, b + size)))
            now = time.perf_counter() - t0
            if now < arrivals[idx[-1]]:
                time.sleep(arrivals[idx[-1]] - now)
            D = [torch.from_numpy(reqs[i]["dist"]).cuda() for i in idx]
            rpp.barcodes_batch(D, [reqs[i]["maxdim"] for i in idx])
            done = time.perf_counter() - t0
            lat += [done - arrivals[i] for i in idx]
        return lat, time.perf_counter() - t0, {"batch": size}

    # One server for the whole sweep, warmed by one closed-loop pass of the
    # stream -- the plain path's workspace is warm the same way (the capacity
    # pass above), and a server is long-lived: its slot workspaces grow to
    # the largest request once, not per measurement.
    slots = 4
    srv = rpp.Server(slots=slots)
    for r in reqs:
        srv.wait(srv.submit(r["dist"], r["maxdim"]))
    print("serving: server warmed", file=sys.stderr, flush=True)

    def served_mode(arrivals):
        st0 = srv.stats()
        tickets = [None] * count
        late = [0.0] * count   # submission time minus arrival time
        t0 = time.perf_counter()

        def submitter():
            for i, (r, a) in enumerate(zip(reqs, arrivals)):
                now = time.perf_counter() - t0
                if now < a:
                    time.sleep(a - now)
                late[i] = max(0.0, time.perf_counter() - t0 - a)
                tickets[i] = srv.submit(r["dist"], r["maxdim"])
        th = threading.Thread(target=submitter)
        th.start()
        lat = []
        for i in range(count):
            while tickets[i] is None:
                time.sleep(0.0005)
            _, ms, _ = srv.wait(tickets[i])
            lat.append(late[i] + ms / 1e3)
        th.join()
        span = time.perf_counter() - t0
        st = srv.stats()
        return lat, span, {"slots": slots, "admitted": st["admitted"] - st0["admitted"],
                           "completed": st["completed"] - st0["completed"],
                           "peak_concurrency": st["peak_concurrency"],
                           "budget_bytes": st["budget_bytes"],
                           "peak_in_flight_bytes": st["peak_in_flight_bytes"],
                           "peak_allocated_bytes": st["peak_allocated_bytes"]}

    def summary(res):
        lat, span, extra = res
        return dict({"barcodes_per_s": round(count / span, 2),
                     "p50_ms": round(_pct(lat, 50) * 1e3, 2),
                     "p99_ms": round(_pct(lat, 99) * 1e3, 2)}, **extra)

    rates = [float(f) for f in args.rates.split(",")]
    sweep = []
    for f in rates:
        lam = f * capacity
        arrivals = np.array([r["arrival_s"] / lam for r in reqs])
        row = {"rate_factor": f, "arrival_rate_per_s": round(lam, 3)}
        for name, fn in (("plain", plain_mode), ("batched", batched_mode),
                         ("served", served_mode)):
            row[name] = summary(fn(arrivals))
            print("serving: rate %.2f x capacity, %s done" % (f, name), file=sys.stderr,
                  flush=True)
        sweep.append(row)
    srv.close()
    main_row = sweep[0]
    out = {
        "metric": "barcodes/sec and p99 latency, served vs batched vs plain (Poisson stream)",
        "value": main_row["served"]["barcodes_per_s"], "unit": "barcodes/s", "n_gpus": 1,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "serving%d" % count, "requests": count,
                   "arrival_rate_per_s": main_row["arrival_rate_per_s"],
                   "rate_rule": "%.2f x plain serial capacity" % rates[0]},
        "plain_serial_capacity_per_s": round(capacity, 2),
        "served": main_row["served"], "batched": main_row["batched"],
        "plain": main_row["plain"],
    }
    if len(sweep) > 1:
        out["sweep"] = sweep
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_requests(rpp, reqs)
    return out


def cpu_baseline_requests(rpp, reqs, n_max=256, k=32):
    """The oracle on a bounded sample of the request stream -- the first k
    requests with n <= n_max, one per host thread -- and the plain GPU path
    on the same sample, both as barcodes/s."""
    import threading
    import oracle
    oracle.build()
    cores = host_threads()
    sample = [r for r in reqs if r["n"] <= n_max][:k]
    queue = list(range(len(sample)))
    lock = threading.Lock()

    def worker():
        while True:
            with lock:
                if not queue:
                    return
                i = queue.pop(0)
            r = sample[i]
            oracle.barcodes(r["dist"], r["n"], r["maxdim"], oracle.enclosing_radius(r["dist"], r["n"]),
                            threads=1, clearing=True)
    t0 = time.perf_counter()
    ths = [threading.Thread(target=worker) for _ in range(cores)]
    for t in ths:
        t.start()
    for t in ths:
        t.join()
    el = time.perf_counter() - t0
    t0 = time.perf_counter()
    for r in sample:
        rpp.barcodes(r["dist"], r["maxdim"])
    gpu_el = time.perf_counter() - t0
    return {"value": round(len(sample) / el, 3), "unit": "barcodes/s", "cores": cores,
            "kind": "oracle", "seconds": round(el, 3),
            "sample": "first %d requests of the stream with n <= %d (threshold = enclosing "
                      "radius, one request per thread)" % (len(sample), n_max),
            "gpu_plain_same_sample_barcodes_per_s": round(len(sample) / gpu_el, 2)}


def bench_copy(args):
    """HBM copy calibration: clone of a 1 GiB float32 tensor (1 GiB read +
    1 GiB written per copy).  Its FETCH_SIZE / WRITE_SIZE counter readings
    against the known bytes give the scale for the counters of the other
    kernels."""
    import torch
    torch.cuda.set_device(0)
    nbytes = 1 << 30
    x = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    y = torch.empty_like(x)
    for _ in range(args.warmup):
        y.copy_(x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        y.copy_(x)
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / args.steps
    print(json.dumps({"metric": "HBM copy bandwidth (read + write)", "value": round(2 * nbytes / el / 1e9, 1),
                      "unit": "GB/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
                      "ms_per_step": round(el * 1e3, 4), "higher_is_better": True,
                      "config": {"workload": "copy1g", "bytes_read": nbytes,
                                 "bytes_written": nbytes}}))


# The paper's averages of the dimension-1 apparent fraction of random edge
# orders (random distance-matrix experiments).
PAPER_APPARENT_FRACTION = {10000: 0.991127743, 20000: 0.993733522}


def bench_perm(args, n0, kind="perm"):
    """Dimension-1 apparent-pair test over all C(n0,2) edges of a matrix
    whose lower triangle is a random order of distinct FP32 values (kind
    "perm") or the greedy deterministic assignment (kind "greedy", about
    half the edges apparent): columns per second through staging +
    enumeration + apparent test + partition, the apparent fraction, and the
    roofline of the apparent kernel."""
    import numpy as np
    import torch
    import paper_2003_07989_amd as rpp
    import workloads
    torch.cuda.set_device(0)
    rpp.load()
    if kind == "greedy":
        d_host = workloads.greedy_assignment_metric(n0)
    else:
        d_host = workloads.random_permutation_metric(n0, 1006)
    dist = torch.from_numpy(d_host).cuda()
    del d_host
    stream = torch.cuda.current_stream()
    os.environ["RPP_COUNT_SCANS"] = "1"
    k, ncols, tally = rpp.apparent_count(dist, 1, n=n0, stream=stream)
    del os.environ["RPP_COUNT_SCANS"]
    for _ in range(args.warmup):
        rpp.apparent_count(dist, 1, n=n0, stream=stream)
    torch.cuda.synchronize()
    steps = max(1, args.steps // 4)
    acc = {"ms_enumerate": 0.0, "ms_apparent": 0.0, "ms_partition": 0.0, "ms_gpu": 0.0}
    t0 = time.perf_counter()
    for _ in range(steps):
        k, ncols, st = rpp.apparent_count(dist, 1, n=n0, stream=stream)
        for key in acc:
            acc[key] += st[key] / steps
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / steps
    kbytes = algorithmic_bytes_apparent(tally, 1)
    kms = acc["ms_apparent"]
    achieved = kbytes / (kms / 1e3) / 1e9
    out = {
        "metric": "columns/sec through the dimension-1 apparent-pair test (%s)"
                  % ("greedy-assignment edge order" if kind == "greedy" else "random edge order"),
        "value": round(ncols / el, 1), "unit": "columns/s", "n_gpus": 1, "steps": steps,
        "warmup": args.warmup, "ms_per_step": round(el * 1e3, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "%s%d" % (kind, n0), "n0": n0, "columns": ncols,
                   "seed": 1006 if kind == "perm" else None},
        "apparent_fraction": k / ncols,
        "paper_average_fraction": PAPER_APPARENT_FRACTION.get(n0) if kind == "perm" else None,
        "lower_bound_fraction": 1.0 / 3.0 if kind == "greedy" else None,
        "upper_bound_fraction": (n0 - 2) / n0,
        "mean_scan": tally["n_scanned"] / ncols,
        "apparent_group": st["apparent_group"],
        "gpu_stage_ms": {key: round(v, 4) for key, v in acc.items()},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic("%s%d" % (kind, n0),
                                                 apparent_kernel_name(1, st["apparent_group"])),
                     "kernel": apparent_kernel_name(1, st["apparent_group"]), "dim": 1,
                     "ms": round(kms, 4), "bytes": kbytes},
    }
    if not args.no_cpu_baseline and kind == "perm":
        out["cpu_baseline"] = cpu_baseline_perm()
    print(json.dumps(out))


def cpu_baseline_perm(n0=500):
    """The oracle's apparent-pair test on a smaller random order (all
    C(n0,2) edges), one thread, as columns/s.  Its cost per column grows
    with n0 (every column builds its full coboundary), so the sample is
    small and the rate is not the same per-column work as at 20000 points."""
    import oracle
    import workloads
    oracle.build()
    d = workloads.random_permutation_metric(n0, 1006)
    t0 = time.perf_counter()
    oracle.apparent_pairs(d, n0, 1)
    el = time.perf_counter() - t0
    return {"value": round(n0 * (n0 - 1) / 2 / el, 1), "unit": "columns/s", "cores": 1,
            "kind": "oracle", "seconds": round(el, 3),
            "sample": "random order on %d points (all %d edges), dimension 1" % (n0, n0 * (n0 - 1) // 2)}


def bench_cloud(args, name: str, cpu: bool = True) -> dict:
    """One named point cloud (workloads.WORKLOADS): W warm-up calls, then K
    timed calls of rpp_barcodes_device on the resident matrix; simplices/s
    of whole-step time, the GPU stage times, and the roofline of the
    dominant kernel of the top dimension."""
    import numpy as np
    import torch
    import paper_2003_07989_amd as rpp
    import workloads

    cfg = workloads.WORKLOADS[name]
    n, maxdim, thr = cfg["n"], cfg["maxdim"], cfg["threshold"]
    d_host = cfg["build"]()
    torch.cuda.set_device(0)
    dist = torch.from_numpy(d_host).cuda()
    stream = torch.cuda.current_stream()
    rpp.load()

    flags = rpp.RPP_SORT_FIRST if args.sort_first else 0
    if args.oblivious:
        flags |= rpp.RPP_OBLIVIOUS_REDUCTION
    # scan tally for the apparent kernel's algorithmic bytes (outside timing)
    os.environ["RPP_COUNT_SCANS"] = "1"
    tally = rpp.barcodes_device(dist, maxdim, thr, flags=flags, stream=stream)
    del os.environ["RPP_COUNT_SCANS"]

    for _ in range(args.warmup):
        rpp.barcodes_device(dist, maxdim, thr, flags=flags, stream=stream)
    torch.cuda.synchronize()
    stage = {k: [0.0] * (maxdim + 1) for k in ("ms_enumerate", "ms_apparent", "ms_partition",
                                                 "ms_sort", "ms_gpu", "ms_host")}
    t0 = time.perf_counter()
    last = None
    for _ in range(args.steps):
        last = rpp.barcodes_device(dist, maxdim, thr, flags=flags, stream=stream)
        for p in range(maxdim + 1):
            for k in stage:
                stage[k][p] += last.stats[p][k]
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ms_step = el * 1e3 / args.steps
    for k in stage:
        stage[k] = [v / args.steps for v in stage[k]]

    # p-simplices with diameter <= the workload's threshold, p = 1..maxdim:
    # every C(n, p+1) without a threshold (the library's truncation at the
    # enclosing radius is an optimisation, not part of the workload)
    if math.isinf(thr):
        simplices = sum(math.comb(n, p + 1) for p in range(1, maxdim + 1))
    else:
        simplices = sum(last.stats[p]["n_simplices"] for p in range(1, maxdim + 1))
    value = simplices / (ms_step / 1e3)
    # GPU-only rate through filtration + apparent test + partition + sorts
    gpu_ms = sum(stage["ms_enumerate"][p] + stage["ms_apparent"][p] + stage["ms_partition"][p]
                 + stage["ms_sort"][p] for p in range(1, maxdim + 1))

    # dominant kernel family: the largest of enumerate / apparent at the top dimension
    top = maxdim
    st = dict(tally.stats[top])
    cand = {
        "apparent": (stage["ms_apparent"][top], algorithmic_bytes_apparent(st, top)),
        "enumerate": (stage["ms_enumerate"][top], algorithmic_bytes_enumerate(st, top)),
    }
    g = st.get("apparent_group", 8)
    if g <= -1000:
        # the apparent test runs inside the enumeration's scatter pass: one
        # stage moving both the filtration's and the test's bytes
        kname = "fused"
        kms = stage["ms_enumerate"][top]
        kbytes = cand["enumerate"][1] + cand["apparent"][1]
    else:
        kname = max(cand, key=lambda k: cand[k][0])
        kms, kbytes = cand[kname]
    achieved = kbytes / (kms / 1e3) / 1e9 if kms > 0 else 0.0
    if kname == "fused":
        kfull = apparent_kernel_name(top, g) + " (count pass + scatter with clearing and apparent test)"
    elif kname == "apparent":
        kfull = apparent_kernel_name(top, g)
    elif g < 0:
        kfull = "k_ext<%d> (count + scatter with clearing)" % top  # sparse enumeration
    else:
        kfull = "k_enum_count<%d>+k_enum_scatter<%d>" % (top, top)
    traffic = measured_traffic(name, kfull)
    roof = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic, "kernel": kfull, "dim": top, "ms": round(kms, 4),
            "bytes": kbytes,
            "measured_gbs": round(traffic / (kms / 1e3) / 1e9, 2) if traffic else None,
            "l2_hit_rate": measured_l2_hit(name, kfull)}

    out = {
        "metric": "simplices/sec through apparent-pair+filtration",
        "value": round(value, 1),
        "unit": "simplices/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": name, "n": n, "maxdim": maxdim,
                   "stage_order": "sort-first" if args.sort_first else "sort-after",
                   "reduction": "oblivious" if args.oblivious else "reduction-matrix",
                   "threshold": "inf" if math.isinf(thr) else thr,
                   "threshold_used": last.threshold_used,
                   "simplices_per_step": simplices},
        "gpu_stages_simplices_per_s": round(simplices / (gpu_ms / 1e3), 1) if gpu_ms else None,
        "stage_ms": {k: [round(x, 4) for x in v] for k, v in stage.items()},
        "counts": {p: {k: last.stats[p][k] for k in ("n_candidates", "n_kept", "n_apparent",
                                                     "n_nonapparent", "n_column_adds")}
                   for p in range(1, maxdim + 1)},
        "n_scanned": {p: tally.stats[p]["n_scanned"] for p in range(1, maxdim + 1)},
        "roofline": roof,
    }
    if cpu and not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(name)
    return out


def bench_latency(args, name: str = "square32") -> dict:
    """Latency per barcode of a small cloud (launch-bound): the median and
    mean over K x 10 calls of rpp_barcodes_device on the resident matrix."""
    import numpy as np
    import torch
    import paper_2003_07989_amd as rpp
    import workloads
    cfg = workloads.WORKLOADS[name]
    dist = torch.from_numpy(cfg["build"]()).cuda()
    stream = torch.cuda.current_stream()
    rpp.load()
    for _ in range(args.warmup):
        rpp.barcodes_device(dist, cfg["maxdim"], cfg["threshold"], stream=stream)
    torch.cuda.synchronize()
    lat, gpu = [], []
    for _ in range(10 * args.steps):
        t0 = time.perf_counter()
        r = rpp.barcodes_device(dist, cfg["maxdim"], cfg["threshold"], stream=stream)
        lat.append(time.perf_counter() - t0)
        gpu.append(sum(s["ms_gpu"] for s in r.stats))
    return {"metric": "latency per barcode (32 points, dims 0-1)", "value":
            round(float(np.median(lat)) * 1e6, 1), "unit": "us", "higher_is_better": False,
            "mean_us": round(float(np.mean(lat)) * 1e6, 1), "calls": len(lat),
            "gpu_stage_ms_mean": round(float(np.mean(gpu)), 4),
            "config": {"workload": name, "n": cfg["n"], "maxdim": cfg["maxdim"]},
            "roofline": "launch-bound: 496 edges and 4960 triangle cofacets per call, far "
                        "below any bandwidth roof"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default=None,
                    help="one workload on its own line (default: the sphere headline with "
                         "every configuration)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="default run: the headline only, without the other configurations")
    ap.add_argument("--sort-first", action="store_true",
                    help="the paper's stage order: sort every kept column before the "
                         "apparent test (default: sort only the non-apparent ones after it)")
    ap.add_argument("--oblivious", action="store_true",
                    help="host reduction in the oblivious form (add a pivot's unreduced "
                         "coboundary) instead of the reduction-matrix form")
    ap.add_argument("--requests", type=int, default=512)
    ap.add_argument("--rates", default="0.8",
                    help="serving: arrival rates as multiples of the plain capacity")
    ap.add_argument("--fd-clouds", default=None,
                    help="first:last+1 clouds for the finite-difference check (with --fd-full: "
                         "every coordinate of those clouds)")
    ap.add_argument("--fd-full", action="store_true",
                    help="circles: finite-difference check of every coordinate")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the hot path runs on a single MI355X and this "
              "build has no multi-GPU path (requested --gpus %d)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    wl = args.workload
    if wl is None:
        out = bench_cloud(args, "sphere4096")
        print("bench: sphere4096 headline done", file=sys.stderr, flush=True)
        if not args.no_extras:
            extras = {}
            extras["square32"] = bench_latency(args)
            print("bench: square32 done", file=sys.stderr, flush=True)
            extras["torus400"] = bench_cloud(args, "torus400", cpu=False)
            print("bench: torus400 done", file=sys.stderr, flush=True)
            extras["serving512"] = bench_serving(args)
            print("bench: serving512 done", file=sys.stderr, flush=True)
            extras["circles64x512"] = bench_circles(args)
            print("bench: circles64x512 done", file=sys.stderr, flush=True)
            out["configs"] = extras
        print(json.dumps(out))
        return
    if wl.startswith("perm"):
        return bench_perm(args, int(wl[4:]))
    if wl.startswith("greedy"):
        return bench_perm(args, int(wl[6:]), kind="greedy")
    if wl == "copy1g":
        return bench_copy(args)
    if wl == "circles64x512":
        print(json.dumps(bench_circles(args)))
        return
    if wl.startswith("serving"):
        print(json.dumps(bench_serving(args)))
        return
    if wl == "square32":
        print(json.dumps(bench_latency(args)))
        return
    print(json.dumps(bench_cloud(args, wl)))


if __name__ == "__main__":
    main()
