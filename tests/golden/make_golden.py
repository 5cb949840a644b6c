"""Write the stored expected barcodes for the full-size workloads.

Calls only the CPU oracle (``oracle/``) on inputs from ``workloads.py``.
The plain standard reduction cannot finish these sizes (a column that
reduces to zero needs on the order of n^2 additions without clearing), so
this script uses the oracle's clearing mode, which the CPU tests pin to the
plain mode bit for bit on smaller inputs.

Output: ``tests/golden/<name>.bars.txt`` with a header (input SHA-256,
sizes, threshold, oracle mode, per-dimension pair and bar counts) and one
line per bar: ``dim birth_hex death_hex birth death`` where *_hex are the
IEEE-754 binary32 bit patterns (exact) and the decimal values are for
reading only.

A second kind of fixture, ``perm<n0>.apparent.txt``, holds the oracle's
dimension-1 apparent pairs of a random edge order on n0 points (all C(n0,2)
edges, no threshold): the input SHA-256, the number of pairs and the SHA-256
of the pair arrays (sigma then tau, little-endian u64, increasing sigma).

Usage: python tests/golden/make_golden.py torus400 [sphere4096 mixture448 perm1500 ...]
"""
from __future__ import annotations

import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads  # noqa: E402


def write(name: str) -> str:
    cfg = workloads.WORKLOADS[name]
    d = cfg["build"]()
    n, maxdim, thr = cfg["n"], cfg["maxdim"], cfg["threshold"]
    if cfg.get("golden_threshold") == "radius":
        # no threshold requested: the oracle runs at the enclosing radius,
        # which leaves every nonzero interval unchanged (the proposition on
        # the enclosing radius, pinned in the CPU tests) and is far cheaper
        thr = oracle.enclosing_radius(d, n)
    digest = hashlib.sha256(d.tobytes()).hexdigest()
    t0 = time.time()
    red = oracle.reduce(d, n, maxdim, thr, clearing=True)
    secs = time.time() - t0
    bars = oracle.bars_from_pairs(red)
    path = os.path.join(HERE, name + ".bars.txt")
    with open(path, "w") as f:
        f.write("# expected barcodes of workload %s, written by tests/golden/make_golden.py\n" % name)
        f.write("# source: CPU oracle, standard reduction with clearing (%.1f s)\n" % secs)
        f.write("# input_sha256 %s\n" % digest)
        f.write("# n %d maxdim %d threshold %r\n" % (n, maxdim, float(thr)))
        for p, r in enumerate(red):
            f.write("# dim %d simplices %d pairs %d bars %d\n"
                    % (p, r["n_simplices"], len(r["sigma"]), len(bars[p][0])))
        for p, (b, dd) in enumerate(bars):
            bb = b.view(np.uint32)
            db = dd.view(np.uint32)
            for i in range(len(b)):
                f.write("%d %08x %08x %.9g %.9g\n" % (p, bb[i], db[i], b[i], dd[i]))
    return path


PERM_SEED = 1006


def pair_digest(sigma, tau) -> str:
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(sigma, dtype="<u8").tobytes())
    h.update(np.ascontiguousarray(tau, dtype="<u8").tobytes())
    return h.hexdigest()


def write_perm(n0: int) -> str:
    d = workloads.random_permutation_metric(n0, PERM_SEED)
    t0 = time.time()
    sigma, tau = oracle.apparent_pairs(d, n0, 1)
    secs = time.time() - t0
    path = os.path.join(HERE, "perm%d.apparent.txt" % n0)
    with open(path, "w") as f:
        f.write("# dimension-1 apparent pairs of a random edge order, written by "
                "tests/golden/make_golden.py\n")
        f.write("# source: CPU oracle apparent-pair test (%.1f s)\n" % secs)
        f.write("input_sha256 %s\n" % hashlib.sha256(d.tobytes()).hexdigest())
        f.write("n0 %d\nseed %d\nedges %d\n" % (n0, PERM_SEED, n0 * (n0 - 1) // 2))
        f.write("pairs %d\n" % len(sigma))
        f.write("pairs_sha256 %s\n" % pair_digest(sigma, tau))
    return path


def read_perm(path: str) -> dict:
    out = {}
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        k, v = line.split()
        out[k] = v if k.endswith("sha256") else int(v)
    return out


def read(path: str):
    """(header dict, bars list per dimension) from a golden file."""
    head = {"dims": {}}
    rows = []
    for line in open(path):
        if line.startswith("#"):
            t = line[1:].split()
            if t and t[0] == "input_sha256":
                head["sha256"] = t[1]
            elif t and t[0] == "n":
                head["n"], head["maxdim"], head["threshold"] = int(t[1]), int(t[3]), float(t[5])
            elif t and t[0] == "dim":
                head["dims"][int(t[1])] = dict(simplices=int(t[3]), pairs=int(t[5]),
                                               bars=int(t[7]))
            continue
        t = line.split()
        if t:
            rows.append((int(t[0]), int(t[1], 16), int(t[2], 16)))
    bars = []
    for p in range(head["maxdim"] + 1):
        sel = [(b, d) for q, b, d in rows if q == p]
        b = np.array([x[0] for x in sel], dtype=np.uint32).view(np.float32)
        d = np.array([x[1] for x in sel], dtype=np.uint32).view(np.float32)
        bars.append((b, d))
    return head, bars


if __name__ == "__main__":
    for name in sys.argv[1:]:
        if name.startswith("perm"):
            print("wrote", write_perm(int(name[4:])), flush=True)
        else:
            print("wrote", write(name), flush=True)
