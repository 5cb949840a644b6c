"""Python side of the CPU oracle -- TEST INFRASTRUCTURE, not the product.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module.  It builds and loads ``rips_oracle.c``
(plain C, gcc) and turns its persistence pairs into barcodes.

Barcode conventions (paper, "Filtering Out Simplices by Diameter Equal to the
Enclosing Radius" and the definition of apparent pairs):
  - a pair (sigma, tau) gives the interval [diam(sigma), diam(tau)); pairs
    with diam(tau) == diam(sigma) have zero persistence and are not reported;
  - a column that reduces to zero and is not the tau of a pair one dimension
    lower is essential: [diam(sigma), +inf);
  - each dimension is sorted by (birth, death), +inf last; zeros are +0.0.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rips_oracle.c")
_LIBDIR = os.path.join(_HERE, "_build")
_LIB = os.path.join(_LIBDIR, "liboracle.so")
MAX_DIM = 5


class _Dim(ctypes.Structure):
    _fields_ = [
        ("n_pairs", ctypes.c_int64),
        ("pair_sigma", ctypes.POINTER(ctypes.c_uint64)),
        ("pair_tau", ctypes.POINTER(ctypes.c_uint64)),
        ("pair_birth", ctypes.POINTER(ctypes.c_float)),
        ("pair_death", ctypes.POINTER(ctypes.c_float)),
        ("n_zero", ctypes.c_int64),
        ("zero_sigma", ctypes.POINTER(ctypes.c_uint64)),
        ("zero_birth", ctypes.POINTER(ctypes.c_float)),
        ("n_simplices", ctypes.c_int64),
        ("n_additions", ctypes.c_int64),
        ("n_cleared", ctypes.c_int64),
    ]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc into oracle/_build/liboracle.so."""
    os.makedirs(_LIBDIR, exist_ok=True)
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread",
                               "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        lib.oracle_reduce.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_int,
                                      ctypes.c_int, ctypes.c_float, ctypes.c_int,
                                      ctypes.c_int, ctypes.POINTER(_Dim)]
        lib.oracle_reduce.restype = ctypes.c_int
        lib.oracle_free.argtypes = [ctypes.POINTER(_Dim), ctypes.c_int]
        lib.oracle_free.restype = None
        lib.oracle_apparent_pairs.argtypes = [
            ctypes.POINTER(ctypes.c_float), ctypes.c_int, ctypes.c_int, ctypes.c_float,
            ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64), ctypes.c_int64]
        lib.oracle_apparent_pairs.restype = ctypes.c_int64
        lib.oracle_count_simplices.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_int,
                                               ctypes.c_int, ctypes.c_float]
        lib.oracle_count_simplices.restype = ctypes.c_int64
        _lib = lib
    return _lib


def _as_dist(dist, n):
    d = np.ascontiguousarray(dist, dtype=np.float32)
    if d.shape != (n * (n - 1) // 2,):
        raise ValueError("condensed distance array must have n*(n-1)/2 entries")
    return d


def _arr(ptr, count, dtype):
    if count == 0:
        return np.zeros(0, dtype=dtype)
    return np.ctypeslib.as_array(ptr, shape=(count,)).astype(dtype, copy=True)


def reduce(dist, n: int, maxdim: int, threshold: float = float("inf"),
           threads: int = 0, clearing: bool = False) -> list:
    """Run the standard reduction for dimensions 0..maxdim.

    ``clearing=False`` (default) reduces every column of every dimension,
    the plain standard algorithm.  ``clearing=True`` leaves out the columns
    that the clearing lemma proves zero; it exists for inputs where the
    plain reduction cannot finish, and the tests pin it to the plain mode.

    Returns one dict per dimension with the full pair list (``sigma``,
    ``tau`` combinatorial indices and their diameters ``birth``, ``death``),
    the zero columns (``zero_sigma``, ``zero_birth``), the number of
    p-simplices with diameter <= threshold (``n_simplices``) and the number
    of column additions."""
    lib = _load()
    d = _as_dist(dist, n)
    out = (_Dim * (maxdim + 1))()
    thr = ctypes.c_float(np.float32(threshold))
    th = threads if threads > 0 else (maxdim + 1)
    rc = lib.oracle_reduce(d.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), n, maxdim,
                           thr, th, 1 if clearing else 0, out)
    if rc != 0:
        raise RuntimeError("oracle_reduce failed (%d)" % rc)
    res = []
    try:
        for p in range(maxdim + 1):
            o = out[p]
            res.append(dict(
                sigma=_arr(o.pair_sigma, o.n_pairs, np.uint64),
                tau=_arr(o.pair_tau, o.n_pairs, np.uint64),
                birth=_arr(o.pair_birth, o.n_pairs, np.float32),
                death=_arr(o.pair_death, o.n_pairs, np.float32),
                zero_sigma=_arr(o.zero_sigma, o.n_zero, np.uint64),
                zero_birth=_arr(o.zero_birth, o.n_zero, np.float32),
                n_simplices=int(o.n_simplices),
                n_additions=int(o.n_additions),
                n_cleared=int(o.n_cleared),
            ))
    finally:
        lib.oracle_free(out, maxdim)
    return res


def canonical(birth, death):
    """(birth, death) float32 arrays sorted by birth then death, +inf last,
    with -0.0 written as +0.0."""
    b = np.asarray(birth, dtype=np.float32) + np.float32(0.0)
    d = np.asarray(death, dtype=np.float32) + np.float32(0.0)
    order = np.lexsort((d, b))
    return b[order], d[order]


def bars_from_pairs(red: list) -> list:
    """Barcodes per dimension from ``reduce`` output."""
    out = []
    prev_tau = np.zeros(0, dtype=np.uint64)
    for p, r in enumerate(red):
        keep = r["death"] > r["birth"]
        ess = ~np.isin(r["zero_sigma"], prev_tau)
        b = np.concatenate([r["birth"][keep], r["zero_birth"][ess]])
        d = np.concatenate([r["death"][keep],
                            np.full(int(ess.sum()), np.inf, dtype=np.float32)])
        out.append(canonical(b, d))
        prev_tau = r["tau"]
    return out


def barcodes(dist, n: int, maxdim: int, threshold: float = float("inf"),
             threads: int = 0, clearing: bool = False) -> list:
    """Per-dimension (birth, death) arrays, canonical order."""
    return bars_from_pairs(reduce(dist, n, maxdim, threshold, threads, clearing))


def apparent_pairs(dist, n: int, p: int, threshold: float = float("inf")):
    """(sigma, tau) cidx arrays of the apparent pairs of dimension (p, p+1),
    found from the definition (oldest cofacet / youngest facet by full
    search)."""
    lib = _load()
    d = _as_dist(dist, n)
    thr = ctypes.c_float(np.float32(threshold))
    dp = d.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
    cnt = lib.oracle_apparent_pairs(dp, n, p, thr, None, None, 0)
    if cnt < 0:
        raise RuntimeError("oracle_apparent_pairs failed (%d)" % cnt)
    s = np.zeros(max(cnt, 1), dtype=np.uint64)
    t = np.zeros(max(cnt, 1), dtype=np.uint64)
    cnt2 = lib.oracle_apparent_pairs(dp, n, p, thr,
                                     s.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                     t.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), cnt)
    assert cnt2 == cnt
    return s[:cnt], t[:cnt]


def count_simplices(dist, n: int, p: int, threshold: float = float("inf")) -> int:
    lib = _load()
    d = _as_dist(dist, n)
    c = lib.oracle_count_simplices(d.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), n, p,
                                   ctypes.c_float(np.float32(threshold)))
    if c < 0:
        raise RuntimeError("oracle_count_simplices failed")
    return int(c)


def enclosing_radius(dist, n: int) -> float:
    """min over points of the max distance to any other point (the paper's
    enclosing radius); 0 for a single point."""
    if n < 2:
        return 0.0
    d = _as_dist(dist, n)
    sq = np.zeros((n, n), dtype=np.float32)
    ii, jj = np.tril_indices(n, -1)
    sq[ii, jj] = d
    sq[jj, ii] = d
    return float(sq.max(axis=1).min())
