"""ctypes binding of the C ABI in include/rpp.h (argument marshalling only).

Every stage of the computation runs inside librpp.so on the GPU (and its
host residual reduction); this module only moves pointers and sizes across
the boundary and copies results into numpy arrays.  PyTorch supplies device
memory and streams.  torch is imported before the library is loaded so that
both share one HIP runtime (torch's runtime carries the same soname).
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass, field

import numpy as np
import torch  # noqa: F401  (must precede loading librpp.so)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librpp.so")

RPP_MAX_DIM = 4
RPP_NOALLOC_MAX_BARS = 262144  # bars rpp_backward_noalloc stages at most
RPP_NO_ENCLOSING_RADIUS = 0x1
RPP_WANT_PAIRS = 0x2
RPP_SORTED_PAIR_STORE = 0x4
RPP_FORCE_SPARSE = 0x8
RPP_FORCE_DENSE = 0x10
RPP_WANT_CRITICAL_EDGES = 0x20
RPP_BATCH_NO_GRAPH = 0x40
RPP_BATCH_AUTOTUNE = 0x80
RPP_OBLIVIOUS_REDUCTION = 0x100
RPP_SORT_FIRST = 0x200
RPP_BATCH_EXACT_SHAPES = 0x400
NO_EDGE = np.uint64(0xFFFFFFFFFFFFFFFF)

ERRORS = {0: "RPP_OK", -1: "RPP_E_INVAL", -2: "RPP_E_DATA", -3: "RPP_E_RANGE",
          -4: "RPP_E_NOMEM", -5: "RPP_E_DEVICE", -6: "RPP_E_CANCELLED"}


class RppError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s (%d): %s" % (ERRORS.get(code, "?"), code, msg))
        self.code = code


class _Stats(ctypes.Structure):
    _fields_ = [(name, ctypes.c_int64) for name in (
        "n_candidates", "n_simplices", "n_thresholded", "n_cleared", "n_kept",
        "n_apparent", "n_nonapparent", "n_host_pairs", "n_essential", "n_bars",
        "n_column_adds", "n_scanned")] + [(name, ctypes.c_float) for name in (
        "ms_gpu", "ms_host", "ms_enumerate", "ms_apparent", "ms_partition", "ms_sort")] + [
        ("apparent_group", ctypes.c_int32)]


class _Bars(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("count", ctypes.c_int64),
                ("birth", ctypes.POINTER(ctypes.c_float)),
                ("death", ctypes.POINTER(ctypes.c_float)),
                ("birth_edge", ctypes.POINTER(ctypes.c_uint64)),
                ("death_edge", ctypes.POINTER(ctypes.c_uint64))]


class _Pairs(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("count", ctypes.c_int64),
                ("sigma", ctypes.POINTER(ctypes.c_uint64)),
                ("tau", ctypes.POINTER(ctypes.c_uint64))]


class _Request(ctypes.Structure):
    _fields_ = [("dist_dev", ctypes.c_void_p), ("n", ctypes.c_int32), ("maxdim", ctypes.c_int32),
                ("threshold", ctypes.c_float)]


class _ServerStats(ctypes.Structure):
    _fields_ = [("slots", ctypes.c_int32), ("budget_bytes", ctypes.c_size_t),
                ("in_flight_bytes", ctypes.c_size_t), ("peak_in_flight_bytes", ctypes.c_size_t),
                ("peak_allocated_bytes", ctypes.c_size_t), ("peak_concurrency", ctypes.c_int32),
                ("admitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("queued", ctypes.c_int64)]


class _Result(ctypes.Structure):
    _fields_ = [("maxdim", ctypes.c_int32), ("n", ctypes.c_int32),
                ("threshold_used", ctypes.c_float), ("enclosing_radius", ctypes.c_float),
                ("dims", ctypes.POINTER(_Bars)), ("stats", ctypes.POINTER(_Stats)),
                ("pairs", ctypes.POINTER(_Pairs))]


_lib = None


def load() -> ctypes.CDLL:
    """Load librpp.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("librpp.so is missing at %s: run __graft_entry__.build() "
                           "(or python -m paper_2003_07989_amd.build) first" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    lib.rpp_barcodes.argtypes = [P(ctypes.c_float), ctypes.c_int32, ctypes.c_int32,
                                 ctypes.c_float, P(P(_Result))]
    lib.rpp_barcodes.restype = ctypes.c_int
    lib.rpp_barcodes_device.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                        ctypes.c_float, ctypes.c_void_p, ctypes.c_size_t,
                                        ctypes.c_void_p, ctypes.c_uint32, P(P(_Result))]
    lib.rpp_barcodes_device.restype = ctypes.c_int
    lib.rpp_workspace_bytes.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_float]
    lib.rpp_workspace_bytes.restype = ctypes.c_size_t
    lib.rpp_apparent_pairs.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                       ctypes.c_float, ctypes.c_void_p, P(ctypes.c_uint64),
                                       P(ctypes.c_uint64), ctypes.c_int64, P(ctypes.c_int64),
                                       P(ctypes.c_int64), P(_Stats)]
    lib.rpp_apparent_pairs.restype = ctypes.c_int
    lib.rpp_pdist_device.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                     ctypes.c_void_p, ctypes.c_void_p]
    lib.rpp_pdist_device.restype = ctypes.c_int
    lib.rpp_backward.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64,
                                 P(ctypes.c_uint64), P(ctypes.c_uint64), P(ctypes.c_float),
                                 P(ctypes.c_float), ctypes.c_void_p, ctypes.c_void_p]
    lib.rpp_backward.restype = ctypes.c_int
    lib.rpp_backward_noalloc.argtypes = lib.rpp_backward.argtypes
    lib.rpp_backward_noalloc.restype = ctypes.c_int
    lib.rpp_barcodes_batch.argtypes = [ctypes.c_int32, P(_Request), ctypes.c_void_p,
                                       ctypes.c_uint32, P(P(_Result))]
    lib.rpp_barcodes_batch.restype = ctypes.c_int
    lib.rpp_server_create.argtypes = [ctypes.c_int32, ctypes.c_size_t, P(ctypes.c_void_p)]
    lib.rpp_server_create.restype = ctypes.c_int
    lib.rpp_server_submit.argtypes = [ctypes.c_void_p, P(ctypes.c_float), ctypes.c_int32,
                                      ctypes.c_int32, ctypes.c_float, ctypes.c_uint32,
                                      P(ctypes.c_uint64)]
    lib.rpp_server_submit.restype = ctypes.c_int
    lib.rpp_server_wait.argtypes = [ctypes.c_void_p, ctypes.c_uint64, P(P(_Result)),
                                    P(ctypes.c_double), P(ctypes.c_double)]
    lib.rpp_server_wait.restype = ctypes.c_int
    lib.rpp_server_cancel.argtypes = [ctypes.c_void_p, ctypes.c_uint64]
    lib.rpp_server_cancel.restype = ctypes.c_int
    lib.rpp_server_stats.argtypes = [ctypes.c_void_p, P(_ServerStats)]
    lib.rpp_server_stats.restype = ctypes.c_int
    lib.rpp_server_destroy.argtypes = [ctypes.c_void_p]
    lib.rpp_server_destroy.restype = None
    lib.rpp_result_free.argtypes = [P(_Result)]
    lib.rpp_result_free.restype = None
    lib.rpp_strerror.argtypes = [ctypes.c_int]
    lib.rpp_strerror.restype = ctypes.c_char_p
    lib.rpp_last_error.argtypes = []
    lib.rpp_last_error.restype = ctypes.c_char_p
    lib.rpp_version.argtypes = []
    lib.rpp_version.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _check(rc: int):
    if rc != 0:
        raise RppError(rc, load().rpp_last_error().decode())


@dataclass
class Barcodes:
    """Result of one cloud: bars[p] = (birth, death) float32 arrays."""
    n: int
    maxdim: int
    threshold_used: float
    enclosing_radius: float
    bars: list
    stats: list
    pairs: list = field(default=None)
    edges: list = field(default=None)   # per dim (birth_edge, death_edge), with critical edges


def _collect(res: "ctypes.POINTER(_Result)") -> Barcodes:
    r = res.contents
    bars, stats, pairs, edges = [], [], None, None
    for p in range(r.maxdim + 1):
        b = r.dims[p]
        cnt = int(b.count)
        if cnt:
            birth = np.ctypeslib.as_array(b.birth, shape=(cnt,)).copy()
            death = np.ctypeslib.as_array(b.death, shape=(cnt,)).copy()
        else:
            birth = np.zeros(0, np.float32)
            death = np.zeros(0, np.float32)
        bars.append((birth, death))
        if bool(b.birth_edge):
            if edges is None:
                edges = []
            if cnt:
                edges.append((np.ctypeslib.as_array(b.birth_edge, shape=(cnt,)).copy(),
                              np.ctypeslib.as_array(b.death_edge, shape=(cnt,)).copy()))
            else:
                edges.append((np.zeros(0, np.uint64), np.zeros(0, np.uint64)))
        s = r.stats[p]
        stats.append({name: getattr(s, name) for name, _ in _Stats._fields_})
    if bool(r.pairs):
        pairs = []
        for p in range(r.maxdim + 1):
            q = r.pairs[p]
            cnt = int(q.count)
            if cnt:
                pairs.append((np.ctypeslib.as_array(q.sigma, shape=(cnt,)).copy(),
                              np.ctypeslib.as_array(q.tau, shape=(cnt,)).copy()))
            else:
                pairs.append((np.zeros(0, np.uint64), np.zeros(0, np.uint64)))
    return Barcodes(int(r.n), int(r.maxdim), float(r.threshold_used),
                    float(r.enclosing_radius), bars, stats, pairs, edges)


def _n_from_len(m: int) -> int:
    n = int((1 + math.isqrt(1 + 8 * m)) // 2)
    if n * (n - 1) // 2 != m:
        raise ValueError("length %d is not n*(n-1)/2" % m)
    return n


def _stream_handle(stream) -> int:
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    return int(getattr(stream, "cuda_stream", stream))


def barcodes_device(dist: torch.Tensor, maxdim: int, threshold: float = math.inf,
                    n: int = None, flags: int = 0, stream=None,
                    workspace: torch.Tensor = None) -> Barcodes:
    """rpp_barcodes_device on a contiguous float32 CUDA tensor holding the
    condensed lower triangle.  workspace: an optional contiguous CUDA tensor
    (any dtype) whose memory the call uses for every device buffer."""
    if not (isinstance(dist, torch.Tensor) and dist.is_cuda and dist.dtype == torch.float32
            and dist.is_contiguous()):
        raise TypeError("dist must be a contiguous float32 CUDA tensor")
    if n is None:
        n = _n_from_len(dist.numel())
    ws_ptr, ws_bytes = None, 0
    if workspace is not None:
        if not (isinstance(workspace, torch.Tensor) and workspace.is_cuda
                and workspace.is_contiguous()):
            raise TypeError("workspace must be a contiguous CUDA tensor")
        ws_ptr = ctypes.c_void_p(workspace.data_ptr())
        ws_bytes = workspace.numel() * workspace.element_size()
    lib = load()
    out = ctypes.POINTER(_Result)()
    rc = lib.rpp_barcodes_device(ctypes.c_void_p(dist.data_ptr() if dist.numel() else 0),
                                 int(n), int(maxdim), ctypes.c_float(threshold), ws_ptr,
                                 ws_bytes, ctypes.c_void_p(_stream_handle(stream)), int(flags),
                                 ctypes.byref(out))
    _check(rc)
    try:
        return _collect(out)
    finally:
        lib.rpp_result_free(out)


def barcodes(dist, maxdim: int, threshold: float = math.inf, n: int = None,
             flags: int = 0, stream=None) -> Barcodes:
    """Barcodes of a condensed distance array (numpy array or tensor); host
    data are copied to the current CUDA device first."""
    if isinstance(dist, torch.Tensor) and dist.is_cuda:
        t = dist.to(torch.float32).contiguous()
    else:
        a = np.ascontiguousarray(np.asarray(dist), dtype=np.float32)
        t = torch.from_numpy(a).cuda()
    return barcodes_device(t, maxdim, threshold, n=n, flags=flags, stream=stream)


def barcodes_host(dist: np.ndarray, maxdim: int, threshold: float = math.inf,
                  n: int = None) -> Barcodes:
    """rpp_barcodes on a host array (the library copies it to the device)."""
    a = np.ascontiguousarray(dist, dtype=np.float32)
    if n is None:
        n = _n_from_len(a.size)
    lib = load()
    out = ctypes.POINTER(_Result)()
    ptr = a.ctypes.data_as(ctypes.POINTER(ctypes.c_float)) if a.size else None
    _check(lib.rpp_barcodes(ptr, int(n), int(maxdim), ctypes.c_float(threshold),
                            ctypes.byref(out)))
    try:
        return _collect(out)
    finally:
        lib.rpp_result_free(out)


def _apparent_call(dist, p, threshold, n, stream, cap, s_arr, t_arr, stats):
    if isinstance(dist, torch.Tensor) and dist.is_cuda:
        t = dist.to(torch.float32).contiguous()
    else:
        t = torch.from_numpy(np.ascontiguousarray(np.asarray(dist), dtype=np.float32)).cuda()
    if n is None:
        n = _n_from_len(t.numel())
    cnt, ncols = ctypes.c_int64(0), ctypes.c_int64(0)
    P64 = ctypes.POINTER(ctypes.c_uint64)
    _check(load().rpp_apparent_pairs(
        ctypes.c_void_p(t.data_ptr()), int(n), int(p), ctypes.c_float(threshold),
        ctypes.c_void_p(_stream_handle(stream)),
        s_arr.ctypes.data_as(P64) if s_arr is not None else None,
        t_arr.ctypes.data_as(P64) if t_arr is not None else None, int(cap),
        ctypes.byref(cnt), ctypes.byref(ncols),
        ctypes.byref(stats) if stats is not None else None))
    return int(cnt.value), int(ncols.value)


def apparent_pairs(dist, p: int, threshold: float = math.inf, n: int = None, stream=None):
    """(sigma, tau, n_columns): apparent pairs of dimension (p, p+1) over all
    p-simplices with diameter <= threshold, in increasing sigma order."""
    k, _ = _apparent_call(dist, p, threshold, n, stream, 0, None, None, None)
    s = np.zeros(max(k, 1), np.uint64)
    u = np.zeros(max(k, 1), np.uint64)
    k2, ncols = _apparent_call(dist, p, threshold, n, stream, k, s, u, None)
    return s[:k2], u[:k2], ncols


def apparent_count(dist, p: int, threshold: float = math.inf, n: int = None, stream=None):
    """Number of apparent pairs of dimension (p, p+1) over all p-simplices
    with diameter <= threshold, without fetching them: (count, n_columns,
    stats dict with the GPU stage times and lanes per column)."""
    st = _Stats()
    k, ncols = _apparent_call(dist, p, threshold, n, stream, 0, None, None, st)
    return k, ncols, {name: getattr(st, name) for name, _ in _Stats._fields_}


def workspace_bytes(n: int, maxdim: int, threshold: float = math.inf) -> int:
    return int(load().rpp_workspace_bytes(int(n), int(maxdim), ctypes.c_float(threshold)))


def version() -> str:
    return load().rpp_version().decode()


def strerror(code: int) -> str:
    return load().rpp_strerror(int(code)).decode()


def pdist_device(points: torch.Tensor, out: torch.Tensor = None, stream=None) -> torch.Tensor:
    """rpp_pdist_device: condensed FP32 distances of an (n, d) float32 CUDA
    tensor (FP64 accumulation, one rounding)."""
    if not (points.is_cuda and points.dtype == torch.float32 and points.dim() == 2):
        raise TypeError("points must be an (n, d) float32 CUDA tensor")
    pts = points.contiguous()
    n, d = pts.shape
    if out is None:
        out = torch.empty(n * (n - 1) // 2, dtype=torch.float32, device=pts.device)
    _check(load().rpp_pdist_device(ctypes.c_void_p(pts.data_ptr()), int(n), int(d),
                                   ctypes.c_void_p(out.data_ptr()),
                                   ctypes.c_void_p(_stream_handle(stream))))
    return out


def backward_points(points: torch.Tensor, birth_edge, death_edge, grad_birth, grad_death,
                    stream=None, out=None, noalloc=False) -> torch.Tensor:
    """rpp_backward: gradient w.r.t. (n, d) float32 CUDA coordinates of a
    loss whose gradient w.r.t. each bar's (birth, death) is given.
    noalloc=True calls rpp_backward_noalloc (bars staged in the library's
    fixed device array); out: a preallocated (n, d) float32 result."""
    pts = points.contiguous()
    n, d = pts.shape
    be = np.ascontiguousarray(birth_edge, dtype=np.uint64)
    de = np.ascontiguousarray(death_edge, dtype=np.uint64)
    gb = np.ascontiguousarray(grad_birth, dtype=np.float32)
    gd = np.ascontiguousarray(grad_death, dtype=np.float32)
    if out is None:
        out = torch.empty_like(pts)
    U64, F32 = ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_float)
    lib = load()
    fn = lib.rpp_backward_noalloc if noalloc else lib.rpp_backward
    _check(fn(ctypes.c_void_p(pts.data_ptr()), int(n), int(d), int(be.size),
              be.ctypes.data_as(U64), de.ctypes.data_as(U64),
              gb.ctypes.data_as(F32), gd.ctypes.data_as(F32),
              ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(_stream_handle(stream))))
    return out


class PointCloudBarcodes(torch.autograd.Function):
    """Differentiable barcodes of a point cloud: forward returns one (k_p, 2)
    float32 tensor of (birth, death) per dimension; backward sends each
    bar's gradient to the endpoints of its critical edges (rpp_backward)."""

    @staticmethod
    def forward(ctx, points, maxdim, threshold=math.inf, flags=0):
        pts = points.detach().contiguous()
        dist = pdist_device(pts)
        res = barcodes_device(dist, maxdim, threshold, flags=flags | RPP_WANT_CRITICAL_EDGES)
        ctx.save_for_backward(pts)
        ctx.edges = res.edges
        ctx.counts = [len(b) for b, _ in res.bars]
        outs = tuple(torch.from_numpy(np.stack([b, d], axis=1)).to(points.device)
                     for b, d in res.bars)
        return outs

    @staticmethod
    def backward(ctx, *grads):
        (pts,) = ctx.saved_tensors
        be, de, gb, gd = [], [], [], []
        for p, g in enumerate(grads):
            e_b, e_d = ctx.edges[p]
            be.append(e_b)
            de.append(e_d)
            if g is None:
                gb.append(np.zeros(ctx.counts[p], np.float32))
                gd.append(np.zeros(ctx.counts[p], np.float32))
            else:
                gh = g.detach().float().cpu().numpy()
                gh = np.where(np.isfinite(gh), gh, 0.0).astype(np.float32)
                gb.append(gh[:, 0])
                gd.append(gh[:, 1])
        grad = backward_points(pts, np.concatenate(be), np.concatenate(de),
                               np.concatenate(gb), np.concatenate(gd))
        return grad, None, None, None


def point_cloud_barcodes(points: torch.Tensor, maxdim: int, threshold: float = math.inf,
                         flags: int = 0):
    """Differentiable barcodes (see PointCloudBarcodes)."""
    return PointCloudBarcodes.apply(points, maxdim, threshold, flags)


def barcodes_batch(dists, maxdims, thresholds=None, flags: int = 0, stream=None) -> list:
    """rpp_barcodes_batch on a list of contiguous float32 CUDA tensors
    (condensed matrices); maxdims / thresholds: one value or one per cloud.
    Returns a list of Barcodes in input order."""
    m = len(dists)
    if not isinstance(maxdims, (list, tuple)):
        maxdims = [maxdims] * m
    if thresholds is None:
        thresholds = [math.inf] * m
    elif not isinstance(thresholds, (list, tuple)):
        thresholds = [thresholds] * m
    reqs = (_Request * max(m, 1))()
    for i, t in enumerate(dists):
        if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
            raise TypeError("each distance array must be a contiguous float32 CUDA tensor")
        reqs[i].dist_dev = t.data_ptr() if t.numel() else None
        reqs[i].n = _n_from_len(t.numel())
        reqs[i].maxdim = int(maxdims[i])
        reqs[i].threshold = float(thresholds[i])
    outs = (ctypes.POINTER(_Result) * max(m, 1))()
    lib = load()
    _check(lib.rpp_barcodes_batch(m, reqs, ctypes.c_void_p(_stream_handle(stream)), int(flags),
                                  outs))
    res = []
    try:
        for i in range(m):
            res.append(_collect(outs[i]))
    finally:
        for i in range(m):
            if bool(outs[i]):
                lib.rpp_result_free(outs[i])
    return res


class Server:
    """Continuous-admission barcode server (rpp_server_*): submit host
    distance arrays, wait for results with per-request latency."""

    def __init__(self, slots: int = 4, hbm_budget_bytes: int = 0):
        self._lib = load()
        h = ctypes.c_void_p()
        rc = self._lib.rpp_server_create(int(slots), int(hbm_budget_bytes), ctypes.byref(h))
        if rc != 0:
            raise RppError(rc, "rpp_server_create failed")
        self._h = h

    def submit(self, dist, maxdim: int, threshold: float = math.inf, flags: int = 0,
               n: int = None) -> int:
        a = np.ascontiguousarray(dist, dtype=np.float32)
        if n is None:
            n = _n_from_len(a.size)
        t = ctypes.c_uint64(0)
        ptr = a.ctypes.data_as(ctypes.POINTER(ctypes.c_float)) if a.size else None
        rc = self._lib.rpp_server_submit(self._h, ptr, int(n), int(maxdim),
                                         ctypes.c_float(threshold), int(flags), ctypes.byref(t))
        if rc != 0:
            raise RppError(rc, "rpp_server_submit failed")
        return int(t.value)

    def wait(self, ticket: int):
        """(Barcodes, latency_ms, queue_ms)."""
        out = ctypes.POINTER(_Result)()
        lat, q = ctypes.c_double(0), ctypes.c_double(0)
        rc = self._lib.rpp_server_wait(self._h, ctypes.c_uint64(ticket), ctypes.byref(out),
                                       ctypes.byref(lat), ctypes.byref(q))
        if rc != 0:
            raise RppError(rc, self._lib.rpp_last_error().decode())
        try:
            return _collect(out), lat.value, q.value
        finally:
            self._lib.rpp_result_free(out)

    def cancel(self, ticket: int):
        """rpp_server_cancel: a queued request never runs, a running one
        stops at its next stage boundary; its wait raises RPP_E_CANCELLED."""
        _check(load().rpp_server_cancel(self._h, int(ticket)))

    def stats(self) -> dict:
        st = _ServerStats()
        self._lib.rpp_server_stats(self._h, ctypes.byref(st))
        return {name: getattr(st, name) for name, _ in _ServerStats._fields_}

    def close(self):
        if self._h:
            self._lib.rpp_server_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
