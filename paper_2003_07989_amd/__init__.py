"""Vietoris-Rips persistence barcodes on the AMD Instinct MI355X.

The data-parallel hot path of arXiv 2003.07989 (Ripser++) -- enumeration
of simplices in combinatorial-number-system order, the threshold and
clearing filter, the apparent-pair test, the column key sorts and H0 by
union-find -- runs as hand-written HIP kernels for gfx950 in ``librpp.so``
behind the C ABI of ``include/rpp.h``.  This package is the thin Python
binding.  Importing it does not load the library; the first call does,
and fails loudly if ``librpp.so`` has not been built.
"""
from ._binding import (NO_EDGE, RPP_BATCH_AUTOTUNE, RPP_BATCH_EXACT_SHAPES, RPP_BATCH_NO_GRAPH,
                       RPP_FORCE_DENSE,
                       RPP_FORCE_SPARSE, RPP_MAX_DIM,
                       RPP_NO_ENCLOSING_RADIUS, RPP_OBLIVIOUS_REDUCTION,
                       RPP_SORT_FIRST, RPP_SORTED_PAIR_STORE,
                       RPP_WANT_CRITICAL_EDGES, RPP_WANT_PAIRS, Barcodes,
                       PointCloudBarcodes, RppError, Server, apparent_count, apparent_pairs,
                       backward_points, barcodes,
                       barcodes_batch,
                       barcodes_device, barcodes_host, load, pdist_device,
                       point_cloud_barcodes, strerror, version, workspace_bytes)

__all__ = ["NO_EDGE", "RPP_BATCH_AUTOTUNE", "RPP_BATCH_EXACT_SHAPES", "RPP_BATCH_NO_GRAPH", "RPP_FORCE_DENSE", "RPP_FORCE_SPARSE", "RPP_MAX_DIM",
           "RPP_NO_ENCLOSING_RADIUS", "RPP_OBLIVIOUS_REDUCTION", "RPP_SORT_FIRST",
           "RPP_SORTED_PAIR_STORE", "RPP_WANT_CRITICAL_EDGES",
           "RPP_WANT_PAIRS", "Barcodes", "PointCloudBarcodes", "RppError", "Server",
           "apparent_count", "apparent_pairs",
           "backward_points", "barcodes", "barcodes_batch", "barcodes_device", "barcodes_host", "load",
           "pdist_device", "point_cloud_barcodes", "strerror", "version", "workspace_bytes"]
