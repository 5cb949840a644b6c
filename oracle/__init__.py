"""CPU oracle for Vietoris-Rips persistence -- TEST INFRASTRUCTURE.

Plain standard reduction (the paper's Algorithm 1) of the full filtered
coboundary matrix, written in C (``rips_oracle.c``) and wrapped in
``oracle.py``.  Only the test suite, ``__graft_entry__.smoke()`` and the
benchmark's CPU-baseline leg may import it; the HIP library never does.
"""
from .oracle import (apparent_pairs, barcodes, bars_from_pairs, build, canonical,
                     count_simplices, enclosing_radius, reduce)

__all__ = ["apparent_pairs", "barcodes", "bars_from_pairs", "build", "canonical",
           "count_simplices", "enclosing_radius", "reduce"]
