"""Weighted graphs (a Markov chain's transition weights, Def. 3.4 with
a_uv = w_uv / sum_x w_ux) as library input.

The library counts a repeated edge with its multiplicity, in A and in the
out-degree, so an edge of integer weight k is passed exactly as k parallel
edges.  This helper builds that CSR on the host; it only rewrites the input
and runs no step of the method.
"""
from __future__ import annotations

import numpy as np


def expand_integer_weights(row_ptr, col, weight):
    """CSR (row_ptr int64[n+1], col int32[m]) with edge e repeated weight[e]
    times, in the same row order.  Weights must be non-negative integers (a
    zero weight drops the edge); anything else raises ValueError."""
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    col = np.asarray(col)
    w = np.asarray(weight)
    if w.shape != col.shape:
        raise ValueError(f"weight has shape {w.shape}, expected {col.shape}")
    wi = np.asarray(w, dtype=np.int64)
    if not np.array_equal(wi, w) or (wi < 0).any():
        raise ValueError("weights must be non-negative integers")
    src = np.repeat(np.arange(len(row_ptr) - 1, dtype=np.int64), np.diff(row_ptr))
    col2 = np.repeat(col, wi).astype(np.int32)
    cnt = np.bincount(np.repeat(src, wi), minlength=len(row_ptr) - 1)
    rp2 = np.zeros(len(row_ptr), dtype=np.int64)
    np.cumsum(cnt, out=rp2[1:])
    return rp2, col2
