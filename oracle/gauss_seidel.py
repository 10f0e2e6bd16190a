"""Block Gauss-Seidel inside one strongly connected component.

Test infrastructure only (see the package docstring).

Sec. 4.3.2 names Gauss-Seidel as an alternative to the power series for the
SCCs that are iterated.  For one component C with M = c A_CC^T (column sums
at most c) and its raised weights W'_C (eq. PR:levels), the fixed point
R = W'_C + M R is approached by sweeps over the component's rows, cut into
`n_blocks` consecutive blocks in the given row order: block b's rows take
W'_C + M R, with R holding this sweep's values for the blocks before b and the
previous sweep's values for b and the blocks after it (inside a block the
update is a Jacobi step).  One block is the Jacobi iteration, which from
R = W'_C is exactly the power series; one row per block is point
Gauss-Seidel.

Certificate: after a sweep the residual W'_C - (I - M) R is non-zero only
through the blocks updated after each row's own update, so its 1-norm is at
most c ||R_new - R_old||_1, and ||R - R*||_1 <= c ||R_new - R_old||_1 / (1 - c).
The sweeps stop once ||R_new - R_old||_1 <= eps (1 - c) ||W'_C||_1, the same
bound as the series' CERT rule.
"""
from __future__ import annotations

import numpy as np


def block_bounds(nv, n_blocks):
    """Row bounds of the blocks: block b holds rows [nv b / B, nv (b+1) / B)."""
    B = max(1, min(int(n_blocks), nv))
    return [(nv * b) // B for b in range(B + 1)]


def block_gauss_seidel(M, Wp, c, eps, n_blocks, max_sweeps=100_000):
    """Block Gauss-Seidel on R = Wp + M R (M dense or scipy sparse, rows are
    destinations, in the order the blocks cut).  Returns (R, sweeps, last),
    last = ||R_new - R_old||_1 of the final sweep."""
    Wp = np.asarray(Wp, dtype=np.float64)
    nv = len(Wp)
    R = Wp.copy()
    thresh = eps * (1.0 - c) * np.abs(Wp).sum()
    if nv == 0 or (thresh == 0.0 and not np.any(Wp)):
        return R, 0, 0.0
    bounds = block_bounds(nv, n_blocks)
    sweeps, last = 0, np.inf
    while sweeps < max_sweeps:
        old = R.copy()
        for b in range(len(bounds) - 1):
            lo, hi = bounds[b], bounds[b + 1]
            R[lo:hi] = Wp[lo:hi] + (M[lo:hi] @ R)
        sweeps += 1
        last = float(np.abs(R - old).sum())
        if last <= thresh:
            break
    return R, sweeps, last
