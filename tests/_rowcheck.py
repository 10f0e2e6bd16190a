"""Row-by-row parity at full size (shared by the GPU tests; not collected).

The oracle's FP64 residual r = W - (I - cA^T)R of the returned R is formed
row by row (Sec. 4.4).  Rows outside SCCs (one-vertex components and CACs)
are solved exactly in one pass (Sec. 4.3, 4.3.1), so their residual must sit
at FP64 rounding level relative to the terms it is formed from; the 1-norm
of the whole residual bounds the relative error of R.  A vertex wrong by a
few units anywhere shows up here even where a relative 1-norm comparison
with a reference over millions of vertices would not."""
import sys

import numpy as np

from oracle.pagerank import residual_rows


def _say(*a):
    print("[gpu-case]", *a, file=sys.stderr, flush=True)


def check_rows(g, comp, comp_type, c, R, eps, W=None, AT=None, ref=None, cert_abs=None, componentwise=True):
    """Asserts the FP64 residual bound <= eps and, for the componentwise
    method (which solves them exactly), rounding-level residuals on every row
    outside an SCC (the plain series iterates those rows like any other);
    with a reference R*, also the rigorous
    per-vertex bound |R_v - R*_v| <= ||R - R*||_1 <= cert_abs.  Prints the
    worst row, the worst SCC and the worst vertex.  Returns (bound, A^T)."""
    W = np.ones(g.n) if W is None else W
    r, scale, AT = residual_rows(g.n, g.row_ptr, g.col, c, W, R, AT)
    bound = float(np.abs(r).sum() / ((1 - c) * np.abs(R).sum()))
    in_scc = comp_type[comp] == 1
    rel = np.abs(r) / np.maximum(scale, 1e-300)
    worst = int(np.argmax(np.where(in_scc, 0.0, rel)))
    _say(f"residual bound {bound:.3e}; worst row outside SCCs: vertex {worst} |r|/scale {rel[worst]:.2e}")
    scc_ids = np.nonzero(comp_type == 1)[0]
    if len(scc_ids):
        K = len(comp_type)
        rs = np.bincount(comp, weights=np.abs(r), minlength=K)[scc_ids]
        Rs = np.bincount(comp, weights=np.abs(R), minlength=K)[scc_ids]
        k = int(np.argmax(rs / ((1 - c) * Rs)))
        _say(f"worst SCC: component {scc_ids[k]}, ||r_C||/((1-c)||R_C||) = {rs[k] / ((1 - c) * Rs[k]):.2e}")
    assert bound <= eps, bound
    if componentwise:
        assert np.all(rel[~in_scc] <= 1e-12), float(rel[worst])
    if ref is not None:
        err = np.abs(R - ref)
        v = int(np.argmax(err / ref))
        _say(f"worst vertex against the reference: {v}, |dR| {err[v]:.3e}, relative {err[v] / ref[v]:.2e}")
        if cert_abs is not None:
            assert np.all(err <= cert_abs * (1 + 1e-9) + 1e-11 * ref)
    return bound, AT
