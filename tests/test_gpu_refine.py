"""GPU parity of the FP64 residual certificate and of iterative refinement
(Sec. 4.4: ||R - R*||_1 <= ||W - (I - cA^T)R||_1 / (1 - c)).

The solve's cert_rel must equal the oracle's FP64 residual bound of the
returned R (same quantity, summed in another order), so it bounds rounding as
well as truncation; with FP32 terms the refinement rounds bring that bound
under eps where the series alone cannot (c = 0.99, or eps below the FP32
rounding floor)."""
import sys

import numpy as np
import pytest

from graphgen import config_graph
from oracle.pagerank import pagerank_power_series, residual_bound, residual_rows

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu-case]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def prm():
    import torch

    import paper_1609_09068_amd as pr

    assert torch.cuda.is_available()
    return pr, torch


@pytest.fixture(scope="module")
def c1(prm):
    pr, torch = prm
    g = config_graph("c1_small")
    part = pr.pr_partition(g.row_ptr, g.col)
    lv = pr.pr_build_levels(part, g.row_ptr, g.col, build_plain=1)
    return g, lv


def _run(prm, lv, g, c, **opts):
    pr, torch = prm
    W = torch.ones(g.n, dtype=torch.float64, device="cuda")
    R = torch.empty_like(W)
    rc, st = pr.pr_solve(lv, c, W, R, **opts)
    torch.cuda.synchronize()
    return rc, st, R.cpu().numpy()


@pytest.mark.parametrize("method", [0, 1])
@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("tail", [0, 1])
def test_certificate_is_the_fp64_residual_bound(prm, c1, method, precision, tail):
    """cert_rel equals the oracle's residual bound of the returned R to within
    the rounding of the two FP64 sums; with refine = -1 it is the truncation
    bound of the series, reported as cert_trunc_rel either way."""
    g, lv = c1
    _say("certificate", method, precision, tail)
    eps = 1e-6 if precision == 0 else 1e-10
    rc, st, R = _run(prm, lv, g, 0.85, method=method, precision=precision, eps=eps, tail_estimate=tail)
    bound, _ = residual_bound(g.n, g.row_ptr, g.col, 0.85, np.ones(g.n), R)
    assert rc == 0 and st["refine_rounds"] == 0
    assert st["cert_rel"] == pytest.approx(bound, rel=1e-3, abs=1e-15), (st["cert_rel"], bound)
    assert bound <= eps
    rc2, st2, R2 = _run(prm, lv, g, 0.85, method=method, precision=precision, eps=eps, tail_estimate=tail, refine=-1)
    assert rc2 == 0 and st2["res_l1"] == 0.0 and st2["cert_rel"] == st2["cert_trunc_rel"]
    assert np.array_equal(R, R2)  # the residual pass does not touch R
    assert st["cert_trunc_rel"] == st2["cert_trunc_rel"]


@pytest.mark.parametrize("method", [0, 1])
def test_refinement_below_the_fp32_floor(prm, c1, method):
    """Mixed precision at eps = 1e-9 (c = 0.85): the FP32 terms alone leave a
    residual bound above eps; refinement rounds (signed correction solves)
    bring the oracle's bound, and the reported one, under eps."""
    g, lv = c1
    _say("refine floor", method)
    eps = 1e-9
    rc0, st0, R0 = _run(prm, lv, g, 0.85, method=method, precision=0, eps=eps, refine=-1)
    b0, AT = residual_bound(g.n, g.row_ptr, g.col, 0.85, np.ones(g.n), R0)
    assert b0 > eps, b0  # the rounding floor of FP32 terms
    rc, st, R = _run(prm, lv, g, 0.85, method=method, precision=0, eps=eps)
    b, _ = residual_bound(g.n, g.row_ptr, g.col, 0.85, np.ones(g.n), R, AT)
    _say("bounds", b0, "->", b, "rounds", st["refine_rounds"], "cert", st["cert_rel"])
    assert rc == 0 and 1 <= st["refine_rounds"] <= 2
    assert b <= eps and st["cert_rel"] == pytest.approx(b, rel=1e-3)
    assert st["edge_iters"] > st0["edge_iters"]  # the correction's terms are counted
    ref, _, _ = pagerank_power_series(g.n, g.row_ptr, g.col, 0.85, np.ones(g.n), eps=1e-14)
    err = np.abs(R - ref)
    assert err.sum() / ref.sum() <= eps
    # rigorous per vertex: |R_v - R*_v| <= ||R - R*||_1 <= cert_abs
    v = int(np.argmax(err))
    _say("worst vertex", v, "abs", err[v], "rel", err[v] / ref[v])
    assert err[v] <= st["cert_abs"] * (1 + 1e-9) + 1e-12 * ref[v]


@pytest.mark.parametrize("tail", [0, 1])
def test_c099_mixed_meets_eps_with_refinement(prm, c1, tail):
    """c = 0.99 in mixed precision, eps = 1e-6: the returned R's FP64 residual
    bound (oracle) is at most eps and equals cert_rel; rows outside SCCs are
    exact up to FP64 rounding."""
    pr, torch = prm
    g, lv = c1
    _say("c=0.99", tail)
    c = 0.99
    rc, st, R = _run(prm, lv, g, c, precision=0, eps=1e-6, tail_estimate=tail)
    r, scale, AT = residual_rows(g.n, g.row_ptr, g.col, c, np.ones(g.n), R)
    bound = np.abs(r).sum() / ((1 - c) * np.abs(R).sum())
    _say("bound", bound, "cert", st["cert_rel"], "rounds", st["refine_rounds"])
    assert rc == 0 and bound <= 1e-6 and st["cert_rel"] == pytest.approx(bound, rel=1e-3)
    part = pr.pr_partition(g.row_ptr, g.col)
    in_scc = part.comp_type[part.comp] == 1
    worst = int(np.argmax(np.where(in_scc, 0.0, np.abs(r) / scale)))
    _say("worst non-SCC row", worst, np.abs(r[worst]) / scale[worst])
    assert np.all(np.abs(r[~in_scc]) <= 1e-12 * scale[~in_scc])


def test_refined_graph_replays_are_bitwise_equal_to_eager(prm, c1):
    """A refined solve replayed from captured graphs (the solve's and the
    correction's, both kept in the plan's graph cache) gives the eager result
    bit for bit, every replay."""
    g, lv = c1
    _say("refine graph replay")
    rc, st, Re = _run(prm, lv, g, 0.85, precision=0, eps=1e-9, use_graph=0)
    assert rc == 0 and st["refine_rounds"] >= 1
    for _ in range(3):
        rc, stg, Rg = _run(prm, lv, g, 0.85, precision=0, eps=1e-9, use_graph=1)
        assert rc == 0 and stg["refine_rounds"] == st["refine_rounds"]
        assert np.array_equal(Re, Rg)


def test_unrefined_bound_above_eps_is_reported(prm, c1):
    """With one round allowed and eps at the FP64 rounding floor the call
    reports what it reached: cert_rel above eps and PR_NOT_CONVERGED, R
    written and far more accurate than the unrefined series."""
    pr, torch = prm
    g, lv = c1
    _say("refine to the FP64 floor")
    rc, st, R = _run(prm, lv, g, 0.85, precision=0, eps=1e-15, refine=1)
    bound, _ = residual_bound(g.n, g.row_ptr, g.col, 0.85, np.ones(g.n), R)
    _say("bound", bound, "cert", st["cert_rel"])
    assert st["refine_rounds"] == 1 and rc == pr._lib.PR_NOT_CONVERGED
    assert st["cert_rel"] > 1e-15 and bound > 1e-15
    assert bound <= 1e-11 and st["cert_rel"] <= 1e-11


@pytest.mark.parametrize("c,want", [(0.85, 0), (0.99, 1)])
def test_auto_precision(prm, c1, c, want):
    """PR_PREC_AUTO: FP32 terms at c = 0.85 and eps 1e-6 (their rounding,
    about 2^-24 / (1-c) = 4e-7, is below eps), FP64 terms at c = 0.99 (6e-6);
    the same result as the explicit choice, bit for bit, and within eps by
    the oracle's residual bound."""
    pr, torch = prm
    g, lv = c1
    rc, st, R = _run(prm, lv, g, c, precision=pr.PR_PREC_AUTO, eps=1e-6, tail_estimate=1)
    rc2, st2, R2 = _run(prm, lv, g, c, precision=want, eps=1e-6, tail_estimate=1)
    bound, _ = residual_bound(g.n, g.row_ptr, g.col, c, np.ones(g.n), R)
    assert rc == 0 and st["precision_used"] == want and st2["precision_used"] == want
    assert np.array_equal(R, R2) and bound <= 1e-6
