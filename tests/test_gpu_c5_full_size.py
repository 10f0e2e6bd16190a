"""GPU parity at the largest single-GPU size: the web-like graph of 20M
vertices and 200M edges (giant SCC of half the vertices, 8% dangling).

 * The host partition is bit-exact with the oracle's (Theorem 3.1: the
   partition is unique, so component ids and levels are one array each).
 * At c = 0.85 and c = 0.99, in mixed precision (FP32 terms), the
   componentwise solve (with and without the tail estimate) and the plain
   series return R whose FP64 residual bound, computed by the oracle, is at
   most 1e-6 (Sec. 4.4: ||R - R*||_1 <= ||W - (I - cA^T)R||_1 / (1 - c)),
   and the solve's own cert_rel is that bound.
 * Row by row, for the componentwise method: every row outside an SCC
   (one-vertex components and CACs, solved exactly in one pass, Sec. 4.3.1)
   has a residual at FP64 rounding level, so no vertex there can be wrong by
   more than rounding; the worst row and the worst SCC are printed."""
import sys
import time

import pytest

from graphgen import config_graph
from oracle.pagerank import transition_T_csr
from oracle.partition import partition_arrays_equal, partition_theorem

from _rowcheck import check_rows

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu-case]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def c5():
    import torch

    import paper_1609_09068_amd as pr

    assert torch.cuda.is_available()
    t0 = time.perf_counter()
    g = config_graph("c5_web_20m", log=lambda *a: _say(f"{time.perf_counter() - t0:.0f}s", *a))
    _say(f"c5 graph n={g.n} m={g.m} in {time.perf_counter() - t0:.0f}s")
    part = pr.pr_partition(g.row_ptr, g.col)
    _say(f"host partition done at {time.perf_counter() - t0:.0f}s: {part.n_comp} components, {part.n_levels} levels")
    lv = pr.pr_build_levels(part, g.row_ptr, g.col, build_plain=1)
    _say(f"plan built at {time.perf_counter() - t0:.0f}s")
    AT = transition_T_csr(g.n, g.row_ptr, g.col)
    _say(f"oracle A^T built at {time.perf_counter() - t0:.0f}s")
    yield pr, torch, g, part, lv, AT
    lv.free()
    part.free()


def test_c5_partition_bit_exact(c5):
    pr, torch, g, part, lv, AT = c5
    t0 = time.perf_counter()
    ref = partition_theorem(g.n, g.row_ptr, g.col)
    _say(f"oracle partition {time.perf_counter() - t0:.0f}s")
    assert partition_arrays_equal(part.as_dict(), ref)


@pytest.mark.parametrize("c", [0.85, 0.99])
@pytest.mark.parametrize("path", ["componentwise", "componentwise+tail", "plain"])
def test_c5_mixed_meets_1e6_row_by_row(c5, c, path):
    pr, torch, g, part, lv, AT = c5
    _say("c5 solve", c, path)
    W = torch.ones(g.n, dtype=torch.float64, device="cuda")
    R = torch.empty_like(W)
    opts = dict(method=1 if path == "plain" else 0, tail_estimate=1 if path.endswith("tail") else 0,
                precision=0, eps=1e-6)
    rc, st = pr.pr_solve(lv, c, W, R, **opts)
    torch.cuda.synchronize()
    Rh = R.cpu().numpy()
    _say(f"rc={rc} cert_rel={st['cert_rel']:.3e} trunc={st['cert_trunc_rel']:.3e} "
         f"rounds={st['refine_rounds']} terms_max={st['iters_max']} ms={st['time_ms']:.1f}")
    assert rc == 0 and st["n_not_converged"] == 0
    bound, _ = check_rows(g, part.comp, part.comp_type, c, Rh, 1e-6, AT=AT, componentwise=path != "plain")
    assert st["cert_rel"] >= 0.999 * bound and st["cert_rel"] <= 1e-6
