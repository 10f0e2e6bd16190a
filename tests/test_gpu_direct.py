"""GPU parity of the direct solve of small SCCs (the paper's choice for small
SCCs in the per-component method dispatch of Sec. 4.3), through the C ABI,
against the oracle's dense per-component solve."""
import sys

import numpy as np
import pytest

from graphgen import config_graph, scc_blocks
from oracle.componentwise import componentwise_solve
from oracle.pagerank import pagerank_dense
from oracle.partition import partition_theorem

pytestmark = pytest.mark.gpu
C = 0.85


def _say(*a):
    print("[gpu-case]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def prm():
    import torch

    import paper_1609_09068_amd as pr

    assert torch.cuda.is_available()
    return pr, torch


def _run(prm, g, W, build, **opts):
    pr, torch = prm
    part = pr.pr_partition(g.row_ptr, g.col)
    lv = pr.pr_build_levels(part, g.row_ptr, g.col, **build)
    Wd = torch.tensor(W, dtype=torch.float64, device="cuda")
    Rd = torch.empty_like(Wd)
    rc, st = pr.pr_solve(lv, C, Wd, Rd, **opts)
    torch.cuda.synchronize()
    return Rd.cpu().numpy(), rc, st, lv


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("limit", [8, 24])
def test_blocks_fp64_match_oracle(prm, seed, limit):
    """Many SCCs of 2-24 vertices: those up to `limit` solved directly, the
    rest by the series at eps 1e-14; equal to the oracle's direct route and
    to the whole-graph dense solve to rounding, with zero terms counted for
    every directly solved SCC."""
    g = scc_blocks(seed)
    W = np.random.default_rng(seed).uniform(0.5, 1.5, g.n)
    _say("direct blocks seed", seed, "limit", limit)
    R, rc, st, lv = _run(prm, g, W, dict(small_cutoff=64), eps=1e-14, precision=1, small_direct=limit)
    assert rc == 0
    Ro, sto = componentwise_solve(g.n, g.row_ptr, g.col, C, W, eps=1e-14, direct_max=limit, return_stats=True)
    Rd = pagerank_dense(g.n, g.row_ptr, g.col, C, W)
    assert np.allclose(R, Ro, rtol=1e-11, atol=0)
    assert np.allclose(R, Rd, rtol=1e-11, atol=0)
    part = partition_theorem(g.n, g.row_ptr, g.col)
    it = lv.debug("iters", n_comp=part["n_comp"])
    # component ids of the library and of the oracle agree (canonical numbering)
    direct = (part["comp_type"] == 1) & (part["comp_size"] <= limit)
    assert direct.sum() >= 3
    assert np.all(it[direct] == 0)
    assert np.all(it[(part["comp_type"] == 1) & ~direct] > 0)
    assert st["cert_rel"] <= 1e-12


def test_direct_is_tolerance_independent(prm):
    """A graph of small SCCs only: with every SCC solved directly the result
    is the dense solve whatever eps asks for."""
    g = scc_blocks(7, nblocks=40, max_size=20)
    W = np.ones(g.n)
    Rd = pagerank_dense(g.n, g.row_ptr, g.col, C, W)
    for eps in (1e-2, 1e-6):
        _say("direct loose eps", eps)
        R, rc, st, _ = _run(prm, g, W, dict(small_cutoff=64), eps=eps, precision=0, small_direct=24)
        assert rc == 0 and st["iters_max"] == 0
        assert np.allclose(R, Rd, rtol=1e-12, atol=0)


def test_config1_mixed_with_direct(prm):
    """The 10k-vertex configuration (SCCs of 5-100 vertices): the direct
    solve of the small ones inside the mixed-precision series stays within
    the 1e-6 bound of the oracle's FP64 direct route, and saves terms."""
    g = config_graph("c1_small")
    W = np.ones(g.n)
    Ro = componentwise_solve(g.n, g.row_ptr, g.col, C, W, eps=1e-13, direct_max=24)
    R0, _, st0, _ = _run(prm, g, W, dict(small_cutoff=64), eps=1e-6)
    _say("c1 direct mixed")
    R1, rc, st1, _ = _run(prm, g, W, dict(small_cutoff=64), eps=1e-6, small_direct=24)
    assert rc == 0
    err = np.abs(R1 - Ro).sum() / Ro.sum()
    assert err <= 1e-6, err
    assert st1["cert_rel"] <= 1e-6
    assert st1["iters_sum"] < st0["iters_sum"]


def test_direct_graph_replay_and_bad_option(prm):
    pr, torch = prm
    g = scc_blocks(3)
    part = pr.pr_partition(g.row_ptr, g.col)
    lv = pr.pr_build_levels(part, g.row_ptr, g.col, small_cutoff=64)
    Wd = torch.ones(g.n, dtype=torch.float64, device="cuda")
    Re = torch.empty_like(Wd)
    pr.pr_solve(lv, C, Wd, Re, small_direct=24)
    eager = Re.cpu().numpy()
    Rg = torch.empty_like(Wd)
    for rep in range(3):
        _say("direct replay", rep)
        Rg.fill_(-1.0)
        rc, _ = pr.pr_solve(lv, C, Wd, Rg, small_direct=24, use_graph=1)
        assert rc == 0 and np.array_equal(Rg.cpu().numpy(), eager)
    with pytest.raises(pr.PRError):
        pr.pr_solve(lv, C, Wd, Rg, small_direct=25)
