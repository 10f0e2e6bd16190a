"""Weighted graphs (integer transition weights passed as parallel edges) on
the GPU against the oracle's weighted dense solve (Def. 3.4 with
a_uv = w_uv / sum_x w_ux)."""
import sys

import numpy as np
import pytest

from graphgen import config_graph, random_digraph, scc_blocks
from oracle.pagerank import pagerank_dense_weighted, pagerank_power_series

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


def _solve(prm, n, rp, col, W, build=None, **opts):
    pr, torch = prm
    part = pr.pr_partition(rp, col)
    lv = pr.pr_build_levels(part, rp, col, **(build or {}))
    Wd = torch.tensor(W, dtype=torch.float64, device="cuda")
    Rd = torch.empty_like(Wd)
    rc, st = pr.pr_solve(lv, C, Wd, Rd, **opts)
    torch.cuda.synchronize()
    assert rc == 0
    return Rd.cpu().numpy(), st


@pytest.mark.parametrize("seed", range(3))
@pytest.mark.parametrize("loops", [False, True])
def test_weighted_fp64_matches_dense(prm, seed, loops):
    pr, _ = prm
    graphs = [random_digraph(800, 3000, seed + 90, loops=loops), scc_blocks(seed + 95, nblocks=30, max_size=40)]
    for g in graphs:
        w = np.random.default_rng(seed).integers(1, 6, g.m)
        W = np.random.default_rng(seed + 1).uniform(0.5, 1.5, g.n)
        ref = pagerank_dense_weighted(g.n, g.row_ptr, g.col, w, C, W, loops=loops)
        rp2, col2 = pr.expand_integer_weights(g.row_ptr, g.col, w)
        for method, build in ((0, dict(small_cutoff=64)), (0, dict(small_cutoff=8, team_edges=256)), (1, {})):
            _say("weighted seed", seed, "loops", loops, "n", g.n, "method", method, build)
            build = dict(build, keep_loops=int(loops))
            R, st = _solve(prm, g.n, rp2, col2, W, build, eps=1e-13, precision=1, method=method)
            np.testing.assert_allclose(R, ref, rtol=1e-10, atol=0)


def test_weighted_config1_mixed(prm):
    """The 10k-vertex configuration with weights 1..4, mixed precision at
    eps 1e-6, with and without the tail estimate, against the oracle's FP64
    series on the same (expanded) graph."""
    pr, _ = prm
    g = config_graph("c1_small")
    w = np.random.default_rng(5).integers(1, 5, g.m)
    rp2, col2 = pr.expand_integer_weights(g.row_ptr, g.col, w)
    W = np.ones(g.n)
    ref, _, _ = pagerank_power_series(g.n, rp2, col2, C, W, eps=1e-13)
    for tail in (0, 1):
        _say("weighted c1 mixed tail", tail)
        R, st = _solve(prm, g.n, rp2, col2, W, eps=1e-6, precision=0, tail_estimate=tail)
        assert np.abs(R - ref).sum() / ref.sum() <= 1e-6 and st["cert_rel"] <= 1e-6
