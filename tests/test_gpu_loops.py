"""GPU parity with self-loops kept in A (build option keep_loops), through the
C ABI, against the oracle's loop-aware routes."""
import sys

import numpy as np
import pytest

from graphgen import config_graph, csr_from_edges, random_digraph, scc_blocks
from oracle.componentwise import componentwise_solve
from oracle.pagerank import pagerank_dense, pagerank_power_series

pytestmark = pytest.mark.gpu
C = 0.85


@pytest.fixture(scope="module")
def prm():
    import torch

    import paper_1609_09068_amd as pr

    assert torch.cuda.is_available()
    return pr, torch


def _with_loops(g, frac, seed):
    rng = np.random.default_rng(seed)
    src = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    lv = rng.choice(g.n, int(frac * g.n), replace=False)
    return csr_from_edges(g.n, np.concatenate([src, lv]), np.concatenate([g.col, lv]), drop_loops=False)


def _solve(prm, g, W, build=None, **opts):
    pr, torch = prm
    part = pr.pr_partition(g.row_ptr, g.col)
    lv = pr.pr_build_levels(part, g.row_ptr, g.col, keep_loops=1, build_plain=1, **(build or {}))
    Wd = torch.tensor(W, dtype=torch.float64, device="cuda")
    Rd = torch.empty_like(Wd)
    rc, st = pr.pr_solve(lv, C, Wd, Rd, **opts)
    torch.cuda.synchronize()
    return Rd.cpu().numpy(), rc, st


TINY = {
    "lone": (1, [(0, 0)]),
    "loop_then_sink": (2, [(0, 0), (0, 1)]),
    "chain_mid_loop": (5, [(0, 1), (1, 1), (1, 2), (2, 3), (3, 3), (3, 4)]),
    "cycle_with_loop": (4, [(0, 1), (1, 2), (2, 3), (3, 0), (2, 2)]),
    "double_loop": (3, [(0, 0), (0, 0), (0, 1), (1, 2), (2, 1)]),
}


@pytest.mark.parametrize("name", sorted(TINY))
@pytest.mark.parametrize("direct", [0, 24])
def test_tiny_loop_graphs_match_dense(prm, name, direct):
    n, edges = TINY[name]
    g = csr_from_edges(n, [a for a, _ in edges], [b for _, b in edges], dedupe=False, drop_loops=False)
    W = np.linspace(0.5, 1.5, n)
    print("[gpu-case] loops tiny", name, direct, file=sys.stderr, flush=True)
    R, rc, st = _solve(prm, g, W, eps=1e-14, precision=1, small_direct=direct)
    assert rc == 0
    assert np.allclose(R, pagerank_dense(n, g.row_ptr, g.col, C, W, loops=True), rtol=1e-12, atol=0)


@pytest.mark.parametrize("seed", range(3))
def test_random_and_blocks_with_loops(prm, seed):
    for g0 in (random_digraph(3000, 9000, seed + 300), scc_blocks(seed + 5)):
        g = _with_loops(g0, 0.2, seed)
        W = np.random.default_rng(seed).uniform(0.5, 1.5, g.n)
        print("[gpu-case] loops random n", g.n, "seed", seed, file=sys.stderr, flush=True)
        R, rc, st = _solve(prm, g, W, eps=1e-13, precision=1)
        Ro = componentwise_solve(g.n, g.row_ptr, g.col, C, W, eps=1e-13, loops=True)
        assert rc == 0 and np.allclose(R, Ro, rtol=1e-10, atol=0)


@pytest.mark.parametrize("method", [0, 1])
def test_config1_with_loops(prm, method):
    g = _with_loops(config_graph("c1_small"), 0.1, 9)
    W = np.ones(g.n)
    ref, _, _ = pagerank_power_series(g.n, g.row_ptr, g.col, C, W, eps=1e-14, loops=True)
    print("[gpu-case] loops c1 method", method, file=sys.stderr, flush=True)
    R, rc, st = _solve(prm, g, W, method=method, eps=1e-10, precision=1)
    assert rc == 0
    assert np.abs(R - ref).sum() / ref.sum() <= 1e-10
    # and the default (loops ignored) is a different vector on the same input
    ref0, _, _ = pagerank_power_series(g.n, g.row_ptr, g.col, C, W, eps=1e-14)
    assert np.abs(ref0 - ref).sum() / ref.sum() > 1e-3
