"""Weighted graphs on the GPU against the oracle's weighted solve (Def. 3.4
with a_uv = w_uv / sum_x w_ux): integer weights passed as parallel edges,
and real weights on a weighted plan (pr_build_levels_weighted)."""
import sys

import numpy as np
import pytest

from graphgen import config_graph, csr_from_edges, random_digraph, scc_blocks
from oracle.pagerank import pagerank_dense_weighted, pagerank_power_series, transition_T_csr

from _rowcheck import check_rows

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


# ---------------------------------------------------------------- real weights
# A weighted plan (pr_build_levels_weighted): the raw weight of every edge in
# every gather, a_uv = w_uv / s_u (Def. 3.4).

def _real_weights(m, seed, zero_frac=0.1):
    """Uniform(0, 2) weights with a fraction set to zero (some vertices then
    lose every out-weight and act as dangling)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(0.0, 2.0, m) * (rng.random(m) >= zero_frac)


def _dag_with_junctions(seed, n=3000):
    """An acyclic graph of deep chains with junctions (vertices with 2-4 CAC
    sources), rows of 5-32 sources and one collector row with 200 sources, so
    every hop kind of the CAC walk is taken."""
    rng = np.random.default_rng(seed)
    src = rng.integers(0, n - 1, 7000)
    hop = np.where(rng.random(7000) < 0.8, 1 + rng.integers(0, 3, 7000), 1 + rng.integers(0, 1500, 7000))
    dst = np.minimum(src + hop, n - 1)
    keep = dst > src
    src, dst = src[keep], dst[keep]
    coll = n - 1
    extra = rng.choice(n - 1, 200, replace=False)
    mid = n // 2
    extra2 = rng.choice(mid, 12, replace=False)
    src = np.concatenate([src, extra, extra2])
    dst = np.concatenate([dst, np.full(200, coll), np.full(12, mid)])
    keep = dst > src
    perm = rng.permutation(n)
    return csr_from_edges(n, perm[src[keep]], perm[dst[keep]])


def _hub_graph(seed):
    """A random digraph whose vertex 0 has more than 2048 in-edges (a gang
    sums such a row in pieces) and lies in the giant SCC."""
    g = random_digraph(3000, 9000, seed)
    src = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    s2 = np.concatenate([src, np.arange(1, g.n), [0] * 50])
    d2 = np.concatenate([g.col, np.zeros(g.n - 1, np.int64), np.arange(1, 51)])
    return csr_from_edges(g.n, s2, d2)


def _ref_weighted(g, w, W, loops=False, c=C):
    if g.n <= 2500:
        return pagerank_dense_weighted(g.n, g.row_ptr, g.col, w, c, W, loops=loops)
    AT = transition_T_csr(g.n, g.row_ptr, g.col, loops=loops, weight=w)
    R, _, _ = pagerank_power_series(g.n, g.row_ptr, g.col, c, W, eps=1e-15, AT=AT)
    return R


def _solve_w(prm, g, w, W, build=None, c=C, **opts):
    pr, torch = prm
    part = pr.pr_partition(g.row_ptr, g.col)
    lv = pr.pr_build_levels(part, g.row_ptr, g.col, weight=w, **(build or {}))
    Wd = torch.tensor(W, dtype=torch.float64, device="cuda")
    Rd = torch.empty_like(Wd)
    rc, st = pr.pr_solve(lv, c, Wd, Rd, **opts)
    torch.cuda.synchronize()
    return Rd.cpu().numpy(), rc, st, lv, part


# (small_cutoff, team_edges): wavefront and workgroup SCCs in a segment, and
# gangs (hub rows included)
@pytest.mark.parametrize("small,team", [(64, 1 << 30), (8, 1 << 30), (8, 256), (1, 200)])
@pytest.mark.parametrize("seed", range(2))
def test_real_weights_fp64_match_the_definition(prm, small, team, seed):
    """FP64 terms at eps 1e-13, componentwise and plain: every vertex within
    rtol 1e-10 of the oracle's weighted solve (dense up to 2500 vertices, else
    the series with the weighted A^T), on a CAC-heavy DAG, SCC blocks, a
    random digraph and a graph with a hub row."""
    graphs = [("dag", _dag_with_junctions(seed + 5)), ("blocks", scc_blocks(seed + 20, nblocks=40, max_size=60)),
              ("random", random_digraph(2000, 6000, seed + 40))]
    if team < 1 << 30:
        graphs.append(("hub", _hub_graph(seed + 60)))
    for name, g in graphs:
        w = _real_weights(g.m, seed + 7)
        W = np.random.default_rng(seed).uniform(0.5, 1.5, g.n)
        ref = _ref_weighted(g, w, W)
        for method in (0, 1):
            _say("real weights fp64", name, "n", g.n, "small", small, "team", team, "method", method)
            R, rc, st, lv, _ = _solve_w(prm, g, w, W, dict(small_cutoff=small, team_edges=team), eps=1e-13,
                                        precision=1, method=method)
            assert rc == 0
            np.testing.assert_allclose(R, ref, rtol=1e-10, atol=0)
            lv.free()


@pytest.mark.parametrize("rpw", [1, 4, 16, 64])
def test_real_weights_all_row_widths_and_direct_solve(prm, rpw):
    """Every rows_per_wave, with and without the direct solve of small SCCs
    (the weighted matrix I - c A_CC^T in LDS), on wavefront SCCs and, with
    wavefront SCCs up to 16 vertices, on workgroup SCCs."""
    g = scc_blocks(33, nblocks=60, max_size=40)
    w = _real_weights(g.m, 3)
    W = np.random.default_rng(4).uniform(0.5, 1.5, g.n)
    ref = _ref_weighted(g, w, W)
    for direct, small in ((0, 64), (24, 64), (40, 16)):
        _say("real weights rpw", rpw, "direct", direct, "small", small)
        R, rc, st, lv, _ = _solve_w(prm, g, w, W, dict(rows_per_wave=rpw, small_cutoff=small), eps=1e-13, precision=1,
                                    small_direct=direct)
        assert rc == 0
        np.testing.assert_allclose(R, ref, rtol=1e-10, atol=0)
        lv.free()


@pytest.mark.parametrize("loops", [False, True])
def test_real_weights_with_loops(prm, loops):
    """Kept self-loops with real weights: R_v = (W' + sources) / (1 - c a_vv)
    for loop vertices outside SCCs, a_vv inside SCCs."""
    g = random_digraph(800, 3000, 90, loops=True)
    w = _real_weights(g.m, 91)
    W = np.random.default_rng(92).uniform(0.5, 1.5, g.n)
    ref = pagerank_dense_weighted(g.n, g.row_ptr, g.col, w, C, W, loops=loops)
    for method in (0, 1):
        _say("real weights loops", loops, "method", method)
        R, rc, st, lv, _ = _solve_w(prm, g, w, W, dict(keep_loops=int(loops), small_cutoff=16), eps=1e-13,
                                    precision=1, method=method)
        assert rc == 0
        np.testing.assert_allclose(R, ref, rtol=1e-10, atol=0)
        lv.free()


def test_integer_weights_equal_the_expanded_graph(prm):
    """Integer weights on a weighted plan and the same weights passed as
    parallel edges on an unweighted plan: two device paths, one answer (FP64,
    rtol 1e-12)."""
    pr, _ = prm
    g = config_graph("c1_small")
    w = np.random.default_rng(5).integers(1, 5, g.m).astype(np.float64)
    W = np.ones(g.n)
    Rw, rc, st, lv, _ = _solve_w(prm, g, w, W, eps=1e-12, precision=1)
    rp2, col2 = pr.expand_integer_weights(g.row_ptr, g.col, w.astype(np.int64))
    Re, st2 = _solve(prm, g.n, rp2, col2, W, eps=1e-12, precision=1)
    assert rc == 0
    np.testing.assert_allclose(Rw, Re, rtol=1e-12, atol=0)
    lv.free()


@pytest.mark.parametrize("c", [0.85, 0.99])
@pytest.mark.parametrize("tail", [0, 1])
def test_real_weights_mixed_config1_row_by_row(prm, c, tail):
    """The 10k-vertex configuration with real weights, FP32 terms, eps 1e-6:
    the oracle's FP64 residual bound with the weighted A^T is at most eps and
    equals cert_rel (refinement rounds at c = 0.99), rows outside SCCs are
    exact to rounding, and the L1 error against the oracle's series is
    within eps."""
    pr, _ = prm
    g = config_graph("c1_small")
    w = _real_weights(g.m, 17)
    W = np.ones(g.n)
    _say("real weights c1 mixed c", c, "tail", tail)
    R, rc, st, lv, part = _solve_w(prm, g, w, W, c=c, eps=1e-6, precision=0, tail_estimate=tail)
    assert rc == 0 and st["n_not_converged"] == 0
    AT = transition_T_csr(g.n, g.row_ptr, g.col, weight=w)
    bound, _ = check_rows(g, part.comp, part.comp_type, c, R, 1e-6, AT=AT)
    assert st["cert_rel"] == pytest.approx(bound, rel=1e-3)
    ref, _, _ = pagerank_power_series(g.n, g.row_ptr, g.col, c, W, eps=1e-14, AT=AT)
    assert np.abs(R - ref).sum() / ref.sum() <= 1e-6
    if c == 0.99:
        assert st["refine_rounds"] >= 1
    lv.free()


def test_weighted_graph_replay_and_warm_start_refused(prm):
    """Captured-graph replays of a weighted solve are bitwise equal to the
    eager solve; a starting-guess network is refused on a weighted plan."""
    pr, torch = prm
    g = config_graph("c1_small")
    w = _real_weights(g.m, 23)
    W = np.ones(g.n)
    Re, rc, st, lv, part = _solve_w(prm, g, w, W, eps=1e-9, precision=0, use_graph=0)
    assert rc == 0
    Wd = torch.tensor(W, dtype=torch.float64, device="cuda")
    for _ in range(3):
        Rd = torch.empty_like(Wd)
        rc, _ = pr.pr_solve(lv, C, Wd, Rd, eps=1e-9, precision=0, use_graph=1)
        torch.cuda.synchronize()
        assert rc == 0 and np.array_equal(Rd.cpu().numpy(), Re)
    net = pr.Mlp.create(seed=1)
    with pytest.raises(pr.PRError) as ei:
        pr.pr_solve(lv, C, Wd, torch.empty_like(Wd), warm_start=net)
    assert ei.value.code == pr._lib.PR_EINVAL
    net.free()
    lv.free()


def _tiny(n, edges):
    return csr_from_edges(n, [a for a, _ in edges], [b for _, b in edges], drop_loops=False)


@pytest.mark.parametrize("case", ["single", "isolated", "zero_chain", "cycle_zero_edge", "fig1_real", "loop_single"])
def test_weighted_edge_cases(prm, case):
    """Degenerate weighted inputs against the dense weighted solve (FP64):
    no edges at all; a chain whose weights are all zero (A = 0, so R = W); a
    5-cycle with one zero-weight edge (still one SCC in the partition, a
    chain in A); the worked example with real weights; a single vertex with a
    weighted self-loop kept (R = W / (1 - c))."""
    loops = case == "loop_single"
    if case == "single":
        g, w = _tiny(1, []), np.zeros(0)
    elif case == "isolated":
        g, w = _tiny(4, []), np.zeros(0)
    elif case == "zero_chain":
        g = _tiny(6, [(i, i + 1) for i in range(5)])
        w = np.zeros(g.m)
    elif case == "cycle_zero_edge":
        g = _tiny(5, [(i, (i + 1) % 5) for i in range(5)])
        w = np.array([0.0 if g.col[e] == 0 else 1.5 for e in range(g.m)])
    elif case == "fig1_real":
        g = _tiny(8, [(0, 1), (0, 2), (1, 3), (2, 4), (2, 5), (1, 5), (4, 5), (6, 7), (3, 1), (7, 6), (1, 6)])
        w = np.linspace(0.25, 2.5, g.m)
    else:
        g, w = _tiny(1, [(0, 0)]), np.array([2.0])
    W = np.linspace(0.5, 1.5, g.n)
    ref = pagerank_dense_weighted(g.n, g.row_ptr, g.col, w, C, W, loops=loops)
    for method in (0, 1):
        _say("weighted edge case", case, "method", method)
        R, rc, st, lv, _ = _solve_w(prm, g, w, W, dict(keep_loops=int(loops)), eps=1e-13, precision=1,
                                    method=method)
        assert rc == 0
        np.testing.assert_allclose(R, ref, rtol=1e-12, atol=0)
        lv.free()
    if case == "zero_chain":
        np.testing.assert_array_equal(R, W)
    if case == "loop_single":  # R of the last solve (the plain series, truncated at eps 1e-13)
        np.testing.assert_allclose(R, W / (1 - C), rtol=1e-12)
