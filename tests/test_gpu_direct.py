"""GPU parity of the direct solve of small SCCs (the paper's choice for small
SCCs in the per-component method dispatch of Sec. 4.3), through the C ABI,
against the oracle's dense per-component solve: SCCs run by one wavefront (up
to 24 vertices) and by one workgroup (up to 80)."""
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
        pr.pr_solve(lv, C, Wd, Rg, small_direct=81)


@pytest.mark.parametrize("seed", range(3))
@pytest.mark.parametrize("limit", [50, 80])
def test_workgroup_blocks_match_oracle(prm, seed, limit):
    """SCCs of 2-80 vertices on a plan whose wavefront SCCs stop at 16
    vertices, so those of 17-80 run on a workgroup: every SCC up to `limit`
    solved directly (zero terms), the rest by the series at eps 1e-14; equal
    to the oracle's direct route and to the whole-graph dense solve."""
    g = scc_blocks(seed + 100, nblocks=30, min_size=2, max_size=80)
    W = np.random.default_rng(seed).uniform(0.5, 1.5, g.n)
    _say("workgroup direct blocks seed", seed, "limit", limit)
    R, rc, st, lv = _run(prm, g, W, dict(small_cutoff=16), eps=1e-14, precision=1, small_direct=limit)
    assert rc == 0
    Ro = componentwise_solve(g.n, g.row_ptr, g.col, C, W, eps=1e-14, direct_max=limit)
    Rd = pagerank_dense(g.n, g.row_ptr, g.col, C, W)
    np.testing.assert_allclose(R, Ro, rtol=1e-11, atol=0)
    np.testing.assert_allclose(R, Rd, rtol=1e-11, atol=0)
    part = partition_theorem(g.n, g.row_ptr, g.col)
    it = lv.debug("iters", n_comp=part["n_comp"])
    scc = part["comp_type"] == 1
    direct = scc & (part["comp_size"] <= limit)
    assert (direct & (part["comp_size"] > 24)).sum() >= 3  # workgroup SCCs among them
    assert np.all(it[direct] == 0)
    assert np.all(it[scc & ~direct] > 0)
    assert st["cert_rel"] <= 1e-12


@pytest.mark.parametrize("precision", [0, 1])
def test_wavefront_and_workgroup_direct_agree_bitwise(prm, precision):
    """SCCs of 2-24 vertices solved directly once as wavefront items (small
    cutoff 64) and once as workgroup items (small cutoff 1): the same
    elimination in the same order, so the same R bit for bit."""
    g = scc_blocks(11, nblocks=40, max_size=24)
    W = np.random.default_rng(12).uniform(0.5, 1.5, g.n)
    _say("direct wave vs workgroup", precision)
    Ra, rca, sta, _ = _run(prm, g, W, dict(small_cutoff=64), eps=1e-10, precision=precision, small_direct=24)
    Rb, rcb, stb, _ = _run(prm, g, W, dict(small_cutoff=1), eps=1e-10, precision=precision, small_direct=24)
    assert rca == 0 and rcb == 0 and sta["iters_max"] == 0 and stb["iters_max"] == 0
    assert np.array_equal(Ra, Rb)
    assert stb["cert_rel"] == pytest.approx(sta["cert_rel"], rel=1e-6, abs=1e-18)


def test_config1_workgroup_direct(prm):
    """The 10k-vertex configuration (200 SCCs, 162 of them of 17-80
    vertices) with wavefront SCCs up to 16 vertices and the direct solve up
    to 80: every SCC solved directly, within the 1e-6 bound of the oracle's
    FP64 direct route in mixed precision; graph replays bitwise equal to the
    eager solve."""
    pr, torch = prm
    g = config_graph("c1_small")
    W = np.ones(g.n)
    Ro = componentwise_solve(g.n, g.row_ptr, g.col, C, W, eps=1e-13, direct_max=80)
    R0, _, st0, _ = _run(prm, g, W, dict(small_cutoff=16), eps=1e-6)
    _say("c1 workgroup direct mixed")
    R1, rc, st1, lv = _run(prm, g, W, dict(small_cutoff=16), eps=1e-6, small_direct=80)
    assert rc == 0
    err = np.abs(R1 - Ro).sum() / Ro.sum()
    assert err <= 1e-6, err
    assert st1["cert_rel"] <= 1e-6
    assert st1["iters_sum"] < st0["iters_sum"]
    part = partition_theorem(g.n, g.row_ptr, g.col)
    it = lv.debug("iters", n_comp=part["n_comp"])
    scc = part["comp_type"] == 1
    assert np.all(it[scc & (part["comp_size"] <= 80)] == 0)
    Wd = torch.ones(g.n, dtype=torch.float64, device="cuda")
    Rg = torch.empty_like(Wd)
    for rep in range(3):
        Rg.fill_(-1.0)
        rc, _ = pr.pr_solve(lv, C, Wd, Rg, eps=1e-6, small_direct=80, use_graph=1)
        assert rc == 0 and np.array_equal(Rg.cpu().numpy(), R1)
