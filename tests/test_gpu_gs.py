"""GPU parity of block Gauss-Seidel sweeps inside workgroup SCCs (solve option
gs_blocks; the alternative to the series that Sec. 4.3.2 names) against the
dense solve and the oracle's block Gauss-Seidel, sweep for sweep."""
import sys

import numpy as np
import pytest

from graphgen import config_graph, scc_blocks
from oracle.gauss_seidel import block_gauss_seidel
from oracle.pagerank import pagerank_dense, pagerank_power_series, residual_bound, transition_T_csr
from oracle.partition import partition_theorem

pytestmark = pytest.mark.gpu
C = 0.85
# every SCC of two or more vertices on one workgroup's register path
SHAPE = dict(small_cutoff=1, team_edges=1 << 30)


def _say(*a):
    print("[gpu-case]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def prm():
    import torch

    import paper_1609_09068_amd as pr

    assert torch.cuda.is_available()
    return pr, torch


def _run(prm, g, W, build, weight=None, **opts):
    pr, torch = prm
    part = pr.pr_partition(g.row_ptr, g.col)
    lv = pr.pr_build_levels(part, g.row_ptr, g.col, weight=weight, **build)
    Wd = torch.tensor(W, dtype=torch.float64, device="cuda")
    Rd = torch.empty_like(Wd)
    rc, st = pr.pr_solve(lv, C, Wd, Rd, **opts)
    torch.cuda.synchronize()
    return Rd.cpu().numpy(), rc, st, lv


@pytest.mark.parametrize("blocks", [1, 4, 8])
@pytest.mark.parametrize("seed", range(2))
def test_fp64_matches_dense_and_oracle_sweeps(prm, blocks, seed):
    """FP64 at eps 1e-12: every vertex within rtol 1e-10 of the dense solve;
    each SCC's sweep count equals the oracle's block Gauss-Seidel on the same
    rows (plan order) and the same W', but for a rounding tie."""
    g = scc_blocks(seed + 40, nblocks=40, max_size=60)
    W = np.random.default_rng(seed).uniform(0.5, 1.5, g.n)
    _say("gs fp64 blocks", blocks, "seed", seed)
    R, rc, st, lv = _run(prm, g, W, SHAPE, eps=1e-12, precision=1, gs_blocks=blocks)
    assert rc == 0 and st["n_not_converged"] == 0
    np.testing.assert_allclose(R, pagerank_dense(g.n, g.row_ptr, g.col, C, W), rtol=1e-10, atol=0)
    assert st["cert_rel"] <= 1e-11
    part = partition_theorem(g.n, g.row_ptr, g.col)
    it = lv.debug("iters", n_comp=part["n_comp"])
    wp = lv.debug("wprime")
    perm = lv.debug("perm")
    vbeg = lv.debug("rank_vbeg")
    rcomp = lv.debug("rank_comp")
    AT = transition_T_csr(g.n, g.row_ptr, g.col).tocsr()
    diff = []
    for r in range(len(rcomp)):
        k = rcomp[r]
        if part["comp_type"][k] != 1:
            continue
        rows = perm[vbeg[r]:vbeg[r + 1]]
        M = (C * AT[rows][:, rows]).tocsr()
        _, sweeps, _ = block_gauss_seidel(M, wp[rows], C, 1e-12, blocks)
        diff.append(int(it[k]) - sweeps)
    diff = np.array(diff)
    _say("SCCs", len(diff), "sweep differences", np.count_nonzero(diff))
    assert len(diff) >= 20 and np.abs(diff).max() <= 1 and np.count_nonzero(diff) <= 2


def test_one_block_is_the_series(prm):
    """One block is the Jacobi iteration: the same number of sweeps as the
    series takes terms, SCC by SCC, and the same result to rounding."""
    pr, _ = prm
    g = scc_blocks(47, nblocks=40, max_size=60)
    W = np.ones(g.n)
    R1, rc1, st1, lv1 = _run(prm, g, W, SHAPE, eps=1e-10, precision=1, gs_blocks=1)
    R0, rc0, st0, lv0 = _run(prm, g, W, SHAPE, eps=1e-10, precision=1)
    part = partition_theorem(g.n, g.row_ptr, g.col)
    i1 = lv1.debug("iters", n_comp=part["n_comp"])
    i0 = lv0.debug("iters", n_comp=part["n_comp"])
    scc = part["comp_type"] == 1
    assert rc1 == 0 and rc0 == 0
    assert np.count_nonzero(i1[scc] != i0[scc]) <= 1 and np.abs(i1[scc] - i0[scc]).max() <= 1
    np.testing.assert_allclose(R1, R0, rtol=1e-11, atol=0)


@pytest.mark.parametrize("c_damp", [0.85, 0.99])
def test_config1_mixed_fewer_sweeps_than_terms(prm, c_damp):
    """The 10k-vertex configuration in mixed precision at eps 1e-6 with four
    blocks: the oracle's FP64 residual bound of R is at most eps and equals
    cert_rel, and the SCCs take fewer sweeps than the series takes terms."""
    pr, torch = prm
    g = config_graph("c1_small")
    W = np.ones(g.n)
    part = pr.pr_partition(g.row_ptr, g.col)
    lv = pr.pr_build_levels(part, g.row_ptr, g.col, **SHAPE)
    Wd = torch.tensor(W, dtype=torch.float64, device="cuda")
    out = {}
    for blocks in (0, 4):
        _say("gs c1 mixed c", c_damp, "blocks", blocks)
        Rd = torch.empty_like(Wd)
        rc, st = pr.pr_solve(lv, c_damp, Wd, Rd, eps=1e-6, precision=0, gs_blocks=blocks)
        torch.cuda.synchronize()
        assert rc == 0
        out[blocks] = (Rd.cpu().numpy(), st)
    R, st = out[4]
    bound, _ = residual_bound(g.n, g.row_ptr, g.col, c_damp, W, R)
    assert bound <= 1e-6 and st["cert_rel"] == pytest.approx(bound, rel=1e-3)
    _say("terms (series)", out[0][1]["iters_sum"], "sweeps (4 blocks)", st["iters_sum"],
         "refinement rounds", out[0][1]["refine_rounds"], st["refine_rounds"])
    if c_damp == 0.85:  # (at 0.99 refinement rounds add their own sweeps and terms)
        assert st["iters_sum"] < out[0][1]["iters_sum"]
    ref, _, _ = pagerank_power_series(g.n, g.row_ptr, g.col, c_damp, W, eps=1e-13)
    assert np.abs(R - ref).sum() / ref.sum() <= 1e-6
    lv.free()


def test_replay_and_refusals(prm):
    pr, torch = prm
    g = scc_blocks(51, nblocks=30, max_size=40)
    R, rc, st, lv = _run(prm, g, np.ones(g.n), SHAPE, eps=1e-8, gs_blocks=4, use_graph=0)
    Wd = torch.ones(g.n, dtype=torch.float64, device="cuda")
    for rep in range(3):
        _say("gs replay", rep)
        Rg = torch.empty_like(Wd)
        rc, _ = pr.pr_solve(lv, C, Wd, Rg, eps=1e-8, gs_blocks=4, use_graph=1)
        torch.cuda.synchronize()
        assert rc == 0 and np.array_equal(Rg.cpu().numpy(), R)
    # the captured graph belongs to its block count: switching counts under
    # replay gives each count's own eager result
    for blocks in (1, 8, 4):
        Re, _, _, _ = _run(prm, g, np.ones(g.n), SHAPE, eps=1e-8, gs_blocks=blocks, use_graph=0)
        Rg = torch.empty_like(Wd)
        rc, _ = pr.pr_solve(lv, C, Wd, Rg, eps=1e-8, gs_blocks=blocks, use_graph=1)
        torch.cuda.synchronize()
        assert rc == 0 and np.array_equal(Rg.cpu().numpy(), Re), blocks
    for bad in (dict(gs_blocks=9), dict(gs_blocks=4, tail_estimate=1), dict(gs_blocks=-1)):
        with pytest.raises(pr.PRError) as ei:
            pr.pr_solve(lv, C, Wd, torch.empty_like(Wd), **bad)
        assert ei.value.code == pr._lib.PR_EINVAL
    lvw = pr.pr_build_levels(pr.pr_partition(g.row_ptr, g.col), g.row_ptr, g.col, weight=np.ones(g.m))
    with pytest.raises(pr.PRError):
        pr.pr_solve(lvw, C, Wd, torch.empty_like(Wd), gs_blocks=4)
