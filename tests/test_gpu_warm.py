"""Warm-started componentwise solve on the GPU against the oracle.

The start does not change the answer (Def. 3.5: R_C = (I - c A_CC^T)^{-1}
W'_C whatever R_0 is), so results are compared with the oracle's R within
the stop rule's bound.  A guess that is always rejected must reproduce the
plain start exactly (same iterations, same R bit for bit), and the
accept/reject decisions follow the oracle's rule evaluated on the oracle's
own (float64) network.
"""
import sys

import numpy as np
import pytest

from graphgen import config_graph, random_digraph, small_plain
from oracle import warmstart as ws
from oracle.componentwise import componentwise_solve
from oracle.pagerank import pagerank_power_series

pytestmark = pytest.mark.gpu
C = 0.85


def _say(*a):
    print("[gpu-case]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def prm():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1609_09068_amd as pr

    return pr, torch


def _solve(pr, torch, g, W, **kw):
    part = pr.pr_partition(g.row_ptr, g.col)
    lv = pr.pr_build_levels(part, g.row_ptr, g.col, **{k: kw.pop(k) for k in list(kw)
                                                        if k in ("team_edges", "small_cutoff", "rows_per_wave")})
    Wd = torch.tensor(W, device="cuda")
    R = torch.empty_like(Wd)
    rc, st = pr.pr_solve(lv, C, Wd, R, **kw)
    return R.cpu().numpy(), st, lv, part


SPLITS = [(64, 65536), (1, 100)]  # (small_cutoff, team_edges): segment items only; gangs


@pytest.mark.parametrize("split", SPLITS)
@pytest.mark.parametrize("precision", [1, 0])
def test_warm_result_matches_oracle(prm, split, precision):
    """Small-config graph: every kind of SCC item, and (second split) the
    larger SCCs on the gang path."""
    pr, torch = prm
    small_cutoff, team_edges = split
    _say("warm parity", split, precision)
    g = small_plain(seed=1)
    W = np.random.default_rng(3).uniform(0.5, 2.0, g.n)
    ref, _, _ = pagerank_power_series(g.n, g.row_ptr, g.col, C, W, eps=1e-13)
    net = pr.Mlp.create(5)
    eps = 1e-10 if precision == 1 else 1e-6
    R, st, lv, _ = _solve(pr, torch, g, W, team_edges=team_edges, small_cutoff=small_cutoff, eps=eps,
                          precision=precision, warm_start=net, warm_scope=1)
    err = np.abs(R - ref).sum() / ref.sum()
    assert err <= (eps if precision == 1 else 1e-6), err
    assert st["ws_accepted"] + st["ws_rejected"] == st["n_iterated"]
    if team_edges == 100:
        assert lv.info()["n_gang_scc"] > 1


@pytest.mark.parametrize("split", SPLITS)
def test_rejected_guess_is_the_plain_start(prm, split):
    pr, torch = prm
    small_cutoff, team_edges = split
    _say("warm rejected", split)
    g = small_plain(seed=1)
    W = np.ones(g.n)
    net = pr.Mlp.create(6)
    th = np.zeros(4545, dtype=np.float32)
    th[-1] = 40.0  # output exp(40) times the scale: never passes the residual test
    net.set_params(th)
    R0, st0, lv0, _ = _solve(pr, torch, g, W, team_edges=team_edges, small_cutoff=small_cutoff, eps=1e-8,
                             precision=1)
    R1, st1, lv1, part = _solve(pr, torch, g, W, team_edges=team_edges, small_cutoff=small_cutoff, eps=1e-8,
                                precision=1, warm_start=net, warm_scope=1)
    assert st1["ws_accepted"] == 0 and st1["ws_rejected"] == st1["n_iterated"] > 0
    np.testing.assert_array_equal(R1, R0)
    np.testing.assert_array_equal(lv1.debug("iters", n_comp=part.n_comp), lv0.debug("iters", n_comp=part.n_comp))
    assert st1["iters_sum"] == st0["iters_sum"]


def test_accept_decisions_follow_the_oracle(prm):
    """The same network (float64 on the CPU, BF16 on the GPU) accepts nearly
    the same components; only guesses whose residual ties with the first
    plain term within rounding may differ."""
    pr, torch = prm
    g = small_plain(seed=1)
    W = np.ones(g.n)
    rng_net = pr.Mlp.create(8)
    th = rng_net.get_params().astype(np.float64)
    # push the guess near the answer: output ~ log(1 + c) on every row
    P = ws.unpack(th)
    P["W3"][:] *= 0.05
    P["b3"][:] = np.log(3.0)
    rng_net.set_params(th.astype(np.float32))
    _, sto = componentwise_solve(g.n, g.row_ptr, g.col, C, W, eps=1e-8, return_stats=True,
                                 warm=th.astype(np.float32).astype(np.float64))
    acc_oracle = int((sto["accepted"] == 1).sum())
    n_scc = int((sto["accepted"] >= 0).sum())
    _, st, _, _ = _solve(pr, torch, g, W, eps=1e-8, precision=1, warm_start=rng_net, warm_scope=1)
    assert st["n_iterated"] == n_scc
    assert abs(st["ws_accepted"] - acc_oracle) <= max(2, n_scc // 20), (st["ws_accepted"], acc_oracle, n_scc)


@pytest.mark.parametrize("scope", [0, 1])
def test_warm_full_size_mixed(prm, scope):
    pr, torch = prm
    _say("warm c2 full", scope)
    g = config_graph("c2_web_1m")
    W = np.ones(g.n)
    ref, _, _ = pagerank_power_series(g.n, g.row_ptr, g.col, C, W, eps=1e-12)
    net = pr.Mlp.create(7)
    R, st, lv, _ = _solve(pr, torch, g, W, eps=1e-6, precision=0, warm_start=net, warm_scope=scope)
    err = np.abs(R - ref).sum() / ref.sum()
    assert err <= 1e-6, err
    n_gang = lv.info()["n_gang_scc"]
    assert n_gang >= 1
    decided = st["ws_accepted"] + st["ws_rejected"]
    assert decided == (n_gang if scope == 0 else st["n_iterated"])


def test_random_graph_warm_fp64(prm):
    pr, torch = prm
    g = random_digraph(3000, 12000, seed=21)
    W = np.random.default_rng(21).uniform(0, 3, g.n)
    ref, _, _ = pagerank_power_series(g.n, g.row_ptr, g.col, C, W, eps=1e-14)
    net = pr.Mlp.create(21)
    R, st, _, _ = _solve(pr, torch, g, W, eps=1e-11, precision=1, warm_start=net, warm_scope=1,
                         team_edges=256, small_cutoff=8)
    assert np.abs(R - ref).sum() / ref.sum() <= 1e-11
