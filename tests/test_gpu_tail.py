"""GPU parity of the certified geometric tail estimate of SCC series (solve
option tail_estimate) against the oracle's same rule and the dense solve."""
import itertools
import sys

import numpy as np
import pytest

from graphgen import config_graph, csr_from_edges, random_digraph, scc_blocks
from oracle.componentwise import componentwise_solve
from oracle.pagerank import pagerank_dense, pagerank_power_series
from oracle.partition import partition_theorem

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


def _run(prm, g, W, build, **opts):
    pr, torch = prm
    part = pr.pr_partition(g.row_ptr, g.col)
    lv = pr.pr_build_levels(part, g.row_ptr, g.col, **build)
    Wd = torch.tensor(W, dtype=torch.float64, device="cuda")
    Rd = torch.empty_like(Wd)
    rc, st = pr.pr_solve(lv, C, Wd, Rd, **opts)
    torch.cuda.synchronize()
    return Rd.cpu().numpy(), rc, st, lv


def test_cycle_stops_after_two_terms(prm):
    m = 8
    g = csr_from_edges(m, np.arange(m), (np.arange(m) + 1) % m)
    for small in (64, 1):  # a wavefront, then a workgroup
        _say("tail cycle small_cutoff", small)
        R, rc, st, _ = _run(prm, g, np.ones(m), dict(small_cutoff=small), eps=1e-10, precision=1, tail_estimate=1)
        assert rc == 0 and st["iters_max"] == 2
        assert np.allclose(R, 1.0 / (1.0 - C), rtol=1e-13, atol=0)


def _hub_graph(seed):
    """A random digraph whose vertex 0 has more than 2048 in-edges (a gang
    sums such a row in pieces) and lies in the giant SCC."""
    g = random_digraph(3000, 9000, seed)
    src = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    s2 = np.concatenate([src, np.arange(1, g.n), [0] * 50])
    d2 = np.concatenate([g.col, np.zeros(g.n - 1, np.int64), np.arange(1, 51)])
    return csr_from_edges(g.n, s2, d2)


# (small_cutoff, team_edges): wavefront and workgroup SCCs in a segment, the
# large-component LDS path (team_edges above every SCC), and gangs (hub rows
# included)
@pytest.mark.parametrize("small,team", [(64, 1 << 30), (8, 1 << 30), (8, 256)])
@pytest.mark.parametrize("seed", range(3))
def test_fp64_matches_oracle_rule(prm, small, team, seed):
    """Per-SCC term counts equal the oracle's tail rule (FP64) but for a
    rounding tie, the result is within eps of the dense solve, and fewer terms
    than the plain rule are taken."""
    graphs = [scc_blocks(seed + 20, nblocks=40, max_size=60), random_digraph(2000, 6000, seed + 40)]
    if team < 1 << 30:
        graphs.append(_hub_graph(seed + 60))
    for g in graphs:
        W = np.random.default_rng(seed).uniform(0.5, 1.5, g.n)
        _say("tail fp64 seed", seed, "small", small, "team", team, "n", g.n)
        build = dict(small_cutoff=small, team_edges=team)
        R, rc, st, lv = _run(prm, g, W, build, eps=1e-9, precision=1, tail_estimate=1)
        _, _, st0, _ = _run(prm, g, W, build, eps=1e-9, precision=1)
        assert rc == 0
        Ro, sto = componentwise_solve(g.n, g.row_ptr, g.col, C, W, eps=1e-9, tail=True, return_stats=True)
        part = partition_theorem(g.n, g.row_ptr, g.col)
        scc = part["comp_type"] == 1
        it = lv.debug("iters", n_comp=part["n_comp"])
        d = np.abs(it[scc].astype(np.int64) - sto["iters"][scc])
        assert d.max() <= 1 and np.count_nonzero(d) <= 2, (it[scc][d > 0], sto["iters"][scc][d > 0])
        big = np.argmax(part["comp_size"][scc])
        assert it[scc][big] == sto["iters"][scc][big]
        Rd = pagerank_dense(g.n, g.row_ptr, g.col, C, W) if g.n <= 2500 else None
        if Rd is not None:
            assert np.abs(R - Rd).sum() / Rd.sum() <= 1e-9
        assert np.abs(R - Ro).sum() / Ro.sum() <= 2e-9
        assert st["iters_sum"] < st0["iters_sum"]
        assert st["cert_rel"] <= 1e-9


@pytest.mark.parametrize("team", [65536, 512])
def test_config1_mixed_and_replay(prm, team):
    pr, torch = prm
    g = config_graph("c1_small")
    W = np.ones(g.n)
    ref, _, _ = pagerank_power_series(g.n, g.row_ptr, g.col, C, W, eps=1e-14)
    part = pr.pr_partition(g.row_ptr, g.col)
    lv = pr.pr_build_levels(part, g.row_ptr, g.col, team_edges=team)
    Wd = torch.tensor(W, device="cuda")
    Re = torch.empty_like(Wd)
    _say("tail c1 mixed team", team)
    rc, st = pr.pr_solve(lv, C, Wd, Re, eps=1e-6, tail_estimate=1)
    eager = Re.cpu().numpy()
    assert rc == 0 and np.abs(eager - ref).sum() / ref.sum() <= 1e-6 and st["cert_rel"] <= 1e-6
    Rg = torch.empty_like(Wd)
    for rep in range(3):
        _say("tail replay", rep)
        Rg.fill_(-1.0)
        rc, _ = pr.pr_solve(lv, C, Wd, Rg, eps=1e-6, tail_estimate=1, use_graph=1)
        assert rc == 0 and np.array_equal(Rg.cpu().numpy(), eager)
    with pytest.raises(pr.PRError):
        pr.pr_solve(lv, C, Wd, Rg, tail_estimate=2)


def _const_net(pr, b3):
    """A network whose output is b3 on every row (zero weights): the same
    guess R_0 = s exp(b3) on the GPU and in the oracle."""
    net = pr.Mlp.create(6)
    th = np.zeros(4545, dtype=np.float32)
    th[-1] = b3
    net.set_params(th)
    return net


def test_gang_rejected_guess_with_tail_is_the_plain_start_tail(prm):
    """Every SCC on the gang path with a guess that always falls back: the
    tail rule must act exactly as without a guess, bit for bit."""
    pr, torch = prm
    from graphgen import small_plain

    g = small_plain(seed=1)
    W = np.random.default_rng(3).uniform(0.5, 2.0, g.n)
    build = dict(small_cutoff=1, team_edges=1)
    _say("tail + rejected guess, gangs")
    R0, rc0, st0, lv0 = _run(prm, g, W, build, eps=1e-10, precision=1, tail_estimate=1)
    R1, rc1, st1, lv1 = _run(prm, g, W, build, eps=1e-10, precision=1, tail_estimate=1,
                             warm_start=_const_net(pr, 40.0))
    assert rc0 == 0 and rc1 == 0
    assert st1["ws_accepted"] == 0 and st1["ws_rejected"] == st1["n_iterated"] > 0
    np.testing.assert_array_equal(R1, R0)
    assert st1["iters_sum"] == st0["iters_sum"]


@pytest.mark.parametrize("precision", [1, 0])
def test_gang_kept_guess_with_tail_matches_oracle(prm, precision):
    """Every SCC on the gang path, constant guess kept for most SCCs: the
    per-SCC term counts follow the oracle's rule (r_0 first, rho from r_2 on)
    but for rounding ties (FP64 terms), the result is within eps, and the
    rule saves terms over the guess alone."""
    pr, torch = prm
    from graphgen import small_plain

    g = small_plain(seed=1)
    W = np.random.default_rng(3).uniform(0.5, 2.0, g.n)
    eps = 1e-10 if precision == 1 else 1e-6
    ref, _, _ = pagerank_power_series(g.n, g.row_ptr, g.col, C, W, eps=1e-13)
    build = dict(small_cutoff=1, team_edges=1)
    net = _const_net(pr, 0.5)
    _say("tail + kept guess, gangs, precision", precision)
    R, rc, st, lv = _run(prm, g, W, build, eps=eps, precision=precision, tail_estimate=1, warm_start=net)
    _, _, st0, _ = _run(prm, g, W, build, eps=eps, precision=precision, warm_start=net)
    assert rc == 0
    assert np.abs(R - ref).sum() / ref.sum() <= eps
    assert st["ws_accepted"] == st0["ws_accepted"] > st["n_iterated"] // 2
    assert st["iters_sum"] < st0["iters_sum"]
    if precision == 1:
        _, sto = componentwise_solve(g.n, g.row_ptr, g.col, C, W, eps=eps, tail=True, return_stats=True,
                                     warm_fn=lambda F, Vs, s: np.full(len(Vs), 0.5))
        part = partition_theorem(g.n, g.row_ptr, g.col)
        scc = part["comp_type"] == 1
        assert abs(st["ws_accepted"] - int((sto["accepted"] == 1).sum())) <= 2
        it = lv.debug("iters", n_comp=part["n_comp"])
        d = np.abs(it[scc].astype(np.int64) - sto["iters"][scc])
        assert d.max() <= 1 and np.count_nonzero(d) <= 4, (it[scc][d > 0], sto["iters"][scc][d > 0])


@pytest.mark.parametrize("small,team", [(64, 1 << 30), (8, 1 << 30), (8, 256)])
def test_guess_on_every_scc_with_tail_matches_oracle(prm, small, team):
    """warm_scope 1 (a guess for every SCC: wavefront, workgroup and gang
    SCCs) with the tail estimate, constant guess kept for most SCCs: per-SCC
    term counts follow the oracle's rule but for rounding ties (FP64), the
    result is within eps, and a guess that always falls back is bit for bit
    the plain-start tail."""
    pr, torch = prm
    from graphgen import small_plain

    g = small_plain(seed=1)
    W = np.random.default_rng(3).uniform(0.5, 2.0, g.n)
    eps = 1e-10
    ref, _, _ = pagerank_power_series(g.n, g.row_ptr, g.col, C, W, eps=1e-13)
    build = dict(small_cutoff=small, team_edges=team)
    _say("tail + guess on every SCC", small, team)
    R, rc, st, lv = _run(prm, g, W, build, eps=eps, precision=1, tail_estimate=1, warm_start=_const_net(pr, 0.5),
                         warm_scope=1)
    assert rc == 0 and np.abs(R - ref).sum() / ref.sum() <= eps
    _, sto = componentwise_solve(g.n, g.row_ptr, g.col, C, W, eps=eps, tail=True, return_stats=True,
                                 warm_fn=lambda F, Vs, s: np.full(len(Vs), 0.5))
    part = partition_theorem(g.n, g.row_ptr, g.col)
    scc = part["comp_type"] == 1
    assert abs(st["ws_accepted"] - int((sto["accepted"] == 1).sum())) <= 2
    it = lv.debug("iters", n_comp=part["n_comp"])
    d = np.abs(it[scc].astype(np.int64) - sto["iters"][scc])
    assert d.max() <= 1 and np.count_nonzero(d) <= 4, (it[scc][d > 0], sto["iters"][scc][d > 0])
    R0, _, st0, _ = _run(prm, g, W, build, eps=eps, precision=1, tail_estimate=1)
    R1, _, st1, _ = _run(prm, g, W, build, eps=eps, precision=1, tail_estimate=1,
                         warm_start=_const_net(pr, 40.0), warm_scope=1)
    assert st1["ws_accepted"] == 0
    np.testing.assert_array_equal(R1, R0)
    assert st1["iters_sum"] == st0["iters_sum"]


def test_web_1m_in_the_timed_launch_shape(prm):
    """The 1M-vertex / 10M-edge web-like graph in the launch shapes the
    benchmark's autotuner picks (rows per wave 64, small cutoff 16, gang
    threshold 16384 or 65536 edges), hipGraph replay, mixed precision, eps
    1e-6: the trained starting guess with the tail estimate, and the plain
    start with it, both within 1e-6 of the oracle's FP64 series, certificates
    included."""
    import os

    pr, torch = prm
    g = config_graph("c2_web_1m")
    W = np.ones(g.n)
    ref, _, _ = pagerank_power_series(g.n, g.row_ptr, g.col, C, W, eps=1e-12)
    part = pr.pr_partition(g.row_ptr, g.col)
    path = os.path.join(os.path.dirname(pr.__file__), "data", "warm_web.prmlp")
    net = pr.Mlp.load_file(path)
    Wd = torch.tensor(W, device="cuda")
    R = torch.empty_like(Wd)
    AT = None
    for team in (16384, 65536):
        lv = pr.pr_build_levels(part, g.row_ptr, g.col, rows_per_wave=64, small_cutoff=16, team_edges=team)
        for opts, rep in itertools.product((dict(warm_start=net), {}), range(2)):
            _say("web 1m timed shape team", team, sorted(opts), "replay", rep)
            R.fill_(-1.0)
            rc, st = pr.pr_solve(lv, C, Wd, R, eps=1e-6, precision=0, tail_estimate=1, use_graph=1, **opts)
            assert rc == 0
            Rh = R.cpu().numpy()
            err = np.abs(Rh - ref).sum() / ref.sum()
            assert err <= 1e-6 and st["cert_rel"] <= 1e-6, (err, st["cert_rel"])
            assert st["n_not_converged"] == 0
            AT = check_rows(g, part.comp, part.comp_type, C, Rh, 1e-6, ref=ref, cert_abs=st["cert_abs"], AT=AT)[1]


def test_tail_is_inert_under_the_papers_stop_rule(prm):
    """The estimate certifies against the 1-norm rule only: with the paper's
    max-norm rule the solve is bit for bit the one without it."""
    pr, torch = prm
    g = scc_blocks(31, nblocks=40, max_size=60)
    W = np.random.default_rng(31).uniform(0.5, 1.5, g.n)
    for team in (1 << 30, 256):
        build = dict(small_cutoff=8, team_edges=team)
        _say("tail under PAPER rule, team", team)
        R0, rc0, st0, _ = _run(prm, g, W, build, stop=pr.PR_STOP_PAPER_MAXABS, tol=1e-9, precision=1)
        R1, rc1, st1, _ = _run(prm, g, W, build, stop=pr.PR_STOP_PAPER_MAXABS, tol=1e-9, precision=1,
                               tail_estimate=1)
        assert rc0 == 0 and rc1 == 0
        np.testing.assert_array_equal(R1, R0)
        assert st1["iters_sum"] == st0["iters_sum"]


def test_tail_with_zero_mass_sccs(prm):
    """SCCs that receive no mass (W = 0 on them and on everything above
    them) skip the series; the rest match the oracle's tail rule."""
    pr, torch = prm
    g = scc_blocks(32, nblocks=40, max_size=60)
    part = partition_theorem(g.n, g.row_ptr, g.col)
    rng = np.random.default_rng(32)
    W = rng.uniform(0.5, 1.5, g.n)
    vlevel = part["comp_level"][part["comp"]]
    W[vlevel >= np.percentile(vlevel, 60)] = 0.0  # the upper levels carry no mass
    for team in (1 << 30, 256):
        build = dict(small_cutoff=8, team_edges=team)
        _say("tail zero-mass SCCs, team", team)
        R, rc, st, lv = _run(prm, g, W, build, eps=1e-9, precision=1, tail_estimate=1)
        Ro, sto = componentwise_solve(g.n, g.row_ptr, g.col, C, W, eps=1e-9, tail=True, return_stats=True)
        assert rc == 0
        np.testing.assert_allclose(R, Ro, rtol=2e-9, atol=1e-300)
        it = lv.debug("iters", n_comp=part["n_comp"])
        scc = part["comp_type"] == 1
        d = np.abs(it[scc].astype(np.int64) - sto["iters"][scc])
        assert d.max() <= 1 and np.count_nonzero(d) <= 2
        dead = scc & (sto["iters"] == 0)
        assert dead.any() and (it[dead] == 0).all()


@pytest.mark.parametrize("seed", range(3))
def test_plain_method_with_tail_matches_oracle(prm, seed):
    """The plain whole-graph series stopped on the tail estimate: the same
    term count as the oracle's whole-graph rule in FP64 (hub rows summed in
    pieces included), R within eps of the dense solve, and a replayed graph
    bitwise equal to the eager solve."""
    pr, torch = prm
    g = _hub_graph(60 + seed)
    W = np.random.default_rng(seed).uniform(0.5, 1.5, g.n)
    _say("plain + tail seed", seed)
    Re, rc, st, lv = _run(prm, g, W, dict(build_plain=1), method=1, eps=1e-9, precision=1, tail_estimate=1)
    Rref, kref, _ = pagerank_power_series(g.n, g.row_ptr, g.col, C, W, eps=1e-9, tail=True)
    _, kplain, _ = pagerank_power_series(g.n, g.row_ptr, g.col, C, W, eps=1e-9)
    dense = pagerank_dense(g.n, g.row_ptr, g.col, C, W)
    _say("terms", st["iters_max"], "oracle", kref, "without the estimate", kplain)
    assert rc == 0 and st["iters_max"] == kref and kref < kplain
    assert np.abs(Re - dense).sum() / dense.sum() <= 1e-9
    assert np.allclose(Re, Rref, rtol=1e-11)
    Wd = torch.tensor(W, dtype=torch.float64, device="cuda")
    Rg = torch.empty_like(Wd)
    for _ in range(2):
        rc, stg = pr.pr_solve(lv, C, Wd, Rg, method=1, eps=1e-9, precision=1, tail_estimate=1, use_graph=1)
        torch.cuda.synchronize()
        assert rc == 0 and np.array_equal(Rg.cpu().numpy(), Re)
