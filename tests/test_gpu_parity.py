"""GPU parity: the HIP path (through the C ABI) against the CPU oracle."""
import sys

import numpy as np
import pytest

from graphgen import config_graph, csr_from_edges, random_digraph
from oracle.componentwise import componentwise_solve
from oracle.pagerank import pagerank_dense, pagerank_power_series
from oracle.partition import partition_arrays_equal, partition_theorem

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


def _solve(prm, g, W, c=C, build=None, **opts):
    pr, torch = prm
    part = pr.pr_partition(g.row_ptr, g.col)
    lv = pr.pr_build_levels(part, g.row_ptr, g.col, **(build or {}))
    Wd = torch.tensor(W, dtype=torch.float64, device="cuda")
    Rd = torch.empty_like(Wd)
    rc, st = pr.pr_solve(lv, c, Wd, Rd, **opts)
    torch.cuda.synchronize()
    return Rd.cpu().numpy(), rc, st, lv, part


def _rel_l1(a, b):
    return float(np.abs(a - b).sum() / max(np.abs(b).sum(), 1e-300))


def _g(n, edges):
    return csr_from_edges(n, [a for a, _ in edges], [b for _, b in edges])


TINY = {
    "fig1": (8, [(0, 1), (0, 2), (1, 3), (2, 4), (2, 5), (1, 5), (4, 5), (6, 7), (3, 1), (7, 6), (1, 6)]),
    "cycle5": (5, [(i, (i + 1) % 5) for i in range(5)]),
    "chain9": (9, [(i, i + 1) for i in range(8)]),
    "star": (7, [(0, i) for i in range(1, 7)] + [(i, 0) for i in range(1, 7)]),
    "isolated": (4, []),
    "single": (1, []),
}


@pytest.mark.parametrize("name", sorted(TINY))
@pytest.mark.parametrize("prec", [0, 1])
def test_tiny_graphs_match_dense(prm, name, prec):
    n, edges = TINY[name]
    g = _g(n, edges)
    W = np.linspace(0.5, 1.5, n)
    _say("tiny", name, "prec", prec)
    R, rc, st, _, _ = _solve(prm, g, W, eps=1e-12, precision=prec)
    ref = pagerank_dense(n, g.row_ptr, g.col, C, W)
    assert rc == 0
    tol = 1e-11 if prec == 1 else 2e-6
    assert _rel_l1(R, ref) <= tol


@pytest.mark.parametrize("seed", range(8))
def test_random_graphs_fp64(prm, seed):
    g = random_digraph(300 + 40 * seed, 900 + 100 * seed, seed)
    W = np.random.default_rng(seed).random(g.n) + 0.01
    _say("random fp64 seed", seed)
    R, rc, st, _, _ = _solve(prm, g, W, eps=1e-12, precision=1)
    ref = pagerank_dense(g.n, g.row_ptr, g.col, C, W)
    assert rc == 0 and _rel_l1(R, ref) <= 1e-11


def test_loops_and_duplicates(prm):
    g = random_digraph(200, 900, 3, loops=True, duplicates=True)
    W = np.ones(g.n)
    _say("loops+duplicates")
    R, rc, _, _, _ = _solve(prm, g, W, eps=1e-12, precision=1)
    ref = pagerank_dense(g.n, g.row_ptr, g.col, C, W)
    assert _rel_l1(R, ref) <= 1e-11


@pytest.fixture(scope="module")
def c1():
    g = config_graph("c1_small")
    W = np.ones(g.n)
    ref, _, _ = pagerank_power_series(g.n, g.row_ptr, g.col, C, W, eps=1e-14)
    return g, W, ref


@pytest.mark.parametrize("rpw", [1, 4, 16, 64])
@pytest.mark.parametrize("small", [0, 16, 256])
def test_config1_fp64_all_kernel_shapes(prm, c1, rpw, small):
    g, W, ref = c1
    build = dict(rows_per_wave=rpw)
    if small:
        build["small_cutoff"] = small
    else:
        build["small_cutoff"] = 1  # every SCC through a workgroup team
        build["team_edges"] = 200  # and most teams with several workgroups
    _say("c1 fp64 rpw", rpw, "small", small)
    R, rc, st, lv, _ = _solve(prm, g, W, build=build, eps=1e-10, precision=1)
    assert rc == 0
    assert _rel_l1(R, ref) <= 1e-10
    assert st["cert_rel"] <= 1e-10


def test_config1_iterations_and_wprime_match_oracle(prm, c1):
    """Per-SCC iteration counts (paper stop rule) and W' after eq. PR:levels."""
    g, W, _ = c1
    part = partition_theorem(g.n, g.row_ptr, g.col)
    Ro, sto = componentwise_solve(g.n, g.row_ptr, g.col, C, W, part=part, stop="paper", tol=1e-9,
                                  return_stats=True)
    _say("c1 paper-mode iterations")
    R, rc, st, lv, p = _solve(prm, g, W, stop=1, tol=1e-9, precision=1)
    assert partition_arrays_equal(p.as_dict(), part)
    it = lv.debug("iters", n_comp=part["n_comp"])
    scc = part["comp_type"] == 1
    # equal except where the max of a term sits within rounding of tol
    diff = np.nonzero(it[scc] != sto["iters"][scc])[0]
    assert len(diff) <= 2, (it[scc][diff], sto["iters"][scc][diff])
    wp = lv.debug("wprime")
    assert np.allclose(wp, sto["wprime"], rtol=1e-12, atol=0)
    assert _rel_l1(R, Ro) <= 1e-9


@pytest.mark.parametrize("prec", [0, 1])
def test_config1_plain(prm, c1, prec):
    g, W, ref = c1
    _say("c1 plain prec", prec)
    R, rc, st, _, _ = _solve(prm, g, W, eps=1e-10 if prec else 1e-6, precision=prec, method=1)
    _, k_or, _ = pagerank_power_series(g.n, g.row_ptr, g.col, C, W, eps=1e-10 if prec else 1e-6)
    assert rc == 0
    if prec:
        assert _rel_l1(R, ref) <= 1e-10
        assert st["iters_max"] == k_or
    else:
        assert _rel_l1(R, ref) <= 1e-6
        assert abs(st["iters_max"] - k_or) <= 1


def test_config1_mixed_precision(prm, c1):
    g, W, ref = c1
    _say("c1 mixed")
    R, rc, st, _, _ = _solve(prm, g, W, eps=1e-6, precision=0)
    assert rc == 0 and _rel_l1(R, ref) <= 1e-6


def test_gangs_and_determinism(prm, c1):
    pr, torch = prm
    g, W, ref = c1
    part = pr.pr_partition(g.row_ptr, g.col)
    lv = pr.pr_build_levels(part, g.row_ptr, g.col, small_cutoff=1, team_edges=100)
    assert lv.info()["n_gang_scc"] > 1
    Wd = torch.tensor(W, device="cuda")
    outs = []
    for rep in range(3):
        _say("determinism rep", rep)
        Rd = torch.empty_like(Wd)
        pr.pr_solve(lv, C, Wd, Rd, eps=1e-8, precision=0)
        outs.append(Rd.cpu().numpy())
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[0], outs[2])
    # FP32 series terms: the error floor sits a few 1e-7 above eps here
    assert _rel_l1(outs[0], ref) <= 1e-6


def test_graph_replay_matches_eager(prm, c1):
    pr, torch = prm
    g, W, _ = c1
    part = pr.pr_partition(g.row_ptr, g.col)
    lv = pr.pr_build_levels(part, g.row_ptr, g.col)
    Wd = torch.tensor(W, device="cuda")
    Re = torch.empty_like(Wd)
    _say("graph: eager")
    pr.pr_solve(lv, C, Wd, Re, eps=1e-8)
    eager = Re.cpu().numpy()
    Rg = torch.empty_like(Wd)
    for rep in range(4):
        _say("graph: replay", rep)
        Rg.fill_(-7.0)
        torch.cuda.synchronize()
        x = torch.randn(1000, device="cuda").sum().item()  # eager work between replays
        rc, st = pr.pr_solve(lv, C, Wd, Rg, eps=1e-8, use_graph=1)
        assert rc == 0 and np.array_equal(Rg.cpu().numpy(), eager), rep
        del x


def test_error_paths(prm, c1):
    pr, torch = prm
    g, W, _ = c1
    part = pr.pr_partition(g.row_ptr, g.col)
    lv = pr.pr_build_levels(part, g.row_ptr, g.col, build_plain=0)
    Wd = torch.tensor(W, device="cuda")
    Rd = torch.zeros_like(Wd)
    for c in (0.0, 1.0, -0.5, float("nan")):
        with pytest.raises(pr.PRError):
            pr.pr_solve(lv, c, Wd, Rd)
    with pytest.raises(pr.PRError):
        pr.pr_solve(lv, C, Wd, Rd, eps=0.0)
    with pytest.raises(pr.PRError):
        pr.pr_solve(lv, C, Wd, Rd, method=1)  # plan without the plain CSR
    _say("error: negative W")
    Wbad = Wd.clone()
    Wbad[5] = -1.0
    with pytest.raises(pr.PRError) as ei:
        pr.pr_solve(lv, C, Wbad, Rd)
    assert ei.value.code == -1
    Wbad[5] = float("inf")
    with pytest.raises(pr.PRError):
        pr.pr_solve(lv, C, Wbad, Rd)
    assert float(Rd.abs().sum()) == 0.0  # nothing written
    _say("error: max_iter")
    rc, st = pr.pr_solve(lv, C, Wd, Rd, max_iter=1)
    assert rc == pr.PR_NOT_CONVERGED and st["n_not_converged"] > 0
    # a partition of another graph is rejected
    g2 = random_digraph(g.n, 3000, 9)
    with pytest.raises(pr.PRError):
        pr.pr_build_levels(part, g2.row_ptr, g2.col)


def test_zero_weights_and_sparse_weights(prm):
    g = config_graph("c1_small", seed=3)
    W = np.zeros(g.n)
    W[::97] = 1.0
    _say("sparse W")
    R, rc, st, _, _ = _solve(prm, g, W, eps=1e-10, precision=1)
    ref, _, _ = pagerank_power_series(g.n, g.row_ptr, g.col, C, W, eps=1e-14)
    assert rc == 0 and _rel_l1(R, ref) <= 1e-10
    W0 = np.zeros(g.n)
    R0, rc, st, _, _ = _solve(prm, g, W0, eps=1e-10, precision=1)
    assert rc == 0 and np.all(R0 == 0.0)


@pytest.mark.parametrize("c", [0.5, 0.99])
def test_damping_extremes(prm, c):
    g = config_graph("c1_small", seed=2)
    W = np.ones(g.n)
    _say("damping", c)
    R, rc, st, _, _ = _solve(prm, g, W, c=c, eps=1e-10, precision=1)
    ref, _, _ = pagerank_power_series(g.n, g.row_ptr, g.col, c, W, eps=1e-14)
    assert rc == 0 and _rel_l1(R, ref) <= 1e-10


@pytest.fixture(scope="module")
def c2():
    g = config_graph("c2_web_1m")
    W = np.ones(g.n)
    ref, k, _ = pagerank_power_series(g.n, g.row_ptr, g.col, C, W, eps=1e-13)
    return g, W, ref


@pytest.mark.parametrize("method", [0, 1])
def test_config2_full_size_mixed(prm, c2, method):
    """1M vertices / 10M edges in the benchmark's launch configuration."""
    g, W, ref = c2
    _say("c2 full size mixed method", method)
    R, rc, st, lv, p = _solve(prm, g, W, eps=1e-6, precision=0, method=method)
    assert rc == 0
    err = _rel_l1(R, ref)
    _say("c2 rel_l1", err, "iters_max", st["iters_max"], "ms", st["time_ms"])
    assert err <= 1e-6
    # row by row: residual bound, exact rows outside SCCs, per-vertex error
    check_rows(g, p.comp, p.comp_type, C, R, 1e-6, ref=ref, cert_abs=st["cert_abs"], componentwise=method == 0)
    # partition of the full graph is bit-exact
    if method == 0:
        assert partition_arrays_equal(p.as_dict(), partition_theorem(g.n, g.row_ptr, g.col))


def test_config3_full_size(prm):
    """5M vertices / 49M edges, 300 levels, no giant SCC: the partition is
    bit-exact with the oracle's, and the benchmark's headline solve (mixed
    precision, gang starting guess, tail estimate, eps 1e-6) and the plain
    method both meet the oracle's FP64 residual bound, which holds at any
    size: ||R - R*||_1 <= ||W - (I - cA^T)R||_1 / (1 - c)."""
    import os

    pr, torch = prm
    g = config_graph("c3_deep_5m")
    W = np.ones(g.n)
    _say("c3 partition")
    part = pr.pr_partition(g.row_ptr, g.col)
    assert partition_arrays_equal(part.as_dict(), partition_theorem(g.n, g.row_ptr, g.col))
    lv = pr.pr_build_levels(part, g.row_ptr, g.col)
    net = pr.Mlp.load_file(os.path.join(os.path.dirname(pr.__file__), "data", "warm_web.prmlp"))
    Wd = torch.tensor(W, device="cuda")
    AT = None
    for method, opts in ((0, dict(warm_start=net, tail_estimate=1)), (1, {})):
        _say("c3 full size method", method, sorted(opts))
        R = torch.empty_like(Wd)
        rc, st = pr.pr_solve(lv, C, Wd, R, eps=1e-6, precision=0, method=method, use_graph=1, **opts)
        assert rc == 0 and st["cert_rel"] <= 1e-6 and st["n_not_converged"] == 0
        bound, AT = check_rows(g, part.comp, part.comp_type, C, R.cpu().numpy(), 1e-6, W=W, AT=AT,
                               componentwise=method == 0)
        assert st["cert_rel"] >= 0.999 * bound


def test_autotuner_sweeps_caches_and_stays_exact(prm, c1, tmp_path, monkeypatch):
    pr, torch = prm
    g, W, ref = c1
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("PR_AUTOTUNE_CACHE", str(cache))
    part = pr.pr_partition(g.row_ptr, g.col)
    _say("autotune sweep")
    lv = pr.pr_build_levels(part, g.row_ptr, g.col, autotune=2)
    info = lv.info()
    assert info["rows_per_wave"] in (1, 4, 16, 64)
    assert info["small_cutoff"] in (16, 64) and info["team_edges"] in (16384, 65536)
    assert info["seg_waves"] in (2, 3)
    lines = cache.read_text().split()
    assert len(lines) == 5 and int(lines[1]) == info["rows_per_wave"] and int(lines[4]) == info["seg_waves"]
    # cached: the same choice without a sweep (the file is not appended to)
    lv2 = pr.pr_build_levels(part, g.row_ptr, g.col, autotune=1)
    keys = ("rows_per_wave", "small_cutoff", "team_edges", "seg_waves")
    assert {k: lv2.info()[k] for k in keys} == {k: info[k] for k in keys}
    assert len(cache.read_text().split()) == 5
    Wd = torch.tensor(W, device="cuda")
    Rd = torch.empty_like(Wd)
    pr.pr_solve(lv2, C, Wd, Rd, eps=1e-10, precision=1)
    assert _rel_l1(Rd.cpu().numpy(), ref) <= 1e-10
    with pytest.raises(pr.PRError):
        pr.pr_build_levels(part, g.row_ptr, g.col, autotune=3)


@pytest.mark.parametrize("L", [255, 256, 1000, 3000])
def test_long_chain_closed_form(prm, L):
    """A chain v1 -> ... -> vL is one CAC spanning several items: with W = 1,
    R_j = (1 - c^j) / (1 - c) (a closed form of the sum over the single path)."""
    pr, torch = prm
    _say("chain", L)
    g = csr_from_edges(L, np.arange(L - 1), np.arange(1, L))
    part = pr.pr_partition(g.row_ptr, g.col)
    assert part.n_comp == 1 and part.comp_type[0] == 0
    lv = pr.pr_build_levels(part, g.row_ptr, g.col)
    Wd = torch.ones(L, dtype=torch.float64, device="cuda")
    Rd = torch.empty_like(Wd)
    pr.pr_solve(lv, C, Wd, Rd, precision=1)
    exact = (1.0 - C ** (np.arange(L) + 1.0)) / (1.0 - C)
    np.testing.assert_allclose(Rd.cpu().numpy(), exact, rtol=1e-13)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_random_dag_cacs(prm, seed):
    """Acyclic graphs: every component is a CAC or a single vertex; many
    vertices have several CAC sources (junctions), chains cross items and
    wavefronts.  Exact up to rounding against the oracle's sweep."""
    pr, torch = prm
    _say("dag", seed)
    rng = np.random.default_rng(seed)
    n = 4000
    # edges i -> j with j > i: mostly short hops (deep chains), some long ones
    src = rng.integers(0, n - 1, 9000)
    hop = np.where(rng.random(9000) < 0.8, 1 + rng.integers(0, 3, 9000), 1 + rng.integers(0, 2000, 9000))
    dst = np.minimum(src + hop, n - 1)
    keep = dst > src
    perm = rng.permutation(n)  # vertex ids not in topological order
    g = csr_from_edges(n, perm[src[keep]], perm[dst[keep]])
    W = rng.uniform(0.1, 2.0, n)
    part = pr.pr_partition(g.row_ptr, g.col)
    assert (part.comp_type == 0).all()
    lv = pr.pr_build_levels(part, g.row_ptr, g.col)
    Wd = torch.tensor(W, device="cuda")
    Rd = torch.empty_like(Wd)
    pr.pr_solve(lv, C, Wd, Rd, precision=1)
    from oracle.componentwise import componentwise_solve

    ref = componentwise_solve(g.n, g.row_ptr, g.col, C, W)
    np.testing.assert_allclose(Rd.cpu().numpy(), ref, rtol=1e-12)
    # bitwise reproducible
    Rd2 = torch.empty_like(Wd)
    pr.pr_solve(lv, C, Wd, Rd2, precision=1)
    assert np.array_equal(Rd.cpu().numpy(), Rd2.cpu().numpy())


@pytest.mark.parametrize("rpw", [16, 64])
@pytest.mark.parametrize("prec", [0, 1])
def test_three_workgroups_per_cu_variant_is_bitwise_equal(prm, c1, rpw, prec):
    """The tail-estimate segment kernel at three workgroups per CU
    (seg_waves = 3) does the same arithmetic in the same order as at two: the
    result is bitwise equal, eager and replayed, and the plan reports the
    variant it runs."""
    pr, torch = prm
    g, W, ref = c1
    part = pr.pr_partition(g.row_ptr, g.col)
    Wd = torch.tensor(W, device="cuda")
    out = {}
    for waves in (2, 3):
        lv = pr.pr_build_levels(part, g.row_ptr, g.col, rows_per_wave=rpw, small_cutoff=64, seg_waves=waves)
        assert lv.info()["seg_waves"] == waves
        for graph in (0, 1, 1):
            _say("seg_waves", waves, "rpw", rpw, "prec", prec, "graph", graph)
            Rd = torch.empty_like(Wd)
            rc, st = pr.pr_solve(lv, C, Wd, Rd, eps=1e-6 if prec == 0 else 1e-10, precision=prec,
                                 tail_estimate=1, use_graph=graph)
            torch.cuda.synchronize()
            assert rc == 0
            out.setdefault(waves, []).append(Rd.cpu().numpy())
        lv.free()
    for r in out[2] + out[3]:
        assert np.array_equal(r, out[2][0])
    assert _rel_l1(out[3][0], ref) <= (1e-6 if prec == 0 else 1e-10)


def test_seg_waves_reports_the_kernel_that_runs(prm, c1):
    """Asked for three workgroups per CU where that variant does not exist
    (4 rows per wavefront, or a weighted plan) the plan reports two."""
    pr, torch = prm
    g, W, ref = c1
    part = pr.pr_partition(g.row_ptr, g.col)
    lv = pr.pr_build_levels(part, g.row_ptr, g.col, rows_per_wave=4, seg_waves=3)
    assert lv.info()["seg_waves"] == 2
    lv.free()
    lv = pr.pr_build_levels(part, g.row_ptr, g.col, weight=np.ones(g.m), rows_per_wave=64, seg_waves=3)
    assert lv.info()["seg_waves"] == 2
    lv.free()
    lv = pr.pr_build_levels(part, g.row_ptr, g.col, rows_per_wave=64, seg_waves=3)
    assert lv.info()["seg_waves"] == 3
    lv.free()
