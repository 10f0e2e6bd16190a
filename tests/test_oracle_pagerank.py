"""Pins for the oracle's PageRank routes (Defs. 3.4-3.6, Sec. 4.3, Sec. 4.4)."""
import itertools
import math

import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

from graphgen import config_graph, csr_from_edges, random_digraph, scc_blocks
from oracle import componentwise as CW
from oracle import pagerank as PR

C = 0.85


def _g(n, edges):
    return csr_from_edges(n, [a for a, _ in edges], [b for _, b in edges])


def _all_routes(g, W, c=C):
    """Every oracle route to R^(3), as (name, vector)."""
    out = [("dense", PR.pagerank_dense(g.n, g.row_ptr, g.col, c, W))]
    out.append(("series", PR.pagerank_power_series(g.n, g.row_ptr, g.col, c, W, eps=1e-15)[0]))
    out.append(("componentwise", CW.componentwise_solve(g.n, g.row_ptr, g.col, c, W, eps=1e-15)))
    return out


# ---------------------------------------------------------------- closed forms

@pytest.mark.parametrize("m", [2, 3, 7])
def test_cycle_and_complete_digraph(m):
    cyc = _g(m, [(i, (i + 1) % m) for i in range(m)])
    full = _g(m, [(i, j) for i in range(m) for j in range(m) if i != j])
    for g in (cyc, full):
        for name, R in _all_routes(g, np.ones(m)):
            assert np.allclose(R, 1.0 / (1.0 - C), rtol=1e-12), name


def test_chain():
    k = 9
    g = _g(k, [(i, i + 1) for i in range(k - 1)])
    expect = np.array([(1 - C ** (j + 1)) / (1 - C) for j in range(k)])
    for name, R in _all_routes(g, np.ones(k)):
        assert np.allclose(R, expect, rtol=1e-13), name


def test_out_tree_and_in_tree():
    b, depth = 3, 3
    nodes = [(0,)]
    edges, index = [], {(0,): 0}
    frontier = [(0,)]
    for _ in range(depth):
        nxt = []
        for p in frontier:
            for j in range(b):
                ch = p + (j,)
                index[ch] = len(index)
                edges.append((index[p], index[ch]))
                nxt.append(ch)
        frontier = nxt
    n = len(index)
    dep = np.array([len(k) - 1 for k in sorted(index, key=index.get)])
    out_tree = _g(n, edges)
    exp_out = np.array([sum((C / b) ** i for i in range(d + 1)) for d in dep])
    for name, R in _all_routes(out_tree, np.ones(n)):
        assert np.allclose(R, exp_out, rtol=1e-13), name
    in_tree = _g(n, [(v, u) for u, v in edges])
    height = depth - dep
    exp_in = np.array([sum((b * C) ** i for i in range(h + 1)) for h in height])
    for name, R in _all_routes(in_tree, np.ones(n)):
        assert np.allclose(R, exp_in, rtol=1e-13), name


def test_bidirected_star():
    m = 6
    g = _g(m + 1, [(0, i) for i in range(1, m + 1)] + [(i, 0) for i in range(1, m + 1)])
    hub = (1 + C * m) / (1 - C * C)
    leaf = 1 + C * hub / m
    for name, R in _all_routes(g, np.ones(m + 1)):
        assert np.isclose(R[0], hub, rtol=1e-12) and np.allclose(R[1:], leaf, rtol=1e-12), name


def test_singletons_keep_their_weight():
    # Sec. 4.3: a component of isolated vertices has R = W (loops ignored)
    rp = np.array([0, 1, 1, 2], dtype=np.int64)
    col = np.array([0, 2], dtype=np.int32)  # vertex 0 has a loop, 2 a loop
    W = np.array([0.3, 2.0, 5.0])
    assert np.allclose(PR.pagerank_dense(3, rp, col, C, W), W)
    assert np.allclose(CW.componentwise_solve(3, rp, col, C, W), W)


def test_duplicate_edges_count_with_multiplicity():
    # 0 -> 1 twice, 0 -> 2 once: a_01 = 2/3, a_02 = 1/3
    rp = np.array([0, 3, 3, 3], dtype=np.int64)
    col = np.array([1, 1, 2], dtype=np.int32)
    W = np.ones(3)
    R = PR.pagerank_dense(3, rp, col, C, W)
    assert np.allclose(R, [1.0, 1 + C * 2 / 3, 1 + C / 3])
    assert np.allclose(CW.componentwise_solve(3, rp, col, C, W, eps=1e-15), R)


# ------------------------------------------------------ independent routes

@pytest.mark.parametrize("seed", range(6))
def test_definition_routes_agree(seed):
    """Def. 3.4 eigenvector rescaled by Def. 3.5 equals the linear solve."""
    g = random_digraph(25, 55, seed)
    rng = np.random.default_rng(seed)
    W = rng.random(g.n) + 0.1
    Rd = PR.pagerank_dense(g.n, g.row_ptr, g.col, C, W)
    R1 = PR.pagerank_r1(g.n, g.row_ptr, g.col, C, W)
    R3 = PR.r3_from_r1(g.n, g.row_ptr, g.col, C, R1, W)
    assert np.allclose(R3, Rd, rtol=1e-10)
    assert np.isclose(np.sum(Rd / np.sum(Rd)), 1.0) and np.allclose(Rd / Rd.sum(), R1, rtol=1e-9)


def test_random_walk_definition():
    """Def. 3.6: expected visit counts of stopped random walks."""
    g = _g(6, [(0, 1), (1, 2), (2, 0), (2, 3), (3, 4), (4, 3), (1, 5)])
    W = np.ones(6)
    est = PR.pagerank_random_walks(g.n, g.row_ptr, g.col, C, W, walks_per_unit=6000, seed=11)
    Rd = PR.pagerank_dense(g.n, g.row_ptr, g.col, C, W)
    assert np.allclose(est, Rd, rtol=0.05)
    # the transposed operator gives clearly different values
    Rwrong = np.linalg.solve(np.eye(6) - C * PR.transition_dense(6, g.row_ptr, g.col), W)
    assert not np.allclose(est, Rwrong, rtol=0.05)


def _path_sums(n, edges, W, c):
    """Sum over every directed path ending at u of W_start * prod c/outdeg."""
    out = {u: [b for a, b in edges if a == u] for u in range(n)}
    R = np.zeros(n)

    def walk(u, weight):
        R[u] += weight
        for v in out[u]:
            walk(v, weight * c / len(out[u]))

    for s in range(n):
        walk(s, W[s])
    return R


@pytest.mark.parametrize("seed", range(5))
def test_brute_force_paths_on_dags(seed):
    rng = np.random.default_rng(100 + seed)
    n = 9
    edges = sorted({(int(a), int(b)) for a, b in rng.integers(0, n, size=(16, 2)) if a < b})
    g = _g(n, edges)
    W = rng.random(n)
    expect = _path_sums(n, edges, W, C)
    for name, R in _all_routes(g, W):
        assert np.allclose(R, expect, rtol=1e-12), name


# ---------------------------------------------------------- stop rules

def test_paper_mode_iterations_on_a_cycle():
    """Sec. 5.2: a bottom-level SCC needs about log(tol)/log(c) iterations;
    on a cycle P_k = c^k exactly, so the listing's rule stops after 128."""
    m = 10
    g = _g(m, [(i, (i + 1) % m) for i in range(m)])
    expect = math.ceil(math.log(1e-9) / math.log(C))
    assert expect == 128
    _, k, _ = PR.pagerank_power_series(g.n, g.row_ptr, g.col, C, np.ones(m), stop="paper", tol=1e-9)
    assert k == expect
    _, st_ = CW.componentwise_solve(g.n, g.row_ptr, g.col, C, np.ones(m), stop="paper", tol=1e-9,
                                    return_stats=True)
    assert st_["iters"].tolist() == [expect]


def test_cert_rule_iterations_on_a_cycle():
    m = 5
    g = _g(m, [(i, (i + 1) % m) for i in range(m)])
    _, k, _ = PR.pagerank_power_series(g.n, g.row_ptr, g.col, C, np.ones(m), eps=1e-6)
    # ||P_k||_1 = c^k m <= eps (1-c) m
    assert k == math.ceil(math.log(1e-6 * (1 - C)) / math.log(C))


@pytest.mark.parametrize("eps", [1e-3, 1e-6, 1e-9])
def test_certificate_bounds_relative_error(eps):
    g = config_graph("c1_small", seed=2)
    W = np.ones(g.n)
    ref, _, _ = PR.pagerank_power_series(g.n, g.row_ptr, g.col, C, W, eps=1e-15)
    Rp, _, _ = PR.pagerank_power_series(g.n, g.row_ptr, g.col, C, W, eps=eps)
    Rc = CW.componentwise_solve(g.n, g.row_ptr, g.col, C, W, eps=eps)
    for R in (Rp, Rc):
        err = np.sum(np.abs(R - ref)) / np.sum(ref)
        assert err <= eps
        assert np.all(R <= ref * (1 + 1e-12))  # monotone from below (Sec. 4.4)


def test_linearity_in_w():
    g = random_digraph(60, 150, 5)
    rng = np.random.default_rng(0)
    W1, W2 = rng.random(g.n), rng.random(g.n)
    f = lambda W: CW.componentwise_solve(g.n, g.row_ptr, g.col, C, W, eps=1e-15)
    assert np.allclose(f(2 * W1 + 3 * W2), 2 * f(W1) + 3 * f(W2), rtol=1e-11)


edge_lists = st.integers(min_value=1, max_value=40).flatmap(
    lambda n: st.tuples(st.just(n), st.lists(
        st.tuples(st.integers(0, n - 1), st.integers(0, n - 1)), max_size=3 * n)))


@settings(max_examples=80, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(edge_lists, st.floats(0.05, 0.99))
def test_property_componentwise_equals_dense(ne, c):
    n, edges = ne
    g = _g(n, edges)
    W = np.linspace(0.5, 1.5, n)
    Rd = PR.pagerank_dense(g.n, g.row_ptr, g.col, c, W)
    Rc = CW.componentwise_solve(g.n, g.row_ptr, g.col, c, W, eps=1e-15)
    assert np.allclose(Rc, Rd, rtol=1e-9, atol=0)


def test_planted_transpose_mistake_is_caught():
    """Using A instead of A^T must fail the chain closed form."""
    k = 6
    g = _g(k, [(i, i + 1) for i in range(k - 1)])
    A = PR.transition_dense(k, g.row_ptr, g.col)
    wrong = np.linalg.solve(np.eye(k) - C * A, np.ones(k))
    expect = np.array([(1 - C ** (j + 1)) / (1 - C) for j in range(k)])
    assert not np.allclose(wrong, expect, rtol=1e-6)


def test_residual_bound_covers_the_error():
    from graphgen import random_digraph
    from oracle.pagerank import pagerank_dense, residual_bound

    g = random_digraph(300, 1500, seed=17)
    c = 0.85
    W = np.random.default_rng(17).uniform(0, 2, g.n)
    exact = pagerank_dense(g.n, g.row_ptr, g.col, c, W)
    rng = np.random.default_rng(3)
    for scale in (1e-3, 1e-6, 0.3):
        R = exact * (1 + scale * rng.normal(size=g.n))
        bound, _ = residual_bound(g.n, g.row_ptr, g.col, c, W, R)
        err = np.abs(R - exact).sum() / np.abs(R).sum()
        assert err <= bound
        assert bound < 50 * err  # and it is not vacuous on these perturbations
    bound, _ = residual_bound(g.n, g.row_ptr, g.col, c, W, exact)
    assert bound < 1e-13


# ------------------------------------------- direct solve of small SCCs

@pytest.mark.parametrize("m", [2, 5, 9])
def test_direct_small_scc_cycle_closed_form(m):
    """A bare m-cycle with W = 1 has R = 1/(1-c) on every vertex, exactly:
    the direct route must hit it to rounding, with no series term counted."""
    g = _g(m, [(i, (i + 1) % m) for i in range(m)])
    R, st = CW.componentwise_solve(g.n, g.row_ptr, g.col, C, np.ones(m), eps=1e-3, direct_max=m,
                                   return_stats=True)
    assert np.allclose(R, 1.0 / (1.0 - C), rtol=1e-14, atol=0)
    assert st["iters"].max() == 0
    # the series at eps 1e-3 is visibly off, so the test does tell the routes apart
    Ri = CW.componentwise_solve(g.n, g.row_ptr, g.col, C, np.ones(m), eps=1e-3)
    assert not np.allclose(Ri, 1.0 / (1.0 - C), rtol=1e-6, atol=0)


@pytest.mark.parametrize("seed", range(5))
def test_direct_small_sccs_equal_dense(seed):
    """Many small SCCs on several levels: direct solves of every SCC up to
    16 vertices plus the series on the larger ones equal the whole-graph
    LAPACK solve (an independent route) to rounding."""
    g = scc_blocks(seed)
    W = np.random.default_rng(seed).uniform(0.5, 1.5, g.n)
    Rd = PR.pagerank_dense(g.n, g.row_ptr, g.col, C, W)
    R, st = CW.componentwise_solve(g.n, g.row_ptr, g.col, C, W, eps=1e-14, direct_max=16, return_stats=True)
    assert np.allclose(R, Rd, rtol=1e-11, atol=0)
    part = CW.partition_theorem(g.n, g.row_ptr, g.col)
    small = (part["comp_type"] == 1) & (part["comp_size"] <= 16)
    assert small.sum() >= 5 and np.all(st["iters"][small] == 0)
    assert np.all(st["iters"][(part["comp_type"] == 1) & ~small] > 0)


def test_direct_planted_sign_mistake_is_caught():
    """(I + cA^T) in place of (I - cA^T) must break the cycle closed form."""
    m = 4
    g = _g(m, [(i, (i + 1) % m) for i in range(m)])
    AT = PR.transition_dense(m, g.row_ptr, g.col).T
    wrong = np.linalg.solve(np.eye(m) + C * AT, np.ones(m))
    assert not np.allclose(wrong, 1.0 / (1.0 - C), rtol=1e-6)


# ------------------------------------------------- self-loops (general A)

def _loopy(n, edges):
    return csr_from_edges(n, [a for a, _ in edges], [b for _, b in edges], drop_loops=False)


def test_loops_closed_forms():
    """Def. 3.4 with a_vv > 0: a lone vertex with a loop has R = w/(1-c); a
    loop plus one edge to a sink gives R_0 = w/(1-c/2) and R_1 = w + c R_0/2;
    the same loop in the middle of a chain (a CAC) scales only its vertex."""
    g = _loopy(1, [(0, 0)])
    R = CW.componentwise_solve(1, g.row_ptr, g.col, C, np.ones(1), loops=True)
    assert np.allclose(R, 1.0 / (1.0 - C), rtol=1e-15)
    g = _loopy(2, [(0, 0), (0, 1)])
    R = CW.componentwise_solve(2, g.row_ptr, g.col, C, np.ones(2), loops=True)
    r0 = 1.0 / (1.0 - C / 2)
    assert np.allclose(R, [r0, 1.0 + C * r0 / 2], rtol=1e-15)
    g = _loopy(3, [(0, 1), (1, 1), (1, 2)])
    R = CW.componentwise_solve(3, g.row_ptr, g.col, C, np.ones(3), loops=True)
    r1 = (1.0 + C) / (1.0 - C / 2)
    assert np.allclose(R, [1.0, r1, 1.0 + C * r1 / 2], rtol=1e-15)
    # the default (loops ignored) differs: the loop is dropped from A and outdeg
    R0 = CW.componentwise_solve(3, g.row_ptr, g.col, C, np.ones(3))
    assert np.allclose(R0, [1.0, 1.0 + C, 1.0 + C * (1.0 + C)], rtol=1e-15)


loop_lists = st.integers(min_value=1, max_value=30).flatmap(
    lambda n: st.tuples(st.just(n), st.lists(
        st.tuples(st.integers(0, n - 1), st.integers(0, n - 1)), max_size=3 * n),
        st.lists(st.integers(0, n - 1), max_size=n)))


@settings(max_examples=80, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(loop_lists, st.floats(0.05, 0.99))
def test_property_loops_componentwise_equals_dense(nel, c):
    """Random graphs with self-loops: the componentwise solve (CAC sweep with
    the loop factor, SCC series with the diagonal, direct small SCCs too)
    equals the dense solve of (I - c A^T) R = W with the loops in A."""
    n, edges, loops = nel
    g = _loopy(n, edges + [(v, v) for v in loops])
    W = np.linspace(0.5, 1.5, n)
    Rd = PR.pagerank_dense(g.n, g.row_ptr, g.col, c, W, loops=True)
    Rc = CW.componentwise_solve(g.n, g.row_ptr, g.col, c, W, eps=1e-15, loops=True)
    assert np.allclose(Rc, Rd, rtol=1e-9, atol=0)
    Rx = CW.componentwise_solve(g.n, g.row_ptr, g.col, c, W, eps=1e-15, loops=True, direct_max=8)
    assert np.allclose(Rx, Rd, rtol=1e-9, atol=0)


def test_loops_planted_missing_factor_is_caught():
    """The CAC sweep run without its loop factor (a_diag omitted) on a chain
    with a looped middle vertex must miss the dense solve."""
    g = _loopy(3, [(0, 1), (1, 1), (1, 2)])
    W = np.ones(3)
    Rd = PR.pagerank_dense(3, g.row_ptr, g.col, C, W, loops=True)
    deg = PR.out_degree(3, g.row_ptr, g.col, loops=True)
    R = np.zeros(3)
    CW._cac_sweep(np.arange(3), W.copy(), np.zeros(3, dtype=np.int64), C, deg, g.row_ptr, g.col, R)
    assert not np.allclose(R, Rd, rtol=1e-6)
    R2 = np.zeros(3)
    AT = PR.transition_T_csr(3, g.row_ptr, g.col, loops=True)
    CW._cac_sweep(np.arange(3), W.copy(), np.zeros(3, dtype=np.int64), C, deg, g.row_ptr, g.col, R2, AT.diagonal())
    assert np.allclose(R2, Rd, rtol=1e-14)


# ------------------------------- geometric tail estimate of an SCC series

@pytest.mark.parametrize("m", [3, 8])
def test_tail_estimate_exact_on_a_cycle(m):
    """On a bare cycle with W = 1 every term is c^k W, so the tail estimate
    is exact: the SCC stops after two terms with R = 1/(1-c), where the plain
    rule needs about log(eps (1-c)) / log(c) terms."""
    g = _g(m, [(i, (i + 1) % m) for i in range(m)])
    R, st = CW.componentwise_solve(m, g.row_ptr, g.col, C, np.ones(m), eps=1e-10, tail=True, return_stats=True)
    assert np.allclose(R, 1.0 / (1.0 - C), rtol=1e-14, atol=0)
    assert st["iters"].max() == 2
    _, st0 = CW.componentwise_solve(m, g.row_ptr, g.col, C, np.ones(m), eps=1e-10, return_stats=True)
    assert st0["iters"].max() == math.ceil(math.log(1e-10 * (1 - C)) / math.log(C))


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("eps", [1e-4, 1e-8])
def test_tail_estimate_meets_the_bound(seed, eps):
    """Random graphs with SCCs: the relative 1-norm error against the dense
    solve stays below eps, and no SCC takes more terms than the plain rule."""
    g = random_digraph(300, 900, seed + 900)
    W = np.random.default_rng(seed).uniform(0.5, 1.5, g.n)
    Rd = PR.pagerank_dense(g.n, g.row_ptr, g.col, C, W)
    R, st = CW.componentwise_solve(g.n, g.row_ptr, g.col, C, W, eps=eps, tail=True, return_stats=True)
    _, st0 = CW.componentwise_solve(g.n, g.row_ptr, g.col, C, W, eps=eps, return_stats=True)
    assert np.abs(R - Rd).sum() / np.abs(Rd).sum() <= eps
    assert np.all(st["iters"] <= st0["iters"]) and st["iters"].sum() < st0["iters"].sum()
    # the certificate c/(1-c) sum(last) bounds the actual error
    assert np.abs(R - Rd).sum() <= C / (1 - C) * st["last"].sum() * (1 + 1e-9)


def test_tail_planted_wrong_candidate_is_caught():
    """Adding the tail on the newest term (rho/(1-rho) P_{k+1}) instead of on
    P_k breaks the residual identity: on a cycle with unequal weights the
    wrong candidate misses the dense solve by far more than eps."""
    m = 5
    g = _g(m, [(i, (i + 1) % m) for i in range(m)] + [(0, 2)])
    W = np.linspace(0.5, 1.5, m)
    Rd = PR.pagerank_dense(m, g.row_ptr, g.col, C, W)
    AT = PR.transition_T_csr(m, g.row_ptr, g.col)
    p0 = W.copy()
    p1 = C * (AT @ p0)
    p2 = C * (AT @ p1)
    rho = np.abs(p1).sum() / np.abs(p0).sum()
    right = p0 + p1 + rho / (1 - rho) * p1
    wrong = p0 + p1 + p2 + rho / (1 - rho) * p2
    r_right = W - right + C * (AT @ right)
    assert np.allclose(r_right, (p2 - rho * p1) / (1 - rho), atol=1e-12)  # the identity the rule uses
    r_wrong = W - wrong + C * (AT @ wrong)
    assert not np.allclose(r_wrong, (p2 - rho * p1) / (1 - rho), atol=1e-6)


# ------------------------------------------- weighted graphs (Markov chains)

def test_weighted_closed_form():
    """0 -> 1 (weight 3), 0 -> 2 (weight 1), 1 -> 0, 2 a sink; W = 1:
    R_0 = 1 + c R_1, R_1 = 1 + (3/4) c R_0, R_2 = 1 + (1/4) c R_0, so
    R_0 = (1 + c) / (1 - 3c^2/4)."""
    rp = np.array([0, 2, 3, 3])
    col = np.array([1, 2, 0])
    w = np.array([3.0, 1.0, 1.0])
    R = PR.pagerank_dense_weighted(3, rp, col, w, C, np.ones(3))
    r0 = (1 + C) / (1 - 0.75 * C * C)
    np.testing.assert_allclose(R, [r0, 1 + 0.75 * C * r0, 1 + 0.25 * C * r0], rtol=1e-14)


@pytest.mark.parametrize("seed", range(3))
def test_unit_weights_are_the_unweighted_definition(seed):
    g = random_digraph(60, 240, seed + 70, loops=True, duplicates=True)
    W = np.random.default_rng(seed).uniform(0.5, 1.5, g.n)
    for loops in (False, True):
        np.testing.assert_allclose(PR.pagerank_dense_weighted(g.n, g.row_ptr, g.col, np.ones(g.m), C, W, loops),
                                   PR.pagerank_dense(g.n, g.row_ptr, g.col, C, W, loops), rtol=1e-13)


@pytest.mark.parametrize("seed", range(3))
def test_integer_weights_as_parallel_edges(seed):
    """An edge of integer weight k passed as k parallel edges (the library's
    input form for weighted graphs) gives the weighted definition, through
    the componentwise oracle and the plain series alike."""
    from paper_1609_09068_amd.weights import expand_integer_weights

    g = random_digraph(300, 1000, seed + 80)
    w = np.random.default_rng(seed).integers(1, 6, g.m)
    W = np.random.default_rng(seed + 1).uniform(0.5, 1.5, g.n)
    Rw = PR.pagerank_dense_weighted(g.n, g.row_ptr, g.col, w, C, W)
    rp2, col2 = expand_integer_weights(g.row_ptr, g.col, w)
    assert rp2[-1] == w.sum()
    R = CW.componentwise_solve(g.n, rp2, col2, C, W, eps=1e-13)
    np.testing.assert_allclose(R, Rw, rtol=1e-11)
    Rp, _, _ = PR.pagerank_power_series(g.n, rp2, col2, C, W, eps=1e-13)
    np.testing.assert_allclose(Rp, Rw, rtol=1e-11)
    # a planted mistake: ignoring the weights is far off
    assert not np.allclose(CW.componentwise_solve(g.n, g.row_ptr, g.col, C, W, eps=1e-13), Rw, rtol=1e-3)


def test_weighted_sparse_transition_closed_form():
    """The sparse weighted A^T (used for the series and the residual of
    weighted graphs) on the closed-form chain above: the series with it gives
    R_0 = (1 + c) / (1 - 3c^2/4); the weights are not normalised by edge
    count (a planted mistake, 1/outdeg, gives R_1 = 1 + c R_0 / 2)."""
    rp = np.array([0, 2, 3, 3])
    col = np.array([1, 2, 0])
    w = np.array([3.0, 1.0, 1.0])
    AT = PR.transition_T_csr(3, rp, col, weight=w)
    R, _, _ = PR.pagerank_power_series(3, rp, col, C, np.ones(3), eps=1e-15, AT=AT)
    r0 = (1 + C) / (1 - 0.75 * C * C)
    np.testing.assert_allclose(R, [r0, 1 + 0.75 * C * r0, 1 + 0.25 * C * r0], rtol=1e-13)
    Ru, _, _ = PR.pagerank_power_series(3, rp, col, C, np.ones(3), eps=1e-15)
    assert abs(Ru[1] - (1 + 0.75 * C * r0)) > 0.1


@pytest.mark.parametrize("seed", range(3))
@pytest.mark.parametrize("loops", [False, True])
def test_weighted_sparse_series_matches_dense(seed, loops):
    """Real weights (some zero, so a vertex can lose every out-weight), with
    repeated edges and loops: the series with the sparse weighted A^T and its
    residual bound agree with the dense weighted solve."""
    g = random_digraph(200, 900, seed + 120, loops=True, duplicates=True)
    rng = np.random.default_rng(seed)
    w = rng.uniform(0.0, 2.0, g.m) * (rng.random(g.m) > 0.1)
    W = rng.uniform(0.5, 1.5, g.n)
    ref = PR.pagerank_dense_weighted(g.n, g.row_ptr, g.col, w, C, W, loops=loops)
    AT = PR.transition_T_csr(g.n, g.row_ptr, g.col, loops=loops, weight=w)
    R, _, _ = PR.pagerank_power_series(g.n, g.row_ptr, g.col, C, W, eps=1e-14, AT=AT)
    np.testing.assert_allclose(R, ref, rtol=1e-11)
    bound, _ = PR.residual_bound(g.n, g.row_ptr, g.col, C, W, ref, AT=AT)
    assert bound < 1e-13
    # the unweighted residual of the weighted answer is not small
    assert PR.residual_bound(g.n, g.row_ptr, g.col, C, W, ref, loops=loops)[0] > 1e-4


def test_weight_expansion_validates_and_drops_zero_weights():
    from paper_1609_09068_amd.weights import expand_integer_weights

    rp = np.array([0, 2, 3, 3])
    col = np.array([1, 2, 0])
    rp2, col2 = expand_integer_weights(rp, col, [2, 0, 3])
    assert rp2.tolist() == [0, 2, 5, 5] and col2.tolist() == [1, 1, 0, 0, 0]
    for bad in ([1.5, 1, 1], [1, -1, 1], [1, 1]):
        with pytest.raises(ValueError):
            expand_integer_weights(rp, col, bad)


@pytest.mark.parametrize("seed", range(2))
def test_tail_estimate_inert_under_the_papers_rule(seed):
    """The estimate certifies against the 1-norm rule only: under the
    paper's max-norm rule the result and the term counts are unchanged."""
    g = random_digraph(300, 900, seed + 910)
    W = np.random.default_rng(seed).uniform(0.5, 1.5, g.n)
    R0, st0 = CW.componentwise_solve(g.n, g.row_ptr, g.col, C, W, stop="paper", tol=1e-9, return_stats=True)
    R1, st1 = CW.componentwise_solve(g.n, g.row_ptr, g.col, C, W, stop="paper", tol=1e-9, tail=True,
                                     return_stats=True)
    np.testing.assert_array_equal(R1, R0)
    np.testing.assert_array_equal(st1["iters"], st0["iters"])


def test_residual_rows_of_exact_and_planted_errors():
    """Pins residual_rows: the dense solution leaves a residual at rounding
    level, and a planted error e at one vertex v (out-degree d) leaves
    r_v = -e and r_u = c e / d at each successor u, nothing elsewhere."""
    g = random_digraph(80, 320, 11)
    W = np.random.default_rng(3).random(g.n) + 0.5
    R = PR.pagerank_dense(g.n, g.row_ptr, g.col, C, W)
    r, scale, _ = PR.residual_rows(g.n, g.row_ptr, g.col, C, W, R)
    assert np.all(np.abs(r) <= 1e-13 * scale)
    outdeg = np.diff(g.row_ptr) - np.array([np.sum(g.col[g.row_ptr[u]:g.row_ptr[u + 1]] == u) for u in range(g.n)])
    v = int(np.argmax(outdeg))
    succ = [int(u) for u in g.col[g.row_ptr[v]:g.row_ptr[v + 1]] if u != v]
    e = 0.125
    R2 = R.copy()
    R2[v] += e
    r2, _, _ = PR.residual_rows(g.n, g.row_ptr, g.col, C, W, R2)
    want = np.zeros(g.n)
    want[v] -= e
    for u in succ:
        want[u] += C * e / outdeg[v]
    assert np.allclose(r2 - r, want, rtol=0, atol=1e-12)


def test_whole_graph_tail_estimate_pins():
    """The whole-graph series with the tail estimate: on a directed cycle
    (P_k = c^k W, rho = c exactly) it stops after two terms with the exact
    R = W/(1-c); on a strongly connected graph it is the componentwise rule on
    its single SCC (same term count, same R up to rounding); on random graphs
    it is within eps of the dense solve and its residual norm is c times the
    returned last norm (the residual identity of the estimate)."""
    n = 12
    g = csr_from_edges(n, list(range(n)), [(i + 1) % n for i in range(n)])
    R, k, _ = PR.pagerank_power_series(n, g.row_ptr, g.col, C, np.ones(n), eps=1e-10, tail=True)
    assert k == 2 and np.allclose(R, 1.0 / (1.0 - C), rtol=1e-14)
    # one SCC: a cycle through every vertex plus random chords
    rng = np.random.default_rng(9)
    n = 300
    order = rng.permutation(n)
    src = list(order) + list(rng.integers(0, n, 900))
    dst = list(np.roll(order, -1)) + list(rng.integers(0, n, 900))
    g = csr_from_edges(n, src, dst)
    W = rng.uniform(0.5, 1.5, n)
    Rp, kp, lp = PR.pagerank_power_series(n, g.row_ptr, g.col, C, W, eps=1e-9, tail=True)
    Rc, st = CW.componentwise_solve(n, g.row_ptr, g.col, C, W, eps=1e-9, tail=True, return_stats=True)
    assert int(st["iters"].max()) == kp and np.allclose(Rp, Rc, rtol=1e-12)
    for seed in range(4):
        g = random_digraph(200, 900, 40 + seed)
        W = np.random.default_rng(seed).uniform(0.5, 1.5, g.n)
        Rt, kt, lt = PR.pagerank_power_series(g.n, g.row_ptr, g.col, C, W, eps=1e-8, tail=True)
        Rn, kn, _ = PR.pagerank_power_series(g.n, g.row_ptr, g.col, C, W, eps=1e-8)
        ref = PR.pagerank_dense(g.n, g.row_ptr, g.col, C, W)
        assert kt <= kn
        assert np.abs(Rt - ref).sum() / ref.sum() <= 1e-8
        r, _, _ = PR.residual_rows(g.n, g.row_ptr, g.col, C, W, Rt)
        assert np.abs(r).sum() == pytest.approx(C * lt, rel=1e-9)
