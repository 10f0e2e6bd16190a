"""Pins for the oracle's SCC/CAC partition (Sec. 4.1, Theorem 3.1)."""
import json
import os

import networkx as nx
import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

from graphgen import config_graph, csr_from_edges, random_digraph
from oracle import partition as P

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _graph(n, edges, dedupe=True, drop_loops=True):
    src = [a for a, _ in edges]
    dst = [b for _, b in edges]
    return csr_from_edges(n, src, dst, dedupe=dedupe, drop_loops=drop_loops)


def _raw_graph(n, edges):
    """CSR that keeps loops and duplicates exactly as given."""
    edges = sorted(edges)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    for a, _ in edges:
        row_ptr[a + 1] += 1
    row_ptr = np.cumsum(row_ptr)
    col = np.array([b for _, b in edges], dtype=np.int32)
    return row_ptr, col


def test_fig1_worked_example():
    fx = json.load(open(os.path.join(GOLDEN, "fig1_partition.json")))
    g = _graph(8, fx["edges"])
    for fn in (P.partition_theorem, P.partition_dfs):
        p = fn(g.n, g.row_ptr, g.col)
        assert p["comp"].tolist() == fx["comp"]
        assert p["comp_level"].tolist() == fx["comp_level"]
        assert p["comp_type"].tolist() == fx["comp_type"]
        assert p["comp_size"].tolist() == fx["comp_size"]
        assert p["n_levels"] == fx["n_levels"]
    lv = P.scc_only_levels(g.n, g.row_ptr, g.col)
    assert lv.tolist() == fx["scc_only_levels"]
    assert int(lv.max()) + 1 == fx["n_levels_scc_only"]


def test_two_vertex_edge_and_single_vertex():
    # Corollary 3.1 proof: one edge between two vertices gives one CAC on one
    # level, while the SCC partition needs two levels; one vertex: equality
    g = _graph(2, [(0, 1)])
    for fn in (P.partition_theorem, P.partition_dfs):
        p = fn(g.n, g.row_ptr, g.col)
        assert p["comp"].tolist() == [0, 0]
        assert p["comp_type"].tolist() == [0]
        assert p["n_levels"] == 1
    assert int(P.scc_only_levels(g.n, g.row_ptr, g.col).max()) + 1 == 2
    g1 = _graph(1, [])
    for fn in (P.partition_theorem, P.partition_dfs):
        p = fn(g1.n, g1.row_ptr, g1.col)
        assert p["comp"].tolist() == [0] and p["n_levels"] == 1
    assert P.scc_only_levels(g1.n, g1.row_ptr, g1.col).tolist() == [0]


def test_empty_graph():
    p = P.partition_theorem(0, np.zeros(1, np.int64), np.zeros(0, np.int32))
    assert p["n_comp"] == 0 and p["n_levels"] == 0


def test_long_chain_is_one_cac():
    n = 3000
    g = _graph(n, [(i, i + 1) for i in range(n - 1)])
    for fn in (P.partition_theorem, P.partition_dfs):
        p = fn(g.n, g.row_ptr, g.col)
        assert p["n_comp"] == 1 and p["n_levels"] == 1 and p["comp_type"].tolist() == [0]


def test_head_blocked_by_scc_below():
    # v -> SCC{1,2} (level 0) and v -> 3 (sink, level 0): no merge, v on level 1
    g = _graph(4, [(0, 1), (1, 2), (2, 1), (0, 3)])
    for fn in (P.partition_theorem, P.partition_dfs):
        p = fn(g.n, g.row_ptr, g.col)
        assert p["comp"].tolist() == [0, 1, 1, 2]
        assert p["comp_level"].tolist() == [1, 0, 0]
        assert p["comp_type"].tolist() == [0, 1, 0]


def test_head_merges_with_all_cacs_one_level_down():
    # 0 -> 1, 0 -> 2 (two sinks): all three form one CAC on level 0;
    # 3 -> 0 then merges too; 4 -> {3, SCC{5,6}} with the SCC on level 0 only
    g = _graph(7, [(0, 1), (0, 2), (3, 0), (4, 3), (4, 5), (5, 6), (6, 5)])
    for fn in (P.partition_theorem, P.partition_dfs):
        p = fn(g.n, g.row_ptr, g.col)
        comp = p["comp"].tolist()
        assert comp[0] == comp[1] == comp[2] == comp[3]
        # 4 sees the CAC on level 0 and the SCC on level 0: blocked, level 1
        assert comp[4] != comp[3]
        assert p["comp_level"][comp[4]] == 1


def test_self_loops_and_duplicates_ignored():
    rp, col = _raw_graph(4, [(0, 0), (0, 1), (0, 1), (1, 2), (2, 2), (2, 1), (3, 3)])
    gref = _graph(4, [(0, 1), (1, 2), (2, 1)])
    for fn in (P.partition_theorem, P.partition_dfs):
        a = fn(4, rp, col)
        b = fn(gref.n, gref.row_ptr, gref.col)
        assert P.partition_arrays_equal(a, b)


def check_invariants(n, row_ptr, col, p):
    comp = p["comp"].astype(np.int64)
    lvl = p["comp_level"].astype(np.int64)
    typ = p["comp_type"]
    size = p["comp_size"]
    k = p["n_comp"]
    # canonical numbering: first appearances are 0, 1, 2, ...
    _, first = np.unique(comp, return_index=True)
    assert np.all(np.diff(first) > 0)
    src = np.repeat(np.arange(n), np.diff(row_ptr))
    dst = np.asarray(col, dtype=np.int64)
    keep = src != dst
    src, dst = src[keep], dst[keep]
    cs, cd = comp[src], comp[dst]
    inter = cs != cd
    # edges between components go strictly down in level (Theorem 3.1, 2)
    assert np.all(lvl[cs[inter]] > lvl[cd[inter]])
    # a component's level is 0 or one more than its highest successor (Def 3.3)
    succmax = np.full(k, -1)
    np.maximum.at(succmax, cs[inter], lvl[cd[inter]])
    assert np.array_equal(lvl, succmax + 1)
    # SCCs are exactly the strongly connected components with >= 2 vertices
    G = nx.DiGraph()
    G.add_nodes_from(range(n))
    G.add_edges_from(zip(src.tolist(), dst.tolist()))
    for s in nx.strongly_connected_components(G):
        s = sorted(s)
        if len(s) >= 2:
            c0 = comp[s[0]]
            assert typ[c0] == 1 and size[c0] == len(s)
            assert np.all(comp[s] == c0)
        else:
            assert typ[comp[s[0]]] == 0
    # CACs: weakly connected, acyclic, induced (Def 2.2)
    for c in np.nonzero(typ == 0)[0]:
        mem = np.nonzero(comp == c)[0]
        H = G.subgraph(mem.tolist())
        assert nx.is_weakly_connected(H)
        assert nx.is_directed_acyclic_graph(H)
    # fixed point of the merge rule: a one-vertex CAC on level L >= 1 must
    # point to an SCC (>= 2 vertices) on level L-1, otherwise it would merge
    for c in np.nonzero((typ == 0) & (size == 1))[0]:
        v = int(np.nonzero(comp == c)[0][0])
        if lvl[c] == 0:
            continue
        succ = dst[src == v]
        below = [d for d in succ if lvl[comp[d]] == lvl[c] - 1]
        assert any(typ[comp[d]] == 1 for d in below)
    # Corollary 3.1: never more levels than the plain SCC partition
    if n:
        assert p["n_levels"] <= int(P.scc_only_levels(n, row_ptr, col).max()) + 1


edge_lists = st.integers(min_value=1, max_value=45).flatmap(
    lambda n: st.tuples(st.just(n), st.lists(
        st.tuples(st.integers(0, n - 1), st.integers(0, n - 1)), max_size=3 * n)))


@settings(max_examples=150, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(edge_lists, st.randoms(use_true_random=False))
def test_property_dfs_equals_theorem_and_invariants(ne, rnd):
    n, edges = ne
    rp, col = _raw_graph(n, edges)  # loops and duplicates kept
    a = P.partition_theorem(n, rp, col)
    b = P.partition_dfs(n, rp, col)
    assert P.partition_arrays_equal(a, b)
    check_invariants(n, rp, col, a)
    # relabelling invariance (Theorem 3.1, 1): the partition is unique, so
    # relabelled vertices land in the relabelled components
    perm = list(range(n))
    rnd.shuffle(perm)
    e2 = [(perm[x], perm[y]) for x, y in edges]
    rnd.shuffle(e2)
    rp2, col2 = _raw_graph(n, e2)
    c = P.partition_theorem(n, rp2, col2)
    d = P.partition_dfs(n, rp2, col2)
    assert P.partition_arrays_equal(c, d)
    inv = np.argsort(perm)
    # same sets: map back and compare as set partitions with equal levels
    comp_back = c["comp"][np.array(perm)] if n else c["comp"]
    lv_back = c["comp_level"][comp_back]
    assert np.array_equal(lv_back, a["comp_level"][a["comp"]])
    pairs = set(zip(a["comp"].tolist(), comp_back.tolist()))
    assert len(pairs) == a["n_comp"] == c["n_comp"]
    del inv


def test_adjacency_order_does_not_matter():
    g = random_digraph(300, 700, 7)
    a = P.partition_dfs(g.n, g.row_ptr, g.col)
    rng = np.random.default_rng(3)
    col2 = g.col.copy()
    for u in range(g.n):
        s, e = g.row_ptr[u], g.row_ptr[u + 1]
        col2[s:e] = rng.permutation(col2[s:e])
    b = P.partition_dfs(g.n, g.row_ptr, col2)
    assert P.partition_arrays_equal(a, b)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_config1_routes_agree(seed):
    g = config_graph("c1_small", seed=seed)
    a = P.partition_theorem(g.n, g.row_ptr, g.col)
    b = P.partition_dfs(g.n, g.row_ptr, g.col)
    assert P.partition_arrays_equal(a, b)
    check_invariants(g.n, g.row_ptr, g.col, a)
    assert int(np.sum(a["comp_type"] == 1)) == 200  # the planted SCC blocks


def test_planted_mistake_is_caught(monkeypatch):
    """A plausible slip in the merge rule (ignoring the SCC block on level
    L-1) must break the Fig. 1 pin."""
    fx = json.load(open(os.path.join(GOLDEN, "fig1_partition.json")))
    g = _graph(8, fx["edges"])
    orig = P.partition_dfs

    def settle_wrong(v, w, typ, level, low):
        if typ[w] is not None:
            level[v] = max(level[v], level[w])  # dropped "+1"
        else:
            level[v] = max(level[v], level[w])
            low[v] = min(low[v], low[w])

    monkeypatch.setattr(P, "_settle_edge", settle_wrong)
    bad = orig(g.n, g.row_ptr, g.col)
    assert bad["comp"].tolist() != fx["comp"] or bad["comp_level"].tolist() != fx["comp_level"]
