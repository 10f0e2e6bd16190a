"""Host-side checks of the C ABI: the library loads, exports every declared
symbol, and its host partition is bit-exact with the oracle (no GPU)."""
import ctypes as C
import os
import re

import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

from graphgen import config_graph, csr_from_edges, random_digraph
from oracle.partition import partition_arrays_equal, partition_theorem

pr = pytest.importorskip("paper_1609_09068_amd")
from paper_1609_09068_amd import _lib  # noqa: E402

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "pr.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(pr_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    names = _declared()
    assert "pr_partition" in names and "pr_solve" in names and "pr_free" in names
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(_lib.EXPORTS)


def test_partition_fig1_and_errors():
    edges = [(0, 1), (0, 2), (1, 3), (2, 4), (2, 5), (1, 5), (4, 5), (6, 7), (3, 1), (7, 6), (1, 6)]
    g = csr_from_edges(8, [a for a, _ in edges], [b for _, b in edges])
    p = pr.pr_partition(g.row_ptr, g.col)
    assert p.comp.tolist() == [0, 1, 2, 1, 2, 2, 3, 3]
    assert p.comp_level.tolist() == [2, 1, 0, 0]
    assert p.comp_type.tolist() == [0, 1, 0, 1]
    assert p.n_levels == 3
    bad = g.col.copy()
    bad[0] = 99
    with pytest.raises(pr.PRError) as ei:
        pr.pr_partition(g.row_ptr, bad)
    assert ei.value.code == _lib.PR_EINVAL
    rp = g.row_ptr.copy()
    rp[3] = rp[2] - 1
    with pytest.raises(pr.PRError):
        pr.pr_partition(rp, g.col)


def test_free_is_idempotent_and_handles_are_checked():
    lib = _lib.load()
    g = random_digraph(10, 20, 0)
    p = pr.pr_partition(g.row_ptr, g.col)
    h = p.handle
    lib.pr_free(h)
    lib.pr_free(h)  # ignored
    lib.pr_free(None)
    lib.pr_free(C.c_void_p(12345))  # unknown: ignored
    k = C.c_int64()
    rc = lib.pr_partition_get(h, None, None, None, None, C.byref(k), None)
    assert rc == _lib.PR_EHANDLE
    p.handle = None


def test_empty_and_single_vertex():
    p = pr.pr_partition(np.zeros(1, np.int64), np.zeros(0, np.int32))
    assert p.n_comp == 0 and p.n_levels == 0
    p = pr.pr_partition(np.zeros(2, np.int64), np.zeros(0, np.int32))
    assert p.comp.tolist() == [0] and p.n_levels == 1


def test_long_chain_no_stack_overflow():
    n = 2_000_000
    src = np.arange(n - 1)
    g = csr_from_edges(n, src, src + 1)
    p = pr.pr_partition(g.row_ptr, g.col)
    assert p.n_comp == 1 and p.n_levels == 1


def test_long_cycle_chain_alternating():
    # SCC pairs linked in a chain: deep DAG of SCCs
    k = 20000
    src, dst = [], []
    for i in range(k):
        a, b = 2 * i, 2 * i + 1
        src += [a, b]
        dst += [b, a]
        if i + 1 < k:
            src.append(b)
            dst.append(2 * (i + 1))
    g = csr_from_edges(2 * k, src, dst)
    a = pr.pr_partition(g.row_ptr, g.col).as_dict()
    b = partition_theorem(g.n, g.row_ptr, g.col)
    assert partition_arrays_equal(a, b)
    assert a["n_levels"] == k


edge_lists = st.integers(min_value=1, max_value=60).flatmap(
    lambda n: st.tuples(st.just(n), st.lists(
        st.tuples(st.integers(0, n - 1), st.integers(0, n - 1)), max_size=3 * n)))


@settings(max_examples=200, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(edge_lists)
def test_property_host_partition_bit_exact(ne):
    n, edges = ne
    edges = sorted(edges)  # loops and duplicates kept
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    for a, _ in edges:
        row_ptr[a + 1] += 1
    row_ptr = np.cumsum(row_ptr)
    col = np.array([b for _, b in edges], dtype=np.int32)
    a = pr.pr_partition(row_ptr, col).as_dict()
    b = partition_theorem(n, row_ptr, col)
    assert partition_arrays_equal(a, b)


@pytest.mark.parametrize("name", ["c1_small", "c4_train_100k"])
def test_config_partitions_bit_exact(name):
    g = config_graph(name)
    a = pr.pr_partition(g.row_ptr, g.col).as_dict()
    b = partition_theorem(g.n, g.row_ptr, g.col)
    assert partition_arrays_equal(a, b)


def _i64(a):
    return np.ascontiguousarray(a, np.int64).ctypes.data_as(C.POINTER(C.c_int64))


def _i32(a):
    return np.ascontiguousarray(a, np.int32).ctypes.data_as(C.POINTER(C.c_int32))


def test_build_rejects_partition_of_another_graph_differing_in_one_edge():
    """The plan build checks that the partition belongs to the graph from a
    fingerprint of every row pointer and column index: a graph with the same
    n and m that differs in one edge, far from any strided sample point, is
    refused before any device work (PR_EINVAL)."""
    lib = _lib.load()
    g = random_digraph(20_000, 200_000, 7)
    p = pr.pr_partition(g.row_ptr, g.col)
    for e in (1, g.m // 4097 + 3, g.m - 2):
        col = g.col.copy()
        col[e] = (col[e] + 1) % g.n
        out = C.c_void_p()
        rc = lib.pr_build_levels(p.handle, g.n, _i64(g.row_ptr), _i32(col), None, None, C.byref(out))
        assert rc == _lib.PR_EINVAL, (e, rc)
        assert b"different graph" in lib.pr_last_error()
    # moving an edge to the next row keeps m but changes two row pointers
    rp = g.row_ptr.copy()
    v = int(np.argmax(np.diff(rp) > 1))
    rp[v + 1] -= 1
    out = C.c_void_p()
    rc = lib.pr_build_levels(p.handle, g.n, _i64(rp), _i32(g.col), None, None, C.byref(out))
    assert rc == _lib.PR_EINVAL and b"different graph" in lib.pr_last_error()


def test_weighted_build_rejects_bad_weights_before_device_work():
    """pr_build_levels_weighted refuses a NULL weight array and a negative,
    NaN or infinite weight with PR_EINVAL (naming the first bad edge) before
    any device work; the Python binding checks the weight array's length."""
    lib = _lib.load()
    g = random_digraph(500, 2000, 11)
    p = pr.pr_partition(g.row_ptr, g.col)
    out = C.c_void_p()
    rc = lib.pr_build_levels_weighted(p.handle, g.n, _i64(g.row_ptr), _i32(g.col), None, None, None, C.byref(out))
    assert rc == _lib.PR_EINVAL and b"weight is NULL" in lib.pr_last_error()
    for bad in (-1.0, float("nan"), float("inf")):
        w = np.ones(g.m)
        w[g.m // 2] = bad
        rc = lib.pr_build_levels_weighted(p.handle, g.n, _i64(g.row_ptr), _i32(g.col),
                                          w.ctypes.data_as(C.POINTER(C.c_double)), None, None, C.byref(out))
        assert rc == _lib.PR_EINVAL, bad
        assert f"weight[{g.m // 2}]".encode() in lib.pr_last_error()
    with pytest.raises(ValueError):
        pr.pr_build_levels(p, g.row_ptr, g.col, weight=np.ones(g.m - 1))


def test_build_rejects_bad_seg_waves_before_device_work():
    lib = _lib.load()
    g = random_digraph(300, 1200, 13)
    p = pr.pr_partition(g.row_ptr, g.col)
    for bad in (1, 4, -2):
        o = pr.build_opts(seg_waves=bad)
        out = C.c_void_p()
        rc = lib.pr_build_levels(p.handle, g.n, _i64(g.row_ptr), _i32(g.col), C.byref(o), None, C.byref(out))
        assert rc == _lib.PR_EINVAL and b"seg_waves" in lib.pr_last_error()
