"""The Barabasi-Albert workload generator (B-A generation subsection of
Sec. 5.1): shape checks only.  The paper's text leaves the edge-orientation
rule open, so parity of the generator itself is unpinned; these tests check
the rule as read (each vertex keeps ceil(log2 E_i) out-edges) and the
qualitative shape the experiments rely on."""
import numpy as np

from graphgen import barabasi_albert
from oracle.partition import partition_theorem


def test_out_degree_rule_and_heavy_in_degree():
    g = barabasi_albert(20_000, 2, seed=11)
    outdeg = np.diff(g.row_ptr)
    # grown vertices created two edges: ceil(log2 2) = 1 kept each (fewer only
    # where a kept edge duplicates one kept from the other end, which the CSR
    # removes; never more)
    assert outdeg[20:].max() <= 1 and outdeg[20:].mean() > 0.99
    indeg = np.bincount(g.col, minlength=g.n)
    assert indeg.max() > 50 * max(indeg.mean(), 1e-9)  # preferential attachment: hubs


def test_five_edges_variant():
    g = barabasi_albert(5_000, 24, seed=12)
    outdeg = np.diff(g.row_ptr)
    assert np.all(outdeg[20:] == 5)  # ceil(log2 24) = 5


def test_seeded_and_cac_dominated():
    a = barabasi_albert(5_000, 2, seed=13)
    b = barabasi_albert(5_000, 2, seed=13)
    assert np.array_equal(a.row_ptr, b.row_ptr) and np.array_equal(a.col, b.col)
    p = partition_theorem(a.n, a.row_ptr, a.col)
    cac_vertices = p["comp_size"][p["comp_type"] == 0].sum()
    assert cac_vertices > 0.6 * a.n  # CAC-dominated, as in the paper's B-A graph
    assert p["comp_size"][p["comp_type"] == 1].max() <= 10  # SCCs stay tiny (mostly 2-cycles)
