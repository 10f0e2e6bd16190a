"""The claim order of the segment kernels' work items, read back from the
plan's own tables and checked on the host.  Workgroups claim items in list
order and a claimed item waits for the values of its sources, so the order
must put every item after the items that hold its sources (eq. PR:levels
pulls from higher levels; inside a CAC, Sec. 4.3.1 sweeps in topological
order); the levels of Theorem 3.1 are claimed from the highest down, and
inside a level, where no edge joins two components, the vertex items come
before the SCC items."""
import sys

import numpy as np
import pytest

from graphgen import config_graph, scc_blocks

pytestmark = pytest.mark.gpu

ITEM_VERTS, ITEM_SMALL, ITEM_MEDIUM = 0, 1, 2


def _say(*a):
    print("[gpu-case]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def pr():
    import torch

    import paper_1609_09068_amd as pr

    assert torch.cuda.is_available()
    return pr


def _check(pr, g, **build):
    part = pr.pr_partition(g.row_ptr, g.col)
    lv = pr.pr_build_levels(part, g.row_ptr, g.col, **build)
    items = lv.debug("items")
    perm = lv.debug("perm")
    rv = lv.debug("rank_vbeg")
    rcomp = lv.debug("rank_comp")
    n = g.n
    pos_of = np.empty(n, np.int64)
    pos_of[perm] = np.arange(n)
    rank_of_pos = np.searchsorted(rv, np.arange(n), side="right") - 1
    level_of_pos = part.comp_level[rcomp[rank_of_pos]]
    item_of = np.full(n, -1, np.int64)
    first = np.empty(len(items), np.int64)
    for q, (k, a, b, _) in enumerate(items):
        lo, hi = (a, b) if k == ITEM_VERTS else ((rv[a], rv[b]) if k == ITEM_SMALL else (rv[a], rv[a + 1]))
        assert lo < hi and np.all(item_of[lo:hi] == -1), "items overlap"
        item_of[lo:hi] = q
        first[q] = lo
        # one level per item
        assert np.all(level_of_pos[lo:hi] == level_of_pos[lo])
    lev = level_of_pos[first]
    # levels from the highest down
    assert np.all(np.diff(lev) <= 0)
    # inside a level: every vertex item before every SCC item
    for L in np.unique(lev):
        kinds = items[lev == L, 0]
        nv = int((kinds == ITEM_VERTS).sum())
        assert np.all(kinds[:nv] == ITEM_VERTS) and np.all(kinds[nv:] != ITEM_VERTS), L
    # every source in an earlier item or the same one (gang rows hold no item)
    src = np.repeat(np.arange(n), np.diff(g.row_ptr))
    iu, iv = item_of[pos_of[src]], item_of[pos_of[np.asarray(g.col)]]
    m = (iu >= 0) & (iv >= 0)
    assert np.all(iu[m] <= iv[m])
    # rows outside every item are exactly the gang SCCs' rows
    gang = item_of < 0
    assert np.all(part.comp_type[rcomp[rank_of_pos[gang]]] == 1)
    info = lv.info()
    assert int(gang.sum()) == info["v_gang"]
    out = dict(items=len(items), verts=int((items[:, 0] == ITEM_VERTS).sum()), gang_rows=int(gang.sum()))
    lv.free()
    part.free()
    return out


@pytest.mark.parametrize("small,team", [(64, 16384), (16, 16384), (1, 200)])
def test_claim_order_c1(pr, small, team):
    g = config_graph("c1_small")
    _say("schedule c1", small, team)
    out = _check(pr, g, small_cutoff=small, team_edges=team)
    assert out["verts"] > 0


def test_claim_order_blocks_with_gangs(pr):
    """SCC blocks on several levels with a gang threshold low enough that
    the larger blocks become gang phases between segments."""
    g = scc_blocks(5, nblocks=60, max_size=60)
    _say("schedule blocks")
    out = _check(pr, g, small_cutoff=8, team_edges=64)
    assert out["gang_rows"] > 0


def test_claim_order_c2(pr):
    """The 1M-vertex web-like graph at the launch shape the autotuner picks
    for it."""
    g = config_graph("c2_web_1m")
    _say("schedule c2")
    out = _check(pr, g, rows_per_wave=64, small_cutoff=64, team_edges=16384)
    assert out["gang_rows"] >= 400000
