"""The SCC/CAC partition of Sec. 4.1.

Test infrastructure only (see the package docstring).

Two independent routes compute the same partition:

* ``partition_theorem`` (primary, scales to tens of millions of vertices):
  strongly connected components from scipy, then the merge process of
  Theorem 3.1 applied bottom-up over the DAG of SCCs.
* ``partition_dfs`` (small graphs): the modified Tarjan depth-first search of
  Sec. 4.1 (Discover / Explore / Finish with a merge-find forest), written
  from the description of those three steps.

Both return the canonical form used everywhere in this project:

  comp[v]        component id; ids are given in order of first appearance
                 while scanning v = 0, 1, ..., n-1 (the numbering pass at the
                 end of Sec. 4.1, with its counter initialised once)
  comp_level[k]  0-based level: components with no edge to another component
                 have level 0 (Def. 3.3 and Fig. 1)
  comp_type[k]   1 for an SCC of two or more vertices, 0 for a CAC (a
                 one-vertex component counts as a CAC, Sec. 3 after Def. 3.3)
  comp_size[k]   number of vertices
  n_levels       1 + the largest level (0 for the empty graph)

Self-loops are ignored in the component finding (Sec. 4.1).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components


def _edges_no_loops(n, row_ptr, col):
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    col = np.asarray(col, dtype=np.int64)
    src = np.repeat(np.arange(n, dtype=np.int64), np.diff(row_ptr))
    keep = src != col
    return src[keep], col[keep]


def canonical_ids(label):
    """Relabel so ids appear in order of first occurrence over v = 0..n-1."""
    label = np.asarray(label)
    if label.size == 0:
        return label.astype(np.int32), 0
    uniq, first = np.unique(label, return_index=True)
    order = np.argsort(first, kind="stable")
    rank = np.empty(len(uniq), dtype=np.int64)
    rank[order] = np.arange(len(uniq))
    pos = np.searchsorted(uniq, label)
    return rank[pos].astype(np.int32), len(uniq)


def _finalise(label, vlevel, vtype):
    comp, k = canonical_ids(label)
    comp_level = np.zeros(k, dtype=np.int32)
    comp_type = np.zeros(k, dtype=np.uint8)
    comp_level[comp] = vlevel
    comp_type[comp] = vtype
    comp_size = np.bincount(comp, minlength=k).astype(np.int32)
    # every member of a component must carry the same level and type
    assert np.all(comp_level[comp] == vlevel)
    assert np.all(comp_type[comp] == vtype)
    n_levels = int(comp_level.max()) + 1 if k else 0
    return dict(comp=comp, comp_level=comp_level, comp_type=comp_type,
                comp_size=comp_size, n_comp=k, n_levels=n_levels)


def scc_labels(n, row_ptr, col):
    src, dst = _edges_no_loops(n, row_ptr, col)
    if n == 0:
        return np.zeros(0, dtype=np.int64), 0
    G = sp.csr_matrix((np.ones(len(src), dtype=np.int8), (src, dst)), shape=(n, n))
    k, lab = connected_components(G, directed=True, connection="strong")
    return lab.astype(np.int64), int(k)


def _heights(k, csrc, cdst):
    """Longest path to a sink in the DAG of SCCs (sinks 0), by peeling sinks."""
    outcnt = np.bincount(csrc, minlength=k)
    order = np.argsort(cdst, kind="stable")
    pred_ptr = np.zeros(k + 1, dtype=np.int64)
    np.cumsum(np.bincount(cdst, minlength=k), out=pred_ptr[1:])
    pred = csrc[order]
    h = np.full(k, -1, dtype=np.int64)
    frontier = np.nonzero(outcnt == 0)[0]
    r = 0
    while frontier.size:
        h[frontier] = r
        lens = pred_ptr[frontier + 1] - pred_ptr[frontier]
        idx = np.repeat(pred_ptr[frontier], lens) + (np.arange(lens.sum()) - np.repeat(np.cumsum(lens) - lens, lens))
        ps = pred[idx]
        np.subtract.at(outcnt, ps, 1)
        cand = np.unique(ps)
        frontier = cand[outcnt[cand] == 0]
        r += 1
    assert np.all(h >= 0)
    return h


def scc_only_levels(n, row_ptr, col):
    """Per-vertex level in the plain SCC partition (the vertex labels of
    Fig. 1): length of the longest path from the vertex's SCC to a sink of
    the DAG of SCCs."""
    lab, k = scc_labels(n, row_ptr, col)
    src, dst = _edges_no_loops(n, row_ptr, col)
    cs, cd = lab[src], lab[dst]
    keep = cs != cd
    h = _heights(k, cs[keep], cd[keep])
    return h[lab]


def partition_theorem(n, row_ptr, col):
    """Theorem 3.1 merge process.

    Starting from the SCC partition, a one-vertex component v becomes the
    head of a merge with every CAC of level L-1 it points to, where L is one
    plus the largest level among its successors, unless it points to an SCC
    of two or more vertices on level L-1; after a merge the new CAC has level
    L-1.  Merges are settled bottom-up (by the height of v's SCC in the DAG of
    SCCs), so every successor's level and type are final when v is settled.
    CACs are then the connected groups of vertices joined by merges."""
    if n == 0:
        return _finalise(np.zeros(0, np.int64), np.zeros(0, np.int32), np.zeros(0, np.uint8))
    lab, k = scc_labels(n, row_ptr, col)
    ssize = np.bincount(lab, minlength=k)
    multi = ssize[lab] >= 2  # vertex in an SCC of two or more vertices
    src, dst = _edges_no_loops(n, row_ptr, col)
    cs, cd = lab[src], lab[dst]
    ext = cs != cd
    esrc, edst = src[ext], dst[ext]
    h = _heights(k, cs[ext], cd[ext])
    # group external edges by the height of their source's SCC
    eh = h[lab[esrc]]
    eorder = np.argsort(eh, kind="stable")
    esrc, edst, eh = esrc[eorder], edst[eorder], eh[eorder]
    hmax = int(h.max())
    ebounds = np.searchsorted(eh, np.arange(hmax + 2))
    vlevel = np.full(n, -1, dtype=np.int64)
    # SCCs grouped by height
    sorder = np.argsort(h, kind="stable")
    sbounds = np.searchsorted(h[sorder], np.arange(hmax + 2))
    members_order = np.argsort(lab, kind="stable")
    mptr = np.zeros(k + 1, dtype=np.int64)
    np.cumsum(ssize, out=mptr[1:])
    merge_src, merge_dst = [], []
    # per-SCC scratch; each SCC is settled in exactly one round
    L = np.zeros(k, dtype=np.int64)
    blocked = np.zeros(k, dtype=bool)
    did = np.zeros(k, dtype=bool)
    for r in range(hmax + 1):
        sccs = sorder[sbounds[r]:sbounds[r + 1]]
        a, b = ebounds[r], ebounds[r + 1]
        s_e, d_e = esrc[a:b], edst[a:b]
        # L(S) = 1 + max level of any successor vertex; 0 without successors
        if b > a:
            assert np.all(vlevel[d_e] >= 0)
            np.maximum.at(L, lab[s_e], vlevel[d_e] + 1)
        Ls = L[sccs]
        single = ssize[sccs] == 1
        # multi-vertex SCCs: level L
        big = sccs[~single]
        if big.size:
            lens = ssize[big]
            idx = np.repeat(mptr[big], lens) + (np.arange(lens.sum()) - np.repeat(np.cumsum(lens) - lens, lens))
            vlevel[members_order[idx]] = np.repeat(L[big], lens)
        # one-vertex SCCs: merge test against successors on level L-1
        sing = sccs[single]
        if sing.size:
            v = members_order[mptr[sing]]
            lvl_v = L[sing].copy()
            if b > a:
                Lsrc = L[lab[s_e]]
                on_below = vlevel[d_e] == Lsrc - 1
                src_single = ssize[lab[s_e]] == 1
                hit = on_below & src_single & multi[d_e]
                blocked[lab[s_e][hit]] = True
                mergeable = on_below & src_single & ~multi[d_e] & ~blocked[lab[s_e]]
                merge_src.append(s_e[mergeable])
                merge_dst.append(d_e[mergeable])
                did[lab[s_e][mergeable]] = True
                lvl_v = np.where(did[sing], lvl_v - 1, lvl_v)
            vlevel[v] = lvl_v
    assert np.all(vlevel >= 0)
    # CACs: connected groups of merge edges among CAC vertices
    if merge_src:
        ms = np.concatenate(merge_src)
        md = np.concatenate(merge_dst)
    else:
        ms = md = np.zeros(0, dtype=np.int64)
    M = sp.csr_matrix((np.ones(len(ms), dtype=np.int8), (ms, md)), shape=(n, n))
    _, cac_lab = connected_components(M, directed=False)
    label = np.where(multi, lab, k + cac_lab)
    vtype = multi.astype(np.uint8)
    return _finalise(label, vlevel.astype(np.int32), vtype)


class _MergeFind:
    """Merge-find forest with union by depth (the .depth value of Sec. 4.1)."""

    def __init__(self, n):
        self.parent = list(range(n))
        self.depth = [1] * n

    def find(self, v):
        root = v
        while self.parent[root] != root:
            root = self.parent[root]
        while self.parent[v] != root:  # path compression
            self.parent[v], v = root, self.parent[v]
        return root

    def merge(self, a, b):
        ra, rb = self.find(a), self.find(b)
        if ra == rb:
            return
        if self.depth[ra] < self.depth[rb]:
            ra, rb = rb, ra
        self.parent[rb] = ra
        if self.depth[ra] == self.depth[rb]:
            self.depth[ra] += 1


def partition_dfs(n, row_ptr, col):
    """Modified Tarjan depth-first search of Sec. 4.1, iterative.

    Discover sets index and lowlink to a running counter and the level to 1
    (levels are 1-based inside the search and shifted to 0-based at the end).
    Explore visits every out-edge (v, w) (loops skipped): an unvisited w is
    searched first; then a w already placed in a component raises v's level to
    at least level(w)+1, while a w still on the stack (same SCC) raises it to at
    least level(w) and lowers v's lowlink to at most lowlink(w).  Finish pops
    an SCC when lowlink equals index; a one-vertex SCC becomes a CAC and, as
    head, is merged with every CAC on level(v)-1 it points to, unless it points
    to an SCC of two or more vertices on that level, in which case nothing is
    merged; after a merge the head's level drops by one.  The merge state
    (``m`` and the candidate list) starts empty once per vertex, before the
    edge loop.
    """
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    col = np.asarray(col, dtype=np.int64)
    nbr = [[int(w) for w in col[row_ptr[v]:row_ptr[v + 1]] if int(w) != v] for v in range(n)]
    index = [0] * n  # 0 = not discovered
    low = [0] * n
    level = [0] * n
    typ = [None] * n  # None while on the stack, "scc" / "cac" once placed
    mf = _MergeFind(n)
    stack = []
    counter = 1
    for root in range(n):
        if index[root]:
            continue
        # frames: [vertex, next edge position]
        index[root] = low[root] = counter
        level[root] = 1
        counter += 1
        stack.append(root)
        frames = [[root, 0]]
        while frames:
            fr = frames[-1]
            v, i = fr
            if i < len(nbr[v]):
                w = nbr[v][i]
                if not index[w]:
                    index[w] = low[w] = counter
                    level[w] = 1
                    counter += 1
                    stack.append(w)
                    frames.append([w, 0])
                    continue  # explore w first; edge (v, w) is settled on return
                fr[1] = i + 1
                _settle_edge(v, w, typ, level, low)
                continue
            # Finish(v)
            frames.pop()
            if low[v] == index[v]:
                size = 0
                while True:
                    w = stack.pop()
                    level[w] = level[v]
                    typ[w] = "scc"
                    mf.merge(w, v)
                    size += 1
                    if w == v:
                        break
                if size == 1:
                    typ[v] = "cac"
                    m = False
                    cand = []
                    for w in nbr[v]:
                        if typ[w] == "scc" and level[w] == level[v] - 1:
                            m = False
                            break
                        if typ[w] == "cac" and level[w] == level[v] - 1:
                            cand.append(w)
                            m = True
                    if m:
                        level[v] -= 1
                        for w in cand:
                            mf.merge(w, v)
            if frames:
                parent = frames[-1]
                pv, pi = parent
                parent[1] = pi + 1
                _settle_edge(pv, v, typ, level, low)
    # numbering pass: counter initialised once, ids by first appearance
    comp_of_head = {}
    comp = np.zeros(n, dtype=np.int64)
    nxt = 0
    for v in range(n):
        h = mf.find(v)
        if h not in comp_of_head:
            comp_of_head[h] = nxt
            nxt += 1
        comp[v] = comp_of_head[h]
    vlevel = np.array([lv - 1 for lv in level], dtype=np.int32)
    vtype = np.array([1 if t == "scc" else 0 for t in typ], dtype=np.uint8)
    return _finalise(comp, vlevel, vtype)


def _settle_edge(v, w, typ, level, low):
    if typ[w] is not None:  # w already belongs to a finished component
        level[v] = max(level[v], level[w] + 1)
    else:  # w is on the stack: same SCC as v
        level[v] = max(level[v], level[w])
        low[v] = min(low[v], low[w])


def partition_arrays_equal(a, b):
    return (a["n_comp"] == b["n_comp"] and a["n_levels"] == b["n_levels"]
            and np.array_equal(a["comp"], b["comp"])
            and np.array_equal(a["comp_level"], b["comp_level"])
            and np.array_equal(a["comp_type"], b["comp_type"])
            and np.array_equal(a["comp_size"], b["comp_size"]))
