"""Serial componentwise PageRank (Sec. 3.3).

Test infrastructure only (see the package docstring).

Levels are solved from the highest down to 0 (Sec. 3.3, steps 1-4).  Before a
level is solved its weights are raised by the rank flowing in from every
higher level (Corollary 3.2 and eq. PR:levels):

    W'_v = W_v + c * sum_{u -> v, level(u) > level(v)} R_u / outdeg(u)

Then, per component of the level (Sec. 3.3, the four-way method choice with
loops ignored):
  * a one-vertex component has R_v = W'_v,
  * a CAC of two or more vertices is solved exactly by the in-degree
    countdown sweep of Sec. 3.3.1 (a vertex enters the queue once all of its
    in-edges inside the CAC have been used),
  * an SCC is solved by the power series of Sec. 3.3.2 restricted to the
    component, started from P_0 = W'_C.
The SCCs of one level are iterated together as one block-diagonal product
(there are no edges between different components of a level), but each keeps
its own stop test and stops contributing once it has converged.
"""
from __future__ import annotations

from collections import deque

import numpy as np

from .pagerank import out_degree, transition_T_csr
from .partition import partition_theorem


def componentwise_solve(n, row_ptr, col, c, W, *, part=None, stop="cert", eps=1e-6,
                        tol=None, max_iter=1_000_000, return_stats=False):
    """Componentwise R^(3).

    Stop rule per SCC C (one term added per iteration, k >= 1):
      "cert":  ||P_k||_1 <= eps (1-c) ||W'_C||_1  (the relative 1-norm error of
               the whole result is then below c*eps; the residual of the
               computed R is non-zero only on SCC rows, where it equals the
               next, unused term of each component's series)
      "paper": max(P_k) < tol.
    """
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    col = np.asarray(col, dtype=np.int64)
    W = np.asarray(W, dtype=np.float64)
    if part is None:
        part = partition_theorem(n, row_ptr, col)
    comp = part["comp"].astype(np.int64)
    clevel = part["comp_level"].astype(np.int64)
    ctype = part["comp_type"]
    csize = part["comp_size"].astype(np.int64)
    vlevel = clevel[comp]
    AT = transition_T_csr(n, row_ptr, col)
    deg = out_degree(n, row_ptr, col)
    nbr_ptr, nbr = row_ptr, col  # out-edges for the CAC sweep
    R = np.zeros(n, dtype=np.float64)
    iters = np.zeros(len(csize), dtype=np.int64)
    last = np.zeros(len(csize), dtype=np.float64)
    wprime = np.zeros(n, dtype=np.float64)
    if n == 0:
        return (R, dict(iters=iters, last=last, wprime=wprime)) if return_stats else R
    order = np.argsort(-vlevel, kind="stable")
    lev_sorted = vlevel[order]
    top = int(vlevel.max())
    for lvl in range(top, -1, -1):
        lo = np.searchsorted(-lev_sorted, -lvl, side="left")
        hi = np.searchsorted(-lev_sorted, -lvl, side="right")
        V = np.sort(order[lo:hi])
        # eq. PR:levels: only higher levels hold non-zero R at this point, and
        # no edge joins two different components of the same level
        Wp = W[V] + c * (AT[V, :] @ R)
        wprime[V] = Wp
        R[V] = 0.0
        cV = comp[V]
        single = (csize[cV] == 1)
        R[V[single]] = Wp[single]
        # CACs of two or more vertices: in-degree countdown sweep
        cac_mask = (ctype[cV] == 0) & ~single
        if np.any(cac_mask):
            _cac_sweep(V[cac_mask], Wp[cac_mask], comp, c, deg, nbr_ptr, nbr, R)
        # SCCs: power series per component
        scc_mask = ctype[cV] == 1
        if np.any(scc_mask):
            Vs = V[scc_mask]
            _scc_series(Vs, Wp[scc_mask], comp, c, AT, R, iters, last, stop, eps, tol, max_iter)
    if return_stats:
        return R, dict(iters=iters, last=last, wprime=wprime)
    return R


def _cac_sweep(Vc, Wp, comp, c, deg, nbr_ptr, nbr, R):
    """Sec. 3.3.1 with loops ignored: v.degree = in-degree inside v's CAC,
    v.rank = W'_v; a vertex is dequeued only after all its in-edges inside the
    CAC have delivered rank, and then pushes c*rank/outdeg along each out-edge
    inside the CAC.  Every vertex and edge is used once."""
    member = {int(v): i for i, v in enumerate(Vc)}
    rank = Wp.astype(np.float64).copy()
    degree = np.zeros(len(Vc), dtype=np.int64)
    for i, v in enumerate(Vc):
        v = int(v)
        for e in range(int(nbr_ptr[v]), int(nbr_ptr[v + 1])):
            u = int(nbr[e])
            if u != v and comp[u] == comp[v] and u in member:
                degree[member[u]] += 1
    q = deque()
    for i in range(len(Vc)):
        if degree[i] == 0:
            q.append(i)
            while q:
                j = q.popleft()
                w = int(Vc[j])
                for e in range(int(nbr_ptr[w]), int(nbr_ptr[w + 1])):
                    u = int(nbr[e])
                    if u == w or comp[u] != comp[w] or u not in member:
                        continue
                    k = member[u]
                    rank[k] += rank[j] * c / deg[w]
                    degree[k] -= 1
                    if degree[k] == 0:
                        q.append(k)
                degree[j] -= 1  # never enqueued again
    assert np.all(degree == -1), "CAC sweep left vertices unvisited (cycle?)"
    R[Vc] = rank


def _scc_series(Vs, Wp, comp, c, AT, R, iters, last, stop, eps, tol, max_iter):
    """Power series of Sec. 3.3.2 on each SCC of one level."""
    sub = AT[Vs, :][:, Vs]  # block diagonal over the level's SCCs
    cid = comp[Vs]
    uniq, local = np.unique(cid, return_inverse=True)
    nc = len(uniq)
    wnorm = np.bincount(local, weights=np.abs(Wp), minlength=nc)
    p = Wp.copy()
    acc = Wp.copy()
    active = wnorm > 0 if stop == "cert" else np.ones(nc, dtype=bool)
    it = np.zeros(nc, dtype=np.int64)
    lastn = wnorm.copy()
    k = 0
    while np.any(active) and k < max_iter:
        p = c * (sub @ p)
        p[~active[local]] = 0.0
        acc += p
        k += 1
        it[active] = k
        pn = np.bincount(local, weights=np.abs(p), minlength=nc)
        lastn[active] = pn[active]
        if stop == "cert":
            done = pn <= eps * (1.0 - c) * wnorm
        else:
            pm = np.zeros(nc)
            np.maximum.at(pm, local, p)
            done = pm < tol
        active &= ~done
    R[Vs] = acc
    iters[uniq] = it
    last[uniq] = lastn
