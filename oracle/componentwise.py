"""Serial componentwise PageRank (Sec. 4.3).

Test infrastructure only (see the package docstring).

Levels are solved from the highest down to 0 (Sec. 4.3, steps 1-4).  Before a
level is solved its weights are raised by the rank flowing in from every
higher level (Corollary 3.2 and eq. PR:levels):

    W'_v = W_v + c * sum_{u -> v, level(u) > level(v)} R_u / outdeg(u)

Then, per component of the level (Sec. 4.3, the four-way method choice with
loops ignored):
  * a one-vertex component has R_v = W'_v,
  * a CAC of two or more vertices is solved exactly by the in-degree
    countdown sweep of Sec. 4.3.1 (a vertex enters the queue once all of its
    in-edges inside the CAC have been used),
  * an SCC is solved by the power series of Sec. 4.3.2 restricted to the
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
                        tol=None, max_iter=1_000_000, return_stats=False, warm=None, warm_fn=None,
                        direct_max=0, loops=False, tail=False):
    """Componentwise R^(3).

    Stop rule per SCC C (one term added per iteration, k >= 1):
      "cert":  ||P_k||_1 <= eps (1-c) ||W'_C||_1  (the relative 1-norm error of
               the whole result is then below c*eps; the residual of the
               computed R is non-zero only on SCC rows, where it equals the
               next, unused term of each component's series)
      "paper": max(P_k) < tol.

    warm: parameters of the starting-guess network (oracle.warmstart); each
    SCC then starts from its prediction R_0 when that passes the residual
    test, else from W'_C as usual.  warm_fn(F, Vs, s) -> y may replace the
    network (F: feature rows of the vertices Vs, s: their component scale),
    e.g. to plant a perfect or a useless guess.  The stats then also hold, per component, the accept flag
    (1 kept, 0 fell back, -1 not an SCC).

    loops: keep self-loops in A (the general definition; the partition does
    not change, a loop being a cycle of one vertex only).  A one-vertex
    component then has R_v = W'_v / (1 - c a_vv), and in the CAC sweep a
    vertex's collected rank is divided by (1 - c a_vv) before it is passed
    on (the loop's own share comes back to it); SCC series use A_CC with its
    diagonal.

    tail: with the CERT rule, an SCC may also stop early on a geometric
    estimate of the rest of its series.  After term P_{k+1} with
    rho = ||P_k||_1 / ||P_{k-1}||_1 < 1, the candidate
    R' = P_0 + ... + P_k + rho/(1-rho) P_k has the residual
    W' - (I - c A_CC^T) R' = (P_{k+1} - rho P_k) / (1 - rho), so
    ||R' - R*_C||_1 <= ||P_{k+1} - rho P_k||_1 / ((1-rho)(1-c)); the SCC stops
    with R' when that is at most eps ||W'_C||_1 (the CERT rule's own bound).
    The plain test is tried first.  Its last-term norm is then the residual
    norm divided by c, so the certificate's c/(1-c) factor gives the bound.
    With a starting guess the same rule runs on the residual series r_k of a
    kept guess (rho from the second new term on: nothing precedes r_0) and
    on the plain series of one that fell back.

    direct_max: SCCs of at most this many vertices are solved directly,
    (I - c A_CC^T) R_C = W'_C with a dense LAPACK solve: the paper's choice
    for small SCCs in the per-component method dispatch of Sec. 4.3 (zero
    iterations, zero last-term norm).
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
    AT = transition_T_csr(n, row_ptr, col, loops)
    deg = out_degree(n, row_ptr, col, loops)
    a_diag = AT.diagonal() if loops else np.zeros(n)
    nbr_ptr, nbr = row_ptr, col  # out-edges for the CAC sweep
    R = np.zeros(n, dtype=np.float64)
    iters = np.zeros(len(csize), dtype=np.int64)
    last = np.zeros(len(csize), dtype=np.float64)
    wprime = np.zeros(n, dtype=np.float64)
    accepted = np.full(len(csize), -1, dtype=np.int64)
    if warm is not None and warm_fn is None:
        from .warmstart import forward

        def warm_fn(F, Vs, sv):
            return forward(warm, F)
    feat = None
    if warm_fn is not None:
        from .warmstart import in_degree

        feat = dict(fn=warm_fn, W=W, indeg=in_degree(n, row_ptr, col), outdeg=out_degree(n, row_ptr, col),
                    accepted=accepted)
    if n == 0:
        return (R, dict(iters=iters, last=last, wprime=wprime, accepted=accepted)) if return_stats else R
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
        R[V[single]] = Wp[single] / (1.0 - c * a_diag[V[single]])
        # CACs of two or more vertices: in-degree countdown sweep
        cac_mask = (ctype[cV] == 0) & ~single
        if np.any(cac_mask):
            _cac_sweep(V[cac_mask], Wp[cac_mask], comp, c, deg, nbr_ptr, nbr, R, a_diag)
        # SCCs: small ones solved directly when asked, the rest by the power
        # series per component
        scc_mask = ctype[cV] == 1
        if direct_max > 0:
            dmask = scc_mask & (csize[cV] <= direct_max)
            if np.any(dmask):
                _scc_direct(V[dmask], Wp[dmask], comp, c, AT, R)
            scc_mask = scc_mask & ~dmask
        if np.any(scc_mask):
            Vs = V[scc_mask]
            _scc_series(Vs, Wp[scc_mask], comp, c, AT, R, iters, last, stop, eps, tol, max_iter, feat, tail)
    if return_stats:
        return R, dict(iters=iters, last=last, wprime=wprime, accepted=accepted)
    return R


def _cac_sweep(Vc, Wp, comp, c, deg, nbr_ptr, nbr, R, a_diag=None):
    """Sec. 4.3.1: v.degree = in-degree inside v's CAC (loops not counted),
    v.rank = W'_v; a vertex is dequeued only after all its in-edges inside the
    CAC have delivered rank; its rank is then final (divided by 1 - c a_vv
    when it has a loop) and it pushes c*rank/outdeg along each out-edge
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
                if a_diag is not None and a_diag[w] != 0.0:
                    rank[j] /= 1.0 - c * a_diag[w]
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


def _scc_direct(Vd, Wp, comp, c, AT, R):
    """Each SCC C among the vertices Vd: R_C = (I - c A_CC^T)^{-1} W'_C, the
    definition (Def. 3.4/3.5) restricted to C, by one dense solve."""
    cid = comp[Vd]
    for C in np.unique(cid):
        m = cid == C
        idx = Vd[m]
        M = np.eye(len(idx)) - c * AT[idx, :][:, idx].toarray()
        R[idx] = np.linalg.solve(M, Wp[m])


def _scc_series(Vs, Wp, comp, c, AT, R, iters, last, stop, eps, tol, max_iter, feat=None, tail=False):
    """Power series of Sec. 4.3.2 on each SCC of one level.

    With a starting guess (feat), a component whose guess passes the residual
    test starts from p = r_0 and R = R_0 + r_0 with no term counted yet; one
    that falls back continues from the state after the plain first term
    (p = P_1, R = W' + P_1, one term counted).  Either way the stop rule is
    then tested on the current term before the next one is formed."""
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

    def stop_test(pv):
        if stop == "cert":
            return np.bincount(local, weights=np.abs(pv), minlength=nc) <= eps * (1.0 - c) * wnorm
        pm = np.zeros(nc)
        np.maximum.at(pm, local, np.abs(pv))
        return pm < tol

    if feat is not None:
        from .warmstart import scc_features

        F, s, R1 = scc_features(Vs, Wp, feat["W"], local, nc, sub, c, feat["indeg"], feat["outdeg"])
        live = s > 0
        y = np.asarray(feat["fn"](F, Vs, s[local]), dtype=np.float64)
        R0 = s[local] * np.exp(y)
        r0 = Wp + c * (sub @ R0) - R0
        p1 = R1 - Wp
        n_r0 = np.bincount(local, weights=np.abs(r0), minlength=nc)
        n_p1 = np.bincount(local, weights=np.abs(p1), minlength=nc)
        keep = live & (n_r0 < n_p1)
        kv = keep[local]
        p = np.where(kv, r0, p1)
        acc = np.where(kv, R0 + r0, R1)
        it = np.where(keep, 0, 1).astype(np.int64)
        lastn = np.where(keep, n_r0, n_p1)
        feat["accepted"][uniq] = keep.astype(np.int64)
        active = live.copy()
        active &= ~stop_test(p)
        p[~active[local]] = 0.0
        # the series continues from the current term p: r_0 (nothing before
        # it in this series) or P_1 (after P_0 = W'_C)
        norm_prev = lastn.copy()
        norm_prev2 = np.where(keep, np.nan, wnorm)
    else:
        norm_prev = wnorm.copy()            # ||P_k||_1 (k = 0: W'_C)
        norm_prev2 = np.full(nc, np.nan)    # ||P_{k-1}||_1, unknown before P_1
    use_tail = tail and stop == "cert"
    while np.any(active) and int(it[active].max()) < max_iter:
        q = c * (sub @ p)
        q[~active[local]] = 0.0
        it[active] += 1
        qn = np.bincount(local, weights=np.abs(q), minlength=nc)
        done = stop_test(q)
        acc_new = acc + q
        if use_tail:
            with np.errstate(invalid="ignore", divide="ignore"):
                rho = norm_prev / norm_prev2
            ok_rho = np.isfinite(rho) & (rho > 0.0) & (rho < 1.0)
            rho_s = np.where(ok_rho, rho, 0.0)
            d = np.bincount(local, weights=np.abs(q - rho_s[local] * p), minlength=nc)
            res = np.where(ok_rho, d / np.where(ok_rho, 1.0 - rho_s, 1.0), np.inf)
            tail_stop = active & ~done & ok_rho & (res <= eps * (1.0 - c) * wnorm)
            if np.any(tail_stop):
                ts = tail_stop[local]
                f = rho_s / np.where(ok_rho, 1.0 - rho_s, 1.0)
                acc_new = np.where(ts, acc + f[local] * p, acc_new)
                qn = np.where(tail_stop, res / c, qn)
                done = done | tail_stop
        acc = acc_new
        lastn[active] = qn[active]
        norm_prev2, norm_prev = norm_prev, qn
        p = q
        active &= ~done
        active &= it < max_iter
    R[Vs] = acc
    iters[uniq] = it
    last[uniq] = lastn
