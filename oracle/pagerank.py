"""Non-normalised PageRank R^(3): definitions and the plain power series.

Test infrastructure only (see the package docstring).

Conventions (Def. 3.4): A is the adjacency matrix with every non-zero row
scaled to sum to one.  Self-loops are ignored by default, as in the
experiments of Sec. 5.2; with loops=True they stay in A (a vertex with a loop
has a_vv > 0 and the loop counts in its out-degree), the general definition.
A repeated edge counts with its multiplicity (the paper assumes simple
graphs, Sec. 3, so this only matters for inputs that are not).  Dangling
vertices have a zero row.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def out_degree(n, row_ptr, col, loops=False):
    """Out-degree, duplicates counted; self-loops only with loops=True."""
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    col = np.asarray(col, dtype=np.int64)
    src = np.repeat(np.arange(n, dtype=np.int64), np.diff(row_ptr))
    keep = (src != col) | loops
    return np.bincount(src[keep], minlength=n).astype(np.int64)


def transition_dense(n, row_ptr, col, loops=False):
    """Dense A of Def. 3.4 (row-normalised; loops dropped unless loops=True)."""
    A = np.zeros((n, n), dtype=np.float64)
    for u in range(n):
        for e in range(int(row_ptr[u]), int(row_ptr[u + 1])):
            v = int(col[e])
            if v != u or loops:
                A[u, v] += 1.0
    s = A.sum(axis=1)
    nz = s > 0
    A[nz] /= s[nz, None]
    return A


def transition_T_csr(n, row_ptr, col, loops=False, weight=None):
    """A^T as a scipy CSR matrix: row v holds a_uv for every edge u->v
    (self-loops only with loops=True).  Unweighted, a_uv = 1/outdeg(u); for a
    weighted graph (Def. 3.4, a Markov chain's transition weights, one weight
    per edge in col order) a_uv = w_uv / s_u with s_u the total weight of u's
    kept out-edges (repeated edges add up; a vertex whose kept out-edges all
    weigh zero has a zero row, like a dangling vertex)."""
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    col = np.asarray(col, dtype=np.int64)
    src = np.repeat(np.arange(n, dtype=np.int64), np.diff(row_ptr))
    keep = (src != col) | loops
    src, dst = src[keep], col[keep]
    if weight is None:
        deg = np.bincount(src, minlength=n).astype(np.float64)
        val = 1.0 / deg[src]
    else:
        wv = np.asarray(weight, dtype=np.float64)[keep]
        s = np.bincount(src, weights=wv, minlength=n)
        val = np.zeros_like(wv)
        np.divide(wv, s[src], out=val, where=s[src] > 0)
    return sp.csr_matrix((val, (dst, src)), shape=(n, n))


def pagerank_dense(n, row_ptr, col, c, W, loops=False):
    """R^(3) as the solution of (I - c A^T) R = W (Sec. 4.3, third method;
    equivalent to Def. 3.5).  LAPACK via numpy; for small n only."""
    A = transition_dense(n, row_ptr, col, loops)
    return np.linalg.solve(np.eye(n) - c * A.T, np.asarray(W, dtype=np.float64))


def pagerank_dense_weighted(n, row_ptr, col, weight, c, W, loops=False):
    """R^(3) of Def. 3.4/3.5 for a weighted graph (a Markov chain's
    transition weights): a_uv = w_uv / sum_x w_ux over the out-edges of u
    (repeated edges add their weights; loops dropped unless loops=True),
    then the dense solve (I - c A^T) R = W."""
    weight = np.asarray(weight, dtype=np.float64)
    A = np.zeros((n, n), dtype=np.float64)
    for u in range(n):
        for e in range(int(row_ptr[u]), int(row_ptr[u + 1])):
            v = int(col[e])
            if v != u or loops:
                A[u, v] += weight[e]
    s = A.sum(axis=1)
    nz = s > 0
    A[nz] /= s[nz, None]
    return np.linalg.solve(np.eye(n) - c * A.T, np.asarray(W, dtype=np.float64))


def pagerank_r1(n, row_ptr, col, c, w):
    """R^(1) of Def. 3.4: the eigenvector of M = c(A + g w^T)^T + (1-c) w e^T
    for eigenvalue one, scaled to unit 1-norm (numpy eigen-solver)."""
    A = transition_dense(n, row_ptr, col)
    w = np.asarray(w, dtype=np.float64)
    w = w / w.sum()
    g = (A.sum(axis=1) == 0).astype(np.float64)
    M = c * (A + np.outer(g, w)).T + (1.0 - c) * np.outer(w, np.ones(n))
    vals, vecs = np.linalg.eig(M)
    k = int(np.argmin(np.abs(vals - 1.0)))
    r = np.real(vecs[:, k])
    return r / r.sum()


def r3_from_r1(n, row_ptr, col, c, R1, W):
    """Def. 3.5: R^(3) = R^(1) ||W||_1 / d with d = 1 - sum(c A^T R^(1))."""
    A = transition_dense(n, row_ptr, col)
    d = 1.0 - np.sum(c * (A.T @ R1))
    return R1 * np.sum(np.abs(W)) / d


def pagerank_random_walks(n, row_ptr, col, c, W, walks_per_unit, seed):
    """Monte-Carlo estimate of Def. 3.6: start round(W_i * walks_per_unit) walks
    at every vertex; each step follows a uniformly chosen out-edge (loops
    ignored) with probability c and stops otherwise or at a dangling vertex.
    R_j is estimated by the number of visits to j divided by walks_per_unit."""
    rng = np.random.default_rng(seed)
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    col = np.asarray(col, dtype=np.int64)
    nbrs = []
    for u in range(n):
        nb = [int(v) for v in col[row_ptr[u]:row_ptr[u + 1]] if int(v) != u]
        nbrs.append(np.array(nb, dtype=np.int64))
    visits = np.zeros(n, dtype=np.float64)
    for i in range(n):
        k = int(round(W[i] * walks_per_unit))
        pos = np.full(k, i, dtype=np.int64)
        while pos.size:
            np.add.at(visits, pos, 1.0)
            cont = rng.random(pos.size) < c
            pos = pos[cont]
            nxt = np.empty_like(pos)
            alive = np.ones(pos.size, dtype=bool)
            for j, u in enumerate(pos):
                nb = nbrs[u]
                if nb.size == 0:
                    alive[j] = False
                else:
                    nxt[j] = nb[rng.integers(0, nb.size)]
            pos = nxt[alive]
    return visits / walks_per_unit


def pagerank_power_series(n, row_ptr, col, c, W, *, stop="cert", eps=1e-6, tol=None,
                          max_iter=1_000_000, AT=None, loops=False, tail=False):
    """The power series of Sec. 4.3.2 on the whole graph (the paper's baseline,
    "method 1" of Sec. 5.2):  P_0 = W,  P_{k+1} = c A^T P_k,  R = sum_k P_k.

    Stop rules (one term P_k is added per iteration, k >= 1):
      "cert":  stop after the first k with ||P_k||_1 <= eps (1-c) ||W||_1.
               Because ||c A^T x||_1 <= c ||x||_1 (Sec. 4.4), the neglected tail
               is at most c/(1-c) ||P_k||_1 <= c eps ||W||_1 <= c eps ||R*||_1,
               a relative 1-norm error below eps.
      "paper": stop after the first k with max(P_k) < tol (the listing of
               Sec. 4.3.2; an absolute max-norm rule).
    tail (with "cert"): the certified geometric tail estimate on the whole
    graph, the rule the componentwise solve applies per SCC.  After term
    P_{k+1}, with rho = ||P_k||_1 / ||P_{k-1}||_1 in (0, 1), the candidate
    R' = P_0 + ... + P_k + rho/(1-rho) P_k has residual W - (I - cA^T)R' =
    (P_{k+1} - rho P_k)/(1-rho); the series stops with R' once that residual's
    norm is at most eps (1-c) ||W||_1 (the plain test is tried first).  The
    returned last norm is then the residual norm divided by c.
    Returns (R, iterations, ||P_K||_1).
    """
    if AT is None:
        AT = transition_T_csr(n, row_ptr, col, loops)
    W = np.asarray(W, dtype=np.float64)
    R = W.copy()
    p = W.copy()
    wnorm = float(np.sum(np.abs(W)))
    k = 0
    last = wnorm
    norm_prev, norm_prev2 = wnorm, None  # ||P_k||_1 and ||P_{k-1}||_1
    while k < max_iter:
        if stop == "cert" and wnorm == 0.0:
            break
        q = c * (AT @ p)
        k += 1
        qn = float(np.sum(np.abs(q)))
        if stop == "cert":
            if qn <= eps * (1.0 - c) * wnorm:
                R += q
                last = qn
                break
            if tail and norm_prev2 is not None and norm_prev2 > 0.0:
                rho = norm_prev / norm_prev2
                if 0.0 < rho < 1.0:
                    res = float(np.sum(np.abs(q - rho * p))) / (1.0 - rho)
                    if res <= eps * (1.0 - c) * wnorm:
                        R += rho / (1.0 - rho) * p
                        last = res / c
                        break
        elif stop == "paper":
            if q.size == 0 or float(np.max(q)) < tol:
                R += q
                last = qn
                break
        else:
            raise ValueError(stop)
        R += q
        last = qn
        norm_prev2, norm_prev = norm_prev, qn
        p = q
    return R, k, last


def residual_rows(n, row_ptr, col, c, W, R, AT=None, loops=False):
    """Per-row residual r = W - (I - c A^T) R of a candidate R (Sec. 4.4), and
    the size of the terms each row's residual is formed from,
    |W| + |R| + c A^T |R| (what its FP64 rounding is relative to).  Returns
    (r, scale, A^T)."""
    if AT is None:
        AT = transition_T_csr(n, row_ptr, col, loops)
    R = np.asarray(R, dtype=np.float64)
    W = np.asarray(W, dtype=np.float64)
    r = W - R + c * (AT @ R)
    scale = np.abs(W) + np.abs(R) + c * (AT @ np.abs(R))
    return r, scale, AT


def residual_bound(n, row_ptr, col, c, W, R, AT=None, loops=False):
    """Certificate of any candidate R (Sec. 4.4): the residual r = W - (I - c A^T) R
    satisfies R* - R = (I - c A^T)^{-1} r, and the column sums of c A^T are at
    most c, so ||R* - R||_1 <= ||r||_1 / (1 - c).  Returns that bound divided
    by ||R||_1 (a relative 1-norm error bound) and A^T for reuse."""
    if AT is None:
        AT = transition_T_csr(n, row_ptr, col, loops)
    R = np.asarray(R, dtype=np.float64)
    r = np.asarray(W, dtype=np.float64) - R + c * (AT @ R)
    return float(np.abs(r).sum() / ((1.0 - c) * np.abs(R).sum())), AT
