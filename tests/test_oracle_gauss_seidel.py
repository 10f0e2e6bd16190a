"""Pins of the block Gauss-Seidel oracle (Sec. 4.3.2 alternative for SCCs)."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle.gauss_seidel import block_bounds, block_gauss_seidel
from oracle.pagerank import pagerank_power_series, transition_T_csr
from graphgen import random_digraph, scc_blocks

C = 0.85


def _scc(seed, n=300, m=1500):
    """The largest SCC of a random digraph: M = c A_CC^T (rows and columns in
    the SCC's vertex order) and a positive W'."""
    g = random_digraph(n, m, seed)
    from scipy.sparse.csgraph import connected_components
    A = sp.csr_matrix((np.ones(g.m), g.col, g.row_ptr), shape=(g.n, g.n))
    _, lab = connected_components(A, directed=True, connection="strong")
    big = np.argmax(np.bincount(lab))
    vs = np.nonzero(lab == big)[0]
    AT = transition_T_csr(g.n, g.row_ptr, g.col)
    M = (C * AT[vs][:, vs]).tocsr()
    Wp = np.random.default_rng(seed).uniform(0.5, 1.5, len(vs))
    return M, Wp


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("blocks", [1, 2, 4, 16])
def test_certificate_bounds_the_error(seed, blocks):
    """||R - R*||_1 <= c ||dR||_1 / (1 - c) <= c eps ||W'||_1 against the
    dense solve, and the residual obeys ||r||_1 <= c ||dR||_1 after every
    number of sweeps."""
    M, Wp = _scc(seed)
    nv = len(Wp)
    Rstar = np.linalg.solve(np.eye(nv) - M.toarray(), Wp)
    for eps in (1e-3, 1e-8):
        R, sweeps, last = block_gauss_seidel(M, Wp, C, eps, blocks)
        err = np.abs(R - Rstar).sum()
        assert err <= C * last / (1 - C) * (1 + 1e-9) + 1e-12
        assert last <= eps * (1 - C) * Wp.sum()
    for k in (1, 2, 5):
        Rk, _, lastk = block_gauss_seidel(M, Wp, C, 0.0, blocks, max_sweeps=k)
        r = Wp - Rk + M @ Rk
        assert np.abs(r).sum() <= C * lastk * (1 + 1e-12) + 1e-13


@pytest.mark.parametrize("seed", range(3))
def test_one_block_is_the_power_series(seed):
    """With one block the sweeps are the series started from W': after k
    sweeps R is the partial sum P_0 + ... + P_k, ||dR|| is ||P_k||, and the
    stop comes after the same number of terms as the series' CERT rule."""
    M, Wp = _scc(seed)
    P, S, norms = Wp.copy(), Wp.copy(), []
    for _ in range(300):
        P = M @ P
        S = S + P
        norms.append(np.abs(P).sum())
    for k in (1, 3, 10):
        Rk, sw, last = block_gauss_seidel(M, Wp, C, 0.0, 1, max_sweeps=k)
        Sk = Wp + sum(np.linalg.matrix_power(M.toarray(), j) @ Wp for j in range(1, k + 1))
        np.testing.assert_allclose(Rk, Sk, rtol=1e-13)
        assert last == pytest.approx(norms[k - 1], rel=1e-10)
    eps = 1e-6
    _, sweeps, _ = block_gauss_seidel(M, Wp, C, eps, 1)
    first = next(k for k, nk in enumerate(norms, 1) if nk <= eps * (1 - C) * Wp.sum())
    assert sweeps == first


def test_point_gauss_seidel_on_a_two_cycle():
    """Two vertices pointing at each other (a_12 = a_21 = 1), W' = (1, 1): point
    Gauss-Seidel from R = W' gives R_1 = 1 + c R_2 then R_2 = 1 + c R_1, an
    error that shrinks by c^2 per sweep (the series shrinks by c per term);
    the exact R is 1/(1-c) for both."""
    M = C * np.array([[0.0, 1.0], [1.0, 0.0]])
    Wp = np.ones(2)
    R1, _, _ = block_gauss_seidel(M, Wp, C, 0.0, 2, max_sweeps=1)
    np.testing.assert_allclose(R1, [1 + C, 1 + C * (1 + C)], rtol=1e-15)
    e = [abs(block_gauss_seidel(M, Wp, C, 0.0, 2, max_sweeps=k)[0][1] - 1 / (1 - C)) for k in (3, 4, 5)]
    np.testing.assert_allclose([e[1] / e[0], e[2] / e[1]], [C * C, C * C], rtol=1e-9)
    # a planted mistake: Jacobi inside the one-row blocks would shrink by c only
    R, sweeps, _ = block_gauss_seidel(M, Wp, C, 1e-10, 2)
    _, sweeps_j, _ = block_gauss_seidel(M, Wp, C, 1e-10, 1)
    assert sweeps < 0.6 * sweeps_j
    np.testing.assert_allclose(R, [1 / (1 - C)] * 2, rtol=1e-9)


@pytest.mark.parametrize("seed", range(3))
def test_more_blocks_need_no_more_sweeps_on_web_like_sccs(seed):
    """On the block SCCs of the synthetic inputs, block Gauss-Seidel with 4 or
    more blocks needs fewer sweeps than the series needs terms (the Stein-
    Rosenberg comparison for this M-matrix splitting)."""
    M, Wp = _scc(seed + 10, n=400, m=2400)
    _, s1, _ = block_gauss_seidel(M, Wp, C, 1e-8, 1)
    _, s4, _ = block_gauss_seidel(M, Wp, C, 1e-8, 4)
    _, s16, _ = block_gauss_seidel(M, Wp, C, 1e-8, 16)
    assert s16 <= s4 <= s1 and s4 < s1


def test_block_bounds():
    assert block_bounds(10, 4) == [0, 2, 5, 7, 10]
    assert block_bounds(3, 8) == [0, 1, 2, 3]
    assert block_bounds(5, 1) == [0, 5]
