"""Pins for the starting-guess network and the warm-started series (CPU)."""
import math

import numpy as np
import pytest

from graphgen import random_digraph, small_plain
from oracle import warmstart as ws
from oracle.componentwise import componentwise_solve
from oracle.pagerank import pagerank_dense


def test_parameter_count():
    # 4*64 + 64 + 64*64 + 64 + 64 + 1
    assert ws.N_PARAMS == 4545


def test_gelu_values():
    # x * Phi(x): Phi(0) = 1/2, Phi(1) = 0.8413447460685429 (standard normal table)
    assert ws.gelu(np.array(0.0)) == 0.0
    assert ws.gelu(np.array(1.0)) == pytest.approx(0.8413447460685429, rel=1e-15)
    assert ws.gelu(np.array(-1.0)) == pytest.approx(-0.15865525393145707, rel=1e-14)
    assert ws.gelu_grad(np.array(0.0)) == 0.5
    # large |x|: identity and zero
    assert ws.gelu(np.array(10.0)) == pytest.approx(10.0)
    assert abs(ws.gelu(np.array(-10.0))) < 1e-20
    x = np.linspace(-4, 4, 41)
    h = 1e-6
    fd = (ws.gelu(x + h) - ws.gelu(x - h)) / (2 * h)
    np.testing.assert_allclose(ws.gelu_grad(x), fd, rtol=1e-8, atol=1e-9)


def test_forward_special_cases():
    th = ws.init_params(3)
    P = ws.unpack(th)
    # zero output layer: the output is the bias
    P["W3"][:] = 0.0
    P["b3"][:] = 0.75
    X = np.random.default_rng(0).normal(size=(9, 4))
    np.testing.assert_array_equal(ws.forward(th, X), np.full(9, 0.75))
    # one-hot path: W1 picks feature 2, W2 identity on unit 0, W3 reads unit 0
    th2 = np.zeros(ws.N_PARAMS)
    Q = ws.unpack(th2)
    Q["W1"][0, 2] = 1.0
    Q["W2"][0, 0] = 1.0
    Q["W3"][0, 0] = 1.0
    y = ws.forward(th2, X)
    np.testing.assert_allclose(y, ws.gelu(ws.gelu(X[:, 2])), rtol=1e-15)


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(1)
    th = ws.init_params(5) * 2.0
    X = rng.normal(size=(7, 4))
    t = rng.normal(size=7)
    L, g = ws.loss_and_grad(th, X, t)
    assert L == pytest.approx(np.mean((ws.forward(th, X) - t) ** 2))
    h = 1e-6
    idx = np.concatenate([rng.choice(ws.N_PARAMS, 200, replace=False), np.arange(ws.N_PARAMS - 65, ws.N_PARAMS)])
    fd = np.empty(len(idx))
    for j, i in enumerate(idx):
        e = np.zeros(ws.N_PARAMS)
        e[i] = h
        fd[j] = (ws.loss_and_grad(th + e, X, t)[0] - ws.loss_and_grad(th - e, X, t)[0]) / (2 * h)
    np.testing.assert_allclose(g[idx], fd, rtol=1e-5, atol=1e-9)


def test_adam_closed_form():
    g1 = np.array([0.5, -2.0, 1e-3, 0.0])
    th = np.array([1.0, 2.0, 3.0, 4.0])
    opt = ws.Adam(4, lr=0.1)
    th1 = opt.step(th, g1)
    # first step: mhat = g, vhat = g^2
    np.testing.assert_allclose(th1, th - 0.1 * g1 / (np.abs(g1) + 1e-8), rtol=1e-14)
    g2 = np.array([1.0, 1.0, -1.0, 2.0])
    th2 = opt.step(th1, g2)
    m = 0.9 * 0.1 * g1 + 0.1 * g2
    v = 0.999 * 0.001 * g1 ** 2 + 0.001 * g2 ** 2
    mhat, vhat = m / (1 - 0.81), v / (1 - 0.999 ** 2)
    np.testing.assert_allclose(th2, th1 - 0.1 * mhat / (np.sqrt(vhat) + 1e-8), rtol=1e-12)


def _graph_with_sccs(seed):
    g = random_digraph(400, 1400, seed=seed)
    return g.n, g.row_ptr, g.col


@pytest.mark.parametrize("seed", [11, 12])
def test_warm_start_does_not_change_the_answer(seed):
    n, rp, col = _graph_with_sccs(seed)
    c = 0.85
    W = np.random.default_rng(seed).uniform(0.5, 2.0, n)
    exact = pagerank_dense(n, rp, col, c, W)
    R, st = componentwise_solve(n, rp, col, c, W, eps=1e-10, return_stats=True, warm=ws.init_params(seed))
    assert np.abs(R - exact).sum() / exact.sum() < 1e-10
    assert (st["accepted"] >= 0).any()


def test_perfect_guess_is_accepted_and_needs_no_terms():
    n, rp, col = _graph_with_sccs(13)
    c = 0.85
    W = np.ones(n)
    exact = pagerank_dense(n, rp, col, c, W)

    def perfect(F, Vs, s):
        return np.log(exact[Vs] / s)

    R, st = componentwise_solve(n, rp, col, c, W, eps=1e-8, return_stats=True, warm_fn=perfect)
    scc = st["accepted"] >= 0
    assert scc.any() and (st["accepted"][scc] == 1).all()
    assert st["iters"][scc].max() <= 1
    assert np.abs(R - exact).sum() / exact.sum() < 1e-12


def test_useless_guess_falls_back_to_the_plain_series():
    n, rp, col = _graph_with_sccs(14)
    c = 0.85
    W = np.ones(n)
    R0, st0 = componentwise_solve(n, rp, col, c, W, eps=1e-9, return_stats=True)

    def huge(F, Vs, s):
        return np.full(len(Vs), 40.0)

    R, st = componentwise_solve(n, rp, col, c, W, eps=1e-9, return_stats=True, warm_fn=huge)
    scc = st["accepted"] >= 0
    assert (st["accepted"][scc] == 0).all()
    np.testing.assert_array_equal(st["iters"], st0["iters"])
    np.testing.assert_allclose(R, R0, rtol=1e-13)


def test_features_on_a_cycle():
    # directed 5-cycle with W = 1: every vertex has in/out-degree 1, no
    # boundary mass, one step gives 1 + c
    n = 5
    rp = np.arange(n + 1)
    col = (np.arange(n) + 1) % n
    c = 0.85
    seen = {}

    def grab(F, Vs, s):
        seen["F"] = F.copy()
        seen["s"] = s.copy()
        return np.zeros(len(Vs))

    componentwise_solve(n, rp, col, c, np.ones(n), eps=1e-8, warm_fn=grab)
    F = seen["F"]
    np.testing.assert_allclose(F[:, 0], math.log(2.0))
    np.testing.assert_allclose(F[:, 1], math.log(2.0))
    np.testing.assert_allclose(F[:, 2], 0.0)
    np.testing.assert_allclose(F[:, 3], math.log1p(1.0 + c))
    np.testing.assert_allclose(seen["s"], 1.0)


def test_small_config_warm_start():
    g = small_plain(seed=1)
    c = 0.85
    W = np.ones(g.n)
    ref, st0 = componentwise_solve(g.n, g.row_ptr, g.col, c, W, eps=1e-12, return_stats=True)
    R, st = componentwise_solve(g.n, g.row_ptr, g.col, c, W, eps=1e-10, return_stats=True,
                                warm=ws.init_params(0))
    assert np.abs(R - ref).sum() / ref.sum() < 1e-10


def test_bf16_rounding():
    # 1 + 2^-8 is a tie between 1 and 1 + 2^-7: nearest even keeps 1
    assert ws.to_bf16(1.0 + 2.0 ** -8) == 1.0
    assert ws.to_bf16(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6
    assert ws.to_bf16(-3.0) == -3.0
    x = np.random.default_rng(2).normal(size=1000)
    assert np.all(np.abs(ws.to_bf16(x) - x) <= 2.0 ** -8 * np.abs(x))


def test_bf16_bound_covers_emulated_rounding():
    rng = np.random.default_rng(7)
    th = ws.init_params(9) * 3.0
    X = np.column_stack([rng.uniform(0, 7, 500), rng.uniform(0, 7, 500), rng.uniform(0, 3, 500),
                         rng.uniform(0, 4, 500)])
    err = np.abs(ws.forward_bf16(th, X) - ws.forward(th, X))
    bound = ws.forward_bf16_bound(th, X)
    assert np.all(err <= bound)
    assert err.max() > 0.0


# ------------------------- the geometric tail estimate after a starting guess

def test_tail_with_useless_guess_is_the_plain_start_tail():
    """A guess that always falls back leaves the plain series, so the tail
    rule must act exactly as without a guess (its rho starts from W'_C)."""
    n, rp, col = _graph_with_sccs(15)
    c = 0.85
    W = np.random.default_rng(15).uniform(0.5, 1.5, n)
    R0, st0 = componentwise_solve(n, rp, col, c, W, eps=1e-9, tail=True, return_stats=True)

    def huge(F, Vs, s):
        return np.full(len(Vs), 40.0)

    R, st = componentwise_solve(n, rp, col, c, W, eps=1e-9, tail=True, return_stats=True, warm_fn=huge)
    scc = st["accepted"] >= 0
    assert (st["accepted"][scc] == 0).all()
    np.testing.assert_array_equal(st["iters"], st0["iters"])
    np.testing.assert_allclose(R, R0, rtol=1e-13)


@pytest.mark.parametrize("m", [4, 7])
def test_tail_with_kept_guess_on_a_cycle(m):
    """Bare cycle, W = 1, guess R_0 = 0.5/(1-c) on every vertex: r_0 = 0.5
    and r_k = 0.5 c^k, all uniform.  The guess is kept (0.5 < c), no ratio
    exists before the second new term, and there the estimate is exact: two
    new terms, R = 1/(1-c)."""
    rp = np.arange(m + 1)
    col = (np.arange(m) + 1) % m
    c = 0.85

    def half(F, Vs, s):
        return np.log(0.5 / (1.0 - c) / s)

    R, st = componentwise_solve(m, rp, col, c, np.ones(m), eps=1e-12, tail=True, return_stats=True, warm_fn=half)
    assert st["accepted"].max() == 1
    assert st["iters"].max() == 2
    np.testing.assert_allclose(R, 1.0 / (1.0 - c), rtol=1e-14)


@pytest.mark.parametrize("seed", [16, 17])
def test_tail_with_noisy_guess_meets_the_bound(seed):
    """Guesses within 5% of the answer (mostly kept): the result is within
    eps of the dense solve, no SCC takes more terms than without the rule,
    and each SCC's residual is at most c times its last-term norm (equal for
    a tail stop: the rule's residual identity)."""
    from graphgen import scc_blocks

    g = scc_blocks(seed, nblocks=30, max_size=40)
    n, rp, col = g.n, g.row_ptr, g.col
    c = 0.85
    eps = 1e-8
    W = np.random.default_rng(seed).uniform(0.5, 1.5, n)
    exact = pagerank_dense(n, rp, col, c, W)
    noise = np.random.default_rng(seed + 1).uniform(-0.05, 0.05, n)

    def noisy(F, Vs, s):
        return np.log(exact[Vs] * (1.0 + noise[Vs]) / s)

    R, st = componentwise_solve(n, rp, col, c, W, eps=eps, tail=True, return_stats=True, warm_fn=noisy)
    _, st0 = componentwise_solve(n, rp, col, c, W, eps=eps, return_stats=True, warm_fn=noisy)
    scc = st["accepted"] >= 0
    assert (st["accepted"][scc] == 1).sum() > scc.sum() // 2
    assert np.abs(R - exact).sum() / exact.sum() <= eps
    assert np.all(st["iters"] <= st0["iters"]) and st["iters"].sum() < st0["iters"].sum()
    from oracle.partition import partition_theorem
    from oracle.pagerank import transition_T_csr

    part = partition_theorem(n, rp, col)
    AT = transition_T_csr(n, rp, col).toarray()
    n_eq = 0
    for C_ in np.nonzero(scc)[0]:
        v = np.nonzero(part["comp"] == C_)[0]
        res = np.abs(st["wprime"][v] - R[v] + c * AT[np.ix_(v, v)] @ R[v]).sum()
        slack = 1e-14 * len(v) * np.abs(R[v]).max()  # rounding of the residual itself
        assert res <= c * st["last"][C_] * (1 + 1e-8) + slack
        n_eq += bool(abs(res - c * st["last"][C_]) <= slack)
    assert n_eq > 0  # some SCCs did stop on the estimate


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_grad_bf16_bound_covers_emulated_rounding(seed):
    """The entrywise first-order gradient bound covers the emulated
    BF16-operand gradient (same rounding decisions as a BF16 kernel), and it
    catches planted mistakes: W2's gradient transposed, or b2's with the
    wrong sign."""
    rng = np.random.default_rng(seed)
    n = 2000
    th = ws.init_params(seed + 10)
    X = np.column_stack([rng.uniform(0, 7, n), rng.uniform(0, 7, n), rng.uniform(0, 3, n),
                         rng.uniform(0.3, 4, n)])
    t = 0.5 * X[:, 3] + rng.normal(0, 0.3, n)
    _, g = ws.loss_and_grad(th, X, t)
    _, ge = ws.loss_and_grad_bf16(th, X, t)
    bound, mag = ws.grad_bf16_bound(th, X, t)
    assert np.all(np.abs(ge - g) <= bound * (1 + 1e-6) + 1e-15)
    assert np.all(bound >= 0) and np.all(mag >= np.abs(g) * (1 - 1e-12))
    w2 = g.copy()
    w2[320:4416] = g[320:4416].reshape(64, 64).T.ravel()
    assert np.any(np.abs(w2 - g) > bound)
    b2 = g.copy()
    b2[4416:4480] *= -1.0
    assert np.any(np.abs(b2 - g) > bound)
