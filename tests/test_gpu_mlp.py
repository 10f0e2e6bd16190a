"""The starting-guess network on the GPU against the float64 oracle.

Forward: the GPU rounds every matrix-product operand to bfloat16 and sums in
float32, so it is compared with the oracle's bfloat16-operand emulation (same
rounding decisions, float64 sums) and with the exact network within the
oracle's first-order rounding bound.  Gradients: bfloat16 operands in the
backward products as well, so the whole gradient vector is compared in
relative 2-norm (3e-2; the forward's relative rounding is 2^-8 per operand
and the backward chains three products).  Adam: the update is float32
arithmetic on the GPU's own gradient, compared with the oracle's update of the
same gradient.
"""
import os
import sys

import numpy as np
import pytest

from oracle import warmstart as ws

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu-case]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def prm():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1609_09068_amd as pr

    return pr, torch


def _features(rng, n):
    # ranges of the real features: log-degrees up to ~7, boundary and one-step terms up to ~4
    return np.column_stack([rng.uniform(0, 7, n), rng.uniform(0, 7, n), rng.uniform(0, 3, n),
                            rng.uniform(0.3, 4, n)]).astype(np.float32)


@pytest.mark.parametrize("n", [1, 15, 16, 64, 1037, 70001])
def test_forward_matches_oracle(prm, n):
    pr, torch = prm
    _say("mlp forward", n)
    rng = np.random.default_rng(n)
    th = (ws.init_params(n) * 2.0).astype(np.float32)
    net = pr.Mlp.create(1)
    net.set_params(th)
    np.testing.assert_array_equal(net.get_params(), th)
    X = _features(rng, n)
    y = net.predict(torch.tensor(X, device="cuda")).cpu().numpy().astype(np.float64)
    th64 = th.astype(np.float64)
    emu = ws.forward_bf16(th64, X.astype(np.float64))
    exact = ws.forward(th64, X.astype(np.float64))
    bound = ws.forward_bf16_bound(th64, X.astype(np.float64))
    assert np.all(np.abs(y - exact) <= bound + 1e-5)
    # against the same rounding decisions: only float32 sums and an occasional
    # one-ulp difference of a rounded activation remain
    assert np.max(np.abs(y - emu)) <= 0.02 * (1.0 + np.max(np.abs(emu)))
    assert np.sqrt(np.mean((y - emu) ** 2)) <= 2e-3 * (1.0 + np.sqrt(np.mean(emu ** 2)))


@pytest.mark.parametrize("n", [16, 999, 20000])
def test_gradient_matches_oracle(prm, n):
    pr, torch = prm
    _say("mlp grad", n)
    rng = np.random.default_rng(100 + n)
    th = ws.init_params(3).astype(np.float32)
    net = pr.Mlp.create(2)
    net.set_params(th)
    X = _features(rng, n)
    t = (0.5 * X[:, 3] + 0.2 * np.sin(X[:, 0]) + rng.normal(0, 0.1, n)).astype(np.float32)
    g, loss = net.grad(torch.tensor(X, device="cuda"), torch.tensor(t, device="cuda"))
    L, g_ref = ws.loss_and_grad(th.astype(np.float64), X.astype(np.float64), t.astype(np.float64))
    assert loss == pytest.approx(L, rel=2e-2)
    rel = np.linalg.norm(g - g_ref) / np.linalg.norm(g_ref)
    assert rel < 3e-2, rel
    # every block of the layout lands in the right place
    for name, lo, hi in [("W1", 0, 256), ("b1", 256, 320), ("W2", 320, 4416), ("b2", 4416, 4480),
                         ("W3", 4480, 4544), ("b3", 4544, 4545)]:
        r = np.linalg.norm(g[lo:hi] - g_ref[lo:hi]) / max(np.linalg.norm(g_ref[lo:hi]), 1e-12)
        assert r < 6e-2, (name, r)


@pytest.mark.parametrize("n", [16, 999, 20000])
def test_gradient_entry_by_entry(prm, n):
    """Every gradient entry against the oracle: within the entrywise
    first-order BF16 rounding bound of the exact gradient (plus float32
    accumulation over at most 2^10 sequential partials, 2^-14 of the
    magnitude gradient); its distance to the oracle's emulation of the same
    BF16 rounding decisions is printed (an operand whose float32 value sits
    next to a rounding boundary may round the other way on the GPU, which
    moves an entry by up to 2^-8 of that row's term)."""
    pr, torch = prm
    _say("mlp grad entrywise", n)
    rng = np.random.default_rng(300 + n)
    th = ws.init_params(7).astype(np.float32)
    net = pr.Mlp.create(2)
    net.set_params(th)
    X = _features(rng, n)
    t = (0.5 * X[:, 3] + 0.2 * np.sin(X[:, 0]) + rng.normal(0, 0.1, n)).astype(np.float32)
    g, _ = net.grad(torch.tensor(X, device="cuda"), torch.tensor(t, device="cuda"))
    g = g.astype(np.float64)
    th64, X64, t64 = th.astype(np.float64), X.astype(np.float64), t.astype(np.float64)
    _, g_ref = ws.loss_and_grad(th64, X64, t64)
    _, g_emu = ws.loss_and_grad_bf16(th64, X64, t64)
    bound, mag = ws.grad_bf16_bound(th64, X64, t64)
    tol = bound + 2.0 ** -14 * mag + 1e-12
    for name, lo, hi in [("W1", 0, 256), ("b1", 256, 320), ("W2", 320, 4416), ("b2", 4416, 4480),
                         ("W3", 4480, 4544), ("b3", 4544, 4545)]:
        d_ex = np.abs(g[lo:hi] - g_ref[lo:hi])
        d_em = np.abs(g[lo:hi] - g_emu[lo:hi])
        e_em = np.abs(g_emu[lo:hi] - g_ref[lo:hi])
        _say(f"  {name}: |gpu-exact|/bound max {np.max(d_ex / tol[lo:hi]):.3e}, |gpu-emu|/mag max "
             f"{np.max(d_em / mag[lo:hi]):.3e}, |emu-exact|/mag max {np.max(e_em / mag[lo:hi]):.3e}")
        assert np.all(d_ex <= tol[lo:hi]), name


def test_gradient_is_deterministic(prm):
    pr, torch = prm
    rng = np.random.default_rng(5)
    net = pr.Mlp.create(3)
    X = torch.tensor(_features(rng, 5000), device="cuda")
    t = torch.tensor(rng.normal(size=5000).astype(np.float32), device="cuda")
    g1, l1 = net.grad(X, t)
    g2, l2 = net.grad(X, t)
    np.testing.assert_array_equal(g1, g2)
    assert l1 == l2


def test_adam_step_matches_oracle(prm):
    pr, torch = prm
    rng = np.random.default_rng(6)
    th = ws.init_params(4).astype(np.float32)
    net = pr.Mlp.create(4)
    net.set_params(th)
    X = torch.tensor(_features(rng, 3000), device="cuda")
    t = torch.tensor(rng.normal(size=3000).astype(np.float32), device="cuda")
    opt = ws.Adam(ws.N_PARAMS, lr=1e-2)
    cur = th.astype(np.float64)
    for step in range(3):
        g, _ = net.grad(X, t)
        net.train_step(X, t, 1e-2)
        cur = opt.step(cur, g.astype(np.float64))
        np.testing.assert_allclose(net.get_params(), cur, rtol=2e-5, atol=2e-6)
        # continue the oracle from the GPU's weights (float32 rounding of each step)
        cur = net.get_params().astype(np.float64)


def test_training_fits_a_smooth_target(prm):
    pr, torch = prm
    rng = np.random.default_rng(8)
    X = _features(rng, 40000)
    t = (np.log1p(X[:, 3]) + 0.1 * X[:, 1] - 0.05 * X[:, 0]).astype(np.float32)
    Xd, td = torch.tensor(X, device="cuda"), torch.tensor(t, device="cuda")
    net = pr.Mlp.create(9)
    first = None
    for step in range(300):
        sel = torch.randint(0, 40000, (2048,), device="cuda", generator=None)
        loss = net.train_step(Xd[sel].contiguous(), td[sel].contiguous(), 3e-3)
        first = loss if first is None else first
    _, final = net.grad(Xd, td)
    assert final < 0.05 * first, (first, final)


def test_save_load_roundtrip(prm, tmp_path):
    pr, torch = prm
    net = pr.Mlp.create(11)
    rng = np.random.default_rng(1)
    X = torch.tensor(_features(rng, 500), device="cuda")
    t = torch.tensor(rng.normal(size=500).astype(np.float32), device="cuda")
    net.train_step(X, t, 1e-3)
    path = tmp_path / "net.bin"
    net.save(path)
    other = pr.Mlp.load_file(path)
    np.testing.assert_array_equal(other.get_params(), net.get_params())
    # the Adam state travels too: the next steps agree
    net.train_step(X, t, 1e-3)
    other.train_step(X, t, 1e-3)
    np.testing.assert_array_equal(other.get_params(), net.get_params())
    bad = tmp_path / "bad.bin"
    bad.write_bytes(b"not a network")
    with pytest.raises(pr.PRError):
        pr.Mlp.load_file(bad)


def test_error_paths(prm):
    pr, torch = prm
    net = pr.Mlp.create(12)
    X = torch.zeros((10, 4), dtype=torch.float32, device="cuda")
    t = torch.zeros(10, dtype=torch.float32, device="cuda")
    with pytest.raises(pr.PRError):
        net.train_step(X, t, -1.0)
    theta = np.zeros(4545, dtype=np.float32)
    theta[7] = np.nan
    with pytest.raises(pr.PRError):
        net.set_params(theta)
    dead = pr.Mlp(net.handle)
    net.free()
    with pytest.raises(pr.PRError):
        dead.get_params()
    dead.handle = None
