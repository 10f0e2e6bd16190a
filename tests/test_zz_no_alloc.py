"""The allocation-free gradient entry point (pr_mlp_grad_noalloc) against
pr_mlp_grad: same kernels, partials in the library's static device array
instead of the network's own buffer, so the gradient and loss agree bit for
bit; two calls in a row, the second on a smaller batch (the array keeps the
first call's partials, which the second must not read)."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu-case]", *a, file=sys.stderr, flush=True)


def test_noalloc_gradient_matches_allocating_entry_point():
    import torch

    import paper_1609_09068_amd as pr

    assert torch.cuda.is_available()
    net = pr.Mlp.create(seed=17)
    rng = np.random.default_rng(5)
    sizes = (200_003, 1_001)  # the second smaller: fewer wavefront partials than the first
    for n in sizes:
        _say("noalloc grad n =", n)
        X = torch.tensor(rng.normal(size=(n, 4)).astype(np.float32), device="cuda")
        t = torch.tensor(rng.normal(size=n).astype(np.float32), device="cuda")
        g_na, l_na = net.grad_noalloc(X, t)
        g_ref, l_ref = net.grad(X, t)
        assert np.all(np.isfinite(g_ref)) and np.abs(g_ref).sum() > 0
        assert np.array_equal(g_na, g_ref), float(np.abs(g_na - g_ref).max())
        assert l_na == l_ref
    # bad arguments are refused before any device work
    with pytest.raises(pr.PRError):
        net.grad_noalloc(X[:0], t[:0])
    net.free()
