"""GPU parity on the Barabasi-Albert workload (about one and about five edges
per vertex), through the C ABI, against the oracle."""
import sys

import numpy as np
import pytest

from graphgen import barabasi_albert
from oracle.componentwise import componentwise_solve
from oracle.pagerank import pagerank_power_series

pytestmark = pytest.mark.gpu
C = 0.85


@pytest.fixture(scope="module")
def prm():
    import torch

    import paper_1609_09068_amd as pr

    assert torch.cuda.is_available()
    return pr, torch


@pytest.mark.parametrize("m,n", [(2, 60_000), (24, 20_000)])
@pytest.mark.parametrize("method", [0, 1])
def test_ba_fp64_matches_oracle(prm, m, n, method):
    pr, torch = prm
    g = barabasi_albert(n, m, seed=77 + m)
    print("[gpu-case] ba m", m, "n", n, "method", method, file=sys.stderr, flush=True)
    part = pr.pr_partition(g.row_ptr, g.col)
    lv = pr.pr_build_levels(part, g.row_ptr, g.col, build_plain=1)
    W = np.random.default_rng(m).uniform(0.5, 1.5, g.n)
    Wd = torch.tensor(W, device="cuda")
    R = torch.empty_like(Wd)
    rc, st = pr.pr_solve(lv, C, Wd, R, method=method, eps=1e-10, precision=1)
    assert rc == 0
    ref, _, _ = pagerank_power_series(g.n, g.row_ptr, g.col, C, W, eps=1e-14)
    err = np.abs(R.cpu().numpy() - ref).sum() / ref.sum()
    assert err <= 1e-10, err
    if method == 0:
        Ro = componentwise_solve(g.n, g.row_ptr, g.col, C, W, eps=1e-10)
        assert np.allclose(R.cpu().numpy(), Ro, rtol=1e-9, atol=0)
