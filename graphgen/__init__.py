"""Seeded synthetic directed graphs shaped like the paper's workloads.

This module only draws graphs (CSR arrays); it holds none of the PageRank or
partition arithmetic.  Both the oracle and the GPU path consume its output.
"""
from .generators import (  # noqa: F401
    Graph,
    barabasi_albert,
    csr_from_edges,
    random_digraph,
    scc_blocks,
    small_plain,
    web_like,
    config_graph,
    CONFIGS,
)
