"""Oracle for componentwise PageRank (Engstrom & Silvestrov, arXiv 1609.09068).

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously-correct CPU
implementation (numpy / scipy, float64) of what the GPU path computes.  It is
imported only by the tests, by the smoke check of the entry module and by the
benchmark's CPU-baseline leg; the product path never calls it.  It shares no
code with the HIP library: no kernels, headers, helpers or tables.

Modules
-------
pagerank      Def. 3.4 / 3.5 (dense solve, eigenvector route), the power
              series of Sec. 4.3.2 with both stop rules.
partition     the SCC/CAC partition of Sec. 4.1: the merge process of
              Theorem 3.1 (primary) and the modified Tarjan DFS (second,
              independent route), canonical component numbering.
componentwise the level-by-level solve of Sec. 4.3 (eq. PR:levels, the CAC
              sweep of Sec. 4.3.1, the power series per SCC).
warmstart     per-vertex features and the 4-64-64-1 GELU network used for the
              learned starting guess (forward, backward, Adam) in float64.
gauss_seidel  block Gauss-Seidel sweeps inside one SCC (the alternative to
              the series that Sec. 4.3.2 names), with its residual certificate.
"""
