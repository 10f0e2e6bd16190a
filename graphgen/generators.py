"""Seeded graph generators.

The paper measures on the Google 2002 web graph and on a Barabasi-Albert graph
(Sec. 5.1).  Neither is available here, so these generators plant the shape
that matters for the componentwise method instead: a block of strongly
connected vertices (a giant SCC for the web-like recipe), many small SCCs, many
acyclic tree/chain regions that become CACs, dangling vertices, heavy-tailed
out-degrees and a DAG of blocks several tens of levels deep (Sec. 5.1 and the
statistics quoted for the web graph there).

A graph is returned as CSR over out-edges: ``row_ptr`` int64[n+1] and
``col`` int32[m]; rows are sorted, there are no self-loops and no duplicate
edges unless a generator is explicitly asked for them.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Graph:
    n: int
    row_ptr: np.ndarray  # int64[n+1]
    col: np.ndarray  # int32[m]
    meta: dict = field(default_factory=dict)

    @property
    def m(self) -> int:
        return int(self.row_ptr[-1])

    def edges(self):
        """(src, dst) int64 arrays in CSR order."""
        src = np.repeat(np.arange(self.n, dtype=np.int64), np.diff(self.row_ptr))
        return src, self.col.astype(np.int64)


def csr_from_edges(n: int, src, dst, *, dedupe: bool = True, drop_loops: bool = True,
                   sort_rows: bool = True) -> Graph:
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    if drop_loops:
        keep = src != dst
        src, dst = src[keep], dst[keep]
    if sort_rows or dedupe:
        key = src * n + dst
        key = np.unique(key) if dedupe else np.sort(key, kind="stable")
        src = key // n
        dst = key - src * n
    counts = np.bincount(src, minlength=n)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    return Graph(n, row_ptr, dst.astype(np.int32))


def random_digraph(n: int, m: int, seed: int, *, loops: bool = False,
                   duplicates: bool = False) -> Graph:
    """Uniform random digraph (tests).  With ``loops``/``duplicates`` the
    self-loops and repeated edges are kept, to exercise the input rules."""
    rng = np.random.default_rng(seed)
    src = rng.integers(0, n, size=m)
    dst = rng.integers(0, n, size=m)
    if duplicates:
        order = np.argsort(src, kind="stable")
        src, dst = src[order], dst[order]
        counts = np.bincount(src, minlength=n)
        row_ptr = np.zeros(n + 1, dtype=np.int64)
        np.cumsum(counts, out=row_ptr[1:])
        if not loops:
            keep = src != dst
            return csr_from_edges(n, src[keep], dst[keep], dedupe=False, drop_loops=False)
        return Graph(n, row_ptr, dst.astype(np.int32))
    return csr_from_edges(n, src, dst, dedupe=True, drop_loops=not loops)


# ---------------------------------------------------------------------------
# helpers
# ---------------------------------------------------------------------------

def scc_blocks(seed: int, nblocks: int = 30, min_size: int = 2, max_size: int = 24, tails: int = 20) -> "Graph":
    """SCC blocks of min_size..max_size vertices (a Hamiltonian cycle plus as
    many random chords), two forward links per block between random pairs of
    blocks (so the blocks sit on several levels), and `tails` one-vertex
    sinks fed from random block vertices.  Many small SCCs: the case of the
    direct small-SCC solve."""
    rng = np.random.default_rng(seed)
    sizes = rng.integers(min_size, max_size + 1, nblocks)
    starts = np.concatenate([[0], np.cumsum(sizes)])
    src, dst = [], []
    for b in range(nblocks):
        v = np.arange(starts[b], starts[b + 1])
        src += list(v)
        dst += list(np.roll(v, -1))
        for _ in range(len(v)):
            src.append(rng.choice(v))
            dst.append(rng.choice(v))
    n0 = int(starts[-1])
    for _ in range(2 * nblocks):
        a, b = sorted(rng.choice(nblocks, 2, replace=False))
        src.append(rng.integers(starts[a], starts[a + 1]))
        dst.append(rng.integers(starts[b], starts[b + 1]))
    for t in range(n0, n0 + tails):
        src.append(rng.integers(0, n0))
        dst.append(t)
    return csr_from_edges(n0 + tails, np.array(src), np.array(dst))


def barabasi_albert(n: int, m: int, seed: int, *, m0: int = 20, seed_degree: float = 5.0,
                    batch_frac: float = 0.01, log=None) -> "Graph":
    """Barabasi-Albert growth, then each vertex keeps ceil(log2 d) of its d
    incident edges as out-edges (the recipe of the paper's B-A experiments,
    Sec. 5.1 and the B-A generation subsection).

    Seed: m0 vertices with uniformly random undirected edges of mean degree
    seed_degree.  Growth: every new vertex joins m distinct existing vertices
    drawn with probability proportional to their degree.  Vertices are added
    in batches of batch_frac of the current size that all draw from the
    degrees at the start of the batch (the exact one-at-a-time process, up to
    that lag).  Thinning: vertex i that created E_i edges (m for a grown
    vertex, its seed edges for a seed vertex) keeps ceil(log2 E_i) of its
    incident edges, chosen uniformly among all of them, as edges i ->
    neighbour; an edge kept from both ends becomes a 2-cycle.  With m = 2 the
    result has about one edge per vertex, with m = 24 about five.  (The
    paper's text leaves open which edges count as originating from a vertex;
    this reading gives its B-A statistics' shape: about one edge per vertex,
    a large CAC, many 2-vertex SCCs.)"""
    rng = np.random.default_rng(seed)
    n_seed_edges = int(round(m0 * seed_degree / 2))
    a = rng.integers(0, m0, n_seed_edges)
    b = rng.integers(0, m0, n_seed_edges)
    keep = a != b
    eu, ev = [a[keep]], [b[keep]]
    ends = np.concatenate([a[keep], b[keep]])  # every edge end once: degree-proportional draws
    pool = [ends]
    pool_len = len(ends)
    v = m0
    while v < n:
        bs = max(1, min(n - v, int(batch_frac * v)))
        flat = np.concatenate(pool) if len(pool) > 1 else pool[0]
        pool = [flat]
        new = np.arange(v, v + bs)
        t = flat[rng.integers(0, pool_len, (bs, m))]
        # distinct targets per vertex: redraw duplicates uniformly among the
        # older vertices (rare once the graph has grown)
        t.sort(axis=1)
        dup = np.zeros_like(t, dtype=bool)
        dup[:, 1:] = t[:, 1:] == t[:, :-1]
        if dup.any():
            t[dup] = rng.integers(0, v, int(dup.sum()))
        src = np.repeat(new, m)
        dst = t.ravel()
        eu.append(src)
        ev.append(dst)
        pool.append(np.concatenate([src, dst]))
        pool_len += 2 * len(src)
        v += bs
    eu = np.concatenate(eu)
    ev = np.concatenate(ev)
    if log:
        log(f"barabasi_albert: grown {n} vertices, {len(eu)} undirected edges")
    created = np.bincount(eu, minlength=n)
    # incident edges per vertex (both ends), then ceil(log2 E_i) kept per vertex
    ends_v = np.concatenate([eu, ev])
    other = np.concatenate([ev, eu])
    order = np.lexsort((rng.random(len(ends_v)), ends_v))  # random order within each vertex
    ends_v, other = ends_v[order], other[order]
    deg = np.bincount(ends_v, minlength=n)
    first = np.concatenate([[0], np.cumsum(deg)[:-1]])
    rank = np.arange(len(ends_v)) - first[ends_v]
    kept = np.minimum(np.ceil(np.log2(np.maximum(created, 1))).astype(np.int64), deg)
    sel = rank < kept[ends_v]
    g = csr_from_edges(n, ends_v[sel], other[sel])
    g.meta.update(dict(kind="barabasi_albert", m=m, m0=m0, seed=seed))
    return g


def _zipf_truncated(rng, size, a, dmax):
    k = np.arange(1, dmax + 1, dtype=np.float64)
    cdf = np.cumsum(k ** (-a))
    cdf /= cdf[-1]
    return np.searchsorted(cdf, rng.random(size), side="right").astype(np.int64) + 1


def _lognormal_sizes(rng, total, median, sigma, min_size):
    """Integer block sizes >= min_size whose sum is exactly ``total``."""
    if total <= 0:
        return np.zeros(0, dtype=np.int64)
    out = []
    acc = 0
    while acc < total:
        batch = max(16, int(1.3 * (total - acc) / max(median, 1)) + 16)
        s = np.maximum(min_size, np.rint(median * np.exp(sigma * rng.standard_normal(batch)))).astype(np.int64)
        out.append(s)
        acc += int(s.sum())
    sizes = np.concatenate(out)
    csum = np.cumsum(sizes)
    k = int(np.searchsorted(csum, total, side="left"))
    sizes = sizes[: k + 1].copy()
    over = int(sizes.sum() - total)
    sizes[-1] -= over
    if sizes[-1] < min_size:
        short = int(sizes[-1])
        sizes = sizes[:-1]
        if len(sizes) == 0:
            return np.array([total], dtype=np.int64)
        sizes[-1] += short
    return sizes


def _segment_ids(sizes):
    return np.repeat(np.arange(len(sizes), dtype=np.int64), sizes)


def _sample_in_ranges(rng, cum, lo, hi):
    """For each (lo, hi) vertex range draw one vertex with probability
    proportional to weight, where ``cum`` is the inclusive prefix sum of the
    weights over the layout order (cum[-1] is the total)."""
    base = np.where(lo > 0, cum[np.maximum(lo - 1, 0)], 0.0)
    top = cum[hi - 1]
    r = base + rng.random(len(lo)) * (top - base)
    # the same search with the queries in increasing order (numpy's binary
    # search then starts from the previous answer: ten times faster on
    # arrays larger than the caches); the result does not depend on the order
    order = np.argsort(r)
    v = np.empty(len(r), dtype=np.int64)
    v[order] = np.searchsorted(cum, r[order], side="right")
    return np.minimum(np.maximum(v, lo), hi - 1)


def _scaled_degrees(rng, n, m_target, a, dmax, mask, floor_deg):
    """Zipf(a) out-degree targets on [1, dmax] for vertices in ``mask``, scaled
    multiplicatively (with randomised rounding) so they sum to ~m_target."""
    raw = _zipf_truncated(rng, n, a, dmax).astype(np.float64)
    raw[~mask] = 0.0
    f = m_target / max(raw.sum(), 1.0)
    for _ in range(6):
        d = raw * f
        d = np.floor(d + rng.random(n)).astype(np.int64)
        d = np.clip(d, 0, dmax)
        d[mask] = np.maximum(d[mask], floor_deg[mask])
        s = d.sum()
        if s == 0:
            break
        if abs(s - m_target) <= 0.002 * m_target:
            break
        f *= m_target / s
    return d


# ---------------------------------------------------------------------------
# configuration 1: the small plain case
# ---------------------------------------------------------------------------

def small_plain(seed: int = 1, n: int = 10_000, n_scc_blocks: int = 200,
                scc_vertices: int = 7_000, cac_vertices: int = 3_000,
                n_dangling: int = 500, n_inter: int = 4_000, intra_deg: float = 6.0) -> Graph:
    """10k-vertex graph: 200 SCCs (Hamiltonian cycle plus random intra edges,
    average intra out-degree ~6), 3,000 vertices in random out-trees and
    chains of 2-50 vertices, 5% dangling vertices, 4,000 edges between blocks
    that follow a random topological order of the blocks."""
    rng = np.random.default_rng(seed)
    assert scc_vertices + cac_vertices == n
    # SCC sizes: U{5..100}, rescaled to the available vertex budget with
    # largest-remainder rounding (every block keeps at least 5 vertices).
    raw = rng.integers(5, 101, size=n_scc_blocks).astype(np.float64)
    share = raw / raw.sum() * scc_vertices
    base = np.maximum(5, np.floor(share).astype(np.int64))
    rem = scc_vertices - int(base.sum())
    if rem > 0:
        order = np.argsort(-(share - np.floor(share)), kind="stable")
        base[order[:rem]] += 1
    elif rem < 0:
        order = np.argsort(-base, kind="stable")
        i = 0
        while rem < 0:
            j = order[i % len(order)]
            if base[j] > 5:
                base[j] -= 1
                rem += 1
            i += 1
    scc_sizes = base
    cac_sizes = []
    left = cac_vertices
    while left > 0:
        s = int(rng.integers(2, 51))
        s = min(s, left)
        if left - s == 1:
            s += 1
        cac_sizes.append(s)
        left -= s
    cac_sizes = np.array(cac_sizes, dtype=np.int64)
    cac_kind = rng.integers(0, 2, size=len(cac_sizes))  # 0 tree, 1 chain

    # blocks: SCC blocks then CAC blocks, shuffled into a random topological order
    kinds = np.concatenate([np.zeros(len(scc_sizes), np.int64), 1 + cac_kind])
    sizes = np.concatenate([scc_sizes, cac_sizes])
    order = rng.permutation(len(sizes))
    kinds, sizes = kinds[order], sizes[order]
    starts = np.zeros(len(sizes) + 1, dtype=np.int64)
    np.cumsum(sizes, out=starts[1:])
    blk = _segment_ids(sizes)
    local = np.arange(n, dtype=np.int64) - starts[blk]

    src_l, dst_l = [], []
    leafish = np.zeros(n, dtype=bool)
    for b in range(len(sizes)):
        s0, s = int(starts[b]), int(sizes[b])
        if kinds[b] == 0:
            cyc = s0 + rng.permutation(s)
            src_l.append(cyc)
            dst_l.append(np.roll(cyc, -1))
            extra = int(round((intra_deg - 1.0) * s))
            extra = min(extra, s * (s - 1) - s)
            if extra > 0:
                es = s0 + rng.integers(0, s, size=3 * extra)
                ed = s0 + rng.integers(0, s, size=3 * extra)
                keep = es != ed
                es, ed = es[keep][:extra], ed[keep][:extra]
                src_l.append(es)
                dst_l.append(ed)
        elif kinds[b] == 1:  # random recursive out-tree
            child = np.arange(1, s, dtype=np.int64)
            parent = np.floor(rng.random(s - 1) * child).astype(np.int64)
            src_l.append(s0 + parent)
            dst_l.append(s0 + child)
            has_child = np.zeros(s, dtype=bool)
            has_child[parent] = True
            leafish[s0 + np.nonzero(~has_child)[0]] = True
        else:  # chain
            src_l.append(s0 + np.arange(s - 1))
            dst_l.append(s0 + np.arange(1, s))
            leafish[s0 + s - 1] = True
    cand = np.nonzero(leafish)[0]
    dangling = np.zeros(n, dtype=bool)
    dangling[rng.choice(cand, size=min(n_dangling, len(cand)), replace=False)] = True

    # inter-block edges: from a block to a later block in the topological order
    src_ok = np.nonzero(~dangling & (blk < len(sizes) - 1))[0]
    es = rng.choice(src_ok, size=n_inter)
    lo = starts[blk[es] + 1]
    ed = lo + np.floor(rng.random(n_inter) * (n - lo)).astype(np.int64)
    src_l.append(es)
    dst_l.append(ed)
    src = np.concatenate(src_l)
    dst = np.concatenate(dst_l)
    perm = rng.permutation(n)
    g = csr_from_edges(n, perm[src], perm[dst])
    g.meta = {"recipe": "small_plain", "seed": seed, "n_scc_blocks": int(n_scc_blocks),
              "n_cac_blocks": int(len(cac_sizes)), "dangling_planted": int(dangling.sum())}
    return g


# ---------------------------------------------------------------------------
# web-like recipe (configurations 2-5)
# ---------------------------------------------------------------------------

def web_like(n: int, m: int, seed: int, *, giant_frac: float = 0.4, cac_frac: float = 0.3,
             dangling_frac: float = 0.10, zipf_a: float = 2.1, dmax: int = 1000,
             n_levels: int = 60, scc_median: float = 12.0, scc_sigma: float = 1.0,
             cac_median: float = 8.0, cac_sigma: float = 1.0, intra_frac: float = 0.75,
             scc_tail_max: int | None = None, level_width: str = "uniform",
             p_next_level: float = 0.5, log=None) -> Graph:
    """Web-like graph built from planted blocks placed on ``n_levels`` planned
    levels.  Edges between blocks only go from a higher planned level to a
    lower one, so the planted SCC blocks are exactly the SCCs and the tree and
    chain blocks are acyclic.  Out-degrees follow a truncated Zipf law scaled
    to ~m edges; edge targets are drawn proportionally to a per-vertex Zipf
    "fitness", so in-degrees are heavy-tailed as well.  ``log`` (optional)
    receives a line as each phase ends."""
    say = log or (lambda *_: None)
    rng = np.random.default_rng(seed)
    n_giant = int(round(giant_frac * n))
    n_cac = int(round(cac_frac * n))
    n_small = n - n_giant - n_cac
    tail = []
    if scc_tail_max:
        s = int(scc_tail_max)
        while s >= 1000 and sum(tail) + s < n_small // 4:
            tail.append(s)
            s //= 2
    small_sizes = _lognormal_sizes(rng, n_small - sum(tail), scc_median, scc_sigma, 2)
    small_sizes = np.concatenate([np.array(tail, dtype=np.int64), small_sizes])
    cac_sizes = _lognormal_sizes(rng, n_cac, cac_median, cac_sigma, 1)
    # kinds: 0 giant SCC, 1 small SCC, 2 out-tree, 3 chain, 4 singleton
    cac_kind = np.where(cac_sizes == 1, 4, 2 + rng.integers(0, 2, size=len(cac_sizes)))
    kinds = np.concatenate([np.zeros(1 if n_giant > 0 else 0, np.int64),
                            np.ones(len(small_sizes), np.int64), cac_kind])
    sizes = np.concatenate([np.array([n_giant] if n_giant > 0 else [], np.int64), small_sizes, cac_sizes])
    nb = len(sizes)
    # planned levels
    if level_width == "pareto":
        w = rng.pareto(1.2, size=n_levels) + 0.05
    else:
        w = np.ones(n_levels)
    lvl = rng.choice(n_levels, size=nb, p=w / w.sum())
    if n_giant > 0:
        lvl[0] = n_levels // 2
    # compress empty levels away
    used = np.unique(lvl)
    lvl = np.searchsorted(used, lvl)
    nl = len(used)
    order = np.lexsort((rng.random(nb), -lvl))
    kinds, sizes, lvl = kinds[order], sizes[order], lvl[order]
    starts = np.zeros(nb + 1, dtype=np.int64)
    np.cumsum(sizes, out=starts[1:])
    blk = _segment_ids(sizes)
    vlvl = lvl[blk]
    vkind = kinds[blk]
    vstart = starts[blk]
    vsize = sizes[blk]
    local = np.arange(n, dtype=np.int64) - vstart
    # level vertex ranges (levels are laid out in descending order)
    lev_lo = np.full(nl, n, dtype=np.int64)
    lev_hi = np.zeros(nl, dtype=np.int64)
    np.minimum.at(lev_lo, vlvl, np.arange(n))
    np.maximum.at(lev_hi, vlvl, np.arange(n) + 1)

    is_scc = vkind <= 1
    say(f"generator: {nb} blocks on {nl} levels planned")
    # --- intra edges -------------------------------------------------------
    # SCC blocks: one random Hamiltonian cycle each
    scc_v = np.nonzero(is_scc)[0]
    key = blk[scc_v] * 2.0 + rng.random(len(scc_v))  # shuffle inside each block
    cyc = scc_v[np.argsort(key, kind="stable")]
    cb = blk[cyc]
    nxt = np.empty_like(cyc)
    nxt[:-1] = cyc[1:]
    nxt[-1] = cyc[0]
    last_of_block = np.ones(len(cyc), dtype=bool)
    last_of_block[:-1] = cb[1:] != cb[:-1]
    first_pos = np.searchsorted(cb, cb, side="left")
    nxt[last_of_block] = cyc[first_pos[last_of_block]]
    cyc_src, cyc_dst = cyc, nxt
    # trees: random recursive out-trees; chains: local i -> i+1
    tree_v = np.nonzero((vkind == 2) & (local > 0))[0]
    tpar = vstart[tree_v] + np.floor(rng.random(len(tree_v)) * local[tree_v]).astype(np.int64)
    chain_v = np.nonzero((vkind == 3) & (local > 0))[0]
    cpar = chain_v - 1
    cac_src = np.concatenate([tpar, cpar])
    cac_dst = np.concatenate([tree_v, chain_v])
    children = np.bincount(cac_src, minlength=n)

    say("generator: block-internal edges drawn")
    # --- degrees -----------------------------------------------------------
    leaf = (~is_scc) & (children == 0)
    n_dang = int(round(dangling_frac * n))
    leaves = np.nonzero(leaf)[0]
    dang = np.zeros(n, dtype=bool)
    if n_dang > 0:
        pick = rng.choice(leaves, size=min(n_dang, len(leaves)), replace=False)
        dang[pick] = True
    active = ~dang
    floor_deg = np.where(is_scc, 1, children).astype(np.int64)
    # ask for ~12% more edges than m: duplicates and edges below the lowest
    # planned level are lost, the surplus is trimmed at the end
    deg = _scaled_degrees(rng, n, int(1.12 * m), zipf_a, dmax, active, floor_deg)
    deg[dang] = 0
    fitness = _zipf_truncated(rng, n, zipf_a, dmax).astype(np.float64)
    cum = np.cumsum(fitness)

    # SCC vertices: ~intra_frac of the degree stays in the block
    scc_intra = np.zeros(n, dtype=np.int64)
    scc_intra[is_scc] = np.maximum(1, np.rint(intra_frac * deg[is_scc])).astype(np.int64)
    scc_intra = np.minimum(scc_intra, np.maximum(vsize - 1, 1) * is_scc)
    extra_intra = np.maximum(scc_intra - 1, 0)
    inter = np.where(is_scc, deg - scc_intra, np.maximum(deg - children, 0))
    inter[vlvl == 0] = 0  # nothing below the lowest planned level

    es = np.repeat(np.arange(n, dtype=np.int64), extra_intra)
    ed = _sample_in_ranges(rng, cum, vstart[es], vstart[es] + vsize[es])
    keep = es != ed
    es, ed = es[keep], ed[keep]

    isrc = np.repeat(np.arange(n, dtype=np.int64), inter)
    sl = vlvl[isrc]
    tgt_lvl = np.where(rng.random(len(isrc)) < p_next_level, sl - 1,
                       np.floor(rng.random(len(isrc)) * sl).astype(np.int64))
    idst = _sample_in_ranges(rng, cum, lev_lo[tgt_lvl], lev_hi[tgt_lvl])

    # structural edges (cycles, trees, chains) first so that de-duplication
    # keeps them; then trim random non-structural edges down to ~m
    n_struct = len(cyc_src) + len(cac_src)
    src = np.concatenate([cyc_src, cac_src, es, isrc])
    dst = np.concatenate([cyc_dst, cac_dst, ed, idst])
    key = src * n + dst
    say(f"generator: {len(key)} candidate edges drawn")
    _, first = np.unique(key, return_index=True)
    say("generator: duplicates removed")
    structural = first < n_struct
    excess = len(first) - m
    if excess > 0:
        cand = np.nonzero(~structural)[0]
        drop = rng.choice(cand, size=min(excess, len(cand)), replace=False)
        keepm = np.ones(len(first), dtype=bool)
        keepm[drop] = False
        first = first[keepm]
    src, dst = src[first], dst[first]
    perm = rng.permutation(n)
    g = csr_from_edges(n, perm[src], perm[dst])
    g.meta = {
        "recipe": "web_like", "seed": seed, "n_target": n, "m_target": m,
        "giant_planted": n_giant, "small_scc_blocks": int(len(small_sizes)),
        "cac_blocks": int(len(cac_sizes)), "planned_levels": int(nl),
        "dangling_planted": int(dang.sum()), "zipf_a": zipf_a, "dmax": dmax,
    }
    return g


# ---------------------------------------------------------------------------
# named configurations
# ---------------------------------------------------------------------------

CONFIGS = {
    # name: (kwargs for the generator, default seed)
    "c1_small": dict(kind="small_plain", seed=1),
    "c2_web_1m": dict(kind="web_like", n=1_000_000, m=10_000_000, seed=2001,
                      giant_frac=0.40, cac_frac=0.30, dangling_frac=0.10, zipf_a=2.1,
                      n_levels=60, scc_median=12, cac_median=8),
    "c3_deep_5m": dict(kind="web_like", n=5_000_000, m=50_000_000, seed=3001,
                       giant_frac=0.0, cac_frac=0.30, dangling_frac=0.10, zipf_a=2.3,
                       n_levels=300, scc_median=6, scc_sigma=0.87, cac_median=8,
                       scc_tail_max=20_000, level_width="pareto"),
    "c4_train_100k": dict(kind="web_like", n=100_000, m=1_000_000, seed=4001,
                          giant_frac=0.40, cac_frac=0.30, dangling_frac=0.10, zipf_a=2.1,
                          n_levels=60, scc_median=12, cac_median=8),
    "c5_web_20m": dict(kind="web_like", n=20_000_000, m=200_000_000, seed=5001,
                       giant_frac=0.50, cac_frac=0.25, dangling_frac=0.08, zipf_a=2.1,
                       n_levels=60, scc_median=12, cac_median=8),
    # the B-A workloads: about one and about five edges per vertex
    "ba_1m_e1": dict(kind="barabasi_albert", n=1_000_000, m=2, seed=6001),
    "ba_1m_e5": dict(kind="barabasi_albert", n=1_000_000, m=24, seed=6002),
}


def config_graph(name: str, seed: int | None = None, **override) -> Graph:
    cfg = dict(CONFIGS[name])
    cfg.update(override)
    kind = cfg.pop("kind")
    s = cfg.pop("seed")
    if seed is not None:
        s = seed
    if kind == "small_plain":
        g = small_plain(seed=s, **cfg)
    elif kind == "barabasi_albert":
        g = barabasi_albert(cfg.pop("n"), cfg.pop("m"), s, **cfg)
    else:
        n = cfg.pop("n")
        m = cfg.pop("m")
        g = web_like(n, m, s, **cfg)
    g.meta["config"] = name
    return g
