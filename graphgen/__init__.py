"""Seeded synthetic graph generators shared by the tests, the oracle checks and
the benchmark.

This module only builds inputs: symmetric integer CSR matrices of the graph
families the method is measured on.  It holds none of the community-detection
arithmetic.  Every generator is deterministic in its seed (numpy's Philox
counter-based bit generator).

A CSR graph is returned as ``(row_ptr int64[n+1], col int32[nnz], w int32[nnz])``
with strictly ascending columns in every row and a symmetric matrix; the
diagonal, when present, is stored once.

Families:
  * ``sbm``        planted-partition stochastic block model (unit weights)
  * ``rmat``       R-MAT (Chakrabarti, Zhan & Faloutsos 2004) edge sampling,
                   symmetrised, duplicate samples summed into the weight,
                   self-loops dropped
  * ``lfr_style``  an LFR-shaped graph (Lancichinetti, Fortunato & Radicchi
                   2008): power-law degrees and community sizes, a mixing
                   fraction of external stubs, configuration-model pairing,
                   integer weights 1..16
  * ``sbm_batch``  many small planted-partition graphs of log-uniform size
  * small fixtures: disjoint cliques, paths, stars, random sparse graphs
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "rng", "csr_from_pairs", "sbm", "rmat", "lfr_style", "lfr_directed", "orient", "random_directed",
    "sbm_batch_sizes",
    "sbm_batch_graph", "sbm_batch", "batch_member_seed", "cliques", "path", "star", "random_sparse", "CONFIG_SEEDS",
    "config_graph",
]

# default seed of each named workload
CONFIG_SEEDS = {"sbm4096": 0x5EED0000, "rmat20": 0x5EED0001, "lfr4m": 0x5EED0002,
                "batch2048": 0x5EED0003, "serve": 0x5EED0004, "lfr1m_dir": 0x5EED0005}


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.Philox(int(seed) & ((1 << 64) - 1)))


def csr_from_pairs(n: int, u: np.ndarray, v: np.ndarray, wt: np.ndarray | None = None,
                   symmetrise: bool = True):
    """CSR of the matrix that sums ``wt`` over every (u, v) pair (and (v, u)
    when ``symmetrise``); a pair with u == v adds its weight to A_uu once."""
    u = np.asarray(u, dtype=np.int64)
    v = np.asarray(v, dtype=np.int64)
    if wt is None:
        wt = np.ones(u.shape[0], dtype=np.int64)
    wt = np.asarray(wt, dtype=np.int64)
    if symmetrise:
        off = u != v
        uu = np.concatenate([u, v[off]])
        vv = np.concatenate([v, u[off]])
        ww = np.concatenate([wt, wt[off]])
    else:
        uu, vv, ww = u, v, wt
    key = uu * n + vv
    order = np.argsort(key, kind="stable")
    key = key[order]
    ww = ww[order]
    if key.size:
        head = np.empty(key.size, dtype=bool)
        head[0] = True
        np.not_equal(key[1:], key[:-1], out=head[1:])
        starts = np.flatnonzero(head)
        uw = np.add.reduceat(ww, starts)
        sel = order[starts]
        rows, cols = uu[sel], vv[sel]
    else:
        uw = ww
        rows, cols = uu, vv
    counts = np.bincount(rows, minlength=n) if n else np.zeros(0, np.int64)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    if uw.size and uw.max() >= 2**31:
        raise ValueError("edge weight does not fit int32")
    return row_ptr, cols.astype(np.int32), uw.astype(np.int32)


def _bernoulli_block_pairs(g, nodes0: int, size: int, p: float):
    """Upper-triangle pairs of a dense block drawn with probability p."""
    iu, ju = np.triu_indices(size, k=1)
    keep = g.random(iu.size) < p
    return iu[keep] + nodes0, ju[keep] + nodes0


def sbm(n: int, block: int, p_in: float, p_out: float, seed: int):
    """Planted-partition SBM: blocks of ``block`` contiguous ids (the last may
    be partial); each pair inside a block is an edge with probability p_in,
    each pair across blocks with probability p_out; unit weights, no loops."""
    g = rng(seed)
    us, vs = [], []
    starts = list(range(0, n, block))
    sizes = [min(block, n - s) for s in starts]
    for s, b in zip(starts, sizes):
        if b >= 2:
            u, v = _bernoulli_block_pairs(g, s, b, p_in)
            us.append(u)
            vs.append(v)
    # external pairs: draw the count, then distinct uniform cross-block pairs
    inside = sum(b * (b - 1) // 2 for b in sizes)
    total = n * (n - 1) // 2
    cross = total - inside
    if cross > 0 and p_out > 0:
        m_out = int(g.binomial(cross, p_out))
        blk = np.repeat(np.arange(len(sizes)), sizes)
        got_u = np.zeros(0, np.int64)
        got_v = np.zeros(0, np.int64)
        while got_u.size < m_out:
            need = (m_out - got_u.size) * 2 + 16
            a = g.integers(0, n, need)
            b = g.integers(0, n, need)
            ok = blk[a] != blk[b]
            a, b = a[ok], b[ok]
            lo, hi = np.minimum(a, b), np.maximum(a, b)
            key = np.concatenate([got_u * n + got_v, lo * n + hi])
            _, first = np.unique(key, return_index=True)
            first.sort()
            key = key[first]
            got_u, got_v = key // n, key % n
        us.append(got_u[:m_out])
        vs.append(got_v[:m_out])
    u = np.concatenate(us) if us else np.zeros(0, np.int64)
    v = np.concatenate(vs) if vs else np.zeros(0, np.int64)
    return csr_from_pairs(n, u, v)


def rmat(scale: int, edge_factor: int, a: float, b: float, c: float, seed: int,
         chunk: int = 1 << 22):
    """R-MAT: edge_factor * 2^scale samples; each of the ``scale`` bit levels
    picks quadrant (0,0),(0,1),(1,0),(1,1) with probabilities a,b,c,d.  The
    samples are symmetrised, duplicates are summed into the weight and
    self-loops are dropped."""
    n = 1 << scale
    m = edge_factor * n
    g = rng(seed)
    keys = []
    t_ab, t_abc = a + b, a + b + c
    for s0 in range(0, m, chunk):
        cnt = min(chunk, m - s0)
        src = np.zeros(cnt, np.int64)
        dst = np.zeros(cnt, np.int64)
        for _lvl in range(scale):
            r = g.random(cnt)
            bit_src = r >= t_ab
            bit_dst = ((r >= a) & (r < t_ab)) | (r >= t_abc)
            src = (src << 1) | bit_src
            dst = (dst << 1) | bit_dst
        keep = src != dst
        src, dst = src[keep], dst[keep]
        keys.append(np.concatenate([src * n + dst, dst * n + src]))
    key = np.sort(np.concatenate(keys))
    head = np.empty(key.size, dtype=bool)
    head[0] = True
    np.not_equal(key[1:], key[:-1], out=head[1:])
    starts = np.flatnonzero(head)
    ukey = key[starts]
    cnt = np.diff(np.append(starts, key.size))
    rows = ukey >> scale
    cols = ukey & (n - 1)
    row_ptr = np.zeros(n + 1, np.int64)
    np.cumsum(np.bincount(rows, minlength=n), out=row_ptr[1:])
    return row_ptr, cols.astype(np.int32), cnt.astype(np.int32)


def _powerlaw_int(g, count: int, expo: float, lo: float, hi: float):
    """Integers from a continuous power law p(x) ~ x^-expo on [lo, hi]
    (inverse-CDF sampling), rounded to the nearest integer."""
    u = g.random(count)
    e1 = 1.0 - expo
    x = (lo**e1 + u * (hi**e1 - lo**e1)) ** (1.0 / e1)
    return np.rint(x).astype(np.int64)


def _powerlaw_mean(expo: float, lo: float, hi: float) -> float:
    e1, e2 = 1.0 - expo, 2.0 - expo
    return (e1 / e2) * (hi**e2 - lo**e2) / (hi**e1 - lo**e1)


def lfr_style(n: int, mean_deg: float, max_deg: int, deg_expo: float, comm_expo: float,
              comm_min: int, comm_max: int, mu: float, w_max: int, seed: int):
    """LFR-shaped graph.  Degrees follow a power law (exponent ``deg_expo``) on
    [k_min, max_deg] with k_min solved so the mean is ``mean_deg``; community
    sizes follow a power law (exponent ``comm_expo``) on [comm_min, comm_max].
    Nodes are placed in communities at random; a node keeps round((1-mu)*k)
    internal stubs (at most its community size - 1) and the rest external.
    Internal stubs are paired at random inside their community, external
    stubs at random over the whole graph; self-loops and repeated pairs are
    dropped.  Each undirected edge gets a weight uniform in 1..w_max.
    Returns (row_ptr, col, w, community_of_node)."""
    g = rng(seed)
    lo_k, hi_k = 1.0, float(max_deg)
    for _ in range(200):  # bisection for k_min giving the requested mean
        mid = 0.5 * (lo_k + hi_k)
        if _powerlaw_mean(deg_expo, mid, max_deg) < mean_deg:
            lo_k = mid
        else:
            hi_k = mid
    kmin = 0.5 * (lo_k + hi_k)
    deg = np.clip(_powerlaw_int(g, n, deg_expo, kmin, max_deg), 1, max_deg)
    # community sizes until they cover n nodes
    sizes = []
    total = 0
    while total < n:
        s = _powerlaw_int(g, 4096, comm_expo, comm_min, comm_max)
        for x in s:
            x = int(min(x, n - total))
            sizes.append(x)
            total += x
            if total >= n:
                break
    sizes = np.array(sizes, np.int64)
    if sizes[-1] < comm_min and sizes.size > 1:  # fold a short tail into the previous one
        sizes[-2] += sizes[-1]
        sizes = sizes[:-1]
    comm = np.repeat(np.arange(sizes.size), sizes)
    comm = comm[g.permutation(n)]
    csize = sizes[comm]
    k_in = np.minimum(np.rint((1.0 - mu) * deg).astype(np.int64), csize - 1)
    k_out = deg - k_in

    def pair_stubs(owner, group):
        # random order inside each group, then consecutive stubs pair up
        r = g.random(owner.size)
        order = np.lexsort((r, group))
        owner, group = owner[order], group[order]
        even = owner.size - (owner.size % 2)
        u, v = owner[0:even:2], owner[1:even:2]
        same = group[0:even:2] == group[1:even:2]
        return u[same], v[same]

    nodes = np.arange(n, dtype=np.int64)
    in_owner = np.repeat(nodes, k_in)
    u1, v1 = pair_stubs(in_owner, comm[in_owner])
    out_owner = np.repeat(nodes, k_out)
    u2, v2 = pair_stubs(out_owner, np.zeros(out_owner.size, np.int64))
    u = np.concatenate([u1, u2])
    v = np.concatenate([v1, v2])
    keep = u != v
    u, v = u[keep], v[keep]
    lo, hi = np.minimum(u, v), np.maximum(u, v)
    key = np.unique(lo * n + hi)
    lo, hi = key // n, key % n
    wt = g.integers(1, w_max + 1, key.size)
    rp, col, w = csr_from_pairs(n, lo, hi, wt)
    return rp, col, w, comm.astype(np.int32)


def lfr_directed(n: int, mean_deg: float, max_deg: int, mu_t: float, mu_w: float, seed: int,
                 deg_expo: float = 2.1, comm_expo: float = 1.1, comm_min: int = 60,
                 comm_max: int = 600, both: float = 0.25, w_max_in: int = 12):
    """A weighted directed graph of the LFR shape: the undirected structure of
    lfr_style (topological mixing mu_t), each edge kept as one arc in a random
    direction or, with probability ``both``, as two arcs; arc weights uniform
    in 1..w_max_in inside a community and in 1..w_max_out across, w_max_out
    chosen so that the share of weight across communities is about mu_w.
    Returns (row_ptr, col, w, community_of_node)."""
    rp, col, _, comm = lfr_style(n, mean_deg, max_deg, deg_expo, comm_expo, comm_min, comm_max,
                                 mu_t, 1, seed)
    # mean external / mean internal weight = (mu_w / mu_t) / ((1 - mu_w) / (1 - mu_t))
    ratio = (mu_w / mu_t) / ((1.0 - mu_w) / (1.0 - mu_t))
    w_max_out = max(1, int(round(ratio * (w_max_in + 1) - 1)))
    n = len(rp) - 1
    u = np.repeat(np.arange(n, dtype=np.int64), np.diff(rp))
    v = col.astype(np.int64)
    up = u < v
    u, v = u[up], v[up]
    g = rng(seed + 1)
    flip = g.random(u.size) < 0.5
    two = g.random(u.size) < both
    su = np.where(flip, v, u)
    sv = np.where(flip, u, v)
    uu = np.concatenate([su, sv[two]])
    vv = np.concatenate([sv, su[two]])
    inside = comm[uu] == comm[vv]
    wt = np.where(inside, g.integers(1, w_max_in + 1, uu.size),
                  g.integers(1, w_max_out + 1, uu.size))
    rpd, cold, wd = csr_from_pairs(n, uu, vv, wt, symmetrise=False)
    return rpd, cold, wd, comm


def sbm_batch_sizes(count: int, n_lo: int, n_hi: int, seed: int):
    """Node counts log-uniform in [n_lo, n_hi] and block sizes uniform in
    16..256 for a batch of planted-partition graphs."""
    g = rng(seed)
    ns = np.rint(np.exp(g.uniform(math.log(n_lo), math.log(n_hi), count))).astype(np.int64)
    bs = g.integers(16, 257, count)
    return ns, bs


def sbm_batch_graph(n: int, block: int, p_in: float, mean_ext_deg: float, seed: int):
    """One member of a batch: p_out chosen so the mean external degree is
    ``mean_ext_deg`` (unused when the graph is a single block)."""
    p_out = 0.0 if n <= block else min(1.0, mean_ext_deg / float(n - block))
    return sbm(n, block, p_in, p_out, seed)


def batch_member_seed(seed: int, index: int) -> int:
    """Seed of member ``index`` of a batch drawn from ``seed``."""
    return int(np.random.SeedSequence([seed & (2**63 - 1), index]).generate_state(1, np.uint64)[0])


def sbm_batch(count: int, n_lo: int, n_hi: int, seed: int, p_in: float = 0.2,
              mean_ext_deg: float = 2.0, indices=None):
    """Members of a batch of planted-partition graphs: node counts
    log-uniform in [n_lo, n_hi], block sizes uniform in 16..256, p_in, and
    p_out for the given mean external degree.  ``indices`` picks members
    (default: all); a member depends only on (seed, index)."""
    ns, bs = sbm_batch_sizes(count, n_lo, n_hi, seed)
    idx = range(count) if indices is None else indices
    return [sbm_batch_graph(int(ns[i]), int(bs[i]), p_in, mean_ext_deg,
                            batch_member_seed(seed, i)) for i in idx]


def config_graph(name: str, seed: int | None = None):
    """The named workloads at their full sizes."""
    s = CONFIG_SEEDS[name] if seed is None else seed
    if name == "sbm4096":
        return sbm(4096, 128, 0.1, 0.002, s)
    if name == "rmat20":
        return rmat(20, 16, 0.57, 0.19, 0.19, s)
    if name == "lfr4m":
        rp, col, w, _ = lfr_style(4_000_000, 20.0, 2000, 2.5, 1.5, 20, 5000, 0.3, 16, s)
        return rp, col, w
    if name == "lfr1m_dir":
        rp, col, w, _ = lfr_directed(1_000_000, 50.0, 100, 0.5, 0.4, s)
        return rp, col, w
    raise KeyError(name)


# ---------------------------------------------------------------- fixtures

def cliques(sizes, isolated: int = 0):
    """Disjoint unit-weight cliques of the given sizes, then isolated nodes."""
    us, vs = [], []
    base = 0
    for s in sizes:
        iu, ju = np.triu_indices(s, k=1)
        us.append(iu + base)
        vs.append(ju + base)
        base += s
    n = base + isolated
    u = np.concatenate(us) if us else np.zeros(0, np.int64)
    v = np.concatenate(vs) if vs else np.zeros(0, np.int64)
    return csr_from_pairs(n, u, v)


def path(n: int):
    u = np.arange(n - 1)
    return csr_from_pairs(n, u, u + 1)


def star(leaves: int):
    u = np.zeros(leaves, np.int64)
    return csr_from_pairs(leaves + 1, u, np.arange(1, leaves + 1))


def random_directed(n: int, m: int, w_max: int, seed: int, loops: bool = False):
    """A directed graph W: m random arcs u -> v (repeats summed), weights
    uniform 1..w_max, stored by source row; with ``loops`` some W_uu > 0."""
    g = rng(seed)
    u = g.integers(0, n, m)
    v = g.integers(0, n, m)
    if not loops:
        keep = u != v
        u, v = u[keep], v[keep]
    wt = g.integers(1, w_max + 1, u.size)
    return csr_from_pairs(n, u, v, wt, symmetrise=False)


def orient(row_ptr, col, w, seed: int, both: float = 0.3, w_max: int = 0):
    """A directed graph from a symmetric CSR: every undirected pair i < j
    keeps both arcs with probability ``both``, else one arc in a random
    direction; loops stay.  Arc weights are the edge's weight, or uniform
    1..w_max per arc when w_max > 0."""
    n = len(row_ptr) - 1
    u = np.repeat(np.arange(n, dtype=np.int64), np.diff(row_ptr))
    v = np.asarray(col, np.int64)
    wt = np.asarray(w, np.int64)
    up = u <= v
    u, v, wt = u[up], v[up], wt[up]
    g = rng(seed)
    keep2 = g.random(u.size) < both
    flip = g.random(u.size) < 0.5
    loop = u == v
    su = np.where(flip & ~loop, v, u)
    sv = np.where(flip & ~loop, u, v)
    extra = keep2 & ~loop
    uu = np.concatenate([su, sv[extra]])
    vv = np.concatenate([sv, su[extra]])
    ww = np.concatenate([wt, wt[extra]])
    if w_max > 0:
        ww = g.integers(1, w_max + 1, uu.size)
    return csr_from_pairs(n, uu, vv, ww, symmetrise=False)


def random_sparse(n: int, m: int, w_max: int, seed: int, loops: bool = False):
    """m random pairs (repeats summed), weights uniform 1..w_max; with
    ``loops`` some diagonal entries appear."""
    g = rng(seed)
    u = g.integers(0, n, m)
    v = g.integers(0, n, m)
    if not loops:
        keep = u != v
        u, v = u[keep], v[keep]
    wt = g.integers(1, w_max + 1, u.size)
    return csr_from_pairs(n, u, v, wt)
