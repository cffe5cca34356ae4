"""Brute-force reference for tiny graphs (n <= ~14), used to pin the oracle.

Every decision here is taken on the modularity numerator recomputed from
scratch for each candidate partition, straight from the weighted modularity
of Sec. 2.4 (with m_w = M2 for a symmetric matrix):

    N_Q(sigma) = sum_ij (M2 * A_ij - k_i * k_j) * [sigma_i == sigma_j],
    Q = N_Q / M2^2.

No gain formula is used: a gain is always N_Q(after) - N_Q(before).  The
steps follow the paper's text (Sec. 3.1-3.5, Algorithm 1), with the same
tie rules and strict tests as the oracle.  Pure Python and numpy, slow by
design.
"""
from __future__ import annotations

import itertools

import numpy as np


def dense(row_ptr, col, w):
    n = len(row_ptr) - 1
    A = np.zeros((n, n), dtype=np.int64)
    for i in range(n):
        for e in range(row_ptr[i], row_ptr[i + 1]):
            A[i, col[e]] += w[e]
    return A


def nq(A, lab) -> int:
    k = A.sum(1)
    m2 = int(k.sum())
    lab = np.asarray(lab)
    same = lab[:, None] == lab[None, :]
    return int(((m2 * A - np.outer(k, k)) * same).sum())


def canonical(lab):
    """Relabel by increasing smallest member."""
    out = np.empty(len(lab), np.int64)
    seen = {}
    for i, c in enumerate(lab):
        if c not in seen:
            seen[c] = len(seen)
        out[i] = seen[c]
    return out


def wcc(a):
    """Components of {(i, a(i))} by repeated label propagation (tiny n)."""
    n = len(a)
    lab = list(range(n))
    changed = True
    while changed:
        changed = False
        for i in range(n):
            j = a[i]
            m = min(lab[i], lab[j])
            if lab[i] != m or lab[j] != m:
                lab[i] = lab[j] = m
                changed = True
    return canonical(lab)


def path_nodes(a, u):
    """u, a(u), a(a(u)), ... until a node repeats."""
    seen = []
    x = u
    while x not in seen:
        seen.append(x)
        x = a[x]
    return seen


def cycle_nodes(a, u):
    p = path_nodes(a, u)
    x = a[p[-1]]
    return p[p.index(x):]


def on_cycle(a, u):
    return u in cycle_nodes(a, u)


def assign(A, qual=None):
    """A gives the neighbours; qual(labels) the quality (default: nq(A, .))."""
    if qual is None:
        qual = lambda lab: nq(A, lab)
    n = A.shape[0]
    single = np.arange(n)
    base = qual(single)
    a = []
    for i in range(n):
        best, bj = None, i
        for j in range(n):
            if j == i or A[i, j] == 0:
                continue
            lab = single.copy()
            lab[i] = j
            g = qual(lab) - base
            if best is None or g > best:
                best, bj = g, j
        a.append(bj if best is not None and best > 0 else i)
    return a


def local_gains(A, lab, qual=None):
    if qual is None:
        qual = lambda lb: nq(A, lb)
    base = qual(lab)
    n = len(lab)
    out = []
    fresh = max(lab) + 1
    for u in range(n):
        l2 = np.array(lab).copy()
        l2[u] = fresh
        out.append((base - qual(l2)) // 2)
    return out


def positive(A, a, qual=None):
    """Split, one optimal bisection at a time, until no node has a negative
    local gain.  Candidate bisections: drop the assignment of one non-cycle
    node, or of two cycle nodes; the best is the largest N_Q gain, ties to
    the lowest (first, second) cut node."""
    if qual is None:
        qual = lambda lb: nq(A, lb)
    a = list(a)
    splits = 0
    while True:
        lab = wcc(a)
        g = local_gains(A, lab, qual)
        bad = sorted({int(lab[u]) for u in range(len(a)) if g[u] < 0})
        if not bad:
            return a, splits
        c = bad[0]
        members = [u for u in range(len(a)) if lab[u] == c]
        cyc = cycle_nodes(a, members[0])
        base = qual(lab)
        best = None
        cands = [(x, x) for x in members if x not in cyc]
        cands += [(min(x, y), max(x, y)) for x, y in itertools.combinations(cyc, 2)]
        for (x, y) in cands:
            a2 = list(a)
            a2[x] = x
            a2[y] = y
            gain = qual(wcc(a2)) - base
            key = (gain, -x, -y)
            if best is None or key > best[0]:
                best = (key, x, y)
        _, x, y = best
        a[x] = x
        a[y] = y
        splits += 1


def maximal_round(A, a, draw, p_threshold, qual=None):
    """One MAXIMAL round (then POSITIVE).  ``draw(i)`` gives node i's 32-bit
    draw.  Returns (new a, valid count)."""
    if qual is None:
        qual = lambda lb: nq(A, lb)
    n = len(a)
    lab = wcc(a)
    base = qual(lab)
    cstar = []
    for i in range(n):
        best, bc = None, lab[i]
        for C in sorted({int(lab[j]) for j in range(n) if A[i, j] > 0 and j != i}):
            if C == lab[i]:
                continue
            l2 = lab.copy()
            l2[i] = C
            gain = qual(l2) - base
            if best is None or gain > best:
                best, bc = gain, C
        cstar.append(bc if best is not None and best > 0 else int(lab[i]))
    valid = 0
    moves = {}
    for i in range(n):
        D = cstar[i]
        if D == lab[i]:
            continue
        # the tail: every node whose pointer path passes through i
        B = [u for u in range(n) if i in path_nodes(a, u)]
        l2 = lab.copy()
        for u in B:
            l2[u] = D
        if qual(l2) - base <= 0:
            continue
        valid += 1
        if draw(i) < p_threshold:
            # best neighbour inside D by the N_Q gain of pairing i with it
            single = np.arange(n)
            sb = qual(single)
            best, bj = None, None
            for j in range(n):
                if j == i or A[i, j] == 0 or lab[j] != D:
                    continue
                ls = single.copy()
                ls[i] = j
                gj = qual(ls) - sb
                if best is None or gj > best:
                    best, bj = gj, j
            moves[i] = bj
    if valid == 0:
        return list(a), 0
    a2 = list(a)
    for i, j in moves.items():
        a2[i] = j
    a2, _ = positive(A, a2, qual)
    return a2, valid


def contract(A, lab):
    lab = np.asarray(lab)
    nc = int(lab.max()) + 1
    S = np.zeros((A.shape[0], nc), np.int64)
    S[np.arange(A.shape[0]), lab] = 1
    return S.T @ A @ S


def run(A, seed, draw_fn, p_threshold=1 << 31, max_rounds=64, max_levels=0):
    """Algorithm 1 on a dense matrix; returns per-level dicts.  A level runs
    MAXIMAL rounds while some move is valid, at most max_rounds of them
    (converged is False when the cap ends it); the run stops after
    max_levels emitted levels when max_levels > 0."""
    n0 = A.shape[0]
    composed = np.arange(n0)
    out = []
    m2 = int(A.sum())
    level = 0
    while m2 > 0:
        n = A.shape[0]
        a = assign(A)
        a, _ = positive(A, a)
        r = 0
        conv = False
        while r < max_rounds:
            a, valid = maximal_round(A, a, lambda i: draw_fn(seed, level, r, i), p_threshold)
            if valid == 0:
                conv = True
                break
            r += 1
        lab = wcc(a)
        nc = int(lab.max()) + 1
        if nc == n:
            break
        composed = lab[composed]
        v = nq(A, lab)
        out.append(dict(labels=composed.copy(), n_c=nc, nq=v, rounds=r, converged=conv))
        level += 1
        if max_levels > 0 and level >= max_levels:
            break
        A = contract(A, lab)
    return out


def set_partitions(n):
    """All set partitions of range(n) as canonical label lists."""
    def rec(i, lab, k):
        if i == n:
            yield list(lab)
            return
        for c in range(k + 1):
            lab.append(c)
            yield from rec(i + 1, lab, max(k, c + 1))
            lab.pop()
    yield from rec(0, [], 0)


# ---------------------------------------------------------------- null models
CONFIG, ER, DIRECTED = 0, 1, 2


def quality(W, lab, kind, num, den, size):
    """The quality of a partition, straight from its definition:
    CONFIG    sum_ij (den*M2*W_ij - num*k_i*k_j)         [same community]
              (Sec. 2.4 modularity with resolution num/den; W symmetric)
    ER        sum_ij (den*W_ij - num*size_i*size_j)      [same community]
              (Sec. 2.2 energy with alpha = 1, beta = p = num/den, the
              Erdos-Renyi null model of Sec. 2.3; size = original nodes)
    DIRECTED  sum_ij (den*m*W_ij - num*kout_i*kin_j)     [same community]
              (Sec. 2.4 with out- and in-strengths; W any nonnegative)
    Each is a positive multiple of the modularity (energy) it names."""
    lab = np.asarray(lab)
    same = lab[:, None] == lab[None, :]
    if kind == CONFIG:
        k = W.sum(1)
        B = den * int(W.sum()) * W - num * np.outer(k, k)
    elif kind == ER:
        B = den * W - num * np.outer(size, size)
    else:
        B = den * int(W.sum()) * W - num * np.outer(W.sum(1), W.sum(0))
    return int((B * same).sum())


def contract_directed(W, lab):
    """W'_CD = sum of W_uv over u in C, v in D (any W)."""
    lab = np.asarray(lab)
    nc = int(lab.max()) + 1
    P = np.zeros((W.shape[0], nc), np.int64)
    P[np.arange(W.shape[0]), lab] = 1
    return P.T @ W @ P


def run_null(W, kind, num, den, seed, draw_fn, p_threshold=1 << 31, max_rounds=64,
             max_levels=0):
    """run() under a null model: every decision on differences of quality();
    neighbours are the nonzeros of W + W^T; each level contracts W (keeping
    its direction) and sums the node sizes.  Per level: labels, n_c, the
    quality of the level's partition, rounds, converged."""
    n0 = W.shape[0]
    composed = np.arange(n0)
    size = np.ones(n0, np.int64)
    out = []
    level = 0
    while int(W.sum()) > 0:
        n = W.shape[0]
        S = W + W.T
        qual = (lambda Wc, sz: (lambda lab: quality(Wc, lab, kind, num, den, sz)))(W, size)
        a = assign(S, qual)
        a, _ = positive(S, a, qual)
        r = 0
        conv = False
        while r < max_rounds:
            a, valid = maximal_round(S, a, lambda i: draw_fn(seed, level, r, i), p_threshold,
                                     qual)
            if valid == 0:
                conv = True
                break
            r += 1
        lab = wcc(a)
        nc = int(lab.max()) + 1
        if nc == n:
            break
        composed = lab[composed]
        out.append(dict(labels=composed.copy(), n_c=nc, nq=qual(lab), rounds=r,
                        converged=conv))
        level += 1
        if max_levels > 0 and level >= max_levels:
            break
        P = np.zeros((n, nc), np.int64)
        P[np.arange(n), lab] = 1
        size = P.T @ size
        W = contract_directed(W, lab)
    return out


# ---------------------------------------------------------------- classical Louvain
def louvain_level(A, max_passes=64):
    """Sequential local moving on a dense symmetric matrix: nodes in id
    order; node i moves to the neighbouring community whose N_Q gain (the
    whole partition recomputed from scratch) is largest, lowest name on ties,
    when that gain is positive.  Communities are named by the node they
    started from.  Returns (canonical labels, passes that moved, converged)."""
    n = A.shape[0]
    c = np.arange(n)
    p = 0
    conv = False
    while p < max_passes:
        moved = 0
        for i in range(n):
            base = nq(A, c)
            best, bc = None, None
            for C in sorted({int(c[j]) for j in range(n) if A[i, j] > 0 and j != i}):
                if C == c[i]:
                    continue
                c2 = c.copy()
                c2[i] = C
                g = nq(A, c2) - base
                if best is None or g > best:
                    best, bc = g, C
            if best is not None and best > 0:
                c[i] = bc
                moved += 1
        if moved == 0:
            conv = True
            break
        p += 1
    return canonical(c), p, conv


def louvain_run(A, max_passes=64, max_levels=0):
    n0 = A.shape[0]
    composed = np.arange(n0)
    out = []
    while int(A.sum()) > 0:
        n = A.shape[0]
        lab, p, conv = louvain_level(A, max_passes)
        nc = int(lab.max()) + 1
        if nc == n:
            break
        composed = lab[composed]
        out.append(dict(labels=composed.copy(), n_c=nc, nq=nq(A, lab), rounds=p,
                        converged=conv))
        if max_levels > 0 and len(out) >= max_levels:
            break
        A = contract(A, lab)
    return out
