"""Oracle: TEST INFRASTRUCTURE ONLY.

A plain sequential CPU implementation of the Synchronised Louvain Method
(arXiv 1702.04645, Algorithm 1 and Sec. 3), written in C in ``slm_oracle.c``
and loaded here through ctypes.  Only the tests, the smoke check and the
CPU-baseline leg of the benchmark may import this package; the GPU library
never does and shares no code with it.

Each wrapper takes numpy arrays (CSR ``row_ptr`` int64, ``col`` int32,
``w`` int32) and returns numpy arrays.  See ``slm_oracle.c`` for the exact
definitions, the integer gain keys and the tie rules.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "slm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain C11, no GPU code)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    lib = C.CDLL(build())
    i64, i32, u64, u32 = C.c_int64, C.c_int32, C.c_uint64, C.c_uint32
    P = C.c_void_p
    sig = {
        "or_mix64": (u64, [u64]),
        "or_draw": (u32, [u64, i32, i32, i32]),
        "or_strength": (i64, [i64, P, P, P, P]),
        "or_assign": (None, [i64, P, P, P, P, i64, P]),
        "or_components": (i64, [i64, P, P, P]),
        "or_local_gain": (None, [i64, P, P, P, P, i64, P, i64, P]),
        "or_positive": (i64, [i64, P, P, P, P, i64, P]),
        "or_sweep": (None, [i64, P, P, P, P, i64, P, i64, P, P, P]),
        "or_maximal_round": (i64, [i64, P, P, P, P, i64, P, u64, i32, i32, u64, P]),
        "or_maximal_round_ex": (i64, [i64, P, P, P, P, i64, P, u64, i32, i32, u64, P, P]),
        "or_modularity_num": (i64, [i64, P, P, P, P, i64, P, i64]),
        "or_modularity": (C.c_double, [i64, i64]),
        "or_contract": (i64, [i64, P, P, P, P, i64, P, P, P]),
        "or_level": (i32, [i64, P, P, P, P, i64, u64, i32, u64, i32, P, P, P]),
        "or_run": (i32, [i64, P, P, P, u64, u64, i32, i32, i32, P, P, P, P, P, P]),
        "or_assign_nm": (None, [i64, P, P, P, P, P, i64, P]),
        "or_local_gain_nm": (None, [i64, P, P, P, P, P, i64, P, i64, P]),
        "or_positive_nm": (i64, [i64, P, P, P, P, P, i64, P]),
        "or_sweep_nm": (None, [i64, P, P, P, P, P, i64, P, i64, P, P, P]),
        "or_maximal_round_nm": (i64, [i64, P, P, P, P, P, i64, P, u64, i32, i32, u64, P, P]),
        "or_modularity_num_nm": (i64, [i64, P, P, P, P, P, i64, P, i64]),
        "or_modularity_nm": (C.c_double, [i64, i64, i64]),
        "or_level_nm": (i32, [i64, P, P, P, P, P, i64, u64, i32, u64, i32, P, P, P]),
        "or_symmetrize": (i64, [i64, P, P, P, P, P, P]),
        "or_null_strengths": (i32, [i32, i64, i64, i64, P, P, P, P, P, P]),
        "or_run_null": (i32, [i64, P, P, P, i32, i64, i64, u64, u64, i32, i32, i32, P, P, P,
                              P, P, P]),
        "or_louvain_level": (i64, [i64, P, P, P, P, i64, i32, P, P, P, P]),
        "or_louvain_run": (i32, [i64, P, P, P, i32, i32, i32, P, P, P, P, P, P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


class Graph:
    """A CSR graph with its strengths k and total M2 (Sec. 2.4)."""

    def __init__(self, row_ptr, col, w):
        self.rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
        self.col = np.ascontiguousarray(col, dtype=np.int32)
        self.w = np.ascontiguousarray(w, dtype=np.int32)
        self.n = int(self.rp.size - 1)
        self.k = np.zeros(max(self.n, 1), np.int64)
        self.m2 = int(_load().or_strength(self.n, _p(self.rp), _p(self.col), _p(self.w),
                                          _p(self.k)))
        self.k = self.k[: self.n]

    def _g(self):
        return (self.n, _p(self.rp), _p(self.col), _p(self.w), _p(self.k))


U32 = 1 << 32
DEFAULT_ACCEPT = 1 << 31  # p = 1/2 as a Q32 threshold


def mix64(z: int) -> int:
    return int(_load().or_mix64(z & (2**64 - 1)))


def draw(seed: int, level: int, rnd: int, node: int) -> int:
    return int(_load().or_draw(seed & (2**64 - 1), level, rnd, node))


def assign(g: Graph) -> np.ndarray:
    a = np.zeros(max(g.n, 1), np.int32)
    _load().or_assign(*g._g(), g.m2, _p(a))
    return a[: g.n]


def components(a: np.ndarray):
    """(canonical labels, number of communities, on-cycle flags) of the
    assignment graph {(i, a(i))}."""
    a = np.ascontiguousarray(a, dtype=np.int32)
    n = a.size
    lab = np.zeros(max(n, 1), np.int32)
    cyc = np.zeros(max(n, 1), np.uint8)
    nc = int(_load().or_components(n, _p(a), _p(lab), _p(cyc)))
    return lab[:n], nc, cyc[:n].astype(bool)


def local_gain(g: Graph, lab: np.ndarray, nc: int) -> np.ndarray:
    lab = np.ascontiguousarray(lab, dtype=np.int32)
    out = np.zeros(max(g.n, 1), np.int64)
    _load().or_local_gain(*g._g(), g.m2, _p(lab), nc, _p(out))
    return out[: g.n]


def positive(g: Graph, a: np.ndarray):
    """POSITIVE on a copy of ``a``; returns (new assignment, splits)."""
    a = np.array(a, dtype=np.int32, copy=True)
    s = int(_load().or_positive(*g._g(), g.m2, _p(a)))
    return a, s


def sweep(g: Graph, lab: np.ndarray, nc: int):
    """The synchronous best-community sweep: (best_c, delta, w_own)."""
    lab = np.ascontiguousarray(lab, dtype=np.int32)
    n = max(g.n, 1)
    best = np.zeros(n, np.int32)
    delta = np.zeros(n, np.int64)
    wown = np.zeros(n, np.int32)
    _load().or_sweep(*g._g(), g.m2, _p(lab), nc, _p(best), _p(delta), _p(wown))
    return best[: g.n], delta[: g.n], wown[: g.n]


def maximal_round(g: Graph, a: np.ndarray, seed: int, level: int, rnd: int,
                  accept_p: int = DEFAULT_ACCEPT, with_repointed: bool = False):
    """One MAXIMAL round followed by POSITIVE on a copy of ``a``.
    Returns (new assignment, valid count, stats dict); with_repointed adds the
    assignment after the re-pointing, before POSITIVE."""
    a = np.array(a, dtype=np.int32, copy=True)
    rep = np.array(a, dtype=np.int32, copy=True)
    st = np.zeros(4, np.int64)
    valid = int(_load().or_maximal_round_ex(*g._g(), g.m2, _p(a), seed & (2**64 - 1), level,
                                            rnd, accept_p, _p(st), _p(rep)))
    stats = dict(candidates=int(st[0]), valid=int(st[1]), accepted=int(st[2]),
                 splits=int(st[3]))
    if with_repointed:
        return a, valid, stats, rep
    return a, valid, stats


def modularity_num(g: Graph, lab: np.ndarray, nc: int) -> int:
    lab = np.ascontiguousarray(lab, dtype=np.int32)
    return int(_load().or_modularity_num(*g._g(), g.m2, _p(lab), nc))


def modularity(nq: int, m2: int) -> float:
    return float(_load().or_modularity(nq, m2))


def contract(g: Graph, lab: np.ndarray, nc: int):
    lab = np.ascontiguousarray(lab, dtype=np.int32)
    rp = np.zeros(nc + 1, np.int64)
    nnz = int(g.rp[-1])
    col = np.zeros(max(nnz, 1), np.int32)
    w = np.zeros(max(nnz, 1), np.int32)
    m = int(_load().or_contract(g.n, _p(g.rp), _p(g.col), _p(g.w), _p(lab), nc, _p(rp),
                                _p(col), _p(w)))
    return rp, col[:m].copy(), w[:m].copy()


def level(g: Graph, seed: int, lvl: int, accept_p: int = DEFAULT_ACCEPT,
          max_rounds: int = 64):
    """One level of Algorithm 1: returns (assignment, rounds, converged, totals)."""
    a = np.zeros(max(g.n, 1), np.int32)
    conv = np.zeros(1, np.int32)
    tot = np.zeros(3, np.int64)
    r = int(_load().or_level(*g._g(), g.m2, seed & (2**64 - 1), lvl, accept_p, max_rounds,
                             _p(a), _p(conv), _p(tot)))
    return a[: g.n], r, bool(conv[0]), dict(valid=int(tot[0]), accepted=int(tot[1]),
                                             splits=int(tot[2]))


def run(row_ptr, col, w, seed: int = 0, accept_p: int = DEFAULT_ACCEPT,
        max_rounds: int = 64, max_levels: int = 0, max_out: int = 32):
    """Full run of Algorithm 1.  Returns a list of per-level dicts with the
    composed labels of the original nodes, n_c, N_Q, Q, rounds, converged."""
    g = Graph(row_ptr, col, w)
    n0 = g.n
    lab = np.zeros((max_out, max(n0, 1)), np.int32)
    nc = np.zeros(max_out, np.int64)
    nq = np.zeros(max_out, np.int64)
    q = np.zeros(max_out, np.float64)
    rounds = np.zeros(max_out, np.int32)
    conv = np.zeros(max_out, np.int32)
    L = int(_load().or_run(n0, _p(g.rp), _p(g.col), _p(g.w), seed & (2**64 - 1), accept_p,
                           max_rounds, max_levels, max_out, _p(lab), _p(nc), _p(nq), _p(q),
                           _p(rounds), _p(conv)))
    out = []
    for l in range(min(L, max_out)):
        out.append(dict(labels=lab[l, :n0].copy(), n_c=int(nc[l]), nq=int(nq[l]), q=float(q[l]),
                        rounds=int(rounds[l]), converged=bool(conv[l])))
    return out


# ---------------------------------------------------------------- null models
CONFIG, ER, DIRECTED = 0, 1, 2  # kinds of or_null_strengths (Sec. 2.2-2.4)


def symmetrize(row_ptr, col, w):
    """S = W + W^T of a CSR W (sorted columns, diagonal 2 W_ii)."""
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    cl = np.ascontiguousarray(col, dtype=np.int32)
    ww = np.ascontiguousarray(w, dtype=np.int32)
    n = rp.size - 1
    rp2 = np.zeros(n + 1, np.int64)
    col2 = np.zeros(max(2 * cl.size, 1), np.int32)
    w2 = np.zeros(max(2 * cl.size, 1), np.int32)
    m = int(_load().or_symmetrize(n, _p(rp), _p(cl), _p(ww), _p(rp2), _p(col2), _p(w2)))
    return rp2, col2[:m].copy(), w2[:m].copy()


class NullGraph:
    """The level-0 graph of a run under a null model: the matrix the levels
    run on (S = W + W^T for DIRECTED, else the symmetric input), the
    strengths x and y, the scale A and M2 = sum of that matrix."""

    def __init__(self, row_ptr, col, w, kind: int = CONFIG, num: int = 1, den: int = 1):
        rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
        cl = np.ascontiguousarray(col, dtype=np.int32)
        ww = np.ascontiguousarray(w, dtype=np.int32)
        self.n = int(rp.size - 1)
        self.kind, self.num, self.den = kind, num, den
        x = np.zeros(max(self.n, 1), np.int64)
        y = np.zeros(max(self.n, 1), np.int64)
        A, m2 = C.c_int64(), C.c_int64()
        st = int(_load().or_null_strengths(kind, num, den, self.n, _p(rp), _p(cl), _p(ww),
                                           _p(x), _p(y), C.byref(A), C.byref(m2)))
        if st == 1:
            raise ValueError("invalid null model")
        if st == 2:
            raise OverflowError("gains of this model could leave int64")
        self.A, self.m2 = int(A.value), int(m2.value)
        self.x, self.y = x, y
        if kind == DIRECTED:
            self.rp, self.col, self.w = symmetrize(rp, cl, ww)
        else:
            self.rp, self.col, self.w = rp, cl, ww
        self._ynull = None if kind != DIRECTED else self.y

    def _g(self):
        return (self.n, _p(self.rp), _p(self.col), _p(self.w), _p(self.x),
                _p(self._ynull) if self._ynull is not None else None, self.A)


def assign_nm(g: NullGraph) -> np.ndarray:
    a = np.zeros(max(g.n, 1), np.int32)
    _load().or_assign_nm(*g._g(), _p(a))
    return a[: g.n]


def local_gain_nm(g: NullGraph, lab, nc: int) -> np.ndarray:
    lab = np.ascontiguousarray(lab, dtype=np.int32)
    out = np.zeros(max(g.n, 1), np.int64)
    _load().or_local_gain_nm(*g._g(), _p(lab), nc, _p(out))
    return out[: g.n]


def positive_nm(g: NullGraph, a):
    a = np.array(a, dtype=np.int32, copy=True)
    s = int(_load().or_positive_nm(*g._g(), _p(a)))
    return a, s


def sweep_nm(g: NullGraph, lab, nc: int):
    lab = np.ascontiguousarray(lab, dtype=np.int32)
    n = max(g.n, 1)
    best = np.zeros(n, np.int32)
    delta = np.zeros(n, np.int64)
    wown = np.zeros(n, np.int32)
    _load().or_sweep_nm(*g._g(), _p(lab), nc, _p(best), _p(delta), _p(wown))
    return best[: g.n], delta[: g.n], wown[: g.n]


def maximal_round_nm(g: NullGraph, a, seed: int, level: int, rnd: int,
                     accept_p: int = DEFAULT_ACCEPT):
    a = np.array(a, dtype=np.int32, copy=True)
    st = np.zeros(4, np.int64)
    valid = int(_load().or_maximal_round_nm(*g._g(), _p(a), seed & (2**64 - 1), level, rnd,
                                            accept_p, _p(st), None))
    return a, valid, dict(candidates=int(st[0]), valid=int(st[1]), accepted=int(st[2]),
                          splits=int(st[3]))


def modularity_num_nm(g: NullGraph, lab, nc: int) -> int:
    lab = np.ascontiguousarray(lab, dtype=np.int32)
    return int(_load().or_modularity_num_nm(*g._g(), _p(lab), nc))


def run_null(row_ptr, col, w, kind: int = CONFIG, num: int = 1, den: int = 1, seed: int = 0,
             accept_p: int = DEFAULT_ACCEPT, max_rounds: int = 64, max_levels: int = 0,
             max_out: int = 32):
    """Full run of Algorithm 1 under a null model; the same per-level dicts
    as run().  The input is symmetric for CONFIG and ER, any CSR for
    DIRECTED."""
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    cl = np.ascontiguousarray(col, dtype=np.int32)
    ww = np.ascontiguousarray(w, dtype=np.int32)
    n0 = rp.size - 1
    lab = np.zeros((max_out, max(n0, 1)), np.int32)
    nc = np.zeros(max_out, np.int64)
    nq = np.zeros(max_out, np.int64)
    q = np.zeros(max_out, np.float64)
    rounds = np.zeros(max_out, np.int32)
    conv = np.zeros(max_out, np.int32)
    L = int(_load().or_run_null(n0, _p(rp), _p(cl), _p(ww), kind, num, den,
                                seed & (2**64 - 1), accept_p, max_rounds, max_levels, max_out,
                                _p(lab), _p(nc), _p(nq), _p(q), _p(rounds), _p(conv)))
    if L == -1:
        raise ValueError("invalid null model")
    if L == -2:
        raise OverflowError("gains of this model could leave int64")
    out = []
    for l in range(min(L, max_out)):
        out.append(dict(labels=lab[l, :n0].copy(), n_c=int(nc[l]), nq=int(nq[l]), q=float(q[l]),
                        rounds=int(rounds[l]), converged=bool(conv[l])))
    return out


# ---------------------------------------------------------------- classical Louvain
def louvain_level(g: Graph, max_passes: int = 64):
    """Sequential local moving of one level: (canonical labels, n_c, passes
    that moved a node, converged, moves)."""
    lab = np.zeros(max(g.n, 1), np.int32)
    p, cv, mv = C.c_int32(), C.c_int32(), C.c_int64()
    nc = int(_load().or_louvain_level(*g._g(), g.m2, max_passes, _p(lab), C.byref(p),
                                      C.byref(cv), C.byref(mv)))
    return lab[: g.n], nc, int(p.value), bool(cv.value), int(mv.value)


def louvain_run(row_ptr, col, w, max_passes: int = 64, max_levels: int = 0, max_out: int = 32):
    """Full classical Louvain run; per-level dicts as run(), with the passes
    of each level under "rounds"."""
    g = Graph(row_ptr, col, w)
    n0 = g.n
    lab = np.zeros((max_out, max(n0, 1)), np.int32)
    nc = np.zeros(max_out, np.int64)
    nq = np.zeros(max_out, np.int64)
    q = np.zeros(max_out, np.float64)
    passes = np.zeros(max_out, np.int32)
    conv = np.zeros(max_out, np.int32)
    L = int(_load().or_louvain_run(n0, _p(g.rp), _p(g.col), _p(g.w), max_passes, max_levels,
                                   max_out, _p(lab), _p(nc), _p(nq), _p(q), _p(passes),
                                   _p(conv)))
    return [dict(labels=lab[l, :n0].copy(), n_c=int(nc[l]), nq=int(nq[l]), q=float(q[l]),
                 rounds=int(passes[l]), converged=bool(conv[l])) for l in range(min(L, max_out))]
