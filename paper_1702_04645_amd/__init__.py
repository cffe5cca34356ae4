"""Python binding of libslm.so, the gfx950 implementation of the Synchronised
Louvain Method (Chiem, Havelange & Van Dooren, arXiv 1702.04645).

Argument marshalling only: every step runs in the HIP kernels behind the C
ABI declared in include/slm.h.  PyTorch provides device memory (the
handles' work space comes from torch's caching allocator through the
library's allocator callbacks, and outputs are torch CUDA tensors) and the
stream (the current torch stream when the graph is created).  The library
must have been built (``python -m paper_1702_04645_amd.build``); importing
this module fails loudly when it is missing.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libslm.so")

(SLM_OK, SLM_E_INVALID, SLM_E_OVERFLOW, SLM_E_NOMEM, SLM_E_DEVICE, SLM_E_STATE, SLM_E_BUSY,
 SLM_E_CANCELLED) = range(8)
_STATUS = {1: "SLM_E_INVALID", 2: "SLM_E_OVERFLOW", 3: "SLM_E_NOMEM", 4: "SLM_E_DEVICE",
           5: "SLM_E_STATE", 6: "SLM_E_BUSY", 7: "SLM_E_CANCELLED"}
SLM_NOALLOC_MAX_COMMUNITIES = 1 << 22  # include/slm.h


class SlmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (_STATUS.get(status, status), msg))
        self.status = status


class Params(C.Structure):
    """slm_params: seed, accept_p (Q32), max_rounds, max_levels, validate."""
    _fields_ = [("seed", C.c_uint64), ("accept_p", C.c_uint64), ("max_rounds", C.c_int32),
                ("max_levels", C.c_int32), ("validate", C.c_int32), ("reserved", C.c_int32)]


_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p)
_FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)


class Model(C.Structure):
    """Null model of a handle (include/slm.h slm_model): kind CONFIG with
    resolution num/den, or ER with p = num/den."""
    _fields_ = [("kind", C.c_int32), ("reserved", C.c_int32), ("num", C.c_int64),
                ("den", C.c_int64)]


MODEL_CONFIG, MODEL_ER, MODEL_DIRECTED = 0, 1, 2


def model(kind: int = MODEL_CONFIG, num: int = 1, den: int = 1) -> Model:
    return Model(kind, 0, num, den)


class _AllocatorC(C.Structure):
    """slm_allocator: ctx, alloc(ctx, bytes, stream), free(ctx, p, stream)."""
    _fields_ = [("ctx", C.c_void_p), ("alloc", _ALLOC_FN), ("free", _FREE_FN)]


class Allocator:
    """A device memory provider for the library.  ``alloc(nbytes, stream)``
    returns a device address (int), or 0 / None when it cannot;
    ``free(address, stream)`` returns it.  The callbacks may run on the
    library's own threads (server lanes).  Keep the object alive as long as
    any handle made with it."""

    def __init__(self, alloc, free):
        def _a(ctx, nbytes, stream):
            try:
                p = alloc(int(nbytes), int(stream or 0))
                return int(p) if p else None
            except Exception:
                return None

        def _f(ctx, ptr, stream):
            try:
                free(int(ptr), int(stream or 0))
            except Exception:
                pass

        self._fa = _ALLOC_FN(_a)
        self._ff = _FREE_FN(_f)
        self.c = _AllocatorC(None, self._fa, self._ff)


def torch_allocator(device=None) -> Allocator:
    """torch's CUDA caching allocator, on the handle's stream."""
    torch = _torch()
    dev = torch.cuda.current_device() if device is None else device
    alloc_fn = torch.cuda.caching_allocator_alloc
    free_fn = torch.cuda.caching_allocator_delete
    return Allocator(lambda nbytes, stream: alloc_fn(nbytes, dev, stream),
                     lambda ptr, stream: free_fn(ptr))


def _allocator(allocator):
    """The Allocator for an ``allocator`` argument: "torch" (the default),
    None (the library's hipMalloc) or an Allocator."""
    if allocator == "torch":
        return torch_allocator()
    if allocator is None or isinstance(allocator, Allocator):
        return allocator
    raise TypeError("allocator must be 'torch', None or an Allocator")


def _aptr(a):
    return C.byref(a.c) if a is not None else None


def params(seed: int = 0, accept_p: int = 1 << 31, max_rounds: int = 64, max_levels: int = 0,
           validate: int = 1) -> Params:
    return Params(seed & (2**64 - 1), accept_p, max_rounds, max_levels, validate, 0)


_lib = None


def lib():
    """The loaded libslm.so (raises when it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libslm.so is not built; run python -m paper_1702_04645_amd.build")
    L = C.CDLL(LIB_PATH)
    P, i32, i64, st = C.c_void_p, C.c_int32, C.c_int64, C.c_int
    pi32, pi64 = C.POINTER(C.c_int32), C.POINTER(C.c_int64)
    sigs = {
        "slm_params_default": (None, [C.POINTER(Params)]),
        "slm_create": (st, [i64, i64, P, C.c_int, P, P, C.c_int, C.c_int, P,
                            C.POINTER(_AllocatorC), C.POINTER(P)]),
        "slm_destroy": (None, [P]),
        "slm_create_model": (st, [i64, i64, P, C.c_int, P, P, C.c_int, C.c_int,
                                  C.POINTER(Model), P, C.POINTER(_AllocatorC), C.POINTER(P)]),
        "slm_level_info": (st, [P, pi32, pi64, pi64, pi64]),
        "slm_reset": (st, [P]),
        "slm_export_level": (st, [P, P, P, P]),
        "slm_assign": (st, [P, P]),
        "slm_components": (st, [P, P, P, P, pi64]),
        "slm_positive": (st, [P, P, pi64]),
        "slm_sweep": (st, [P, P, i64, P, P, P]),
        "slm_round": (st, [P, C.POINTER(Params), i32, i32, P, pi64]),
        "slm_level": (st, [P, C.POINTER(Params), i32, P, pi64, pi32, pi32]),
        "slm_modularity": (st, [P, P, i64, pi64, C.POINTER(C.c_double)]),
        "slm_contract": (st, [P, P, i64]),
        "slm_run": (st, [P, C.POINTER(Params), C.POINTER(P)]),
        "slm_louvain_level": (st, [P, C.POINTER(Params), P, pi64, pi32, pi32]),
        "slm_louvain_run": (st, [P, C.POINTER(Params), C.POINTER(P)]),
        "slm_result_num_levels": (st, [P, pi32]),
        "slm_result_level": (st, [P, i32, pi64, C.POINTER(C.POINTER(C.c_int32)), pi64,
                                  C.POINTER(C.c_double), pi32, pi32]),
        "slm_result_free": (None, [P]),
        "slm_result_times": (st, [P, pi64, pi64]),
        "slm_timing_enable": (st, [P, C.c_int]),
        "slm_timing_read": (st, [P, C.POINTER(C.c_double), pi64, pi64, pi64]),
        "slm_set_option": (st, [P, C.c_char_p, i64]),
        "slm_last_error": (C.c_char_p, []),
        "slm_batch_create": (st, [i32, P, C.c_int, P, C.POINTER(_AllocatorC), C.POINTER(P)]),
        "slm_batch_size": (st, [P, pi32]),
        "slm_batch_run": (st, [P, C.POINTER(Params), P, P]),
        "slm_batch_solve": (st, [i32, P, C.POINTER(Params), P, P, C.POINTER(_AllocatorC), P]),
        "slm_server_create": (st, [P, C.POINTER(_AllocatorC), C.POINTER(P)]),
        "slm_server_cancel": (st, [P, C.c_uint64]),
        "slm_server_submit": (st, [P, P, C.c_uint64, C.POINTER(C.c_uint64)]),
        "slm_server_poll": (st, [P, C.c_uint64, C.POINTER(P)]),
        "slm_server_wait": (st, [P, C.c_uint64, C.POINTER(P)]),
        "slm_server_stats": (st, [P, pi64, pi64, pi64]),
        "slm_server_destroy": (None, [P]),
        "slm_modularity_noalloc": (st, [i64, i64, P, P, P, P, i64, pi64,
                                        C.POINTER(C.c_double), P]),
    }
    for name, (res, args) in sigs.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def exported_symbols():
    return [n for n in lib().__dict__ if n.startswith("slm_")]


def _check(status: int):
    if status != SLM_OK:
        raise SlmError(status, lib().slm_last_error().decode())


def _torch():
    import torch
    return torch


def _dev_i32(n: int):
    torch = _torch()
    return torch.empty(max(n, 1), dtype=torch.int32, device="cuda")


def _ptr(t):
    return C.c_void_p(t.data_ptr())


def _on_stream(stream, fn, *args, tensors=()):
    """Runs library call fn(*args), whose device work goes to ``stream``,
    ordered against torch's current stream when the two differ: ``stream``
    first waits for the work queued on the current stream (which made the
    inputs), and the current stream then waits for ``stream`` (whose work
    writes the outputs); ``tensors`` are marked as used on ``stream``, so the
    caching allocator does not hand their memory out again before that work
    is done."""
    torch = _torch()
    cur = torch.cuda.current_stream()
    other = stream is not None and stream != cur
    if other:
        stream.wait_stream(cur)
    _check(fn(*args))
    if other:
        for t in tensors:
            t.record_stream(stream)
        cur.wait_stream(stream)


@dataclass
class LevelResult:
    labels: np.ndarray
    n_c: int
    nq: int
    q: float
    rounds: int
    converged: bool


class Graph:
    """A handle on a symmetric integer CSR graph resident in HBM.

    ``row_ptr`` (int32 or int64), ``col`` and ``w`` (int32) are numpy arrays
    (host) or torch CUDA tensors (device).  The handle's device memory comes
    from ``allocator`` ("torch": torch's caching allocator; None: the
    library's hipMalloc; or an Allocator)."""

    def __init__(self, row_ptr, col, w, validate: bool = True, stream=None,
                 allocator="torch", model: Model | None = None):
        torch = _torch()
        self._h = C.c_void_p()
        self._alloc = _allocator(allocator)
        on_dev = isinstance(row_ptr, torch.Tensor) and row_ptr.is_cuda
        if on_dev:
            rp, cl, ww = row_ptr.contiguous(), col.contiguous().to(torch.int32), \
                w.contiguous().to(torch.int32)
            rp_bytes = rp.element_size()
            n = rp.numel() - 1
            nnz = cl.numel()
            self._keep = (rp, cl, ww)
            args = (_ptr(rp), _ptr(cl), _ptr(ww))
        else:
            rp = np.ascontiguousarray(row_ptr)
            if rp.dtype not in (np.int32, np.int64):
                rp = rp.astype(np.int64)
            cl = np.ascontiguousarray(col, dtype=np.int32)
            ww = np.ascontiguousarray(w, dtype=np.int32)
            rp_bytes = rp.dtype.itemsize
            n = rp.size - 1
            nnz = cl.size
            self._keep = (rp, cl, ww)
            args = (rp.ctypes.data_as(C.c_void_p), cl.ctypes.data_as(C.c_void_p),
                    ww.ctypes.data_as(C.c_void_p))
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        if on_dev and stream != torch.cuda.current_stream():
            stream.wait_stream(torch.cuda.current_stream())  # the inputs were made there
        if model is None:
            _check(lib().slm_create(n, nnz, args[0], rp_bytes, args[1], args[2], int(on_dev),
                                    int(validate), C.c_void_p(stream.cuda_stream),
                                    _aptr(self._alloc), C.byref(self._h)))
        else:
            _check(lib().slm_create_model(n, nnz, args[0], rp_bytes, args[1], args[2],
                                          int(on_dev), int(validate), C.byref(model),
                                          C.c_void_p(stream.cuda_stream), _aptr(self._alloc),
                                          C.byref(self._h)))
        self._keep = None
        self.n0 = n
        self.nnz0 = nnz

    def close(self):
        if self._h:
            lib().slm_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -------------------------------------------------------------- level state
    def level_info(self):
        lv, n, nnz, m2 = C.c_int32(), C.c_int64(), C.c_int64(), C.c_int64()
        _check(lib().slm_level_info(self._h, C.byref(lv), C.byref(n), C.byref(nnz), C.byref(m2)))
        return dict(level=lv.value, n=n.value, nnz=nnz.value, m2=m2.value)

    def reset(self):
        _check(lib().slm_reset(self._h))

    def export_level(self):
        info = self.level_info()
        rp = np.zeros(info["n"] + 1, np.int64)
        col = np.zeros(max(info["nnz"], 1), np.int32)
        w = np.zeros(max(info["nnz"], 1), np.int32)
        _check(lib().slm_export_level(self._h, rp.ctypes.data_as(C.c_void_p),
                                      col.ctypes.data_as(C.c_void_p),
                                      w.ctypes.data_as(C.c_void_p)))
        return rp, col[: info["nnz"]], w[: info["nnz"]]

    # -------------------------------------------------------------- steps
    def assign(self):
        n = self.level_info()["n"]
        a = _dev_i32(n)
        _on_stream(self.stream, lib().slm_assign, self._h, _ptr(a), tensors=(a,))
        return a[:n]

    def components(self, a):
        torch = _torch()
        n = self.level_info()["n"]
        a = a.to(torch.int32).contiguous()
        lab = _dev_i32(n)
        cyc = torch.empty(max(n, 1), dtype=torch.uint8, device="cuda")
        nc = C.c_int64()
        _on_stream(self.stream, lib().slm_components, self._h, _ptr(a), _ptr(lab), _ptr(cyc),
                   C.byref(nc), tensors=(a, lab, cyc))
        return lab[:n], nc.value, cyc[:n]

    def positive(self, a):
        torch = _torch()
        a = a.to(torch.int32).clone()
        sp = C.c_int64()
        _on_stream(self.stream, lib().slm_positive, self._h, _ptr(a), C.byref(sp), tensors=(a,))
        return a, sp.value

    def sweep(self, lab, nc: int):
        torch = _torch()
        n = self.level_info()["n"]
        lab = lab.to(torch.int32).contiguous()
        best = _dev_i32(n)
        delta = torch.empty(max(n, 1), dtype=torch.int64, device="cuda")
        wown = _dev_i32(n)
        _on_stream(self.stream, lib().slm_sweep, self._h, _ptr(lab), int(nc), _ptr(best),
                   _ptr(delta), _ptr(wown), tensors=(lab, best, delta, wown))
        return best[:n], delta[:n], wown[:n]

    def round(self, a, p: Params, level: int, rnd: int):
        torch = _torch()
        a = a.to(torch.int32).clone()
        st = (C.c_int64 * 4)()
        _on_stream(self.stream, lib().slm_round, self._h, C.byref(p), level, rnd, _ptr(a), st,
                   tensors=(a,))
        return a, dict(candidates=st[0], valid=st[1], accepted=st[2], splits=st[3])

    def level(self, p: Params, level: int):
        n = self.level_info()["n"]
        lab = _dev_i32(n)
        nc, r, cv = C.c_int64(), C.c_int32(), C.c_int32()
        _on_stream(self.stream, lib().slm_level, self._h, C.byref(p), level, _ptr(lab),
                   C.byref(nc), C.byref(r), C.byref(cv), tensors=(lab,))
        return lab[:n], nc.value, r.value, bool(cv.value)

    def modularity(self, lab, nc: int):
        torch = _torch()
        lab = lab.to(torch.int32).contiguous()
        nq, q = C.c_int64(), C.c_double()
        _on_stream(self.stream, lib().slm_modularity, self._h, _ptr(lab), int(nc), C.byref(nq),
                   C.byref(q), tensors=(lab,))
        return nq.value, q.value

    def contract(self, lab, nc: int):
        torch = _torch()
        lab = lab.to(torch.int32).contiguous()
        _on_stream(self.stream, lib().slm_contract, self._h, _ptr(lab), int(nc), tensors=(lab,))

    def run(self, p: Params | None = None):
        if p is None:
            p = params()
        res = C.c_void_p()
        _check(lib().slm_run(self._h, C.byref(p), C.byref(res)))
        return _take_result(res, self.n0)

    def louvain_level(self, p: Params | None = None):
        """Classical Louvain local moving of the current level: (labels, n_c,
        passes, converged)."""
        if p is None:
            p = params()
        n = self.level_info()["n"]
        lab = _dev_i32(n)
        nc, ps, cv = C.c_int64(), C.c_int32(), C.c_int32()
        _on_stream(self.stream, lib().slm_louvain_level, self._h, C.byref(p), _ptr(lab),
                   C.byref(nc), C.byref(ps), C.byref(cv), tensors=(lab,))
        return lab[:n], nc.value, ps.value, bool(cv.value)

    def louvain_run(self, p: Params | None = None):
        """Full classical Louvain run (rounds = passes per level)."""
        if p is None:
            p = params()
        res = C.c_void_p()
        _check(lib().slm_louvain_run(self._h, C.byref(p), C.byref(res)))
        return _take_result(res, self.n0)

    # -------------------------------------------------------------- timing
    def set_option(self, name: str, value: int):
        """Tuning knob of the sweep (`slm_set_option`); results never change."""
        _check(lib().slm_set_option(self._h, name.encode(), int(value)))

    def timing(self, enable: bool = True):
        _check(lib().slm_timing_enable(self._h, int(enable)))

    def timing_read(self):
        ms, sw, en, by = C.c_double(), C.c_int64(), C.c_int64(), C.c_int64()
        _check(lib().slm_timing_read(self._h, C.byref(ms), C.byref(sw), C.byref(en), C.byref(by)))
        return dict(sweep_ms=ms.value, sweeps=sw.value, entries=en.value, bytes=by.value)


def _take_result(res, n0: int):
    """Copies an slm_result into a list of LevelResult and frees it."""
    try:
        L = C.c_int32()
        _check(lib().slm_result_num_levels(res, C.byref(L)))
        out = []
        for l in range(L.value):
            nc, nq, q = C.c_int64(), C.c_int64(), C.c_double()
            r, cv = C.c_int32(), C.c_int32()
            labp = C.POINTER(C.c_int32)()
            _check(lib().slm_result_level(res, l, C.byref(nc), C.byref(labp), C.byref(nq),
                                          C.byref(q), C.byref(r), C.byref(cv)))
            labels = np.ctypeslib.as_array(labp, shape=(n0,)).copy() if n0 else \
                np.zeros(0, np.int32)
            out.append(LevelResult(labels, nc.value, nq.value, q.value, r.value, bool(cv.value)))
        return out
    finally:
        lib().slm_result_free(res)


class _Desc(C.Structure):
    _fields_ = [("n", C.c_int64), ("nnz", C.c_int64), ("row_ptr", C.c_void_p),
                ("col", C.c_void_p), ("w", C.c_void_p)]


def _descs(graphs):
    """slm_graph_desc array of host CSR triples, and the arrays it points to."""
    keep = []
    descs = (_Desc * len(graphs))()
    for i, (rp, col, w) in enumerate(graphs):
        rp = np.ascontiguousarray(rp, dtype=np.int64)
        cl = np.ascontiguousarray(col, dtype=np.int32)
        ww = np.ascontiguousarray(w, dtype=np.int32)
        keep.append((rp, cl, ww))
        descs[i] = _Desc(rp.size - 1, cl.size, rp.ctypes.data, cl.ctypes.data, ww.ctypes.data)
    return descs, keep


def _seed_array(seeds, count):
    if seeds is None:
        return None
    sd = np.ascontiguousarray([int(x) & (2**64 - 1) for x in seeds], dtype=np.uint64)
    assert sd.size == count
    return sd


def batch_solve(graphs, p: Params | None = None, seeds=None, stream=None, allocator="torch"):
    """One-shot batched run (slm_batch_solve) of a list of host CSR triples;
    returns one list of LevelResult per graph."""
    torch = _torch()
    if p is None:
        p = params()
    a = _allocator(allocator)
    descs, keep = _descs(graphs)
    G = len(graphs)
    sd = _seed_array(seeds, G)
    if stream is None:
        stream = torch.cuda.current_stream()
    outs = (C.c_void_p * max(G, 1))()
    _check(lib().slm_batch_solve(G, descs, C.byref(p),
                                 sd.ctypes.data_as(C.c_void_p) if sd is not None else None,
                                 C.c_void_p(stream.cuda_stream), _aptr(a), outs))
    return [_take_result(C.c_void_p(outs[i]), keep[i][0].size - 1) for i in range(G)]


class Batch(Graph):
    """Many independent graphs (a list of host CSR triples) in one handle,
    run together as one disjoint union.  The single-step methods inherited
    from Graph act on the level-0 union."""

    def __init__(self, graphs, validate: bool = True, stream=None, allocator="torch"):
        torch = _torch()
        self._h = C.c_void_p()
        self._alloc = _allocator(allocator)
        descs, keep = _descs(graphs)
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        _check(lib().slm_batch_create(len(graphs), descs, int(validate),
                                      C.c_void_p(stream.cuda_stream), _aptr(self._alloc),
                                      C.byref(self._h)))
        self.sizes = [k[0].size - 1 for k in keep]
        self.n0 = int(sum(self.sizes))
        self.nnz0 = int(sum(k[1].size for k in keep))

    def __len__(self):
        return len(self.sizes)

    def set_option(self, name: str, value: int):
        """Tuning knob of the sweep (`slm_set_option`); results never change."""
        _check(lib().slm_set_option(self._h, name.encode(), int(value)))

    def run(self, p: Params | None = None, seeds=None):
        """Full runs of every graph; returns one list of LevelResult per graph."""
        if p is None:
            p = params()
        G = len(self.sizes)
        sd = _seed_array(seeds, G)
        outs = (C.c_void_p * G)()
        _check(lib().slm_batch_run(self._h, C.byref(p),
                                   sd.ctypes.data_as(C.c_void_p) if sd is not None else None,
                                   outs))
        res = []
        for i in range(G):
            res.append(_take_result(C.c_void_p(outs[i]), self.sizes[i]))
        return res


class _ServerCfg(C.Structure):
    _fields_ = [("node_capacity", C.c_int64), ("entry_capacity", C.c_int64),
                ("max_members", C.c_int32), ("lanes", C.c_int32), ("large_nodes", C.c_int64),
                ("large_lanes", C.c_int32), ("validate", C.c_int32), ("queue_cap", C.c_int32),
                ("params", Params)]


class Server:
    """Serving loop of the library: requests run as they arrive, admitted at
    level boundaries while they fit a lane's capacity.  ``lanes`` lanes in
    all, ``large_lanes`` of them for graphs above ``large_nodes`` nodes;
    ``queue_cap`` requests may wait per class (0: no cap; a full queue makes
    submit raise SLM_E_BUSY)."""

    def __init__(self, node_capacity: int = 0, entry_capacity: int = 0, max_members: int = 0,
                 lanes: int = 1, large_nodes: int = 1 << 62, large_lanes: int = 0,
                 validate: bool = True, p: Params | None = None, queue_cap: int = 0,
                 allocator="torch"):
        self._h = C.c_void_p()
        self._alloc = _allocator(allocator)
        cfg = _ServerCfg(node_capacity, entry_capacity, max_members, lanes, large_nodes,
                         large_lanes, int(validate), int(queue_cap),
                         p if p is not None else params())
        _check(lib().slm_server_create(C.byref(cfg), _aptr(self._alloc), C.byref(self._h)))
        self._n0 = {}

    def submit(self, row_ptr, col, w, seed: int = 0) -> int:
        rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
        cl = np.ascontiguousarray(col, dtype=np.int32)
        ww = np.ascontiguousarray(w, dtype=np.int32)
        d = _Desc(rp.size - 1, cl.size, rp.ctypes.data, cl.ctypes.data, ww.ctypes.data)
        t = C.c_uint64()
        _check(lib().slm_server_submit(self._h, C.byref(d), seed & (2**64 - 1), C.byref(t)))
        self._n0[t.value] = rp.size - 1
        return t.value

    def cancel(self, ticket: int):
        """Cancels a request; its poll / wait then raises SLM_E_CANCELLED."""
        _check(lib().slm_server_cancel(self._h, ticket))

    def poll(self, ticket: int):
        """The levels of a finished request (once), else None."""
        res = C.c_void_p()
        _check(lib().slm_server_poll(self._h, ticket, C.byref(res)))
        if not res.value:
            return None
        return _take_result(res, self._n0.pop(ticket))

    def wait(self, ticket: int):
        res = C.c_void_p()
        _check(lib().slm_server_wait(self._h, ticket, C.byref(res)))
        return _take_result(res, self._n0.pop(ticket))

    def wait_timed(self, ticket: int):
        """(levels, seconds from submission to the end of the last level)."""
        res = C.c_void_p()
        _check(lib().slm_server_wait(self._h, ticket, C.byref(res)))
        a, b = C.c_int64(), C.c_int64()
        _check(lib().slm_result_times(res, C.byref(a), C.byref(b)))
        return _take_result(res, self._n0.pop(ticket)), (b.value - a.value) / 1e9

    def stats(self):
        a, b, c = C.c_int64(), C.c_int64(), C.c_int64()
        _check(lib().slm_server_stats(self._h, C.byref(a), C.byref(b), C.byref(c)))
        return dict(submitted=a.value, completed=b.value, reserved_bytes=c.value)

    def close(self):
        if self._h:
            lib().slm_server_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def run(row_ptr, col, w, seed: int = 0, accept_p: int = 1 << 31, max_rounds: int = 64,
        max_levels: int = 0):
    """Full run of Algorithm 1 on the GPU; returns a list of LevelResult."""
    with Graph(row_ptr, col, w) as g:
        return g.run(params(seed, accept_p, max_rounds, max_levels))


def modularity_noalloc(row_ptr, col, w, lab, nc: int, stream=None):
    """N_Q and Q of a labelling of a device CSR through slm_modularity_noalloc
    (no handle, no device allocation).  ``row_ptr`` int64, ``col``, ``w`` and
    ``lab`` int32 CUDA tensors."""
    torch = _torch()
    for t in (row_ptr, col, w, lab):
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.is_contiguous()):
            raise TypeError("row_ptr, col, w and lab must be contiguous CUDA tensors")
    if row_ptr.dtype != torch.int64 or col.dtype != torch.int32 or w.dtype != torch.int32 \
            or lab.dtype != torch.int32:
        raise TypeError("row_ptr must be int64; col, w and lab int32")
    if stream is None:
        stream = torch.cuda.current_stream()
    n = row_ptr.numel() - 1
    if lab.numel() < n:
        raise ValueError("lab holds fewer than n labels")
    nq, q = C.c_int64(), C.c_double()
    _on_stream(stream, lib().slm_modularity_noalloc, n, col.numel(), _ptr(row_ptr), _ptr(col),
               _ptr(w), _ptr(lab), int(nc), C.byref(nq), C.byref(q),
               C.c_void_p(stream.cuda_stream), tensors=(row_ptr, col, w, lab))
    return nq.value, q.value
