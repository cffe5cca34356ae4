"""Host-side checks of the C-ABI library: it loads, exports every entry
point include/slm.h declares, and rejects bad arguments before touching a
device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    src = open(os.path.join(ROOT, "include", "slm.h")).read()
    return sorted(set(re.findall(r"\b(slm_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared()
    for must in ("slm_create", "slm_sweep", "slm_contract", "slm_run", "slm_destroy"):
        assert must in names


def test_library_exports_every_declared_symbol():
    import paper_1702_04645_amd as slm
    lib = slm.lib()
    for name in declared():
        assert hasattr(lib, name), name


def test_invalid_arguments_are_rejected_without_a_device():
    import paper_1702_04645_amd as slm
    lib = slm.lib()
    h = C.c_void_p()
    rp = np.zeros(3, np.int64)
    # bad row_ptr width
    st = lib.slm_create(2, 0, rp.ctypes.data_as(C.c_void_p), 3, None, None, 0, 1, None,
                        None, C.byref(h))
    assert st == slm.SLM_E_INVALID and b"row_ptr" in lib.slm_last_error()
    # negative size
    st = lib.slm_create(-1, 0, rp.ctypes.data_as(C.c_void_p), 8, None, None, 0, 1, None,
                        None, C.byref(h))
    assert st == slm.SLM_E_INVALID
    # n too large
    st = lib.slm_create(1 << 31, 0, rp.ctypes.data_as(C.c_void_p), 8, None, None, 0, 1, None,
                        None, C.byref(h))
    assert st == slm.SLM_E_OVERFLOW
    # missing entries
    st = lib.slm_create(2, 2, rp.ctypes.data_as(C.c_void_p), 8, None, None, 0, 1, None,
                        None, C.byref(h))
    assert st == slm.SLM_E_INVALID
    # an allocator without a free callback is rejected before any device call
    half = slm._AllocatorC(None, slm._ALLOC_FN(lambda c, n, s: None), slm._FREE_FN())
    rp2 = np.zeros(3, np.int64)
    st = lib.slm_create(2, 0, rp2.ctypes.data_as(C.c_void_p), 8, None, None, 0, 1, None,
                        C.byref(half), C.byref(h))
    assert st == slm.SLM_E_INVALID and b"allocator" in lib.slm_last_error()
    p = slm.Params()
    lib.slm_params_default(C.byref(p))
    assert p.accept_p == 1 << 31 and p.max_rounds == 64 and p.validate == 1


def test_batch_arguments_are_rejected_without_a_device():
    import paper_1702_04645_amd as slm
    lib = slm.lib()
    h = C.c_void_p()
    # no graphs
    assert lib.slm_batch_create(0, None, 1, None, None, C.byref(h)) == slm.SLM_E_INVALID

    def descs(*graphs):
        arr = (slm._Desc * len(graphs))()
        for i, (rp, col, w) in enumerate(graphs):
            arr[i] = slm._Desc(rp.size - 1, col.size, rp.ctypes.data, col.ctypes.data,
                               w.ctypes.data)
        return arr

    ok = (np.array([0, 1, 2], np.int64), np.array([1, 0], np.int32), np.array([1, 1], np.int32))
    # an asymmetric member
    bad = (np.array([0, 1, 1], np.int64), np.array([1], np.int32), np.array([1], np.int32))
    d = descs(ok, bad)
    assert lib.slm_batch_create(2, d, 1, None, None, C.byref(h)) == slm.SLM_E_INVALID
    assert b"symmetric" in lib.slm_last_error()
    # a member whose total weight reaches 2^31
    big = (np.array([0, 1, 2], np.int64), np.array([1, 0], np.int32),
           np.array([2**30, 2**30], np.int32))
    d = descs(ok, big)
    assert lib.slm_batch_create(2, d, 1, None, None, C.byref(h)) == slm.SLM_E_OVERFLOW
    # row_ptr not ending at nnz (validation off still checks it)
    short = (np.array([0, 1, 1], np.int64), np.array([1, 0], np.int32), np.array([1, 1], np.int32))
    d = descs(short)
    assert lib.slm_batch_create(1, d, 0, None, None, C.byref(h)) == slm.SLM_E_INVALID
    # the one-shot batch run checks like slm_batch_create and returns nothing
    outs = (C.c_void_p * 2)()
    p = slm.params()
    assert lib.slm_batch_solve(0, None, C.byref(p), None, None, None, outs) == slm.SLM_E_INVALID
    d = descs(ok, bad)
    assert lib.slm_batch_solve(2, d, C.byref(p), None, None, None, outs) == slm.SLM_E_INVALID
    assert outs[0] is None and outs[1] is None
    assert lib.slm_batch_solve(2, d, None, None, None, None, outs) == slm.SLM_E_INVALID


def test_server_arguments_are_rejected_without_a_device():
    import paper_1702_04645_amd as slm
    lib = slm.lib()
    h = C.c_void_p()
    for lanes, large, ncap, qcap in ((17, 0, 0, 0), (0, 0, 0, 0), (1, 0, -5, 0), (2, 2, 0, 0),
                                     (2, -1, 0, 0), (1, 0, 0, -1)):
        cfg = slm._ServerCfg(ncap, 0, 0, lanes, 0, large, 1, qcap, slm.params())
        assert lib.slm_server_create(C.byref(cfg), None, C.byref(h)) == slm.SLM_E_INVALID
    bad = slm.params(accept_p=(1 << 32) + 1)
    cfg = slm._ServerCfg(0, 0, 0, 1, 0, 0, 1, 0, bad)
    assert lib.slm_server_create(C.byref(cfg), None, C.byref(h)) == slm.SLM_E_INVALID
    # an allocator without a free callback
    half = slm._AllocatorC(None, slm._ALLOC_FN(lambda c, n, s: None), slm._FREE_FN())
    cfg = slm._ServerCfg(0, 0, 0, 1, 0, 0, 1, 0, slm.params())
    assert lib.slm_server_create(C.byref(cfg), C.byref(half), C.byref(h)) == slm.SLM_E_INVALID
    assert b"allocator" in lib.slm_last_error()
    # cancel on no server
    assert lib.slm_server_cancel(None, 1) == slm.SLM_E_INVALID


def test_set_option_rejects_without_a_device():
    import paper_1702_04645_amd as slm
    lib = slm.lib()
    assert lib.slm_set_option(None, b"hub_table_bits", 8) == slm.SLM_E_INVALID
    assert b"null" in lib.slm_last_error()


def test_noalloc_rejects_sizes_without_a_device():
    """slm_modularity_noalloc checks its sizes before touching a device."""
    import paper_1702_04645_amd as slm
    lib = slm.lib()
    big = slm.SLM_NOALLOC_MAX_COMMUNITIES + 1
    dummy = C.c_void_p(1)  # never dereferenced: the call fails first
    st = lib.slm_modularity_noalloc(big, 0, dummy, None, None, dummy, big, None, None, None)
    assert st == slm.SLM_E_INVALID and b"at most" in lib.slm_last_error()
    st = lib.slm_modularity_noalloc(-1, 0, dummy, None, None, dummy, 0, None, None, None)
    assert st == slm.SLM_E_INVALID
    st = lib.slm_modularity_noalloc(4, 0, dummy, None, None, dummy, 5, None, None, None)
    assert st == slm.SLM_E_INVALID and b"community count" in lib.slm_last_error()
    st = lib.slm_modularity_noalloc(1 << 31, 0, dummy, None, None, dummy, 0, None, None, None)
    assert st == slm.SLM_E_OVERFLOW
