"""slm_modularity_noalloc, the entry point that allocates nothing, against
slm_modularity on a handle of the same graph (and the oracle's N_Q): equal
N_Q and bit-identical Q on two calls in a row, the second on a smaller
graph, then on a contracted level, and its error paths."""
import ctypes as C

import numpy as np
import pytest

import graphgen as gg
import oracle
from gpu_common import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def slm():
    import torch
    assert torch.cuda.is_available()
    import paper_1702_04645_amd as slm
    slm.lib()
    return slm


def _dev(rp, col, w):
    import torch
    return (torch.from_numpy(np.ascontiguousarray(rp, np.int64)).cuda(),
            torch.from_numpy(np.ascontiguousarray(col, np.int32)).cuda(),
            torch.from_numpy(np.ascontiguousarray(w, np.int32)).cuda())


def _check_level(slm, g, rp, col, w, lab, nc):
    """noalloc == handle == oracle for one labelling of one graph."""
    import torch
    nq_h, q_h = g.modularity(lab, nc)
    d = _dev(rp, col, w)
    nq_n, q_n = slm.modularity_noalloc(*d, lab.to(torch.int32).contiguous(), nc)
    og = oracle.Graph(rp, col, w)
    nq_o = oracle.modularity_num(og, lab.cpu().numpy(), nc)
    say("  n=%d nc=%d N_Q handle %d noalloc %d oracle %d" % (rp.size - 1, nc, nq_h, nq_n, nq_o))
    assert nq_n == nq_h == nq_o
    assert q_n == q_h


def test_two_calls_second_smaller(slm):
    graphs = [("rmat12", gg.rmat(12, 16, 0.57, 0.19, 0.19, 77)),
              ("cliques", gg.cliques([3, 5, 8, 13], isolated=3))]
    for name, (rp, col, w) in graphs:
        say("noalloc", name)
        with slm.Graph(rp, col, w) as g:
            a = g.assign()
            lab, nc, _ = g.components(a)
            _check_level(slm, g, rp, col, w, lab, nc)


def test_contracted_level_and_repeat(slm):
    rp, col, w = gg.sbm(3000, 60, 0.2, 0.004, 9)
    with slm.Graph(rp, col, w) as g:
        a = g.assign()
        a, _ = g.positive(a)
        lab, nc, _ = g.components(a)
        _check_level(slm, g, rp, col, w, lab, nc)
        g.contract(lab, nc)
        rp1, col1, w1 = g.export_level()
        a1 = g.assign()
        lab1, nc1, _ = g.components(a1)
        say("level 1")
        _check_level(slm, g, rp1, col1, w1, lab1, nc1)
        # the singleton labelling of the level (every community one node)
        import torch
        ident = torch.arange(rp1.size - 1, dtype=torch.int32, device="cuda")
        _check_level(slm, g, rp1, col1, w1, ident, rp1.size - 1)


def test_errors(slm):
    import torch
    rp, col, w = gg.cliques([4, 4])
    d = _dev(rp, col, w)
    lab = torch.zeros(rp.size - 1, dtype=torch.int32, device="cuda")
    lab[3] = 5  # out of range for n_c = 2
    with pytest.raises(slm.SlmError) as e:
        slm.modularity_noalloc(*d, lab, 2)
    assert e.value.status == slm.SLM_E_INVALID and "label" in str(e.value)
    # a good call right after the failed one
    lab[3] = 0
    nq, q = slm.modularity_noalloc(*d, lab, 2)
    og = oracle.Graph(rp, col, w)
    assert nq == oracle.modularity_num(og, lab.cpu().numpy(), 2)
    # community count beyond the fixed work space: rejected before any launch
    lib = slm.lib()
    st = lib.slm_modularity_noalloc(slm.SLM_NOALLOC_MAX_COMMUNITIES + 1, 0,
                                    C.c_void_p(d[0].data_ptr()), None, None,
                                    C.c_void_p(lab.data_ptr()),
                                    slm.SLM_NOALLOC_MAX_COMMUNITIES + 1, None, None, None)
    assert st == slm.SLM_E_INVALID and b"at most" in lib.slm_last_error()
