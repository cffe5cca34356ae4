"""Calls of the binding on a handle made with a stream of its own.  Their
inputs are made on torch's current stream and their outputs are read there,
so each call must be ordered against it both ways.  The current stream is
kept busy by a spin kernel just before each input is written, so a call that
read its input without waiting would see memory not written yet.  Every step
(ASSIGN, POSITIVE, COMPONENTS, the sweep, N_Q, one MAXIMAL round, AGGREGATE)
must equal the oracle bit for bit, as on the current stream."""
import numpy as np
import pytest

import oracle
from gpu_common import oracle_states, say, small_graphs

pytestmark = pytest.mark.gpu

SPIN = 20_000_000  # cycles of the spin kernel (about 10 ms)


@pytest.fixture(scope="module")
def slm():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1702_04645_amd as slm
    slm.lib()
    return slm


def _late(x):
    """x on the device, written on the current stream after a spin."""
    import torch
    src = torch.as_tensor(np.ascontiguousarray(x), device="cuda")
    torch.cuda.synchronize()
    torch.cuda._sleep(SPIN)
    out = torch.empty_like(src)
    out.copy_(src)
    return out


def _np(t):
    return t.cpu().numpy()


@pytest.mark.parametrize("name", ["rmat12", "mixed_hub", "sbm1000"])
def test_side_stream_steps(slm, name):
    import torch
    rp, col, w = small_graphs()[name]
    say("side stream", name)
    g_or, a0, a1, lab1, nc1 = oracle_states(rp, col, w)
    side = torch.cuda.Stream()
    with slm.Graph(rp, col, w, stream=side) as g:
        assert np.array_equal(_np(g.assign()), a0)
        a1_g, s_g = g.positive(_late(a0))
        assert np.array_equal(_np(a1_g), a1)
        lab_o, nc_o, cyc_o = oracle.components(a1)
        lab, nc, cyc = g.components(_late(a1))
        assert nc == nc_o and np.array_equal(_np(lab), lab_o)
        assert np.array_equal(_np(cyc).astype(bool), cyc_o)
        b_o, d_o, w_o = oracle.sweep(g_or, lab1, nc1)
        b, d, wo = g.sweep(_late(lab1), nc1)
        assert np.array_equal(_np(b), b_o) and np.array_equal(_np(d), d_o)
        assert np.array_equal(_np(wo), w_o)
        nq, _ = g.modularity(_late(lab1), nc1)
        assert nq == oracle.modularity_num(g_or, lab1, nc1)
        a2_o, v_o, st_o = oracle.maximal_round(g_or, a1, 5, 0, 0)
        a2_g, st_g = g.round(_late(a1), slm.params(seed=5), 0, 0)
        assert st_g["valid"] == v_o and np.array_equal(_np(a2_g), a2_o)
        rp_o, col_o, w_o2 = oracle.contract(g_or, lab1, nc1)
        g.contract(_late(lab1), nc1)
        rp_g, col_g, w_g = g.export_level()
        assert np.array_equal(rp_g, rp_o) and np.array_equal(col_g, col_o)
        assert np.array_equal(w_g, w_o2)


def test_side_stream_noalloc(slm):
    import torch
    rp, col, w = small_graphs()["rmat12"]
    g_or, a0, a1, lab1, nc1 = oracle_states(rp, col, w)
    side = torch.cuda.Stream()
    nq, _ = slm.modularity_noalloc(_late(rp.astype(np.int64)), _late(col), _late(w),
                                   _late(lab1), nc1, stream=side)
    assert nq == oracle.modularity_num(g_or, lab1, nc1)
