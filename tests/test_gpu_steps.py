"""Step-by-step parity of the GPU path (through the C ABI) with the CPU
oracle: ASSIGN, COMPONENTS, POSITIVE, the MAXIMAL sweep, one MAXIMAL round,
one level, modularity and AGGREGATE.  Integer results must be bit-exact."""
import numpy as np
import pytest

import oracle
from gpu_common import neighbour_assignment, oracle_states, say, small_graphs

pytestmark = pytest.mark.gpu

GRAPHS = small_graphs()
NAMES = sorted(GRAPHS)


@pytest.fixture(scope="module")
def slm():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1702_04645_amd as slm
    slm.lib()
    return slm


def _t(x):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x), device="cuda")


def _np(t):
    return t.cpu().numpy()


@pytest.mark.parametrize("name", NAMES)
def test_assign(slm, name):
    rp, col, w = GRAPHS[name]
    say("assign", name, rp.size - 1, col.size)
    g_or = oracle.Graph(rp, col, w)
    with slm.Graph(rp, col, w) as g:
        info = g.level_info()
        assert info["m2"] == g_or.m2 and info["n"] == g_or.n
        a = _np(g.assign())
    assert np.array_equal(a, oracle.assign(g_or))


@pytest.mark.parametrize("name", NAMES)
def test_components(slm, name):
    rp, col, w = GRAPHS[name]
    say("components", name)
    a = neighbour_assignment(rp, col, 7)
    lab_o, nc_o, cyc_o = oracle.components(a)
    with slm.Graph(rp, col, w) as g:
        lab, nc, cyc = g.components(_t(a))
        assert nc == nc_o
        assert np.array_equal(_np(lab), lab_o)
        assert np.array_equal(_np(cyc).astype(bool), cyc_o)


@pytest.mark.parametrize("name", NAMES)
def test_positive(slm, name):
    rp, col, w = GRAPHS[name]
    say("positive", name)
    g_or = oracle.Graph(rp, col, w)
    starts = [oracle.assign(g_or), neighbour_assignment(rp, col, 11)]
    with slm.Graph(rp, col, w) as g:
        for a0 in starts:
            a_o, s_o = oracle.positive(g_or, a0)
            a_g, s_g = g.positive(_t(a0))
            assert np.array_equal(_np(a_g), a_o)
            assert s_g == s_o


@pytest.mark.parametrize("name", NAMES)
def test_sweep(slm, name):
    rp, col, w = GRAPHS[name]
    say("sweep", name)
    g_or, a0, a1, lab1, nc1 = oracle_states(rp, col, w)
    n = rp.size - 1
    rg = np.random.default_rng(2)
    labs = [(lab1, nc1), (np.arange(n, dtype=np.int32), n)]
    r = rg.integers(0, max(2, n // 7), n)
    _, inv = np.unique(r, return_inverse=True)
    lab_r, nc_r, _ = oracle.components(np.arange(n, dtype=np.int32))  # identity
    first = {}
    canon = np.empty(n, np.int32)
    for i, c in enumerate(inv):
        canon[i] = first.setdefault(int(c), len(first))
    labs.append((canon, len(first)))
    with slm.Graph(rp, col, w) as g:
        for lab, nc in labs:
            b_o, d_o, w_o = oracle.sweep(g_or, lab, nc)
            b, d, wo = g.sweep(_t(lab), nc)
            assert np.array_equal(_np(b), b_o)
            assert np.array_equal(_np(d), d_o)
            assert np.array_equal(_np(wo), w_o)


@pytest.mark.parametrize("name", ["star5000", "mixed_hub"])
@pytest.mark.parametrize("bits,pairs", [(4, 8), (6, 1), (5, 3072), (11, 100)])
def test_sweep_hub_passes(slm, name, bits, pairs):
    """Hub rows with small partition tables: partitions cut into many passes,
    and passes that fill the table cut again, give the same sweep."""
    rp, col, w = GRAPHS[name]
    say("sweep hub passes", name, bits, pairs)
    g_or, a0, a1, lab1, nc1 = oracle_states(rp, col, w)
    n = rp.size - 1
    r = np.random.default_rng(4).integers(0, max(2, n // 3), n)
    first = {}
    canon = np.array([first.setdefault(int(c), len(first)) for c in r], np.int32)
    labs = [(lab1, nc1), (np.arange(n, dtype=np.int32), n), (canon, len(first))]
    with slm.Graph(rp, col, w) as g:
        g.set_option("hub_table_bits", bits)
        g.set_option("hub_pass_pairs", pairs)
        for lab, nc in labs:
            b_o, d_o, w_o = oracle.sweep(g_or, lab, nc)
            b, d, wo = g.sweep(_t(lab), nc)
            assert np.array_equal(_np(b), b_o)
            assert np.array_equal(_np(d), d_o)
            assert np.array_equal(_np(wo), w_o)
        with pytest.raises(slm.SlmError):
            g.set_option("hub_table_bits", 12)
        with pytest.raises(slm.SlmError):
            g.set_option("no_such_option", 1)


@pytest.mark.parametrize("name", NAMES)
def test_round(slm, name):
    rp, col, w = GRAPHS[name]
    say("round", name)
    g_or, a0, a1, lab1, nc1 = oracle_states(rp, col, w)
    with slm.Graph(rp, col, w) as g:
        a_o, a_g = a1, a1
        for rnd in range(3):
            for acc in (1 << 31, 1 << 32):
                p = slm.params(seed=5, accept_p=acc)
                a_o2, v_o, st_o = oracle.maximal_round(g_or, a_o, 5, 0, rnd, acc)
                a_g2, st_g = g.round(_t(a_o), p, 0, rnd)
                assert st_g["valid"] == v_o
                assert st_g["candidates"] == st_o["candidates"]
                assert st_g["accepted"] == st_o["accepted"]
                assert np.array_equal(_np(a_g2), a_o2)
            a_o = a_o2


@pytest.mark.parametrize("name", NAMES)
def test_level_modularity_contract(slm, name):
    rp, col, w = GRAPHS[name]
    say("level", name)
    g_or = oracle.Graph(rp, col, w)
    a_o, r_o, c_o, _ = oracle.level(g_or, 3, 0)
    lab_o, nc_o, _ = oracle.components(a_o)
    with slm.Graph(rp, col, w) as g:
        lab, nc, r, c = g.level(slm.params(seed=3), 0)
        assert (nc, r, c) == (nc_o, r_o, c_o)
        assert np.array_equal(_np(lab), lab_o)
        nq, q = g.modularity(lab, nc)
        nq_o = oracle.modularity_num(g_or, lab_o, nc_o)
        assert nq == nq_o and q == oracle.modularity(nq_o, g_or.m2)
        if nc < g_or.n:
            g.contract(lab, nc)
            rp2, col2, w2 = g.export_level()
            rp_o, col_o, w_o = oracle.contract(g_or, lab_o, nc_o)
            assert np.array_equal(rp2, rp_o)
            assert np.array_equal(col2, col_o) and np.array_equal(w2, w_o)
            assert g.level_info()["m2"] == g_or.m2
        g.reset()
        assert g.level_info()["level"] == 0
