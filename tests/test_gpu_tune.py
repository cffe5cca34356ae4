"""The launch autotuner: every option it tries leaves the sweep unchanged
(it checks that itself), and the options it returns give the oracle's sweep."""
import numpy as np
import pytest

import oracle
from gpu_common import oracle_states, say, small_graphs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def slm():
    import torch
    assert torch.cuda.is_available()
    import paper_1702_04645_amd as slm
    slm.lib()
    return slm


@pytest.mark.parametrize("name", ["mixed_hub", "rmat12"])
def test_autotune_keeps_results(slm, name, tmp_path):
    import torch
    from paper_1702_04645_amd import autotune
    rp, col, w = small_graphs()[name]
    say("autotune", name)
    g_or, _, _, lab1, nc1 = oracle_states(rp, col, w)
    with slm.Graph(rp, col, w) as g:
        res = autotune.tune(g, reps=2, blocks=1, passes=1)
        for k, v in res["options"].items():
            assert v in autotune.CANDIDATES[k]
        path = tmp_path / "tuned.json"
        autotune.save(path, res)
        autotune.apply(g, autotune.load(path)["options"])
        b, d, o = g.sweep(torch.from_numpy(lab1).cuda(), nc1)
    b_o, d_o, w_o = oracle.sweep(g_or, lab1, nc1)
    assert np.array_equal(b.cpu().numpy(), b_o)
    assert np.array_equal(d.cpu().numpy(), d_o)
    assert np.array_equal(o.cpu().numpy(), w_o)
