"""The package has no CPU path: without its HIP library (or without a GPU)
every entry raises instead of computing, and no module or source of the
package reads the oracle, which is test infrastructure only."""
import os
import re
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
PKG = os.path.join(ROOT, "paper_1702_04645_amd")


def _graph():
    # a 4-cycle with unit weights
    rp = np.array([0, 2, 4, 6, 8], np.int64)
    col = np.array([1, 3, 0, 2, 1, 3, 0, 2], np.int32)
    return rp, col, np.ones(8, np.int32)


def test_missing_library_raises(monkeypatch):
    import paper_1702_04645_amd as slm
    monkeypatch.setattr(slm, "LIB_PATH", os.path.join(ROOT, "no_such_dir", "libslm.so"))
    monkeypatch.setattr(slm, "_lib", None)
    with pytest.raises(ImportError):
        slm.lib()
    with pytest.raises(ImportError):
        slm.exported_symbols()
    rp, col, w = _graph()
    # without the library (and, here, without a GPU) no entry returns a result
    for call in (lambda: slm.run(rp, col, w),
                 lambda: slm.Graph(rp, col, w, allocator=None),
                 lambda: slm.batch_solve([(rp, col, w)], allocator=None),
                 lambda: slm.Server(lanes=1)):
        with pytest.raises((ImportError, RuntimeError, AssertionError)):
            call()


def test_package_never_reads_the_oracle():
    pat = re.compile(r"^\s*(import\s+oracle|from\s+oracle\b)|liboracle|slm_oracle", re.M)
    found = []
    for dirpath, _, files in os.walk(PKG):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".h")):
                path = os.path.join(dirpath, f)
                if pat.search(open(path, encoding="utf-8").read()):
                    found.append(os.path.relpath(path, ROOT))
    assert not found, found
    for f in ("bench.py", "__graft_entry__.py"):
        src = open(os.path.join(ROOT, f), encoding="utf-8").read()
        # only the CPU-baseline leg of the bench and smoke's check may call it
        assert "import oracle" not in src.split("def ", 1)[0], f
