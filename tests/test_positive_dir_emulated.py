"""The directed model's POSITIVE kernel (Sec. 2.4 and 3.3; k_positive_dir),
compiled for the host by g++ with the emulation header in tests/emu (one
thread per lane, real barriers and wavefront exchanges), against the
oracle's POSITIVE under the directed model on the POSITIVE inputs of the
first level of oracle runs (the assignment after ASSIGN and after the first
MAXIMAL rounds' re-pointing) and on random assignments of every node to a
neighbour, with cycles of any length.  Community and member orders are shuffled (on
the device they come from atomics), and lanes other than 0 are held back
after every barrier (or all lanes by random amounts), so that a read of
shared state that a single thread changes before the next barrier shows up
as a stuck barrier or a different result.  Needs no GPU."""
import os
import re
import shutil
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.join(ROOT, "tests"))

import graphgen as gg  # noqa: E402
import oracle  # noqa: E402
from gpu_common import neighbour_assignment, small_graphs  # noqa: E402

CSRC = os.path.join(ROOT, "paper_1702_04645_amd", "csrc")
EMU = os.path.join(ROOT, "tests", "emu")
WORKGROUPS = {"wg256": 256, "wg64": 64}

pytestmark = pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")


def _kernel_source():
    s = open(os.path.join(CSRC, "k_positive_dir.hip")).read()
    s, k = re.subn(r"^#define PD_BS (\d+)(.*)$", r"#ifndef PD_BS\n#define PD_BS \1\2\n#endif", s,
                   flags=re.M)
    assert k == 1
    s, k = re.subn(r"k_positive_dir<<<.*>>>\(A\);", "(void)A; (void)s;", s)
    assert k == 1
    return s


@pytest.fixture(scope="module")
def emulators(tmp_path_factory):
    d = tmp_path_factory.mktemp("positive_dir_emu")
    (d / "k_positive_dir_emu.inc").write_text(_kernel_source())
    out = {}
    for name, bs in WORKGROUPS.items():
        exe = str(d / ("emu_" + name))
        cmd = ["g++", "-std=c++20", "-O1", "-pthread", "-I", EMU, "-I", CSRC, "-I", str(d),
               "-DPD_BS=%d" % bs, os.path.join(EMU, "positive_dir_emu.cpp"), "-o", exe]
        r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
        assert r.returncode == 0, r.stderr[-3000:]
        out[name] = exe
    return out


def _p(a):
    import ctypes
    return a.ctypes.data_as(ctypes.c_void_p)


def positive_inputs(rp, col, w, num, den, seed, max_rounds=6):
    """The assignments the first level of an oracle run under the directed
    model hands to POSITIVE (ASSIGN's, then the first rounds' re-pointed
    ones), and two random assignments of every node to a neighbour or
    itself (cycles of any length), with the level's null-model graph."""
    ng = oracle.NullGraph(rp, col, w, oracle.DIRECTED, num, den)
    out = []
    if ng.n == 0 or ng.m2 == 0:
        return ng, out
    a = oracle.assign_nm(ng)
    out.append(a.copy())
    a, _ = oracle.positive_nm(ng, a)
    for r in range(max_rounds):
        a2 = np.array(a, dtype=np.int32, copy=True)
        rep = np.array(a, dtype=np.int32, copy=True)
        st = np.zeros(4, np.int64)
        valid = int(oracle._load().or_maximal_round_nm(*ng._g(), _p(a2), seed, 0, r,
                                                        oracle.DEFAULT_ACCEPT, _p(st), _p(rep)))
        if valid == 0:
            break
        out.append(rep.copy())
        a = a2
    for r in range(2):
        out.append(neighbour_assignment(ng.rp, ng.col, seed + 10 + r).astype(np.int32))
    return ng, out


def run_emulator(exe, cases, order, skew_us, tmp):
    fin, fout = str(tmp / "cases.bin"), str(tmp / "out.bin")
    with open(fin, "wb") as f:
        for ng, a in cases:
            np.array([ng.n, ng.col.size, ng.A, order, 1], np.int64).tofile(f)
            ng.rp.astype(np.int64).tofile(f)
            ng.col.astype(np.int32).tofile(f)
            ng.w.astype(np.int32).tofile(f)
            ng.x[: ng.n].astype(np.int32).tofile(f)
            ng.y[: ng.n].astype(np.int32).tofile(f)
            a.astype(np.int32).tofile(f)
    r = subprocess.run([exe, fin, fout, str(skew_us)], capture_output=True, text=True,
                       timeout=900)
    assert r.returncode == 0, "emulated kernel stopped (%d):\n%s" % (r.returncode,
                                                                    r.stderr[-6000:])
    res = []
    with open(fout, "rb") as f:
        for ng, a in cases:
            hdr = np.fromfile(f, np.int64, 3)
            res.append((hdr, np.fromfile(f, np.int32, ng.n)))
    return res


def _cases():
    cases = []
    graphs = small_graphs()
    for name in ["random0", "random1", "random2", "random3", "random4", "random5", "path200",
                 "cliques", "sbm1000"]:
        rp, col, w = graphs[name]
        d = gg.orient(rp, col, w, 17 + len(name), both=0.3,
                      w_max=0 if name.startswith("star") else 6)
        for num, den in ((1, 1), (3, 2)) if name.startswith("random") else ((1, 1),):
            ng, inputs = positive_inputs(*d, num, den, seed=4)
            cases += [(ng, a) for a in inputs]
    for s in range(4):
        rg = np.random.default_rng(900 + s)
        n = int(rg.integers(5, 400))
        d = gg.random_directed(n, int(rg.integers(n, 5 * n)), 9, 900 + s, loops=(s % 2 == 0))
        ng, inputs = positive_inputs(*d, 1, 1, seed=4)
        cases += [(ng, a) for a in inputs]
    return cases


@pytest.mark.parametrize("config,skew", [("wg256", 20), ("wg64", -30)])
def test_emulated_directed_positive_matches_oracle(emulators, config, skew, tmp_path):
    cases = _cases()
    assert len(cases) < 250
    order = 7 + WORKGROUPS[config] + abs(skew)
    res = run_emulator(emulators[config], cases, order, skew_us=skew, tmp=tmp_path)
    splits = flagged = 0
    for (ng, a), (hdr, a_got) in zip(cases, res):
        a_exp, s_exp = oracle.positive_nm(ng, a)
        assert hdr[1] == 0, "loop bound tripped (code %d)" % hdr[1]
        assert hdr[0] == s_exp
        assert np.array_equal(a_got, a_exp)
        splits += int(hdr[0])
        flagged += int(hdr[2])
    # the cases exercise the kernel: many communities split, many splits
    assert flagged > 30 and splits > 60, (flagged, splits)
