"""Per-increment metrics (FFTG_METRICS=<path>: one JSON line per member and
increment, the same numbers the call returns) and roctx ranges
(FFTG_TRACE=1: the solve runs unchanged with the ranges on)."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

import synth
from tests.gpu_util import tensor6

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_metrics_lines_match_the_returned_stats(tmp_path):
    print("metrics jsonl", flush=True)
    from paper_1601_05970_amd import fftg
    path = str(tmp_path / "m.jsonl")
    w = synth.small_random((9, 7, 5), 0.4, 1, E_eq=0.01, n_inc=2)
    v = synth.small_random((5, 5, 5), 0.3, 2, E_eq=0.01, n_inc=2)
    o = fftg.fftg_options_default()
    os.environ["FFTG_METRICS"] = path
    try:
        pl = fftg.Plan(w.phase, w.materials, o)
        h = fftg.History(pl)
        single = [h.solve_increment(tensor6(w.dE(n))) for n in (1, 2)]
        plans = [fftg.Plan(x.phase, x.materials, o) for x in (w, v)]
        hists = [fftg.History(p) for p in plans]
        b = fftg.Batch(plans, hists)
        batched = [b.solve_increment(np.array([tensor6(x.dE(n)) for x in (w, v)])) for n in (1, 2)]
        b.close()
    finally:
        del os.environ["FFTG_METRICS"]
    lines = [json.loads(l) for l in open(path)]
    assert len(lines) == 2 + 2 * 2
    expect = single + [s for st in batched for s in st]
    grids = [[9, 7, 5]] * 2 + [[9, 7, 5], [5, 5, 5]] * 2
    for rec, st, g in zip(lines, expect, grids):
        assert rec["grid"] == g and rec["precision"] == "fp64" and rec["status"] == 0
        assert rec["newton"] == st["newton_iters"] and rec["cg"] == st["cg_iters"]
        assert rec["total_cg"] == st["total_cg"] and rec["converged"] == 1
        assert np.allclose(rec["Sigma"], st["Sigma"], rtol=0, atol=0)
        assert abs(rec["rel_equilibrium"] - st["rel_equilibrium"]) <= 1e-5 * max(st["rel_equilibrium"], 1e-300)
    assert [r["increment"] for r in lines[:2]] == [1, 2]


def test_solve_with_roctx_ranges():
    """FFTG_TRACE is read once per process, so the traced solve runs in a
    child process (one at a time on the device)."""
    print("roctx ranges", flush=True)
    code = (
        "import numpy as np, synth\n"
        "from paper_1601_05970_amd import fftg\n"
        "w = synth.small_random((7, 7, 7), 0.4, 3, E_eq=0.01, n_inc=2)\n"
        "pl = fftg.Plan(w.phase, w.materials, fftg.fftg_options_default())\n"
        "h = fftg.History(pl)\n"
        "from tests.gpu_util import tensor6\n"
        "st = [h.solve_increment(tensor6(w.dE(n))) for n in (1, 2)]\n"
        "print('traced', st[-1]['converged'], st[-1]['total_cg'])\n")
    env = dict(os.environ, FFTG_TRACE="1", PYTHONPATH=ROOT + os.pathsep + os.environ.get("PYTHONPATH", ""))
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, stdout=subprocess.PIPE,
                       stderr=subprocess.STDOUT, text=True, timeout=240)
    assert r.returncode == 0, r.stdout[-3000:]
    assert "traced True" in r.stdout
