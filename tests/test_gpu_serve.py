"""Served requests give the same results as the same requests solved alone
(within the stated tolerance: 1e-10 FP64, 1e-6 mixed), with arrivals that
overlap work already on the device: 15^3 requests join a class that is
already stepping (its batch is rebuilt on the join and kept otherwise), and
63^3 requests run in classes of their own beside the small ones."""
import numpy as np
import pytest

import synth
from tests.gpu_util import tensor6, to_host

pytestmark = pytest.mark.gpu


def _requests():
    shapes = [(9, 9, 9), (15, 15, 15), (11, 13, 7), (15, 15, 15), (9, 11, 13), (13, 13, 13), (63, 63, 63),
              (15, 15, 15), (63, 63, 63)]
    precs = ["fp64", "mixed", "fp64", "fp64", "mixed", "mixed", "fp64", "fp64", "mixed"]
    arrivals = [0.0, 0.0, 0.002, 0.004, 0.006, 0.05, 0.01, 0.2, 0.3]
    out = []
    for i, (sh, pr, t) in enumerate(zip(shapes, precs, arrivals)):
        w = synth.small_random(sh, 0.35, 10 + i, E_eq=0.01, n_inc=3 + (i % 2))
        w.precision = pr
        out.append(synth.Request(i, t, w))
    return out


def _alone(w):
    from paper_1601_05970_amd import fftg
    o = fftg.fftg_options_default()
    o.tol_newton, o.tol_cg = w.tol_newton, w.tol_cg
    o.precision = fftg.FFTG_MIXED if w.precision == "mixed" else fftg.FFTG_FP64
    pl = fftg.Plan(w.phase, w.materials, o)
    h = fftg.History(pl)
    return [h.solve_increment(tensor6(w.dE(n)))["Sigma"] for n in range(1, w.n_inc + 1)]


def test_served_results_equal_alone():
    print("serve alone vs mix", flush=True)
    from paper_1601_05970_amd.serve import FftgExecutor, Server, summarize
    reqs = _requests()
    srv = Server(FftgExecutor(), 16 * 10 ** 9)
    recs = srv.run(reqs)
    assert all(r.status == "ok" for r in recs), [(r.rid, r.status, r.error) for r in recs]
    by_id = {r.rid: r for r in recs}       # the server reports in arrival order
    for q in reqs:
        r = by_id[q.rid]
        ref = np.array(_alone(q.workload))
        got = np.array(r.sigma)
        tol = 1e-10 if q.workload.precision == "fp64" else 1e-6
        assert got.shape == ref.shape
        assert np.max(np.abs(got - ref)) <= tol * np.max(np.abs(ref)), (q.rid, q.workload.precision)
    s = summarize(recs)
    assert s["ok"] == len(reqs)


def test_executor_checkpoint_restore_replays_an_increment():
    """The state the server restores before splitting an increment: a
    checkpoint taken at an increment boundary (pinned host buffer), one
    increment solved, the checkpoint restored and the same increment solved
    again gives the same Sigma and strain bit for bit."""
    print("serve checkpoint/restore", flush=True)
    from paper_1601_05970_amd import fftg
    from paper_1601_05970_amd.serve import FftgExecutor
    w = synth.small_random((15, 15, 15), 0.35, 3, E_eq=0.01, n_inc=3)
    q = synth.Request(0, 0.0, w)
    ex = FftgExecutor()
    h = ex.admit(q)
    k = ex.klass(q)
    ex.step(k, [h], [w.dE(1)])
    ck = ex.checkpoint(h)
    a = ex.step(k, [h], [w.dE(2)])[0]
    sa = to_host(h[1].get_field(fftg.FFTG_FIELD_STRAIN))
    ex.restore(h, ck)
    b = ex.step(k, [h], [w.dE(2)])[0]
    sb = to_host(h[1].get_field(fftg.FFTG_FIELD_STRAIN))
    assert a["ok"] and b["ok"] and a["Sigma"] == b["Sigma"]
    assert np.array_equal(sa, sb)
    ex.release(h)
