"""Scheduler of the continuous-batching server against a scripted executor
(no GPU): admission by memory footprint, FIFO order, isolation of failures,
deferred admission on allocation failure, and that every request's
increments are applied in order."""
import threading
import time

import numpy as np
import pytest

from paper_1601_05970_amd.serve import Executor, Server, summarize


class FakeWorkload:
    def __init__(self, shape, n_inc, precision="fp64"):
        self.shape, self.n_inc, self.precision = shape, n_inc, precision

    def dE(self, n):
        return np.full((3, 3), float(n))


class FakeReq:
    def __init__(self, rid, arrival, shape, n_inc, precision="fp64"):
        self.rid, self.arrival = rid, arrival
        self.workload = FakeWorkload(shape, n_inc, precision)


class ScriptedExecutor(Executor):
    """Footprint = voxels; step sleeps 0.5 ms per member; request ids listed
    in fail_at fail at that increment; oom_once makes the first admit of an
    id raise MemoryError."""

    def __init__(self, fail_at=None, oom_once=()):
        self.fail_at = fail_at or {}
        self.oom_once = set(oom_once)
        self.lock = threading.Lock()
        self.live = {}
        self.seen_dE = {}
        self.admit_order = []
        self.max_live_bytes = 0

    def footprint(self, req):
        return int(np.prod(req.workload.shape))

    def klass(self, req):
        return (req.workload.precision, max(req.workload.shape) > 20)

    def admit(self, req):
        with self.lock:
            if req.rid in self.oom_once:
                self.oom_once.discard(req.rid)
                raise MemoryError("scripted")
            self.live[req.rid] = self.footprint(req)
            self.max_live_bytes = max(self.max_live_bytes, sum(self.live.values()))
            self.admit_order.append(req.rid)
        return {"rid": req.rid, "inc": 0}

    def step(self, klass, handles, dEs):
        time.sleep(0.0005 * len(handles))
        out = []
        for h, dE in zip(handles, dEs):
            h["inc"] += 1
            self.seen_dE.setdefault(h["rid"], []).append(float(dE[0, 0]))
            ok = self.fail_at.get(h["rid"]) != h["inc"]
            out.append({"ok": ok, "Sigma": [float(h["inc"])] * 6, "cg": 3, "error": "" if ok else "scripted"})
        return out

    def release(self, h):
        with self.lock:
            del self.live[h["rid"]]


def _stream(n, seed=0):
    rng = np.random.default_rng(seed)
    t, out = 0.0, []
    for i in range(n):
        t += float(rng.exponential(0.002))
        shape = (int(rng.choice([9, 15, 31])),) * 3
        out.append(FakeReq(i, t, shape, int(rng.integers(2, 6)), "fp64" if i % 2 else "mixed"))
    return out


def test_all_requests_complete_in_order_within_budget():
    reqs = _stream(30)
    ex = ScriptedExecutor()
    budget = 3 * 31 ** 3
    srv = Server(ex, budget)
    recs = srv.run(reqs)
    assert all(r.status == "ok" for r in recs)
    assert ex.max_live_bytes <= budget and srv.max_used <= budget
    assert ex.admit_order == sorted(ex.admit_order)          # FIFO admission
    for r, q in zip(recs, reqs):
        assert r.admitted >= r.arrival - 1e-9 and r.finished >= r.admitted
        assert r.done_inc == q.workload.n_inc == len(r.sigma)
        assert ex.seen_dE[q.rid] == [float(n) for n in range(1, q.workload.n_inc + 1)]
    assert not ex.live
    s = summarize(recs)
    assert s["ok"] == 30 and s["p99_latency_s"] >= s["p50_latency_s"] > 0


def test_failure_is_isolated_and_memory_is_returned():
    reqs = _stream(12, 1)
    ex = ScriptedExecutor(fail_at={3: 1, 7: 2})
    srv = Server(ex, 10 ** 9)
    recs = srv.run(reqs)
    st = {r.rid: r.status for r in recs}
    assert st[3] == "failed" and st[7] == "failed"
    assert all(v == "ok" for k, v in st.items() if k not in (3, 7))
    assert srv.used == 0 and not ex.live


def test_allocation_failure_defers_admission():
    reqs = _stream(8, 2)
    ex = ScriptedExecutor(oom_once=[2, 5])
    srv = Server(ex, 10 ** 9)
    recs = srv.run(reqs)
    assert all(r.status == "ok" for r in recs)
    assert any("deferred" in e for e in srv.errors)


def test_oversized_request_is_rejected():
    reqs = [FakeReq(0, 0.0, (31, 31, 31), 2), FakeReq(1, 0.0, (9, 9, 9), 2)]
    srv = Server(ScriptedExecutor(), 1000)
    recs = srv.run(reqs)
    assert recs[0].status == "rejected" and recs[1].status == "ok"
