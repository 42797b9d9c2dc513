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


class SplittingExecutor(ScriptedExecutor):
    """Steps of request `rid` fail while its dE exceeds `limit` (a load step
    too large for Newton); checkpoint / restore copy the scripted state."""

    def __init__(self, rid, limit):
        super().__init__()
        self.rid, self.limit = rid, limit
        self.restores = 0

    def step(self, klass, handles, dEs):
        out = super().step(klass, handles, dEs)
        for h, dE, o in zip(handles, dEs, out):
            if h["rid"] == self.rid and float(dE[0, 0]) > self.limit:
                o.update(ok=False, error="scripted Newton cap")
        return out

    def checkpoint(self, h):
        return dict(h)

    def restore(self, h, ck):
        h.update(ck)
        self.restores += 1


def test_failed_increment_is_split_and_the_request_completes():
    """Request 0's steps fail while dE > 0.9 (increment n has dE = n): the
    server restores the state and halves the failing sub-step, so increment
    1 runs as 0.5 x 2, increment 2 as 0.5 x 4, increment 3 as 0.75 x 4 and
    increment 4 as 0.5 x 8 (three halvings, the limit); the converged
    sub-steps add up to each increment, one Sigma is recorded per increment,
    and with max_split = 0 the same request fails."""
    reqs = [FakeReq(0, 0.0, (9, 9, 9), 4), FakeReq(1, 0.0, (9, 9, 9), 3)]
    ex = SplittingExecutor(0, 0.9)
    srv = Server(ex, 10 ** 9, max_split=3)
    recs = srv.run(reqs)
    r0 = recs[0]
    assert r0.status == "ok" and recs[1].status == "ok"
    assert len(r0.sigma) == r0.n_inc == 4 and r0.done_inc == 4
    seen = ex.seen_dE[0]
    assert abs(sum(v for v in seen if v <= ex.limit) - (1 + 2 + 3 + 4)) < 1e-12
    assert sorted(set(v for v in seen if v <= ex.limit)) == [0.5, 0.75]
    assert r0.splits == ex.restores > 0
    assert summarize(recs)["split_increments"] == r0.splits
    assert not ex.live
    ex2 = SplittingExecutor(0, ex.limit)
    recs2 = Server(ex2, 10 ** 9, max_split=0).run(reqs)
    assert recs2[0].status == "failed" and recs2[1].status == "ok"


def test_split_depth_is_bounded():
    """A step that fails at every size fails the request after max_split
    halvings of one increment."""
    reqs = [FakeReq(0, 0.0, (9, 9, 9), 2)]
    ex = SplittingExecutor(0, -1.0)      # every dE fails
    recs = Server(ex, 10 ** 9, max_split=2).run(reqs)
    assert recs[0].status == "failed" and recs[0].splits == 2   # 1 -> 1/2 -> 1/4, which fails at the limit
    assert ex.seen_dE[0] == [1.0, 0.5, 0.25]
