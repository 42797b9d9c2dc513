"""Continuous-batching server for RVE solve requests.

Each request is one RVE (phase map, materials, mean-strain path of n_inc
increments, FP64 or mixed precision).  The server

* admits arrived requests first-in first-out while the sum of their device
  footprints (fftg_footprint_bytes) fits the memory budget; a request that
  does not fit waits until finished requests free memory;
* keeps every admitted request's plan and history (strain, plastic history,
  Krylov work buffers) resident on the device until it completes;
* groups active requests into classes (precision x grid size); each class
  is advanced by its own worker thread on its own HIP stream, one increment
  of every member per step, through one batched launch sequence
  (fftg_batch_solve_increment) whose batch object persists until the class's
  membership changes.  Requests that arrive while a class is busy join it at
  the next increment boundary, and different classes overlap on the device:
  a request never waits on the Newton loop of a request of another size;
* records arrival, admission and completion times, so latency percentiles
  and throughput follow from the records;
* optionally (max_split > 0) splits an increment whose Newton iteration
  fails (iteration cap, breakdown) into two halves, up to max_split times:
  the request's state is copied to host memory at every increment boundary
  and restored before the halves run.  Algorithm 1 with a large load step
  can stall on an elasto-plastic microstructure (the Newton update keeps
  the same size from one iteration to the next) where half the step
  converges; the split path follows the same mean-strain path with finer
  increments.

The executor interface (footprint / admit / step / release) separates the
scheduling logic from the device, so the scheduler is testable on the CPU
with a scripted executor.
"""
from __future__ import annotations

import dataclasses
import threading
import time
from collections import deque
from typing import Any, Callable, Dict, List, Optional, Sequence

import numpy as np


@dataclasses.dataclass
class Record:
    rid: int
    arrival: float
    precision: str
    shape: tuple
    n_inc: int
    footprint: int
    admitted: Optional[float] = None
    finished: Optional[float] = None
    done_inc: int = 0
    status: str = "pending"           # pending / active / ok / failed / rejected
    sigma: List[List[float]] = dataclasses.field(default_factory=list)
    cg_iters: int = 0
    error: str = ""
    # sub-steps left in the current increment: (fraction of its dE, halvings)
    parts: List[Any] = dataclasses.field(default_factory=lambda: [(1.0, 0)])
    splits: int = 0

    @property
    def latency(self) -> Optional[float]:
        return None if self.finished is None else self.finished - self.arrival


class Executor:
    """Device side of the server (interface)."""

    def footprint(self, req) -> int:
        raise NotImplementedError

    def klass(self, req) -> Any:
        """Scheduling class of a request (members of a class step together)."""
        raise NotImplementedError

    def admit(self, req) -> Any:
        """Creates the device state of a request; raises MemoryError if it
        cannot be allocated."""
        raise NotImplementedError

    def step(self, klass, handles: Sequence[Any], dEs: Sequence[np.ndarray]) -> List[dict]:
        """One increment for every handle; returns per-handle dicts with
        keys ok (bool), Sigma (6 floats), cg (int), error (str)."""
        raise NotImplementedError

    def release(self, handle) -> None:
        raise NotImplementedError

    def checkpoint(self, handle) -> Any:
        """Host copy of a request's state at an increment boundary, for
        splitting an increment that fails; None when not supported."""
        return None

    def restore(self, handle, ckpt) -> None:
        raise NotImplementedError


def _tensor6(E):
    return [E[0, 0], E[1, 1], E[2, 2], E[1, 2], E[0, 2], E[0, 1]]


class FftgExecutor(Executor):
    """Executor on libfftg: one plan + history per request, one HIP stream
    per class, batched increments per class through a batch that is kept
    while the class's members stay the same."""

    def __init__(self, size_split: int = 0):
        import torch
        from . import fftg
        self.torch, self.fftg = torch, fftg
        self.size_split = size_split     # > 0: two size bands instead of one class per grid size
        self.streams: Dict[Any, Any] = {}
        self.batches: Dict[Any, Any] = {}   # class -> (member key, fftg.Batch)
        self.ckpt_bufs: Dict[int, Any] = {}  # id(history) -> pinned host buffer
        self.lock = threading.Lock()

    def footprint(self, req) -> int:
        w = req.workload
        prec = self.fftg.FFTG_MIXED if w.precision == "mixed" else self.fftg.FFTG_FP64
        return self.fftg.fftg_footprint_bytes(*w.shape, prec)

    def klass(self, req):
        w = req.workload
        if self.size_split > 0:
            return (w.precision, "large" if max(w.shape) > self.size_split else "small")
        return (w.precision, tuple(w.shape))

    def _stream(self, k):
        with self.lock:
            if k not in self.streams:
                self.streams[k] = self.torch.cuda.Stream()
            return self.streams[k]

    def admit(self, req):
        fftg = self.fftg
        w = req.workload
        o = fftg.fftg_options_default()
        o.tol_newton, o.tol_cg = w.tol_newton, w.tol_cg
        o.precision = fftg.FFTG_MIXED if w.precision == "mixed" else fftg.FFTG_FP64
        try:
            plan = fftg.Plan(w.phase, w.materials, o, stream=self._stream(self.klass(req)))
            hist = fftg.History(plan)
        except fftg.FFTGError as e:
            if e.status == fftg.FFTG_E_NOMEM:
                raise MemoryError(str(e))
            raise
        return (plan, hist)

    def _batch(self, klass, plans, hists):
        """The class's batch over exactly these members (rebuilt only when the
        membership changed since the last step)."""
        key = tuple(id(h) for h in hists)
        with self.lock:
            old = self.batches.get(klass)
            if old is not None and old[0] == key:
                return old[1]
            if old is not None:
                del self.batches[klass]
        if old is not None:
            old[1].close()
        b = self.fftg.Batch(plans, hists)
        with self.lock:
            self.batches[klass] = (key, b)
        return b

    def step(self, klass, handles, dEs):
        plans = [h[0] for h in handles]
        hists = [h[1] for h in handles]
        if len(handles) == 1:
            with self.lock:
                old = self.batches.pop(klass, None)
            if old is not None:
                old[1].close()
            st = [hists[0].solve_increment(_tensor6(dEs[0]), raise_on_error=False)]
        else:
            st = self._batch(klass, plans, hists).solve_increment(np.array([_tensor6(d) for d in dEs]),
                                                                   raise_on_error=False)
        out = []
        for s in st:
            ok = bool(s["converged"])   # Newton converged (no breakdown, no cap)
            err = ""
            if not ok:
                res = s.get("newton_res") or [float("nan")]
                err = (f"status {s['status']} after {s.get('newton_iters', len(res))} Newton iterations, "
                       f"last residual {res[-1]:.3g}")
            out.append({"ok": ok, "Sigma": s["Sigma"], "cg": s["total_cg"], "error": err})
        return out

    def checkpoint(self, handle):
        """The history's state in a pinned host buffer kept per request
        (fftg_history_save); the buffer is reused at every step."""
        plan, hist = handle
        with self.lock:
            buf = self.ckpt_bufs.get(id(hist))
        if buf is None:
            buf = self.torch.empty(hist.checkpoint_bytes(), dtype=self.torch.uint8, pin_memory=True)
            with self.lock:
                self.ckpt_bufs[id(hist)] = buf
        n = hist.save_into(buf.data_ptr(), buf.numel())
        return (buf, n)

    def restore(self, handle, ckpt):
        plan, hist = handle
        buf, n = ckpt
        hist.restore_from(buf.data_ptr(), n)

    def release(self, handle):
        plan, hist = handle
        with self.lock:
            self.ckpt_bufs.pop(id(hist), None)
        # a batch that covers this member is dropped first (it refers to the history)
        with self.lock:
            drop = [k for k, (key, _) in self.batches.items() if id(hist) in key]
            gone = [self.batches.pop(k)[1] for k in drop]
        for b in gone:
            b.close()
        hist.close()
        plan.close()


class Server:
    """Admission + per-class stepping workers; see the module docstring."""

    def __init__(self, executor: Executor, mem_budget: int, clock: Callable[[], float] = time.perf_counter,
                 verbose: bool = False, max_split: int = 0):
        self.ex = executor
        self.verbose = verbose
        self.max_split = int(max_split)
        self.budget = int(mem_budget)
        self.clock = clock
        self.cv = threading.Condition()
        self.used = 0
        self.max_used = 0
        self.active: Dict[Any, List[Any]] = {}     # class -> [(record, handle, request)]
        self.busy: Dict[Any, bool] = {}
        self.errors: List[str] = []

    # -------------------------------------------------------------- workers
    def _worker(self, k, t0, stop):
        while True:
            with self.cv:
                while not self.active.get(k) and not stop.is_set():
                    self.cv.wait(0.05)
                if stop.is_set() and not self.active.get(k):
                    return
                members = list(self.active[k])
                self.busy[k] = True
            handles = [m[1] for m in members]
            parts = [m[0].parts[0] for m in members]
            dEs = [m[2].workload.dE(m[0].done_inc + 1) * f for m, (f, _) in zip(members, parts)]
            ckpts = [None] * len(members)
            if self.max_split > 0:
                try:
                    ckpts = [self.ex.checkpoint(h) for h in handles]
                except Exception as e:   # no checkpoint: the step runs without the split fallback
                    self.errors.append(f"checkpoint failed: {e!r}")
                    ckpts = [None] * len(members)
            try:
                res = self.ex.step(k, handles, dEs)
            except Exception as e:  # the whole step failed: fail its members only
                res = [{"ok": False, "Sigma": [0.0] * 6, "cg": 0, "error": repr(e)} for _ in members]
            # members whose sub-step failed and may be split: restored before
            # the next step (this thread owns the class's members between steps)
            for (rec, h, req), r, (f, depth), ck in zip(members, res, parts, ckpts):
                if r["ok"] or ck is None or depth >= self.max_split:
                    continue
                try:
                    self.ex.restore(h, ck)
                    r["split"] = True
                except Exception as e:
                    r["error"] = f"{r.get('error', '')}; restore failed: {e!r}"
            now = self.clock() - t0
            finished = []
            with self.cv:
                for (rec, h, req), r, (f, depth) in zip(members, res, parts):
                    rec.cg_iters += int(r.get("cg", 0))
                    if not r["ok"]:
                        if r.get("split"):
                            rec.parts[0:1] = [(0.5 * f, depth + 1), (0.5 * f, depth + 1)]
                            rec.splits += 1
                            continue
                        rec.status, rec.error, rec.finished = "failed", r.get("error", ""), now
                        finished.append((rec, h))
                        continue
                    rec.parts.pop(0)
                    if rec.parts:
                        continue             # more sub-steps of this increment
                    rec.parts = [(1.0, 0)]
                    rec.sigma.append(list(r["Sigma"]))
                    rec.done_inc += 1
                    if rec.done_inc == rec.n_inc:
                        rec.status, rec.finished = "ok", now
                        finished.append((rec, h))
                done_ids = {id(rec) for rec, _ in finished}
                self.active[k] = [m for m in self.active[k] if id(m[0]) not in done_ids]
                self.busy[k] = False
            for rec, h in finished:
                if self.verbose:
                    why = f" in increment {rec.done_inc + 1} of {rec.n_inc}: {rec.error}" if rec.status == "failed" else ""
                    print(f"serve: request {rec.rid} {rec.status} shape {rec.shape} {rec.precision} "
                          f"latency {rec.latency:.3f} s{why}", flush=True)
                try:
                    self.ex.release(h)
                finally:
                    with self.cv:
                        self.used -= rec.footprint
                        self.cv.notify_all()

    # ------------------------------------------------------------------ run
    def run(self, requests: Sequence[Any], poll: float = 0.002) -> List[Record]:
        reqs = sorted(requests, key=lambda r: r.arrival)
        recs = {}
        pending = deque()
        for q in reqs:
            w = q.workload
            rec = Record(q.rid, q.arrival, w.precision, tuple(w.shape), w.n_inc, int(self.ex.footprint(q)))
            recs[q.rid] = rec
            pending.append(q)
        stop = threading.Event()
        workers: Dict[Any, threading.Thread] = {}
        t0 = self.clock()
        while pending:
            now = self.clock() - t0
            with self.cv:
                while pending and pending[0].arrival <= now:
                    q = pending[0]
                    rec = recs[q.rid]
                    if rec.footprint > self.budget:
                        rec.status, rec.error, rec.finished = "rejected", "larger than the memory budget", now
                        pending.popleft()
                        continue
                    if self.used + rec.footprint > self.budget:
                        break                      # FIFO: wait for memory
                    self.used += rec.footprint     # reserve before allocating
                    self.max_used = max(self.max_used, self.used)
                    self.cv.release()
                    try:
                        h = self.ex.admit(q)
                    except MemoryError as e:
                        self.cv.acquire()
                        self.used -= rec.footprint
                        self.errors.append(f"admission of {q.rid} deferred: {e}")
                        break                      # retry when something finishes
                    except Exception as e:
                        self.cv.acquire()
                        self.used -= rec.footprint
                        rec.status, rec.error, rec.finished = "failed", repr(e), self.clock() - t0
                        pending.popleft()
                        continue
                    self.cv.acquire()
                    pending.popleft()
                    rec.admitted = self.clock() - t0
                    rec.status = "active"
                    k = self.ex.klass(q)
                    self.active.setdefault(k, []).append((rec, h, q))
                    if k not in workers:
                        th = threading.Thread(target=self._worker, args=(k, t0, stop), daemon=True)
                        workers[k] = th
                        th.start()
                    self.cv.notify_all()
                # sleep until the next arrival, or until a completion frees memory
                if pending:
                    head = recs[pending[0].rid]
                    if self.used + head.footprint > self.budget:
                        wait = 0.05                       # woken by a completion
                    else:
                        wait = min(max(pending[0].arrival - (self.clock() - t0), 0.0), 0.05)
                    if wait > 0:
                        self.cv.wait(wait)
        # drain
        with self.cv:
            while any(self.active.get(k) for k in self.active):
                self.cv.wait(0.05)
        stop.set()
        for th in workers.values():
            th.join()
        return [recs[q.rid] for q in reqs]


def summarize(records: Sequence[Record]) -> dict:
    ok = [r for r in records if r.status == "ok"]
    lat = np.array([r.latency for r in ok]) if ok else np.array([np.nan])
    t_end = max((r.finished for r in records if r.finished is not None), default=0.0)
    t_start = min((r.arrival for r in records), default=0.0)
    vox_cg = sum(r.cg_iters * int(np.prod(r.shape)) for r in ok)
    return {"requests": len(records), "ok": len(ok),
            "failed": sum(r.status == "failed" for r in records),
            "rejected": sum(r.status == "rejected" for r in records),
            "p50_latency_s": float(np.percentile(lat, 50)), "p99_latency_s": float(np.percentile(lat, 99)),
            "mean_latency_s": float(np.mean(lat)),
            "throughput_req_s": len(ok) / max(t_end - t_start, 1e-9),
            "voxel_cg_iters_per_s": vox_cg / max(t_end - t_start, 1e-9),
            "makespan_s": t_end - t_start,
            "split_increments": sum(r.splits for r in records),
            "failures": [{"rid": r.rid, "shape": list(r.shape), "precision": r.precision,
                          "increment": r.done_inc + 1, "of": r.n_inc, "error": r.error}
                         for r in records if r.status == "failed"]}


def main(argv=None):
    import argparse
    import json
    import os
    import sys
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import synth
    import torch

    ap = argparse.ArgumentParser(description="Poisson request stream through the continuous-batching server")
    ap.add_argument("--requests", type=int, default=24)
    ap.add_argument("--rate-factors", default="0.5,0.8,1.0",
                    help="arrival rates as fractions of the measured saturated throughput")
    ap.add_argument("--sizes", default="31,63,127,255")
    ap.add_argument("--weights", default="0.4,0.3,0.2,0.1")
    ap.add_argument("--budget-gb", type=float, default=0.0, help="0: 80 %% of free device memory")
    ap.add_argument("--max-split", type=int, default=3,
                    help="halvings allowed for an increment whose Newton iteration fails (0: fail the request)")
    args = ap.parse_args(argv)
    sizes = tuple(int(s) for s in args.sizes.split(","))
    weights = tuple(float(s) for s in args.weights.split(","))
    if len(weights) != len(sizes) or min(weights) < 0 or sum(weights) <= 0:
        ap.error("--weights needs one non-negative weight per size")
    weights = tuple(w / sum(weights) for w in weights)   # renormalised over the sizes given
    free, _ = torch.cuda.mem_get_info()
    budget = int(args.budget_gb * 1e9) if args.budget_gb > 0 else int(0.8 * free)
    ex = FftgExecutor()
    # saturated throughput: every request present at t = 0
    base = synth.serving_stream(args.requests, rate=1e9, sizes=sizes, weights=weights)
    for q in base:
        q.arrival = 0.0
    srv = Server(ex, budget, verbose=True, max_split=args.max_split)
    sat = summarize(srv.run(base))
    out = {"saturated": sat, "budget_bytes": budget, "max_used_bytes": srv.max_used, "runs": []}
    print(json.dumps({"saturated": sat}), flush=True)
    for f in [float(x) for x in args.rate_factors.split(",") if x]:
        lam = f * sat["throughput_req_s"]
        reqs = synth.serving_stream(args.requests, rate=lam, sizes=sizes, weights=weights)
        srv = Server(ex, budget, verbose=True, max_split=args.max_split)
        s = summarize(srv.run(reqs))
        s["rate_factor"], s["rate_req_s"] = f, lam
        out["runs"].append(s)
        print(json.dumps(s), flush=True)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
