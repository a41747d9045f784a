"""Continuous-batching solve server on one GPU: a host scheduler over the
C-ABI (no arithmetic here: every factorisation and solve runs in the
library's kernels).

A job asks for x = A^{-1} b (nrhs right-hand sides) for the matrix of one
size class.  A *factor* job takes a fresh copy of the pre-assembled
H-matrix of its size, factors it and solves; a *repeat* job solves with a
factor that is already resident, chosen when it arrives.  The server

* admits factor jobs while the device bytes of their slots (one bound
  handle per slot, `hlu_required_bytes`) fit the HBM budget, first in first
  out but letting a later job pass one that does not fit yet, and evicts
  the least recently used idle resident factors to make room;
* keeps factored matrices resident in their slots for repeat jobs (a slot
  with waiting repeat jobs is pinned);
* coalesces the waiting right-hand sides of one resident factor into one
  solve call of at most `max_nrhs` columns (the library refines every
  column on its own, so a column's result does not depend on its
  companions);
* factors the small matrices admitted together by one batched persistent
  launch (`hlu_batch_*`), larger ones alone, each slot on a stream of its
  own, from a pool of worker threads (the C calls release the interpreter
  lock).

The device side sits behind a backend object so that the policy can be
exercised on the host with a simulated backend.
"""
from __future__ import annotations

import collections
import math
import queue
import threading
import time
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Job:
    jid: int
    key: int                  # size class (number of unknowns)
    nrhs: int
    arrival: float            # seconds after the start of the run
    repeat: bool = False      # solve with a resident factor
    keep_x: bool = False      # keep the solution (host copy) for checking
    # filled in by the server
    slot: int = -1
    batched: bool = False
    admitted: float = math.nan
    done: float = math.nan
    x: object = None
    b: object = None
    error: str = ""

    @property
    def latency(self):
        return self.done - self.arrival


@dataclass
class Slot:
    sid: int
    key: int
    nbytes: int
    handle: object = None     # backend object (created by the first task)
    busy: bool = False
    factored: bool = False
    pins: int = 0             # repeat jobs waiting for this factor
    pending: collections.deque = field(default_factory=collections.deque)
    last_use: float = 0.0


class Server:
    """Runs a list of jobs against `backend` (see `GpuBackend`)."""

    def __init__(self, backend, budget_bytes, max_nrhs=64, threads=4, batch_max_key=5120,
                 batch_max=16, seed=0, rhs=None, max_factor_tasks=2):
        self.be = backend
        self.budget = int(budget_bytes)
        self.max_nrhs = int(max_nrhs)
        self.threads = int(threads)
        self.batch_max_key = int(batch_max_key)
        self.batch_max = int(batch_max)
        self.rng = np.random.default_rng(seed)
        self.rhs = rhs                      # rhs(job, n) -> host array (n, nrhs)
        # factor tasks in flight at most (admission waits beyond that, so
        # the solves that complete jobs never queue behind many factors)
        self.max_factor_tasks = max(1, int(max_factor_tasks))
        self.slots = {}
        self.used = 0
        self.peak_used = 0
        self.next_sid = 0
        self.solve_calls = []               # columns per solve call
        self.factor_launches = []           # matrices per factor launch
        self.evictions = 0
        self.fallback_repeats = 0

    # -- slot bookkeeping (dispatcher thread only) ------------------------
    def _free_slot(self, key):
        """An idle, unpinned slot of this size with nothing waiting (least
        recently used first; empty slots before resident factors)."""
        best = None
        for s in self.slots.values():
            if s.key != key or s.busy or s.pins or s.pending:
                continue
            rank = (s.factored, s.last_use)
            if best is None or rank < (best.factored, best.last_use):
                best = s
        return best

    def _evict_for(self, nbytes):
        """Drop idle, unpinned slots (least recently used first) until
        nbytes fit; False if they cannot."""
        idle = sorted((s for s in self.slots.values()
                       if not s.busy and not s.pins and not s.pending),
                      key=lambda s: s.last_use)
        room = self.budget - self.used
        victims = []
        for s in idle:
            if room >= nbytes:
                break
            victims.append(s)
            room += s.nbytes
        if room < nbytes:
            return False
        for s in victims:
            del self.slots[s.sid]
            self.used -= s.nbytes
            self.be.drop_slot(s.handle)
            self.evictions += 1
        return True

    def _take_slot(self, key):
        s = self._free_slot(key)
        if s is not None:
            return s
        nbytes = self.be.slot_bytes(key)
        if nbytes > self.budget:
            raise ValueError(f"a slot of size {key} ({nbytes} B) exceeds the budget")
        if self.used + nbytes > self.budget and not self._evict_for(nbytes):
            return None
        s = Slot(self.next_sid, key, nbytes)
        self.next_sid += 1
        self.slots[s.sid] = s
        self.used += nbytes
        self.peak_used = max(self.peak_used, self.used)
        return s

    # -- tasks (worker threads) -------------------------------------------
    def _task_factor(self, group):
        """group: [(slot, job)], factored together when more than one."""
        try:
            for s, _ in group:
                if s.handle is None:
                    s.handle = self.be.new_slot(s.key)
            self.be.factor([s.handle for s, _ in group])
            return ("factored", group, "")
        except Exception as e:  # reported per job
            return ("factored", group, f"{type(e).__name__}: {e}")

    def _task_solve(self, slot, jobs, now_fn):
        try:
            bs = []
            for j in jobs:
                if j.b is None:
                    j.b = self.rhs(j, self.be.size(slot.key))
                bs.append(j.b)
            xs = self.be.solve(slot.handle, bs)
            t = now_fn()
            for j, x in zip(jobs, xs):
                j.done = t
                j.x = x if j.keep_x else None
                j.b = None if not j.keep_x else j.b
            return ("solved", (slot, jobs), "")
        except Exception as e:
            t = now_fn()
            for j in jobs:
                j.done = t
            return ("solved", (slot, jobs), f"{type(e).__name__}: {e}")

    # -- main loop ---------------------------------------------------------
    def run(self, jobs, progress=None):
        """Serves `jobs` (their arrival times are seconds after the call);
        progress(done, total), if given, is called after every completion."""
        jobs = sorted(jobs, key=lambda j: j.arrival)
        t0 = time.perf_counter()
        now = lambda: time.perf_counter() - t0  # noqa: E731
        done_q = queue.Queue()
        pool = ThreadPoolExecutor(max_workers=self.threads)
        waiting = collections.deque()         # factor jobs not yet admitted
        nxt = 0
        remaining = len(jobs)
        in_flight = 0
        factor_tasks = 0

        def submit(fn, *a):
            nonlocal in_flight, factor_tasks
            in_flight += 1
            factor_tasks += fn == self._task_factor
            fut = pool.submit(fn, *a)
            fut.add_done_callback(lambda f: done_q.put(f.result()))

        try:
            while remaining:
                t = now()
                # arrivals up to now
                while nxt < len(jobs) and jobs[nxt].arrival <= t:
                    j = jobs[nxt]
                    nxt += 1
                    if j.repeat:
                        resident = [s for s in self.slots.values() if s.factored]
                        if resident:
                            s = resident[int(self.rng.integers(len(resident)))]
                            j.key = s.key
                            j.slot = s.sid
                            j.admitted = t
                            s.pins += 1
                            s.pending.append(j)
                            continue
                        self.fallback_repeats += 1
                        j.repeat = False
                    waiting.append(j)
                # admission of factor jobs (FIFO, later ones may pass): a
                # large matrix takes a factor task of its own, the small ones
                # admitted now share one batched task
                small = []
                budget_tasks = self.max_factor_tasks - factor_tasks
                for j in list(waiting):
                    big = j.key > self.batch_max_key
                    if not big and len(small) >= self.batch_max:
                        continue
                    need = 1 if big or not small else 0
                    if need > budget_tasks:
                        continue
                    s = self._take_slot(j.key)
                    if s is None:
                        continue
                    waiting.remove(j)
                    budget_tasks -= need
                    s.busy = True
                    s.factored = False
                    j.slot = s.sid
                    j.admitted = t
                    if big:
                        self.factor_launches.append(1)
                        submit(self._task_factor, [(s, j)])
                    else:
                        small.append((s, j))
                for q in range(0, len(small), self.batch_max):
                    grp = small[q:q + self.batch_max]
                    for s, j in grp:
                        j.batched = len(grp) > 1
                    self.factor_launches.append(len(grp))
                    submit(self._task_factor, grp)
                # coalesced solves on resident, idle slots
                for s in self.slots.values():
                    if s.busy or not s.factored or not s.pending:
                        continue
                    take, cols = [], 0
                    while s.pending and cols + s.pending[0].nrhs <= self.max_nrhs:
                        j = s.pending.popleft()
                        take.append(j)
                        cols += j.nrhs
                    if not take:   # a job wider than max_nrhs
                        j = s.pending.popleft()
                        j.error, j.done = "nrhs exceeds max_nrhs", now()
                        if j.repeat:
                            s.pins -= 1
                        remaining -= 1
                        continue
                    s.busy = True
                    self.solve_calls.append(cols)
                    submit(self._task_solve, s, take, now)
                if not remaining:
                    break
                # wait for a completion or the next arrival
                timeout = None
                if nxt < len(jobs):
                    timeout = max(0.0, jobs[nxt].arrival - now())
                if in_flight == 0 and timeout is None:
                    # nothing running and nothing arriving while jobs wait:
                    # the budget cannot hold what they need
                    raise RuntimeError(f"{remaining} jobs cannot be admitted within the budget")
                try:
                    msg = done_q.get(timeout=timeout)
                except queue.Empty:
                    msg = None
                while msg is not None:
                    in_flight -= 1
                    kind, payload, err = msg
                    tt = now()
                    if kind == "factored":
                        factor_tasks -= 1
                        for s, j in payload:
                            s.busy = False
                            s.last_use = tt
                            if err:
                                j.error, j.done = err, tt
                                remaining -= 1
                            else:
                                s.factored = True
                                s.pending.appendleft(j)   # its own right-hand sides
                    else:
                        s, js = payload
                        s.busy = False
                        s.last_use = tt
                        for j in js:
                            if j.repeat:
                                s.pins -= 1
                            if err:
                                j.error = err
                        remaining -= len(js)
                        if progress is not None:
                            progress(len(jobs) - remaining, len(jobs))
                    try:
                        msg = done_q.get_nowait()
                    except queue.Empty:
                        msg = None
        finally:
            pool.shutdown(wait=True)
        return jobs


def summarize(jobs, keys):
    """Latency percentiles (ms) per size class and overall, and throughput."""
    ok = [j for j in jobs if not j.error]
    out = {"jobs": len(jobs), "errors": len(jobs) - len(ok)}
    if not ok:
        return out
    span = max(j.done for j in ok) - min(j.arrival for j in ok)
    out["jobs_per_s"] = len(ok) / span if span > 0 else math.inf
    lat = np.array([j.latency for j in ok]) * 1e3
    out["p50_ms"] = float(np.percentile(lat, 50))
    out["p99_ms"] = float(np.percentile(lat, 99))
    per = {}
    for k in keys:
        lk = np.array([j.latency for j in ok if j.key == k]) * 1e3
        if len(lk):
            per[str(k)] = {"jobs": int(len(lk)), "p50_ms": float(np.percentile(lk, 50)),
                           "p99_ms": float(np.percentile(lk, 99))}
    out["per_size"] = per
    out["repeat_jobs"] = sum(j.repeat for j in ok)
    return out


class GpuBackend:
    """Slots are clones of one pre-assembled master handle per size class,
    each with its own buffer and stream."""

    def __init__(self, masters, workers=None, device="cuda"):
        import torch
        from .binding import Batch
        self.torch = torch
        self.Batch = Batch
        self.masters = dict(masters)          # key -> assembled HLU
        self.workers = dict(workers or {})    # key -> dataflow workgroups (0: all)
        self.device = device
        self._lock = threading.Lock()

    def size(self, key):
        return self.masters[key].n

    def slot_bytes(self, key):
        return self.masters[key].required_bytes + 256

    def new_slot(self, key):
        torch = self.torch
        st = torch.cuda.Stream(device=self.device)
        with torch.cuda.stream(st):
            h = self.masters[key].clone(bind=True, stream=st)
        h.set_workers(self.workers.get(key, 0))
        st.synchronize()
        return {"h": h, "stream": st, "fresh": True, "key": key}

    def drop_slot(self, slot):
        if slot is not None:
            slot["stream"].synchronize()
            slot["h"] = None

    def factor(self, slots):
        if len(slots) == 1:
            s = slots[0]
            if not s["fresh"]:
                s["h"].reset(stream=s["stream"])
            s["fresh"] = False
            s["h"].factor(stream=s["stream"])
            s["h"].sync(stream=s["stream"])
            return
        st = slots[0]["stream"]
        for s in slots:
            s["stream"].synchronize()
            if not s["fresh"]:
                s["h"].reset(stream=st)
            s["fresh"] = False
        b = self.Batch([s["h"] for s in slots], device=self.device)
        b.factor(stream=st)
        b.sync(stream=st)
        for s in slots:
            s["h"].sync(stream=st)

    def solve(self, slot, bs):
        torch = self.torch
        h, st = slot["h"], slot["stream"]
        cols = [b.shape[1] for b in bs]
        with torch.cuda.stream(st):
            B = torch.from_numpy(np.ascontiguousarray(np.concatenate(bs, axis=1).T)).to(
                self.device, non_blocking=False)
            X = torch.empty_like(B)
            h.solve_cm(B, X, stream=st)
            st.synchronize()
            h.sync(stream=st)
            x = X.cpu().numpy().T
        out, c = [], 0
        for k in cols:
            out.append(np.ascontiguousarray(x[:, c:c + k]))
            c += k
        return out
