"""Scheduling policy of the solve server on the host, with a simulated
backend (sleeps for the device work; a "solve" returns b / n so that every
job's columns can be traced through coalescing)."""
import threading
import time

import numpy as np
import pytest

from paper_1906_00874_amd.serve import Job, Server, summarize


class FakeBackend:
    def __init__(self, nbytes, t_factor, t_solve):
        self.nbytes, self.t_factor, self.t_solve = nbytes, t_factor, t_solve
        self.lock = threading.Lock()
        self.live = 0
        self.max_live = 0
        self.created = 0
        self.dropped = 0
        self.factored = []
        self.factoring = 0
        self.max_factoring = 0

    def size(self, key):
        return key

    def slot_bytes(self, key):
        return self.nbytes[key]

    def new_slot(self, key):
        with self.lock:
            self.created += 1
            self.live += self.nbytes[key]
            self.max_live = max(self.max_live, self.live)
        return {"key": key, "factored": False}

    def drop_slot(self, slot):
        if slot is not None:
            with self.lock:
                self.dropped += 1
                self.live -= self.nbytes[slot["key"]]

    def factor(self, slots):
        with self.lock:
            self.factoring += 1
            self.max_factoring = max(self.max_factoring, self.factoring)
        time.sleep(max(self.t_factor[s["key"]] for s in slots))
        for s in slots:
            s["factored"] = True
        with self.lock:
            self.factored.append(len(slots))
            self.factoring -= 1

    def solve(self, slot, bs):
        assert slot["factored"]
        cols = sum(b.shape[1] for b in bs)
        time.sleep(self.t_solve[slot["key"]] * (1 + cols / 64))
        return [b / slot["key"] for b in bs]


def rhs(job, n):
    return np.random.default_rng(1000 + job.jid).standard_normal((n, job.nrhs))


def make_jobs(n, keys, probs, rate, repeat_frac, seed, max_nrhs=64):
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, n))
    k = rng.choice(keys, size=n, p=probs)
    r = rng.integers(1, max_nrhs + 1, size=n)
    rep = rng.random(n) < repeat_frac
    return [Job(i, int(k[i]), int(r[i]), float(t[i]), repeat=bool(rep[i]), keep_x=True)
            for i in range(n)]


KEYS = [8, 16, 32, 64]
NBYTES = {8: 10, 16: 40, 32: 160, 64: 640}
TF = {8: 0.002, 16: 0.004, 32: 0.01, 64: 0.03}
TS = {8: 0.001, 16: 0.001, 32: 0.002, 64: 0.004}


def check_results(jobs):
    for j in jobs:
        assert not j.error, j.error
        assert j.done >= j.arrival
        assert j.x is not None and j.x.shape == (j.key, j.nrhs)
        np.testing.assert_array_equal(j.x, rhs(j, j.key) / j.key)


def test_all_jobs_served_and_results_routed():
    jobs = make_jobs(150, KEYS, [.4, .3, .2, .1], rate=400.0, repeat_frac=0.3, seed=5)
    be = FakeBackend(NBYTES, TF, TS)
    srv = Server(be, budget_bytes=4000, threads=4, batch_max_key=16, rhs=rhs, seed=1)
    out = srv.run(jobs)
    check_results(out)
    assert srv.peak_used <= 4000 and be.max_live <= 4000
    assert max(srv.solve_calls) <= 64
    assert sum(srv.solve_calls) == sum(j.nrhs for j in out)
    assert all(s.pins == 0 and not s.pending and not s.busy for s in srv.slots.values())
    assert any(j.repeat for j in out)
    s = summarize(out, KEYS)
    assert s["errors"] == 0 and s["jobs"] == 150 and s["p99_ms"] >= s["p50_ms"]


def test_coalescing_and_batching_under_a_burst():
    # everything arrives at once: the small factor jobs are batched and the
    # repeat jobs on one resident factor share solve calls
    first = [Job(i, 8, 4, 0.0, keep_x=True) for i in range(6)]
    later = [Job(100 + i, 8, 7, 0.05, repeat=True, keep_x=True) for i in range(20)]
    be = FakeBackend(NBYTES, TF, {8: 0.02})
    srv = Server(be, budget_bytes=10_000, threads=2, batch_max_key=16, batch_max=4, rhs=rhs)
    out = srv.run(first + later)
    check_results(out)
    assert max(srv.factor_launches) == 4 and sum(srv.factor_launches) == 6
    assert any(j.batched for j in out)
    # 20 repeat jobs of 7 columns: at most 9 per call, so calls of > 7 columns exist
    assert max(srv.solve_calls) > 7 and max(srv.solve_calls) <= 64


def test_small_budget_forces_eviction_and_queueing():
    jobs = make_jobs(60, KEYS, [.25, .25, .25, .25], rate=1000.0, repeat_frac=0.2, seed=9)
    be = FakeBackend(NBYTES, TF, TS)
    srv = Server(be, budget_bytes=700, threads=3, batch_max_key=16, rhs=rhs)
    out = srv.run(jobs)
    check_results(out)
    assert srv.peak_used <= 700 and be.max_live <= 700
    assert srv.evictions > 0 and be.dropped == srv.evictions


def test_budget_below_one_slot_is_an_error():
    be = FakeBackend(NBYTES, TF, TS)
    srv = Server(be, budget_bytes=100, rhs=rhs)
    with pytest.raises(ValueError):
        srv.run([Job(0, 64, 1, 0.0)])


def test_repeat_without_resident_factor_becomes_factor_job():
    be = FakeBackend(NBYTES, TF, TS)
    srv = Server(be, budget_bytes=10_000, rhs=rhs)
    out = srv.run([Job(0, 16, 3, 0.0, repeat=True, keep_x=True)])
    check_results(out)
    assert srv.fallback_repeats == 1 and not out[0].repeat


@pytest.mark.parametrize("cap", [1, 3])
def test_factor_tasks_in_flight_are_capped(cap):
    jobs = make_jobs(80, KEYS, [.25, .25, .25, .25], rate=2000.0, repeat_frac=0.2, seed=4)
    be = FakeBackend(NBYTES, TF, TS)
    srv = Server(be, budget_bytes=5000, threads=4, batch_max_key=16, rhs=rhs,
                 max_factor_tasks=cap)
    out = srv.run(jobs)
    check_results(out)
    assert be.max_factoring <= cap
