"""Model of the dataflow executor's scheduling protocol, run on the CPU with
random interleavings (no GPU).

The persistent executor (`df_run` in csrc/kernels.hip) takes tickets on a
FIFO ring of ready ops; an op's workgroup decrements its successors'
in-degrees, keeps the lowest ready position among the first NT successors
and runs it next without the ring, pushes the other ready ones (reserving a
slot, then storing the op), and counts the op as finished.  A workgroup
whose ticket is never filled (kept ops bypass the ring) leaves once every
op has finished.  This model executes that protocol one shared-memory step
at a time under a random scheduler and checks, on random DAGs and on the
dependency graph of a real factor schedule, that every op runs exactly
once, only after all of its predecessors, that the ring never overflows and
that every worker leaves.  It also checks that the exit on the finished
counter is needed: without it, a worker holding an unfilled ticket waits
forever once an op has been kept."""
import random

import numpy as np
import pytest


class Hang(Exception):
    pass


def simulate(succ, workers, chunk, seed, finished_exit=True, max_steps=3_000_000):
    rng = random.Random(seed)
    n = len(succ)
    indeg = [0] * n
    for u in range(n):
        for v in succ[u]:
            indeg[v] += 1
    ready0 = [u for u in range(n) if indeg[u] == 0]
    ring = [-1] * n
    for i, u in enumerate(ready0):
        ring[i] = u
    st = {"head": 0, "tail": len(ready0), "finished": 0}
    remaining_preds = list(indeg)
    runs = [0] * n

    def worker():
        nxt = -1
        while True:
            v, nxt = nxt, -1
            if v < 0:
                s = st["head"]
                st["head"] += 1
                yield
                if s < n:
                    while True:
                        v = ring[s]
                        yield
                        if v >= 0:
                            break
                        if finished_exit and st["finished"] >= n:
                            break
                if v < 0:
                    return
            assert remaining_preds[v] == 0, f"op {v} ran before a predecessor"
            runs[v] += 1
            yield
            readyl = []
            for pos, t in enumerate(succ[v]):
                indeg[t] -= 1
                remaining_preds[t] -= 1
                if indeg[t] == 0:
                    readyl.append((pos, t))
                yield
            first = [x for x in readyl if x[0] < chunk]
            keep = min(first) if first else None
            for pos, t in readyl:
                if keep is not None and pos == keep[0]:
                    continue
                slot = st["tail"]
                st["tail"] += 1
                yield
                assert slot < n, "ring overflow"
                ring[slot] = t
                yield
            if keep is not None:
                nxt = keep[1]
            st["finished"] += 1
            yield

    gens = [worker() for _ in range(workers)]
    alive = list(range(workers))
    steps = 0
    while alive:
        w = rng.choice(alive)
        try:
            next(gens[w])
        except StopIteration:
            alive.remove(w)
        steps += 1
        if steps > max_steps:
            raise Hang(f"no progress after {steps} steps")
    assert runs == [1] * n, "an op ran twice or never"
    return st


def random_dag(seed, n, maxsucc):
    rng = random.Random(seed)
    succ = []
    for u in range(n):
        later = list(range(u + 1, n))
        succ.append(sorted(rng.sample(later, min(len(later), rng.randint(0, maxsucc)))))
    return succ


@pytest.mark.parametrize("seed", range(60))
def test_random_dags(seed):
    rng = random.Random(1000 + seed)
    n = rng.randint(1, 160)
    succ = random_dag(seed, n, rng.randint(0, 10))
    simulate(succ, workers=rng.randint(1, 9), chunk=rng.randint(1, 6), seed=seed)


def test_factor_schedule_graph():
    """The dependency graph of a real factor schedule (n = 1280, leaf 32),
    as the planner emits it (CSR successors in schedule order)."""
    import paper_1906_00874_amd as P
    from hlu_inputs import icosphere
    xyz, area = icosphere(3)
    h = P.HLU(xyz, area, device="cpu", assemble=False, leaf=32, eta=2.0, eps=1e-6, cap=32,
              precision=P.PREC_MIXED, max_nrhs=2)
    off, su = h.schedule_graph(0)
    n = len(off) - 1
    succ = [sorted(int(x) for x in su[off[i]:off[i + 1]]) for i in range(n)]
    assert n > 1000 and sum(len(s) for s in succ) > n
    for seed in range(3):
        simulate(succ, workers=16, chunk=256, seed=seed, max_steps=20_000_000)


def test_exit_on_finished_counter_is_needed():
    """A chain 0 -> 1 -> 2: every op is kept by its predecessor's worker, so
    no ticket but the first is ever filled; without the exit on the finished
    counter the other workers wait forever."""
    succ = [[1], [2], []]
    simulate(succ, workers=3, chunk=4, seed=0)
    with pytest.raises(Hang):
        simulate(succ, workers=3, chunk=4, seed=0, finished_exit=False, max_steps=200_000)
