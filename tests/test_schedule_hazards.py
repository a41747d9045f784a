"""Memory hazards of the static schedules (host logic, no GPU).

Every op of a schedule reads and writes column segments of panels in the
device buffer (the operand roles of each op type are those of the op table:
leaf factorisation, leaf solves, panel products, truncations, dense updates,
zeroing, the leaf inverses, and the solve's H-matvec updates and inverse
applications).  Two ops that touch overlapping
bytes, one of them writing, must be ordered: for the wave executor they must
sit in different waves, in the right order; for the dataflow executor a path
of dependency edges must lead from the earlier to the later one.  The check
replays each schedule in its order over elementary byte intervals, with the
panels taken at their full static capacity, and is run with and without
reuse of the scratch region as a ring.
"""
import numpy as np
import pytest

import paper_1906_00874_amd as P
from hlu_inputs import icosphere

OP_GETRF, OP_TRSM_L, OP_TRSM_UT, OP_TRSM_U, OP_PGEMM, OP_TRUNC, OP_ADDD, OP_ZERO, \
    OP_MVT, OP_MVROW, OP_TRINV, OP_INVAPPLY = range(12)


def _segs(r, write, out):
    if r["kind"] == 1 or r["rows"] <= 0 or r["cols"] <= 0:
        return
    es = 8 if r["dt"] == 0 else 4
    ptr, ld, rows, cols = int(r["ptr"]), int(r["ld"]), int(r["rows"]), int(r["cols"])
    if r["trans"]:
        rows, cols = cols, rows
    for j in range(cols):
        out.append((ptr + j * ld * es, ptr + (j * ld + rows) * es, write))
    if r["rankp"]:
        out.append((int(r["rankp"]), int(r["rankp"]) + 4, write and False))


def accesses(o, terms):
    """(lo, hi, write) byte ranges of one op."""
    t, p, a = int(o["type"]), o["p"], []
    if t == OP_GETRF:
        _segs(p[0], True, a)
        a.append((int(p[1]["ptr"]), int(p[1]["ptr"]) + 4 * int(p[0]["rows"]), True))
    elif t in (OP_TRSM_L, OP_TRSM_UT, OP_TRSM_U):
        _segs(p[0], False, a)
        _segs(p[1], True, a)
        if t == OP_TRSM_L:
            a.append((int(p[2]["ptr"]), int(p[2]["ptr"]) + 4 * int(p[0]["rows"]), False))
    elif t == OP_PGEMM:
        _segs(p[0], False, a)
        if o["i0"] == 1:
            _segs(p[1], False, a)
        _segs(p[2], False, a)
        _segs(p[3], True, a)
    elif t == OP_TRUNC:
        _segs(p[0], True, a)
        _segs(p[1], True, a)
        a.append((int(p[0]["rankp"]), int(p[0]["rankp"]) + 4, True))
        for q in range(int(o["i0"]), int(o["i0"]) + int(o["i1"])):
            _segs(terms[q]["X"], False, a)
            _segs(terms[q]["Y"], False, a)
    elif t == OP_ADDD:
        _segs(p[0], True, a)
        _segs(p[1], False, a)
        _segs(p[2], False, a)
    elif t == OP_ZERO:
        _segs(p[0], True, a)
    elif t == OP_MVT:
        _segs(p[0], False, a)
        _segs(p[2], False, a)
        _segs(p[3], True, a)
        if o["i2"] == 1:   # accumulates onto p3
            _segs(p[3], False, a)
    elif t == OP_MVROW:
        _segs(p[3], True, a)
        if o["i2"] == 1:
            _segs(p[0], False, a)
        if int(o["i0"]) == -1:   # one term carried in the op
            _segs(p[1], False, a)
            _segs(p[2], False, a)
        else:
            for q in range(int(o["i0"]), int(o["i0"]) + int(o["i1"])):
                _segs(terms[q]["X"], False, a)
                _segs(terms[q]["Y"], False, a)
    elif t == OP_TRINV:
        _segs(p[0], False, a)
        a.append((int(p[1]["ptr"]), int(p[1]["ptr"]) + 4 * int(p[0]["rows"]), False))
        _segs(p[2], True, a)
        _segs(p[3], True, a)
    elif t == OP_INVAPPLY:
        _segs(p[0], False, a)
        _segs(p[1], True, a)
    else:
        raise AssertionError(f"unknown op type {t}")
    return a


def hazards(h, which):
    """Unordered conflicting pairs (wave order, dependency paths)."""
    ops, waves, terms = h.schedule_ops(which)
    off, su = h.schedule_graph(which)
    n = len(ops)
    assert n > 0 and np.all(np.diff(waves) >= 0)
    acc = [accesses(ops[k], terms) for k in range(n)]
    bounds = np.unique(np.array([x for a in acc for (lo, hi, _) in a for x in (lo, hi)],
                                dtype=np.int64))
    # ancestors of every op as an integer bitset (edges run forward)
    preds = [[] for _ in range(n)]
    for u in range(n):
        for v in su[off[u]:off[u + 1]]:
            assert v > u, "dependency edge against the schedule order"
            preds[v].append(u)
    anc = [0] * n
    for v in range(n):
        m = 0
        for u in preds[v]:
            m |= anc[u] | (1 << u)
        anc[v] = m
    last_w = np.full(len(bounds), -1, dtype=np.int64)
    readers = [[] for _ in range(len(bounds))]
    bad_wave, bad_dag = [], []

    def need(a, b):
        if a < 0 or a == b:
            return
        if not waves[a] < waves[b]:
            bad_wave.append((a, b))
        if not (anc[b] >> a) & 1:
            bad_dag.append((a, b))

    for k in range(n):
        rd = [(lo, hi) for (lo, hi, w) in acc[k] if not w]
        wr = [(lo, hi) for (lo, hi, w) in acc[k] if w]
        for lo, hi in rd:
            for iv in range(np.searchsorted(bounds, lo), np.searchsorted(bounds, hi)):
                need(int(last_w[iv]), k)
                readers[iv].append(k)
        for lo, hi in wr:
            for iv in range(np.searchsorted(bounds, lo), np.searchsorted(bounds, hi)):
                need(int(last_w[iv]), k)
                for r in readers[iv]:
                    need(r, k)
                last_w[iv] = k
                readers[iv] = []
    return bad_wave, bad_dag


@pytest.mark.parametrize("ring", [0, 32768])
def test_factor_and_solve_schedules_are_hazard_free(ring):
    xyz, area = icosphere(2)
    h = P.HLU(xyz, area, assemble=False, leaf=16, eta=2.0, eps=1e-6, cap=16,
              precision=P.PREC_MIXED, max_nrhs=2, cap_mv=0, refine_tol=0.0,
              scratch_cap=ring)
    st = h.stats()
    if ring:
        assert st["bytes_scratch"] <= ring
    for which in (0, 1):
        bad_wave, bad_dag = hazards(h, which)
        assert not bad_wave, f"schedule {which}: unordered in waves {bad_wave[:5]}"
        assert not bad_dag, f"schedule {which}: no dependency path {bad_dag[:5]}"


def test_scratch_ring_shrinks_scratch():
    xyz, area = icosphere(2)
    kw = dict(assemble=False, leaf=16, eta=2.0, eps=1e-6, cap=16, precision=P.PREC_MIXED,
              max_nrhs=1, cap_mv=0, refine_tol=0.0)
    full = P.HLU(xyz, area, scratch_cap=0, **kw).stats()["bytes_scratch"]
    ring = P.HLU(xyz, area, scratch_cap=32768, **kw).stats()["bytes_scratch"]
    assert ring <= 32768 < full


@pytest.mark.parametrize("operation", [0, 2])
def test_scratch_is_written_before_it_is_read(operation):
    """Without a ring the scratch panels are not zero-filled: the first panel
    product into each row range overwrites it.  Every scratch byte an op
    reads (at full static capacity) was written by an earlier op of the
    schedule, and there is no zeroing op at all; the H-LU plan and the
    inverse plan (identity and zero blocks) are both checked."""
    xyz, area = icosphere(2)
    h = P.HLU(xyz, area, assemble=False, leaf=16, eta=2.0, eps=1e-6, cap=16,
              precision=P.PREC_MIXED, max_nrhs=2, cap_mv=0, refine_tol=0.0, operation=operation)
    st = h.stats()
    lo_s, hi_s = st["offset_scratch"], st["offset_scratch"] + st["bytes_scratch"]
    ops, waves, terms = h.schedule_ops(0)
    assert not np.any(ops["type"] == OP_ZERO)
    assert np.any((ops["type"] == OP_PGEMM) & ((ops["i2"] & 1) == 1))
    acc = [accesses(ops[k], terms) for k in range(len(ops))]
    bounds = np.unique(np.array([x for a in acc for (lo, hi, _) in a for x in (lo, hi)]
                                + [lo_s, hi_s], dtype=np.int64))
    written = np.zeros(len(bounds), dtype=bool)
    unread = 0
    for k in range(len(ops)):
        for lo, hi, w in acc[k]:
            if w or hi <= lo_s or lo >= hi_s:
                continue
            a, b = np.searchsorted(bounds, lo), np.searchsorted(bounds, hi)
            unread += int((~written[a:b]).sum())
        for lo, hi, w in acc[k]:
            if w:
                written[np.searchsorted(bounds, lo):np.searchsorted(bounds, hi)] = True
    assert unread == 0


def test_solve_vtx_split_over_multi_leaf_sources():
    """A V^T X product whose source cluster has several leaves is emitted as
    two ops on the same T slot: the rows of every leaf but the one the sweep
    solves last (writing T), then that leaf's rows alone, accumulating
    (i2 = 1), ordered by a dependency path.  The two parts' rows of V (and of
    X) are adjacent, the accumulating one after the first in the forward
    sweep and before it in the backward sweep, and it covers one leaf."""
    xyz, area = icosphere(3)
    h = P.HLU(xyz, area, assemble=False, leaf=64, eta=2.0, eps=1e-5, cap=32,
              precision=P.PREC_MIXED, max_nrhs=4, cap_mv=64, eps_mv=1e-12, refine_tol=0.0)
    ops, waves, terms = h.schedule_ops(1)
    off, su = h.schedule_graph(1)
    n = len(ops)
    mvt = np.flatnonzero(ops["type"] == OP_MVT)
    acc = [k for k in mvt if ops["i2"][k] == 1]
    assert acc, "no multi-leaf source in this schedule"
    succ = [set(su[off[u]:off[u + 1]]) for u in range(n)]

    def reaches(u, v):
        seen, todo = {u}, [u]
        while todo:
            x = todo.pop()
            for y in succ[x]:
                if y == v:
                    return True
                if y not in seen and y < v:
                    seen.add(y)
                    todo.append(y)
        return False

    for k in acc:
        t = int(ops["p"][k, 3]["ptr"])
        rest = [r for r in mvt if r < k and ops["i2"][r] == 0 and int(ops["p"][r, 3]["ptr"]) == t]
        assert rest, f"accumulating product {k} without a first part"
        r = rest[-1]
        assert 0 < int(ops["p"][k, 0]["rows"]) <= 64
        assert int(ops["p"][k, 2]["rows"]) == int(ops["p"][k, 0]["rows"])
        assert int(ops["p"][r, 2]["rows"]) == int(ops["p"][r, 0]["rows"])
        assert reaches(r, k), f"no dependency path from {r} to {k}"
        for q in (0, 2):
            es = 8 if int(ops["p"][k, q]["dt"]) == 0 else 4
            pa, ra = int(ops["p"][k, q]["ptr"]), int(ops["p"][k, q]["rows"])
            pr, rr = int(ops["p"][r, q]["ptr"]), int(ops["p"][r, q]["rows"])
            assert pa == pr + rr * es or pr == pa + ra * es, (k, r, q)
