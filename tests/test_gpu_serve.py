"""Serving on the GPU: per-column refinement independence, clones of one
plan, and the continuous-batching server against alone runs (bitwise)."""
import sys

import numpy as np
import pytest

from hlu_inputs import icosphere, rhs_normal

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu-test]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    import paper_1906_00874_amd as P
    return P


KW = dict(leaf=32, eta=2.0, eps=1e-6, cap=32, eps_mv=1e-12, cap_mv=64, refine_tol=1e-10,
          refine_max_iter=10, max_nrhs=64)


def _solve(h, b, torch):
    bc = torch.tensor(np.ascontiguousarray(b.T), device="cuda")
    xc = torch.empty_like(bc)
    h.solve_cm(bc, xc)
    st, inf = h.sync(check=True)
    return xc.cpu().numpy().T, inf


def test_columns_refined_independently(P):
    import torch
    xyz, area = icosphere(3)
    h = P.HLU(xyz, area, precision=P.PREC_MIXED, **KW)
    h.set_executor(1)
    h.factor()
    h.sync()
    b = rhs_normal(3, h.n, 40)
    b[:, 7] *= 1e-3          # columns of very different scale share the call
    x_all, inf = _solve(h, b, torch)
    _say("coalesced 40 columns: iters", inf.iters, "eta", inf.eta_final)
    assert inf.eta_final <= 1e-10
    for j0, j1 in [(0, 1), (7, 8), (5, 12), (39, 40)]:
        xs, _ = _solve(h, np.ascontiguousarray(b[:, j0:j1]), torch)
        assert np.array_equal(xs, x_all[:, j0:j1]), (j0, j1)


def test_clone_matches_original(P):
    import torch
    xyz, area = icosphere(3)
    h = P.HLU(xyz, area, precision=P.PREC_MIXED, **KW)
    h.set_executor(1)
    c = h.clone(bind=True)
    c.set_workers(16)
    for q in (h, c):
        q.factor()
        q.sync()
    L0, U0 = h.export_factors()
    L1, U1 = c.export_factors()
    assert np.array_equal(L0, L1) and np.array_equal(U0, U1)
    b = rhs_normal(4, h.n, 3)
    x0, _ = _solve(h, b, torch)
    x1, _ = _solve(c, b, torch)
    assert np.array_equal(x0, x1)
    # the clone outlives the original handle (shared plan)
    del h
    c.reset()
    c.factor()
    c.sync()
    x2, _ = _solve(c, b, torch)
    assert np.array_equal(x2, x1)


def test_server_matches_alone_runs(P):
    import torch
    from paper_1906_00874_amd.serve import GpuBackend, Job, Server, summarize
    masters = {}
    for lv in (3, 4):
        xyz, area = icosphere(lv)
        m = P.HLU(xyz, area, precision=P.PREC_MIXED, **KW)
        m.set_executor(1)
        masters[m.n] = m
    rng = np.random.default_rng(21)
    jobs = []
    for i in range(24):
        key = 1280 if rng.random() < 0.6 else 5120
        jobs.append(Job(i, key, int(rng.integers(1, 33)), float(i) * 0.01,
                        repeat=bool(i >= 6 and rng.random() < 0.4), keep_x=True))

    def rhs(job, n):
        return rhs_normal(500 + job.jid, n, job.nrhs)

    be = GpuBackend(masters, workers={1280: 32, 5120: 64})
    srv = Server(be, budget_bytes=6 * max(m.required_bytes for m in masters.values()),
                 max_nrhs=64, threads=4, batch_max_key=5120, batch_max=8, seed=3, rhs=rhs)
    out = srv.run(jobs)
    s = summarize(out, [1280, 5120])
    _say("served", s, "launches", srv.factor_launches, "solve cols", srv.solve_calls)
    assert s["errors"] == 0, [j.error for j in out if j.error][:3]
    for j in out:
        h = masters[j.key].clone(bind=True)
        h.factor()
        h.sync()
        xa, _ = _solve(h, rhs(j, h.n), torch)
        assert np.array_equal(xa, j.x), (j.jid, j.key, j.repeat, j.batched)
        del h
