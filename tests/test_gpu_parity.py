"""Device path against the oracle (MI355X only, through the C-ABI)."""
import math
import os
import sys

import numpy as np
import pytest

import oracle as O
from hlu_inputs import icosphere, rhs_normal, rhs_uniform

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu-test]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1906_00874_amd as P
    return P


def _cm_blocks(torch, mats):
    """list of (b x b) numpy arrays -> device tensor (count, b, b) holding
    each block column-major (row q of the tensor slice = column q)."""
    arr = np.ascontiguousarray(np.stack([m.T for m in mats]))
    t = torch.tensor(arr, dtype=torch.float64, device="cuda").contiguous()
    assert t.is_contiguous()
    return t


# ---------------------------------------------------------------- leaf getrf
@pytest.mark.parametrize("b", [1, 2, 11, 31, 32, 33, 63, 64])
def test_getrf_batched_vs_oracle(P, b):
    import torch
    _say("getrf", b)
    rng = np.random.default_rng(b)
    mats = [rng.standard_normal((b, b)) for _ in range(7)]
    mats.append(np.abs(rng.standard_normal((b, b))) + np.eye(b) * b)   # diagonally dominant
    a = _cm_blocks(torch, mats)
    piv, info = P.getrf_batched(a)
    torch.cuda.synchronize()
    got = a.cpu().numpy()
    piv = piv.cpu().numpy()
    info = info.cpu().numpy()
    for q, m in enumerate(mats):
        ref = m.copy()
        rp, ri = O.getrf(ref)
        assert np.array_equal(piv[q], rp), q
        assert info[q] == ri
        # contraction disabled on both sides: the elimination is bit-exact
        assert np.array_equal(got[q].T, ref), (q, np.abs(got[q].T - ref).max())


def test_getrf_zero_pivot_and_singular(P):
    import torch
    m = np.array([[0.0, 1.0, 2.0], [0.0, 3.0, 4.0], [0.0, 5.0, 7.0]])
    z = np.zeros((3, 3))
    a = _cm_blocks(torch, [m, z])
    piv, info = P.getrf_batched(a)
    torch.cuda.synchronize()
    assert info.cpu().numpy().tolist() == [1, 1]
    assert piv.cpu().numpy()[0, 0] == 0


# ---------------------------------------------------------------- truncation
def _trunc_case(P, m, n, kc, kx, cap, eps, fixed=0, seed=0, decay=0.6, offset=False):
    import torch
    rng = np.random.default_rng(seed)
    U0 = rng.standard_normal((m, kc)) * decay ** np.arange(kc)
    V0 = rng.standard_normal((n, kc))
    X = rng.standard_normal((m, kx)) * decay ** np.arange(kx) * 0.3
    Y = rng.standard_normal((n, kx))
    Ud = torch.zeros((cap, m), dtype=torch.float64, device="cuda")
    Vd = torch.zeros((cap, n), dtype=torch.float64, device="cuda")
    Ud[:kc] = torch.tensor(U0.T, device="cuda")
    Vd[:kc] = torch.tensor(V0.T, device="cuda")
    Xd = torch.tensor(X.T.copy(), device="cuda")
    Yd = torch.tensor(Y.T.copy(), device="cuda")
    k = P.truncate_add(Ud, Vd, kc, Xd, Yd, cap, eps, fixed)
    torch.cuda.synchronize()
    Ug = Ud.cpu().numpy()[:k].T
    Vg = Vd.cpu().numpy()[:k].T
    rule = O.Rule(eps=eps, cap=cap, fixed=fixed)
    Uo, Vo = O.truncate(np.hstack([U0, -X]), np.hstack([V0, Y]), rule)
    D = U0 @ V0.T - X @ Y.T
    return k, Ug, Vg, Uo, Vo, D, rule


@pytest.mark.parametrize("m,n,kc,kx,eps", [(40, 30, 8, 8, 1e-6), (300, 200, 16, 16, 1e-6),
                                           (64, 65, 32, 32, 1e-5), (1, 9, 0, 3, 1e-6),
                                           (700, 90, 20, 24, 1e-8), (17, 5, 3, 30, 1e-6)])
def test_truncate_vs_oracle(P, m, n, kc, kx, eps):
    _say("truncate", m, n, kc, kx, eps)
    k, Ug, Vg, Uo, Vo, D, rule = _trunc_case(P, m, n, kc, kx, 32, eps, seed=m + n)
    ko = Uo.shape[1]
    nd = np.linalg.norm(D)
    # Eckart-Young: both are best approximations at the chosen rank; the
    # rank may differ by one when a singular value sits on the threshold
    assert abs(k - ko) <= 1
    sig = np.linalg.svd(D, compute_uv=False)
    tail = math.sqrt(float(np.sum(sig[k:] ** 2)))
    err = np.linalg.norm(D - Ug @ Vg.T)
    assert err <= max(eps * nd * 1.05, tail * 1.05 + 1e-12 * nd)
    if k == ko:
        assert np.linalg.norm(Ug @ Vg.T - Uo @ Vo.T) <= max(2 * eps * nd, 1e-11 * nd)


def test_truncate_fixed_rank_and_cap(P):
    k, Ug, Vg, Uo, Vo, D, _ = _trunc_case(P, 80, 70, 16, 16, 32, 0.0, fixed=8, seed=3, decay=0.8)
    assert k == 8
    sig = np.linalg.svd(D, compute_uv=False)
    assert np.linalg.norm(D - Ug @ Vg.T) == pytest.approx(math.sqrt(np.sum(sig[8:] ** 2)), rel=1e-6)
    k, Ug, Vg, Uo, Vo, D, _ = _trunc_case(P, 80, 70, 5, 20, 5, 1e-14, seed=4, decay=0.95)
    assert k == 5
    sig = np.linalg.svd(D, compute_uv=False)
    assert np.linalg.norm(D - Ug @ Vg.T) == pytest.approx(math.sqrt(np.sum(sig[5:] ** 2)), rel=1e-6)


@pytest.mark.parametrize("kx,eps", [(100, 1e-6), (64, 1e-5), (33, 1e-6)])
def test_truncate_multi_term_passes(P, kx, eps):
    """An update wider than the stack admits is added in several passes;
    each pass discards at most eps of the norm of its own sum (ranks stay
    below the capacity here, so no pass is capped)."""
    _say("truncate multi-term", kx, eps)
    k, Ug, Vg, Uo, Vo, D, rule = _trunc_case(P, 300, 250, 8, kx, 32, eps, seed=kx, decay=0.5)
    assert not any(l[3] for l in rule.log)
    nd = np.linalg.norm(D)
    passes = math.ceil(kx / 32)
    err = np.linalg.norm(D - Ug @ Vg.T)
    assert err <= passes * 1.5 * eps * nd + 1e-12 * nd
    # the rank is never below the single-shot optimum for the same tolerance
    assert k >= Uo.shape[1] - 1


# ---------------------------------------------------------------- H-LU
def _hlu(P, level, leaf, **kw):
    xyz, area = icosphere(level)
    _say("plan+assemble", level, leaf, kw)
    return xyz, area, P.HLU(xyz, area, leaf=leaf, eta=kw.pop("eta", 2.0), **kw)


def test_hlu_eta0_matches_block_lu(P):
    """eta = 0: every block dense; the device factors equal the oracle's
    dense block LU with leaf-local pivoting (pivots bit-equal)."""
    xyz, area = icosphere(2)
    _, _, h = _hlu(P, 2, 16, eta=0.0, eps=1e-6, kernel=P.KERNEL_POINT)
    h.factor()
    h.sync()
    Lg, Ug = h.export_factors()
    pg = h.export_pivots()
    H = O.HMatrix(xyz, area, 16, 0.0, O.Rule(eps=1e-6), reading=O.READING_POINT)
    A = H.to_dense()
    O.factor(H)
    Lo, Uo = O.factors_dense(H)
    for lf in H.leaves:
        blk = [b for b in O.leaves_of(H.block) if b.t is lf and b.s is lf][0]
        assert np.array_equal(pg[lf.off:lf.off + lf.size], blk.piv)
    sc = np.abs(A).max()
    assert np.abs(Lg - Lo).max() <= 1e-12 * sc
    assert np.abs(Ug - Uo).max() <= 1e-12 * sc
    assert np.linalg.norm(A - Lg @ Ug) / np.linalg.norm(A) < 1e-14


@pytest.mark.parametrize("level,leaf,eps,fixed,prec", [
    (3, 32, 1e-6, 0, 0), (3, 32, 0.0, 8, 0), (4, 32, 1e-6, 0, 0), (3, 32, 1e-6, 0, 1),
    (4, 32, 1e-5, 0, 1)])
def test_hlu_factor_accuracy(P, level, leaf, eps, fixed, prec):
    """|A - Lhat U|_F / |A|_F <= 10 eps_trunc + |A - A_H| with the exact A."""
    xyz, area, h = _hlu(P, level, leaf, eps=eps if eps else 1e-6, fixed_rank=fixed, precision=prec)
    h.factor()
    st, inf = h.sync()
    Lg, Ug = h.export_factors()
    perm = h.perm()
    A = O.dense_matrix(xyz, area)[np.ix_(perm, perm)]
    rel = np.linalg.norm(A - Lg @ Ug) / np.linalg.norm(A)
    _say("factor accuracy", level, leaf, eps, fixed, prec, rel, "max rank", inf.max_rank,
         "cap hits", inf.cap_hits)
    if fixed:
        # fixed rank 8: the largest discarded block tail is ~1e-4 relative
        # (oracle's truncation log); the global error stays far below it
        assert rel < 1e-5
    else:
        assert rel <= 11 * eps


@pytest.mark.parametrize("prec", [0, 1])
def test_hlu_solve_vs_oracle_and_refinement(P, prec):
    xyz, area, h = _hlu(P, 3, 32, eps=1e-6, precision=prec, refine_tol=1e-10)
    import torch
    h.factor()
    h.sync()
    b = rhs_normal(11, h.n, 4)
    x = h.solve(torch.tensor(b, device="cuda")).cpu().numpy()
    st, inf = h.sync(check=False)
    assert st == 0, (st, inf.eta_final)
    eta = O.backward_error(xyz, area, x, b)
    _say("solve+IR", prec, "iters", inf.iters, "eta dev", inf.eta_final, "eta exact", eta)
    assert eta <= 1e-10
    H = O.HMatrix(xyz, area, 32, 2.0, O.Rule(eps=1e-6, cap=32))
    O.factor(H)
    xo, hist = O.refine(H, b, tol=1e-10)
    kappa = 4.0
    assert np.abs(x - xo).max() / np.abs(xo).max() <= 4 * kappa * max(eta, hist[-1]) * 10


def test_hlu_solve_without_refinement_vs_oracle(P):
    import torch
    xyz, area, h = _hlu(P, 3, 32, fixed_rank=8)
    h.factor()
    h.sync()
    x_true = rhs_uniform(0, h.n)
    A = O.dense_matrix(xyz, area)
    b = A @ x_true
    x = h.solve(torch.tensor(b, device="cuda")).cpu().numpy()
    H = O.HMatrix(xyz, area, 32, 2.0, O.Rule(fixed=8))
    O.factor(H)
    xo = O.solve(H, b)
    xd = np.linalg.solve(A, b)
    e_g = np.linalg.norm(x - xd) / np.linalg.norm(xd)
    e_o = np.linalg.norm(xo - xd) / np.linalg.norm(xd)
    _say("C1 solve errors gpu", e_g, "oracle", e_o)
    assert e_g < 1e-5 and e_o < 1e-5
    assert np.linalg.norm(x - xo) / np.linalg.norm(xo) < 1e-5


def test_matvec_vs_exact(P):
    import torch
    xyz, area, h = _hlu(P, 4, 32, eps=1e-6)
    x = rhs_normal(7, h.n, 3)
    y = h.matvec(torch.tensor(x, device="cuda")).cpu().numpy()
    ye = O.exact_matvec(xyz, area, x)
    rel = np.linalg.norm(y - ye) / np.linalg.norm(ye)
    _say("matvec rel", rel)
    assert rel < 1e-11


def test_solve_argument_and_state_errors(P):
    import torch
    xyz, area, h = _hlu(P, 2, 16)
    b = torch.zeros((h.n, 1), dtype=torch.float64, device="cuda")
    with pytest.raises(P.HLUError) as e:
        h.solve(b)
    assert e.value.status == 6
    h.factor()
    with pytest.raises(P.HLUError) as e:
        h.factor()
    assert e.value.status == 6
    with pytest.raises(P.HLUError) as e:
        h.solve(torch.zeros((h.n, 40), dtype=torch.float64, device="cuda"))
    assert e.value.status == 1
    h.reset()
    h.factor()
    h.sync()


@pytest.mark.parametrize("prec", [0, 1])
def test_graph_replays_match_eager(P, prec):
    """The graph of the schedule replayed several times (with eager work and
    synchronisations in between) gives bitwise the eager factors and solve."""
    import torch
    xyz, area, h = _hlu(P, 3, 32, eps=1e-6, precision=prec, max_nrhs=4)
    b = torch.tensor(rhs_normal(5, h.n, 3), device="cuda")
    h.set_graph(False)
    h.factor()
    h.sync()
    L0, U0 = h.export_factors()
    x0 = h.solve(b).cpu().numpy()
    h.set_graph(True)
    for rep in range(3):
        h.reset()
        junk = torch.randn(1000, device="cuda").sum()       # eager work between replays
        torch.cuda.synchronize()
        h.factor()
        h.sync()
        L, U = h.export_factors()
        x = h.solve(b).cpu().numpy()
        assert np.array_equal(L, L0) and np.array_equal(U, U0), rep
        assert np.array_equal(x, x0), rep
        del junk


@pytest.mark.parametrize("level,prec,graph", [(3, 0, 0), (3, 1, 1), (4, 1, 1)])
def test_dataflow_executor_matches_waves(P, level, prec, graph):
    """The persistent dataflow executor runs the same ops on the same inputs
    (every read/write conflict is an edge, and writers of the same rows keep
    their program order), so its factors and its solutions (with refinement)
    are bitwise the wave executor's; replayed twice."""
    import torch
    xyz, area, h = _hlu(P, level, 32, eps=1e-6, precision=prec, max_nrhs=4)
    b = torch.tensor(rhs_normal(5, h.n, 3), device="cuda")
    h.set_graph(graph)
    h.set_executor(0)
    h.factor()
    h.sync()
    L0, U0 = h.export_factors()
    p0 = h.export_pivots()
    x0 = h.solve(b).cpu().numpy()
    st0, inf0 = h.sync(check=False)
    h.set_executor(1)
    for rep in range(2):
        h.reset()
        h.factor()
        st, inf = h.sync(check=False)
        assert st == 0, (rep, P.lib.hlu_last_error())
        L, U = h.export_factors()
        assert np.array_equal(h.export_pivots(), p0)
        assert np.array_equal(L, L0) and np.array_equal(U, U0), rep
        x = h.solve(b).cpu().numpy()
        st, inf = h.sync(check=False)
        assert st == st0 and inf.iters == inf0.iters, (rep, P.lib.hlu_last_error())
        assert np.array_equal(x, x0), rep


@pytest.mark.parametrize("slack,workers,graph", [(0.02, 4, 0), (0.2, 16, 1), (1.0, 2, 0)])
def test_priority_rings_match_one_ring(P, slack, workers, graph):
    """Near-critical ops flagged from a factorisation's own records go to a
    second ready ring served by dedicated workgroups; the ops and their
    inputs are the same, so the factors are bitwise those of one ring.  The
    last case flags every op that has predecessors (the high ring carries
    almost all of the schedule through two workgroups); clearing the flags
    restores one ring."""
    xyz, area, h = _hlu(P, 4, 32, eps=1e-6, precision=P.PREC_MIXED, max_nrhs=2)
    h.set_graph(graph)
    h.set_executor(1)
    h.factor()
    st, _ = h.sync(check=False)
    assert st == 0
    L0, U0 = h.export_factors()
    p0 = h.export_pivots()
    nf = h.set_priorities(slack, workers)
    assert nf > 0
    for rep in range(2):
        h.reset()
        h.factor()
        st, _ = h.sync(check=False)
        assert st == 0, (rep, P.lib.hlu_last_error())
        L, U = h.export_factors()
        assert np.array_equal(h.export_pivots(), p0)
        assert np.array_equal(L, L0) and np.array_equal(U, U0), rep
    assert h.set_priorities(slack, 0) == 0
    h.reset()
    h.factor()
    st, _ = h.sync(check=False)
    assert st == 0
    L, U = h.export_factors()
    assert np.array_equal(L, L0) and np.array_equal(U, U0)


def test_batched_factor_matches_alone(P):
    """One persistent launch over the union of several matrices' schedules
    (sphere and ellipsoids of different sizes) gives, matrix by matrix, the
    factors and pivots of factoring each alone (the same ops on the same
    data); repeated after a reset."""
    from hlu_inputs.geometry import ellipsoid_surface
    geo = [icosphere(3), ellipsoid_surface(3, (1.5, 0.7, 1.0)), icosphere(4),
           ellipsoid_surface(2, (0.6, 1.8, 1.2))]
    hs = [P.HLU(x, a, leaf=32, eta=2.0, eps=1e-6, cap=32, precision=P.PREC_MIXED, max_nrhs=1)
          for x, a in geo]
    ref = []
    for h in hs:
        h.set_executor(1)
        h.factor()
        st, inf = h.sync(check=False)
        assert st == 0
        ref.append((h.export_factors(), h.export_pivots()))
    _say("batched", [h.n for h in hs])
    bt = P.Batch(hs)
    for rep in range(2):
        for h in hs:
            h.reset()
        bt.factor()
        bt.sync()
        for h, ((L0, U0), p0) in zip(hs, ref):
            st, inf = h.sync(check=False)
            assert st == 0, P.lib.hlu_last_error()
            L, U = h.export_factors()
            assert np.array_equal(h.export_pivots(), p0)
            assert np.array_equal(L, L0) and np.array_equal(U, U0), rep


def test_scratch_ring_reuse(P):
    """H-GEMM temporaries sharing a ring: a ring that never wraps changes
    nothing (bitwise); a tight ring (regions reused, deferred truncations
    flushed early) keeps the factor accurate, and the wave and dataflow
    executors, which take the reuse order from the same program order,
    agree bitwise."""
    xyz, area = icosphere(4)
    A = O.dense_matrix(xyz, area)
    kw = dict(leaf=32, eta=2.0, eps=1e-6, cap=32, precision=P.PREC_MIXED, max_nrhs=1,
              cap_mv=0, refine_tol=0.0)
    h0 = P.HLU(xyz, area, **kw)
    big = int(h0.stats()["bytes_scratch"]) * 2 + (1 << 20)
    h0.set_executor(1)
    h0.factor()
    h0.sync()
    L0, U0 = h0.export_factors()
    h2 = P.HLU(xyz, area, scratch_cap=big, **kw)
    h2.set_executor(1)
    h2.factor()
    h2.sync()
    L2, U2 = h2.export_factors()
    assert np.array_equal(L2, L0) and np.array_equal(U2, U0)
    h1 = P.HLU(xyz, area, scratch_cap=2 << 20, **kw)
    _say("ring", h1.stats()["bytes_scratch"], "vs", h0.stats()["bytes_scratch"])
    assert h1.stats()["bytes_scratch"] <= 2 << 20
    h1.set_executor(0)
    h1.factor()
    h1.sync()
    Lw, Uw = h1.export_factors()
    h1.set_executor(1)
    h1.reset()
    h1.factor()
    h1.sync()
    Ld, Ud = h1.export_factors()
    assert np.array_equal(Lw, Ld) and np.array_equal(Uw, Ud)
    perm = h1.perm()
    rel = np.linalg.norm(A[np.ix_(perm, perm)] - Ld @ Ud) / np.linalg.norm(A)
    assert rel <= 11 * 1e-6, rel


def test_refinement_not_converged_is_reported(P):
    """A very loose factorisation with one refinement step cannot reach the
    target: the solve reports NOT_CONVERGED instead of a silent answer."""
    import torch
    xyz, area, h = _hlu(P, 3, 32, eps=1e-1, cap=2, refine_tol=1e-15, refine_max_iter=1)
    h.factor()
    h.sync()
    b = torch.tensor(rhs_normal(3, h.n, 1), device="cuda")
    h.solve(b)
    st, inf = h.sync(check=False)
    assert st == 5
    assert inf.eta_final > 1e-15


def test_autotuned_batch_matches_alone_at_the_chosen_shape(P):
    """The autotuner picks a (truncation stack width, workers) pair by timing
    the batch; at that choice the batch still equals each matrix factored
    alone with the same stack width, bit for bit, and a narrow stack (32)
    keeps the factor accuracy bound |A - Lhat U| <= 10 eps |A| (+ |A - A_H|)."""
    from hlu_inputs.geometry import ellipsoid_surface
    from paper_1906_00874_amd import autotune
    geo = [icosphere(3), ellipsoid_surface(3, (1.5, 0.7, 1.0)), ellipsoid_surface(2, (0.6, 1.8, 1.2))]
    hs = [P.HLU(x, a, leaf=32, eta=2.0, eps=1e-6, cap=32, precision=P.PREC_MIXED, max_nrhs=1)
          for x, a in geo]
    for h in hs:
        h.set_executor(1)
    bt = P.Batch(hs)
    res = autotune.tune_batch(bt, hs, reps=1, log=_say)
    _say("autotune choice", res["trunc_width"], res["workers"], res["table"])
    assert res["trunc_width"] in autotune.WIDTHS and res["workers"] in autotune.WORKERS
    assert len(res["table"]) == len(autotune.WIDTHS) + len(autotune.WORKERS) - 1
    for h in hs:
        h.reset()
    bt.factor()
    bt.sync()
    got = [(h.export_factors(), h.export_pivots()) for h in hs]
    for h, ((L0, U0), p0) in zip(hs, got):
        h.reset()
        h.set_tuning(res["trunc_width"])
        h.factor()
        st, inf = h.sync(check=False)
        assert st == 0
        L, U = h.export_factors()
        assert np.array_equal(h.export_pivots(), p0)
        assert np.array_equal(L, L0) and np.array_equal(U, U0)
    xyz, area = geo[0]
    h = hs[0]
    h.reset()
    h.set_tuning(32)
    h.factor()
    h.sync()
    Lg, Ug = h.export_factors()
    A = O.dense_matrix(xyz, area)[np.ix_(h.perm(), h.perm())]
    rel = np.linalg.norm(A - Lg @ Ug) / np.linalg.norm(A)
    _say("stack width 32: |A - LU|/|A|", rel)
    assert rel <= 11 * 1e-6


@pytest.mark.parametrize("kernel,reading,geo,prec", [
    (2, O.READING_LOG1D, "segment", 0), (3, O.READING_LOG2D, "circle", 1)])
def test_log_kernels_factor_and_refined_solve(P, kernel, reading, geo, prec):
    """Second workloads of Sec. 6.1: the d = 1 (-log r on [0, 1]) and d = 2
    (-log(r)/(2 pi) on a circle) kernels, n = 4096: factor accuracy against
    the exact matrix, refined backward error against the exact operator and
    the solution against the oracle's (P9(b) bound)."""
    import torch
    from hlu_inputs import circle, segment
    xyz, h = (segment if geo == "segment" else circle)(4096)
    _say("log kernel", kernel, geo, "precision", prec)
    hl = P.HLU(xyz, h, kernel=kernel, leaf=32, eta=2.0, eps=1e-6, cap=32, precision=prec,
               refine_tol=1e-10, max_nrhs=4)
    hl.set_executor(1)
    hl.factor()
    st, inf = hl.sync(check=False)
    assert st == 0
    Lg, Ug = hl.export_factors()
    perm = hl.perm()
    A = O.dense_matrix(xyz, h, reading)[np.ix_(perm, perm)]
    rel = np.linalg.norm(A - Lg @ Ug) / np.linalg.norm(A)
    del Lg, Ug, A
    b = rhs_normal(17, hl.n, 4)
    x = hl.solve(torch.tensor(b, device="cuda")).cpu().numpy()
    st, inf = hl.sync(check=False)
    assert st == 0
    eta = O.backward_error(xyz, h, x, b, reading)
    H = O.HMatrix(xyz, h, 32, 2.0, O.Rule(eps=1e-6, cap=32), reading=reading)
    O.factor(H)
    xo, hist = O.refine(H, b, tol=1e-10)
    e = np.abs(x - xo).max() / np.abs(xo).max()
    _say("log kernel", kernel, "|A - LU|/|A|", rel, "iters", inf.iters, "eta", eta,
         "|x - x_oracle|", e)
    assert rel <= 11 * 1e-6
    assert eta <= 1e-10 and inf.eta_final <= 1e-10
    assert e <= 4 * 4.0 * max(eta, hist[-1], 1e-12)
