"""Planted mistakes in the oracle, on the CPU.

Each plausible slip (a lost absolute value in the pivot search, a dropped
column scaling, a missing Sigma in the truncated factors, a sign flip in the
low-rank update, a permutation applied after the solve instead of before,
the larger box diameter or the distance of the box centres in the
admissibility condition) must be caught by the checks the oracle's pins use.  Every check runs on the
unmodified oracle first, so a failure under a mutant is the mutant's doing.
"""
import math

import numpy as np
import scipy.linalg as sla

import oracle.hlu as OH


# ------------------------------------------------------------------ checks
def _getrf_ok(fn, b=33, seed=7):
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((b, b))
    lu_ref, piv_ref = sla.lu_factor(a.copy())
    a2 = a.copy()
    piv, info = fn(a2)
    return (info == 0 and np.array_equal(piv, piv_ref)
            and np.allclose(a2, lu_ref, rtol=1e-12, atol=1e-12 * np.abs(lu_ref).max()))


def _truncate_ok(fn, m=200, n=150, K=40, eps=1e-6, seed=11):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((m, K)) * 0.5 ** np.arange(K)
    Y = rng.standard_normal((n, K))
    D = X @ Y.T
    nd = np.linalg.norm(D)
    sig = np.linalg.svd(D, compute_uv=False)
    tails = np.sqrt(np.concatenate([np.cumsum((sig ** 2)[::-1])[::-1], [0.0]]))
    k_ref = int(np.argmax(tails <= eps * nd))
    U, V = fn(X, Y, OH.Rule(eps=eps, cap=1000))
    err = np.linalg.norm(D - U @ V.T)
    return U.shape[1] == k_ref and abs(err - tails[k_ref]) <= 1e-6 * tails[k_ref] + 1e-13 * nd


def _blocktree_ok(level=3, leaf=32, eta=2.0):
    """Every node of Algorithm 2's block tree against the admissibility
    condition written out here: low-rank leaves admissible, partitioned
    nodes and dense leaves not."""
    from hlu_inputs import icosphere
    xyz, _ = icosphere(level)
    root, _, _ = OH.cluster_tree(xyz, leaf)

    def adm(t, s):
        gap = np.maximum(0.0, np.maximum(s.lo - t.hi, t.lo - s.hi))
        dist = float(np.sqrt(np.sum(gap * gap)))
        dmin = min(float(np.sqrt(np.sum((t.hi - t.lo) ** 2))),
                   float(np.sqrt(np.sum((s.hi - s.lo) ** 2))))
        return dist > 0 and dmin <= eta * dist

    stack = [OH.block_tree(root, root, eta)]
    while stack:
        b = stack.pop()
        if (b.kind == "R") != adm(b.t, b.s):
            return False
        if b.kind == "H":
            stack.extend(c for row in b.sons for c in row)
    return True


def _hlu_ok():
    """H-LU of a mixed-structure matrix at tight tolerance reproduces A."""
    rng = np.random.default_rng(3)
    npt = 256
    pts = rng.standard_normal((npt, 3))
    pts /= np.linalg.norm(pts, axis=1, keepdims=True)
    pts[:, 2] *= 0.5
    area = np.full(npt, 4 * math.pi / npt)
    H = OH.HMatrix(pts, area, 8, 1.0, OH.Rule(eps=1e-13, cap=10 ** 6))
    A = H.to_dense()
    OH.factor(H)
    Lh, U = OH.factors_dense(H)
    return np.linalg.norm(A - Lh @ U) / np.linalg.norm(A) < 1e-11


# ----------------------------------------------------------------- mutants
def _getrf_no_abs(a):
    b = a.shape[0]
    piv = np.zeros(b, dtype=np.int64)
    for k in range(b):
        p = k + int(np.argmax(a[k:, k]))          # slip: signed maximum
        piv[k] = p
        if p != k:
            a[[k, p], :] = a[[p, k], :]
        a[k + 1:, k] = a[k + 1:, k] / a[k, k]
        a[k + 1:, k + 1:] -= np.outer(a[k + 1:, k], a[k, k + 1:])
    return piv, 0


def _getrf_no_scale(a):
    b = a.shape[0]
    piv = np.zeros(b, dtype=np.int64)
    for k in range(b):
        p = k + int(np.argmax(np.abs(a[k:, k])))
        piv[k] = p
        if p != k:
            a[[k, p], :] = a[[p, k], :]
        # slip: multipliers left unscaled by the pivot
        a[k + 1:, k + 1:] -= np.outer(a[k + 1:, k] / a[k, k], a[k, k + 1:])
    return piv, 0


def _truncate_no_sigma(X, Y, rule):
    Qx, Rx = np.linalg.qr(X, mode="reduced")
    Qy, Ry = np.linalg.qr(Y, mode="reduced")
    u, sig, vt = np.linalg.svd(Rx @ Ry.T, full_matrices=False)
    k = rule.choose(sig)
    return Qx @ u[:, :k], Qy @ vt[:k].T          # slip: Sigma dropped


def _add_lr_sign(C, X, Y, rule):
    if C.kind == "F":
        C.F -= X @ Y.T
    elif C.kind == "R":
        # slip: the update enters the stack with a plus sign
        C.U, C.V = OH.truncate(np.hstack([C.U, X]), np.hstack([C.V, Y]), rule)
    else:
        for i, ti in enumerate(C.t.sons):
            for j, sj in enumerate(C.s.sons):
                _add_lr_sign(C.sons[i][j], X[OH._rows(C.t, ti)], Y[OH._rows(C.s, sj)], rule)


def _admissible_max_diam(t, s, eta):
    gap = np.maximum(0.0, np.maximum(s.lo - t.hi, t.lo - s.hi))
    dist = float(np.linalg.norm(gap))
    if eta <= 0.0 or dist <= 0.0:
        return False
    return max(t.diam(), s.diam()) <= eta * dist     # slip: max instead of min


def _admissible_centre_distance(t, s, eta):
    # slip: distance between the box centres instead of the gap between boxes
    dist = float(np.linalg.norm(0.5 * (t.lo + t.hi) - 0.5 * (s.lo + s.hi)))
    if eta <= 0.0 or dist <= 0.0:
        return False
    return min(t.diam(), s.diam()) <= eta * dist


def _fwd_late_perm(Lb, Y):
    if Lb.kind == "F":
        # slip: the leaf's row interchanges applied after the solve
        Y[:] = sla.solve_triangular(Lb.F, Y, lower=True, unit_diagonal=True, check_finite=False)
        OH.apply_piv(Lb.piv, Y)
        return
    t0, t1 = Lb.t.sons
    Y0, Y1 = Y[OH._rows(Lb.t, t0)], Y[OH._rows(Lb.t, t1)]
    _fwd_late_perm(Lb.sons[0][0], Y0)
    Y1 -= OH.mul(Lb.sons[1][0], Y0)
    _fwd_late_perm(Lb.sons[1][1], Y1)


# ------------------------------------------------------------------- tests
def test_getrf_checks_catch_slips():
    assert _getrf_ok(OH.getrf)
    assert not _getrf_ok(_getrf_no_abs)
    assert not _getrf_ok(_getrf_no_scale)


def test_truncate_check_catches_missing_sigma():
    assert _truncate_ok(OH.truncate)
    assert not _truncate_ok(_truncate_no_sigma)


def test_hlu_check_catches_update_sign(monkeypatch):
    assert _hlu_ok()
    monkeypatch.setattr(OH, "add_lr", _add_lr_sign)
    assert not _hlu_ok()


def test_hlu_check_catches_late_permutation(monkeypatch):
    monkeypatch.setattr(OH, "fwd", _fwd_late_perm)
    assert not _hlu_ok()


def test_blocktree_check_catches_admissibility_slips(monkeypatch):
    assert _blocktree_ok()
    monkeypatch.setattr(OH, "admissible", _admissible_max_diam)
    assert not _blocktree_ok()
    monkeypatch.setattr(OH, "admissible", _admissible_centre_distance)
    assert not _blocktree_ok()
