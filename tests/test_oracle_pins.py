"""Pins of the oracle against mathematics and library routines (CPU only).

Each test checks the oracle against something other than itself: LAPACK,
numpy's SVD, a brute-force dense block LU written here, closed forms on the
sphere, and structural invariants of Algorithms 1 and 2.
"""
import math

import numpy as np
import pytest
import scipy.linalg as sla

import oracle as O
import oracle.hlu as OH
from hlu_inputs import icosphere, rhs_normal


# ---------------------------------------------------------------- geometry
@pytest.mark.parametrize("level", [0, 1, 2, 3, 4])
def test_icosphere_counts_and_area(level):
    xyz, area = icosphere(level)
    assert xyz.shape == (20 * 4 ** level, 3)
    # flat triangles inscribed in the sphere: total area below 4 pi and
    # converging to it; centroids strictly inside the unit sphere
    assert area.sum() < 4 * math.pi
    r = np.linalg.norm(xyz, axis=1)
    assert r.max() < 1.0
    if level >= 3:
        assert abs(area.sum() - 4 * math.pi) / (4 * math.pi) < 5e-3


# ---------------------------------------------------------------- Algorithm 1
def _check_cluster(c, xyz_p, leaf):
    pts = xyz_p[c.off:c.off + c.size]
    assert np.array_equal(pts.min(axis=0), c.lo) and np.array_equal(pts.max(axis=0), c.hi)
    if c.sons:
        assert c.size > leaf
        s0, s1 = c.sons
        assert s0.off == c.off and s1.off == c.off + s0.size
        assert s0.size + s1.size == c.size and s0.size > 0 and s1.size > 0
        d = int(np.argmax(c.hi - c.lo))
        mid = 0.5 * (c.lo[d] + c.hi[d])
        assert np.all(xyz_p[s0.off:s0.off + s0.size, d] < mid)
        assert np.all(xyz_p[s1.off:s1.off + s1.size, d] >= mid)
        for s in c.sons:
            _check_cluster(s, xyz_p, leaf)
    else:
        assert c.size <= leaf


@pytest.mark.parametrize("level,leaf", [(3, 32), (4, 32), (3, 64), (2, 1)])
def test_cluster_tree_invariants(level, leaf):
    xyz, _ = icosphere(level)
    root, perm, leaves = O.cluster_tree(xyz, leaf)
    assert np.array_equal(np.sort(perm), np.arange(xyz.shape[0]))
    _check_cluster(root, xyz[perm], leaf)
    offs = [l.off for l in leaves]
    assert offs == sorted(offs)
    assert sum(l.size for l in leaves) == xyz.shape[0]


def test_cluster_tree_coincident_points_median_split():
    xyz = np.zeros((10, 3))
    root, perm, leaves = O.cluster_tree(xyz, 3)
    assert np.array_equal(np.sort(perm), np.arange(10))
    assert all(l.size <= 3 for l in leaves)
    assert root.sons[0].size == 5


# ---------------------------------------------------------------- Algorithm 2
def _coverage(H):
    n = H.n
    cnt = np.zeros((n, n), dtype=np.int32)
    for b in O.leaves_of(H.block):
        cnt[b.t.off:b.t.off + b.t.size, b.s.off:b.s.off + b.s.size] += 1
    return cnt


@pytest.mark.parametrize("eta", [0.0, 0.5, 2.0])
def test_block_tree_partition_and_admissibility(eta):
    xyz, area = icosphere(3)
    H = O.HMatrix(xyz, area, 32, eta, O.Rule(eps=1e-6))
    assert np.all(_coverage(H) == 1)
    for b in O.leaves_of(H.block):
        gap = np.maximum(0.0, np.maximum(b.s.lo - b.t.hi, b.t.lo - b.s.hi))
        dist = np.linalg.norm(gap)
        diam = min(np.linalg.norm(b.t.hi - b.t.lo), np.linalg.norm(b.s.hi - b.s.lo))
        if b.kind == "R":
            assert eta > 0 and dist > 0 and diam <= eta * dist
            assert b.t is not b.s
        else:
            assert not b.t.sons or not b.s.sons
    if eta == 0.0:
        assert H.stats()["lowrank"] == 0


def test_kernel_entries_direct():
    xyz, area = icosphere(2)
    i, j = 3, 17
    r = np.linalg.norm(xyz[i] - xyz[j])
    A = O.kernel_entries(xyz, area, [i, j], [i, j], O.READING_WEIGHTED)
    assert A[0, 1] == pytest.approx(area[j] / (4 * math.pi * r), rel=1e-15)
    assert A[1, 0] == pytest.approx(area[i] / (4 * math.pi * r), rel=1e-15)
    assert A[0, 0] == pytest.approx(math.sqrt(area[i]) / (2 * math.pi) + 1.0, rel=1e-15)
    B = O.kernel_entries(xyz, area, [i, j], [i, j], O.READING_POINT)
    assert B[0, 1] == pytest.approx(1.0 / (4 * math.pi * r), rel=1e-15)


# ---------------------------------------------------------------- leaf getrf
@pytest.mark.parametrize("b", [1, 2, 11, 31, 32, 33, 63, 64])
def test_getrf_matches_lapack(b):
    rng = np.random.default_rng(100 + b)
    a = rng.standard_normal((b, b))
    lu_ref, piv_ref = sla.lu_factor(a.copy())
    a2 = a.copy()
    piv, info = O.getrf(a2)
    assert info == 0
    assert np.array_equal(piv, piv_ref)
    assert np.allclose(a2, lu_ref, rtol=1e-12, atol=1e-12 * np.abs(lu_ref).max())


def test_getrf_zero_pivot_info():
    a = np.array([[0.0, 1.0, 2.0], [0.0, 3.0, 4.0], [0.0, 5.0, 7.0]])
    piv, info = O.getrf(a)
    assert info == 1
    assert piv[0] == 0


def test_getrf_ties_take_first_index():
    a = np.array([[1.0, 2.0], [-1.0, 5.0]])
    piv, _ = O.getrf(a)
    assert piv[0] == 0


# ---------------------------------------------------------------- truncation
def _decaying(m, n, K, rng, decay=0.5):
    X = rng.standard_normal((m, K)) * decay ** np.arange(K)
    Y = rng.standard_normal((n, K))
    return X, Y


@pytest.mark.parametrize("m,n,K,eps", [(40, 30, 12, 1e-3), (200, 150, 40, 1e-6),
                                       (20, 70, 30, 1e-8), (5, 9, 16, 1e-2)])
def test_truncate_eckart_young(m, n, K, eps):
    rng = np.random.default_rng(m * n + K)
    X, Y = _decaying(m, n, K, rng)
    D = X @ Y.T
    sig = np.linalg.svd(D, compute_uv=False)
    rule = O.Rule(eps=eps, cap=1000)
    U, V = O.truncate(X, Y, rule)
    k = U.shape[1]
    # smallest k whose discarded tail meets the bound, computed from the
    # dense product's singular values
    tails = np.sqrt(np.concatenate([np.cumsum((sig ** 2)[::-1])[::-1], [0.0]]))
    k_ref = int(np.argmax(tails <= eps * np.linalg.norm(D)))
    assert k == k_ref
    err = np.linalg.norm(D - U @ V.T)
    assert err == pytest.approx(tails[k], rel=1e-6, abs=1e-13 * np.linalg.norm(D))
    assert err <= eps * np.linalg.norm(D) * (1 + 1e-8)


def test_truncate_cap_and_fixed():
    rng = np.random.default_rng(7)
    X, Y = _decaying(60, 50, 20, rng, decay=0.9)
    rule = O.Rule(eps=1e-12, cap=5)
    U, V = O.truncate(X, Y, rule)
    assert U.shape[1] == 5 and rule.log[-1][3]
    rule = O.Rule(fixed=3)
    U, V = O.truncate(X, Y, rule)
    sig = np.linalg.svd(X @ Y.T, compute_uv=False)
    assert np.linalg.norm(X @ Y.T - U @ V.T) == pytest.approx(
        np.sqrt(np.sum(sig[3:] ** 2)), rel=1e-8)


def test_truncate_zero_and_rank_deficient():
    X = np.zeros((10, 4))
    Y = np.ones((8, 4))
    U, V = O.truncate(X, Y, O.Rule(eps=1e-6))
    assert U.shape[1] == 0
    rng = np.random.default_rng(1)
    a = rng.standard_normal((30, 2))
    X = np.hstack([a, a])          # rank 2 stack of 4 columns
    Y = rng.standard_normal((25, 4))
    U, V = O.truncate(X, Y, O.Rule(eps=1e-10))
    assert U.shape[1] == 2
    assert np.allclose(U @ V.T, X @ Y.T, atol=1e-12)


# ---------------------------------------------------------------- H-LU pins
def _block_lu_bruteforce(A, leaves):
    """Dense block LU with partial pivoting confined to each diagonal leaf,
    written independently: Schur complements eliminated leaf by leaf."""
    n = A.shape[0]
    S = A.copy()
    Lh = np.zeros((n, n))
    U = np.zeros((n, n))
    pivs = []
    for lf in leaves:
        a, b = lf.off, lf.off + lf.size
        lu, piv = sla.lu_factor(S[a:b, a:b].copy())
        pivs.append(piv)
        P = np.eye(b - a)
        for k, p in enumerate(piv):
            P[[k, p]] = P[[p, k]]
        L = np.tril(lu, -1) + np.eye(b - a)
        Uk = np.triu(lu)
        Lh[a:b, a:b] = P.T @ L
        U[a:b, a:b] = Uk
        # U row panel and L column panel from the current Schur complement
        U[a:b, b:] = sla.solve_triangular(L, P @ S[a:b, b:], lower=True, unit_diagonal=True)
        Lh[b:, a:b] = sla.solve_triangular(Uk.T, S[b:, a:b].T, lower=True).T
        S[b:, b:] -= Lh[b:, a:b] @ U[a:b, b:]
    return Lh, U, pivs


def test_hlu_eta0_equals_block_lu():
    """eta = 0: no admissible blocks, the H-LU is the dense block LU with
    pivoting restricted to the diagonal leaves."""
    xyz, area = icosphere(2)
    H = O.HMatrix(xyz, area, 16, 0.0, O.Rule(eps=1e-6), reading=O.READING_POINT)
    A = H.to_dense()
    Lr, Ur, pivs = _block_lu_bruteforce(A, H.leaves)
    O.factor(H)
    Lh, U = O.factors_dense(H)
    for lf, p in zip(H.leaves, pivs):
        blk = [b for b in O.leaves_of(H.block) if b.t is lf and b.s is lf][0]
        assert np.array_equal(blk.piv, p)
    sc = np.abs(A).max()
    assert np.abs(Lh - Lr).max() < 1e-12 * sc * 100
    assert np.abs(U - Ur).max() < 1e-12 * sc * 100
    assert np.linalg.norm(A - Lh @ U) / np.linalg.norm(A) < 1e-14


def test_hlu_single_leaf_is_lapack():
    xyz, area = icosphere(1)             # n = 80, leaf 100 -> one dense block
    H = O.HMatrix(xyz, area, 100, 2.0, O.Rule(eps=1e-6))
    A = H.to_dense()
    O.factor(H)
    lu, piv = sla.lu_factor(A)
    assert np.array_equal(H.block.piv, piv)
    assert np.allclose(H.block.F, lu, atol=1e-13)


def test_hgemm_cases_against_dense():
    """Every product kind in a factorisation at tight tolerance: the H-LU of
    a mixed-structure matrix reproduces A to the truncation accuracy."""
    O.CASES.clear()
    rng = np.random.default_rng(3)
    pts = rng.standard_normal((384, 3))
    pts /= np.linalg.norm(pts, axis=1, keepdims=True)
    pts[:, 2] *= 0.5
    area = np.full(384, 4 * math.pi / 384)
    H = O.HMatrix(pts, area, 8, 1.0, O.Rule(eps=1e-13, cap=10 ** 6))
    A = H.to_dense()
    O.factor(H)
    Lh, U = O.factors_dense(H)
    assert np.linalg.norm(A - Lh @ U) / np.linalg.norm(A) < 1e-11
    kinds = set(O.CASES)
    for needed in ("RRR", "FFF", "HHH", "RFF", "FRF", "HFR", "FHR", "HHR"):
        assert any(k == needed for k in kinds), (needed, kinds)


def test_hgemm_direct_random_blocks():
    """gemm(C, A, B) on blocks of an assembled H-matrix against C - A B."""
    xyz, area = icosphere(3)
    H = O.HMatrix(xyz, area, 16, 1.0, O.Rule(eps=1e-13, cap=10 ** 6))
    D = H.to_dense()
    A10 = H.block.sons[1][0]
    A01 = H.block.sons[0][1]
    C = H.block.sons[1][1]
    n0 = H.block.t.sons[0].size
    ref = D[n0:, n0:] - D[n0:, :n0] @ D[:n0, n0:]
    O.gemm(C, A10, A01, H.rule)
    got = np.zeros_like(ref)
    for b in O.leaves_of(C):
        got[b.t.off - n0:b.t.off - n0 + b.t.size, b.s.off - n0:b.s.off - n0 + b.s.size] = \
            b.F if b.kind == "F" else b.U @ b.V.T
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-11


# ---------------------------------------------------------------- accuracy gates
@pytest.fixture(scope="module")
def c1_factored():
    xyz, area = icosphere(3)
    rule = O.Rule(eps=1e-6, cap=32)
    H = O.HMatrix(xyz, area, 32, 2.0, rule)
    AH = H.to_dense()
    nlog = len(rule.log)
    O.factor(H)
    return xyz, area, H, AH, rule, nlog


def test_construction_accuracy(c1_factored):
    xyz, area, H, AH, rule, _ = c1_factored
    A = O.dense_matrix(xyz, area)[np.ix_(H.perm, H.perm)]
    assert np.linalg.norm(A - AH) / np.linalg.norm(A) <= 1e-6


def test_factor_accuracy(c1_factored):
    xyz, area, H, AH, rule, _ = c1_factored
    Lh, U = O.factors_dense(H)
    assert np.linalg.norm(AH - Lh @ U) / np.linalg.norm(AH) <= 10 * 1e-6


def test_refinement_backward_error(c1_factored):
    xyz, area, H, AH, rule, _ = c1_factored
    b = rhs_normal(11, H.n, 3)
    x, hist = O.refine(H, b, tol=1e-10)
    assert hist[-1] <= 1e-10
    assert len(hist) <= 4
    # the solve of the exact system agrees with LAPACK's dense solve
    xd = np.linalg.solve(O.dense_matrix(xyz, area), b)
    assert np.linalg.norm(x - xd) / np.linalg.norm(xd) < 1e-9


def _zonal(l, z):
    return np.polynomial.legendre.Legendre.basis(l)(z)


@pytest.mark.parametrize("level,delta", [(3, 2.0e-2), (4, 1.0e-2)])
def test_sphere_closed_form(level, delta):
    """Weighted reading on the unit sphere: A = I + V_h with V the single
    layer operator, whose eigenvalues on degree-l harmonics are 1/(2l+1), so
    A Y_l ~ (1 + 1/(2l+1)) Y_l up to an O(h) discretisation error."""
    xyz, area = icosphere(level)
    A = O.dense_matrix(xyz, area)
    z = xyz[:, 2] / np.linalg.norm(xyz, axis=1)
    for l in range(4):
        y = _zonal(l, z)
        lam = 1.0 + 1.0 / (2 * l + 1)
        assert np.linalg.norm(A @ y - lam * y) / np.linalg.norm(y) < delta


def test_sphere_closed_form_through_hlu(c1_factored):
    xyz, area, H, AH, rule, _ = c1_factored
    z = xyz[:, 2] / np.linalg.norm(xyz, axis=1)
    for l in range(4):
        y = _zonal(l, z)
        lam = 1.0 + 1.0 / (2 * l + 1)
        x = O.solve(H, y)
        assert np.linalg.norm(x - y / lam) / np.linalg.norm(y) < 2.0e-2 / lam


def test_hmatvec_matches_dense(c1_factored):
    xyz, area, _, _, _, _ = c1_factored
    H = O.HMatrix(xyz, area, 32, 2.0, O.Rule(eps=1e-10, cap=64))
    x = rhs_normal(5, H.n, 2)
    y = O.hmatvec(H, x)
    yd = O.dense_matrix(xyz, area) @ x
    assert np.linalg.norm(y - yd) / np.linalg.norm(yd) < 1e-9


def test_zero_pivot_reported():
    """Two identical rows inside one leaf give an exactly zero pivot."""
    xyz, area = icosphere(2)
    H = O.HMatrix(xyz, area, 16, 0.0, O.Rule(eps=1e-6), reading=O.READING_POINT)
    lf = H.leaves[0]
    r0, r1 = lf.off, lf.off + 1
    for b in O.leaves_of(H.block):
        if b.t is lf:
            b.F[r1 - b.t.off] = b.F[r0 - b.t.off]
    info = O.factor(H)
    assert lf.off < info <= lf.off + lf.size


# ---------------------------------------------------------------- Algorithm 2, both sides
def _admissible_here(t, s, eta):
    """The admissibility condition of Sec. 2 (with eta), written out here:
    the smaller of the two box diameters against eta times the Euclidean
    gap between the axis-parallel boxes."""
    gap = [max(0.0, s.lo[d] - t.hi[d], t.lo[d] - s.hi[d]) for d in range(3)]
    dist = math.sqrt(sum(g * g for g in gap))
    dt = math.sqrt(sum((t.hi[d] - t.lo[d]) ** 2 for d in range(3)))
    ds = math.sqrt(sum((s.hi[d] - s.lo[d]) ** 2 for d in range(3)))
    return eta > 0 and dist > 0 and min(dt, ds) <= eta * dist


def _walk(b):
    yield b
    if b.kind == "H":
        for row in b.sons:
            for c in row:
                yield from _walk(c)


@pytest.mark.parametrize("level,leaf,eta", [(3, 32, 2.0), (4, 32, 2.0), (3, 16, 0.5)])
def test_block_tree_every_node_against_admissibility(level, leaf, eta):
    """Algorithm 2 on every node of the block tree: a low-rank leaf is
    admissible; a partitioned node and a dense leaf are not (a dense leaf
    also has a leaf cluster on one side)."""
    xyz, _ = icosphere(level)
    root, _, _ = O.cluster_tree(xyz, leaf)
    bt = O.block_tree(root, root, eta)
    kinds = {"R": 0, "H": 0, "F": 0}
    for b in _walk(bt):
        kinds[b.kind] += 1
        if b.kind == "R":
            assert _admissible_here(b.t, b.s, eta)
        else:
            assert not _admissible_here(b.t, b.s, eta)
            if b.kind == "H":
                assert b.t.sons and b.s.sons
            else:
                assert not b.t.sons or not b.s.sons
    assert all(v > 0 for v in kinds.values())


# leaves / dense blocks / low-rank blocks of the sphere workloads at eta 2,
# counted by an independent throwaway implementation of Algorithms 1 and 2
# (NumPy, written separately from this oracle before it existed)
INDEPENDENT_COUNTS = [
    (3, 32, 52, 418, 894),
    (4, 32, 217, 1845, 3922),
    (5, 32, 875, 7645, 18096),
    (5, 64, 437, 4395, 7924),
]


@pytest.mark.parametrize("level,leaf,nleaves,ndense,nlr", INDEPENDENT_COUNTS)
def test_block_counts_match_independent_count(level, leaf, nleaves, ndense, nlr):
    xyz, _ = icosphere(level)
    root, _, leaves = O.cluster_tree(xyz, leaf)
    bt = O.block_tree(root, root, 2.0)
    nf = sum(1 for b in O.leaves_of(bt) if b.kind == "F")
    nr = sum(1 for b in O.leaves_of(bt) if b.kind == "R")
    assert (len(leaves), nf, nr) == (nleaves, ndense, nlr)


# ---------------------------------------------------------------- randomised compression
@pytest.fixture(scope="module")
def large_admissible_blocks():
    """Exact entries of two admissible blocks of the level-5 sphere at leaf
    64 whose smaller side exceeds the dense-SVD limit (so the oracle's
    assembly takes its randomised range finder for them)."""
    xyz, area = icosphere(5)
    root, perm, _ = O.cluster_tree(xyz, 64)
    bt = O.block_tree(root, root, 2.0)
    big = [b for b in O.leaves_of(bt) if b.kind == "R" and min(b.t.size, b.s.size) > 384]
    big.sort(key=lambda b: b.t.size * b.s.size)
    pick = [big[0], big[-1]]
    xp, ap = xyz[perm], area[perm]
    out = []
    for b in pick:
        rows = np.arange(b.t.off, b.t.off + b.t.size)
        cols = np.arange(b.s.off, b.s.off + b.s.size)
        out.append(O.kernel_entries(xp, ap, rows, cols))
    return out


@pytest.mark.parametrize("which", [0, 1])
@pytest.mark.parametrize("eps", [1e-5, 1e-6])
def test_randomised_compression_eckart_young(large_admissible_blocks, which, eps):
    """The randomised range finder with power iterations (the oracle's
    assembly of large admissible blocks) against the dense SVD of the same
    exact block: the rank rule's choice to within one and the error within
    the tolerance."""
    A = large_admissible_blocks[which]
    assert min(A.shape) > 384
    nA = np.linalg.norm(A)
    sig = np.linalg.svd(A, compute_uv=False)
    tails = np.sqrt(np.concatenate([np.cumsum((sig ** 2)[::-1])[::-1], [0.0]]))
    k_ref = int(np.argmax(tails <= eps * nA))
    rule = O.Rule(eps=eps, cap=32)
    U, V = OH._compress_block(A, rule, np.random.default_rng(0))
    k = U.shape[1]
    assert abs(k - k_ref) <= 1, (k, k_ref)
    err = np.linalg.norm(A - U @ V.T)
    assert err <= eps * nA * (1 + 1e-6)
    # not much worse than the best approximation of the same rank
    assert err <= 1.5 * tails[k] + 1e-14 * nA


def test_randomised_compression_fixed_rank(large_admissible_blocks):
    A = large_admissible_blocks[1]
    sig = np.linalg.svd(A, compute_uv=False)
    U, V = OH._compress_block(A, O.Rule(fixed=8), np.random.default_rng(1))
    assert U.shape[1] == 8
    best = math.sqrt(float(np.sum(sig[8:] ** 2)))
    assert np.linalg.norm(A - U @ V.T) <= 1.05 * best
