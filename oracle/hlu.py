"""Oracle: hierarchical matrix, H-LU, solve and refinement in plain FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).  The code follows the
paper's steps in its order and notation, with library primitives (matmul,
SVD, QR, triangular solve) as single steps and no blocking or fusion beyond
what the method states:

* cluster tree: Algorithm 1 (Sec. 2), bounding boxes as described there;
* block tree: Algorithm 2 with the admissibility condition of Sec. 2;
* storage types: dense, low-rank X = A B^* (Sec. 3.1, "Low-rank blocks"),
  and 2x2 partitioned blocks (Sec. 2, hmatrix structure);
* H-LU: the sequence O1.1-O5.5 of Sec. 3.1 applied recursively, with the
  partitioned triangular solve O2.1-O2.6 of Sec. 5.2;
* low-rank arithmetic: matrix-vector and matrix-matrix products, triangular
  solves on the k columns of the factors, and addition followed by an SVD
  that discards small singular values (Sec. 3.1, "Low-rank blocks").

Readings where the paper is silent:
* split: longest bbox axis (lowest axis on ties), box midpoint, strict '<'
  to son 0, stable order; median split if a son would be empty;
* admissible(t,s): eta > 0, dist > 0 and min(diam t, diam s) <= eta*dist,
  diam/dist Euclidean on the tight axis-parallel boxes;
* pivoting: partial pivoting inside each diagonal leaf (first index of the
  largest |a|), row swaps applied lazily (rows of already computed L blocks
  stay unswapped, so A = Lhat U with Lhat's diagonal leaf blocks P^T L);
* truncation: smallest k whose discarded singular values have Frobenius
  norm <= eps * Frobenius norm of the block, capped at `cap`; or a fixed k;
* H-GEMM with mixed structures: product kinds as in the standard
  H-arithmetic of Grasedyck and Hackbusch (cited in Sec. 1); a low-rank
  target with partitioned operands is split into four virtual low-rank sons,
  updated recursively and agglomerated by one truncated addition;
* every truncated addition happens right after its product.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sla

FOUR_PI = 4.0 * math.pi

READING_WEIGHTED = 0   # A_ij = area_j / (4 pi |x_i - x_j|)
READING_POINT = 1      # A_ij = 1 / (4 pi |x_i - x_j|)
READING_LOG1D = 2      # A_ij = -h_j log|x_i - x_j|            (d = 1)
READING_LOG2D = 3      # A_ij = -h_j log|x_i - x_j| / (2 pi)   (d = 2)

# model flop count of the executed operations (getrf 2b^3/3 - b^2/2 + 5b/6,
# triangular solve m^2 n, product 2 m n k, truncation as in `truncate`);
# reset by the caller, used only to express timings as GFLOP/s
FLOPS = [0.0]


def _count(f):
    FLOPS[0] += f


# ---------------------------------------------------------------------------
# kernel entries (Sec. 6.1, d = 3 Laplace kernel g(x,y) = 1/(4 pi |x-y|))
# ---------------------------------------------------------------------------
def kernel_entries(xyz, area, rows, cols, reading=READING_WEIGHTED):
    """Dense block A[rows, cols] of the collocation matrix.

    Off-diagonal entries are the d=3 Laplace kernel between centroids, weighted
    by the column panel's area in the weighted reading.  The self term is
    2*sqrt(area_i/pi)/(4 pi)*sqrt(pi) + 1.0 in both readings.
    Parity: pinned by the closed-form sphere test (zonal harmonics) and by
    direct entry checks in the tests.
    """
    rows = np.asarray(rows)
    cols = np.asarray(cols)
    d = xyz[rows][:, None, :] - xyz[cols][None, :, :]
    r = np.sqrt(np.einsum("ijk,ijk->ij", d, d))
    same = rows[:, None] == cols[None, :]
    if reading in (READING_LOG1D, READING_LOG2D):
        return _log_entries(r, same, area[rows], area[cols], reading)
    with np.errstate(divide="ignore"):
        g = 1.0 / (FOUR_PI * r)
    if reading == READING_WEIGHTED:
        g = g * area[cols][None, :]
    diag = 2.0 * np.sqrt(area[rows] / math.pi) / FOUR_PI * math.sqrt(math.pi) + 1.0
    g = np.where(same, diag[:, None], g)
    return g


def _log_entries(r, same, h_rows, h_cols, reading):
    """d = 1 and d = 2 Laplace kernels of Sec. 6.1 (-log r and -log(r)/(2 pi))
    collocated at panel midpoints with one-point quadrature over the column
    panel (weight: its length h_j), plus the identity.  The self term is the
    kernel integrated exactly over the straight panel of length h around its
    midpoint: the integral of -log|t| over [-h/2, h/2] is h (1 - log(h/2)).
    Parity: pinned by the integral itself (numerical quadrature), by the
    continuous operator applied to 1 on [0, 1] (d = 1) and by the circle's
    Fourier modes (d = 2) in the tests."""
    scale = 1.0 if reading == READING_LOG1D else 1.0 / (2.0 * math.pi)
    with np.errstate(divide="ignore"):
        g = -np.log(r) * h_cols[None, :] * scale
    diag = h_rows * (1.0 - np.log(0.5 * h_rows)) * scale + 1.0
    return np.where(same, diag[:, None], g)


def dense_matrix(xyz, area, reading=READING_WEIGHTED):
    n = xyz.shape[0]
    idx = np.arange(n)
    return kernel_entries(xyz, area, idx, idx, reading)


def exact_matvec(xyz, area, x, reading=READING_WEIGHTED, rows=None, chunk=512):
    """y = A[rows,:] x by direct summation (no compression).  x: n or n x k."""
    n = xyz.shape[0]
    rows = np.arange(n) if rows is None else np.asarray(rows)
    x2 = x.reshape(n, -1)
    out = np.empty((rows.size, x2.shape[1]))
    cols = np.arange(n)
    for a in range(0, rows.size, chunk):
        blk = kernel_entries(xyz, area, rows[a:a + chunk], cols, reading)
        out[a:a + chunk] = blk @ x2
    return out.reshape((rows.size,) + x.shape[1:])


def exact_inf_norm(xyz, area, reading=READING_WEIGHTED, chunk=512):
    """max_i sum_j |A_ij| by direct summation."""
    n = xyz.shape[0]
    cols = np.arange(n)
    best = 0.0
    for a in range(0, n, chunk):
        blk = kernel_entries(xyz, area, np.arange(a, min(n, a + chunk)), cols, reading)
        best = max(best, float(np.abs(blk).sum(axis=1).max()))
    return best


# ---------------------------------------------------------------------------
# cluster tree (Algorithm 1)
# ---------------------------------------------------------------------------
class Cluster:
    __slots__ = ("off", "size", "lo", "hi", "sons", "leaf_id", "level")

    def __init__(self, off, size, lo, hi, level):
        self.off, self.size, self.lo, self.hi = off, size, lo, hi
        self.sons = []
        self.leaf_id = -1
        self.level = level

    @property
    def is_leaf(self):
        return not self.sons

    def diam(self):
        return float(np.linalg.norm(self.hi - self.lo))


def cluster_tree(xyz, leaf_size):
    """Algorithm 1: bisect the degrees of freedom while size > C_lf.

    Returns (root, perm, leaves).  perm[p] is the original index of the point
    at cluster position p; clusters cover contiguous ranges of positions.
    """
    perm = []
    leaves = []

    def build(idx, level):
        pts = xyz[idx]
        lo, hi = pts.min(axis=0), pts.max(axis=0)
        c = Cluster(len(perm), idx.size, lo, hi, level)
        if idx.size > leaf_size:
            d = int(np.argmax(hi - lo))
            mid = 0.5 * (lo[d] + hi[d])
            mask = pts[:, d] < mid
            left, right = idx[mask], idx[~mask]
            if left.size == 0 or right.size == 0:
                order = np.lexsort((idx, pts[:, d]))
                srt = idx[order]
                left, right = srt[: idx.size // 2], srt[idx.size // 2:]
            c.sons = [build(left, level + 1), build(right, level + 1)]
        else:
            c.leaf_id = len(leaves)
            leaves.append(c)
            perm.extend(idx.tolist())
        return c

    root = build(np.arange(xyz.shape[0]), 0)
    # offsets: leaves appended in DFS order, so fix internal offsets
    def fix(c):
        if c.sons:
            for s in c.sons:
                fix(s)
            c.off = c.sons[0].off
    fix(root)
    return root, np.array(perm, dtype=np.int64), leaves


# ---------------------------------------------------------------------------
# block tree (Algorithm 2) and storage
# ---------------------------------------------------------------------------
def admissible(t, s, eta):
    """min(diam t, diam s) <= eta * dist(t, s) on the bounding boxes."""
    gap = np.maximum(0.0, np.maximum(s.lo - t.hi, t.lo - s.hi))
    dist = float(np.linalg.norm(gap))
    if eta <= 0.0 or dist <= 0.0:
        return False
    return min(t.diam(), s.diam()) <= eta * dist


class Block:
    """One node of the block tree: kind 'F' (dense), 'R' (low-rank U V^T) or
    'H' (2x2 sons)."""
    __slots__ = ("t", "s", "kind", "F", "U", "V", "sons", "piv", "info")

    def __init__(self, t, s, kind):
        self.t, self.s, self.kind = t, s, kind
        self.F = self.U = self.V = None
        self.sons = None
        self.piv = None
        self.info = 0

    @property
    def shape(self):
        return (self.t.size, self.s.size)


def block_tree(t, s, eta):
    """Algorithm 2."""
    if admissible(t, s, eta):
        return Block(t, s, "R")
    if t.sons and s.sons:
        b = Block(t, s, "H")
        b.sons = [[block_tree(ti, sj, eta) for sj in s.sons] for ti in t.sons]
        return b
    return Block(t, s, "F")


def leaves_of(b):
    if b.kind == "H":
        for row in b.sons:
            for c in row:
                yield from leaves_of(c)
    else:
        yield b


# ---------------------------------------------------------------------------
# truncation rule and the SVD-based recompression (Sec. 3.1)
# ---------------------------------------------------------------------------
class Rule:
    """Rank choice after an SVD: fixed rank, or smallest k with
    ||sigma_{k+1:}||_2 <= eps ||sigma||_2, capped at cap."""

    def __init__(self, eps=0.0, cap=32, fixed=0):
        self.eps, self.cap, self.fixed = float(eps), int(cap), int(fixed)
        self.log = []          # (k, discarded tail, block norm, capped)

    def choose(self, sig, norm2=None):
        sig = np.asarray(sig, dtype=np.float64)
        tot2 = float(np.sum(sig * sig)) if norm2 is None else float(norm2)
        # tail2[k] = sum_{i>=k} sigma_i^2
        tail2 = np.concatenate([np.cumsum((sig * sig)[::-1])[::-1], [0.0]])
        if norm2 is not None:
            head = np.concatenate([[0.0], np.cumsum(sig * sig)])
            tail2 = np.maximum(tot2 - head, 0.0)
        if self.fixed > 0:
            k = min(self.fixed, sig.size)
            capped = False
        else:
            thr = (self.eps ** 2) * tot2
            k = int(np.argmax(tail2 <= thr)) if np.any(tail2 <= thr) else sig.size
            capped = k > self.cap
            k = min(k, self.cap)
        self.log.append((k, math.sqrt(max(tail2[k], 0.0)), math.sqrt(tot2), capped))
        return k


def truncate(X, Y, rule):
    """Best rank-k approximation of X Y^T (Sec. 3.1, addition of low-rank
    matrices): QR of both stacks, SVD of R_X R_Y^T, keep the leading k
    singular triplets; Sigma goes into the left factor.
    Parity: pinned against numpy's SVD of the dense product (Eckart-Young)."""
    m, K = X.shape
    n = Y.shape[0]
    if K == 0 or m == 0 or n == 0:
        rule.log.append((0, 0.0, 0.0, False))
        return np.zeros((m, 0)), np.zeros((n, 0))
    Qx, Rx = np.linalg.qr(X, mode="reduced")
    Qy, Ry = np.linalg.qr(Y, mode="reduced")
    M = Rx @ Ry.T
    u, sig, vt = np.linalg.svd(M, full_matrices=False)
    k = rule.choose(sig)
    U = Qx @ (u[:, :k] * sig[:k])
    V = Qy @ vt[:k].T
    # QR of both stacks, core product, SVD (Golub-Van Loan count), recombination
    _count(2.0 * (m + n) * K * K - 4.0 * K ** 3 / 3.0 + 2.0 * K ** 3 + 21.0 * K ** 3
           + 2.0 * (m + n) * K * k)
    return U, V


# ---------------------------------------------------------------------------
# assembly of the H-matrix (dense near field; SVD-compressed far field)
# ---------------------------------------------------------------------------
def _compress_block(Ablk, rule, rng, dense_limit=384, oversample=10, power=2):
    m, n = Ablk.shape
    norm2 = float(np.sum(Ablk * Ablk))
    if min(m, n) <= dense_limit:
        u, sig, vt = np.linalg.svd(Ablk, full_matrices=False)
        k = rule.choose(sig)
        return u[:, :k] * sig[:k], vt[:k].T
    # randomised range finder with power iterations (Halko, Martinsson,
    # Tropp 2011, Alg. 4.4), then SVD of the projected block
    ell = min(min(m, n), (rule.fixed if rule.fixed > 0 else rule.cap) + oversample)
    Om = rng.standard_normal((n, ell))
    Q, _ = np.linalg.qr(Ablk @ Om)
    for _ in range(power):
        W, _ = np.linalg.qr(Ablk.T @ Q)
        Q, _ = np.linalg.qr(Ablk @ W)
    B = Q.T @ Ablk
    u, sig, vt = np.linalg.svd(B, full_matrices=False)
    k = rule.choose(sig, norm2=None if rule.fixed > 0 else norm2)
    return (Q @ u[:, :k]) * sig[:k], vt[:k].T


class HMatrix:
    """An assembled H-matrix in cluster order plus its trees."""

    def __init__(self, xyz, area, leaf_size, eta, rule, reading=READING_WEIGHTED,
                 seed=0):
        self.xyz, self.area = np.asarray(xyz, np.float64), np.asarray(area, np.float64)
        self.n = self.xyz.shape[0]
        self.reading = reading
        self.rule = rule
        self.root, self.perm, self.leaves = cluster_tree(self.xyz, leaf_size)
        self.xyz_p = self.xyz[self.perm]
        self.area_p = self.area[self.perm]
        self.block = block_tree(self.root, self.root, eta)
        rng = np.random.default_rng(seed)
        for b in leaves_of(self.block):
            rows = np.arange(b.t.off, b.t.off + b.t.size)
            cols = np.arange(b.s.off, b.s.off + b.s.size)
            Ablk = kernel_entries(self.xyz_p, self.area_p, rows, cols, reading)
            if b.kind == "F":
                b.F = Ablk
            else:
                b.U, b.V = _compress_block(Ablk, rule, rng)
        self.factored = False

    # -- structure statistics -------------------------------------------------
    def stats(self):
        nf = nr = 0
        for b in leaves_of(self.block):
            if b.kind == "F":
                nf += 1
            else:
                nr += 1
        return dict(n=self.n, leaves=len(self.leaves), dense=nf, lowrank=nr)

    def to_dense(self):
        """Expand the (unfactored) H-matrix to a dense array in cluster order."""
        A = np.zeros((self.n, self.n))
        for b in leaves_of(self.block):
            sl = (slice(b.t.off, b.t.off + b.t.size), slice(b.s.off, b.s.off + b.s.size))
            A[sl] = b.F if b.kind == "F" else b.U @ b.V.T
        return A


# ---------------------------------------------------------------------------
# products of a block with a dense panel (Sec. 3.1 low-rank products)
# ---------------------------------------------------------------------------
def mul(M, X):
    """M X for a block of any kind; X has |s| rows."""
    if M.kind == "F":
        _count(2.0 * M.F.shape[0] * M.F.shape[1] * X.shape[1])
        return M.F @ X
    if M.kind == "R":
        _count(2.0 * M.U.shape[1] * X.shape[1] * (M.U.shape[0] + M.V.shape[0]))
        return M.U @ (M.V.T @ X)
    out = np.zeros((M.t.size, X.shape[1]))
    for i, ti in enumerate(M.t.sons):
        ri = slice(ti.off - M.t.off, ti.off - M.t.off + ti.size)
        for j, sj in enumerate(M.s.sons):
            cj = slice(sj.off - M.s.off, sj.off - M.s.off + sj.size)
            out[ri] += mul(M.sons[i][j], X[cj])
    return out


def mulT(M, X):
    """M^T X for a block of any kind; X has |t| rows."""
    if M.kind == "F":
        _count(2.0 * M.F.shape[0] * M.F.shape[1] * X.shape[1])
        return M.F.T @ X
    if M.kind == "R":
        _count(2.0 * M.U.shape[1] * X.shape[1] * (M.U.shape[0] + M.V.shape[0]))
        return M.V @ (M.U.T @ X)
    out = np.zeros((M.s.size, X.shape[1]))
    for i, ti in enumerate(M.t.sons):
        ri = slice(ti.off - M.t.off, ti.off - M.t.off + ti.size)
        for j, sj in enumerate(M.s.sons):
            cj = slice(sj.off - M.s.off, sj.off - M.s.off + sj.size)
            out[cj] += mulT(M.sons[i][j], X[ri])
    return out


def _rows(parent, child):
    return slice(child.off - parent.off, child.off - parent.off + child.size)


# ---------------------------------------------------------------------------
# dense leaf LU with partial pivoting
# ---------------------------------------------------------------------------
def getrf(a):
    """Right-looking unblocked Gaussian elimination with partial pivoting,
    in place.  Pivot = first index of the largest |a_ik|; a zero pivot sets
    info (1-based column) and skips the scaling, as LAPACK's getrf does.
    Returns (piv, info) with piv[k] the row swapped with row k (0-based).
    Parity: pinned against scipy.linalg.lu_factor (LAPACK)."""
    b = a.shape[0]
    piv = np.zeros(b, dtype=np.int64)
    info = 0
    for k in range(b):
        p = k + int(np.argmax(np.abs(a[k:, k])))
        piv[k] = p
        if a[p, k] != 0.0:
            if p != k:
                a[[k, p], :] = a[[p, k], :]
            a[k + 1:, k] = a[k + 1:, k] / a[k, k]
        elif info == 0:
            info = k + 1
        a[k + 1:, k + 1:] -= np.outer(a[k + 1:, k], a[k, k + 1:])
    _count(getrf_flops(b))
    return piv, info


def apply_piv(piv, Y):
    for k, p in enumerate(piv):
        if p != k:
            Y[[k, p]] = Y[[p, k]]


# ---------------------------------------------------------------------------
# triangular solves on panels (Sec. 3.1; partitioned RHS O2.1-O2.6)
# ---------------------------------------------------------------------------
def fwd(Lb, Y):
    """Y := L^{-1} P Y for the factored diagonal block Lb (rows of Y = t),
    leaf permutations applied after the updates from earlier leaves."""
    if Lb.kind == "F":
        apply_piv(Lb.piv, Y)
        Y[:] = sla.solve_triangular(Lb.F, Y, lower=True, unit_diagonal=True,
                                    check_finite=False)
        _count(float(Y.shape[0]) ** 2 * Y.shape[1])
        return
    t0, t1 = Lb.t.sons
    Y0, Y1 = Y[_rows(Lb.t, t0)], Y[_rows(Lb.t, t1)]
    fwd(Lb.sons[0][0], Y0)
    Y1 -= mul(Lb.sons[1][0], Y0)
    fwd(Lb.sons[1][1], Y1)


def bwdT(Ub, Y):
    """Y := U^{-T} Y (forward substitution with U^T), rows of Y = t."""
    if Ub.kind == "F":
        Y[:] = sla.solve_triangular(Ub.F, Y, lower=False, trans="T",
                                    check_finite=False)
        _count(float(Y.shape[0]) ** 2 * Y.shape[1])
        return
    t0, t1 = Ub.t.sons
    Y0, Y1 = Y[_rows(Ub.t, t0)], Y[_rows(Ub.t, t1)]
    bwdT(Ub.sons[0][0], Y0)
    Y1 -= mulT(Ub.sons[0][1], Y0)
    bwdT(Ub.sons[1][1], Y1)


def bwd(Ub, Y):
    """Y := U^{-1} Y (backward substitution), rows of Y = t."""
    if Ub.kind == "F":
        Y[:] = sla.solve_triangular(Ub.F, Y, lower=False, check_finite=False)
        _count(float(Y.shape[0]) ** 2 * Y.shape[1])
        return
    t0, t1 = Ub.t.sons
    Y0, Y1 = Y[_rows(Ub.t, t0)], Y[_rows(Ub.t, t1)]
    bwd(Ub.sons[1][1], Y1)
    Y0 -= mul(Ub.sons[0][1], Y1)
    bwd(Ub.sons[0][0], Y0)


def trsm_l(Lb, B, rule):
    """B := L^{-1} P B for a block B = (t, s) of any kind (O1.2 / O2)."""
    if B.kind == "R":
        fwd(Lb, B.U)
    elif B.kind == "F":
        fwd(Lb, B.F)
    else:
        for j in range(2):
            trsm_l(Lb.sons[0][0], B.sons[0][j], rule)
        for j in range(2):
            gemm(B.sons[1][j], Lb.sons[1][0], B.sons[0][j], rule)
        for j in range(2):
            trsm_l(Lb.sons[1][1], B.sons[1][j], rule)


def trsm_u(B, Ub, rule):
    """B := B U^{-1} for a block B = (s, t) of any kind (O1.3 / O3)."""
    if B.kind == "R":
        bwdT(Ub, B.V)
    elif B.kind == "F":
        Ft = np.ascontiguousarray(B.F.T)
        bwdT(Ub, Ft)
        B.F = Ft.T.copy()
    else:
        for i in range(2):
            trsm_u(B.sons[i][0], Ub.sons[0][0], rule)
        for i in range(2):
            gemm(B.sons[i][1], B.sons[i][0], Ub.sons[0][1], rule)
        for i in range(2):
            trsm_u(B.sons[i][1], Ub.sons[1][1], rule)


# ---------------------------------------------------------------------------
# H-GEMM  C := C - A B  with truncation (O1.4 / O4)
# ---------------------------------------------------------------------------
def add_lr(C, X, Y, rule):
    """C := C - X Y^T, C of any kind; truncated when C is low-rank."""
    if C.kind == "F":
        _count(2.0 * X.shape[0] * Y.shape[0] * X.shape[1])
        C.F -= X @ Y.T
    elif C.kind == "R":
        C.U, C.V = truncate(np.hstack([C.U, -X]), np.hstack([C.V, Y]), rule)
    else:
        for i, ti in enumerate(C.t.sons):
            for j, sj in enumerate(C.s.sons):
                add_lr(C.sons[i][j], X[_rows(C.t, ti)], Y[_rows(C.s, sj)], rule)


# how often each product kind was taken (read by the tests to check that a
# workload exercises every case)
CASES = {}


def _case(name):
    CASES[name] = CASES.get(name, 0) + 1


def gemm(C, A, B, rule):
    """C := C - A B following the product kinds of standard H-arithmetic."""
    _case(A.kind + B.kind + C.kind)
    if A.kind == "R":
        add_lr(C, A.U, mulT(B, A.V), rule)
    elif B.kind == "R":
        add_lr(C, mul(A, B.U), B.V, rule)
    elif A.kind == "F" and B.kind == "F":
        if A.s.is_leaf:
            add_lr(C, A.F, B.F.T, rule)          # rank |r| product
        else:
            D = A.F @ B.F                          # t and s are leaves
            _count(2.0 * A.F.shape[0] * A.F.shape[1] * B.F.shape[1])
            if C.kind == "F":
                C.F -= D
            else:
                add_lr(C, D, np.eye(C.s.size), rule)
    elif A.kind == "H" and B.kind == "F":      # s is a leaf
        add_lr(C, mul(A, B.F), np.eye(C.s.size), rule)
    elif A.kind == "F" and B.kind == "H":      # t is a leaf
        add_lr(C, np.eye(C.t.size), mulT(B, A.F.T), rule)
    else:                                       # both partitioned
        if C.kind == "H":
            for i in range(2):
                for j in range(2):
                    for l in range(2):
                        gemm(C.sons[i][j], A.sons[i][l], B.sons[l][j], rule)
        elif C.kind == "R":
            # four virtual low-rank sons, recursive update, agglomeration
            sons = [[None, None], [None, None]]
            for i, ti in enumerate(C.t.sons):
                for j, sj in enumerate(C.s.sons):
                    v = Block(ti, sj, "R")
                    v.U = C.U[_rows(C.t, ti)].copy()
                    v.V = C.V[_rows(C.s, sj)].copy()
                    sons[i][j] = v
            for i in range(2):
                for j in range(2):
                    for l in range(2):
                        gemm(sons[i][j], A.sons[i][l], B.sons[l][j], rule)
            Xs, Ys = [], []
            for i, ti in enumerate(C.t.sons):
                for j, sj in enumerate(C.s.sons):
                    v = sons[i][j]
                    Xp = np.zeros((C.t.size, v.U.shape[1]))
                    Yp = np.zeros((C.s.size, v.V.shape[1]))
                    Xp[_rows(C.t, ti)] = v.U
                    Yp[_rows(C.s, sj)] = v.V
                    Xs.append(Xp)
                    Ys.append(Yp)
            C.U, C.V = truncate(np.hstack(Xs), np.hstack(Ys), rule)
        else:
            raise AssertionError("dense target with two partitioned operands")


# ---------------------------------------------------------------------------
# H-LU (O1.1 - O5.5, recursive)
# ---------------------------------------------------------------------------
class _ZeroPivot(Exception):
    pass


def lu(Ab, rule, info):
    if Ab.kind == "F":
        Ab.piv, inf = getrf(Ab.F)
        if inf:
            # the leaf elimination itself finishes (LAPACK semantics); the
            # solves that would use the singular U are not attempted
            info[0] = Ab.t.off + inf
            raise _ZeroPivot()
        return
    assert Ab.kind == "H", "diagonal blocks are never admissible"
    A00, A01 = Ab.sons[0]
    A10, A11 = Ab.sons[1]
    lu(A00, rule, info)
    trsm_l(A00, A01, rule)
    trsm_u(A10, A00, rule)
    gemm(A11, A10, A01, rule)
    lu(A11, rule, info)


def factor(H):
    """Factor H in place.  Returns the first zero-pivot position (1-based in
    cluster order) or 0."""
    info = [0]
    try:
        lu(H.block, H.rule, info)
    except _ZeroPivot:
        return info[0]
    H.factored = True
    return info[0]


# ---------------------------------------------------------------------------
# the other H-arithmetic operations on the same primitives (Sec. 2: H2Lib
# offers H-matrix multiplication and inversion beside the H-LU)
# ---------------------------------------------------------------------------
def _blank(b, fill):
    """A block tree with b's structure; leaves from fill(leaf) -> (F) or
    (U, V)."""
    c = Block(b.t, b.s, b.kind)
    if b.kind == "H":
        c.sons = [[_blank(x, fill) for x in row] for row in b.sons]
    elif b.kind == "F":
        c.F = fill(b)
    else:
        c.U, c.V = fill(b)
    return c


def _zero(b):
    return np.zeros((b.t.size, b.s.size)) if b.kind == "F" else \
        (np.zeros((b.t.size, 0)), np.zeros((b.s.size, 0)))


def _ident(b):
    if b.kind == "F":
        return np.eye(b.t.size) if b.t is b.s else np.zeros((b.t.size, b.s.size))
    return np.zeros((b.t.size, 0)), np.zeros((b.s.size, 0))


def _negate(b):
    for lf in leaves_of(b):
        if lf.kind == "F":
            lf.F = -lf.F
        else:
            lf.U = -lf.U


def hmul(HA, HB, rule):
    """C ~= A B in H-format on A's block tree (A and B on the same trees):
    C starts at zero and takes the H-GEMM C := C - A B of the H-LU (every
    update truncated to the rule), then its sign is flipped.  Returns the
    root block of C (cluster order)."""
    C = _blank(HA.block, _zero)
    gemm(C, HA.block, HB.block, rule)
    _negate(C)
    return C


def hinv(HA, rule):
    """X ~= A^{-1} in H-format through the first steps of the H-LU of the
    doubled matrix [A I; I 0] (Sec. 3.1): LU of A, the two triangular solves
    on the identity blocks, and the Schur-complement update of the zero
    block, which then holds -A^{-1}; its sign is flipped.  A is factored in
    place.  Returns the root block of X (cluster order)."""
    I12 = _blank(HA.block, _ident)
    I21 = _blank(HA.block, _ident)
    X = _blank(HA.block, _zero)
    info = [0]
    lu(HA.block, rule, info)
    trsm_l(HA.block, I12, rule)
    trsm_u(I21, HA.block, rule)
    gemm(X, I21, I12, rule)
    _negate(X)
    return X


def block_dense(b, n):
    """Dense n x n expansion of a block tree (cluster order)."""
    A = np.zeros((n, n))
    for lf in leaves_of(b):
        sl = (slice(lf.t.off, lf.t.off + lf.t.size), slice(lf.s.off, lf.s.off + lf.s.size))
        A[sl] = lf.F if lf.kind == "F" else lf.U @ lf.V.T
    return A


def solve(H, b):
    """x = A_H^{-1} b in the caller's original point order (b: n or n x k)."""
    assert H.factored
    shape = b.shape
    Y = np.array(b.reshape(H.n, -1)[H.perm], dtype=np.float64)
    fwd(H.block, Y)
    bwd(H.block, Y)
    x = np.empty_like(Y)
    x[H.perm] = Y
    return x.reshape(shape)


def hmatvec(H, x):
    """y = A_H x with the unfactored H-matrix (original point order)."""
    assert not H.factored
    shape = x.shape
    X = x.reshape(H.n, -1)[H.perm]
    Y = mul(H.block, X)
    y = np.empty_like(Y)
    y[H.perm] = Y
    return y.reshape(shape)


def factors_dense(H):
    """(Lhat, U) dense in cluster order: A_H ~= Lhat U, with the diagonal leaf
    blocks of Lhat equal to P^T L (lazy pivoting)."""
    n = H.n
    Lh = np.zeros((n, n))
    U = np.zeros((n, n))
    for b in leaves_of(H.block):
        rs = slice(b.t.off, b.t.off + b.t.size)
        cs = slice(b.s.off, b.s.off + b.s.size)
        M = b.F if b.kind == "F" else b.U @ b.V.T
        if b.t is b.s:
            L = np.tril(M, -1) + np.eye(b.t.size)
            P = np.eye(b.t.size)
            apply_piv(b.piv, P)       # P: rows swapped as in the elimination
            Lh[rs, cs] = P.T @ L
            U[rs, cs] = np.triu(M)
        elif b.t.off > b.s.off:
            Lh[rs, cs] = M
        else:
            U[rs, cs] = M
    return Lh, U


# ---------------------------------------------------------------------------
# iterative refinement with the exact operator
# ---------------------------------------------------------------------------
def backward_error(xyz, area, x, b, reading=READING_WEIGHTED, anorm=None, rows=None):
    """max_j ||r_j||_inf / (||A||_inf ||x_j||_inf + ||b_j||_inf), exact A.
    With `rows`, the residual is sampled on those rows only."""
    x2 = x.reshape(x.shape[0], -1)
    b2 = b.reshape(b.shape[0], -1)
    if anorm is None:
        anorm = exact_inf_norm(xyz, area, reading)
    Ax = exact_matvec(xyz, area, x2, reading, rows=rows)
    bb = b2 if rows is None else b2[rows]
    r = bb - Ax
    eta = np.abs(r).max(axis=0) / (anorm * np.abs(x2).max(axis=0) + np.abs(b2).max(axis=0))
    return float(eta.max())


def refine(H, b, tol=1e-10, max_iter=10, anorm=None):
    """x0 = solve(b); repeat r = b - A x (exact), x += solve(r) until the
    backward error is <= tol.  Returns (x, history)."""
    if anorm is None:
        anorm = exact_inf_norm(H.xyz, H.area, H.reading)
    x = solve(H, b)
    hist = []
    for _ in range(max_iter + 1):
        x2, b2 = x.reshape(H.n, -1), b.reshape(H.n, -1)
        r = b2 - exact_matvec(H.xyz, H.area, x2, H.reading)
        eta = float((np.abs(r).max(axis=0) /
                     (anorm * np.abs(x2).max(axis=0) + np.abs(b2).max(axis=0))).max())
        hist.append(eta)
        if eta <= tol or len(hist) > max_iter:
            break
        x = x + solve(H, r.reshape(b.shape))
    return x, hist


# ---------------------------------------------------------------------------
# flop model (per executed op) for GFLOP/s figures
# ---------------------------------------------------------------------------
def getrf_flops(b):
    return 2.0 * b ** 3 / 3.0 - b * b / 2.0 + 5.0 * b / 6.0
