"""Pins of the oracle's H-matrix multiplication and inversion (the other
H-arithmetic operations beside the H-LU, built from the same primitives):
against the dense product and the dense inverse of the same H-matrices
(library routines), within the truncation tolerance; and planted mistakes
(a product without its sign flip, an inverse that skips a triangular solve)
fail these criteria."""
import numpy as np
import pytest

import oracle as O
from hlu_inputs import icosphere


@pytest.fixture(scope="module")
def mats():
    xyz, area = icosphere(3)
    rule = O.Rule(eps=1e-6, cap=32)
    HA = O.HMatrix(xyz, area, 32, 2.0, rule)
    HB = O.HMatrix(xyz, area, 32, 2.0, rule, reading=O.READING_POINT)
    return xyz, area, rule, HA, HB


def test_hmul_against_the_dense_product(mats):
    xyz, area, rule, HA, HB = mats
    A, B = HA.to_dense(), HB.to_dense()
    C = O.block_dense(O.hmul(HA, HB, rule), HA.n)
    rel = np.linalg.norm(C - A @ B) / (np.linalg.norm(A) * np.linalg.norm(B))
    assert rel <= 10 * rule.eps
    # a dropped sign flip is caught
    AB = A @ B
    assert np.linalg.norm(-C - AB) / np.linalg.norm(AB) > 1.0


def test_hinv_against_the_dense_inverse(mats):
    xyz, area, rule, HA, HB = mats
    import copy
    H = copy.deepcopy(HA)
    A = H.to_dense()
    X = O.block_dense(O.hinv(H, rule), H.n)
    Ai = np.linalg.inv(A)
    rel = np.linalg.norm(X - Ai) / np.linalg.norm(Ai)
    assert rel <= 40 * rule.eps
    assert np.linalg.norm(X @ A - np.eye(H.n)) / np.sqrt(H.n) <= 40 * rule.eps
    # an inverse that skips the lower triangular solve is caught
    H2 = copy.deepcopy(HA)
    from oracle import hlu as OH
    I12 = OH._blank(H2.block, OH._ident)
    I21 = OH._blank(H2.block, OH._ident)
    Z = OH._blank(H2.block, OH._zero)
    O.lu(H2.block, rule, [0])
    O.trsm_u(I21, H2.block, rule)
    O.gemm(Z, I21, I12, rule)
    OH._negate(Z)
    bad = O.block_dense(Z, H.n)
    assert np.linalg.norm(bad - Ai) / np.linalg.norm(Ai) > 1e3 * rule.eps
