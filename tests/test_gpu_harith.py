"""H-matrix multiplication and inversion on the device (MI355X, through the
C-ABI): PRODUCT and INVERSE plans run the H-GEMM and the first H-LU steps of
a doubled H-matrix (include/hlu.h, hlu_operation).  Checked against the
exact dense product / inverse of the kernel matrices and against the
oracle's H-multiplication / H-inversion on the same trees."""
import sys

import numpy as np
import pytest

import oracle as O
from hlu_inputs import icosphere

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


def _orig(Xc, perm):
    X = np.zeros_like(Xc)
    X[np.ix_(perm, perm)] = Xc
    return X


@pytest.mark.parametrize("prec", [0, 1])
def test_hmul_vs_dense_and_oracle(P, prec):
    xyz, area = icosphere(3)
    eps = 1e-6
    _say("H-product n", xyz.shape[0], "precision", prec)
    h = P.HLU(xyz, area, leaf=32, eta=2.0, eps=eps, cap=32, cap_mv=0, precision=prec,
              operation=P.OP_PRODUCT, kernel_b=P.KERNEL_POINT)
    h.set_executor(1)
    h.factor()
    st, inf = h.sync(check=False)
    assert st == 0
    C = h.export_result()
    A = O.dense_matrix(xyz, area)
    B = O.dense_matrix(xyz, area, O.READING_POINT)
    nAB = np.linalg.norm(A) * np.linalg.norm(B)
    rel = np.linalg.norm(C - A @ B) / nAB
    rule = O.Rule(eps=eps, cap=32)
    HA = O.HMatrix(xyz, area, 32, 2.0, rule)
    HB = O.HMatrix(xyz, area, 32, 2.0, rule, reading=O.READING_POINT)
    Co = _orig(O.block_dense(O.hmul(HA, HB, rule), HA.n), HA.perm)
    ro = np.linalg.norm(Co - A @ B) / nAB
    rp = np.linalg.norm(C - Co) / nAB
    _say("H-product: |C - A B| device", rel, "oracle", ro, "|C_dev - C_orc|", rp, "cap hits",
         inf.cap_hits)
    assert rel <= 10 * eps and ro <= 10 * eps and rp <= 20 * eps


@pytest.mark.parametrize("prec", [0, 1])
def test_hinv_vs_dense_and_oracle(P, prec):
    import copy
    xyz, area = icosphere(3)
    eps = 1e-6
    _say("H-inverse n", xyz.shape[0], "precision", prec)
    h = P.HLU(xyz, area, leaf=32, eta=2.0, eps=eps, cap=32, cap_mv=0, precision=prec,
              operation=P.OP_INVERSE)
    h.set_executor(1)
    h.factor()
    st, inf = h.sync(check=False)
    assert st == 0 and inf.info == 0
    X = h.export_result()
    A = O.dense_matrix(xyz, area)
    Ai = np.linalg.inv(A)
    rel = np.linalg.norm(X - Ai) / np.linalg.norm(Ai)
    res = np.linalg.norm(X @ A - np.eye(A.shape[0])) / np.sqrt(A.shape[0])
    rule = O.Rule(eps=eps, cap=32)
    HA = O.HMatrix(xyz, area, 32, 2.0, rule)
    Xo = _orig(O.block_dense(O.hinv(copy.deepcopy(HA), rule), HA.n), HA.perm)
    rp = np.linalg.norm(X - Xo) / np.linalg.norm(Ai)
    _say("H-inverse: |X - A^-1|/|A^-1|", rel, "|XA - I|/sqrt(n)", res, "|X_dev - X_orc|", rp,
         "cap hits", inf.cap_hits)
    assert rel <= 40 * eps and res <= 40 * eps and rp <= 80 * eps


def test_product_and_inverse_plans_refuse_lu_calls(P):
    import torch
    xyz, area = icosphere(2)
    h = P.HLU(xyz, area, leaf=16, eta=2.0, eps=1e-6, cap=32, cap_mv=0, operation=P.OP_INVERSE)
    h.factor()
    h.sync()
    with pytest.raises(P.HLUError) as e:
        h.solve(torch.zeros(h.n, dtype=torch.float64, device="cuda"))
    assert e.value.status == 6
    with pytest.raises(P.HLUError) as e:
        h.export_factors()
    assert e.value.status == 6
