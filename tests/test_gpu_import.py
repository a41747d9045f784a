"""One H-matrix, two factorisations: the oracle's assembled A_H is
imported into the device handle (hlu_import_blocks), so the device and the
oracle factor the very same blocks (MI355X only, through the C-ABI).

Bounds (Sec. 3.1 recursion with truncation to eps after the products):
|A_H - Lhat U|_F <= 10 eps |A_H|_F on either side, hence the two factor
operators differ by at most 20 eps |A_H|_F.  The first diagonal leaf sees no
update before its LU, so its pivots (and, in FP64, its factors) are equal
bit for bit; later leaves see Schur complements that differ by the
truncation error, and their pivots are reported and must agree for nearly
all leaves."""
import sys

import numpy as np
import pytest

import oracle as O
from hblocks import write_blocks
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


@pytest.mark.parametrize("prec,leaf,eps", [(0, 32, 1e-6), (1, 64, 1e-5)])
def test_same_A_H_factors_vs_oracle(P, tmp_path, prec, leaf, eps):
    xyz, area = icosphere(4)
    _say("import: n", xyz.shape[0], "leaf", leaf, "eps", eps, "precision", prec)
    H = O.HMatrix(xyz, area, leaf, 2.0, O.Rule(eps=eps, cap=32))
    path = tmp_path / "a_h.bin"
    write_blocks(H, path)
    A_H = H.to_dense()
    h = P.HLU(xyz, area, leaf=leaf, eta=2.0, eps=eps, cap=32, precision=prec)
    assert np.array_equal(h.perm(), H.perm)
    h.import_blocks(path)
    h.set_executor(1)
    h.factor()
    st, inf = h.sync(check=False)
    assert st == 0 and inf.info == 0
    Lg, Ug = h.export_factors()
    pg = h.export_pivots()
    assert O.factor(H) == 0
    Lo, Uo = O.factors_dense(H)
    nA = np.linalg.norm(A_H)
    e_g = np.linalg.norm(A_H - Lg @ Ug) / nA
    e_o = np.linalg.norm(A_H - Lo @ Uo) / nA
    e_go = np.linalg.norm(Lg @ Ug - Lo @ Uo) / nA
    diag = {b.t.off: b for b in O.leaves_of(H.block) if b.t is b.s}
    same = [np.array_equal(pg[lf.off:lf.off + lf.size], diag[lf.off].piv) for lf in H.leaves]
    _say("same A_H: |A_H - LU| device", e_g, "oracle", e_o, "|LU_dev - LU_orc|", e_go,
         "leaves with equal pivots", sum(same), "/", len(same))
    assert e_g <= 10 * eps and e_o <= 10 * eps
    assert e_go <= 20 * eps
    assert same[0]
    assert sum(same) >= 0.9 * len(same)
    if prec == 0:
        lf = H.leaves[0]
        sl = slice(lf.off, lf.off + lf.size)
        assert np.array_equal(Lg[sl, sl], Lo[sl, sl])
        assert np.array_equal(Ug[sl, sl], Uo[sl, sl])
