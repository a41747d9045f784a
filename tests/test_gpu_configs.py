"""Device path against the oracle at the workloads' own settings (MI355X
only, through the C-ABI).

* n = 20480 (level-5 icosphere), leaf 64, eta 2, eps 1e-6, capacity 32,
  FP64, 8 right-hand sides ~ N(0,1) seed 1, dataflow executor.  The oracle's
  solutions of the same inputs are stored on 256 sampled rows
  (tests/golden/c2_oracle.npz, written by make_c2_oracle.py from the oracle
  alone).
* n = 5120 (level 4), leaf 64, eps 1e-5, mixed precision: the oracle runs
  in the test.

Bounds (forward errors, infinity norm, kappa_inf <= 4 for this operator):
* unrefined: |A - Lhat U| <= 10 eps |A| on either side, so each solution is
  within kappa * 10 eps of the exact one, and the two within twice that;
* refined: both backward errors are at most max(eta, eps_mv), so the two
  solutions agree to 4 kappa max(eta) (the device measures its eta with the
  eps_mv = 1e-12 operator copy).
"""
import os
import sys

import numpy as np
import pytest

import oracle as O
from hlu_inputs import config_inputs, icosphere, rhs_normal

pytestmark = pytest.mark.gpu

KAPPA = 4.0
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c2_oracle.npz")


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


def _solve(torch, h, b, tol):
    h.set_refinement(tol, 10)
    x = h.solve(torch.tensor(b, device="cuda")).cpu().numpy()
    st, inf = h.sync(check=False)
    assert st == 0, (st, inf.eta_final)
    return x, inf


@pytest.fixture(scope="module")
def c2(P):
    import torch
    g = np.load(GOLD)
    xyz, area, cfg = config_inputs("c2")
    n = xyz.shape[0]
    _say("c2 plan+assemble n", n)
    h = P.HLU(xyz, area, leaf=cfg["leaf"], eta=cfg["eta"], eps=cfg["eps"], cap=cfg["cap"],
              eps_mv=1e-12, cap_mv=64, precision=P.PREC_FP64, refine_tol=1e-10,
              max_nrhs=cfg["nrhs"])
    h.set_executor(1)
    _say("c2 factor")
    h.factor()
    st, inf = h.sync(check=False)
    assert st == 0 and inf.info == 0
    b = rhs_normal(cfg["seed"], n, cfg["nrhs"])
    return torch, h, g, b, xyz, area


def test_c2_unrefined_vs_oracle(c2):
    torch, h, g, b, xyz, area = c2
    x0, inf = _solve(torch, h, b, 0.0)
    assert inf.iters == 0
    rows = g["rows"]
    xr = g["xr"]
    sc = g["xr_inf"]
    e_dev = (np.abs(x0[rows] - xr).max(axis=0) / sc).max()
    e_orc = (np.abs(g["x0"] - xr).max(axis=0) / sc).max()
    e_pair = (np.abs(x0[rows] - g["x0"]).max(axis=0) / sc).max()
    _say("c2 unrefined errors vs refined oracle: device", e_dev, "oracle", e_orc,
         "device vs oracle", e_pair)
    eps = 1e-6
    assert e_dev <= KAPPA * 10 * eps
    assert e_orc <= KAPPA * 10 * eps
    assert e_pair <= 2 * KAPPA * 10 * eps


def test_c2_refined_vs_oracle(c2):
    torch, h, g, b, xyz, area = c2
    x, inf = _solve(torch, h, b, 1e-10)
    rows = g["rows"]
    eta_s = O.backward_error(xyz, area, x, b, anorm=float(g["anorm"]), rows=rows)
    bound = 4 * KAPPA * max(inf.eta_final, float(g["hist"][-1]), eta_s, 1e-12)
    rel = (np.abs(x[rows] - g["xr"]).max(axis=0) / g["xr_inf"]).max()
    _say("c2 refined: iters", inf.iters, "eta device", inf.eta_final, "eta exact sampled",
         eta_s, "oracle eta", g["hist"][-1], "|x - x_oracle|", rel, "bound", bound)
    assert inf.eta_final <= 1e-10 and eta_s <= 1e-10
    assert 1 <= inf.iters <= 3
    assert rel <= bound


def test_mixed_leaf64_vs_oracle(P):
    """n = 5120, leaf 64 (the headline leaf), eps 1e-5, mixed precision:
    factor accuracy against the exact matrix, unrefined and refined
    solutions against the oracle's."""
    import torch
    xyz, area = icosphere(4)
    n = xyz.shape[0]
    eps = 1e-5
    _say("mixed leaf 64 n", n)
    h = P.HLU(xyz, area, leaf=64, eta=2.0, eps=eps, cap=32, eps_mv=1e-12, cap_mv=64,
              precision=P.PREC_MIXED, refine_tol=1e-10, max_nrhs=8)
    h.set_executor(1)
    h.factor()
    st, inf = h.sync(check=False)
    assert st == 0
    Lg, Ug = h.export_factors()
    perm = h.perm()
    A = O.dense_matrix(xyz, area)
    Ap = A[np.ix_(perm, perm)]
    rel = np.linalg.norm(Ap - Lg @ Ug) / np.linalg.norm(Ap)
    del Ap, Lg, Ug
    b = rhs_normal(13, n, 8)
    x0, inf0 = _solve(torch, h, b, 0.0)
    xr, infr = _solve(torch, h, b, 1e-10)
    H = O.HMatrix(xyz, area, 64, 2.0, O.Rule(eps=eps, cap=32))
    O.factor(H)
    x0o = O.solve(H, b)
    xro, hist = O.refine(H, b, tol=1e-10)
    xd = np.linalg.solve(A, b)
    sc = np.abs(xd).max(axis=0)
    e_dev = (np.abs(x0 - xd).max(axis=0) / sc).max()
    e_orc = (np.abs(x0o - xd).max(axis=0) / sc).max()
    e_pair = (np.abs(x0 - x0o).max(axis=0) / sc).max()
    eta_d = O.backward_error(xyz, area, xr, b)
    bound = 4 * KAPPA * max(infr.eta_final, hist[-1], eta_d, 1e-12)
    e_ref = (np.abs(xr - xro).max(axis=0) / np.abs(xro).max(axis=0)).max()
    _say("mixed leaf 64: |A - LU|/|A|", rel, "unrefined dev", e_dev, "oracle", e_orc, "pair",
         e_pair, "refined iters", infr.iters, "eta", eta_d, "|x - x_oracle|", e_ref,
         "bound", bound)
    assert rel <= 11 * eps
    assert e_dev <= KAPPA * 10 * eps and e_orc <= KAPPA * 10 * eps
    assert e_pair <= 2 * KAPPA * 10 * eps
    assert eta_d <= 1e-10 and infr.eta_final <= 1e-10
    assert e_ref <= bound
