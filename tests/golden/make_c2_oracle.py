"""Writes c2_oracle.npz: the oracle's solutions of the n = 20480 workload
(level-5 icosphere, weighted d=3 Laplace collocation, leaf 64, eta 2,
eps 1e-6 with rank capacity 32, FP64, 8 right-hand sides ~ N(0,1) seed 1),
stored on a fixed sample of rows.

Only the oracle and the shared input generators run here.  Stored:
  rows       sampled row indices (original point order)
  x0         unrefined solution x0 = solve(b) on those rows (n_rows x 8)
  xr         solution refined with the exact operator to eta <= 1e-10
  x0_inf, xr_inf   per-column max |x| over all rows
  hist       backward-error history of the refinement
  anorm      exact ||A||_inf
  factor_s   oracle factor time (host, informational)

Run:  python tests/golden/make_c2_oracle.py   (about 3 minutes, one core)
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402
from hlu_inputs import config_inputs, rhs_normal  # noqa: E402


def main():
    xyz, area, cfg = config_inputs("c2")
    n = xyz.shape[0]
    b = rhs_normal(cfg["seed"], n, cfg["nrhs"])
    t = time.perf_counter()
    H = O.HMatrix(xyz, area, cfg["leaf"], cfg["eta"], O.Rule(eps=cfg["eps"], cap=cfg["cap"]))
    print(f"assembled n={n} in {time.perf_counter() - t:.1f} s: {H.stats()}", flush=True)
    t = time.perf_counter()
    info = O.factor(H)
    factor_s = time.perf_counter() - t
    assert info == 0
    print(f"factored in {factor_s:.1f} s", flush=True)
    anorm = O.exact_inf_norm(xyz, area)
    x0 = O.solve(H, b)
    xr, hist = O.refine(H, b, tol=1e-10, anorm=anorm)
    print("refinement history", hist, flush=True)
    rows = np.sort(np.random.default_rng(41).choice(n, 256, replace=False))
    np.savez(os.path.join(HERE, "c2_oracle.npz"), rows=rows, x0=x0[rows], xr=xr[rows],
             x0_inf=np.abs(x0).max(axis=0), xr_inf=np.abs(xr).max(axis=0),
             hist=np.array(hist), anorm=np.array(anorm), factor_s=np.array(factor_s))


if __name__ == "__main__":
    main()
