"""Pins of the oracle's d = 1 and d = 2 Laplace kernels (Sec. 6.1:
-log|x-y| and -log|x-y| / (2 pi)), independent of its own formulas:

* the self term equals the kernel integrated over the panel by adaptive
  quadrature (scipy.integrate.quad);
* d = 1 on [0, 1]: A 1 - 1 converges to the continuous operator applied to
  1, (V1)(x) = 1 - x log x - (1 - x) log(1 - x), at first order in h;
* d = 2 on the circle of radius rho: the Fourier modes are eigenfunctions,
  V cos(k t) = rho / (2k) cos(k t) (k >= 1) and V 1 = -rho log(rho);
* the oracle's H-LU on both kernels: factor accuracy against the dense
  matrix and refinement to 1e-10 against the exact operator;
* planted mistakes (a dropped 1/(2 pi), a flipped sign, a self term without
  the exact panel integral) fail these criteria.
"""
import math

import numpy as np
import pytest
from scipy import integrate

import oracle as O
from hlu_inputs import circle, rhs_normal, segment


def _self_quad(h, scale):
    f = lambda t: -math.log(abs(t)) * scale  # noqa: E731
    a, _ = integrate.quad(f, -h / 2, 0.0)
    b, _ = integrate.quad(f, 0.0, h / 2)
    return a + b + 1.0


@pytest.mark.parametrize("reading,scale", [(O.READING_LOG1D, 1.0),
                                           (O.READING_LOG2D, 1.0 / (2 * math.pi))])
def test_self_term_is_the_panel_integral(reading, scale):
    for h in (1e-3, 0.05, 0.7):
        xyz = np.zeros((2, 3))
        xyz[1, 0] = 5.0
        A = O.kernel_entries(xyz, np.array([h, h]), np.arange(2), np.arange(2), reading)
        assert abs(A[0, 0] - _self_quad(h, scale)) <= 1e-12 * abs(A[0, 0])


def _v1_error(n, entries=None):
    xyz, h = segment(n)
    A = (entries or O.dense_matrix)(xyz, h, O.READING_LOG1D)
    x = xyz[:, 0]
    v1 = 1.0 - x * np.log(x) - (1.0 - x) * np.log(1.0 - x)
    return float(np.abs(A.sum(axis=1) - 1.0 - v1).max())


def _mode_error(n, k, entries=None, rho=0.5):
    xyz, h = circle(n, rho)
    A = (entries or O.dense_matrix)(xyz, h, O.READING_LOG2D)
    t = np.arctan2(xyz[:, 1], xyz[:, 0])
    u = np.cos(k * t)
    lam = 1.0 + (rho / (2 * k) if k else -rho * math.log(rho))
    return float(np.abs(A @ u - lam * u).max())


def test_log1d_converges_to_the_continuous_operator():
    e = [_v1_error(n) for n in (256, 1024)]
    assert e[0] <= 0.2 / 256 and e[1] <= 0.2 / 1024
    assert e[0] / e[1] >= 3.0


@pytest.mark.parametrize("k", [0, 1, 3])
def test_log2d_circle_modes(k):
    e = [_mode_error(n, k) for n in (256, 1024)]
    assert e[0] <= 0.2 / 256 and e[1] <= 0.2 / 1024
    assert e[0] / e[1] >= 3.0


def _mutant(kind):
    base = O.kernel_entries

    def entries(xyz, area, rows, cols, reading):
        A = base(xyz, area, rows, cols, reading)
        rows, cols = np.asarray(rows), np.asarray(cols)
        same = rows[:, None] == cols[None, :]
        if kind == "no_2pi" and reading == O.READING_LOG2D:
            A = np.where(same, A, A * 2 * math.pi)
        elif kind == "sign":
            A = np.where(same, A, -A)
        elif kind == "self":
            h = area[rows]
            scale = 1.0 if reading == O.READING_LOG1D else 1 / (2 * math.pi)
            A = np.where(same, (-h * np.log(h) * scale + 1.0)[:, None], A)
        return A

    def dense(xyz, area, reading):
        idx = np.arange(xyz.shape[0])
        return entries(xyz, area, idx, idx, reading)
    return dense


@pytest.mark.parametrize("kind", ["no_2pi", "sign", "self"])
def test_planted_kernel_mistakes_are_caught(kind):
    bad = _mutant(kind)
    caught_1d = _v1_error(256, bad) > 0.2 / 256
    caught_2d = any(_mode_error(256, k, bad) > 0.2 / 256 for k in (0, 1, 3))
    assert caught_2d if kind == "no_2pi" else (caught_1d and caught_2d)


@pytest.mark.parametrize("reading,geo", [(O.READING_LOG1D, segment), (O.READING_LOG2D, circle)])
def test_oracle_hlu_on_log_kernels(reading, geo):
    xyz, h = geo(1024)
    eps = 1e-6
    H = O.HMatrix(xyz, h, 32, 2.0, O.Rule(eps=eps, cap=32), reading=reading)
    st = H.stats()
    assert st["lowrank"] > 0 and st["dense"] > 0
    A_H = H.to_dense()
    A = O.dense_matrix(xyz, h, reading)[np.ix_(H.perm, H.perm)]
    assert np.linalg.norm(A - A_H) / np.linalg.norm(A) <= eps
    assert O.factor(H) == 0
    Lh, U = O.factors_dense(H)
    assert np.linalg.norm(A_H - Lh @ U) / np.linalg.norm(A_H) <= 10 * eps
    b = rhs_normal(5, xyz.shape[0], 2)
    x, hist = O.refine(H, b, tol=1e-10)
    assert hist[-1] <= 1e-10
    assert O.backward_error(xyz, h, x, b, reading) <= 1e-10
