"""Pins of the oracle's V-cycle (the "some multigrid steps" of Algorithm 1,
step 1) against closed-form smoother error propagation on exact eigenvectors,
symmetry, and contraction on the Laplacian."""
import numpy as np
import pytest
from numpy.polynomial import chebyshev as C

from oracle import fem
from oracle.multigrid import Hierarchy, MGOptions, gershgorin_rho
from workloads import lognormal_kappa


def _sine_mode(n, m, k):
    i = np.arange(1, n)
    s = np.outer(np.sin(k * np.pi * i / n), np.sin(m * np.pi * i / n))  # rows y, cols x
    return s.ravel()


def _setup(n_c, n_f, kappa=None):
    A, _ = fem.assemble(2, n_f, kappa=kappa)
    return Hierarchy(2, A, n_c, n_f)


def test_jacobi_closed_form_on_sine_modes():
    # For the 5-point Laplacian, D = 4 I and sin(m pi x) sin(k pi y) is an
    # eigenvector with D^{-1} A eigenvalue t = (4 - 2cos(m pi h) - 2cos(k pi h))/4.
    n = 16
    hier = _setup(4, n)
    lv = hier.levels[-1]
    for (m, k) in [(1, 1), (3, 7), (15, 15), (8, 2)]:
        s = _sine_mode(n, m, k)
        t = (4 - 2 * np.cos(m * np.pi / n) - 2 * np.cos(k * np.pi / n)) / 4
        x = hier.jacobi(lv, s, np.zeros_like(s), 0.8, 3)
        assert np.allclose(x, (1 - 0.8 * t) ** 3 * s, atol=1e-13)


def test_chebyshev_closed_form_on_sine_modes():
    # Error propagation of the Chebyshev semi-iteration of degree s on [a, b]:
    # p(t) = T_s((theta - t)/delta) / T_s(theta/delta).
    n = 16
    hier = _setup(4, n)
    lv = hier.levels[-1]
    assert gershgorin_rho(lv.A) == pytest.approx(2.0, abs=1e-14)
    b = lv.rho
    a = b / 4
    theta, delta = (a + b) / 2, (b - a) / 2
    for deg in (1, 2, 4, 5):
        Ts = np.zeros(deg + 1); Ts[deg] = 1
        for (m, k) in [(1, 2), (5, 9), (15, 14), (12, 3)]:
            s = _sine_mode(n, m, k)
            t = (4 - 2 * np.cos(m * np.pi / n) - 2 * np.cos(k * np.pi / n)) / 4
            p = C.chebval((theta - t) / delta, Ts) / C.chebval(theta / delta, Ts)
            x = hier.chebyshev(lv, s, np.zeros_like(s), 4.0, deg)
            assert np.allclose(x, p * s, atol=1e-12)


@pytest.mark.parametrize("smoother,nu", [("jacobi", 2), ("cheb", 4)])
def test_vcycle_is_symmetric_and_contracts(smoother, nu):
    kap = lognormal_kappa(2, 32, seed=2)
    hier = _setup(4, 32, kappa=kap)
    A = hier.levels[-1].A
    opts = MGOptions(smoother, nu, nu, 0.8, 4.0, 1)
    rng = np.random.default_rng(0)
    f, g = rng.standard_normal(A.shape[0]), rng.standard_normal(A.shape[0])
    L = len(hier.levels) - 1
    Bf = hier.vcycle(L, np.zeros_like(f), f, opts)
    Bg = hier.vcycle(L, np.zeros_like(g), g, opts)
    assert g @ Bf == pytest.approx(f @ Bg, rel=1e-11)
    # energy-norm contraction of the error over 5 cycles
    xs = rng.standard_normal(A.shape[0])
    rhs = A @ xs
    x = np.zeros_like(rhs)
    e0 = np.sqrt((xs - x) @ A @ (xs - x))
    for _ in range(5):
        x = hier.vcycle(L, x, rhs, opts)
    e5 = np.sqrt((xs - x) @ A @ (xs - x))
    assert (e5 / e0) ** (1 / 5) < 0.35
    for _ in range(40):
        x = hier.vcycle(L, x, rhs, opts)
    assert np.max(np.abs(x - xs)) < 1e-10 * np.max(np.abs(xs))


def test_hierarchy_coarse_operators_are_rediscretisations():
    hier = _setup(4, 32)
    for lv in hier.levels:
        A_direct, _ = fem.assemble(2, lv.n)
        assert abs(lv.A - A_direct).max() < 1e-13
