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


def _krylov_minimiser(A, x0, f, k):
    """Brute force: the x in x0 + span{r0, A r0, ..., A^{k-1} r0} of least
    A-norm error, from the normal equations of an orthonormal basis."""
    r0 = f - A @ x0
    K = np.empty((len(f), k))
    v = r0.copy()
    for j in range(k):
        K[:, j] = v
        v = A @ v
    Q, _ = np.linalg.qr(K)
    # min_y (x0 + Q y - x*)^T A (x0 + Q y - x*)  =>  (Q^T A Q) y = Q^T r0
    y = np.linalg.solve(Q.T @ (A @ Q), Q.T @ r0)
    return x0 + Q @ y


def test_cg_smoother_is_the_krylov_minimiser_and_terminates():
    # the paper's smoother (Section 5: CG steps for pre- and post-smoothing):
    # k steps of CG from x0 give the A-norm-optimal point of the k-th Krylov
    # space; on n unknowns with n distinct eigenvalues it is exact after n
    hier = _setup(4, 16)
    lv = hier.levels[-1]
    A = lv.A.toarray()
    rng = np.random.default_rng(3)
    f = rng.standard_normal(A.shape[0])
    x0 = rng.standard_normal(A.shape[0])
    for k in (1, 2, 3):
        x = hier.cg(lv, x0, f, k)
        xb = _krylov_minimiser(A, x0, f, k)
        assert np.max(np.abs(x - xb)) < 1e-10 * np.max(np.abs(xb))
    # finite termination on a small system: 3 x 3 interior nodes of the 4-cell
    # mesh has 9 unknowns with 6 distinct eigenvalues
    small = _setup(2, 4)
    lv4 = small.levels[-1]
    A4 = lv4.A.toarray()
    f4 = rng.standard_normal(A4.shape[0])
    x = small.cg(lv4, np.zeros_like(f4), f4, 9)
    assert np.max(np.abs(A4 @ x - f4)) < 1e-12
    # an exact solution already: the zero denominator leaves x unchanged
    xs = np.linalg.solve(A4, f4)
    assert np.array_equal(small.cg(lv4, xs.copy(), A4 @ xs, 2), xs) or \
        np.max(np.abs(small.cg(lv4, xs.copy(), A4 @ xs, 2) - xs)) < 1e-14


def test_cg_smoothed_vcycle_contracts():
    # one V-cycle with 2 CG pre- and post-smoothing steps (the paper's
    # multigrid step) reduces the A-norm error of the Laplacian by about 0.14
    # per cycle (damped Jacobi 2/2: 0.25); with a rough kappa the plain
    # (unpreconditioned) CG smoother is weaker but still contracts (about 0.63
    # against Jacobi's 0.5)
    for kap, bound in ((None, 0.2), (lognormal_kappa(2, 64, seed=2, sigma=1.0), 0.7)):
        hier = _setup(8, 64, kappa=kap)
        opts = MGOptions("cg", 2, 2, vcycles=1)
        A = hier.levels[-1].A
        rng = np.random.default_rng(5)
        xs = rng.standard_normal(A.shape[0])
        f = A @ xs
        x = np.zeros_like(f)
        errs = []
        for _ in range(4):
            x = hier.vcycle(len(hier.levels) - 1, x, f, opts)
            errs.append(np.sqrt((x - xs) @ (A @ (x - xs))))
        e0 = np.sqrt(xs @ (A @ xs))
        rates = [errs[0] / e0] + [errs[i + 1] / errs[i] for i in range(3)]
        assert max(rates) < bound, rates
