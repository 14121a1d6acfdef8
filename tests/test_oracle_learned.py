"""Pins of the learned smoother's oracle (oracle/learned.py)."""
import numpy as np
import pytest

from oracle import fem, learned as LN
from oracle.multigrid import Hierarchy, MGOptions

torch = pytest.importorskip("torch")


def _weights(seed, scale=0.3):
    rng = np.random.default_rng(seed)
    return scale * rng.standard_normal((LN.CH, 27)), scale * rng.standard_normal((LN.CH, 27))


def test_bf16_rounding_matches_torch_and_ties_to_even():
    x = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, -3.14159, 1e-3, 65504.0, 7.0e-39])
    assert LN.bf16(x)[1] == 1.0                 # halfway: down to the even mantissa
    assert LN.bf16(x)[2] == 1 + 2 ** -6         # halfway: up to the even mantissa
    r = np.random.default_rng(0).standard_normal(4000) * 10.0 ** np.random.default_rng(1).integers(-8, 8, 4000)
    for v in (x, r):
        ref = torch.from_numpy(v.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
        np.testing.assert_array_equal(LN.bf16(v), ref)


def test_forward_equals_direct_loops():
    W1, W2 = _weights(2)
    rho = np.random.default_rng(3).standard_normal((4, 4, 4))
    d, _, _ = LN.forward(rho, W1, W2)
    np.testing.assert_allclose(d, LN.forward_loops(rho, W1, W2), rtol=1e-12, atol=1e-12)


def test_forward_is_positively_homogeneous_and_zero_without_output_weights():
    W1, W2 = _weights(4)
    rho = np.random.default_rng(5).standard_normal((5, 5, 5))
    d = LN.forward(rho, W1, W2)[0]
    np.testing.assert_allclose(LN.forward(2.5 * rho, W1, W2)[0], 2.5 * d, rtol=1e-12)
    assert np.all(LN.forward(rho, W1, 0 * W2)[0] == 0)


def test_identity_channels_give_damped_jacobi_of_the_multigrid_oracle():
    """Channel 0 passes rho, channel 1 passes -rho: h0 - h1 = rho, so the step is
    x + omega D^{-1} (f - A x), the Jacobi sweep of oracle.multigrid."""
    n = 8
    A, _ = fem.assemble(3, n)
    hier = Hierarchy(3, A, 4, n)
    lv = hier.levels[-1]
    W1 = np.zeros((LN.CH, 27))
    W2 = np.zeros((LN.CH, 27))
    omega = 6.0 / 7.0
    W1[0, 13], W1[1, 13] = 1.0, -1.0
    W2[0, 13], W2[1, 13] = omega, -omega
    rng = np.random.default_rng(6)
    x, f = rng.standard_normal((2, A.shape[0]))
    got = LN.step_matrix(lv.A, lv.D, x, f, W1, W2, bf=False)
    np.testing.assert_allclose(got, Hierarchy.jacobi(lv, x, f, omega, 1), rtol=1e-12, atol=1e-12)
    # the constant-coefficient stencil of the module is the assembled stiffness
    h = 1.0 / n
    np.testing.assert_allclose(LN.laplace7(x.reshape(7, 7, 7), h).reshape(-1), lv.A @ x, rtol=1e-12, atol=1e-12)
    assert np.allclose(lv.D, 6 * h)


def test_gradient_matches_central_differences():
    W1, W2 = _weights(7, 0.5)
    R = np.random.default_rng(8).standard_normal((2, 5, 5, 5))
    w0 = 0.25
    L, g1, g2 = LN.loss_and_grad(R, w0, W1, W2)
    rng = np.random.default_rng(9)
    eps = 1e-6
    for which, W, G in ((1, W1, g1), (2, W2, g2)):
        for _ in range(6):
            c, t = rng.integers(0, LN.CH), rng.integers(0, 27)
            Wp, Wm = W.copy(), W.copy()
            Wp[c, t] += eps
            Wm[c, t] -= eps
            args_p = (Wp, W2) if which == 1 else (W1, Wp)
            args_m = (Wm, W2) if which == 1 else (W1, Wm)
            fd = (LN.loss_and_grad(R, w0, *args_p)[0] - LN.loss_and_grad(R, w0, *args_m)[0]) / (2 * eps)
            assert abs(fd - G[c, t]) <= 1e-6 * max(1.0, abs(fd)), (which, c, t, fd, G[c, t])


def test_learned_vcycle_reduces_to_jacobi_vcycle():
    """The multigrid oracle's learned smoother with Jacobi-equivalent weights
    reproduces its Jacobi V-cycle."""
    n = 8
    A, _ = fem.assemble(3, n)
    hier = Hierarchy(3, A, 2, n)
    omega = 6.0 / 7.0
    W1 = np.zeros((LN.CH, 27))
    W2 = np.zeros((LN.CH, 27))
    W1[0, 13], W1[1, 13] = 1.0, -1.0
    W2[0, 13], W2[1, 13] = omega, -omega
    rng = np.random.default_rng(10)
    x, f = rng.standard_normal((2, A.shape[0]))
    oj = MGOptions("jacobi", 1, 1, omega, 6.0, 1)
    ol = MGOptions("learned", 1, 1, omega, 6.0, 1, weights=(W1, W2), learned_bf16=False)
    L = len(hier.levels) - 1
    np.testing.assert_allclose(hier.vcycle(L, x, f, ol), hier.vcycle(L, x, f, oj), rtol=1e-11, atol=1e-12)


def test_adam_first_step_moves_by_the_learning_rate():
    W = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -7.0, 1e-3])
    W1, m, v = LN.adam_step(W, g, np.zeros(3), np.zeros(3), 1, lr=0.01)
    np.testing.assert_allclose(W1, W - 0.01 * np.sign(g), rtol=1e-6)
