"""Pins of the oracle's Algorithms 1 and 2 against the definition (dense
generalized eigensolve of the full pencil), brute-force Rayleigh-Ritz on the
fine mesh, exact fixed points, Theorem 3.1's mesh-independent rate and
Remark 3.2's orthogonality bound."""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import pasm
from oracle.multigrid import default_options
from workloads import lognormal_kappa


@pytest.fixture(scope="module")
def small2d():
    return pasm.make_problem(2, 8, 64)


def _align(u, v, M):
    return u if float(u @ (M @ v)) >= 0 else -u


def test_converges_to_dense_discrete_eigenpairs(small2d):
    prob = small2d
    w, V = pasm.discrete_eigenpairs(prob.A, prob.M, 4)
    for bvp in (pasm.ExactBVP(prob.A),
                pasm.MultigridBVP(prob, default_options(2, "jacobi", 2, 2, 2))):
        r = pasm.solve(prob, 4, bvp, tol=1e-13)
        assert np.max(np.abs(r["lam"] - w) / w) < 1e-11
        for i in range(4):
            u = _align(r["U"][i], V[:, i], prob.M)
            d = u - V[:, i]
            assert np.sqrt(d @ prob.M @ d) < 1e-5
            assert r["U"][i] @ prob.M @ r["U"][i] == pytest.approx(1.0, rel=1e-12)
    # the selected Ritz index differs from i for the third eigenpair
    assert r["picks"][2][0] == 1


def test_exact_eigenpair_is_a_fixed_point(small2d):
    prob = small2d
    w, V = pasm.discrete_eigenpairs(prob.A, prob.M, 4)
    mg = pasm.MultigridBVP(prob, default_options(2, "cheb", 4, 4, 2))
    for i in range(4):
        out = pasm.correction_step(prob, w[i], V[:, i], mg)
        assert out["lam"] == pytest.approx(w[i], rel=1e-12)
        u = _align(out["u"], V[:, i], prob.M)
        assert np.max(np.abs(u - V[:, i])) < 1e-9 * np.max(np.abs(V[:, i]))


def test_augmented_pencil_equals_bruteforce_rayleigh_ritz(small2d):
    prob = small2d
    lam0, U0, _, _ = pasm.coarse_start(prob, 4)
    bvp = pasm.MultigridBVP(prob, default_options(2, "jacobi", 2, 2, 1))
    i = 2
    out = pasm.correction_step(prob, lam0[i], U0[i], bvp)
    ut = out["ut"]
    Vb = np.hstack([prob.P.toarray(), ut[:, None]])     # fine basis of V_H + span{u~}
    Ar = Vb.T @ (prob.A @ Vb)
    Mr = Vb.T @ (prob.M @ Vb)
    mu_bf, Z_bf = sla.eigh(Ar, Mr)
    Ahat, Mhat = pasm.augmented_pencil(prob.AH, prob.MH, out["b"], out["c"], out["beta"], out["zeta"])
    mu = sla.eigh(Ahat, Mhat, eigvals_only=True)
    assert np.max(np.abs(mu - mu_bf) / np.abs(mu_bf)) < 1e-9
    # brute-force selection: component along u~ measured on the fine mesh
    scores = [abs(float((Vb @ Z_bf[:, j]) @ (prob.M @ ut))) for j in range(len(mu_bf))]
    j = int(np.argmax(scores))
    assert out["lam"] == pytest.approx(mu_bf[j], rel=1e-9)
    unew = Vb @ Z_bf[:, j]
    unew = _align(unew, out["u"], prob.M)
    assert np.max(np.abs(unew - out["u"])) < 1e-7


def test_rate_depends_on_H_not_h():
    # Theorem 3.1 / Remark 3.1: the contraction factor gamma is bounded
    # independently of the fine mesh.  Measured on the slowest of the first four
    # eigenpairs, from per-iteration eigenvalue error ratios above rounding.
    rates = []
    for nf in (32, 64):
        prob = pasm.make_problem(2, 8, nf)
        w, _ = pasm.discrete_eigenpairs(prob.A, prob.M, 4)
        r = pasm.solve(prob, 4, pasm.ExactBVP(prob.A), tol=1e-14, which=[3])
        err = np.abs(np.array(r["hist"][0]) - w[3]) / w[3]
        ratios = [err[t + 1] / err[t] for t in range(1, len(err) - 1) if err[t + 1] > 1e-11]
        rates.append(float(np.median(ratios)))
    assert rates[0] < 0.3 and rates[1] < 0.3
    assert 0.8 < rates[0] / rates[1] < 1.25


def test_orthogonality_bound_remark_3_2(small2d):
    prob = small2d
    w, V = pasm.discrete_eigenpairs(prob.A, prob.M, 4)
    r = pasm.solve(prob, 4, pasm.ExactBVP(prob.A), tol=1e-6)
    res = []
    for i in range(4):
        u = _align(r["U"][i], V[:, i], prob.M)
        d = u - V[:, i]
        res.append(np.sqrt(d @ prob.M @ d))
    G = r["U"] @ (prob.M @ r["U"].T)
    for i in range(4):
        for j in range(i + 1, 4):
            assert abs(G[i, j]) <= res[i] + res[j] + res[i] * res[j] + 1e-15


def test_fine_equal_coarse_skips_augmentation():
    prob = pasm.make_problem(2, 8, 8)
    theta = sla.eigh(prob.AH, prob.MH, eigvals_only=True)
    r = pasm.solve(prob, 3, pasm.ExactBVP(prob.A), tol=1e-13, max_iter=3)
    assert np.allclose(r["lam"], theta[:3], rtol=1e-13)


def test_variable_kappa_and_potential_fixed_point_and_convergence():
    # With a coefficient and a potential the exact discrete eigenpairs are still
    # fixed points of Algorithm 1, and the lowest one is reached from the coarse
    # start.  (Higher ones need a finer V_H when the coefficient splits the
    # near-degenerate pairs; Remark 3.1.)
    kap = lognormal_kappa(2, 32, seed=4, sigma=0.5)
    prob = pasm.make_problem(2, 8, 32, kappa=kap, centre=[0.3, 0.7])
    w, V = pasm.discrete_eigenpairs(prob.A, prob.M, 4)
    mg = pasm.MultigridBVP(prob, default_options(2, "cheb", 4, 4, 2))
    for i in range(4):
        out = pasm.correction_step(prob, w[i], V[:, i], mg)
        assert out["lam"] == pytest.approx(w[i], rel=1e-11)
    r = pasm.solve(prob, 1, mg, tol=1e-13)
    assert abs(r["lam"][0] - w[0]) / w[0] < 1e-11


def test_3d_with_degenerate_pairs():
    prob = pasm.make_problem(3, 4, 8)
    w, V = pasm.discrete_eigenpairs(prob.A, prob.M, 4)
    # the Kuhn mesh keeps an exact double eigenvalue (axis permutations)
    assert abs(w[1] - w[2]) < 1e-10 * w[1]
    r = pasm.solve(prob, 4, pasm.MultigridBVP(prob, default_options(3, "jacobi", 2, 2, 2)), tol=1e-13)
    lam = np.sort(r["lam"])
    assert np.max(np.abs(lam - w) / w) < 1e-10
    # cluster subspace check for the double eigenvalue
    idx = [i for i in range(4) if abs(r["lam"][i] - w[1]) < 1e-8 * w[1]]
    assert len(idx) == 2
    Ug = r["U"][idx].T
    Qa, _ = np.linalg.qr(V[:, 1:3])
    Qb, _ = np.linalg.qr(Ug)
    s = np.linalg.svd(Qa.T @ Qb, compute_uv=False)
    assert np.min(s) > 1 - 1e-8


def test_paper_multigrid_step_reaches_the_same_fixed_points(small2d):
    # the paper's boundary value solver (one V-cycle with 2 CG pre- and
    # post-smoothing steps, Section 5) changes the speed only: the same
    # discrete eigenpairs
    from oracle.multigrid import MGOptions
    prob = small2d
    w, _ = pasm.discrete_eigenpairs(prob.A, prob.M, 4)
    r = pasm.solve(prob, 4, pasm.MultigridBVP(prob, MGOptions("cg", 2, 2, vcycles=1)), tol=1e-13)
    assert np.max(np.abs(r["lam"] - w) / w) < 1e-11


def test_example2_operator_solve_reaches_discrete_eigenpairs():
    # the second example of Section 5 (full tensor and potential, 3D) at a
    # small size: Algorithm 2 with the paper's multigrid step reaches the
    # discrete eigenpairs of its pencil
    from oracle import fem
    from oracle.multigrid import MGOptions
    prob = pasm.make_problem(3, 4, 16, tensor=fem.example2_tensor, potential=fem.example2_potential)
    w, _ = pasm.discrete_eigenpairs(prob.A, prob.M, 1)
    r = pasm.solve(prob, 1, pasm.MultigridBVP(prob, MGOptions("cg", 2, 2, vcycles=1)), tol=1e-13)
    assert abs(r["lam"][0] - w[0]) / w[0] < 1e-11
