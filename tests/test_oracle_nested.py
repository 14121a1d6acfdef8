"""Pins of the oracle's nested schedule (Algorithm 2, step 2(A)).

* The intermediate problems are the restrictions of the forms to the nested
  spaces: for constant coefficients they equal the direct assembly on that
  mesh (Galerkin = rediscretisation for P1 on nested Kuhn meshes).
* The correction step's fixed points on a level are that level's discrete
  eigenpairs, so many steps per level end step 2(A) on the discrete
  eigenpairs of h_{n-1}.
* The nested start is much closer to the finest discrete eigenpairs than the
  coarse start (its error is the O(h^2) gap between consecutive meshes), and
  step 2(B) then converges to them.
"""
import numpy as np
import pytest

from oracle import fem
from oracle import pasm as O
from oracle.multigrid import default_options


def test_level_problem_is_the_direct_assembly_on_that_mesh():
    prob = O.make_problem(2, 4, 32)
    for n in (8, 16):
        lp = O.level_problem(prob, n)
        A, M = fem.assemble(2, n)
        assert abs(lp.A - A).max() < 1e-13
        assert abs(lp.M - M).max() < 1e-17
        assert np.max(np.abs(lp.AH - prob.AH)) < 1e-13
        # the level's own prolongation from V_H composes with the rest to P
        Pk = O.prolongation(2, n, 32)
        assert abs(Pk @ lp.P - prob.P).max() < 1e-15
    prob3 = O.make_problem(3, 2, 8)
    lp = O.level_problem(prob3, 4)
    A, M = fem.assemble(3, 4)
    assert abs(lp.A - A).max() < 1e-13 and abs(lp.M - M).max() < 1e-17


def test_many_steps_per_level_end_on_the_discrete_eigenpairs_of_2h():
    prob = O.make_problem(2, 8, 64)
    k = 4
    r = O.solve_nested(prob, k, lambda lp: O.ExactBVP(lp.A), varpi=25)
    lp = O.level_problem(prob, 32)
    w2h, _ = O.discrete_eigenpairs(lp.A, lp.M, k)
    assert np.max(np.abs(r["lam_start"] - w2h) / w2h) < 1e-11
    # the start is M_h-normalised on the finest mesh (the nested mass matrices
    # are restrictions of each other)
    for i in range(k):
        assert r["U_start"][i] @ (prob.M @ r["U_start"][i]) == pytest.approx(1.0, rel=1e-12)


def test_nested_start_is_close_and_step_2b_converges():
    prob = O.make_problem(2, 8, 128)
    k = 4
    w, _ = O.discrete_eigenpairs(prob.A, prob.M, k)
    theta, _, _, _ = O.coarse_start(prob, k)
    mg = lambda lp: O.MultigridBVP(lp, default_options(2, "cheb", 4, 4, 2))  # noqa: E731
    r = O.solve_nested(prob, k, mg, varpi=1, varpi_n=8)
    e_coarse = np.abs(theta - w) / w
    e_start = np.abs(r["lam_start"] - w) / w
    assert np.all(e_start < 0.05 * e_coarse), (e_start, e_coarse)
    assert np.max(np.abs(r["lam"] - w) / w) < 1e-11
    # against the plain schedule (Algorithm 2 without step 2(A)): the same
    # fixed points
    plain = O.solve(prob, k, mg(prob), tol=1e-13)
    assert np.max(np.abs(plain["lam"] - r["lam"]) / w) < 1e-11


def test_two_levels_have_no_intermediate_step():
    prob = O.make_problem(2, 8, 16)
    r = O.solve_nested(prob, 3, lambda lp: O.ExactBVP(lp.A), varpi=2)
    theta, U0, _, _ = O.coarse_start(prob, 3)
    assert np.array_equal(r["lam_start"], theta)
    assert np.max(np.abs(r["U_start"] - U0)) < 1e-15
