"""Why some coarse spaces cannot serve the wanted eigenpairs (oracle, exact BVP
solves, reduced fine meshes).

Theorem 3.1 and Remark 3.1: the correction step contracts only when V_H is
fine enough for the eigenvalue sought (eta(V_H) small against lambda and the
spectral gap).  These tests reproduce, with the oracle and exact boundary
value solves (no multigrid, no GPU), the three cases where a configured coarse
space is too coarse, at fine meshes small enough for the CPU:

* 2D Laplacian, 20 eigenpairs, H = 1/16: several exact discrete eigenpairs are
  repelling fixed points (a 1e-4 perturbation grows by orders of magnitude per
  step) and a third of the processes from the coarse start never converge;
  with H = 1/32 the same eigenpairs attract and every process converges.
* rough coefficient (log kappa ~ N(0, 1) i.i.d. per fine element): the
  Galerkin coarse Ritz values sit 25-45 % above the discrete eigenvalues and
  only the lowest process converges, at H = 1/16 and H = 1/32 alike.
* 3D cube, 40 eigenpairs, H = 1/8: the cube's multiple eigenvalues; most
  processes settle nowhere or on another member of their cluster.
"""
import numpy as np
import pytest

import workloads as W
from oracle import pasm as O

pytestmark = pytest.mark.slow


def _errors_vs_own(r, w):
    """Per process: relative error of the final eigenvalue against the
    discrete eigenvalue of its own start index, and the smallest error over
    its history."""
    idx = r["index"]
    fin = np.abs(r["lam"] - w[idx]) / w[idx]
    best = np.array([np.min(np.abs(np.array(h) - w[i]) / w[i]) for h, i in zip(r["hist"], idx)])
    return fin, best


def _perturbed_step_errors(prob, w, V, j, bvp, steps, eps=1e-4, seed=0):
    rng = np.random.default_rng(seed + j)
    d = rng.standard_normal(V.shape[0])
    d -= V[:, j] * (V[:, j] @ (prob.M @ d))
    d /= np.sqrt(d @ (prob.M @ d))
    u = V[:, j] + eps * d
    u /= np.sqrt(u @ (prob.M @ u))
    lam = float(u @ (prob.A @ u))
    errs = []
    for _ in range(steps):
        out = O.correction_step(prob, lam, u, bvp)
        lam, u = out["lam"], out["u"]
        errs.append(abs(lam - w[j]) / w[j])
    return np.array(errs)


def test_laplace_20_pairs_need_a_finer_coarse_space_than_H16():
    n = 128
    w_all = {}
    for nc in (16, 32):
        prob = O.make_problem(2, nc, n)
        w, V = O.discrete_eigenpairs(prob.A, prob.M, 20)
        w_all[nc] = (prob, w, V, O.ExactBVP(prob.A))
    # from the coarse start (Algorithm 2, h_1 = H)
    prob, w, V, bvp = w_all[16]
    r = O.solve(prob, 20, bvp, tol=0.0, max_iter=30, workers=8)
    fin, best = _errors_vs_own(r, w)
    assert np.sum(fin <= 1e-8) <= 14
    assert np.sum(fin > 1e-3) >= 4
    prob32, w32, V32, bvp32 = w_all[32]
    r = O.solve(prob32, 20, bvp32, tol=0.0, max_iter=10, workers=8)
    _, best32 = _errors_vs_own(r, w32)
    assert np.all(best32 <= 1e-8)
    # the exact eigenpairs themselves: repelling at H = 1/16, attracting at 1/32
    for j in (10, 17, 18, 19):
        e16 = _perturbed_step_errors(prob, w, V, j, bvp, 6)
        assert e16[-1] > 1e3 * e16[1], (j, e16)
        e32 = _perturbed_step_errors(prob32, w32, V32, j, bvp32, 6)
        assert e32[-1] < 1e-12, (j, e32)


def test_rough_coefficient_defeats_the_coarse_space():
    n = 128
    kap = W.lognormal_kappa(2, n, seed=0, sigma=1.0)
    for nc, k, its in ((16, 20, 20), (32, 10, 15)):
        prob = O.make_problem(2, nc, n, kappa=kap)
        w, _ = O.discrete_eigenpairs(prob.A, prob.M, k)
        r = O.solve(prob, k, O.ExactBVP(prob.A), tol=0.0, max_iter=its, workers=8)
        start_gap = r["lam0"] / w - 1.0
        assert np.all(start_gap > 0.25), (nc, start_gap)
        fin, best = _errors_vs_own(r, w)
        assert np.sum(best <= 1e-8) <= 2, (nc, best)
        assert best[0] <= 1e-8  # the lowest one still converges


def test_cube_clusters_with_100_pairs_scale_coarse_space():
    # 40 eigenpairs of the cube at H = 1/8, h = 1/16 (the configured 100 at
    # h = 1/128 behave alike; this size runs in seconds)
    prob = O.make_problem(3, 8, 16)
    w, _ = O.discrete_eigenpairs(prob.A, prob.M, 48)
    r = O.solve(prob, 40, O.ExactBVP(prob.A), tol=0.0, max_iter=25, workers=8)
    # any member of a cluster is a correct answer for any process of it
    anyv = np.array([np.min(np.abs(l - w) / w) for l in r["lam"]])
    assert np.sum(anyv <= 1e-8) <= 14
    # the failures sit in multiple eigenvalues (relative gap < 1e-6)
    mult = np.array([np.sum(np.abs(w - wi) <= 1e-6 * wi) for wi in w[:40]])
    bad = np.flatnonzero(anyv > 1e-8)
    assert np.mean(mult[bad] >= 2) > 0.6
