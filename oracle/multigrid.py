"""Geometric multigrid V-cycle for the boundary value problem of Algorithm 1 (oracle).

TEST INFRASTRUCTURE ONLY (see the package header).

Algorithm 1, step 1 solves a(u_hat, v) = lambda b(u, v) "by some multigrid
steps".  The paper fixes neither the smoother nor the cycle; the reading used
throughout this project (and by the GPU library, implemented independently) is:

  * levels: the nested meshes between H and h (ratio 2), coarse operators by the
    Galerkin rule A_{l-1} = P_l^T A_l P_l, the coarsest level (= V_H) solved
    exactly;
  * one V-cycle V(l, x, f):
        x <- S_pre(x, f)                       (pre-smoothing)
        r_c <- P_l^T (f - A_l x)               (residual, restriction)
        e_c <- V(l-1, 0, r_c)                  (coarse correction; exact on V_H)
        x <- x + P_l e_c                       (prolongation)
        x <- S_post(x, f)                      (post-smoothing)
  * the boundary value problem starts from x = u (the current eigenvector
    approximation, as in the contraction assumption of Theorem 3.1) and runs a
    fixed number of V-cycles;
  * smoothers, with D = diag(A_l):
        damped Jacobi, nu sweeps:   x <- x + omega D^{-1} (f - A x)
        learned (3D): nu steps of the convolutional corrector of
        oracle.learned, x <- x + N(D^{-1} (f - A x))
        Chebyshev of degree s on D^{-1} A over [rho/alpha, rho], rho the
        Gershgorin bound max_i sum_j |a_ij| / a_ii.  Written here in the
        two-vector (direction, residual) form of the Chebyshev semi-iteration.
        conjugate gradients (the smoother of the paper's experiments, Section
        5: one multigrid step with 2 CG steps for pre- and post-smoothing):
        nu steps of plain CG on A x = f from the current x.

Parity status: pinned.  The smoothers are checked against the closed-form
error propagation of Jacobi ((1 - omega t)^nu) and of Chebyshev (the scaled
Chebyshev polynomial) on exact eigenvectors of D^{-1} A, CG against the
A-norm minimiser over the Krylov space computed by brute force and its
finite termination, and the V-cycle against its contraction on the Laplacian
(tests/test_oracle_multigrid.py).
"""
from __future__ import annotations

import dataclasses
from typing import List

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .transfer import galerkin, level_sizes, prolongation


@dataclasses.dataclass
class Level:
    n: int
    A: sp.csr_matrix
    D: np.ndarray
    rho: float
    P: sp.csr_matrix = None      # prolongation from the next coarser level to this one


@dataclasses.dataclass
class MGOptions:
    smoother: str = "jacobi"     # "jacobi" | "cheb" | "learned" | "cg"
    nu_pre: int = 2
    nu_post: int = 2
    omega: float = 0.8
    cheb_alpha: float = 4.0
    vcycles: int = 2
    weights: tuple = None        # (W1, W2) of the learned smoother (oracle.learned)
    learned_bf16: bool = True    # round the learned smoother's operands as the GPU does


def default_options(dim: int, smoother: str, nu_pre: int, nu_post: int, vcycles: int) -> MGOptions:
    """Jacobi weight 4/5 (2D) or 6/7 (3D); Chebyshev interval [rho/4, rho]
    (2D) or [rho/6, rho] (3D)."""
    omega = 4.0 / 5.0 if dim == 2 else 6.0 / 7.0
    alpha = 4.0 if dim == 2 else 6.0
    return MGOptions(smoother, nu_pre, nu_post, omega, alpha, vcycles)


def gershgorin_rho(A: sp.csr_matrix) -> float:
    D = A.diagonal()
    rowsum = np.asarray(abs(A).sum(axis=1)).ravel()
    return float(np.max(rowsum / D))


class Hierarchy:
    """Galerkin multigrid hierarchy from V_H (level 0) to V_h (last level)."""

    def __init__(self, dim: int, A_fine: sp.csr_matrix, n_coarse: int, n_fine: int):
        sizes = level_sizes(n_coarse, n_fine)
        self.dim = dim
        levels: List[Level] = [None] * len(sizes)
        A = A_fine.tocsr()
        for l in range(len(sizes) - 1, -1, -1):
            levels[l] = Level(sizes[l], A, A.diagonal().copy(), gershgorin_rho(A))
            if l > 0:
                P = prolongation(dim, sizes[l - 1], sizes[l])
                levels[l].P = P
                A = galerkin(P, A)
        self.levels = levels
        A0 = levels[0].A.toarray()
        self.coarse_chol = sla.cho_factor(A0, lower=True)

    # -- smoothers -------------------------------------------------------
    @staticmethod
    def jacobi(lv: Level, x: np.ndarray, f: np.ndarray, omega: float, nu: int) -> np.ndarray:
        for _ in range(nu):
            x = x + omega * (f - lv.A @ x) / lv.D
        return x

    @staticmethod
    def chebyshev(lv: Level, x: np.ndarray, f: np.ndarray, alpha: float, degree: int) -> np.ndarray:
        """Chebyshev semi-iteration on D^{-1} A x = D^{-1} f over [rho/alpha, rho].

        theta = centre, delta = half width, sigma = theta/delta;
        r0 = D^{-1}(f - A x0), d0 = r0/theta, then for each further step
        rho_{j+1} = 1/(2 sigma - rho_j),
        d_{j+1} = rho_{j+1} rho_j d_j + (2 rho_{j+1}/delta) r_{j+1}.
        """
        if degree <= 0:
            return x
        a = lv.rho / alpha
        b = lv.rho
        theta = 0.5 * (b + a)
        delta = 0.5 * (b - a)
        sigma = theta / delta
        rho_j = 1.0 / sigma
        r = (f - lv.A @ x) / lv.D
        d = r / theta
        for j in range(degree):
            x = x + d
            if j == degree - 1:
                break
            r = r - (lv.A @ d) / lv.D
            rho_next = 1.0 / (2.0 * sigma - rho_j)
            d = rho_next * rho_j * d + (2.0 * rho_next / delta) * r
            rho_j = rho_next
        return x

    @staticmethod
    def cg(lv: Level, x: np.ndarray, f: np.ndarray, nu: int) -> np.ndarray:
        """nu steps of (unpreconditioned) conjugate gradients on A x = f:
        r = f - A x, p = r; then per step alpha = r.r / p.Ap, x += alpha p,
        r -= alpha Ap, beta = r_new.r_new / r.r, p = r + beta p.  A zero
        denominator (an exact solution already) leaves x as it is."""
        if nu <= 0:
            return x
        x = x.copy()
        r = f - lv.A @ x
        p = r.copy()
        rr = float(r @ r)
        for j in range(nu):
            q = lv.A @ p
            pq = float(p @ q)
            alpha = rr / pq if pq != 0.0 else 0.0
            x = x + alpha * p
            if j == nu - 1:
                break
            r = r - alpha * q
            rr_new = float(r @ r)
            beta = rr_new / rr if rr != 0.0 else 0.0
            p = r + beta * p
            rr = rr_new
        return x

    def smooth(self, lv: Level, x, f, opts: MGOptions, nu: int):
        if opts.smoother == "cg":
            return self.cg(lv, x, f, nu)
        if opts.smoother == "jacobi":
            return self.jacobi(lv, x, f, opts.omega, nu)
        if opts.smoother == "cheb":
            return self.chebyshev(lv, x, f, opts.cheb_alpha, nu)
        if opts.smoother == "learned":
            from . import learned
            for _ in range(nu):
                x = learned.step_matrix(lv.A, lv.D, x, f, opts.weights[0], opts.weights[1], opts.learned_bf16)
            return x
        raise ValueError(opts.smoother)

    # -- cycle -----------------------------------------------------------
    def coarse_solve(self, f: np.ndarray) -> np.ndarray:
        return sla.cho_solve(self.coarse_chol, f)

    def vcycle(self, l: int, x: np.ndarray, f: np.ndarray, opts: MGOptions) -> np.ndarray:
        if l == 0:
            return self.coarse_solve(f)
        lv = self.levels[l]
        x = self.smooth(lv, x, f, opts, opts.nu_pre)
        rc = lv.P.T @ (f - lv.A @ x)
        ec = self.vcycle(l - 1, np.zeros_like(rc), rc, opts)
        x = x + lv.P @ ec
        x = self.smooth(lv, x, f, opts, opts.nu_post)
        return x

    def solve(self, x0: np.ndarray, f: np.ndarray, opts: MGOptions) -> np.ndarray:
        """opts.vcycles V-cycles on the finest level starting from x0."""
        x = x0.copy()
        L = len(self.levels) - 1
        for _ in range(opts.vcycles):
            x = self.vcycle(L, x, f, opts)
        return x
