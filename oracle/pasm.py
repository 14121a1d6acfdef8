"""Algorithms 1 and 2 of the paper, plainly, in FP64 (oracle).

TEST INFRASTRUCTURE ONLY (see the package header).

Definition of the result.  The scheme is a fixed-point iteration whose fixed
points are the discrete eigenpairs of the pencil A_h x = lambda M_h x
(Section 2, the discrete eigenproblem): if (lambda, u) is such a pair, the
boundary value problem of Algorithm 1 returns u itself and the augmented space
V_H + span{u} contains it, so Rayleigh-Ritz returns it again.  The reference
values are therefore `discrete_eigenpairs` (dense LAPACK, or shift-invert
Lanczos for large meshes).

Algorithm.  `correction_step` is Algorithm 1 (One Correction Step):
  1. f = lambda M_h u; u~ = approximate solution of A_h u^ = f, either exact
     (sparse LU) or by the V-cycles of `multigrid` started from u;
  2. the augmented pencil of Section 3.1 (matrix form):
         [[A_H, b], [b^T, beta]] z = mu [[M_H, c], [c^T, zeta]] z,
         b = P^T A_h u~, c = P^T M_h u~, beta = u~^T A_h u~, zeta = u~^T M_h u~,
     solved densely; the output is the eigenvector with the largest component
     along u~, measured by |b(u_H + alpha u~, u~)| = |u_H . c + alpha zeta|.
`solve` is Algorithm 2 with h_1 = H: the coarse eigenproblem gives the start
(lambda_i = theta_i, u_i = P q_i) and each eigenpair is corrected on the
finest mesh independently, with no orthogonalisation between them.

Readings of points the paper leaves open (all documented with the design):
  * eigenvectors are M-normalised (u^T M_h u = 1), the normalisation of the
    dense solver; the selection score uses these M^-normalised vectors;
  * inside an augmented eigenvalue of multiplicity > 1 the vector with the
    largest component along u~ is the projection of the score functional onto
    that eigenspace; ties between scores (relative 1e-12) go to the eigenvalue
    closest to the previous one, then to the lower index;
  * sign: b(u_new, u~) > 0;
  * if u~ lies in V_H (zeta - |projection|^2 <= 1e-13 zeta) the augmentation is
    skipped and the coarse Ritz pair with the largest score is taken.

Parity status: pinned (fixed point equals dense eigh of the full pencil on
small meshes; the augmented solve equals brute-force Rayleigh-Ritz on the
fine mesh; tests/test_oracle_pasm.py).
"""
from __future__ import annotations

import dataclasses
import os
import time
from typing import List, Optional

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .fem import assemble, quadratic_potential
from .multigrid import Hierarchy, MGOptions, default_options
from .transfer import galerkin, level_sizes, prolongation

TIE_RTOL = 1e-12
CLUSTER_RTOL = 1e-12
SKIP_RTOL = 1e-13


# ---------------------------------------------------------------------------
# problem set-up
# ---------------------------------------------------------------------------
@dataclasses.dataclass
class Problem:
    dim: int
    n_coarse: int
    n_fine: int
    A: sp.csr_matrix          # fine stiffness (+ potential)
    M: sp.csr_matrix          # fine mass
    P: sp.csr_matrix          # composite prolongation V_H -> V_h
    AH: np.ndarray            # Galerkin P^T A P (dense)
    MH: np.ndarray            # Galerkin P^T M P (dense)


def make_problem(dim: int, n_coarse: int, n_fine: int, kappa=None, centre=None, tensor=None,
                 potential=None) -> Problem:
    """The discrete problem on the fine mesh with its coarse space: centre
    gives the potential |x - c|^2; tensor / potential are callables of the
    centroids (the second example of Section 5: fem.example2_tensor,
    fem.example2_potential)."""
    pot = potential if potential is not None else (None if centre is None else quadratic_potential(centre))
    A, M = assemble(dim, n_fine, kappa=kappa, potential=pot, tensor=tensor)
    P = prolongation(dim, n_coarse, n_fine)
    AH = galerkin(P, A).toarray()
    MH = galerkin(P, M).toarray()
    return Problem(dim, n_coarse, n_fine, A, M, P, AH, MH)


# ---------------------------------------------------------------------------
# the definition: discrete eigenpairs of (A_h, M_h)
# ---------------------------------------------------------------------------
def discrete_eigenpairs(A: sp.spmatrix, M: sp.spmatrix, k: int, dense_limit: int = 6000):
    """The k smallest eigenpairs of A x = lambda M x, x^T M x = 1."""
    N = A.shape[0]
    if N <= dense_limit:
        w, V = sla.eigh(A.toarray(), M.toarray(), subset_by_index=[0, k - 1])
        return w, V
    w, V = spla.eigsh(A.tocsc(), k=k, M=M.tocsc(), sigma=0.0, which="LM", tol=1e-14)
    order = np.argsort(w)
    w, V = w[order], V[:, order]
    V = V / np.sqrt(np.einsum("ij,ij->j", V, M @ V))[None, :]
    return w, V


# ---------------------------------------------------------------------------
# Algorithm 1, step 2: augmented eigenproblem and selection
# ---------------------------------------------------------------------------
def augmented_pencil(AH, MH, b, c, beta, zeta):
    N = AH.shape[0]
    Ahat = np.empty((N + 1, N + 1)); Mhat = np.empty((N + 1, N + 1))
    Ahat[:N, :N] = AH; Ahat[:N, N] = b; Ahat[N, :N] = b; Ahat[N, N] = beta
    Mhat[:N, :N] = MH; Mhat[:N, N] = c; Mhat[N, :N] = c; Mhat[N, N] = zeta
    return Ahat, Mhat


def select_eigvec(mu: np.ndarray, Z: np.ndarray, mvec: np.ndarray, lam_prev: float):
    """Pick the M^-normalised eigenvector z with the largest |z . mvec|.

    mvec is the score functional (= [c; zeta] for the augmented pencil, so that
    z . mvec = b(u_H + alpha u~, u~)).  Returns (index, mu, z, score).
    """
    m = len(mu)
    # canonical representative of each eigenvalue cluster
    cand = []
    j = 0
    while j < m:
        jj = j + 1
        while jj < m and abs(mu[jj] - mu[j]) <= CLUSTER_RTOL * max(abs(mu[j]), abs(mu[jj])):
            jj += 1
        Zc = Z[:, j:jj]
        s = Zc.T @ mvec
        ns = float(np.linalg.norm(s))
        z = Zc @ (s / ns) if (jj - j > 1 and ns > 0) else Zc[:, 0]
        cand.append((j, float(np.mean(mu[j:jj])), z, abs(float(z @ mvec))))
        j = jj
    best = max(c[3] for c in cand)
    ties = [c for c in cand if c[3] >= best * (1.0 - TIE_RTOL)]
    ties.sort(key=lambda c: (abs(c[1] - lam_prev), c[0]))
    return ties[0]


def correction_step(prob: Problem, lam: float, u: np.ndarray, bvp) -> dict:
    """Algorithm 1 for one eigenpair.  `bvp(f, x0)` returns u~ ~= A^{-1} f."""
    f = lam * (prob.M @ u)
    ut = bvp(f, u)
    Au = prob.A @ ut
    Mu = prob.M @ ut
    b = prob.P.T @ Au
    c = prob.P.T @ Mu
    beta = float(ut @ Au)
    zeta = float(ut @ Mu)
    N = prob.AH.shape[0]
    # u~ in V_H: the augmented mass is singular, keep the coarse Ritz pairs
    resid = zeta - float(c @ np.linalg.solve(prob.MH, c))
    if resid <= SKIP_RTOL * zeta:
        theta, Q = sla.eigh(prob.AH, prob.MH)
        j, mu, z, score = select_eigvec(theta, Q, c, lam)
        unew = prob.P @ z
        alpha = 0.0
    else:
        Ahat, Mhat = augmented_pencil(prob.AH, prob.MH, b, c, beta, zeta)
        w, Z = sla.eigh(Ahat, Mhat)
        mvec = np.concatenate([c, [zeta]])
        j, mu, z, score = select_eigvec(w, Z, mvec, lam)
        unew = prob.P @ z[:N] + z[N] * ut
        alpha = float(z[N])
    s = float(unew @ (prob.M @ ut))
    if s < 0:
        unew = -unew
        alpha = -alpha
    return dict(lam=float(mu), u=unew, index=int(j), score=float(score), alpha=alpha,
                b=b, c=c, beta=beta, zeta=zeta, ut=ut)


# ---------------------------------------------------------------------------
# boundary value problem solvers
# ---------------------------------------------------------------------------
class ExactBVP:
    """Sparse LU of A_h, factored once."""

    def __init__(self, A: sp.csr_matrix):
        self.lu = spla.splu(A.tocsc(), permc_spec="MMD_AT_PLUS_A")

    def __call__(self, f, x0):
        return self.lu.solve(f)


class MultigridBVP:
    """The V-cycles of `multigrid`, started from the current eigenvector."""

    def __init__(self, prob: Problem, opts: MGOptions):
        self.h = Hierarchy(prob.dim, prob.A, prob.n_coarse, prob.n_fine)
        self.opts = opts

    def __call__(self, f, x0):
        return self.h.solve(x0, f, self.opts)


# ---------------------------------------------------------------------------
# Algorithm 2 with h_1 = H
# ---------------------------------------------------------------------------
def coarse_start(prob: Problem, k: int):
    """Step 1 of Algorithm 2 on V_H: theta_i, and u_i = P q_i."""
    theta, Q = sla.eigh(prob.AH, prob.MH)
    return theta[:k].copy(), (prob.P @ Q[:, :k]).T.copy(), theta, Q


_WORKER = {}


def _worker_init():
    # one BLAS thread per worker process: the workers already fill the cores
    try:
        from threadpoolctl import threadpool_limits
        _WORKER["limits"] = threadpool_limits(limits=1)
    except ImportError:  # pragma: no cover
        pass


def _worker_run(i):
    prob, bvp, lam0, u0, tol, max_iter = (_WORKER[k] for k in
                                          ("prob", "bvp", "lam0", "u0", "tol", "max_iter"))
    return _iterate_one(prob, bvp, float(lam0[i]), u0[i].copy(), tol, max_iter)


def _iterate_one(prob, bvp, lam, u, tol, max_iter):
    hist = [lam]
    stamps = [time.perf_counter()]
    picks = []
    for _ in range(max_iter):
        out = correction_step(prob, lam, u, bvp)
        dl = abs(out["lam"] - lam) / abs(out["lam"])
        lam, u = out["lam"], out["u"]
        hist.append(lam)
        stamps.append(time.perf_counter())
        picks.append(out["index"])
        if dl < tol:
            break
    return lam, u, hist, stamps, picks


def solve(prob: Problem, k: int, bvp, tol: float = 1e-13, max_iter: int = 60,
          workers: int = 1, which: Optional[List[int]] = None, start=None):
    """Algorithm 2: every eigenpair corrected independently until its relative
    eigenvalue change drops below tol.  Returns dict with lam (k,), U (k, N),
    per-eigenpair histories, timestamps and selected Ritz indices.  start:
    (lambda, U) of the coarse start when already formed by coarse_start."""
    lam0, U0 = start if start is not None else coarse_start(prob, k)[:2]
    idx = list(range(k)) if which is None else list(which)
    if workers <= 1:
        res = [_iterate_one(prob, bvp, float(lam0[i]), U0[i].copy(), tol, max_iter) for i in idx]
    else:
        import multiprocessing as mp
        _WORKER.update(prob=prob, bvp=bvp, lam0=lam0, u0=U0, tol=tol, max_iter=max_iter)
        with mp.get_context("fork").Pool(workers, initializer=_worker_init) as pool:
            res = pool.map(_worker_run, idx, chunksize=1)
        _WORKER.clear()
    lam = np.array([r[0] for r in res])
    U = np.stack([r[1] for r in res])
    return dict(lam=lam, U=U, hist=[r[2] for r in res], stamps=[r[3] for r in res],
                picks=[r[4] for r in res], lam0=lam0[idx], index=idx)


def _record_one(prob, bvp, lam, u, steps, sample):
    rec = []
    for _ in range(steps):
        out = correction_step(prob, lam, u, bvp)
        lam, u = out["lam"], out["u"]
        rec.append((lam, out["index"], out["score"], out["beta"], out["zeta"], u[sample].copy(),
                    float(np.max(np.abs(u)))))
    return rec


def _worker_record(i):
    prob, bvp, lam0, u0, steps, sample = (_WORKER[k] for k in
                                          ("prob", "bvp", "lam0", "u0", "steps", "sample"))
    return _record_one(prob, bvp, float(lam0[i]), u0[i].copy(), steps, sample)


def record_steps(prob: Problem, k: int, bvp, steps: int, sample: np.ndarray, workers: int = 1):
    """The first `steps` correction steps (Algorithm 1) of each of the k
    processes of Algorithm 2 (h_1 = H) from the coarse start.  Returns the
    start (theta_i, and the coarse vectors q_i as columns) and, per step and
    process: lambda, the selected augmented index, its score, beta = a(u~, u~),
    zeta = b(u~, u~), the new u at the `sample` node indices and max |u|."""
    lam0, U0, theta, Q = coarse_start(prob, k)
    if workers <= 1:
        res = [_record_one(prob, bvp, float(lam0[i]), U0[i].copy(), steps, sample) for i in range(k)]
    else:
        import multiprocessing as mp
        _WORKER.update(prob=prob, bvp=bvp, lam0=lam0, u0=U0, steps=steps, sample=sample)
        with mp.get_context("fork").Pool(workers, initializer=_worker_init) as pool:
            res = pool.map(_worker_record, range(k), chunksize=1)
        _WORKER.clear()
    field = lambda f: np.array([[res[i][t][f] for i in range(k)] for t in range(steps)])  # noqa: E731
    return dict(theta=lam0, Q=Q[:, :k].copy(), lam=field(0), index=field(1), score=field(2), beta=field(3),
                zeta=field(4), u_sample=field(5), u_max=field(6))


# ---------------------------------------------------------------------------
# Algorithm 2 with the nested levels of step 2(A)
# ---------------------------------------------------------------------------
def level_problem(prob: Problem, n_level: int) -> Problem:
    """The problem on the intermediate space V_{h_k} (h_k = 1/n_level) of the
    hierarchy between V_H and V_h.  V_{h_k} is a subspace of V_h, so the
    forms a(.,.) and b(.,.) restricted to it are the Galerkin products
    P^T A_h P and P^T M_h P with P the prolongation V_{h_k} -> V_h."""
    if n_level == prob.n_fine:
        return prob
    Pk = prolongation(prob.dim, n_level, prob.n_fine)
    A = galerkin(Pk, prob.A)
    M = galerkin(Pk, prob.M)
    PH = prolongation(prob.dim, prob.n_coarse, n_level)
    return Problem(prob.dim, prob.n_coarse, n_level, A, M, PH, prob.AH, prob.MH)


def solve_nested(prob: Problem, k: int, make_bvp, varpi: int = 1, varpi_n: int = 0,
                 which: Optional[List[int]] = None):
    """Algorithm 2 with h_1 = H and its nested step 2(A):
      1. the coarse eigenpairs (theta_i, q_i) on V_H = V_{h_1};
      2(A). for every intermediate level h_2, ..., h_{n-1} (ratio 2): start
         from the previous level's result (a function of the coarser space is
         also one of the finer space: its nodal values are the prolongation),
         then `varpi` correction steps (Algorithm 1 with the coarse space V_H,
         on that level);
      2(B). `varpi_n` correction steps on the finest level.
    make_bvp(level_problem) gives the boundary value solver of a level.
    Returns the finest-level start (after 2(A)) and the final eigenpairs,
    with per-process eigenvalue histories over the whole schedule."""
    sizes = level_sizes(prob.n_coarse, prob.n_fine)
    theta, Q = sla.eigh(prob.AH, prob.MH)
    idx = list(range(k)) if which is None else list(which)
    lam = theta[idx].copy()
    coarse = Q[:, idx].T.copy()              # u_i as functions of V_H (coarse nodal values)
    hist = [[float(l)] for l in lam]
    cur_n = prob.n_coarse
    U = coarse
    for n_l in sizes[1:-1]:
        lp = level_problem(prob, n_l)
        Pstep = prolongation(prob.dim, cur_n, n_l)
        U = (Pstep @ U.T).T.copy()
        bvp = make_bvp(lp)
        for i in range(len(idx)):
            for _ in range(varpi):
                out = correction_step(lp, float(lam[i]), U[i], bvp)
                lam[i], U[i] = out["lam"], out["u"]
                hist[i].append(float(lam[i]))
        cur_n = n_l
    Pstep = prolongation(prob.dim, cur_n, prob.n_fine)
    U = (Pstep @ U.T).T.copy()
    lam_start, U_start = lam.copy(), U.copy()
    if varpi_n > 0:
        bvp = make_bvp(prob)
        for i in range(len(idx)):
            for _ in range(varpi_n):
                out = correction_step(prob, float(lam[i]), U[i], bvp)
                lam[i], U[i] = out["lam"], out["u"]
                hist[i].append(float(lam[i]))
    return dict(lam_start=lam_start, U_start=U_start, lam=lam, U=U, hist=hist, index=idx)


def mg_options_for(workload) -> MGOptions:
    return default_options(workload.dim, workload.smoother, workload.nu_pre,
                           workload.nu_post, workload.vcycles)


def cpu_count() -> int:
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        return os.cpu_count() or 1
