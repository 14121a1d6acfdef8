"""Pins of the oracle's two eigensolver pieces that the full-size references
rest on.

* `discrete_eigenpairs`, shift-invert Lanczos branch (used above 6000 unknowns,
  so for every stored 1M-node value): forced on small meshes with exact
  (3D Kuhn cube) and near-degenerate (2D "/" square) eigenvalues and compared
  with the dense branch, multiplicities included.
* The stored 1M-node eigenvalues: the continuum eigenvalues of the unit square
  are pi^2 (m^2 + n^2) (Example 1's operator; the discrete ones converge at
  O(h^2), Corollary 3.1), so every cluster of the stored list must have the
  size of the continuum multiplicity and lie within the O(h^2) error of it.
  A missed member of a pair would shift the whole list and fail this.
* `select_eigvec` (Algorithm 1, step 2: the eigenvector with the largest
  component along u~) inside a repeated eigenvalue, against brute force over
  the eigenspace, and its independence of the basis the dense solver returns.
"""
import math
import os

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import fem
from oracle import pasm as O

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _cluster_starts(w, rtol):
    starts = [0]
    for j in range(1, len(w)):
        if (w[j] - w[j - 1]) > rtol * w[j]:
            starts.append(j)
    return starts + [len(w)]


def _subspace_gap(V1, V2, M):
    """Largest principal angle (sine) between two M-orthonormal bases."""
    s = np.linalg.svd(V1.T @ (M @ V2), compute_uv=False)
    return float(np.sqrt(max(0.0, 1.0 - np.min(s) ** 2)))


@pytest.mark.parametrize("dim,n,k", [(2, 64, 12), (3, 8, 12), (3, 12, 10)])
def test_lanczos_branch_equals_dense_branch(dim, n, k):
    A, M = fem.assemble(dim, n)
    wd, Vd = O.discrete_eigenpairs(A, M, k)                      # dense LAPACK
    wl, Vl = O.discrete_eigenpairs(A, M, k, dense_limit=0)       # shift-invert Lanczos
    # the dense generalized solver's eigenvalues carry errors up to ~1e-12
    # (its Cholesky reduction); the Rayleigh quotients of its vectors are
    # second-order accurate and pin the Lanczos values far tighter
    assert np.max(np.abs(wl - wd) / wd) < 1e-11
    rq = np.einsum("ij,ij->j", Vd, A @ Vd) / np.einsum("ij,ij->j", Vd, M @ Vd)
    assert np.max(np.abs(wl - rq) / rq) < 1e-13
    # multiplicities: the same clusters (exact ones in 3D, rel. gaps down to
    # 3e-6 in 2D), and the same invariant subspaces
    st = _cluster_starts(wd, 1e-9)
    assert st == _cluster_starts(wl, 1e-9)
    if dim == 3:
        assert any(b - a >= 2 for a, b in zip(st[:-1], st[1:])), "expected an exact multiple eigenvalue"
    for a, b in zip(st[:-1], st[1:]):
        assert _subspace_gap(Vd[:, a:b], Vl[:, a:b], M) < 1e-7
    # M-orthonormal
    G = Vl.T @ (M @ Vl)
    assert np.max(np.abs(G - np.eye(k))) < 1e-10


def _continuum_unit_square(count):
    vals = sorted((m * m + q * q) for m in range(1, 40) for q in range(1, 40))
    return np.array(vals[:count], dtype=np.float64) * math.pi ** 2


def test_stored_1m_node_eigenvalues_have_the_continuum_multiplicities():
    w = np.loadtxt(os.path.join(GOLDEN, "lap2d-H32-h1024-k20.eigenvalues.txt"), comments="#")
    h = 1.0 / 1024
    lam = _continuum_unit_square(len(w) + 4)
    # discrete above continuum (min-max, Section 2), O(h^2) close: the "/"
    # mesh's first-order error term is bounded by (m^4 + n^4) h^2 / 12
    # relative to pi^2 (m^2 + n^2); 40 (m^2+n^2) h^2 covers m^2+n^2 <= 40
    rel = (w - lam[:len(w)]) / lam[:len(w)]
    assert np.all(rel > 0.0)
    assert np.all(rel < 40.0 * (lam[:len(w)] / math.pi ** 2) * h * h)
    # the same cluster pattern: continuum multiplicities 1 or 2 (m != n)
    # against discrete clusters at a relative gap far above the splitting
    # of the pairs (<= 2e-5 here) and far below the continuum gaps (>= 0.04)
    st_w = _cluster_starts(w, 1e-3)
    st_c = _cluster_starts(lam[:len(w)], 1e-3)
    assert st_w == st_c


def _pencil_with_double_eigenvalue(n, seed):
    rng = np.random.default_rng(seed)
    B = rng.standard_normal((n, n))
    M = B @ B.T + n * np.eye(n)
    # M-orthonormal basis: V = L^{-T} W with M = L L^T, W orthogonal
    L = np.linalg.cholesky(M)
    W, _ = np.linalg.qr(rng.standard_normal((n, n)))
    V = np.linalg.solve(L.T, W)
    w = np.array([1.0, 2.0, 2.0] + list(np.linspace(3.0, 9.0, n - 3)))
    Minv_mult = M @ V
    A = Minv_mult @ np.diag(w) @ Minv_mult.T
    return A, M, rng.standard_normal(n)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_select_eigvec_inside_repeated_eigenvalue_is_bruteforce_maximum(seed):
    n = 9
    A, M, mvec = _pencil_with_double_eigenvalue(n, seed)
    mu, Z = sla.eigh(A, M)
    assert abs(mu[1] - mu[2]) < 1e-12 * mu[2]
    j, m_sel, z, score = O.select_eigvec(mu, Z, mvec, lam_prev=2.0)
    # brute force: every M-normalised direction cos t z1 + sin t z2 of the
    # double eigenvalue's eigenspace, and every other eigenvector
    t = np.linspace(0.0, np.pi, 200001)
    Zt = np.outer(Z[:, 1], np.cos(t)) + np.outer(Z[:, 2], np.sin(t))
    s_space = np.abs(mvec @ Zt)
    s_other = [abs(float(mvec @ Z[:, i])) for i in range(n) if i not in (1, 2)]
    best = max(float(np.max(s_space)), max(s_other))
    assert score >= best * (1 - 1e-9)
    assert score == pytest.approx(abs(float(z @ mvec)), rel=1e-13)
    assert float(z @ (M @ z)) == pytest.approx(1.0, rel=1e-12)
    if float(np.max(s_space)) > max(s_other):
        assert j == 1 and m_sel == pytest.approx(2.0, rel=1e-12)
        # z is an eigenvector of the double eigenvalue
        assert np.max(np.abs(A @ z - 2.0 * (M @ z))) < 1e-9 * np.max(np.abs(A @ z))
        # and the brute-force maximiser up to sign
        zb = Zt[:, int(np.argmax(s_space))]
        zb = zb if zb @ (M @ z) > 0 else -zb
        assert np.max(np.abs(zb - z)) < 1e-4 * np.max(np.abs(z))


def test_select_eigvec_does_not_depend_on_the_eigenspace_basis():
    n = 9
    A, M, mvec = _pencil_with_double_eigenvalue(n, 5)
    mu, Z = sla.eigh(A, M)
    # make the double eigenvalue the winner: put the functional into its eigenspace
    mvec = M @ (0.3 * Z[:, 1] - 0.8 * Z[:, 2]) + 1e-3 * mvec
    sel = [O.select_eigvec(mu, Z, mvec, 2.0)]
    for ang in (0.3, 1.1, 2.5):
        R = np.array([[math.cos(ang), -math.sin(ang)], [math.sin(ang), math.cos(ang)]])
        Z2 = Z.copy()
        Z2[:, 1:3] = Z[:, 1:3] @ R
        sel.append(O.select_eigvec(mu, Z2, mvec, 2.0))
    for j, m_sel, z, score in sel[1:]:
        assert j == sel[0][0]
        assert score == pytest.approx(sel[0][3], rel=1e-12)
        z0 = sel[0][2]
        zz = z if z @ (M @ z0) > 0 else -z
        assert np.max(np.abs(zz - z0)) < 1e-12 * np.max(np.abs(z0))


def test_select_eigvec_tie_goes_to_the_eigenvalue_nearest_the_previous_one():
    # two distinct eigenvalues with exactly equal scores: the reading takes
    # the one nearest the previous eigenvalue, then the lower index
    M = np.eye(3)
    mu = np.array([1.0, 2.0, 3.0])
    Z = np.eye(3)
    mvec = np.array([0.5, 0.1, 0.5])
    assert O.select_eigvec(mu, Z, mvec, 2.9)[0] == 2
    assert O.select_eigvec(mu, Z, mvec, 1.2)[0] == 0
    assert O.select_eigvec(mu, Z, mvec, 2.0)[0] == 0
