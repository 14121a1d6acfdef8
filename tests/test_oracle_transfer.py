"""Pins of the oracle's prolongation and Galerkin operators (Section 3, nested
P1 spaces) against brute-force point evaluation and direct coarse assembly."""
import itertools

import numpy as np
import pytest

from oracle import fem, transfer
from workloads import lognormal_kappa


def _brute_eval(dim, n, values, x):
    """Evaluate the P1 function with nodal `values` (full mesh) at point x by
    testing every simplex for non-negative barycentric coordinates."""
    X = fem.kuhn_elements(dim, n)
    ids = fem.node_ids(X, n)
    P = X.astype(float) / n
    for e in range(X.shape[0]):
        B = (P[e, 1:] - P[e, 0]).T            # columns: edge vectors
        lam = np.linalg.solve(B, x - P[e, 0])
        bary = np.concatenate([[1 - lam.sum()], lam])
        if np.all(bary >= -1e-12):
            return float(bary @ values[ids[e]])
    raise AssertionError("point outside the mesh")


@pytest.mark.parametrize("dim,nc,nf", [(2, 2, 4), (2, 3, 6), (3, 2, 4)])
def test_prolongation_is_pointwise_evaluation(dim, nc, nf):
    rng = np.random.default_rng(0)
    vc = rng.standard_normal((nc + 1) ** dim)
    P = transfer.prolongation(dim, nc, nf, full=True)
    vf = P @ vc
    coords = fem.all_node_coords(dim, nf)
    for q in rng.choice(len(coords), size=min(40, len(coords)), replace=False):
        x = coords[q] / nf
        assert vf[q] == pytest.approx(_brute_eval(dim, nc, vc, x), abs=1e-12)


@pytest.mark.parametrize("dim", [2, 3])
def test_prolongation_reproduces_affine_functions(dim):
    g = np.array([0.7, -1.3, 2.0][:dim])
    f = lambda x: x @ g + 0.25
    P = transfer.prolongation(dim, 4, 16 if dim == 2 else 8, full=True)
    vc = fem.interpolate(f, dim, 4, full=True)
    vf = fem.interpolate(f, dim, 16 if dim == 2 else 8, full=True)
    assert np.max(np.abs(P @ vc - vf)) < 1e-13


@pytest.mark.parametrize("dim,nc,nf", [(2, 4, 16), (3, 2, 8)])
def test_composite_equals_product(dim, nc, nf):
    direct = transfer.prolongation(dim, nc, nf)
    prod = None
    n = nc
    while n < nf:
        step = transfer.prolongation(dim, n, 2 * n)
        prod = step if prod is None else step @ prod
        n *= 2
    assert abs(direct - prod).max() < 1e-15


@pytest.mark.parametrize("dim,nc", [(2, 4), (2, 8), (3, 2), (3, 4)])
def test_galerkin_equals_direct_coarse_assembly_constant(dim, nc):
    A_f, M_f = fem.assemble(dim, 2 * nc)
    A_c, M_c = fem.assemble(dim, nc)
    P = transfer.prolongation(dim, nc, 2 * nc)
    assert abs(transfer.galerkin(P, A_f) - A_c).max() < 1e-13
    assert abs(transfer.galerkin(P, M_f) - M_c).max() < 1e-16


def _children_mean(dim, nc, kappa_f):
    """Arithmetic mean of the fine coefficient over the 2^d children of every
    coarse simplex; children found by locating fine centroids."""
    nf = 2 * nc
    Xf = fem.kuhn_elements(dim, nf)
    cen = Xf.astype(float).mean(axis=1) / nf * nc           # in coarse cell units
    cell = np.floor(cen).astype(int)
    xi = cen - cell
    perms = list(itertools.permutations(range(dim)))
    order = np.argsort(-xi, axis=1)
    p = np.array([perms.index(tuple(o)) for o in order])
    cid = np.zeros(len(cell), dtype=int)
    stride = 1
    for a in range(dim):
        cid += cell[:, a] * stride
        stride *= nc
    coarse = cid * len(perms) + p
    tot = np.bincount(coarse, weights=kappa_f, minlength=nc ** dim * len(perms))
    cnt = np.bincount(coarse, minlength=nc ** dim * len(perms))
    assert np.all(cnt == 2 ** dim)
    return tot / cnt


def test_galerkin_equals_mean_coefficient_rediscretisation_2d():
    nc = 8
    kap = lognormal_kappa(2, 2 * nc, seed=0)
    A_f, _ = fem.assemble(2, 2 * nc, kappa=kap)
    A_c, _ = fem.assemble(2, nc, kappa=_children_mean(2, nc, kap))
    P = transfer.prolongation(2, nc, 2 * nc)
    G = transfer.galerkin(P, A_f)
    assert abs(G - A_c).max() < 1e-12 * abs(A_c).max()


def test_galerkin_of_potential_is_seven_point_2d():
    nc = 8
    pot = fem.quadratic_potential([0.3, 0.6])
    A_f, _ = fem.assemble(2, 2 * nc, potential=pot)
    A0, _ = fem.assemble(2, 2 * nc)
    P = transfer.prolongation(2, nc, 2 * nc)
    G = (transfer.galerkin(P, A_f - A0)).toarray()
    m = nc - 1
    for r in range(G.shape[0]):
        i, j = r % m, r // m
        for q in np.flatnonzero(np.abs(G[r]) > 1e-15):
            di, dj = q % m - i, q // m - j
            assert (di, dj) in {(0, 0), (1, 0), (-1, 0), (0, 1), (0, -1), (1, 1), (-1, -1)}
