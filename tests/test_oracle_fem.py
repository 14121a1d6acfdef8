"""Pins of the oracle's P1 assembly (Section 2) against facts fixed by the
mathematics, not by the oracle: hand-derived stencils, exact integrals of
linear functions, an independent quadrature rule, the continuum eigenvalues
pi^2 (m^2 + n^2) with O(h^2) convergence, and the min-max upper bound."""
import itertools
import math

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import fem
from workloads import lognormal_kappa


def _node(n, *c):
    """Interior index of interior node c (x fastest)."""
    idx = 0
    stride = 1
    for a in c:
        idx += (a - 1) * stride
        stride *= n - 1
    return idx


def test_stiffness_and_mass_stencil_2d():
    # Hand derivation: each interior node touches 6 right triangles of area h^2/2;
    # legs couple with -1/2 per triangle, hypotenuses with 0.  Mass: |T|/12 (1+delta).
    n = 8
    h = 1.0 / n
    A, M = fem.assemble(2, n)
    i, j = 4, 4
    r = _node(n, i, j)
    row_a = A[r].toarray().ravel()
    row_m = M[r].toarray().ravel()
    expect_a = {(0, 0): 4.0, (1, 0): -1.0, (-1, 0): -1.0, (0, 1): -1.0, (0, -1): -1.0,
                (1, 1): 0.0, (-1, -1): 0.0, (1, -1): 0.0, (-1, 1): 0.0}
    expect_m = {(0, 0): 0.5, (1, 0): 1 / 12, (-1, 0): 1 / 12, (0, 1): 1 / 12, (0, -1): 1 / 12,
                (1, 1): 1 / 12, (-1, -1): 1 / 12, (1, -1): 0.0, (-1, 1): 0.0}
    for (dx, dy), v in expect_a.items():
        assert row_a[_node(n, i + dx, j + dy)] == pytest.approx(v, abs=1e-14)
    for (dx, dy), v in expect_m.items():
        assert row_m[_node(n, i + dx, j + dy)] == pytest.approx(v * h * h, abs=1e-16)
    assert np.count_nonzero(np.abs(row_a) > 1e-14) == 5
    assert np.count_nonzero(np.abs(row_m) > 1e-18) == 7


def test_stiffness_and_mass_stencil_3d():
    # Kuhn tetrahedra: 24 around each node; axis edges in 6 tets, face diagonals
    # (1,1,0)-type in 4, the body diagonal (1,1,1) in 6.  |T| = h^3/6, M_T = |T|/20 (1+delta).
    n = 6
    h = 1.0 / n
    A, M = fem.assemble(3, n)
    c = (3, 3, 3)
    r = _node(n, *c)
    row_a = A[r].toarray().ravel()
    row_m = M[r].toarray().ravel()
    for off in itertools.product((-1, 0, 1), repeat=3):
        q = _node(n, *(c[a] + off[a] for a in range(3)))
        s = sum(abs(o) for o in off)
        same_sign = all(o >= 0 for o in off) or all(o <= 0 for o in off)
        if s == 0:
            ea, em = 6.0 * h, 0.4 * h ** 3
        elif s == 1:
            ea, em = -1.0 * h, h ** 3 / 20
        elif s == 2 and same_sign:
            ea, em = 0.0, h ** 3 / 30
        elif s == 3 and same_sign:
            ea, em = 0.0, h ** 3 / 20
        else:
            ea, em = 0.0, 0.0
        assert row_a[q] == pytest.approx(ea, abs=1e-14)
        assert row_m[q] == pytest.approx(em, abs=1e-17)


def test_variable_kappa_edge_weights_2d():
    # The edge (i,j)-(i+1,j) is a leg of the lower triangle of cell (i,j) and of
    # the upper triangle of cell (i,j-1); each leg couples with -kappa_T/2.
    n = 6
    kap = lognormal_kappa(2, n, seed=3)
    A, _ = fem.assemble(2, n, kappa=kap)

    def kl(ci, cj):
        return kap[2 * (ci + n * cj)]

    def ku(ci, cj):
        return kap[2 * (ci + n * cj) + 1]

    i, j = 2, 3
    a_e = A[_node(n, i, j), _node(n, i + 1, j)]
    a_n = A[_node(n, i, j), _node(n, i, j + 1)]
    # vertical edge (i,j)-(i,j+1): leg of the upper triangle of cell (i,j) and of
    # the lower triangle of cell (i-1,j)
    assert a_e == pytest.approx(-(kl(i, j) + ku(i, j - 1)) / 2, rel=1e-14)
    assert a_n == pytest.approx(-(ku(i, j) + kl(i - 1, j)) / 2, rel=1e-14)
    assert abs(A[_node(n, i, j), _node(n, i + 1, j + 1)]) < 1e-14


@pytest.mark.parametrize("dim", [2, 3])
def test_linear_functions_integrated_exactly(dim):
    # For affine f = g.x + c0 (its own interpolant): a(f,f) = sum_T kappa_T |T| |g|^2,
    # b(f,f) = int f^2 = |mean|^2 + var with x ~ U(0,1)^d.
    n = 4
    g = np.array([1.0, -2.0, 0.5][:dim])
    c0 = 0.3
    kap = lognormal_kappa(dim, n, seed=1)
    A, M = fem.assemble(dim, n, kappa=kap, full=True)
    f = fem.interpolate(lambda x: x @ g + c0, dim, n, full=True)
    vol = (1.0 / n) ** dim / math.factorial(dim)
    assert f @ (A @ f) == pytest.approx(np.sum(kap) * vol * (g @ g), rel=1e-12)
    mean = c0 + 0.5 * g.sum()
    var = (g @ g) / 12.0
    assert f @ (M @ f) == pytest.approx(mean ** 2 + var, rel=1e-12)
    assert M.sum() == pytest.approx(1.0, rel=1e-13)
    assert np.max(np.abs(A @ np.ones(A.shape[0]))) < 1e-12


@pytest.mark.parametrize("dim", [2, 3])
def test_mass_against_independent_quadrature(dim):
    # Degree-2 exact rules: 2D edge midpoints (weights 1/3); 3D the 4-point rule
    # with barycentric (a, b, b, b), a = 0.5854101966249685, b = 0.1381966011250105.
    n = 3
    rng = np.random.default_rng(7)
    _, M = fem.assemble(dim, n, full=True)
    N = (n + 1) ** dim
    u, v = rng.standard_normal(N), rng.standard_normal(N)
    X = fem.kuhn_elements(dim, n)
    ids = fem.node_ids(X, n)
    vol = (1.0 / n) ** dim / math.factorial(dim)
    if dim == 2:
        pts = np.array([[0.5, 0.5, 0.0], [0.0, 0.5, 0.5], [0.5, 0.0, 0.5]])
    else:
        a, b = 0.5854101966249685, 0.1381966011250105
        pts = np.array([[a, b, b, b], [b, a, b, b], [b, b, a, b], [b, b, b, a]])
    wq = 1.0 / pts.shape[0]
    uq = pts @ u[ids].T          # (q, E)
    vq = pts @ v[ids].T
    integral = vol * wq * np.sum(uq * vq)
    assert u @ (M @ v) == pytest.approx(integral, rel=1e-12)


def _continuum_2d(count):
    vals = sorted(m * m + k * k for m in range(1, 8) for k in range(1, 8))
    return np.pi ** 2 * np.array(vals[:count], dtype=float)


def test_eigenvalues_converge_at_order_h2_2d():
    # Corollary 3.1: |lambda - lambda_h| = O(h^2); eigenvalues of the unit square
    # are pi^2 (m^2 + n^2).  Discrete ones are upper bounds (min-max).
    exact = _continuum_2d(4)
    errs = []
    for n in (8, 16, 32):
        A, M = fem.assemble(2, n)
        w = sla.eigh(A.toarray(), M.toarray(), eigvals_only=True, subset_by_index=[0, 3])
        assert np.all(w > 0) and np.all(np.diff(w) >= 0)
        assert np.all(w >= exact * (1 - 1e-14))
        errs.append(w - exact)
    errs = np.array(errs)
    ratios = errs[:-1] / errs[1:]
    assert np.all(ratios[-1] > 3.6) and np.all(ratios[-1] < 4.4)


def test_eigenvalues_converge_at_order_h2_3d():
    exact = 3 * np.pi ** 2
    errs = []
    for n in (4, 8, 16):
        A, M = fem.assemble(3, n)
        if A.shape[0] < 2000:
            w = sla.eigh(A.toarray(), M.toarray(), eigvals_only=True, subset_by_index=[0, 0])[0]
        else:
            import scipy.sparse.linalg as spla
            w = spla.eigsh(A.tocsc(), k=1, M=M.tocsc(), sigma=0, which="LM")[0][0]
        assert w >= exact
        errs.append(w - exact)
    r = errs[1] / errs[2]
    assert 3.4 < r < 4.6


def test_rayleigh_quotient_expansion_is_exact():
    # Lemma 2.1 for the discrete pencil: for any w and eigenpair (lam, u),
    # a(w,w)/b(w,w) - lam = a(w-u,w-u)/b(w,w) - lam b(w-u,w-u)/b(w,w).
    n = 10
    kap = lognormal_kappa(2, n, seed=5)
    A, M = fem.assemble(2, n, kappa=kap)
    lam, U = sla.eigh(A.toarray(), M.toarray(), subset_by_index=[0, 2])
    rng = np.random.default_rng(11)
    for i in range(3):
        u = U[:, i] * 3.7
        w = u + 0.1 * rng.standard_normal(u.shape)
        bw = w @ M @ w
        lhs = (w @ A @ w) / bw - lam[i]
        d = w - u
        rhs = (d @ A @ d) / bw - lam[i] * (d @ M @ d) / bw
        assert lhs == pytest.approx(rhs, rel=1e-9, abs=1e-12)


def test_stencil_built_stiffness_3d_equals_assembly():
    from stencil_ops import constant_stiffness_3d
    for n in (4, 8):
        A, _ = fem.assemble(3, n)
        B = constant_stiffness_3d(n)
        assert abs(A - B).max() < 1e-15


# ---------------------------------------------------------------------------
# the full diffusion tensor of the second example (Section 5.2)
# ---------------------------------------------------------------------------
def test_tensor_identity_equals_the_scalar_assembly():
    A0, M0 = fem.assemble(3, 4)
    A1, M1 = fem.assemble(3, 4, tensor=lambda x: np.repeat(np.eye(3)[None], x.shape[0], axis=0))
    assert abs(A1 - A0).max() < 1e-14 and abs(M1 - M0).max() == 0.0


def test_constant_tensor_integrates_linear_functions_exactly():
    # a(u, v) = int grad u . C grad v = a^T C b over the unit cube for
    # u = a.x, v = b.x (the centroid rule is exact for a constant tensor)
    C = np.array([[2.0, 0.3, -0.2], [0.3, 1.5, 0.4], [-0.2, 0.4, 1.2]])
    A, _ = fem.assemble(3, 3, full=True, tensor=lambda x: np.repeat(C[None], x.shape[0], axis=0))
    x = fem.all_node_coords(3, 3).astype(np.float64) / 3
    rng = np.random.default_rng(0)
    for _ in range(3):
        a, b = rng.standard_normal(3), rng.standard_normal(3)
        assert (x @ a) @ (A @ (x @ b)) == pytest.approx(a @ C @ b, rel=1e-12)


def test_example2_operator_is_a_symmetric_15_point_stencil():
    n = 6
    A, M = fem.assemble(3, n, tensor=fem.example2_tensor, potential=fem.example2_potential)
    assert abs(A - A.T).max() < 1e-15
    assert np.min(np.linalg.eigvalsh(A.toarray())) > 0.0
    # couplings only along the Kuhn edges +-(1,0,0) .. +-(1,1,1)
    m = n - 1
    allowed = {0}
    for o in [(1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 1, 0), (1, 0, 1), (0, 1, 1), (1, 1, 1)]:
        d = o[0] + o[1] * m + o[2] * m * m
        allowed |= {d, -d}
    Ac = A.tocoo()
    offs = set((Ac.col - Ac.row).tolist())
    assert offs <= allowed
    # the off-axis couplings are really there (the identity tensor has none)
    assert any(abs(A[i, i + 1 + m]) > 1e-12 for i in range(10))
    # phi = exp(prod(x - 1/2)) enters as phi M at element centroids: with the
    # identity tensor the difference to the Laplacian is that mass term
    A2, _ = fem.assemble(3, n, potential=fem.example2_potential)
    A3, _ = fem.assemble(3, n)
    D = (A2 - A3).toarray()
    assert np.min(np.linalg.eigvalsh(D)) > 0.0


def test_example2_galerkin_levels_stay_15_point():
    from oracle.transfer import galerkin, prolongation
    A, _ = fem.assemble(3, 8, tensor=fem.example2_tensor, potential=fem.example2_potential)
    Ac = galerkin(prolongation(3, 4, 8), A).tocoo()
    m = 3
    allowed = {0}
    for o in [(1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 1, 0), (1, 0, 1), (0, 1, 1), (1, 1, 1)]:
        d = o[0] + o[1] * m + o[2] * m * m
        allowed |= {d, -d}
    big = np.abs(Ac.data) > 1e-14 * np.abs(Ac.data).max()
    assert set((Ac.col - Ac.row)[big].tolist()) <= allowed
