"""P1 finite elements on the uniform Kuhn simplex mesh of the unit box (oracle).

TEST INFRASTRUCTURE ONLY (see the package header).

Follows Section 2 of the paper: the model problem -div(A grad u) = lambda u with
homogeneous Dirichlet data, its weak form a(u,v) = lambda b(u,v) with
a(u,v) = int A grad u . grad v and b(u,v) = int u v, and the linear
finite element space V_h on a shape-regular simplicial mesh.  The diffusion
tensor is taken as kappa(x) I with kappa constant on every element, and the
optional zeroth-order term of the second example (Section 5.2) is added as
int V u v with V evaluated at the element centroid.

The mesh is the Kuhn (Freudenthal) split of the uniform cubic grid: every cell
with origin o is cut into d! simplices, simplex `p` having the vertex path
o, o+e[pi0], o+e[pi0]+e[pi1], ..., o+(1,...,1) for pi the p-th permutation.
In 2D this is the "/" split into two right triangles.  Element order and the
node numbering (x fastest) are the ones documented in `workloads`.

Assembly is element by element with the textbook formulas
    K_T = kappa_T |T| G G^T       (G = gradients of the barycentric functions)
    M_T = |T| (1 + delta_ij) / ((d+1)(d+2))
    V_T = V(centroid_T) M_T
summed into global sparse matrices; Dirichlet nodes are then removed.

Parity status: pinned.  The stencils are checked against closed forms derived
by hand from the element integrals, the bilinear forms against an independent
quadrature rule, and the discrete eigenvalues against the O(h^2) convergence to
pi^2 (m^2 + n^2) and the min-max upper bound (tests/test_oracle_fem.py).
"""
from __future__ import annotations

import itertools
import math
from typing import Callable, Optional, Tuple

import numpy as np
import scipy.sparse as sp


def node_ids(coords: np.ndarray, n: int) -> np.ndarray:
    """Global node number of integer node coordinates (..., d), x fastest."""
    d = coords.shape[-1]
    out = np.zeros(coords.shape[:-1], dtype=np.int64)
    stride = 1
    for a in range(d):
        out += coords[..., a].astype(np.int64) * stride
        stride *= n + 1
    return out


def all_node_coords(dim: int, n: int) -> np.ndarray:
    """Integer coordinates of all (n+1)^d nodes in global order (x fastest)."""
    idx = np.arange((n + 1) ** dim)
    return np.stack([(idx // (n + 1) ** a) % (n + 1) for a in range(dim)], axis=1)


def interior_mask(dim: int, n: int) -> np.ndarray:
    c = all_node_coords(dim, n)
    return np.all((c > 0) & (c < n), axis=1)


def kuhn_elements(dim: int, n: int) -> np.ndarray:
    """Integer vertex coordinates of every simplex, shape (n^d * d!, d+1, d).

    Element order: cell index (x fastest) major, permutation index minor.
    """
    cells = np.arange(n ** dim)
    origin = np.stack([(cells // n ** a) % n for a in range(dim)], axis=1)  # (C, d)
    perms = list(itertools.permutations(range(dim)))
    eye = np.eye(dim, dtype=np.int64)
    verts = np.zeros((n ** dim, len(perms), dim + 1, dim), dtype=np.int64)
    for p, perm in enumerate(perms):
        v = origin.copy()
        verts[:, p, 0, :] = v
        for m, axis in enumerate(perm):
            v = v + eye[axis]
            verts[:, p, m + 1, :] = v
    return verts.reshape(-1, dim + 1, dim)


def element_geometry(X: np.ndarray, h: float) -> Tuple[np.ndarray, np.ndarray]:
    """Volumes |T| and barycentric gradients G (E, d+1, d) of simplices X*h."""
    P = X.astype(np.float64) * h
    d = X.shape[-1]
    B = P[:, 1:, :] - P[:, :1, :]                     # rows: edge vectors from vertex 0
    vol = np.abs(np.linalg.det(B)) / math.factorial(d)
    # x - v0 = B^T lam  =>  lam = B^{-T} (x - v0); grad lam_m = row m of B^{-T}
    C = np.linalg.inv(np.transpose(B, (0, 2, 1)))
    G = np.concatenate([-C.sum(axis=1, keepdims=True), C], axis=1)
    return vol, G


def _scatter(nodes: np.ndarray, local: np.ndarray, size: int) -> sp.csr_matrix:
    nl = nodes.shape[1]
    rows = np.repeat(nodes, nl, axis=1).ravel()
    cols = np.tile(nodes, (1, nl)).ravel()
    return sp.coo_matrix((local.ravel(), (rows, cols)), shape=(size, size)).tocsr()


def assemble(dim: int, n: int,
             kappa: Optional[np.ndarray] = None,
             potential: Optional[Callable[[np.ndarray], np.ndarray]] = None,
             full: bool = False,
             tensor: Optional[Callable[[np.ndarray], np.ndarray]] = None):
    """Stiffness A (with the potential term, if any) and mass M.

    kappa: per-element coefficient (None means 1).
    potential: V(x) evaluated at element centroids, x of shape (E, d).
    tensor: the diffusion tensor A(x) (E, d, d) evaluated at element
            centroids (None means the identity): K_T = kappa_T |T| G A_T G^T.
    full: if True return matrices over all nodes, else over interior nodes only
          (homogeneous Dirichlet condition, Section 2).
    """
    h = 1.0 / n
    X = kuhn_elements(dim, n)
    E = X.shape[0]
    vol, G = element_geometry(X, h)
    kap = np.ones(E) if kappa is None else np.asarray(kappa, dtype=np.float64)
    assert kap.shape == (E,)
    if tensor is None:
        K_loc = (kap * vol)[:, None, None] * np.einsum("eid,ejd->eij", G, G)
    else:
        centroid = X.astype(np.float64).mean(axis=1) * h
        At = np.asarray(tensor(centroid), dtype=np.float64)
        assert At.shape == (E, dim, dim)
        K_loc = (kap * vol)[:, None, None] * np.einsum("eid,edf,ejf->eij", G, At, G)
    ref_mass = (np.ones((dim + 1, dim + 1)) + np.eye(dim + 1)) / ((dim + 1) * (dim + 2))
    M_loc = vol[:, None, None] * ref_mass[None]
    if potential is not None:
        centroid = X.astype(np.float64).mean(axis=1) * h
        K_loc = K_loc + np.asarray(potential(centroid))[:, None, None] * M_loc
    nodes = node_ids(X, n)
    size = (n + 1) ** dim
    A = _scatter(nodes, K_loc, size)
    M = _scatter(nodes, M_loc, size)
    if full:
        return A, M
    keep = np.flatnonzero(interior_mask(dim, n))
    return A[keep][:, keep].tocsr(), M[keep][:, keep].tocsr()


def interpolate(f: Callable[[np.ndarray], np.ndarray], dim: int, n: int,
                full: bool = False) -> np.ndarray:
    """Nodal interpolant of f (vectorised over points (N, d)) on the mesh."""
    x = all_node_coords(dim, n).astype(np.float64) / n
    v = np.asarray(f(x), dtype=np.float64)
    return v if full else v[interior_mask(dim, n)]


def quadratic_potential(centre) -> Callable[[np.ndarray], np.ndarray]:
    """V(x) = |x - c|^2 (the confining potential of the uneven batch)."""
    c = np.asarray(centre, dtype=np.float64)
    return lambda x: np.sum((x - c[None, :]) ** 2, axis=1)


def example2_tensor(x: np.ndarray) -> np.ndarray:
    """The diffusion tensor of the second example (Section 5.2):
    A(x) = I + (x - 1/2)(x - 1/2)^T, for points x (E, 3)."""
    y = x - 0.5
    return np.eye(x.shape[1])[None] + y[:, :, None] * y[:, None, :]


def example2_potential(x: np.ndarray) -> np.ndarray:
    """The zeroth-order coefficient of the second example:
    phi(x) = exp((x1 - 1/2)(x2 - 1/2)(x3 - 1/2))."""
    return np.exp(np.prod(x - 0.5, axis=1))

