"""Prolongation between nested Kuhn meshes and Galerkin coarse operators (oracle).

TEST INFRASTRUCTURE ONLY (see the package header).

Section 3 builds a nested family V_H (= V_{h_1}) in V_{h_2} in ... in V_{h_n}
by regular refinement with ratio beta (here beta = 2).  Because the spaces are
nested, a coarse P1 function is also a fine P1 function; its fine nodal values
are obtained by evaluating the coarse basis functions at the fine nodes.  This
module does exactly that by point location: the coarse simplex holding a fine
node is found from the sort order of the node's local cell coordinates (the
Kuhn simplex with permutation pi holds the points whose local coordinates are
ordered xi[pi0] >= xi[pi1] >= ...), and the barycentric weights are read off
that order.  No stencil formula is assumed.

The coarse matrices of the augmented problem (Section 3.1, the matrix form of
the small eigenproblem) are A_H = P^T A_h P and M_H = P^T M_h P with P the
composite prolongation; the multigrid hierarchy uses the same Galerkin rule.

Parity status: pinned (Galerkin products equal direct coarse assembly; the
interpolant of a coarse P1 function is reproduced; tests/test_oracle_transfer.py).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .fem import all_node_coords, interior_mask, node_ids


def prolongation(dim: int, n_coarse: int, n_fine: int, full: bool = False) -> sp.csr_matrix:
    """Matrix P with (P v_H)(fine node) = v_H(fine node) for v_H in V_H.

    n_fine must be a multiple of n_coarse.  With full=False, rows and columns
    are restricted to interior nodes (coarse boundary values are zero).
    """
    assert n_fine % n_coarse == 0
    xf = all_node_coords(dim, n_fine)                   # (Nf, d) integer coords
    t = xf * n_coarse                                   # position in units of 1/n_fine of coarse cells
    cell = np.minimum(t // n_fine, n_coarse - 1)        # coarse cell index per axis
    xi = (t - cell * n_fine).astype(np.float64) / n_fine  # local coordinates in [0, 1]
    order = np.argsort(-xi, axis=1, kind="stable")      # xi[pi0] >= xi[pi1] >= ...
    xs = np.take_along_axis(xi, order, axis=1)
    nf = xf.shape[0]
    rows, cols, vals = [], [], []
    vert = cell.copy()
    # vertex 0 = cell origin, weight 1 - xi[pi0]
    w = 1.0 - xs[:, 0]
    rows.append(np.arange(nf)); cols.append(node_ids(vert, n_coarse)); vals.append(w)
    for m in range(dim):
        step = np.zeros_like(vert)
        np.put_along_axis(step, order[:, m:m + 1], 1, axis=1)
        vert = vert + step
        w = xs[:, m] - (xs[:, m + 1] if m + 1 < dim else 0.0)
        rows.append(np.arange(nf)); cols.append(node_ids(vert, n_coarse)); vals.append(w)
    rows = np.concatenate(rows); cols = np.concatenate(cols); vals = np.concatenate(vals)
    nz = vals != 0.0
    P = sp.coo_matrix((vals[nz], (rows[nz], cols[nz])),
                      shape=(nf, (n_coarse + 1) ** dim)).tocsr()
    if full:
        return P
    keep_f = np.flatnonzero(interior_mask(dim, n_fine))
    keep_c = np.flatnonzero(interior_mask(dim, n_coarse))
    return P[keep_f][:, keep_c].tocsr()


def level_sizes(n_coarse: int, n_fine: int):
    """Cells per side of every level, coarse to fine, ratio 2 (Section 3)."""
    sizes = [n_coarse]
    while sizes[-1] < n_fine:
        sizes.append(sizes[-1] * 2)
    assert sizes[-1] == n_fine, "fine/coarse ratio must be a power of two"
    return sizes


def galerkin(P: sp.csr_matrix, A: sp.csr_matrix) -> sp.csr_matrix:
    """Coarse operator P^T A P."""
    return (P.T @ A @ P).tocsr()
