"""Operators of the uniform constant-coefficient meshes built from their
stencils instead of element by element, for fine grids where the oracle's
assembly loop takes minutes.  Pinned to the assembly at small sizes in
test_oracle_fem.py (the mesh is translation invariant, so the stencil of one
interior node fixes every row)."""
import numpy as np
import scipy.sparse as sp


def constant_stiffness_3d(n: int) -> sp.csr_matrix:
    """Interior stiffness of the Kuhn mesh with kappa = 1: h (6 at the centre,
    -1 at the six axis neighbours), nodes ordered x fastest."""
    m = n - 1
    h = 1.0 / n
    T = sp.diags([-np.ones(m - 1), 2.0 * np.ones(m), -np.ones(m - 1)], [-1, 0, 1])
    I = sp.identity(m)
    return (h * (sp.kron(sp.kron(I, I), T) + sp.kron(sp.kron(I, T), I) + sp.kron(sp.kron(T, I), I))).tocsr()
