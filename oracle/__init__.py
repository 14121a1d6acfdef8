"""Plain, slow, FP64 CPU oracle for the parallel augmented subspace method.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import anything from this package.  The GPU
library never calls it and shares no code with it.

Contents
--------
fem        P1 finite elements on the uniform Kuhn simplex mesh (2D "/" triangles,
           3D Kuhn tetrahedra): element-by-element assembly of the stiffness,
           mass and potential matrices (Section 2, the discrete eigenproblem).
transfer   nodal-interpolation prolongation between nested meshes and the
           Galerkin coarse operators (Section 3, the nested spaces V_H, V_{h_k}).
multigrid  the V-cycle used as "some multigrid steps" for the boundary value
           problem of Algorithm 1, step 1 (Jacobi / Chebyshev smoothing).
pasm       Algorithm 1 (one correction step) and Algorithm 2 (the parallel
           augmented subspace scheme), with the definition of the result
           (the discrete eigenpairs of the pencil) beside it.
learned    the learned convolutional smoother (not in the paper; an
           alternative smoother for the multigrid steps of Algorithm 1):
           forward map, training loss and its gradient, Adam update.

Every function states which part of the paper it follows.  Parity status of
every function is listed in its module header.
"""
