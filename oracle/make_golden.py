"""Write the stored expected values under tests/golden/ (oracle only).

TEST INFRASTRUCTURE ONLY.  Each file holds the k smallest discrete
eigenvalues of the P1 pencil (A_h, M_h) of one workload (Section 2, the
discrete eigenproblem), computed by `oracle.pasm.discrete_eigenpairs`
(dense LAPACK for small meshes, shift-invert Lanczos otherwise), one value per
line with 17 significant digits.

    python -m oracle.make_golden [name ...]
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import fem  # noqa: E402
from oracle.pasm import discrete_eigenpairs  # noqa: E402

GOLDEN = os.path.join(ROOT, "tests", "golden")


def golden_path(name: str) -> str:
    return os.path.join(GOLDEN, f"{name}.eigenvalues.txt")


def write(w: W.Workload, extra: int = 2) -> str:
    if w.kappa != "one" or w.potential != "none":
        raise ValueError("golden values are written for constant-coefficient workloads")
    t = time.time()
    A, M = fem.assemble(w.dim, w.n_fine)
    lam, _ = discrete_eigenpairs(A, M, w.k + extra)
    path = golden_path(w.name)
    with open(path, "w") as f:
        f.write(f"# {w.name}: {w.k + extra} smallest discrete eigenvalues of the P1 pencil\n")
        f.write(f"# dim={w.dim} h=1/{w.n_fine} interior dofs={A.shape[0]}; written by oracle/make_golden.py\n")
        for v in lam:
            f.write(f"{v:.17g}\n")
    print(f"{path}: {time.time() - t:.1f} s")
    return path


def read(name: str) -> np.ndarray:
    return np.loadtxt(golden_path(name), comments="#")


if __name__ == "__main__":
    names = sys.argv[1:] or [W.LAP2D_SMALL.name, W.LAP2D_LARGE.name]
    for wl in W.ALL:
        if wl.name in names:
            write(wl)
