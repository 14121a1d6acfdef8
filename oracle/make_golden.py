"""Write the stored expected values under tests/golden/ (oracle only).

TEST INFRASTRUCTURE ONLY.  Everything here calls `oracle` and the seeded input
generators of `workloads`; nothing comes from the GPU library.

Files
-----
<name>.eigenvalues.txt
    the k (+2) smallest discrete eigenvalues of the P1 pencil (A_h, M_h)
    (Section 2, the discrete eigenproblem) from `discrete_eigenpairs` (dense
    LAPACK for small meshes, shift-invert Lanczos otherwise), 17 digits.
<name>.vectors.npz
    the same eigenpairs' vectors (M-normalised) at 256 seeded sample nodes
    (`workloads.sample_nodes(N, 256, seed=1)`): full vectors of 1M nodes are
    too large to store, and a cluster subspace is identified by its rows at
    enough nodes.
<name>.step1.npz, <name>.steps3.npz
    the first correction steps (Algorithm 1) of every process of Algorithm 2
    with h_1 = H, from the coarse start (theta_i, u_i = P q_i), with the
    workload's own V-cycles in FP64 (oracle.multigrid): per step and process
    lambda, the selected augmented index, its score, beta = a(u~, u~),
    zeta = b(u~, u~), u at 256 seeded sample nodes (seed 2) and max |u|.
    step1 files also hold the start itself (theta_i and the coarse vectors
    q_i), so that a test can hand the identical start to the library.

    python -m oracle.make_golden [target ...]

targets: eigenvalues, vectors, kappa-step1, batch-step1, cube-step1,
ex2-step1, laplace-steps3 (default: all).
"""
from __future__ import annotations

import dataclasses
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import fem  # noqa: E402
from oracle import pasm as O  # noqa: E402
from oracle.pasm import discrete_eigenpairs  # noqa: E402

GOLDEN = os.path.join(ROOT, "tests", "golden")
SAMPLES = 256


def golden_path(name: str, kind: str = "eigenvalues.txt") -> str:
    return os.path.join(GOLDEN, f"{name}.{kind}")


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
    print(f"{path}: {time.time() - t:.1f} s", flush=True)
    return path


def read(name: str) -> np.ndarray:
    return np.loadtxt(golden_path(name), comments="#")


def _meta(**kw) -> np.ndarray:
    return np.array(json.dumps(dict(kw, writer="oracle/make_golden.py")))


def write_vectors(w: W.Workload, extra: int = 2) -> str:
    """Discrete eigenvectors of a constant-coefficient workload at sample nodes."""
    t = time.time()
    A, M = fem.assemble(w.dim, w.n_fine)
    lam, V = discrete_eigenpairs(A, M, w.k + extra)
    sample = W.sample_nodes(A.shape[0], SAMPLES, seed=1)
    path = golden_path(w.name, "vectors.npz")
    np.savez_compressed(path, lam=lam, sample=sample, v_sample=V[sample, :].T.copy(),
                        v_max=np.max(np.abs(V), axis=0),
                        meta=_meta(what="discrete eigenpairs (Section 2) at sample nodes", workload=w.name,
                                   dim=w.dim, n_fine=w.n_fine, normalisation="u^T M u = 1, sign arbitrary"))
    print(f"{path}: {time.time() - t:.1f} s", flush=True)
    return path


def _steps(name, prob, wl: W.Workload, steps: int, workers: int, keep_start: bool, **meta) -> str:
    t = time.time()
    bvp = O.MultigridBVP(prob, O.mg_options_for(wl))
    N = prob.A.shape[0]
    sample = W.sample_nodes(N, SAMPLES, seed=2)
    rec = O.record_steps(prob, wl.k, bvp, steps, sample, workers=workers)
    if not keep_start:
        rec.pop("Q")
    kind = "step1.npz" if steps == 1 else f"steps{steps}.npz"
    path = golden_path(name, kind)
    np.savez_compressed(path, sample=sample, **rec,
                        meta=_meta(what=f"first {steps} correction steps (Algorithm 1) of Algorithm 2, h_1 = H, "
                                        f"from the coarse start, FP64 V-cycles of the workload", workload=name,
                                   dim=prob.dim, n_coarse=prob.n_coarse, n_fine=prob.n_fine, k=wl.k,
                                   smoother=wl.smoother, nu=[wl.nu_pre, wl.nu_post], vcycles=wl.vcycles, **meta))
    print(f"{path}: {time.time() - t:.1f} s", flush=True)
    return path


def write_kappa_step1(workers: int) -> str:
    wl = W.KAPPA2D_MIXED
    kap = W.lognormal_kappa(2, wl.n_fine, seed=wl.seed)
    prob = O.make_problem(2, wl.n_coarse, wl.n_fine, kappa=kap)
    return _steps(wl.name, prob, wl, 1, workers, True, kappa="lognormal sigma 1 seed 0")


def write_batch_step1(workers: int) -> str:
    wl = W.BATCH2D_UNEVEN
    pos, inst = W.batch_member_at(1024, seed=wl.seed)
    prob = O.make_problem(2, wl.n_coarse, inst.n_fine, kappa=inst.kappa, centre=inst.centre)
    return _steps(f"{wl.name}-member{pos}", prob, wl, 1, workers, True, member=pos,
                  centre=[float(c) for c in inst.centre])


def write_cube_step1(workers: int) -> str:
    wl = W.LAP3D
    prob = O.make_problem(3, wl.n_coarse, wl.n_fine)
    return _steps(wl.name, prob, wl, 1, workers, True)


EX2_PAIRS = 16  # processes recorded for the second example (of its 200)


def write_ex2_step1(workers: int) -> str:
    """The second example (full tensor and potential on the cube, the
    paper's CG(2) multigrid step): the first EX2_PAIRS processes' first
    step; each process is independent of the others."""
    wl = W.EX2_3D
    prob = O.make_problem(3, wl.n_coarse, wl.n_fine, tensor=fem.example2_tensor, potential=fem.example2_potential)
    sub = dataclasses.replace(wl, k=EX2_PAIRS)
    return _steps(wl.name, prob, sub, 1, workers, True, pairs_of=wl.k,
                  coefficients="A = I + (x-1/2)(x-1/2)^T, phi = exp(prod(x_i - 1/2)) at element centroids")


def write_laplace_steps3(workers: int) -> str:
    wl = W.LAP2D_LARGE_H64
    prob = O.make_problem(2, wl.n_coarse, wl.n_fine)
    return _steps(wl.name, prob, wl, 3, workers, False)


if __name__ == "__main__":
    targets = sys.argv[1:] or ["eigenvalues", "vectors", "kappa-step1", "batch-step1", "cube-step1",
                               "ex2-step1", "laplace-steps3"]
    workers = min(8, O.cpu_count())
    for tg in targets:
        if tg == "eigenvalues":
            for wl in (W.LAP2D_SMALL, W.LAP2D_LARGE):
                write(wl)
        elif tg == "vectors":
            write_vectors(W.LAP2D_LARGE)
        elif tg == "kappa-step1":
            write_kappa_step1(workers)
        elif tg == "batch-step1":
            write_batch_step1(workers)
        elif tg == "cube-step1":
            write_cube_step1(workers)
        elif tg == "ex2-step1":
            write_ex2_step1(workers)
        elif tg == "laplace-steps3":
            write_laplace_steps3(workers)
        else:
            raise SystemExit(f"unknown target {tg}")
