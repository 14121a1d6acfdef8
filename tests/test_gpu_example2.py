"""GPU parity of the general 3D operator: the second example of Section 5,
-div(A grad u) + phi u = lambda u on the unit cube with
A = I + (x - 1/2)(x - 1/2)^T and phi = exp(prod (x_i - 1/2)) at element
centroids (and 3D per-element kappa through the same 15-point path).

The library assembles the fine 15-point stencil and its Galerkin levels on
the host and runs unfused 15-point kernels; every level's operator, V-cycles
(Jacobi, Chebyshev, CG), one correction step and whole solves are compared
with the oracle (element-by-element sparse assembly, Galerkin products)."""
import sys

import numpy as np
import pytest

import paper_1908_10251_amd as P
import workloads as W
from oracle import fem, pasm as O
from oracle.multigrid import Hierarchy, MGOptions, default_options

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _ex2(nf):
    ten, phi = W.example2_elements(nf)
    A, M = fem.assemble(3, nf, tensor=fem.example2_tensor, potential=fem.example2_potential)
    return ten, phi, A, M


SM = {"jacobi": P.PASM_JACOBI, "cheb": P.PASM_CHEBYSHEV, "cg": P.PASM_CG}


@pytest.mark.parametrize("nc,nf", [(4, 16), (4, 32)])
def test_example2_operator_every_level(nc, nf):
    _say(f"example 2 operators H=1/{nc} h=1/{nf}")
    ten, phi, A, M = _ex2(nf)
    hier = Hierarchy(3, A, nc, nf)
    k = 2
    with P.Solver(3, 1 / nc, 1 / nf, k, tensor=ten, potential=phi, opts=P.options()) as s:
        assert P.pasm_num_levels(s.ctx) == len(hier.levels)
        rng = np.random.default_rng(4)
        for l, lv in enumerate(hier.levels):
            x = rng.standard_normal((k, lv.A.shape[0]))
            y = torch.zeros(k, lv.A.shape[0], dtype=torch.float64, device="cuda")
            P.pasm_apply_operator(s.ctx, l, P.PASM_OP_STIFFNESS, _t(x), y)
            ref = (lv.A @ x.T).T
            err = np.max(np.abs(y.cpu().numpy() - ref)) / np.max(np.abs(ref))
            _say(f"  level {l}: {err:.2e}")
            assert err < 1e-13, (l, err)
        x = rng.standard_normal((k, M.shape[0]))
        y = torch.zeros_like(_t(x))
        P.pasm_apply_operator(s.ctx, len(hier.levels) - 1, P.PASM_OP_MASS, _t(x), y)
        assert np.max(np.abs(y.cpu().numpy() - (M @ x.T).T)) / np.max(np.abs((M @ x.T).T)) < 1e-14


@pytest.mark.parametrize("smoother,nu", [("jacobi", 2), ("cheb", 2), ("cg", 2)])
@pytest.mark.parametrize("precision", [P.PASM_FP64, P.PASM_MIXED])
def test_example2_vcycle_matches_oracle(smoother, nu, precision):
    nc, nf = 4, 32
    _say(f"example 2 vcycle {smoother} nu={nu} prec={precision}")
    ten, phi, A, _ = _ex2(nf)
    hier = Hierarchy(3, A, nc, nf)
    opts = MGOptions("cg", nu, nu, vcycles=1) if smoother == "cg" else default_options(3, smoother, nu, nu, 1)
    k = 2
    rng = np.random.default_rng(6)
    N = A.shape[0]
    f = rng.standard_normal((k, N))
    x0 = rng.standard_normal((k, N))
    o = P.options(precision=precision, smoother=SM[smoother], nu_pre=nu, nu_post=nu, vcycles=1)
    with P.Solver(3, 1 / nc, 1 / nf, k, tensor=ten, potential=phi, opts=o) as s:
        for ncyc in (1, 2):
            xg = _t(x0)
            P.pasm_vcycle(s.ctx, _t(f), xg, ncyc)
            xg = xg.cpu().numpy()
            for r in range(k):
                xr = x0[r].copy()
                for _ in range(ncyc):
                    xr = hier.vcycle(len(hier.levels) - 1, xr, f[r], opts)
                err = np.max(np.abs(xg[r] - xr)) / np.max(np.abs(xr))
                tol = 1e-12 * (nf / 64) ** 2 if precision == P.PASM_FP64 else 2e-5
                tol = max(tol, 1e-12)
                _say(f"  ncyc={ncyc} rhs={r} err={err:.2e} tol={tol:.1e}")
                assert err < tol


# FP64: the oracle's step to rounding.  Mixed: the V-cycle runs in FP32 on
# FP64 residuals and its correction is added in FP64 inside the border pass;
# against the FP64 step, 1e-8 on lambda and 1e-6 on u, beta and zeta.
@pytest.mark.parametrize("precision,lam_tol,tol", [(P.PASM_FP64, 1e-11, 1e-8), (P.PASM_MIXED, 1e-8, 1e-6)])
@pytest.mark.parametrize("nf,k", [(32, 4), (64, 6)])
def test_example2_one_step_matches_oracle(precision, lam_tol, tol, nf, k):
    nc = 4
    _say(f"example 2 one correction step H=1/{nc} h=1/{nf} k={k} (CG(2) V-cycle) prec={precision}")
    ten, phi, _, _ = _ex2(nf)
    prob = O.make_problem(3, nc, nf, tensor=fem.example2_tensor, potential=fem.example2_potential)
    lam0, U0, _, _ = O.coarse_start(prob, k)
    bvp = O.MultigridBVP(prob, MGOptions("cg", 2, 2, vcycles=1))
    o = P.options(precision=precision, smoother=P.PASM_CG, nu_pre=2, nu_post=2, vcycles=1)
    with P.Solver(3, 1 / nc, 1 / nf, k, tensor=ten, potential=phi, opts=o) as s:
        theta, _ = P.pasm_coarse_eigenpairs(s.ctx)
        assert np.max(np.abs(theta[:k] - lam0) / lam0) < 1e-12
        P.pasm_set_state(s.ctx, lam0, U0)
        s.iterate()
        lam, U = s.eigenpairs()
        bz, _, _ = P.pasm_last_borders(s.ctx, k)
    btol = 1e-11 if precision == P.PASM_FP64 else tol
    for i in range(k):
        ref = O.correction_step(prob, lam0[i], U0[i], bvp)
        eu = np.max(np.abs(U[i] - ref["u"])) / np.max(np.abs(ref["u"]))
        _say(f"  pair {i}: lambda {abs(lam[i] - ref['lam']) / ref['lam']:.1e} u {eu:.1e} "
             f"beta {abs(bz[i, 0] / ref['beta'] - 1):.1e} zeta {abs(bz[i, 1] / ref['zeta'] - 1):.1e}")
        assert bz[i, 0] == pytest.approx(ref["beta"], rel=btol)
        assert bz[i, 1] == pytest.approx(ref["zeta"], rel=btol)
        assert abs(lam[i] - ref["lam"]) / ref["lam"] < lam_tol, (i, lam[i], ref["lam"])
        assert eu < tol


@pytest.mark.parametrize("smoother,precision", [("cg", P.PASM_FP64), ("jacobi", P.PASM_FP64),
                                                ("cg", P.PASM_MIXED)])
def test_example2_solve_reaches_discrete_eigenvalues(smoother, precision):
    nc, nf, k = 4, 16, 4
    _say(f"example 2 solve H=1/{nc} h=1/{nf} k={k} {smoother} prec={precision}")
    ten, phi, A, M = _ex2(nf)
    w, _ = O.discrete_eigenpairs(A, M, k + 2)
    o = P.options(precision=precision, smoother=SM[smoother], nu_pre=2, nu_post=2, vcycles=1 if smoother == "cg" else 2,
                  tol=1e-12, max_iter=80)
    with P.Solver(3, 1 / nc, 1 / nf, k, tensor=ten, potential=phi, opts=o) as s:
        its = s.solve(allow_notconv=True)
        lam, U = s.eigenpairs()
    # the cube's axis permutations keep exact multiplicities: sorted lists
    err = np.max(np.abs(np.sort(lam) - w[:k]) / w[:k])
    _say(f"  {its} steps, max rel err {err:.2e}")
    assert err < (1e-10 if precision == P.PASM_FP64 else 1e-8)
    for i in range(k):
        assert U[i] @ (M @ U[i]) == pytest.approx(1.0, abs=1e-10)


def test_kappa_3d_through_the_general_operator():
    nc, nf, k = 4, 16, 2
    _say("3D per-element kappa, lowest eigenpairs")
    kap = W.lognormal_kappa(3, nf, seed=5, sigma=0.5)
    A, M = fem.assemble(3, nf, kappa=kap)
    w, _ = O.discrete_eigenpairs(A, M, k)
    o = P.options(smoother=P.PASM_JACOBI, nu_pre=2, nu_post=2, vcycles=2, tol=1e-12, max_iter=80)
    with P.Solver(3, 1 / nc, 1 / nf, k, kappa=kap, opts=o) as s:
        s.solve(allow_notconv=True)
        lam, _ = s.eigenpairs(False)
    assert abs(lam[0] - w[0]) / w[0] < 1e-10
