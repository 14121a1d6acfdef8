"""GPU parity of the paper's multigrid step: V-cycles with conjugate-gradient
pre- and post-smoothing (PASM_CG; Section 5 uses one V-cycle with 2 CG steps
on each side), against the oracle's CG-smoothed V-cycle.

CG is not a fixed polynomial: its step lengths are ratios of inner products
over the whole level.  The library forms them from workgroup partial sums
added in a fixed order, the oracle with NumPy's sums; the two agree to
rounding, which the coarse-grid correction amplifies like the other FP64
V-cycles (the bound grows with (n/64)^2 from 1e-12), and FP32 cycles to 2e-5.
Whole solves with this smoother must reach the discrete eigenpairs."""
import sys

import numpy as np
import pytest

import paper_1908_10251_amd as P
from oracle import fem, pasm as O
from oracle.multigrid import Hierarchy, MGOptions
from workloads import lognormal_kappa, quadratic_potential_elements

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _opts(nu=2, vcycles=1, precision=P.PASM_FP64, tol=1e-10, max_iter=60):
    return P.options(precision=precision, smoother=P.PASM_CG, nu_pre=nu, nu_post=nu, vcycles=vcycles, tol=tol,
                     max_iter=max_iter)


VC = [
    # dim, nc, nf, kappa sigma, potential scale
    (2, 8, 64, None, 0.0),
    (2, 4, 64, 1.0, 0.0),
    (2, 32, 512, None, 0.0),
    (2, 4, 64, 0.5, 300.0),
    (3, 4, 16, None, 0.0),
    (3, 4, 32, None, 0.0),
]


@pytest.mark.parametrize("dim,nc,nf,sig,vscale", VC)
@pytest.mark.parametrize("precision", [P.PASM_FP64, P.PASM_MIXED])
@pytest.mark.parametrize("nu", [1, 2])
def test_cg_vcycle_matches_oracle(dim, nc, nf, sig, vscale, precision, nu):
    _say(f"CG vcycle dim={dim} H=1/{nc} h=1/{nf} sigma={sig} V={vscale} prec={precision} nu={nu}")
    kap = None if sig is None else lognormal_kappa(dim, nf, seed=13, sigma=sig)
    vel = vfn = None
    if vscale:
        c = (0.4, 0.3)
        vel = quadratic_potential_elements(nf, c, vscale)
        vfn = lambda x: vscale * fem.quadratic_potential(c)(x)  # noqa: E731
    A, _ = fem.assemble(dim, nf, kappa=kap, potential=vfn)
    hier = Hierarchy(dim, A, nc, nf)
    opts = MGOptions("cg", nu, nu, vcycles=1)
    k = 2
    rng = np.random.default_rng(17)
    N = A.shape[0]
    f = rng.standard_normal((k, N))
    x0 = rng.standard_normal((k, N))
    with P.Solver(dim, 1 / nc, 1 / nf, k, kappa=kap, potential=vel, opts=_opts(nu, precision=precision)) as s:
        for ncyc in (1, 2):
            xg = _t(x0)
            P.pasm_vcycle(s.ctx, _t(f), xg, ncyc)
            xg = xg.cpu().numpy()
            for r in range(k):
                xr = x0[r].copy()
                for _ in range(ncyc):
                    xr = hier.vcycle(len(hier.levels) - 1, xr, f[r], opts)
                err = np.max(np.abs(xg[r] - xr)) / np.max(np.abs(xr))
                tol = 1e-12 * max(1.0, (nf / 64) ** 2) if precision == P.PASM_FP64 else 2e-5
                _say(f"  ncyc={ncyc} rhs={r} err={err:.2e} tol={tol:.1e}")
                assert err < tol, (ncyc, r, err)


def test_cg_vcycle_from_an_exact_solution_stays_there():
    # f = A x*: the residual of x* is rounding only and CG's steps must not
    # blow it up (zero denominators give zero steps)
    _say("CG vcycle at an exact solution")
    A, _ = fem.assemble(2, 64)
    rng = np.random.default_rng(19)
    xs = rng.standard_normal((1, A.shape[0]))
    f = (A @ xs.T).T
    with P.Solver(2, 1 / 8, 1 / 64, 1, opts=_opts(2)) as s:
        xg = _t(xs)
        P.pasm_vcycle(s.ctx, _t(f), xg, 1)
        d = np.max(np.abs(xg.cpu().numpy() - xs)) / np.max(np.abs(xs))
    assert d < 1e-12


def test_one_correction_step_with_the_papers_multigrid_step():
    # Algorithm 1 with one V-cycle of CG(2) smoothing, from identical states
    nc, nf, k = 8, 256, 4
    _say(f"one step, CG(2) V-cycle, H=1/{nc} h=1/{nf}")
    prob = O.make_problem(2, nc, nf)
    lam0, U0, _, _ = O.coarse_start(prob, k)
    bvp = O.MultigridBVP(prob, MGOptions("cg", 2, 2, vcycles=1))
    with P.Solver(2, 1 / nc, 1 / nf, k, opts=_opts(2)) as s:
        P.pasm_set_state(s.ctx, lam0, U0)
        s.iterate()
        lam, U = s.eigenpairs()
    for i in range(k):
        ref = O.correction_step(prob, lam0[i], U0[i], bvp)
        assert abs(lam[i] - ref["lam"]) / ref["lam"] < 1e-11, (i, lam[i], ref["lam"])
        assert np.max(np.abs(U[i] - ref["u"])) / np.max(np.abs(ref["u"])) < 1e-8


@pytest.mark.parametrize("dim,nc,nf,k,precision", [(2, 8, 64, 4, P.PASM_FP64), (2, 8, 64, 4, P.PASM_MIXED),
                                                   (3, 4, 16, 1, P.PASM_FP64), (2, 8, 256, 4, P.PASM_FP64)])
def test_cg_solve_reaches_discrete_eigenpairs(dim, nc, nf, k, precision):
    _say(f"CG solve dim={dim} H=1/{nc} h=1/{nf} k={k} prec={precision}")
    prob = O.make_problem(dim, nc, nf)
    w, _ = O.discrete_eigenpairs(prob.A, prob.M, k)
    with P.Solver(dim, 1 / nc, 1 / nf, k, opts=_opts(2, tol=1e-12, precision=precision)) as s:
        its = s.solve()
        lam, _ = s.eigenpairs(False)
    err = np.max(np.abs(lam - w) / w)
    _say(f"  {its} steps, max rel err {err:.2e}")
    assert err < (1e-10 if precision == P.PASM_FP64 else 1e-8)
