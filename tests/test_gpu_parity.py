"""GPU parity: the HIP library (through its C ABI) against the CPU oracle.

Operators and V-cycles element by element; one correction step (Algorithm 1)
from identical states; whole solves (Algorithm 2) against the discrete
eigenpairs.  Tolerances: FP64 paths 1e-12..1e-10 relative (rounding order
only), mixed-precision V-cycles 1e-5 relative per cycle (FP32 arithmetic on
FP64 residuals), eigenvalues of mixed solves 1e-8 relative."""
import sys

import numpy as np
import pytest

import paper_1908_10251_amd as P
from oracle import fem, pasm as O
from oracle.multigrid import Hierarchy, MGOptions, default_options
from workloads import lognormal_kappa, quadratic_potential_elements

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _opts(smoother="jacobi", nu=2, vcycles=2, precision=P.PASM_FP64, tol=1e-10, max_iter=60, fused=True,
          exhaustive=False):
    return P.options(precision=precision, smoother=P.PASM_CHEBYSHEV if smoother == "cheb" else P.PASM_JACOBI,
                     nu_pre=nu, nu_post=nu, vcycles=vcycles, tol=tol, max_iter=max_iter, fused=fused,
                     exhaustive=exhaustive)


# potential V = scale |x - c|^2 of the uneven batch, scaled up so that the
# mass-type term is a visible part of the operator
POT_CENTRE = (0.3, 0.6)
POT_SCALE = 400.0


def _potential(nf, pot):
    """(per-element values for the library, callable for the oracle) or Nones."""
    if not pot:
        return None, None
    return (quadratic_potential_elements(nf, POT_CENTRE, POT_SCALE),
            lambda x: POT_SCALE * fem.quadratic_potential(POT_CENTRE)(x))


CASES = [
    # dim, nc, nf, kappa-sigma (None: kappa = 1), potential
    (2, 8, 64, None, False),
    (2, 4, 32, 1.0, False),
    (3, 4, 16, None, False),
    (2, 4, 32, None, True),
    (2, 4, 32, 1.0, True),
]


@pytest.mark.parametrize("dim,nc,nf,sig,pot", CASES)
def test_operators_every_level(dim, nc, nf, sig, pot):
    _say(f"operators dim={dim} H=1/{nc} h=1/{nf} sigma={sig} potential={pot}")
    kap = None if sig is None else lognormal_kappa(dim, nf, seed=7, sigma=sig)
    vel, vfn = _potential(nf, pot)
    A, M = fem.assemble(dim, nf, kappa=kap, potential=vfn)
    hier = Hierarchy(dim, A, nc, nf)
    k = 3
    with P.Solver(dim, 1 / nc, 1 / nf, k, kappa=kap, potential=vel, opts=_opts()) as s:
        assert P.pasm_num_levels(s.ctx) == len(hier.levels)
        rng = np.random.default_rng(1)
        for l, lv in enumerate(hier.levels):
            N = lv.A.shape[0]
            x = rng.standard_normal((k, N))
            y = torch.zeros(k, N, dtype=torch.float64, device="cuda")
            P.pasm_apply_operator(s.ctx, l, P.PASM_OP_STIFFNESS, _t(x), y)
            ref = (lv.A @ x.T).T
            err = np.max(np.abs(y.cpu().numpy() - ref)) / np.max(np.abs(ref))
            assert err < 1e-13, (l, err)
        x = rng.standard_normal((k, M.shape[0]))
        y = torch.zeros_like(_t(x))
        P.pasm_apply_operator(s.ctx, len(hier.levels) - 1, P.PASM_OP_MASS, _t(x), y)
        ref = (M @ x.T).T
        assert np.max(np.abs(y.cpu().numpy() - ref)) / np.max(np.abs(ref)) < 1e-14


VC = [
    (2, 8, 64, None, "jacobi", 2, False),
    (2, 8, 64, None, "cheb", 4, False),
    (2, 4, 64, 1.0, "cheb", 4, False),
    (3, 4, 16, None, "jacobi", 2, False),
    # fine grids of 512 cells and more take the marching smoother with fused
    # transfers; 513 nodes per side leave ragged strips and segments
    (2, 32, 512, None, "cheb", 4, False),
    (2, 64, 512, None, "jacobi", 2, False),
    # odd step counts: strip halos rounded up to an even width
    (2, 32, 512, None, "jacobi", 3, False),
    # per-element kappa on marching levels (FP32 cycles take the edge-weight
    # marching smoother): ragged strips and bands, odd step counts
    (2, 32, 512, 1.0, "cheb", 4, False),
    (2, 16, 256, 1.0, "jacobi", 3, False),
    # general 7-point operators (potential term), Galerkin coarse levels
    (2, 4, 64, 1.0, "cheb", 4, True),
    (2, 8, 64, None, "jacobi", 2, True),
]


@pytest.mark.parametrize("dim,nc,nf,sig,smoother,nu,pot", VC)
@pytest.mark.parametrize("precision", [P.PASM_FP64, P.PASM_MIXED])
@pytest.mark.parametrize("fused", [True, False])
def test_vcycle_matches_oracle(dim, nc, nf, sig, smoother, nu, pot, precision, fused):
    _say(f"vcycle dim={dim} H=1/{nc} h=1/{nf} sigma={sig} {smoother} pot={pot} prec={precision} fused={fused}")
    kap = None if sig is None else lognormal_kappa(dim, nf, seed=3, sigma=sig)
    vel, vfn = _potential(nf, pot)
    A, _ = fem.assemble(dim, nf, kappa=kap, potential=vfn)
    hier = Hierarchy(dim, A, nc, nf)
    opts = default_options(dim, smoother, nu, nu, 1)
    k = 2
    rng = np.random.default_rng(2)
    N = A.shape[0]
    f = rng.standard_normal((k, N))
    x0 = rng.standard_normal((k, N))
    with P.Solver(dim, 1 / nc, 1 / nf, k, kappa=kap, potential=vel,
                  opts=_opts(smoother, nu, precision=precision, fused=fused)) as s:
        # host transfers of the state must leave the grids' zero boundary intact
        lam, U = s.eigenpairs()
        P.pasm_set_state(s.ctx, lam, U)
        for ncyc in (2, 1, 2):
            xg = _t(x0)
            P.pasm_vcycle(s.ctx, _t(f), xg, ncyc)
            xg = xg.cpu().numpy()
            for r in range(k):
                xr = x0[r].copy()
                for _ in range(ncyc):
                    xr = hier.vcycle(len(hier.levels) - 1, xr, f[r], opts)
                err = np.max(np.abs(xg[r] - xr)) / np.max(np.abs(xr))
                # rounding of the residuals is amplified by the coarse-grid
                # correction, up to cond(A_h) ~ h^-2: the FP64 bound grows
                # with (nf/64)^2 from 1e-12 at 64 cells
                tol = 1e-12 * max(1.0, (nf / 64) ** 2) if precision == P.PASM_FP64 else 2e-5
                _say(f"  ncyc={ncyc} rhs={r} err={err:.2e} tol={tol:.1e}")
                assert err < tol, (ncyc, r, err)


@pytest.mark.parametrize("precision", [P.PASM_FP64, P.PASM_MIXED])
def test_vcycle_kappa_2048_matches_oracle(precision):
    # the rough-coefficient workload's mesh and coefficient (4.2M nodes,
    # log kappa ~ N(0, 1) per element, H = 1/32, Chebyshev 4/4): one and two
    # V-cycles on one right-hand side against the oracle's
    nc, nf = 32, 2048
    _say(f"vcycle kappa h=1/{nf} H=1/{nc} cheb 4/4 prec={precision}")
    kap = lognormal_kappa(2, nf, seed=0, sigma=1.0)
    A, _ = fem.assemble(2, nf, kappa=kap)
    hier = Hierarchy(2, A, nc, nf)
    opts = default_options(2, "cheb", 4, 4, 1)
    rng = np.random.default_rng(8)
    N = A.shape[0]
    f = rng.standard_normal((1, N))
    x0 = rng.standard_normal((1, N))
    with P.Solver(2, 1 / nc, 1 / nf, 1, kappa=kap, opts=_opts("cheb", 4, precision=precision)) as s:
        for ncyc in (1, 2):
            xg = _t(x0)
            P.pasm_vcycle(s.ctx, _t(f), xg, ncyc)
            xg = xg.cpu().numpy()[0]
            xr = x0[0].copy()
            for _ in range(ncyc):
                xr = hier.vcycle(len(hier.levels) - 1, xr, f[0], opts)
            err = np.max(np.abs(xg - xr)) / np.max(np.abs(xr))
            tol = 1e-12 * (nf / 64) ** 2 if precision == P.PASM_FP64 else 2e-5
            _say(f"  ncyc={ncyc} err={err:.2e} tol={tol:.1e}")
            assert err < tol


@pytest.mark.parametrize("smoother,nu", [("cheb", 4), ("jacobi", 3), ("cheb", 2), ("jacobi", 1)])
def test_vcycle_kappa_odd_rhs_count_matches_oracle(smoother, nu):
    # FP32 cycles on edge-weight levels march two right-hand sides per
    # wavefront: three right-hand sides leave a ragged last pair, and every
    # step count has its own kernel.  Each right-hand side against the
    # oracle's V-cycle, and the first one against a context of one
    # right-hand side (a partner must not leak into it).
    nc, nf, k = 8, 512, 3
    _say(f"vcycle kappa h=1/{nf} k={k} {smoother} nu={nu} mixed")
    kap = lognormal_kappa(2, nf, seed=21, sigma=1.0)
    A, _ = fem.assemble(2, nf, kappa=kap)
    hier = Hierarchy(2, A, nc, nf)
    opts = default_options(2, smoother, nu, nu, 1)
    rng = np.random.default_rng(23)
    N = A.shape[0]
    f = rng.standard_normal((k, N))
    x0 = rng.standard_normal((k, N))
    o = _opts(smoother, nu, precision=P.PASM_MIXED)
    with P.Solver(2, 1 / nc, 1 / nf, k, kappa=kap, opts=o) as s:
        xg = _t(x0)
        P.pasm_vcycle(s.ctx, _t(f), xg, 2)
        xg = xg.cpu().numpy()
    with P.Solver(2, 1 / nc, 1 / nf, 1, kappa=kap, opts=o) as s1:
        x1 = _t(x0[:1])
        P.pasm_vcycle(s1.ctx, _t(f[:1]), x1, 2)
        x1 = x1.cpu().numpy()[0]
    for r in range(k):
        xr = x0[r].copy()
        for _ in range(2):
            xr = hier.vcycle(len(hier.levels) - 1, xr, f[r], opts)
        err = np.max(np.abs(xg[r] - xr)) / np.max(np.abs(xr))
        _say(f"  rhs={r} err={err:.2e}")
        assert err < 2e-5, (r, err)
    d = np.max(np.abs(xg[0] - x1)) / np.max(np.abs(x1))
    _say(f"  rhs 0 alone vs with partners: {d:.2e}")
    assert d < 1e-6


@pytest.mark.parametrize("smoother,nu", [("cheb", 4), ("jacobi", 2), ("cheb", 1)])
def test_vcycle_kappa_potential_odd_rhs_count_matches_oracle(smoother, nu):
    # kappa and a potential: the general 7-point operator (its diagonal and
    # the "/" diagonal couplings streamed with the edge weights) marches in
    # FP32 on the levels of 256 cells and more; three right-hand sides leave
    # a ragged last pair.  Each right-hand side against the oracle's V-cycle.
    nc, nf, k = 8, 512, 3
    _say(f"vcycle kappa + potential h=1/{nf} k={k} {smoother} nu={nu} mixed")
    kap = lognormal_kappa(2, nf, seed=31, sigma=1.0)
    vel, vfn = _potential(nf, True)
    A, _ = fem.assemble(2, nf, kappa=kap, potential=vfn)
    hier = Hierarchy(2, A, nc, nf)
    opts = default_options(2, smoother, nu, nu, 1)
    rng = np.random.default_rng(33)
    N = A.shape[0]
    f = rng.standard_normal((k, N))
    x0 = rng.standard_normal((k, N))
    o = _opts(smoother, nu, precision=P.PASM_MIXED)
    with P.Solver(2, 1 / nc, 1 / nf, k, kappa=kap, potential=vel, opts=o) as s:
        xg = _t(x0)
        P.pasm_vcycle(s.ctx, _t(f), xg, 2)
        xg = xg.cpu().numpy()
    for r in range(k):
        xr = x0[r].copy()
        for _ in range(2):
            xr = hier.vcycle(len(hier.levels) - 1, xr, f[r], opts)
        err = np.max(np.abs(xg[r] - xr)) / np.max(np.abs(xr))
        _say(f"  rhs={r} err={err:.2e}")
        assert err < 2e-5, (r, err)


@pytest.mark.parametrize("nf,smoother,pre,post", [(256, "cheb", 4, 4), (512, "jacobi", 2, 2), (256, "cheb", 3, 1),
                                                  (512, "cheb", 1, 4), (256, "jacobi", 1, 1), (512, "jacobi", 3, 3)])
def test_paired_smoothing_phases_equal_single_cycles(nf, smoother, pre, post):
    # cycles in a row run the finest post-smoothing of one cycle and the
    # pre-smoothing of the next in one pass; one cycle per call runs them as
    # two passes: the same arithmetic (the two kernels may contract different
    # products into fused multiply-adds, so equal to rounding).  Odd step
    # counts and reflected bands whose last row carries a coarse node are
    # among the cases.
    _say(f"paired phases h=1/{nf} {smoother} pre={pre} post={post}")
    nc, k = 8, 3
    rng = np.random.default_rng(5)
    o = P.options(smoother=P.PASM_CHEBYSHEV if smoother == "cheb" else P.PASM_JACOBI, nu_pre=pre, nu_post=post)
    with P.Solver(2, 1 / nc, 1 / nf, k, opts=o) as s:
        N = P.pasm_num_dofs(s.ctx)
        f = _t(rng.standard_normal((k, N)))
        x0 = rng.standard_normal((k, N))
        xa = _t(x0)
        P.pasm_vcycle(s.ctx, f, xa, 3)
        xb = _t(x0)
        for _ in range(3):
            P.pasm_vcycle(s.ctx, f, xb, 1)
        rel = float(torch.max(torch.abs(xa - xb)) / torch.max(torch.abs(xb)))
        _say(f"  paired vs single cycles: {rel:.2e}")
        assert rel < 1e-13
        assert float(torch.max(torch.abs(xa - _t(x0)))) > 0.0


_HIER_3D = {}


def _hier_3d(nc, nf):
    # stiffness from its stencil (pinned to the assembly in test_oracle_fem.py):
    # assembling 128^3 element by element takes minutes
    if (nc, nf) not in _HIER_3D:
        from stencil_ops import constant_stiffness_3d
        _HIER_3D[(nc, nf)] = Hierarchy(3, constant_stiffness_3d(nf), nc, nf)
    return _HIER_3D[(nc, nf)]


@pytest.mark.parametrize("smoother,nu", [("jacobi", 2), ("cheb", 2), ("jacobi", 1)])
@pytest.mark.parametrize("precision", [P.PASM_FP64, P.PASM_MIXED])
@pytest.mark.parametrize("fused", [True, False])
def test_vcycle_3d_128_matches_oracle(smoother, nu, precision, fused):
    # 128 cells per side: with fusion the finest level takes the marching
    # smoother (slabs of 32 rows overlapping by 2 nu, 127 rows leave a ragged
    # last slab); FP64 V-cycles start from a nonzero x, mixed ones from 0
    nc, nf, k = 8, 128, 2
    _say(f"vcycle 3d H=1/{nc} h=1/{nf} {smoother} nu={nu} prec={precision} fused={fused}")
    hier = _hier_3d(nc, nf)
    opts = default_options(3, smoother, nu, nu, 1)
    rng = np.random.default_rng(11)
    N = hier.levels[-1].A.shape[0]
    f = rng.standard_normal((k, N))
    x0 = rng.standard_normal((k, N))
    with P.Solver(3, 1 / nc, 1 / nf, k, opts=_opts(smoother, nu, precision=precision, fused=fused)) as s:
        for ncyc in (2, 1):
            xg = _t(x0)
            P.pasm_vcycle(s.ctx, _t(f), xg, ncyc)
            xg = xg.cpu().numpy()
            for r in range(k):
                xr = x0[r].copy()
                for _ in range(ncyc):
                    xr = hier.vcycle(len(hier.levels) - 1, xr, f[r], opts)
                err = np.max(np.abs(xg[r] - xr)) / np.max(np.abs(xr))
                tol = 1e-12 * (nf / 64) ** 2 if precision == P.PASM_FP64 else 2e-5
                _say(f"  ncyc={ncyc} rhs={r} err={err:.2e} tol={tol:.1e}")
                assert err < tol, (ncyc, r, err)


def _clusters(vals, rtol=1e-10):
    out, cur = [], [0]
    for i in range(1, len(vals)):
        if abs(vals[i] - vals[cur[-1]]) <= rtol * abs(vals[i]):
            cur.append(i)
        else:
            out.append(cur)
            cur = [i]
    out.append(cur)
    return out


ONE_STEP = [
    (2, 8, 64, None, "jacobi", 2, 4, False),
    (2, 8, 64, None, "cheb", 4, 4, False),
    (2, 4, 32, 0.5, "cheb", 4, 2, False),
    (3, 4, 16, None, "jacobi", 2, 4, False),
    (2, 8, 64, 0.5, "cheb", 4, 3, True),
]


# Larger grids for the paths that only they take: a finest level of 512
# (marching smoother; in FP64 the last post-smoothing also forms the borders)
# and a coarse space of 3969 (dense coarse products on the FP64 matrix cores).
ONE_STEP_LARGE = [
    (2, 16, 512, None, "cheb", 4, 3, False),
    (2, 64, 128, None, "cheb", 4, 2, False),
]


@pytest.mark.parametrize("dim,nc,nf,sig,smoother,nu,k,pot", ONE_STEP)
@pytest.mark.parametrize("exhaustive", [False, True])
def test_one_correction_step_matches_oracle(dim, nc, nf, sig, smoother, nu, k, pot, exhaustive):
    """Algorithm 1 from the same state: the coarse start, then a perturbed state."""
    _one_step_check(dim, nc, nf, sig, smoother, nu, k, pot, exhaustive, perturbed=True)


@pytest.mark.parametrize("dim,nc,nf,sig,smoother,nu,k,pot", ONE_STEP_LARGE)
def test_one_correction_step_large_matches_oracle(dim, nc, nf, sig, smoother, nu, k, pot):
    """As above from the coarse start (the oracle's dense pencils of order
    N_H + 1 make the perturbed state too slow at N_H = 3969)."""
    _one_step_check(dim, nc, nf, sig, smoother, nu, k, pot, False, perturbed=nc < 64)


def _one_step_check(dim, nc, nf, sig, smoother, nu, k, pot, exhaustive, perturbed):
    _say(f"one step dim={dim} H=1/{nc} h=1/{nf} sigma={sig} {smoother} k={k} pot={pot} exhaustive={exhaustive}")
    kap = None if sig is None else lognormal_kappa(dim, nf, seed=5, sigma=sig)
    vel, _ = _potential(nf, pot)
    prob = O.make_problem(dim, nc, nf, kappa=kap)
    if pot:
        # the oracle's problem with the same scaled potential
        A, M = fem.assemble(dim, nf, kappa=kap, potential=_potential(nf, pot)[1])
        prob = O.Problem(dim, nc, nf, A, M, prob.P, (prob.P.T @ A @ prob.P).toarray(), prob.MH)
    bvp = O.MultigridBVP(prob, default_options(dim, smoother, nu, nu, 2))
    lam0, U0, _, _ = O.coarse_start(prob, k)
    rng = np.random.default_rng(4)
    U1 = U0 + 0.05 * rng.standard_normal(U0.shape) * np.max(np.abs(U0))
    lam1 = np.array([(u @ prob.A @ u) / (u @ prob.M @ u) for u in U1])
    # the coarse pencil's rounding (two different dense eigensolvers) grows
    # with its condition, which scales as H^-2
    cs = max(1.0, (nc / 8) ** 2)
    with P.Solver(dim, 1 / nc, 1 / nf, k, kappa=kap, potential=vel, opts=_opts(smoother, nu, exhaustive=exhaustive)) as s:
        states = ((lam0, U0, True), (lam1, U1, False)) if perturbed else ((lam0, U0, True),)
        for lam_in, U_in, from_setup in states:
            if not from_setup:
                P.pasm_set_state(s.ctx, lam_in, U_in)
            else:
                lg, Ug = P.pasm_eigenpairs(s.ctx, k)
                assert np.max(np.abs(lg - lam0) / lam0) < 1e-13 * cs
                # start vectors: equal up to sign, or the same subspace inside a
                # cluster of equal coarse eigenvalues (any basis is valid there)
                for grp in _clusters(lam0):
                    if len(grp) == 1:
                        i = grp[0]
                        ui = Ug[i] if Ug[i] @ U0[i] >= 0 else -Ug[i]
                        assert np.max(np.abs(ui - U0[i])) < 1e-11 * cs * np.max(np.abs(U0[i]))
                    else:
                        Qa, _ = np.linalg.qr(U0[grp].T)
                        Qb, _ = np.linalg.qr(Ug[grp].T)
                        assert np.min(np.linalg.svd(Qa.T @ Qb, compute_uv=False)) > 1 - 1e-12 * cs
                U_in = Ug
            s.iterate()
            lg, Ug = P.pasm_eigenpairs(s.ctx, k)
            rank, score, flags = P.pasm_last_selection(s.ctx, k)
            theta, Qg = P.pasm_coarse_eigenpairs(s.ctx)
            bz, pg, qg = P.pasm_last_borders(s.ctx, k)
            assert np.max(np.abs(theta - O.coarse_start(prob, k)[2]) / theta) < 1e-12 * cs
            assert np.max(np.abs(Qg.T @ prob.MH @ Qg - np.eye(len(theta)))) < 1e-11 * cs
            for i in range(k):
                ref = O.correction_step(prob, lam_in[i], U_in[i], bvp)
                assert bz[i, 0] == pytest.approx(ref["beta"], rel=1e-11), (i, bz[i], ref["beta"], ref["zeta"])
                assert bz[i, 1] == pytest.approx(ref["zeta"], rel=1e-11), (i, bz[i], ref["beta"], ref["zeta"])
                np.testing.assert_allclose(pg[i], Qg.T @ ref["b"], rtol=0, atol=1e-10 * np.max(np.abs(pg[i])))
                np.testing.assert_allclose(qg[i], Qg.T @ ref["c"], rtol=0, atol=1e-10 * np.max(np.abs(qg[i])))
                # the arrowhead reduction of the same borders, solved densely
                zp = bz[i, 1] - qg[i] @ qg[i]
                gv = (pg[i] - theta * qg[i]) / np.sqrt(zp)
                rho = (bz[i, 0] - 2 * qg[i] @ pg[i] + qg[i] @ (theta * qg[i])) / zp
                Ar = np.diag(np.concatenate([theta, [rho]]))
                Ar[:-1, -1] = gv
                Ar[-1, :-1] = gv
                wa, Va = np.linalg.eigh(Ar)
                ja = int(np.argmax(np.abs(Va[:-1].T @ qg[i] + Va[-1] * np.sqrt(zp))))
                assert abs(lg[i] - wa[ja]) / wa[ja] < 1e-11, (i, lg[i], wa[ja], ref["lam"])
                assert abs(lg[i] - ref["lam"]) / ref["lam"] < 1e-11, (i, lg[i], ref["lam"])
                assert rank[i] == ref["index"], (i, rank[i], ref["index"])
                assert score[i] == pytest.approx(ref["score"], rel=1e-8)
                d = np.max(np.abs(Ug[i] - ref["u"])) / np.max(np.abs(ref["u"]))
                assert d < 1e-8, (i, d)


def _mnorm_dist(u, v, M):
    v = v if u @ (M @ v) >= 0 else -v
    d = u - v
    return float(np.sqrt(d @ (M @ d)))


@pytest.mark.parametrize("precision", [P.PASM_FP64, P.PASM_MIXED])
def test_small_laplace_solve_matches_discrete_eigenpairs(precision):
    """The 2D workload H = 1/8, h = 1/64, k = 4, Jacobi 2/2, 2 V-cycles."""
    _say(f"solve lap2d H=1/8 h=1/64 k=4 prec={precision}")
    prob = O.make_problem(2, 8, 64)
    w, V = O.discrete_eigenpairs(prob.A, prob.M, 4)
    with P.Solver(2, 1 / 8, 1 / 64, 4, opts=_opts("jacobi", 2, precision=precision, tol=1e-12)) as s:
        its = s.solve()
        lam, U = s.eigenpairs()
    assert its <= 20
    tol = 1e-10 if precision == P.PASM_FP64 else 1e-8
    assert np.max(np.abs(lam - w) / w) < tol
    for i in range(4):
        assert _mnorm_dist(U[i], V[:, i], prob.M) < 1e-6
        assert U[i] @ prob.M @ U[i] == pytest.approx(1.0, abs=1e-10)


def test_small_laplace_iteration_history_matches_oracle():
    """Same trajectory as the oracle's Algorithm 2 with the same V-cycles."""
    _say("history lap2d H=1/8 h=1/64 k=4")
    prob = O.make_problem(2, 8, 64)
    bvp = O.MultigridBVP(prob, default_options(2, "jacobi", 2, 2, 2))
    ref = O.solve(prob, 4, bvp, tol=1e-10)
    with P.Solver(2, 1 / 8, 1 / 64, 4, opts=_opts("jacobi", 2, tol=1e-10)) as s:
        hist = [s.eigenpairs(False)[0]]
        for _ in range(max(len(h) for h in ref["hist"]) - 1):
            s.iterate()
            hist.append(s.eigenpairs(False)[0])
    for i in range(4):
        for t, lr in enumerate(ref["hist"][i]):
            assert abs(hist[t][i] - lr) / lr < 1e-10, (i, t)


@pytest.mark.parametrize("nc,nf,smoother,nu", [(8, 64, "cheb", 4), (8, 256, "cheb", 4), (16, 512, "jacobi", 2),
                                               (8, 256, "jacobi", 1)])
def test_iterate_n_equals_single_steps(nc, nf, smoother, nu):
    # n steps with one synchronisation.  From 256 cells on, each step but the
    # last leaves its prolongation (u = P Q y' + s u~, f = lambda M u) to the
    # next step's first marching pre-smoothing, which forms both in its pass
    # with the stand-alone prolongation's arithmetic: the same eigenvalues
    # and vectors bit for bit as n single steps, and the same stop test
    _say(f"iterate_n H=1/{nc} h=1/{nf} {smoother} nu={nu}")
    with P.Solver(2, 1 / nc, 1 / nf, 4, opts=_opts(smoother, nu)) as s:
        with pytest.raises(P.PasmError):
            P.pasm_iterate_n(s.ctx, 0)
        P.pasm_restart(s.ctx)
        flags = [P.pasm_iterate(s.ctx) for _ in range(3)]
        lam1, U1 = s.eigenpairs()
        P.pasm_restart(s.ctx)
        flag = P.pasm_iterate_n(s.ctx, 3)
        lam2, U2 = s.eigenpairs()
        assert np.array_equal(lam1, lam2)
        assert np.array_equal(U1, U2)
        assert flag == flags[-1]
        # and continuing: one more step each way agrees too
        assert P.pasm_iterate_n(s.ctx, 1) in (True, False)


def test_restart_matches_the_start_after_setup():
    # set-up forms u_i = P q_i with the dense product Q e_i; a restart gathers
    # the column q_i instead and fuses the first right-hand side into the
    # prolongation: the same iterates to rounding
    _say("restart vs set-up start")
    with P.Solver(2, 1 / 8, 1 / 64, 4, opts=_opts("cheb", 4)) as s:
        hist0 = []
        for _ in range(3):
            s.iterate()
            hist0.append(s.eigenpairs()[0])
        U0 = s.eigenpairs()[1]
        P.pasm_restart(s.ctx)
        hist1 = []
        for _ in range(3):
            s.iterate()
            hist1.append(s.eigenpairs()[0])
        U1 = s.eigenpairs()[1]
    assert np.max(np.abs(np.array(hist1) - np.array(hist0)) / np.array(hist0)) < 1e-12
    assert np.max(np.abs(U1 - U0)) < 1e-10 * np.max(np.abs(U0))


def test_restart_start_read_first_equals_fused_start():
    # from 256 cells on, a restart leaves u_i = P q_i and theta_i M u_i to
    # the next step's first marching pre-smoothing; a caller that reads u in
    # between gets them from the stand-alone prolongation (the same
    # arithmetic): the same iterates bit for bit either way
    _say("restart: start read first vs formed in the first pass")
    with P.Solver(2, 1 / 8, 1 / 256, 4, opts=_opts("cheb", 4)) as s:
        P.pasm_restart(s.ctx)
        lam0, U0 = s.eigenpairs()
        assert np.all(np.isfinite(U0)) and np.max(np.abs(U0)) > 0.0
        for _ in range(2):
            s.iterate()
        la, Ua = s.eigenpairs()
        P.pasm_restart(s.ctx)
        assert P.pasm_iterate_n(s.ctx, 2) in (True, False)
        lb, Ub = s.eigenpairs()
    assert np.array_equal(la, lb)
    assert np.array_equal(Ua, Ub)


def test_fine_equal_coarse_returns_coarse_ritz_pairs():
    _say("h = H")
    prob = O.make_problem(2, 8, 8)
    w, _ = O.discrete_eigenpairs(prob.A, prob.M, 3)
    with P.Solver(2, 1 / 8, 1 / 8, 3, opts=_opts()) as s:
        s.iterate()
        lam, _ = s.eigenpairs(False)
        _, _, flags = P.pasm_last_selection(s.ctx, 3)
    assert np.max(np.abs(lam - w) / w) < 1e-12
    assert np.all(flags & 1)


@pytest.mark.parametrize("precision", [P.PASM_FP64, P.PASM_MIXED])
def test_3d_solve_with_degenerate_pair(precision):
    _say(f"solve lap3d H=1/4 h=1/16 k=4 prec={precision}")
    prob = O.make_problem(3, 4, 16)
    w, V = O.discrete_eigenpairs(prob.A, prob.M, 4)
    with P.Solver(3, 1 / 4, 1 / 16, 4, opts=_opts("jacobi", 2, tol=1e-12, precision=precision)) as s:
        s.solve()
        lam, U = s.eigenpairs()
    assert np.max(np.abs(np.sort(lam) - w) / w) < (1e-10 if precision == P.PASM_FP64 else 1e-8)
    # the double eigenvalue: compare subspaces
    idx = [i for i in range(4) if abs(lam[i] - w[1]) < 1e-8 * w[1]]
    assert len(idx) == 2
    Qa, _ = np.linalg.qr(V[:, 1:3])
    Qb, _ = np.linalg.qr(U[idx].T)
    assert np.min(np.linalg.svd(Qa.T @ Qb, compute_uv=False)) > 1 - 1e-10


@pytest.mark.parametrize("vcycles", [1, 2])
def test_3d_mixed_one_step_matches_oracle(vcycles):
    # mixed precision on the cube: the step's residuals form lambda M u
    # from u (f is never stored) and the last FP32 correction is added in
    # the border pass; against the oracle's FP64 step, 1e-8 on lambda and
    # 1e-6 on u
    nc, nf, k = 4, 32, 4
    _say(f"one mixed 3D step H=1/{nc} h=1/{nf} k={k} vcycles={vcycles}")
    prob = O.make_problem(3, nc, nf)
    lam0, U0, _, _ = O.coarse_start(prob, k)
    bvp = O.MultigridBVP(prob, default_options(3, "jacobi", 2, 2, vcycles))
    o = P.options(precision=P.PASM_MIXED, smoother=P.PASM_JACOBI, nu_pre=2, nu_post=2, vcycles=vcycles)
    with P.Solver(3, 1 / nc, 1 / nf, k, opts=o) as s:
        P.pasm_set_state(s.ctx, lam0, U0)
        s.iterate()
        lam, U = s.eigenpairs()
        bz, _, _ = P.pasm_last_borders(s.ctx, k)
    for i in range(k):
        ref = O.correction_step(prob, lam0[i], U0[i], bvp)
        eu = np.max(np.abs(U[i] - ref["u"])) / np.max(np.abs(ref["u"]))
        _say(f"  pair {i}: lambda {abs(lam[i] - ref['lam']) / ref['lam']:.1e} u {eu:.1e}")
        assert bz[i, 0] == pytest.approx(ref["beta"], rel=1e-6)
        assert bz[i, 1] == pytest.approx(ref["zeta"], rel=1e-6)
        assert abs(lam[i] - ref["lam"]) / ref["lam"] < 1e-8
        assert eu < 1e-6


@pytest.mark.parametrize("nc,nf,k", [(6, 192, 5), (5, 160, 3)])
def test_2d_mixed_kappa_one_step_ragged_strips(nc, nf, k):
    # mixed precision with a rough per-element kappa on grids whose interior
    # (191, 159 nodes per side) leaves a partial last strip and band in the
    # row-marching border pass (strips of 60 columns) and in the marching
    # smoother, and a coarse space that is no power of two; against the
    # oracle's FP64 step, 1e-8 on lambda and 1e-6 on u and the borders
    _say(f"one mixed kappa step H=1/{nc} h=1/{nf} k={k}")
    kap = lognormal_kappa(2, nf, seed=12, sigma=1.0)
    prob = O.make_problem(2, nc, nf, kappa=kap)
    lam0, U0, _, _ = O.coarse_start(prob, k)
    bvp = O.MultigridBVP(prob, default_options(2, "cheb", 4, 4, 2))
    with P.Solver(2, 1 / nc, 1 / nf, k, kappa=kap, opts=_opts("cheb", 4, precision=P.PASM_MIXED)) as s:
        P.pasm_set_state(s.ctx, lam0, U0)
        s.iterate()
        lam, U = s.eigenpairs()
        bz, _, _ = P.pasm_last_borders(s.ctx, k)
    for i in range(k):
        ref = O.correction_step(prob, lam0[i], U0[i], bvp)
        eu = np.max(np.abs(U[i] - ref["u"])) / np.max(np.abs(ref["u"]))
        _say(f"  pair {i}: lambda {abs(lam[i] - ref['lam']) / ref['lam']:.1e} u {eu:.1e}")
        assert bz[i, 0] == pytest.approx(ref["beta"], rel=1e-6)
        assert bz[i, 1] == pytest.approx(ref["zeta"], rel=1e-6)
        assert abs(lam[i] - ref["lam"]) / ref["lam"] < 1e-8
        assert eu < 1e-6


def test_variable_kappa_lowest_eigenpair():
    _say("solve kappa2d H=1/8 h=1/64 k=1")
    kap = lognormal_kappa(2, 64, seed=4, sigma=0.5)
    prob = O.make_problem(2, 8, 64, kappa=kap)
    w, _ = O.discrete_eigenpairs(prob.A, prob.M, 1)
    for prec, tol in ((P.PASM_FP64, 1e-10), (P.PASM_MIXED, 1e-8)):
        with P.Solver(2, 1 / 8, 1 / 64, 1, kappa=kap, opts=_opts("cheb", 4, precision=prec, tol=1e-12)) as s:
            s.solve()
            lam, _ = s.eigenpairs(False)
        assert abs(lam[0] - w[0]) / w[0] < tol


def test_kappa_and_potential_lowest_eigenpair():
    """-div(kappa grad u) + V u = lambda u: the operator family of the uneven batch."""
    _say("solve kappa+V 2d H=1/8 h=1/64 k=1")
    kap = lognormal_kappa(2, 64, seed=6, sigma=0.5)
    vel, vfn = _potential(64, True)
    A, M = fem.assemble(2, 64, kappa=kap, potential=vfn)
    w, _ = O.discrete_eigenpairs(A, M, 1)
    for prec, tol in ((P.PASM_FP64, 1e-10), (P.PASM_MIXED, 1e-8)):
        with P.Solver(2, 1 / 8, 1 / 64, 1, kappa=kap, potential=vel,
                      opts=_opts("cheb", 4, precision=prec, tol=1e-12)) as s:
            s.solve()
            lam, _ = s.eigenpairs(False)
        assert abs(lam[0] - w[0]) / w[0] < tol
