"""GPU: context state across entry points, and the error paths of the ABI.

* A restart leaves the start u_i = P q_i and its right-hand side theta_i M u_i
  to the next step's first pass (2D FP64 marching levels).  Building-block
  calls in between must not change what the next step computes: after a
  V-cycle on caller data the same iterates to rounding (the right-hand side
  is formed again, by another kernel), after an eigenvalue-only query
  bit-identical ones (nothing is enqueued).
* Non-finite input is refused at the boundary (pasm_set_state), the context
  stays usable; the iteration cap gives PASM_E_NOTCONV.
"""
import sys

import numpy as np
import pytest

import paper_1908_10251_amd as P

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _opts(**kw):
    base = dict(smoother=P.PASM_CHEBYSHEV, nu_pre=4, nu_post=4, vcycles=2, tol=1e-10)
    base.update(kw)
    return P.options(**base)


def test_restart_vcycle_iterate_equals_restart_iterate():
    # 256 cells: the marching finest level, so the restart's start is pending
    # when pasm_vcycle runs; the V-cycle overwrites the right-hand side buffer
    # with the caller's f, and the following step must form lambda M u again
    _say("restart -> vcycle(nrhs < k) -> iterate vs restart -> iterate, H=1/8 h=1/256 k=4")
    k = 4
    with P.Solver(2, 1 / 8, 1 / 256, k, opts=_opts()) as s:
        N = P.pasm_num_dofs(s.ctx)
        P.pasm_restart(s.ctx)
        s.iterate()
        lam_a, U_a = s.eigenpairs()
        P.pasm_restart(s.ctx)
        rng = np.random.default_rng(3)
        f = torch.from_numpy(rng.standard_normal((2, N))).cuda()
        x = torch.zeros(2, N, dtype=torch.float64, device="cuda")
        P.pasm_vcycle(s.ctx, f, x, 1)
        assert float(torch.max(torch.abs(x))) > 0.0
        s.iterate()
        lam_b, U_b = s.eigenpairs()
    # the two orders form theta M u with different kernels (in the first
    # pass, or the stand-alone mass product after the V-cycle reused the
    # buffer), equal to rounding; a step on the caller's f would be O(1) off
    assert np.max(np.abs(lam_a - lam_b) / lam_a) < 1e-13
    assert np.max(np.abs(U_a - U_b)) < 1e-11 * np.max(np.abs(U_a))


def test_mixed_kappa_restart_vcycle_iterate_equals_restart_iterate():
    # mixed precision with edge weights: the prolongation that forms u also
    # forms the next step's first FP32 residual (f = lambda M u is never
    # stored).  A V-cycle in between reuses that buffer, so the following
    # step must form its residual again from u.  Set-state in between
    # likewise.
    from workloads import lognormal_kappa
    _say("mixed kappa: restart -> vcycle -> iterate vs restart -> iterate, H=1/8 h=1/256 k=3")
    k, nf = 3, 256
    kap = lognormal_kappa(2, nf, seed=31, sigma=1.0)
    with P.Solver(2, 1 / 8, 1 / nf, k, kappa=kap, opts=_opts(precision=P.PASM_MIXED)) as s:
        N = P.pasm_num_dofs(s.ctx)
        P.pasm_restart(s.ctx)
        s.iterate()
        s.iterate()
        lam_a, U_a = s.eigenpairs()
        P.pasm_restart(s.ctx)
        s.iterate()
        rng = np.random.default_rng(4)
        f = torch.from_numpy(rng.standard_normal((2, N))).cuda()
        x = torch.zeros(2, N, dtype=torch.float64, device="cuda")
        P.pasm_vcycle(s.ctx, f, x, 1)
        s.iterate()
        lam_b, U_b = s.eigenpairs()
        # a state set from the host: the residual of the old state is stale
        P.pasm_restart(s.ctx)
        s.iterate()
        lam_1, U_1 = s.eigenpairs()
        P.pasm_restart(s.ctx)
        P.pasm_set_state(s.ctx, lam_1, U_1)
        s.iterate()
        lam_c, U_c = s.eigenpairs()
    for lam, U in ((lam_b, U_b), (lam_c, U_c)):
        dl = np.max(np.abs(lam_a - lam) / lam_a)
        du = np.max(np.abs(U_a - U)) / np.max(np.abs(U_a))
        _say(f"  lambda {dl:.1e}, u {du:.1e}")
        # FP32 cycles: the residuals may differ in their last bits (two
        # kernels form them); a residual of the wrong state would be O(1)
        assert dl < 1e-9 and du < 1e-5


def test_eigenvalue_only_query_changes_nothing():
    # an eigenvalue-only read between a restart and the steps enqueues no
    # work: the steps then form the start in their first pass as usual
    _say("restart -> eigenvalues only -> iterate_n(2) vs restart -> iterate_n(2), h=1/256")
    with P.Solver(2, 1 / 8, 1 / 256, 4, opts=_opts()) as s:
        P.pasm_restart(s.ctx)
        P.pasm_iterate_n(s.ctx, 2)
        lam_a, U_a = s.eigenpairs()
        P.pasm_restart(s.ctx)
        lam0, _ = s.eigenpairs(vectors=False)
        P.pasm_iterate_n(s.ctx, 2)
        lam_b, U_b = s.eigenpairs()
    assert np.all(np.isfinite(lam0))
    assert np.array_equal(lam_a, lam_b)
    assert np.array_equal(U_a, U_b)


def test_non_finite_state_is_refused_and_context_survives():
    _say("set_state with NaN / inf -> PASM_E_INVALID; the context still iterates")
    k = 3
    with P.Solver(2, 1 / 8, 1 / 64, k, opts=_opts(smoother=P.PASM_JACOBI, nu_pre=2, nu_post=2)) as s:
        s.iterate()
        lam, U = s.eigenpairs()
        bad = U.copy()
        bad[1, 17] = np.nan
        with pytest.raises(P.PasmError) as e:
            P.pasm_set_state(s.ctx, lam, bad)
        assert e.value.status == P.PASM_E_INVALID
        assert "non-finite" in str(e.value)
        bad[1, 17] = np.inf
        with pytest.raises(P.PasmError):
            P.pasm_set_state(s.ctx, lam, bad)
        lam_bad = lam.copy()
        lam_bad[0] = np.nan
        with pytest.raises(P.PasmError):
            P.pasm_set_state(s.ctx, lam_bad, U)
        # the refused calls changed nothing: the state is still (lam, U)
        lam2, U2 = s.eigenpairs()
        assert np.array_equal(lam, lam2) and np.array_equal(U, U2)
        s.iterate()
        assert np.all(np.isfinite(s.eigenpairs(False)[0]))


def test_iteration_cap_reports_not_converged():
    _say("solve with max_iter = 1 -> PASM_E_NOTCONV")
    with P.Solver(2, 1 / 8, 1 / 64, 4, opts=_opts(max_iter=1, tol=1e-14)) as s:
        with pytest.raises(P.PasmError) as e:
            s.solve()
        assert e.value.status == P.PASM_E_NOTCONV
        assert s.solve(allow_notconv=True) == 1
