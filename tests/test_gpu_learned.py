"""GPU parity of the learned smoother (3D Kuhn-mesh Laplacian levels).

The inference step and the training gradient are compared with the oracle's
arithmetic (oracle/learned.py, which rounds the same operands to bfloat16);
the differences left come from FP32 accumulation on the GPU and the rare
bfloat16 rounding decision that FP32 and FP64 sums take differently, which
bounds them well below 1e-2 of the result while any wrong tap, channel or
sign is O(1).  Whole solves with the learned smoother (and with weights that
force the Jacobi fallback) must reach the discrete eigenvalues."""
import sys

import numpy as np
import pytest

import paper_1908_10251_amd as P
from oracle import fem, learned as LN, pasm as O
from oracle.multigrid import Hierarchy, MGOptions

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

NC, NF, K = 4, 32, 4


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _opts(precision, nu=2, tol=1e-10, max_iter=80):
    return P.options(precision=precision, smoother=P.PASM_LEARNED, nu_pre=nu, nu_post=nu, vcycles=2, tol=tol,
                     max_iter=max_iter)


def _weights(seed, scale):
    rng = np.random.default_rng(seed)
    return (scale * rng.standard_normal((2, 16, 27))).astype(np.float32)


@pytest.mark.parametrize("precision", [P.PASM_FP64, P.PASM_MIXED])
def test_learned_step_matches_oracle(precision):
    _say(f"learned step prec={precision}")
    with P.Solver(3, 1 / NC, 1 / NF, K, opts=_opts(precision)) as s:
        W = _weights(11, 0.3)
        P.pasm_learned_set_weights(s.ctx, W)
        W64 = W.astype(np.float64)
        rng = np.random.default_rng(12)
        for level in (2, 3):
            n = NC << level
            m = n - 1
            h = 1.0 / n
            x = rng.standard_normal((2, m ** 3))
            f = 6 * h * rng.standard_normal((2, m ** 3))
            out = torch.zeros(2, m ** 3, dtype=torch.float64, device="cuda")
            P.pasm_learned_step(s.ctx, level, _t(x), _t(f), out)
            out = out.cpu().numpy()
            for r in range(2):
                if precision == P.PASM_MIXED:  # the cycle type holds x and f in FP32
                    xr, fr = x[r].astype(np.float32).astype(np.float64), f[r].astype(np.float32).astype(np.float64)
                else:
                    xr, fr = x[r], f[r]
                ref = LN.smooth_step(xr.reshape(m, m, m), fr.reshape(m, m, m), h, W64[0], W64[1], bf=True).reshape(-1)
                scale = np.max(np.abs(ref - xr))
                err = np.max(np.abs(out[r] - ref)) / scale
                _say(f"  level {level} rhs {r}: err {err:.2e} (|delta| max {scale:.2e})")
                assert err < 3e-3, (level, r, err)
                assert np.mean(np.abs(out[r] - ref)) / scale < 2e-5


def test_learned_gradient_matches_oracle():
    _say("learned loss and gradient")
    with P.Solver(3, 1 / NC, 1 / NF, K, opts=_opts(P.PASM_MIXED)) as s:
        W = _weights(13, 0.2)
        P.pasm_learned_set_weights(s.ctx, W)
        level, m = 2, (NC << 2) - 1
        h = 1.0 / (NC << 2)
        R = np.random.default_rng(14).standard_normal((3, m ** 3)).astype(np.float32).astype(np.float64)
        loss, g = P.pasm_learned_loss_grad(s.ctx, level, _t(R))
        W64 = W.astype(np.float64)
        Lr, g1, g2 = LN.loss_and_grad(R.reshape(3, m, m, m), h, W64[0], W64[1], bf=True)
        _say(f"  loss {loss:.6e} oracle {Lr:.6e}")
        assert abs(loss - Lr) / Lr < 1e-4
        for got, ref in ((g[0], g1), (g[1], g2)):
            err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
            _say(f"  grad err {err:.2e}")
            assert err < 1e-3


@pytest.mark.parametrize("precision", [P.PASM_MIXED, P.PASM_FP64])
def test_learned_solve_reaches_discrete_eigenvalues(precision):
    _say(f"learned solve prec={precision}")
    prob = O.make_problem(3, NC, NF)
    w, _ = O.discrete_eigenpairs(prob.A, prob.M, K)
    with P.Solver(3, 1 / NC, 1 / NF, K, opts=_opts(precision, tol=1e-12)) as s:
        rep0 = P.pasm_learned_report(s.ctx)
        _say(f"  set-up: {rep0}")
        assert rep0["train_steps"] > 0 and rep0["loss_last"] < rep0["loss_first"]
        assert 0 < rep0["learned_rate"] < 1 and 0 < rep0["plain_rate"] < 1
        P.pasm_learned_enable(s.ctx, True)  # whatever the speed test decided
        s.solve(allow_notconv=True)
        lam, _ = s.eigenpairs(False)
        rep = P.pasm_learned_report(s.ctx)
        _say(f"  after solve: {rep}")
        assert rep["cycles_learned"] + rep["cycles_fallback"] > 0 or not rep["enabled"]
    tol = 1e-8 if precision == P.PASM_MIXED else 1e-10
    assert np.max(np.abs(np.sort(lam) - w) / w) < tol
    assert rep["cycles_learned"] > 0


def test_bad_weights_fall_back_to_jacobi():
    """An anti-smoother (x - omega rho) is rejected every cycle; the plain
    cycles still solve the problem."""
    _say("learned fallback")
    prob = O.make_problem(3, NC, NF)
    w, _ = O.discrete_eigenpairs(prob.A, prob.M, K)
    with P.Solver(3, 1 / NC, 1 / NF, K, opts=_opts(P.PASM_MIXED, tol=1e-12)) as s:
        W = np.zeros((2, 16, 27), dtype=np.float32)
        W[0, 0, 13], W[0, 1, 13] = 1.0, -1.0
        W[1, 0, 13], W[1, 1, 13] = -1.5, 1.5
        P.pasm_learned_set_weights(s.ctx, W)
        P.pasm_learned_enable(s.ctx, True)
        before = P.pasm_learned_report(s.ctx)
        s.solve(allow_notconv=True)
        lam, _ = s.eigenpairs(False)
        rep = P.pasm_learned_report(s.ctx)
    assert rep["cycles_fallback"] > before["cycles_fallback"]
    assert np.max(np.abs(np.sort(lam) - w) / w) < 1e-8


def test_learned_vcycle_matches_oracle():
    """One library V-cycle with the trained weights against the oracle's
    learned V-cycle with the same weights (FP64 cycle)."""
    _say("learned vcycle")
    A, _ = fem.assemble(3, NF)
    hier = Hierarchy(3, A, NC, NF)
    rng = np.random.default_rng(15)
    N = A.shape[0]
    f = rng.standard_normal((2, N))
    x0 = rng.standard_normal((2, N))
    with P.Solver(3, 1 / NC, 1 / NF, K, opts=_opts(P.PASM_FP64)) as s:
        W = P.pasm_learned_weights(s.ctx).astype(np.float64)
        P.pasm_learned_enable(s.ctx, True)
        # no fallback: a cycle is redone only if it grows the residual 1e6-fold
        P.pasm_learned_set_threshold(s.ctx, 1e6)
        before = P.pasm_learned_report(s.ctx)
        xg = _t(x0)
        P.pasm_vcycle(s.ctx, _t(f), xg, 1)
        xg = xg.cpu().numpy()
        rep = P.pasm_learned_report(s.ctx)
    # the learned cycle ran and was kept
    assert before["enabled"] and rep["cycles_fallback"] == before["cycles_fallback"]
    assert rep["cycles_learned"] == before["cycles_learned"] + 1
    opts = MGOptions("learned", 1, 1, 6.0 / 7.0, 6.0, 1, weights=(W[0], W[1]), learned_bf16=True)
    for r in range(2):
        ref = hier.vcycle(len(hier.levels) - 1, x0[r], f[r], opts)
        err = np.max(np.abs(xg[r] - ref)) / np.max(np.abs(ref))
        _say(f"  rhs {r}: err {err:.2e}")
        assert err < 2e-3
