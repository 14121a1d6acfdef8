"""GPU parity of batches of uneven instances (one launch per level for all
members, recorded graph per iteration, autotuned smoothing tiles).

Each member is the operator family of the uneven batch: -div(kappa grad u)
+ V u with log-normal kappa per element and V = s |x - c|^2, on its own fine
mesh.  The batch is checked against the oracle's correction step member by
member, against single-instance contexts, graph replays against eager
launches, every tile height against the others, and a mixed-precision solve
against the discrete eigenvalues."""
import sys

import numpy as np
import pytest

import paper_1908_10251_amd as P
from oracle import fem, pasm as O
from oracle.multigrid import default_options
from workloads import lognormal_kappa, quadratic_potential_elements

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

H = 1 / 8
FINE = [32, 64, 16, 64]          # uneven: 3, 4, 2 and 4 levels
CENTRES = [(0.3, 0.6), (0.7, 0.2), (0.5, 0.5), (0.1, 0.9)]
VSCALE = 200.0


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _members(sigma=0.5):
    out = []
    for i, (nf, c) in enumerate(zip(FINE, CENTRES)):
        kap = lognormal_kappa(2, nf, seed=20 + i, sigma=sigma)
        vel = quadratic_potential_elements(nf, c, VSCALE)
        out.append((nf, c, kap, vel))
    return out


def _oracle_problem(nf, c, kap):
    A, M = fem.assemble(2, nf, kappa=kap, potential=lambda x: VSCALE * fem.quadratic_potential(c)(x))
    base = O.make_problem(2, int(round(1 / H)), nf)
    return O.Problem(2, base.n_coarse, nf, A, M, base.P, (base.P.T @ A @ base.P).toarray(), base.MH)


def _opts(precision=P.PASM_FP64, nu=4, fused=True, tol=1e-10, max_iter=60):
    return P.options(precision=precision, smoother=P.PASM_CHEBYSHEV, nu_pre=nu, nu_post=nu, vcycles=2, tol=tol,
                     max_iter=max_iter, fused=fused)


@pytest.mark.parametrize("fused", [False, True])
def test_batch_one_step_matches_oracle_per_member(fused):
    """From the oracle's coarse start of every member, one batched correction
    step equals the oracle's Algorithm 1 with the same V-cycles."""
    _say(f"batch one step fused={fused}")
    k = 3
    mem = _members()
    with P.Batch(H, k, [(1 / nf, kap, vel) for nf, _, kap, vel in mem], opts=_opts(fused=fused)) as b:
        refs = []
        for i, (nf, c, kap, vel) in enumerate(mem):
            prob = _oracle_problem(nf, c, kap)
            lam0, U0, _, _ = O.coarse_start(prob, k)
            lg, _ = b.eigenpairs(i, False)
            assert np.max(np.abs(lg - lam0) / lam0) < 1e-12, (i, lg, lam0)
            P.pasm_batch_set_state(b.b, i, lam0, U0)
            bvp = O.MultigridBVP(prob, default_options(2, "cheb", 4, 4, 2))
            refs.append([O.correction_step(prob, lam0[j], U0[j], bvp) for j in range(k)])
        b.iterate()
        for i in range(len(mem)):
            lg, Ug = b.eigenpairs(i)
            for j in range(k):
                ref = refs[i][j]
                assert abs(lg[j] - ref["lam"]) / ref["lam"] < 1e-11, (i, j, lg[j], ref["lam"])
                d = np.max(np.abs(Ug[j] - ref["u"])) / np.max(np.abs(ref["u"]))
                assert d < 1e-8, (i, j, d)


def test_batch_large_members_mixed_one_step_matches_oracle():
    """Members of 256 and 512 cells march their FP32 levels of 256 cells and
    more in one launch per phase, each pair of right-hand sides with its
    member's coefficient planes and smoothing scale; an odd number of
    right-hand sides per member marches them one per wavefront.  One batched
    mixed-precision step from the oracle's coarse starts against the
    oracle's FP64 step per member."""
    _say("batch, members of 256 and 512 cells, k = 3, mixed: one step")
    k = 3
    mem = []
    for i, (nf, c) in enumerate([(256, (0.3, 0.6)), (512, (0.7, 0.2))]):
        kap = lognormal_kappa(2, nf, seed=40 + i, sigma=0.5)
        mem.append((nf, c, kap, quadratic_potential_elements(nf, c, VSCALE)))
    with P.Batch(H, k, [(1 / nf, kap, vel) for nf, _, kap, vel in mem], opts=_opts(precision=P.PASM_MIXED)) as b:
        refs = []
        for i, (nf, c, kap, vel) in enumerate(mem):
            prob = _oracle_problem(nf, c, kap)
            lam0, U0, _, _ = O.coarse_start(prob, k)
            P.pasm_batch_set_state(b.b, i, lam0, U0)
            bvp = O.MultigridBVP(prob, default_options(2, "cheb", 4, 4, 2))
            refs.append([O.correction_step(prob, lam0[j], U0[j], bvp) for j in range(k)])
        b.iterate()
        for i in range(len(mem)):
            lg, Ug = b.eigenpairs(i)
            for j in range(k):
                ref = refs[i][j]
                el = abs(lg[j] - ref["lam"]) / ref["lam"]
                d = np.max(np.abs(Ug[j] - ref["u"])) / np.max(np.abs(ref["u"]))
                _say(f"  member {i} pair {j}: lambda {el:.2e}, u {d:.2e}")
                assert el < 1e-8, (i, j, el)
                assert d < 1e-6, (i, j, d)


def test_batch_equals_single_instances():
    """Three iterations of the batch give each member's single-context history."""
    _say("batch vs single contexts")
    k = 3
    mem = _members()
    hist_b = []
    with P.Batch(H, k, [(1 / nf, kap, vel) for nf, _, kap, vel in mem], opts=_opts()) as b:
        for _ in range(3):
            b.iterate()
            hist_b.append(b.eigenvalues())
    for i, (nf, _, kap, vel) in enumerate(mem):
        with P.Solver(2, H, 1 / nf, k, kappa=kap, potential=vel, opts=_opts()) as s:
            for t in range(3):
                s.iterate()
                lam, _ = s.eigenpairs(False)
                err = np.max(np.abs(lam - hist_b[t][i]) / lam)
                assert err < 1e-11, (i, t, err)


def test_batch_graph_replays_equal_eager_launches():
    """The recorded iteration replayed (with eager work and synchronisations
    between replays) gives bit-identical eigenvalues to launching the same
    kernels one by one."""
    _say("batch graph vs eager")
    k = 2
    mem = _members()
    with P.Batch(H, k, [(1 / nf, kap, vel) for nf, _, kap, vel in mem],
                 opts=_opts(precision=P.PASM_MIXED)) as b:
        runs = []
        for graph in (True, False, True, True):
            P.pasm_batch_use_graph(b.b, graph)
            P.pasm_batch_restart(b.b)
            torch.cuda.synchronize()
            h = []
            for _ in range(3):
                b.iterate()
                h.append(b.eigenvalues())
            runs.append(np.array(h))
        for r in runs[1:]:
            assert np.array_equal(r, runs[0])


def test_batch_restart_matches_the_start_after_setup():
    """A restart (columns of each member's Q gathered, lambda = theta per
    member) gives the iterates of the start that set-up forms with the dense
    products."""
    _say("batch restart vs set-up start")
    k = 2
    mem = _members()
    with P.Batch(H, k, [(1 / nf, kap, vel) for nf, _, kap, vel in mem], opts=_opts()) as b:
        runs = []
        for restart in (False, True):
            if restart:
                P.pasm_batch_restart(b.b)
            h = []
            for _ in range(3):
                b.iterate()
                h.append(b.eigenvalues())
            runs.append(np.array(h))
    assert np.max(np.abs(runs[1] - runs[0]) / runs[0]) < 1e-12


def test_batch_every_tile_height_agrees():
    _say("batch tiles")
    k = 2
    mem = _members()
    with P.Batch(H, k, [(1 / nf, kap, vel) for nf, _, kap, vel in mem], opts=_opts(nu=2)) as b:
        rows, ms = P.pasm_batch_tuning(b.b)
        L = P.pasm_batch_num_levels(b.b)
        assert len(rows) == L
        for l in range(1, L):
            assert rows[l] in (0, 2, 4, 8)
            cand = [c for c, t in zip((0, 2, 4, 8), ms[l]) if t >= 0]
            assert rows[l] in cand and len(cand) >= 2
            assert ms[l][(0, 2, 4, 8).index(rows[l])] == min(t for t in ms[l] if t >= 0)
        out = {}
        for r in (0, 2, 4):
            P.pasm_batch_set_tiles(b.b, [0] + [r] * (L - 1))
            P.pasm_batch_restart(b.b)
            b.iterate()
            b.iterate()
            out[r] = b.eigenvalues()
        for r in (2, 4):
            assert np.max(np.abs(out[r] - out[0]) / out[0]) < 1e-12, r
        with pytest.raises(P.PasmError):
            P.pasm_batch_set_tiles(b.b, [0] + [3] * (L - 1))


def test_batch_tile_height_8_agrees():
    # the tallest fused tile (8 x 4 LDS rows per workgroup) fits the LDS with
    # FP32 V-cycles: compared with per-step smoothing and with height 4 on the
    # same start, to the mixed-precision bar
    _say("batch tile height 8 (mixed)")
    k = 2
    mem = _members()
    with P.Batch(H, k, [(1 / nf, kap, vel) for nf, _, kap, vel in mem],
                 opts=_opts(precision=P.PASM_MIXED, nu=2)) as b:
        rows, ms = P.pasm_batch_tuning(b.b)
        L = P.pasm_batch_num_levels(b.b)
        t8 = [0] + [8 if ms[l][3] >= 0 else 4 for l in range(1, L)]
        assert any(t == 8 for t in t8[1:]), ms
        out = {}
        for name, tiles in (("0", [0] * L), ("4", [0] + [4] * (L - 1)), ("8", t8)):
            P.pasm_batch_set_tiles(b.b, tiles)
            P.pasm_batch_restart(b.b)
            b.iterate()
            b.iterate()
            out[name] = b.eigenvalues()
        for name in ("4", "8"):
            d = np.max(np.abs(out[name] - out["0"]) / out["0"])
            _say(f"  tiles {name} vs per-step: {d:.2e}")
            assert d < 1e-8, name


def test_batch_mixed_solve_reaches_discrete_eigenvalues():
    _say("batch mixed solve")
    k = 2
    mem = _members()
    with P.Batch(H, k, [(1 / nf, kap, vel) for nf, _, kap, vel in mem],
                 opts=_opts(precision=P.PASM_MIXED, tol=1e-12, max_iter=80)) as b:
        b.solve(allow_notconv=True)
        for i, (nf, c, kap, vel) in enumerate(mem):
            prob = _oracle_problem(nf, c, kap)
            w, V = O.discrete_eigenpairs(prob.A, prob.M, 1)
            lam, U = b.eigenpairs(i)
            assert abs(lam[0] - w[0]) / w[0] < 1e-8, (i, lam[0], w[0])
            u = U[0] if U[0] @ (prob.M @ V[:, 0]) >= 0 else -U[0]
            d = u - V[:, 0]
            assert np.sqrt(d @ (prob.M @ d)) < 1e-4, i
