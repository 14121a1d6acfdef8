"""GPU: graph replay of correction steps (pasm_use_graph) against eager steps.

Two contexts with identical set-up run the same sequence of entry points, one
with the replay on; a replayed step launches the same kernels with the same
arguments, so the eigenvalues and eigenvectors must agree bit for bit after
every call.  The sequences mix pasm_iterate (each step's prolongation formed
by the stand-alone pass) and pasm_iterate_n (prolongations left to the next
step's first pass), with eigenvector reads (which settle a pending
prolongation) and host synchronisations between the replays, so every
recorded graph is replayed several times from both kinds of state (the
states recur every few steps: the eigenvalue buffers rotate with period 3 and
u alternates between two buffers).  The replay counter must show that graphs
actually ran.
"""
import sys

import numpy as np
import pytest

import paper_1908_10251_amd as P
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _run(dim, H, h, k, opts, kappa=None, calls=None):
    calls = calls or [("n", 3), ("n", 3), ("1", 1), ("1", 1), ("1", 1), ("n", 2), ("1", 1), ("1", 1),
                      ("n", 3), ("n", 3), ("1", 1), ("1", 1), ("1", 1), ("1", 1), ("n", 4), ("n", 2)]
    out = {}
    for graph in (False, True):
        seq = []
        with P.Solver(dim, H, h, k, kappa=kappa, opts=opts) as s:
            P.pasm_use_graph(s.ctx, graph)
            P.pasm_restart(s.ctx)
            for kind, n in calls:
                if kind == "n":
                    P.pasm_iterate_n(s.ctx, n)
                else:
                    s.iterate()
                seq.append(s.eigenpairs())
            stats = P.pasm_graph_stats(s.ctx)
        out[graph] = (seq, stats)
    (eager, st0), (replay, st1) = out[False], out[True]
    assert st0 == (False, 0, 0), st0
    assert st1[0] and st1[2] > 0, st1
    for t, ((la, Ua), (lb, Ub)) in enumerate(zip(eager, replay)):
        assert np.array_equal(la, lb), (t, np.max(np.abs(la - lb)))
        assert np.array_equal(Ua, Ub), (t, np.max(np.abs(Ua - Ub)))
    _say(f"  {len(eager)} calls agree bit for bit; graphs held {st1[1]}, steps replayed {st1[2]}")
    return st1


def test_graph_replay_fp64_laplace_marching():
    _say("graph replay: 2D FP64 Laplacian, H=1/8 h=1/256 k=4, Chebyshev 4/4")
    opts = P.options(smoother=P.PASM_CHEBYSHEV, nu_pre=4, nu_post=4, vcycles=2)
    _run(2, 1 / 8, 1 / 256, 4, opts)


def test_graph_replay_mixed_rough_coefficient():
    _say("graph replay: 2D mixed, log-normal kappa, H=1/8 h=1/256 k=6")
    kappa = W.lognormal_kappa(2, 256, seed=3)
    opts = P.options(precision=P.PASM_MIXED, smoother=P.PASM_CHEBYSHEV, nu_pre=4, nu_post=4, vcycles=2)
    _run(2, 1 / 8, 1 / 256, 6, opts, kappa=kappa)


def test_graph_replay_cg_smoothing():
    _say("graph replay: 2D FP64, the paper's CG(2) multigrid step, H=1/8 h=1/128 k=4")
    opts = P.options(smoother=P.PASM_CG, nu_pre=2, nu_post=2, vcycles=1)
    _run(2, 1 / 8, 1 / 128, 4, opts)


def test_graph_replay_mixed_cube():
    _say("graph replay: 3D mixed Laplacian, H=1/4 h=1/32 k=5")
    opts = P.options(precision=P.PASM_MIXED, smoother=P.PASM_CHEBYSHEV, nu_pre=4, nu_post=4, vcycles=2)
    _run(3, 1 / 4, 1 / 32, 5, opts)


def test_graph_replay_off_while_profiling():
    # steps that record profiling events run unrecorded
    _say("graph replay with profiling on: no graphs recorded")
    opts = P.options(smoother=P.PASM_CHEBYSHEV, nu_pre=4, nu_post=4, vcycles=2)
    with P.Solver(2, 1 / 8, 1 / 256, 4, opts=opts) as s:
        P.pasm_use_graph(s.ctx, True)
        P.pasm_profile(s.ctx, 0, True)
        for _ in range(4):
            P.pasm_iterate_n(s.ctx, 2)
        assert P.pasm_graph_stats(s.ctx) == (True, 0, 0)
        launches, ms, _ = P.pasm_profile_read(s.ctx, 0)
        assert launches > 0 and ms > 0.0
        P.pasm_profile(s.ctx, 0, False)
        for _ in range(12):
            P.pasm_iterate_n(s.ctx, 2)
        assert P.pasm_graph_stats(s.ctx)[2] > 0
        P.pasm_use_graph(s.ctx, False)
        assert P.pasm_graph_stats(s.ctx)[:2] == (False, 0)
