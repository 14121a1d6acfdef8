"""GPU: the allocation-free loss/gradient entry point against the allocating one.

pasm_learned_loss_grad_noalloc carves every device buffer out of the
library's fixed per-GPU scratch array.  It runs the same kernels on the same
inputs as pasm_learned_loss_grad, so the loss and the gradient must agree;
two calls in a row (the second on a smaller level with fewer samples) check
that nothing of the first call's scratch contents leaks into the second.
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


def test_noalloc_loss_grad_equals_allocating_entry_point():
    opts = P.options(precision=P.PASM_MIXED, smoother=P.PASM_LEARNED, nu_pre=2, nu_post=2, vcycles=2)
    with P.Solver(3, 1 / 4, 1 / 32, 4, opts=opts) as s:
        rng = np.random.default_rng(21)
        W = (0.2 * rng.standard_normal((2, 16, 27))).astype(np.float32)
        P.pasm_learned_set_weights(s.ctx, W)
        # the 32-cell level with 8 samples (the largest the scratch holds),
        # then the 16-cell level with 3
        for level, ns in ((3, 8), (2, 3), (3, 2)):
            m = (4 << level) - 1
            _say(f"no-alloc loss/grad: level {level} ({m + 1} cells), {ns} samples")
            R = rng.standard_normal((ns, m ** 3)).astype(np.float32).astype(np.float64)
            Rt = torch.from_numpy(R).cuda()
            la, ga = P.pasm_learned_loss_grad(s.ctx, level, Rt)
            lb, gb = P.pasm_learned_loss_grad_noalloc(s.ctx, level, Rt)
            _say(f"  loss {la:.9e} / {lb:.9e}, grad max diff {np.max(np.abs(ga - gb)):.2e}")
            assert lb == pytest.approx(la, rel=1e-12, abs=0.0)
            assert np.max(np.abs(gb - ga)) <= 1e-12 * np.max(np.abs(ga))
        # beyond the scratch size: refused with a clear message, context intact
        R = rng.standard_normal((9, 31 ** 3))
        with pytest.raises(P.PasmError) as e:
            P.pasm_learned_loss_grad_noalloc(s.ctx, 3, torch.from_numpy(R).cuda())
        assert e.value.status == P.PASM_E_INVALID and "scratch" in str(e.value)
        R = rng.standard_normal((2, 15 ** 3))
        la, ga = P.pasm_learned_loss_grad(s.ctx, 2, torch.from_numpy(R).cuda())
        lb, gb = P.pasm_learned_loss_grad_noalloc(s.ctx, 2, torch.from_numpy(R).cuda())
        assert lb == pytest.approx(la, rel=1e-12, abs=0.0)
