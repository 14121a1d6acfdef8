"""Learned convolutional smoother for structured 3D V-cycles (oracle).

TEST INFRASTRUCTURE ONLY (see the package header).

Not part of the paper: this is the smoother of the learned-corrector growth
direction.  It replaces damped Jacobi inside the V-cycle of Algorithm 1,
step 1 ("some multigrid steps") on the 3D Kuhn-mesh Laplacian levels, and is
defined here by its arithmetic, which the GPU path must reproduce:

  rho     = (f - A x) / D                    D = the (constant) diagonal of A
  z1[c]   = sum_t W1[c, t] rho(v + t)         t in {-1,0,1}^3, c = 0..15
  h[c]    = max(z1[c], 0)                     zero outside the interior nodes
  delta   = sum_{c,t} W2[c, t] h[c](v + t)
  x_new   = x + delta

Taps are ordered t = (dx, dy, dz) -> (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1).
Fields live on the interior nodes of an n^3-cell grid ((n-1)^3 values, x
fastest); positions outside the interior count as zero (Dirichlet data).
With `bf16=True` the inputs of every contraction are rounded to bfloat16
(round to nearest even) exactly where the GPU rounds them: rho, W1, h, W2 in
the forward pass, the output gradient g and the hidden gradient in the
backward pass; sums are exact (FP64 here, FP32 on the GPU).

Training loss over residual samples r_s (the residuals that plain V-cycles
present to the smoother):
    L = (1/S) sum_s ||r_s - A delta_s||^2 / ||r_s||^2
i.e. the residual left after the correction, relative to the one before.
Its gradient (`loss_and_grad`) is pinned against central finite
differences; the forward pass against a direct loop over nodes and taps.

Parity status: pinned (tests/test_oracle_learned.py).
"""
from __future__ import annotations

import itertools

import numpy as np

CH = 16
TAPS = [(dx, dy, dz) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def bf16(a: np.ndarray) -> np.ndarray:
    """Round to bfloat16 (nearest, ties to even), returned as float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = ((u + 0x7FFF + lsb) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _rnd(a, on):
    return bf16(a) if on else np.asarray(a, dtype=np.float64)


def shift(u: np.ndarray, t) -> np.ndarray:
    """out(v) = u(v + t) on an (m, m, m) array indexed [z, y, x]; zero outside."""
    dx, dy, dz = t
    m = u.shape[0]
    out = np.zeros_like(u)
    src = [slice(max(0, d), m + min(0, d)) for d in (dz, dy, dx)]
    dst = [slice(max(0, -d), m + min(0, -d)) for d in (dz, dy, dx)]
    out[tuple(dst)] = u[tuple(src)]
    return out


def laplace7(u: np.ndarray, w0: float) -> np.ndarray:
    """A u for the 3D Kuhn-mesh stiffness with constant coefficient:
    w0 * (6 u - the six axis neighbours), zero Dirichlet data."""
    s = sum(shift(u, t) for t in [(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)])
    return w0 * (6.0 * u - s)


def forward(rho: np.ndarray, W1: np.ndarray, W2: np.ndarray, bf=False):
    """delta = N(rho) and the intermediates (z1, h) for one field rho (m, m, m)."""
    r = _rnd(rho, bf)
    w1 = _rnd(W1, bf)
    w2 = _rnd(W2, bf)
    z1 = np.zeros((CH,) + rho.shape)
    sh = [shift(r, t) for t in TAPS]
    for c in range(CH):
        for ti in range(27):
            z1[c] += w1[c, ti] * sh[ti]
    h = _rnd(np.maximum(z1, 0.0), bf)
    delta = np.zeros_like(rho)
    for c in range(CH):
        for ti, t in enumerate(TAPS):
            delta += w2[c, ti] * shift(h[c], t)
    return delta, z1, h


def forward_loops(rho, W1, W2):
    """The same map by explicit loops over nodes (tiny grids only)."""
    m = rho.shape[0]
    get = lambda a, z, y, x: a[z, y, x] if 0 <= z < m and 0 <= y < m and 0 <= x < m else 0.0
    h = np.zeros((CH, m, m, m))
    for c, z, y, x in itertools.product(range(CH), range(m), range(m), range(m)):
        s = sum(W1[c, ti] * get(rho, z + t[2], y + t[1], x + t[0]) for ti, t in enumerate(TAPS))
        h[c, z, y, x] = max(s, 0.0)
    out = np.zeros_like(rho)
    for z, y, x in itertools.product(range(m), range(m), range(m)):
        out[z, y, x] = sum(W2[c, ti] * get(h[c], z + t[2], y + t[1], x + t[0])
                           for c in range(CH) for ti, t in enumerate(TAPS))
    return out


def smooth_step(x: np.ndarray, f: np.ndarray, w0: float, W1, W2, bf=False) -> np.ndarray:
    """One learned smoothing step x <- x + N((f - A x) / D), D = 6 w0."""
    rho = (f - laplace7(x, w0)) / (6.0 * w0)
    delta, _, _ = forward(rho, W1, W2, bf)
    return x + delta


def loss_and_grad(R: np.ndarray, w0: float, W1, W2, bf=False):
    """Loss L over samples R (S, m, m, m) and its gradient (dW1, dW2).

    With bf=True the backward pass rounds g (the gradient at delta) and the
    hidden gradient to bfloat16 before they enter a contraction, and uses
    the rounded forward values, as the GPU does."""
    S = R.shape[0]
    w1 = _rnd(W1, bf)
    w2 = _rnd(W2, bf)
    L = 0.0
    dW1 = np.zeros((CH, 27))
    dW2 = np.zeros((CH, 27))
    for s in range(S):
        r = R[s]
        nr = float(np.sum(r * r))
        rho = r / (6.0 * w0)
        delta, z1, h = forward(rho, W1, W2, bf)
        res = r - laplace7(delta, w0)
        L += float(np.sum(res * res)) / nr / S
        g = _rnd(-2.0 / (S * nr) * laplace7(res, w0), bf)   # dL/d delta
        rr = _rnd(rho, bf)
        # delta = sum_{c,t} w2[c,t] h[c](v+t): dW2[c,t] = sum_v g(v) h[c](v+t)
        gh = np.zeros_like(h)
        for c in range(CH):
            for ti, t in enumerate(TAPS):
                dW2[c, ti] += float(np.sum(g * shift(h[c], t)))
                gh[c] += w2[c, ti] * shift(g, (-t[0], -t[1], -t[2]))
        gh = _rnd(gh * (z1 > 0.0), bf)
        for c in range(CH):
            for ti, t in enumerate(TAPS):
                dW1[c, ti] += float(np.sum(gh[c] * shift(rr, t)))
    return L, dW1, dW2


def adam_step(W, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step t >= 1) of W with gradient g; returns (W, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return W - lr * mh / (np.sqrt(vh) + eps), m, v


def step_matrix(A, D, x: np.ndarray, f: np.ndarray, W1, W2, bf=False) -> np.ndarray:
    """The learned step on a level given as a sparse matrix A with diagonal D
    (interior nodes of an m^3 grid, x fastest): x + N((f - A x) / D)."""
    m = round(len(x) ** (1.0 / 3.0))
    rho = ((f - A @ x) / D).reshape(m, m, m)
    delta, _, _ = forward(rho, W1, W2, bf)
    return x + delta.reshape(-1)
