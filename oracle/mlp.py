"""FP64 oracle of the learned coarse-cell proposal (a small MLP over the
projected vector Z of eq. (12)).  Test infrastructure only: see the package
docstring.

The paper searches eq. (14) with a k-d tree (Section 3, Algorithm 1 steps
3-4 offline, step 3 online); the proposal replaces that search structure:
an MLP maps the normalised projection to a few cells of a coarse grid whose
fine directions are then scored exactly.  Everything here is the plain
textbook definition: affine layers, the exact erf GELU, softmax
cross-entropy, their analytic gradients and one Adam update.
"""
from __future__ import annotations

import numpy as np
from scipy.special import erf


def gelu(x):
    """GELU(x) = x * Phi(x) = x/2 * (1 + erf(x / sqrt 2))."""
    return 0.5 * x * (1.0 + erf(x / np.sqrt(2.0)))


def gelu_grad(x):
    """d GELU / dx = Phi(x) + x * phi(x)."""
    return 0.5 * (1.0 + erf(x / np.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / np.sqrt(2.0 * np.pi)


def mlp_forward(params, f):
    """Logits of the 3-layer MLP f -> GELU(f W1^T + b1) -> GELU(. W2^T + b2)
    -> . W3^T + b3.  params = (W1, b1, W2, b2, W3, b3) with W_l [out, in].
    Returns (logits, cache)."""
    W1, b1, W2, b2, W3, b3 = params
    a1 = f @ W1.T + b1
    h1 = gelu(a1)
    a2 = h1 @ W2.T + b2
    h2 = gelu(a2)
    logits = h2 @ W3.T + b3
    return logits, (f, a1, h1, a2, h2)


def softmax_xent(logits, labels):
    """Mean softmax cross-entropy and its gradient w.r.t. the logits."""
    m = logits.max(axis=1, keepdims=True)
    e = np.exp(logits - m)
    p = e / e.sum(axis=1, keepdims=True)
    n = logits.shape[0]
    loss = -np.mean(np.log(p[np.arange(n), labels]))
    g = p.copy()
    g[np.arange(n), labels] -= 1.0
    return loss, g / n, p


def mlp_backward(params, cache, dlogits):
    """Analytic gradients of the MLP for upstream gradient dlogits.
    Returns (dW1, db1, dW2, db2, dW3, db3)."""
    W1, b1, W2, b2, W3, b3 = params
    f, a1, h1, a2, h2 = cache
    dW3 = dlogits.T @ h2
    db3 = dlogits.sum(axis=0)
    dh2 = dlogits @ W3
    da2 = dh2 * gelu_grad(a2)
    dW2 = da2.T @ h1
    db2 = da2.sum(axis=0)
    dh1 = da2 @ W2
    da1 = dh1 * gelu_grad(a1)
    dW1 = da1.T @ f
    db1 = da1.sum(axis=0)
    return dW1, db1, dW2, db2, dW3, db3


def adam_step(p, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba) with bias correction at step t >= 1.
    Returns (p', m', v')."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def coarse_cells(fine: np.ndarray, coarse: np.ndarray, tie: float = 1e-12) -> np.ndarray:
    """cell[q] = index c of the coarse direction closest to fine direction q
    (largest dot product of unit vectors; within ``tie`` the lowest c)."""
    fu = fine / np.linalg.norm(fine, axis=1, keepdims=True)
    cu = coarse / np.linalg.norm(coarse, axis=1, keepdims=True)
    cell = np.empty(fu.shape[0], dtype=np.int64)
    for a in range(0, fu.shape[0], 2048):
        d = fu[a:a + 2048] @ cu.T
        best = d.max(axis=1, keepdims=True)
        cell[a:a + 2048] = np.argmax(d >= best - tie, axis=1)
    return cell


def proposal_features(z: np.ndarray) -> np.ndarray:
    """Network input for projected vectors z [F, K] (complex, eq. (12) with S
    folded in): [Re z, Im z] / ||z||, 0 for z = 0."""
    f = np.concatenate([z.real, z.imag], axis=1)
    n = np.linalg.norm(f, axis=1, keepdims=True)
    return np.where(n > 0, f / np.where(n > 0, n, 1.0), 0.0)
