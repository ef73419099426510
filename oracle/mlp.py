"""FP64 reference of the warm-start network (test infrastructure).

Not part of the paper: the learned warm start of the dual PCGP is a system
pattern added around Algorithm 3.  A 3-layer perceptron with ReLU,

    h1 = relu(X W1^T + b1),  h2 = relu(h1 W2^T + b2),  Y = h2 W3^T + b3,

maps per-interface-node features to the change of that node's multiplier
rows between load steps.  The loss is the masked mean squared error

    L = 1/(2 N) sum_i sum_j M_ij (Y_ij - T_ij)^2

(M masks the zero-padded rows of nodes with fewer than 21 multipliers).
The GPU keeps weights and activations in bfloat16 with FP32 accumulation;
`bf16` rounds a float64 array the same way (round to nearest even on the
upper 16 bits of the float32 value) so the oracle can run on identical
inputs.  Parity of the oracle itself is pinned by central finite
differences of L (tests/test_oracle_mlp.py).
"""

from __future__ import annotations

import numpy as np

DIMS = (31, 256, 256, 21)


def bf16(x: np.ndarray) -> np.ndarray:
    """Round to bfloat16 (nearest, ties to even) and return float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def forward(p, X, round_bf16: bool = False):
    r = bf16 if round_bf16 else (lambda a: a)
    a1 = X @ p["W1"].T + p["b1"]
    h1 = r(np.maximum(a1, 0.0))
    a2 = h1 @ p["W2"].T + p["b2"]
    h2 = r(np.maximum(a2, 0.0))
    Y = h2 @ p["W3"].T + p["b3"]
    return Y, dict(X=X, a1=a1, h1=h1, a2=a2, h2=h2)


def loss(Y, T, M):
    N = Y.shape[0]
    return 0.5 * float(np.sum(M * (Y - T) ** 2)) / N


def backward(p, cache, Y, T, M):
    """Gradients of the masked MSE loss with respect to all parameters."""
    N = Y.shape[0]
    dY = M * (Y - T) / N
    g = {}
    g["W3"] = dY.T @ cache["h2"]
    g["b3"] = dY.sum(axis=0)
    dh2 = dY @ p["W3"]
    da2 = dh2 * (cache["a2"] > 0)
    g["W2"] = da2.T @ cache["h1"]
    g["b2"] = da2.sum(axis=0)
    dh1 = da2 @ p["W2"]
    da1 = dh1 * (cache["a1"] > 0)
    g["W1"] = da1.T @ cache["X"]
    g["b1"] = da1.sum(axis=0)
    return g


def adam(p, g, state, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma and Ba, 2015) in place; state holds m, v, t."""
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    for k in p:
        m = state.setdefault("m_" + k, np.zeros_like(p[k]))
        v = state.setdefault("v_" + k, np.zeros_like(p[k]))
        m[:] = b1 * m + (1 - b1) * g[k]
        v[:] = b2 * v + (1 - b2) * g[k] ** 2
        mh = m / (1 - b1 ** t)
        vh = v / (1 - b2 ** t)
        p[k] -= lr * mh / (np.sqrt(vh) + eps)
    return p
