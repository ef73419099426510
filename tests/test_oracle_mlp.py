"""Pins of the oracle MLP: analytic gradients equal central finite
differences of the loss, bf16 rounding matches the bfloat16 definition, and
Adam reduces the loss on a fixed batch."""

import numpy as np

from oracle import mlp
import workloads


def small_problem(seed=0, n=12):
    rng = np.random.default_rng(seed)
    dims = (5, 7, 6, 4)
    p = workloads.mlp_init(seed, dims)
    for k in p:
        if k.startswith("b"):
            p[k] = rng.standard_normal(p[k].shape) * 0.1
    X = rng.standard_normal((n, dims[0]))
    T = rng.standard_normal((n, dims[-1]))
    M = (rng.random((n, dims[-1])) > 0.3).astype(float)
    return p, X, T, M


def test_gradients_match_finite_differences():
    p, X, T, M = small_problem()
    Y, cache = mlp.forward(p, X)
    g = mlp.backward(p, cache, Y, T, M)
    h = 1e-6
    for k in p:
        flat = p[k].ravel()
        for idx in range(flat.size):
            old = flat[idx]
            flat[idx] = old + h
            lp = mlp.loss(mlp.forward(p, X)[0], T, M)
            flat[idx] = old - h
            lm = mlp.loss(mlp.forward(p, X)[0], T, M)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            assert abs(fd - g[k].ravel()[idx]) <= 1e-7 * max(1.0, abs(fd)), (k, idx)


def test_bf16_rounding_definition():
    # exactly representable values are unchanged; halfway cases round to even
    vals = np.array([1.0, -2.5, 0.15625, 2.0 ** 100])
    assert np.array_equal(mlp.bf16(vals), vals.astype(np.float32).astype(np.float64))
    one = np.float32(1.0).view(np.uint32)
    up = np.array([one + 0x8000], dtype=np.uint32).view(np.float32)       # 1 + 2^-8, a tie
    assert mlp.bf16(up.astype(np.float64))[0] == 1.0                      # ties to even (down)
    up2 = np.array([one + 0x18000], dtype=np.uint32).view(np.float32)     # 1 + 3*2^-8, a tie
    assert mlp.bf16(up2.astype(np.float64))[0] == float(np.array([one + 0x20000], dtype=np.uint32).view(np.float32)[0])
    x = np.random.default_rng(1).standard_normal(1000)
    rel = np.abs(mlp.bf16(x) - x) / np.abs(x)
    assert rel.max() <= 2.0 ** -8


def test_adam_reduces_loss():
    p, X, T, M = small_problem(3, n=64)
    st = {}
    l0 = mlp.loss(mlp.forward(p, X)[0], T, M)
    for _ in range(200):
        Y, c = mlp.forward(p, X)
        mlp.adam(p, mlp.backward(p, c, Y, T, M), st, lr=1e-2)
    assert mlp.loss(mlp.forward(p, X)[0], T, M) < 0.5 * l0


def _two_steps(adam, lr=1e-3, eps=1e-8):
    """A scalar parameter theta = 0 driven by the gradients +1, then -1."""
    p = {"w": np.zeros(1)}
    st = {}
    adam(p, {"w": np.array([1.0])}, st, lr=lr, b1=0.9, b2=0.999, eps=eps)
    t1 = p["w"][0]
    adam(p, {"w": np.array([-1.0])}, st, lr=lr, b1=0.9, b2=0.999, eps=eps)
    return t1, p["w"][0]


def test_adam_closed_form_first_two_steps():
    """Adam (Kingma and Ba 2015, Algorithm 1) from zero moments.  Step 1: the
    bias-corrected moments are g and g^2, so theta moves by -lr g/(|g| + eps),
    i.e. -lr for g = 1.  Step 2 with g = -1: m = 0.9*0.1 - 0.1 = -0.01 and
    m_hat = -0.01/(1 - 0.81) = -1/19; v = 0.999*0.001 + 0.001 = 0.001999 and
    v_hat = 0.001999/(1 - 0.998001) = 1, so theta moves by +lr/19.  Variants
    without the bias correction, or with beta1 and beta2 swapped, move
    differently and fail the same check."""
    lr, eps = 1e-3, 1e-8
    t1, t2 = _two_steps(mlp.adam, lr, eps)
    assert abs(t1 - (-lr / (1.0 + eps))) <= 1e-15
    assert abs(t2 - (t1 + lr * (1.0 / 19.0) / (1.0 + eps))) <= 1e-15

    def no_bias_correction(p, g, state, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        for k in p:
            m = state.setdefault("m_" + k, np.zeros_like(p[k]))
            v = state.setdefault("v_" + k, np.zeros_like(p[k]))
            m[:] = b1 * m + (1 - b1) * g[k]
            v[:] = b2 * v + (1 - b2) * g[k] ** 2
            p[k] -= lr * m / (np.sqrt(v) + eps)

    def swapped_betas(p, g, state, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        return mlp.adam(p, g, state, lr=lr, b1=b2, b2=b1, eps=eps)

    for bad in (no_bias_correction, swapped_betas):
        b1_, b2_ = _two_steps(bad, lr, eps)
        assert abs(b1_ - t1) > 1e-6 or abs(b2_ - t2) > 1e-6
