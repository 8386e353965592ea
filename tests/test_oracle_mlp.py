"""Pins of the FP64 perceptron oracle: finite differences, Adam's first step,
and a loss that decreases on a learnable toy problem."""
import numpy as np

import gwsynth
from oracle import mlp


def _params(n_in=5, width=7, n_out=3, seed=1):
    p = gwsynth.mlp_init(n_in, width, n_out, seed=seed)
    rng = np.random.default_rng(seed)
    p["b1"] = rng.standard_normal(width) * 0.1
    p["b2"] = rng.standard_normal(width) * 0.1
    p["b3"] = rng.standard_normal(n_out) * 0.1
    p["W3"] = p["W3"] * 10
    return p


def test_silu_derivative_finite_difference():
    z = np.linspace(-6, 6, 101)
    h = 1e-6
    fd = (mlp.silu(z + h) - mlp.silu(z - h)) / (2 * h)
    np.testing.assert_allclose(mlp.dsilu(z), fd, rtol=1e-8, atol=1e-10)


def test_gradients_finite_difference():
    rng = np.random.default_rng(2)
    p = _params()
    x = rng.standard_normal((11, 5))
    t = rng.standard_normal((11, 3))
    mask = (rng.uniform(size=(11, 3)) > 0.2).astype(float)
    y, cache = mlp.forward(p, x, keep=True)
    L, dy = mlp.loss(y, t, mask)
    g, dx = mlp.backward(p, cache, dy)
    h = 1e-6
    for name in p:
        flat = p[name].reshape(-1)
        for idx in rng.choice(flat.size, size=min(6, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + h
            Lp = mlp.loss(mlp.forward(p, x), t, mask)[0]
            flat[idx] = old - h
            Lm = mlp.loss(mlp.forward(p, x), t, mask)[0]
            flat[idx] = old
            fd = (Lp - Lm) / (2 * h)
            assert abs(g[name].reshape(-1)[idx] - fd) <= 1e-6 * max(1.0, abs(fd)), name
    # input gradient
    for (r, c) in [(0, 0), (3, 4), (10, 2)]:
        old = x[r, c]
        x[r, c] = old + h
        Lp = mlp.loss(mlp.forward(p, x), t, mask)[0]
        x[r, c] = old - h
        Lm = mlp.loss(mlp.forward(p, x), t, mask)[0]
        x[r, c] = old
        assert abs(dx[r, c] - (Lp - Lm) / (2 * h)) <= 1e-6


def test_adam_first_step_is_signed_lr():
    # With bias correction, the first Adam step is lr * g / (|g| + eps') ~ lr * sign(g).
    p = {"a": np.array([1.0, -2.0, 3.0])}
    g = {"a": np.array([0.5, -1e-3, 40.0])}
    m = {"a": np.zeros(3)}
    v = {"a": np.zeros(3)}
    p2, m, v = mlp.adam_step(dict(p), g, m, v, step=1, lr=0.01, eps=1e-12)
    np.testing.assert_allclose(p2["a"], p["a"] - 0.01 * np.sign(g["a"]), rtol=0, atol=1e-10)


def test_training_reduces_loss():
    rng = np.random.default_rng(4)
    p = gwsynth.mlp_init(3, 16, 1, seed=3)
    x = rng.uniform(-1, 1, (256, 3))
    t = (np.sin(2 * x[:, :1]) + x[:, 1:2] * x[:, 2:3])
    m = {k: np.zeros_like(a) for k, a in p.items()}
    v = {k: np.zeros_like(a) for k, a in p.items()}
    L0 = None
    for step in range(1, 301):
        y, cache = mlp.forward(p, x, keep=True)
        L, dy = mlp.loss(y, t)
        if L0 is None:
            L0 = L
        g, _ = mlp.backward(p, cache, dy)
        p, m, v = mlp.adam_step(p, g, m, v, step, lr=3e-3)
    assert L < 0.1 * L0


def test_bf16_rounding_known_values():
    from oracle.precision import round_bf16, split_bf16
    # 1 + 2^-8 is halfway between 1 and 1 + 2^-7: ties to even -> 1
    x = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, 1 + 2 ** -7 + 2 ** -20, -2.5, 3.0e38, 1e-40],
                 dtype=np.float32)
    r = round_bf16(x)
    assert r[0] == 1.0 and r[1] == 1.0 and r[2] == np.float32(1 + 2 ** -6)
    assert r[3] == np.float32(1 + 2 ** -7) and r[4] == -2.5
    # bf16 has 8 significant bits: unit roundoff 2^-8
    rng = np.random.default_rng(0)
    y = rng.standard_normal(10000).astype(np.float32) * 10.0 ** rng.uniform(-5, 5, 10000)
    assert np.all(np.abs(round_bf16(y) - y) <= 2.0 ** -8 * np.abs(y))
    hi, lo = split_bf16(y)
    assert np.all(np.abs(y.astype(np.float64) - hi - lo) <= 2.0 ** -16 * np.abs(y))
