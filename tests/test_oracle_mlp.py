"""Pins for the fp64 cost-model MLP reference (no GPU): analytic gradients
against central finite differences, closed forms of the forward pass and of
the first Adam step (Kingma & Ba 2015, Algorithm 1)."""
import numpy as np

import oracle


def _params(rng, K=6, scale=0.5):
    return {"W1": rng.normal(0, scale, (4, 64)), "b1": rng.normal(0, 0.1, 64),
            "W2": rng.normal(0, scale / 4, (64, 64)), "b2": rng.normal(0, 0.1, 64),
            "W3": rng.normal(0, scale / 4, (64, K)), "b3": rng.normal(0, 0.1, K)}


def test_forward_closed_forms():
    rng = np.random.default_rng(1)
    p = _params(rng)
    for k in ("W1", "W2", "W3"):
        p[k] = np.zeros_like(p[k])
    X = rng.normal(size=(5, 4))
    out, _ = oracle.mlp_forward(p, X)
    np.testing.assert_array_equal(out, np.tile(p["b3"], (5, 1)))
    # one hidden unit on, identity-like path: out = relu(x0) * a * b
    p = {k: np.zeros_like(v) for k, v in _params(rng).items()}
    p["W1"][0, 0] = 1.0
    p["W2"][0, 0] = 2.0
    p["W3"][0, 1] = 3.0
    X = np.array([[1.5, 0, 0, 0], [-2.0, 0, 0, 0]])
    out, _ = oracle.mlp_forward(p, X)
    np.testing.assert_allclose(out[:, 1], [1.5 * 6.0, 0.0])


def test_loss_mask():
    out = np.array([[1.0, 2.0], [3.0, 4.0]])
    T = np.array([[0.0, 0.0], [0.0, 0.0]])
    mask = np.array([[1, 0], [0, 1]])
    assert oracle.mlp_loss(out, T, mask) == (1.0 + 16.0) / 2
    assert oracle.mlp_loss(out, T, np.zeros((2, 2))) == 0.0


def test_gradients_vs_finite_differences():
    rng = np.random.default_rng(2)
    p = _params(rng)
    X = rng.normal(size=(9, 4))
    T = rng.normal(size=(9, 6))
    mask = (rng.random((9, 6)) < 0.7).astype(np.float64)
    out, cache = oracle.mlp_forward(p, X)
    g = oracle.mlp_backward(p, cache, out, T, mask)
    eps = 1e-6
    for key, val in p.items():
        flat = val.reshape(-1)
        idx = rng.choice(flat.size, size=min(flat.size, 25), replace=False)
        for i in idx:
            old = flat[i]
            flat[i] = old + eps
            lp = oracle.mlp_loss(oracle.mlp_forward(p, X)[0], T, mask)
            flat[i] = old - eps
            lm = oracle.mlp_loss(oracle.mlp_forward(p, X)[0], T, mask)
            flat[i] = old
            fd = (lp - lm) / (2 * eps)
            an = g[key].reshape(-1)[i]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)), (key, i, fd, an)


def test_adam_first_step_closed_form():
    # t = 1: mhat = g, vhat = g^2, so the step is lr * g / (|g| + eps)
    rng = np.random.default_rng(3)
    p = _params(rng)
    g = {k: rng.normal(size=v.shape) for k, v in p.items()}
    z = {k: np.zeros_like(v) for k, v in p.items()}
    newp, m, v = oracle.adam_step(p, g, z, z, 1, lr=0.01)
    for k in p:
        np.testing.assert_allclose(newp[k], p[k] - 0.01 * g[k] / (np.abs(g[k]) + 1e-8), rtol=1e-10, atol=1e-15)
        np.testing.assert_allclose(m[k], 0.1 * g[k])
        np.testing.assert_allclose(v[k], 0.001 * g[k] ** 2)


def test_training_reduces_loss():
    rng = np.random.default_rng(4)
    p = _params(rng)
    X = rng.normal(size=(64, 4))
    T = np.stack([X[:, 0] * 2 - X[:, 1], X[:, 2] ** 2], axis=1)
    p["W3"] = p["W3"][:, :2]
    p["b3"] = p["b3"][:2]
    mask = np.ones_like(T)
    m = {k: np.zeros_like(v) for k, v in p.items()}
    v = {k: np.zeros_like(val) for k, val in p.items()}
    first = None
    for t in range(1, 301):
        out, cache = oracle.mlp_forward(p, X)
        loss = oracle.mlp_loss(out, T, mask)
        first = loss if first is None else first
        g = oracle.mlp_backward(p, cache, out, T, mask)
        p, m, v = oracle.adam_step(p, g, m, v, t, lr=3e-3)
    assert loss < 0.2 * first
