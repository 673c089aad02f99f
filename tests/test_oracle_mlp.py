"""Pins of the MLP oracle: GELU closed form and derivative, loss gradients by
central differences, one Adam step by hand.  CPU only."""
import math

import numpy as np

from oracle import mlp


def test_gelu_closed_form_and_derivative():
    a = np.linspace(-5, 5, 41)
    # Phi(0) = 1/2, Phi(-inf) = 0: gelu(0) = 0, gelu(a) -> a for large a
    assert mlp.gelu(np.array([0.0]))[0] == 0.0
    assert abs(mlp.gelu(np.array([8.0]))[0] - 8.0) < 1e-12
    assert abs(mlp.gelu(np.array([1.0]))[0] - 0.8413447460685429) < 1e-15
    h = 1e-6
    fd = (mlp.gelu(a + h) - mlp.gelu(a - h)) / (2 * h)
    assert np.abs(fd - mlp.gelu_grad(a)).max() < 1e-8


def test_gradients_by_central_differences():
    rng = np.random.default_rng(0)
    sizes = [7, 11, 9, 5]
    Ws, bs = mlp.init_params(sizes, 1)
    X = rng.normal(size=(6, 7))
    T = rng.normal(size=(6, 5))
    loss, gW, gb = mlp.loss_and_grads(Ws, bs, X, T)
    h = 1e-6
    for l in range(len(Ws)):
        for (i, j) in [(0, 0), (2, 3), (sizes[l] - 1, sizes[l + 1] - 1)]:
            Wp = [w.copy() for w in Ws]
            Wm = [w.copy() for w in Ws]
            Wp[l][i, j] += h
            Wm[l][i, j] -= h
            fd = (mlp.loss_and_grads(Wp, bs, X, T)[0] - mlp.loss_and_grads(Wm, bs, X, T)[0]) / (2 * h)
            assert abs(fd - gW[l][i, j]) < 1e-7 * max(1.0, abs(fd))
        bp = [b.copy() for b in bs]
        bm = [b.copy() for b in bs]
        bp[l][1] += h
        bm[l][1] -= h
        fd = (mlp.loss_and_grads(Ws, bp, X, T)[0] - mlp.loss_and_grads(Ws, bm, X, T)[0]) / (2 * h)
        assert abs(fd - gb[l][1]) < 1e-7 * max(1.0, abs(fd))


def test_adam_first_step_is_sign_step():
    """With zero moments, the first bias-corrected Adam step is
    -lr * g / (|g| + eps), i.e. -lr * sign(g) for |g| >> eps."""
    g = np.array([0.5, -2.0, 1e-3])
    p, m, v = mlp.adam_step(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, lr=0.01)
    assert np.allclose(p, -0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)
