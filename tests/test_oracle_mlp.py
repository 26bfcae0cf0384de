"""Pins of the FP64 network reference: analytic gradients against central
finite differences (the definition of the derivative) and the closed form of
Adam's first bias-corrected step (each parameter moves by lr * sign(grad))."""
import numpy as np

from oracle import mlp


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(0)
    sizes = [7, 8, 8, 5]
    params = mlp.init_params(sizes, seed=1)
    for p in params[1::2]:
        p += rng.normal(size=p.shape) * 0.1
    x = rng.normal(size=(6, 7))
    t = rng.normal(size=(6, 5))
    y, cache = mlp.forward(params, x)
    grads = mlp.backward(params, cache, y, t)
    h = 1e-6
    for p, gp in zip(params, grads):
        flat = p.reshape(-1)
        gflat = gp.reshape(-1)
        for i in range(flat.size):
            old = flat[i]
            flat[i] = old + h
            lp = mlp.mse(mlp.forward(params, x)[0], t)
            flat[i] = old - h
            lm = mlp.mse(mlp.forward(params, x)[0], t)
            flat[i] = old
            fd = (lp - lm) / (2 * h)
            assert abs(fd - gflat[i]) < 1e-7 * max(1.0, abs(fd))


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(2)
    p = [rng.normal(size=(4, 3))]
    g = [rng.normal(size=(4, 3))]
    m = [np.zeros((4, 3))]
    v = [np.zeros((4, 3))]
    p0 = p[0].copy()
    mlp.adam_step(p, g, m, v, step=1, lr=1e-2, eps=0.0)
    assert np.allclose(p[0], p0 - 1e-2 * np.sign(g[0]), rtol=0, atol=1e-15)
