"""Pins of the FP64 surrogate-network reference: gradients vs central
differences and an Adam step vs its textbook update."""
import numpy as np

from oracle import mlp


def test_mlp_gradients_match_central_differences():
    layers = (6, 7, 5, 4, 1)
    params = mlp.init_params(3, layers)
    rng = np.random.default_rng(0)
    x = rng.normal(size=(9, 6))
    y = rng.normal(size=9)
    _, grads = mlp.loss_and_grads(params, x, y)
    h = 1e-6
    for k, P in enumerate(params):
        flat = P.reshape(-1)
        for j in range(0, flat.size, max(1, flat.size // 7)):
            old = flat[j]
            flat[j] = old + h
            lp, _ = mlp.loss_and_grads(params, x, y)
            flat[j] = old - h
            lm, _ = mlp.loss_and_grads(params, x, y)
            flat[j] = old
            fd = (lp - lm) / (2 * h)
            assert abs(fd - grads[k].reshape(-1)[j]) <= 1e-7 * max(1.0, abs(fd))


def test_mlp_forward_shapes_and_silu():
    params = mlp.init_params(1)
    assert [p.shape for p in params] == [(256, 6), (256,), (256, 256), (256,), (256, 256), (256,), (1, 256), (1,)]
    assert sum(p.size for p in params) == 133633
    z = np.array([-3.0, 0.0, 2.0])
    assert np.allclose(mlp.silu(z), z / (1 + np.exp(-z)))
    assert mlp.silu(np.array([0.0]))[0] == 0.0


def test_adam_first_step_moves_by_lr():
    """With bias correction the first Adam step is lr * g/|g| per element."""
    params = [np.array([1.0, -2.0, 3.0])]
    grads = [np.array([0.5, -4.0, 1e-3])]
    m = [np.zeros(3)]
    v = [np.zeros(3)]
    mlp.adam_step(params, grads, m, v, 1, lr=0.01, eps=0.0)
    assert np.allclose(params[0], [1.0 - 0.01, -2.0 + 0.01, 3.0 - 0.01])
