"""Pin of the oracle network gradient by central finite differences."""
import numpy as np

from oracle import mlp


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(0)
    n_in, h, n_out, rows = 7, 6, 5, 4
    n = n_in * h + h + h * h + h + h * n_out + n_out
    theta = rng.standard_normal(n) * 0.5
    X = rng.standard_normal((rows, n_in))
    T = rng.standard_normal((rows, n_out))
    loss, g = mlp.loss_and_grad(theta, X, T, n_in, h, n_out)
    eps = 1e-6
    num = np.zeros(n)
    for i in range(n):
        tp, tm = theta.copy(), theta.copy()
        tp[i] += eps
        tm[i] -= eps
        num[i] = (mlp.loss_and_grad(tp, X, T, n_in, h, n_out)[0] - mlp.loss_and_grad(tm, X, T, n_in, h, n_out)[0]) / (2 * eps)
    assert np.linalg.norm(num - g) / np.linalg.norm(g) < 1e-6


def test_forward_relu_structure():
    n_in, h, n_out = 3, 4, 2
    n = n_in * h + h + h * h + h + h * n_out + n_out
    theta = np.zeros(n)
    theta[-n_out:] = [1.5, -2.0]          # b3 only
    Y, _ = mlp.forward(theta, np.ones((5, n_in)), n_in, h, n_out)
    assert np.allclose(Y, [[1.5, -2.0]] * 5)
