"""Pins of the float64 network oracle: gradients by central differences, the
no-hidden-layer case against linear least squares, the Cholesky target map."""
import numpy as np

from oracle import mlp
from paper_2107_10800_amd import workloads as W


def test_param_count():
    assert mlp.n_params() == 20245
    assert W.mlp_init_weights().size == 20245


def test_gradient_central_differences():
    sizes = (7, 8, 6, 21)
    rng = np.random.default_rng(0)
    flat = rng.standard_normal(mlp.n_params(sizes)) * 0.5
    X = rng.standard_normal((5, 7))
    T = rng.standard_normal((5, 21))
    loss, g = mlp.loss_and_grad(flat, X, T, sizes)
    h = 1e-6
    fd = np.zeros_like(flat)
    for k in range(len(flat)):
        e = np.zeros_like(flat)
        e[k] = h
        fd[k] = (mlp.loss_and_grad(flat + e, X, T, sizes)[0]
                 - mlp.loss_and_grad(flat - e, X, T, sizes)[0]) / (2 * h)
    assert np.abs(g - fd).max() <= 1e-7 * max(1.0, np.abs(fd).max())
    assert abs(loss - np.mean((mlp.forward(flat, X, sizes)[0] - T) ** 2)) == 0.0


def test_no_hidden_layer_is_least_squares():
    # with no hidden layer the network is affine: its MSE minimiser is the
    # least-squares solution, where the gradient vanishes
    sizes = (7, 21)
    rng = np.random.default_rng(1)
    X = rng.standard_normal((200, 7))
    T = X @ rng.standard_normal((7, 21)) + 0.1 * rng.standard_normal((200, 21))
    Xa = np.column_stack([X, np.ones(len(X))])
    sol, *_ = np.linalg.lstsq(Xa, T, rcond=None)
    flat = mlp.pack([(sol[:7].T, sol[7])])
    _, g = mlp.loss_and_grad(flat, X, T, sizes)
    assert np.abs(g).max() < 1e-12
    # Adam from zero approaches the same minimum
    f = np.zeros_like(flat)
    m = np.zeros_like(f)
    v = np.zeros_like(f)
    for t in range(1, 3001):
        _, gg = mlp.loss_and_grad(f, X, T, sizes)
        f, m, v = mlp.adam(f, gg, m, v, t, 1e-2)
    assert abs(mlp.loss_and_grad(f, X, T, sizes)[0]
               - mlp.loss_and_grad(flat, X, T, sizes)[0]) < 1e-6


def test_cholesky_target_round_trip():
    rng = np.random.default_rng(2)
    B = rng.standard_normal((4, 6, 6))
    Nt = B @ B.transpose(0, 2, 1) + 0.1 * np.eye(6)
    y = mlp.target_from_mobility(Nt, a=1.3, eta=0.7)
    back = mlp.mobility_from_output(y, a=1.3, eta=0.7)
    assert np.allclose(back, Nt, rtol=1e-12, atol=1e-13)
    # the diagonal is carried as log L_ii
    Sc = mlp.scaling(1.3, 0.7)
    L0 = np.linalg.cholesky(Sc[:, None] * Nt[0] * Sc[None, :])
    assert np.allclose(np.exp(y[0, mlp.DIAG]), np.diag(L0), rtol=1e-13)
    assert list(mlp.DIAG) == [0, 2, 5, 9, 14, 20]


def test_features_double_cover():
    th = np.array([[0.5, 0.5, 0.5, 0.5], [-0.5, 0.5, -0.5, 0.5]])
    x = mlp.features([3.0, 4.0], th, [0, 1])
    assert np.all(x[:, 1] >= 0)
    assert np.allclose(x[1, 1:5], [0.5, -0.5, 0.5, -0.5])
    assert np.allclose(x[:, 5:], [[1, 0], [0, 1]])


def test_adam_first_step_is_sign_descent():
    # with zero moments the bias-corrected first step is lr * g / (|g| + eps):
    # every weight moves by lr against the sign of its gradient
    rng = np.random.default_rng(3)
    flat = rng.standard_normal(50)
    g = rng.standard_normal(50) * np.logspace(-3, 2, 50)
    new, m, v = mlp.adam(flat, g, np.zeros(50), np.zeros(50), 1, lr=1e-2)
    assert np.allclose(new - flat, -1e-2 * np.sign(g), rtol=1e-4, atol=0)
    # a constant gradient keeps the step at lr (moments track g and g^2 exactly)
    new2, _, _ = mlp.adam(new, g, m, v, 2, lr=1e-2)
    assert np.allclose(new2 - new, -1e-2 * np.sign(g), rtol=1e-4, atol=0)


def test_adam_minimises_a_quadratic():
    rng = np.random.default_rng(4)
    A = rng.standard_normal((6, 6))
    H = A @ A.T + np.eye(6)
    xs = rng.standard_normal(6)
    x, m, v = np.zeros(6), np.zeros(6), np.zeros(6)
    for t in range(1, 3001):
        lr = 0.05 * (0.5 * (1 + np.cos(np.pi * t / 3000)) + 1e-3)
        x, m, v = mlp.adam(x, H @ (x - xs), m, v, t, lr=lr)
    assert np.linalg.norm(x - xs) <= 1e-3 * np.linalg.norm(xs)
