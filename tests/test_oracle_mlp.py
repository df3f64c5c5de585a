"""Pins of the preconditioner network oracle (oracle/mlp.py): backpropagation
against central finite differences, closed forms of a network reduced to its
output bias, the first Adam step, and the block target/feature definitions."""
import numpy as np

from oracle import mlp
from paper_1408_5092_amd import inputs


def _data(seed, n=37):
    rng = np.random.default_rng(seed)
    X = rng.normal(0.0, 1.0, (n, mlp.F))
    t = np.exp(rng.normal(0.0, 0.5, n))
    return X, t


def test_gradient_matches_finite_differences():
    p = inputs.mlp_init(3).astype(np.float64)
    p += np.random.default_rng(4).normal(0.0, 0.05, p.shape)  # nonzero biases too
    X, t = _data(5)
    L, g = mlp.loss_and_grad(p, X, t)
    assert abs(L - mlp.loss(p, X, t)) < 1e-14
    rng = np.random.default_rng(6)
    idx = np.concatenate([rng.choice(mlp.N_PARAMS, 60, replace=False), [0, 512, 576, 4672, 4736, 4800]])
    h = 1e-6
    for k in idx:
        e = np.zeros_like(p)
        e[k] = h
        fd = (mlp.loss(p + e, X, t) - mlp.loss(p - e, X, t)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-7 + 1e-5 * abs(g[k]), k


def test_output_bias_only_closed_form():
    p = np.zeros(mlp.N_PARAMS)
    b3 = 0.3
    p[-1] = b3
    X, t = _data(7)
    s = np.log1p(np.exp(b3))
    r = np.log(s) - np.log(t)
    L, g = mlp.loss_and_grad(p, X, t)
    assert abs(L - np.mean(r ** 2)) < 1e-14
    sig = 1.0 / (1.0 + np.exp(-b3))
    assert abs(g[-1] - np.mean(2.0 * r) * sig / s) < 1e-14
    # with zero weights only the output bias and the last layer's weights can move
    assert np.all(g[:-65] == 0.0)


def test_initial_scale_is_jacobi():
    p = inputs.mlp_init(0).astype(np.float64)
    p[:-1] = 0.0
    assert abs(mlp.forward(p, np.zeros((3, mlp.F))) - 1.0).max() < 1e-7  # float32 bias


def test_first_adam_step():
    p = np.ones(5)
    g = np.array([0.5, -2.0, 1e-3, 0.0, 3.0])
    p1, m, v = mlp.adam_step(p, np.zeros(5), np.zeros(5), g, 1, 0.01)
    # bias-corrected first step: lr * g / (|g| + eps)
    np.testing.assert_allclose(p1, p - 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)


def test_block_target_and_features():
    rng = np.random.default_rng(8)
    d = np.exp(rng.normal(0.0, 1.0, (3, 5)))
    b = rng.normal(0.0, 1.0, (3, 5))
    e0 = 1.7 * (b / d)
    assert abs(mlp.block_target(d, b, e0) - 1.7) < 1e-14
    assert mlp.block_target(d, np.zeros((3, 5)), e0) is None
    f = mlp.block_features(np.full((2, 4), 3.0), b[:2, :4], 2.0 * np.linalg.norm(b[:2, :4]), 5, 12)
    np.testing.assert_allclose(f, [np.log(3.0), 0.0, 0.0, 0.0, np.log(2), np.log(4), -np.log(2.0), 0.5],
                               rtol=0, atol=1e-14)
