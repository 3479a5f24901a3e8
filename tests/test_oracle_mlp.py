"""Pins of the closure network's FP64 oracle (no GPU): the analytic gradient
against central finite differences, the first Adam step against its closed
form, and the features/targets against their definitions in moment space."""
import numpy as np
import pytest


@pytest.fixture(scope="module")
def mlp():
    import oracle.mlp as m
    return m


def _data(mlp, B=16, seed=0):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(B, mlp.NIN))
    T = rng.normal(size=(B, mlp.NREG))
    flag = rng.integers(0, 2, B)
    p = mlp.init(rng.uniform(-1, 1, mlp.NPARAM)) + 0.05 * rng.normal(size=mlp.NPARAM)
    return p, X, T, flag


def test_sizes(mlp):
    assert mlp.NPARAM == 64 * 10 + 64 + 64 * 64 + 64 + 8 * 64 + 8 == 5384


def test_gradient_matches_finite_differences(mlp):
    p, X, T, flag = _data(mlp)
    loss, g = mlp.loss_grad(p, X, T, flag)
    rng = np.random.default_rng(1)
    idx = rng.choice(mlp.NPARAM, 60, replace=False)
    h = 1e-6
    for k in idx:
        e = np.zeros_like(p)
        e[k] = h
        fd = (mlp.loss_grad(p + e, X, T, flag)[0] - mlp.loss_grad(p - e, X, T, flag)[0]) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1e-3, abs(g[k])) + 1e-9, (k, fd, g[k])


def test_loss_pieces(mlp):
    # zero network: MSE = mean(T^2), cross-entropy = log 2
    p = np.zeros(mlp.NPARAM)
    _, X, T, flag = _data(mlp)
    loss, _ = mlp.loss_grad(p, X, T, flag)
    assert abs(loss - (np.mean(np.sum(T * T, axis=1) / 6) + np.log(2))) < 1e-12


def test_first_adam_step(mlp):
    # with bias correction the first step is -lr * g / (|g| + eps)
    rng = np.random.default_rng(2)
    p, g = rng.normal(size=50), rng.normal(size=50)
    p1, m, v = mlp.adam(p, g, np.zeros(50), np.zeros(50), 1, lr=1e-3)
    np.testing.assert_allclose(p1, p - 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12)


def test_features_and_targets(oracle, mlp):
    # an equilibrium node has zero non-equilibrium features and targets
    f9 = oracle.equilibrium(3, 2, 1.1, 0.03, -0.02)
    x = mlp.features(oracle, f9, 0.1)
    np.testing.assert_allclose(x[:4], [0.1, 0.03, -0.02, np.log(0.1)], atol=1e-14)
    assert np.max(np.abs(x[4:])) < 1e-15
    f36 = oracle.equilibrium(6, 4, 1.1, 0.03, -0.02)
    assert np.max(np.abs(mlp.targets(oracle, f36))) < 1e-15
    # the closure coefficients enter the lift exactly where D2Q9 lacks them
    rng = np.random.default_rng(3)
    y = rng.normal(size=6)
    c = mlp.closure_coeffs(y, np.zeros(6), np.ones(6), 1.1)
    up = oracle.project(3, 2, 6, 4, f9, c)
    back = mlp.targets(oracle, up)
    np.testing.assert_allclose(back, y, atol=1e-13)
