"""Pins for the learned-start oracle (descriptors, network, gradients, Adam)."""

import math

import numpy as np

from oracle import mlp


def test_descriptors_match_brute_force_image_sum():
    n, a = 6, 5.0
    pos = np.array([[0.3, 4.6, 2.2], [2.9, 1.1, 4.9]])
    w = mlp.widths(4, 0.5, 4.0)
    d = mlp.descriptors(n, a, pos, w)
    h = a / n
    rng = np.random.default_rng(1)
    for idx in rng.choice(n ** 3, 6, replace=False):
        x = np.array([idx % n, (idx // n) % n, idx // (n * n)]) * h
        for k, wk in enumerate(w):
            s = 0.0
            reach = int(math.ceil(wk * 10 / a)) + 1
            for p in pos:
                for l1 in range(-reach, reach + 1):
                    for l2 in range(-reach, reach + 1):
                        for l3 in range(-reach, reach + 1):
                            r = x - p - a * np.array([l1, l2, l3])
                            s += math.exp(-(r @ r) / (2 * wk * wk))
            assert abs(d[idx, k] - s) < 1e-12 * max(1.0, s)
    np.testing.assert_allclose(w[[0, -1]], [0.5, 4.0])
    assert np.allclose(w[1:] / w[:-1], w[1] / w[0])


def test_activation_derivatives():
    z = np.linspace(-30, 30, 301)
    d = 1e-6
    np.testing.assert_allclose(mlp.silu_grad(z), (mlp.silu(z + d) - mlp.silu(z - d)) / (2 * d),
                               atol=1e-8)
    np.testing.assert_allclose(mlp.softplus(np.array([-800.0, 0.0, 800.0])),
                               [0.0, math.log(2.0), 800.0], atol=1e-300)


def test_gradient_matches_central_differences():
    shapes = mlp.layer_shapes(5, 7, 3)
    theta = mlp.init_params(shapes, 3)
    rng = np.random.default_rng(4)
    u = rng.standard_normal((40, 5))
    t = rng.uniform(0.5, 2.0, 40)
    loss, g = mlp.loss_and_grad(theta, shapes, u, t)
    assert g.shape == theta.shape == (mlp.param_count(shapes),)
    for i in rng.choice(len(theta), 25, replace=False):
        e = np.zeros_like(theta)
        e[i] = 1e-6
        num = (mlp.loss_and_grad(theta + e, shapes, u, t)[0] -
               mlp.loss_and_grad(theta - e, shapes, u, t)[0]) / 2e-6
        assert abs(g[i] - num) < 1e-7 * max(1e-3, abs(num)), i


def test_first_adam_step_closed_form():
    rng = np.random.default_rng(6)
    theta = rng.standard_normal(10)
    g = rng.standard_normal(10) * 1e-3
    new, m, v = mlp.adam_step(theta, np.zeros(10), np.zeros(10), g, 1, lr=1e-3)
    np.testing.assert_allclose(new, theta - 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12)


def test_density_is_normalised():
    shapes = mlp.layer_shapes(4, 8, 2)
    theta = mlp.init_params(shapes, 9)
    u = np.random.default_rng(2).standard_normal((216, 4))
    rho = mlp.density(theta, shapes, u, 12.0, 0.5)
    assert abs(0.5 ** 3 * rho.sum() - 12.0) < 1e-12 and rho.min() > 0
