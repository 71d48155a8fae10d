"""Pins of the FP64 refinement-network oracle (oracle/mlp.py)."""
import math

import numpy as np
import pytest

from oracle import mlp


@pytest.fixture(scope="module")
def setup():
    rng = np.random.default_rng(0)
    q = rng.uniform(0, 1, size=(64, 3))
    target = 0.05 * rng.standard_normal((64, 3))
    B = mlp.rff_matrix(8.0, seed=1)
    p = mlp.init_params(seed=2)
    return q, target, B, p


def test_shapes_and_parameter_count(setup):
    q, target, B, p = setup
    assert sum(v.size for v in p.values()) == 66435
    assert np.all(B == np.rint(B))
    pred, _ = mlp.forward(p, q, B)
    assert pred.shape == (64, 3)


def test_features_are_periodic(setup):
    q, _, B, _ = setup
    np.testing.assert_allclose(mlp.features(q, B), mlp.features(q + np.array([1.0, -2.0, 3.0]), B),
                               atol=1e-10)


def test_gelu_matches_definition_and_derivative():
    x = np.linspace(-6, 6, 101)
    from scipy.stats import norm
    np.testing.assert_allclose(mlp.gelu(x), x * norm.cdf(x), atol=1e-14)
    h = 1e-6
    np.testing.assert_allclose(mlp.gelu_grad(x), (mlp.gelu(x + h) - mlp.gelu(x - h)) / (2 * h),
                               atol=1e-8)


def test_backward_matches_central_differences(setup):
    q, target, B, p = setup
    _, g = mlp.loss_and_grad(p, q, target, B)
    rng = np.random.default_rng(5)
    h = 1e-6
    for name in mlp.NAMES:
        for _ in range(4):
            idx = tuple(rng.integers(0, s) for s in p[name].shape)
            old = p[name][idx]
            p[name][idx] = old + h
            lp = mlp.loss(mlp.forward(p, q, B)[0], target)
            p[name][idx] = old - h
            lm = mlp.loss(mlp.forward(p, q, B)[0], target)
            p[name][idx] = old
            fd = (lp - lm) / (2 * h)
            assert abs(fd - g[name][idx]) <= 1e-7 * max(1.0, abs(fd)) + 1e-9, (name, idx, fd, g[name][idx])


def test_backward_matches_torch_autograd_fp64(setup):
    torch = pytest.importorskip("torch")
    q, target, B, p = setup
    _, g = mlp.loss_and_grad(p, q, target, B)
    tp = {k: torch.tensor(v, dtype=torch.float64, requires_grad=True) for k, v in p.items()}
    h = torch.tensor(mlp.features(q, B), dtype=torch.float64)
    for i in range(1, 5):
        h = torch.nn.functional.gelu(h @ tp[f"W{i}"].T + tp[f"b{i}"])
    out = h @ tp["W5"].T + tp["b5"]
    L = ((out - torch.tensor(target)) ** 2).sum(dim=1).mean()
    L.backward()
    for k in mlp.NAMES:
        np.testing.assert_allclose(g[k], tp[k].grad.numpy(), rtol=1e-10, atol=1e-13)


def test_zero_output_layer_bias_gradient_closed_form(setup):
    q, target, B, p = setup
    p = {k: v.copy() for k, v in p.items()}
    p["W5"][:] = 0.0
    _, g = mlp.loss_and_grad(p, q, target, B)
    expect = 2.0 * (p["b5"][None, :] - target).mean(axis=0)
    np.testing.assert_allclose(g["b5"], expect, rtol=1e-12)
    for i in range(1, 5):
        assert np.all(g[f"W{i}"] == 0.0)


def test_adam_first_step_is_lr_times_sign():
    # with zero moments the bias-corrected first step is -lr * g / (|g| + eps)
    p = {k: np.ones(3) for k in mlp.NAMES}
    g = {k: np.array([2.0, -0.5, 1e-3]) for k in mlp.NAMES}
    m = {k: np.zeros(3) for k in mlp.NAMES}
    v = {k: np.zeros(3) for k in mlp.NAMES}
    mlp.adam_step(p, g, m, v, t=1, lr=0.01)
    for k in mlp.NAMES:
        np.testing.assert_allclose(p[k], 1.0 - 0.01 * g[k] / (np.abs(g[k]) + 1e-8), rtol=1e-12)


def test_training_reduces_loss_on_a_smooth_field():
    rng = np.random.default_rng(3)
    q = rng.uniform(0, 1, size=(256, 3))
    target = 0.05 * np.stack([np.sin(2 * np.pi * q[:, 0]), np.cos(2 * np.pi * q[:, 1]),
                              np.sin(2 * np.pi * (q[:, 0] + q[:, 2]))], axis=1)
    B = mlp.rff_matrix(2.0, seed=1)
    p = mlp.init_params(seed=2)
    m = {k: np.zeros_like(v) for k, v in p.items()}
    v = {k: np.zeros_like(x) for k, x in p.items()}
    l0 = mlp.loss(mlp.forward(p, q, B)[0], target)
    for t in range(1, 151):
        _, g = mlp.loss_and_grad(p, q, target, B)
        mlp.adam_step(p, g, m, v, t, lr=mlp.cosine_lr(t, 150, 3e-3, 1e-4))
    l1 = mlp.loss(mlp.forward(p, q, B)[0], target)
    assert l1 < 0.05 * l0


def test_minimal_image_range():
    d = np.array([-0.75, -0.5, -0.25, 0.0, 0.5, 0.75])
    np.testing.assert_allclose(mlp.minimal_image(d), [0.25, 0.5, -0.25, 0.0, 0.5, -0.25])
