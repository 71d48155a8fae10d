"""Pins of the FP64 refinement-network oracle (oracle/mlp.py)."""
import math

import numpy as np
import pytest

from oracle import mlp
import workloads as W


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


# ------------------------------------------------------- bf16 operands
def test_bf16_round_known_values_and_ties_to_even():
    v = np.array([1.0, 1.0 + 2.0 ** -8, 1.0 + 2.0 ** -9, 1.0 + 3 * 2.0 ** -9, -2.5, 0.0, 3.0e38])
    got = mlp.bf16_round(v)
    # bf16 keeps 7 stored bits: the spacing at 1 is 2^-7, so 1 + 2^-8 is the
    # halfway point and rounds to the even neighbour, 1.0
    assert got[0] == 1.0 and got[1] == 1.0 and got[2] == 1.0
    assert got[3] == 1.0 + 2.0 ** -7      # above halfway: up
    assert got[4] == -2.5 and got[5] == 0.0
    assert np.isfinite(got[6]) and abs(got[6] - 3.0e38) / 3.0e38 < 2.0 ** -8


def test_bf16_round_matches_torch_conversion():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(5)
    a = (rng.standard_normal(20000) * np.exp(rng.uniform(-20, 20, 20000))).astype(np.float32)
    ref = torch.from_numpy(a).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(mlp.bf16_round(a), ref)


def test_bf16_forward_rounds_the_product_operands(setup):
    # the activations the bf16 mode feeds to the products are bf16 values,
    # and the output moves by about the operands' rounding (2^-9 relative)
    q, target, B, p = setup
    out64, _ = mlp.forward(p, q, B)
    out16, (hs, _) = mlp.forward(p, q, B, operands="bf16")
    for h in hs:
        np.testing.assert_array_equal(h, mlp.bf16_round(h))
    rel = np.linalg.norm(out16 - out64) / np.linalg.norm(out64)
    assert 1e-5 < rel < 3e-2, rel


# ------------------------------------------------------------ placement
def test_barycentric_coordinates_in_the_table():
    rng = np.random.default_rng(7)
    p = rng.uniform(0, 1, size=(5000, 3))
    tet, lam = mlp.barycentric_in_table(p)
    assert np.all(tet >= 0)
    np.testing.assert_allclose(lam.sum(axis=1), 1.0, atol=1e-12)
    assert lam.min() >= -1e-12
    rec = np.zeros_like(p)
    for m in range(4):
        corners = np.array([mlp.corner_offset(mlp.TET_TABLE[t][m]) for t in tet])
        rec += lam[:, m:m + 1] * corners
    np.testing.assert_allclose(rec, p, atol=1e-12)


def test_placement_of_an_undisplaced_lattice():
    # raw with s = 0 and hybrid with any constant s put every fine tracer at
    # its Lagrangian point; coarse tracers keep their data
    n, r = 4, 3
    xyz = [np.asarray(a) for a in W.undisplaced(n)]
    q = mlp.fine_points((n, n, n), r).astype(np.float64)
    raw = mlp.place(xyz, (n, n, n), r, np.zeros_like(q))
    np.testing.assert_allclose(raw, q, atol=1e-7)
    s = np.full_like(q, 0.123)
    hyb = mlp.place(xyz, (n, n, n), r, s, s_coarse=np.full((n ** 3, 3), 0.123))
    np.testing.assert_allclose(hyb, q, atol=2e-7)


def test_hybrid_placement_with_zero_network_is_the_affine_map():
    # s = 0: the residuals are the coarse positions minus their points, so a
    # fine tracer lands on the affine map of its coarse tetrahedron
    n, r = 5, 2
    xyz = W.zeldovich(n, 2, 1.0)
    q = mlp.fine_points((n, n, n), r).astype(np.float64)
    got = mlp.place(xyz, (n, n, n), r, np.zeros_like(q), s_coarse=np.zeros((n ** 3, 3)))
    # the midpoint of coarse edge 0-1 of cube (1, 2, 3) is fine tracer (3, 4, 6)
    f = n * r
    fid = 3 + f * (4 + f * 6)
    c0 = 1 + n * (2 + n * 3)
    c1 = 2 + n * (2 + n * 3)
    X = np.stack([np.asarray(a, dtype=np.float64) for a in xyz], axis=1)
    mid = X[c0] + 0.5 * mlp.minimal_image(X[c1] - X[c0])
    np.testing.assert_allclose(got[fid], mlp.wrap_f32(mid, 1.0), atol=1e-7)
