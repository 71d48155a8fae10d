"""Refinement network on the GPU (bf16 MFMA kernels) against the FP64 oracle,
and the refined lattices through the projector."""
import numpy as np
import pytest

import oracle as O
from oracle import mlp
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tess():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1208_3206_amd as t
    return t


def bf16_round(a):
    import torch
    return torch.from_numpy(np.asarray(a, dtype=np.float32)).to(torch.bfloat16).to(torch.float64).numpy()


def as_dict(flat):
    out, off = {}, 0
    shapes = {"W1": (128, 128), "b1": (128,), "W2": (128, 128), "b2": (128,), "W3": (128, 128),
              "b3": (128,), "W4": (128, 128), "b4": (128,), "W5": (3, 128), "b5": (3,)}
    for k in mlp.NAMES:
        n = int(np.prod(shapes[k]))
        out[k] = np.asarray(flat[off:off + n], dtype=np.float64).reshape(shapes[k])
        off += n
    return out


def reference(params_flat, B, q, target):
    """FP64 oracle with the weights rounded to bf16 as the GPU uses them."""
    p = as_dict(params_flat)
    for k in ("W1", "W2", "W3", "W4", "W5"):
        p[k] = bf16_round(p[k])
    pred, cache = mlp.forward(p, q.astype(np.float64), B)
    return mlp.loss(pred, target), mlp.backward(p, cache, pred, target), pred


def problem(n, seed):
    rng = np.random.default_rng(seed)
    q = (rng.integers(0, 64, size=(n, 3)) / 64.0).astype(np.float32)
    target = (0.03 * np.sin(2 * np.pi * (q @ np.array([[1, 2, 0], [0, 1, 3], [2, 0, 1]]).T))
              ).astype(np.float32)
    B = mlp.rff_matrix(8.0, seed=1).astype(np.float32)
    params = mlp.flatten(mlp.init_params(seed=2)).astype(np.float32)
    return q, target, B, params


def test_forward_matches_oracle(tess):
    import torch
    q, target, B, params = problem(1000, 0)
    loss, grad, pred = tess.mlp_loss_grad(params, B, torch.from_numpy(q).cuda(),
                                          torch.from_numpy(target).cuda(), want_pred=True)
    rl, _, rpred = reference(params, B.astype(np.float64), q, target.astype(np.float64))
    got = pred.cpu().numpy().astype(np.float64)
    err = np.linalg.norm(got - rpred) / np.linalg.norm(rpred)
    print(f"forward: rel L2 {err:.3e}, loss {loss:.6e} vs {rl:.6e}", flush=True)
    assert err < 2e-2
    assert abs(loss - rl) / rl < 2e-2


@pytest.mark.parametrize("n", [64, 1000, 8192])
def test_gradients_match_oracle(tess, n):
    import torch
    q, target, B, params = problem(n, n)
    loss, grad = tess.mlp_loss_grad(params, B, torch.from_numpy(q).cuda(), torch.from_numpy(target).cuda())
    rl, rg, _ = reference(params, B.astype(np.float64), q, target.astype(np.float64))
    g = as_dict(grad)
    for k in mlp.NAMES:
        a, b = g[k].ravel(), rg[k].ravel()
        rel = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)
        cos = float(a @ b / (np.linalg.norm(a) * np.linalg.norm(b) + 1e-300))
        print(f"n={n} {k}: rel L2 {rel:.3e} cos {cos:.6f}", flush=True)
        assert rel < 3e-2 and cos > 0.999, k


def test_zero_output_weights_bias_gradient(tess):
    import torch
    q, target, B, params = problem(512, 3)
    params = params.copy()
    params[66048:66048 + 384] = 0.0  # W5
    loss, grad = tess.mlp_loss_grad(params, B, torch.from_numpy(q).cuda(), torch.from_numpy(target).cuda())
    b5 = params[66432:66435].astype(np.float64)
    expect = 2.0 * (b5[None, :] - target.astype(np.float64)).mean(axis=0)
    np.testing.assert_allclose(grad[66432:66435], expect, rtol=1e-4, atol=1e-7)
    assert np.all(grad[:4 * 16512] == 0.0)


def test_linear_refinement_keeps_the_image(tess):
    import torch
    n = 16
    xyz = W.zeldovich(n, 5, 3.0)
    lat = tess.build(*[torch.from_numpy(a).cuda() for a in xyz], (n, n, n))
    fine, rep = tess.refine(lat, r=2, mode="linear")
    view = W.z_view(96)
    a = tess.project(lat, view).cpu().numpy().astype(np.float64)
    b = tess.project(fine, view).cpu().numpy().astype(np.float64)
    err = np.abs(a - b).max() / np.abs(a).max()
    print(f"linear r=2: max rel diff {err:.3e}", flush=True)
    assert rep["fine_tracers"] == (2 * n) ** 3
    assert err < 1e-3
    assert abs(a.sum() - b.sum()) / a.sum() < 1e-5


def test_training_reduces_the_loss_and_places_vertices(tess):
    import torch
    n = 16
    xyz = W.zeldovich(n, 4, 3.0)
    lat = tess.build(*[torch.from_numpy(a).cuda() for a in xyz], (n, n, n))
    fine, rep, w = tess.refine(lat, r=2, mode="mlp", steps=300, batch=1024, lr0=3e-3, lr1=1e-4,
                               want_weights=True)
    print(f"train: loss {rep['loss_first']:.3e} -> {rep['loss_last']:.3e}, {rep['train_ms']:.0f} ms", flush=True)
    assert rep["loss_last"] < 0.2 * rep["loss_first"]
    assert np.all(np.isfinite(w))
    img = tess.project(fine, W.z_view(64)).cpu().numpy()
    assert np.all(np.isfinite(img)) and abs(img.mean() - 1.0) < 0.02
