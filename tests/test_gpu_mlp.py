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
    """FP64 oracle with the products' operands rounded to bf16, as the GPU takes
    them (the backward's products take the same bf16 weights)."""
    p = as_dict(params_flat)
    for k in ("W1", "W2", "W3", "W4", "W5"):
        p[k] = mlp.bf16_round(p[k])
    pred, cache = mlp.forward(p, q.astype(np.float64), B, operands="bf16")
    return mlp.loss(pred, target), mlp.backward(p, cache, pred, target), pred


def problem(n, seed):
    rng = np.random.default_rng(seed)
    q = (rng.integers(0, 64, size=(n, 3)) / 64.0).astype(np.float32)
    target = (0.03 * np.sin(2 * np.pi * (q @ np.array([[1, 2, 0], [0, 1, 3], [2, 0, 1]]).T))
              ).astype(np.float32)
    B = W.rff_frequencies(8.0, seed=1)
    params = W.network_params(seed=2)
    return q, target, B, params


def test_forward_matches_oracle(tess):
    import torch
    q, target, B, params = problem(1000, 0)
    loss, grad, pred = tess.mlp_loss_grad(params, B, torch.from_numpy(q).cuda(),
                                          torch.from_numpy(target).cuda(), want_pred=True)
    rl, _, rpred = reference(params, B.astype(np.float64), q, target.astype(np.float64))
    got = pred.cpu().numpy().astype(np.float64)
    err = np.linalg.norm(got - rpred) / np.linalg.norm(rpred)
    print(f"forward: rel L2 {err:.3e}, max abs {np.abs(got - rpred).max():.3e}, "
          f"loss {loss:.6e} vs {rl:.6e}", flush=True)
    assert err < 1e-3
    assert abs(loss - rl) / rl < 2e-3


@pytest.mark.parametrize("n", [1, 17, 1000, 40000])
def test_fused_inference_matches_oracle_and_training_forward(tess, n):
    # the inference kernel (whole network per 16-sample tile, layers computed
    # transposed with permuted input columns) against the oracle's bf16-operand
    # forward pass and the training path's layer-by-layer forward; n covers a
    # partial tile, several blocks and a ragged tail
    import torch
    q, target, B, params = problem(n, 100 + n)
    qd = torch.from_numpy(q).cuda()
    pred = tess.mlp_forward(params, B, qd).cpu().numpy().astype(np.float64)
    _, _, rpred = reference(params, B.astype(np.float64), q, target.astype(np.float64))
    err = np.linalg.norm(pred - rpred) / np.linalg.norm(rpred)
    _, _, tpred = tess.mlp_loss_grad(params, B, qd, torch.from_numpy(target).cuda(), want_pred=True)
    tpred = tpred.cpu().numpy().astype(np.float64)
    d = np.abs(pred - tpred).max() / np.abs(tpred).max()
    dl2 = np.linalg.norm(pred - tpred) / np.linalg.norm(tpred)
    print(f"fused inference n={n}: rel L2 vs oracle {err:.3e}, vs training forward rel L2 {dl2:.3e} "
          f"max {d:.3e}", flush=True)
    assert err < 1e-3
    # the same operands, summed in another order (the columns of each 32-wide
    # k block are permuted), so now and then a bf16 activation rounds the
    # other way (one bf16 ulp, 2^-8 relative, on one of 512 activations)
    assert dl2 < 2e-4 and d < 1e-2


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
        print(f"n={n} {k}: rel L2 {rel:.3e} cos {cos:.7f}", flush=True)
        assert rel <= 1e-2 and cos >= 0.9999, k


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
    # the r-fold sub-lattice's tetrahedra nest in the coarse ones (pin C11),
    # so the LINEAR refinement's image is the coarse lattice's: the GPU image
    # of the fine lattice against the oracle's image of the coarse one
    import torch
    n = 16
    xyz = W.zeldovich(n, 5, 3.0)
    lat = tess.build(*[torch.from_numpy(a).cuda() for a in xyz], (n, n, n))
    fine, rep = tess.refine(lat, r=2, mode="linear")
    view = W.z_view(96)
    got = tess.project(fine, view).cpu().numpy()
    ref, _ = O.project_region(*xyz, (n, n, n), view)
    tau = 1e-6 * np.abs(ref).mean()
    err = (np.abs(got.astype(np.float64) - ref) / np.maximum(np.abs(ref), tau)).max()
    mass = abs(got.astype(np.float64).sum() - ref.sum()) / ref.sum()
    print(f"linear r=2 vs the oracle's coarse image: max rel {err:.3e}, mass {mass:.3e}", flush=True)
    assert rep["fine_tracers"] == (2 * n) ** 3
    # the fine positions are the affine maps rounded to FP32: the image moves
    # by that rounding (~1e-7 of a cell), far inside the projection's bar
    assert err <= 1e-4 and mass <= 1e-6


def test_adam_step_matches_oracle(tess):
    # one bias-corrected update from a state with non-zero moments (step 7)
    rng = np.random.default_rng(11)
    p = W.network_params(seed=4)
    m = (1e-3 * rng.standard_normal(p.size)).astype(np.float32)
    v = (1e-6 * rng.uniform(0.0, 1.0, p.size) ** 2).astype(np.float32)
    g = (1e-3 * rng.standard_normal(p.size)).astype(np.float32)
    gp, gm, gv = tess.mlp_adam(p, m, v, g, step=7, lr=1e-3)
    P, G, M, V = (as_dict(a.astype(np.float64)) for a in (p, g, m, v))
    mlp.adam_step(P, G, M, V, t=7, lr=1e-3)
    for got, ref, what in ((gp, P, "params"), (gm, M, "m"), (gv, V, "v")):
        r = mlp.flatten(ref)
        err = np.abs(got.astype(np.float64) - r).max() / np.abs(r).max()
        print(f"adam {what}: max rel {err:.3e}", flush=True)
        assert err <= 1e-6, what
    # the update itself, to the FP32 rounding of the parameters it moves
    du = gp.astype(np.float64) - p
    dr = mlp.flatten(P) - p
    assert np.abs(du - dr).max() <= 1e-6 * np.abs(dr).max() + 2.0 ** -24 * np.abs(p).max()


@pytest.mark.parametrize("mode", ["mlp_raw", "mlp"])
def test_refined_positions_match_oracle_inference(tess, mode):
    # the placed fine tracers from given weights (no training) against the
    # oracle's placement with its bf16-operand inference; coarse tracers
    # keep their data exactly
    import torch
    n, r = 12, 2
    xyz = W.zeldovich(n, 4, 4.0)
    lat = tess.build(*[torch.from_numpy(a).cuda() for a in xyz], (n, n, n))
    B = W.rff_frequencies(8.0, seed=1)
    params = W.network_params(seed=6, out_scale=0.1)
    fine, _ = tess.refine(lat, r=r, mode=mode, steps=0, rff_B=B, weights_in=params)
    got = torch.stack(fine.positions(), dim=1).cpu().numpy().astype(np.float64)
    p = as_dict(params)
    s_fine, _ = mlp.forward(p, mlp.fine_points((n, n, n), r).astype(np.float64), B.astype(np.float64),
                            operands="bf16")
    s_coarse = None
    if mode == "mlp":
        s_coarse, _ = mlp.forward(p, mlp.fine_points((n, n, n), 1).astype(np.float64), B.astype(np.float64),
                                  operands="bf16")
    ref = mlp.place(xyz, (n, n, n), r, s_fine, s_coarse=s_coarse).astype(np.float64)
    d = np.abs(mlp.minimal_image(got - ref)).max(axis=1) * (n * r)   # in fine cells
    f = n * r
    ids = np.arange(f ** 3)
    coarse = ((ids % f) % r == 0) & (((ids // f) % f) % r == 0) & ((ids // (f * f)) % r == 0)
    q99, q999 = np.quantile(d, 0.99), np.quantile(d, 0.999)
    print(f"{mode}: position error in fine cells: max {d.max():.3e}, 99.9% {q999:.3e}, 99% {q99:.3e}",
          flush=True)
    assert np.all(d[coarse] == 0.0)
    assert q99 <= 1e-3
    assert d.max() <= 2e-2


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
