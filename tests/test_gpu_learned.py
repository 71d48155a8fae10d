"""Learned refinement judged against a high-resolution lattice of the same field.

The 64^3 lattice of the seeded field (modes |k| <= 16, D = 5) is refined r = 4
times, with vertices placed by the network trained on the lattice's own (q, x)
pairs (plus its residuals interpolated from the coarse tracers), and rendered
at 2048^2; the reference is the 256^3 lattice of the same analytic field.  The
gain test: the learned image is closer to the reference (relative L1) than the
plain 64^3 image; the linear refinement (nested tetrahedra) reproduces the
plain image.
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tess():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1208_3206_amd as t
    return t


def l1(img, ref):
    return float((img - ref).abs().sum() / ref.abs().sum())


def test_learned_refinement_beats_plain_coarse_lattice(tess):
    import torch
    w, wr = W.LEARNED, W.LEARNED_REF
    view = W.z_view(w.width, w.height)
    dev = lambda xyz: [torch.from_numpy(a).cuda() for a in xyz]
    ref_lat = tess.build(*dev(W.zeldovich(wr.n, wr.kmax, wr.growth[0])), (wr.n,) * 3)
    ref = tess.project(ref_lat, view).double()
    del ref_lat
    coarse = tess.build(*dev(W.zeldovich(w.n, w.kmax, w.growth[0])), (w.n,) * 3)
    plain = tess.project(coarse, view).double()
    fine_lin, _ = tess.refine(coarse, r=4, mode="linear")
    lin = tess.project(fine_lin, view).double()
    del fine_lin
    fine, rep = tess.refine(coarse, r=4, mode="mlp")
    learned = tess.project(fine, view).double()
    e_plain, e_lin, e_mlp = l1(plain, ref), l1(lin, ref), l1(learned, ref)
    print(f"L1 vs 256^3: plain 64^3 {e_plain:.4f}, linear r=4 {e_lin:.4f}, learned r=4 {e_mlp:.4f}; "
          f"loss {rep['loss_first']:.3e} -> {rep['loss_last']:.3e}, train {rep['train_ms']:.0f} ms, "
          f"infer {rep['infer_ms']:.1f} ms", flush=True)
    assert rep["loss_last"] < 0.25 * rep["loss_first"]
    assert abs(e_lin - e_plain) < 1e-3 * e_plain + 1e-6
    assert e_mlp < e_plain
