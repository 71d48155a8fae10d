"""tess_project_noalloc (the allocation-free projection) against tess_project
through the C ABI: two calls in a row, the second with a smaller input, each
held to the projection's parity bar against tess_project's image (and the
oracle's); then a call captured into a graph in global capture mode, where
any allocation would fail the capture, replayed against the eager image."""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tess():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1208_3206_amd as t
    return t


def dev(arrs):
    import torch
    return [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in arrs]


def check(got, ref, what):
    got = got.astype(np.float64)
    tau = 1e-6 * np.abs(ref).mean()
    r = np.abs(got - ref) / np.maximum(np.abs(ref), tau)
    covered = np.abs(ref) > 1e-3 * np.abs(ref).mean()
    mass = abs(got.sum() - ref.sum()) / abs(ref.sum())
    print(f"{what}: max rel {r.max():.3e}, covered {r[covered].max():.3e}, mass {mass:.3e}", flush=True)
    assert r.max() <= 1e-4 and r[covered].max() <= 1e-6 and mass <= 1e-6, what


def test_noalloc_matches_project_on_two_calls(tess):
    import torch
    cases = [
        # 8 pixels per lattice cell: the edge form, periodic wrap
        (24, W.zeldovich(24, 8, 6.0, seed=3), W.z_view(192, 160)),
        # smaller: 12^3 into a rotated 96 x 80 window (per-tetrahedron form)
        (12, W.zeldovich(12, 4, 4.0, seed=4), W.rotated_view(W.random_rotations(1, seed=9)[0], 96, 80)),
    ]
    for n, xyz, view in cases:
        lat = tess.build(*dev(xyz), (n, n, n))
        out = torch.full((view["height"], view["width"]), -7.0, dtype=torch.float32, device="cuda")
        tess.project_noalloc(lat, view, out)
        ref_img = tess.project(lat, view)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        check(got, ref_img.cpu().numpy().astype(np.float64), f"noalloc vs tess_project, {n}^3")
        orc, _ = O.project_region(*xyz, (n, n, n), view)
        check(got, orc, f"noalloc vs oracle, {n}^3")


def test_noalloc_overflow_and_capacity_error(tess):
    import torch
    n = 16
    xyz = W.zeldovich(n, 5, 4.0, seed=5)
    lat = tess.build(*dev(xyz), (n, n, n))
    view = W.z_view(120, 88)
    out = torch.empty((88, 120), dtype=torch.float32, device="cuda")
    # a capped pair list: the overflow raster draws the image
    tess.project_noalloc(lat, view, out, tune=tess.make_tune(pair_capacity=64))
    torch.cuda.synchronize()
    orc, _ = O.project_region(*xyz, (n, n, n), view)
    check(out.cpu().numpy(), orc, "noalloc through the overflow raster")
    # a lattice too large for the scratch is refused with TESS_ECAPACITY
    big = 64
    zb = [torch.zeros(big ** 3, dtype=torch.float32, device="cuda") for _ in range(3)]
    lb = tess.build(*zb, (big, big, big))
    with pytest.raises(tess.TessError, match="scratch"):
        tess.project_noalloc(lb, W.z_view(512), torch.empty((512, 512), device="cuda"))


def test_noalloc_in_a_graph_captured_in_global_mode(tess):
    import torch
    n = 16
    xyz = W.zeldovich(n, 5, 4.0, seed=6)
    lat = tess.build(*dev(xyz), (n, n, n))
    view = W.z_view(128, 112)
    s = torch.cuda.Stream()
    out = torch.empty((112, 128), dtype=torch.float32, device="cuda")
    with torch.cuda.stream(s):
        tess.project_noalloc(lat, view, out)
    s.synchronize()
    eager = out.clone()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s, capture_error_mode="global"):
        tess.project_noalloc(lat, view, out)
    for _ in range(3):
        out.fill_(-1.0)
        g.replay()
        torch.cuda.synchronize()
        torch.testing.assert_close(out, eager, rtol=2.4e-7, atol=1e-9)
        tess.project(lat, W.z_view(64, 64))  # other work between replays
        torch.cuda.synchronize()
