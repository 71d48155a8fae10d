"""Benchmark: column-density projection of the 256^3 Zel'dovich lattice to 2048^2.

One step = one full tess_project call (setup, binning, raster, finalize) of the
100,663,296-tetrahedron lattice onto a 2048 x 2048 image, inputs resident in
HBM.  Prints one JSON line (see the field list at the bottom).

  python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X: 256 CUs x 4 SIMD x 16 lanes at 2.4 GHz.  The raster's FP64 FMA,
# add, multiply, min, max and floor issue at one lane-operation per lane per
# clock (the rate of unpacked FP32), so that is the ceiling of its arithmetic.
PEAK_VALU_OPS = 256 * 4 * 16 * 2.4e9          # 3.93e13 lane-ops/s
# The raster's unit of work is a kink: one crease crossing one pixel row of a
# tile (tess_stats.kinks).  Its algorithmic FP64 arithmetic: step the crossing
# along the crease, floor it, the fraction phi from the crossing (2), and the
# two second-difference entries D*phi and D - D*phi (2).
OPS_PER_KINK = 6
# A perspective view's raster evaluates every pixel of a footprint's box (the
# chord is not piecewise linear along a row; tess_stats.kinks counts those
# pixels): 4 faces x (n . d, 2; the quotient h / n . d, 1; the min or max, 1),
# the ray length |(pu, pv, 1)| (3) and q times the chord (3).
OPS_PER_RAY_PIXEL = 22
# Its LDS traffic: two FP64 read-modify-writes.
LDS_BYTES_PER_KINK = 2 * 16
PEAK_LDS_BYTES = 256 * 128 * 2.4e9            # 128 B/clk/CU: 78.6 TB/s
# A raster that visits every covered pixel needs at least 16 lane-operations
# per fragment (4 plane evaluations, 2 min/max, subtract and clamp, a
# compensated add); reported alongside as the fragment-equivalent rate.
OPS_PER_FRAGMENT = 16
# k_raster's HBM bytes at stress 2048^2 from rocprofv3 FETCH_SIZE / WRITE_SIZE
# passes (KiB per dispatch), scaled by what the same counters read for 1 GiB
# read and written by a device copy and read by a sum (--copy-probe: both
# read back half their bytes, the write counter all); valid only for the
# sources they were taken on.
TRAFFIC = {
    "sources": ["paper_1208_3206_amd/csrc/tess_kernels.hip", "paper_1208_3206_amd/csrc/tess_tet.h",
                "paper_1208_3206_amd/csrc/tess_internal.h"],
    "workload": "stress_256^3_to_2048^2", "tile": [32, 512], "block": 1024,
    "sha256": "946348e51242f5fc4224eedefa6189e91ca0dea5dc6aea1e21062f10b9e75107",
    "fetch_kib": 46861873.6, "write_kib": 1427621.1, "fetch_scale": 2.0, "write_scale": 1.0,
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="stress_256^3_to_2048^2")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--tile-rows", type=int, default=0)
    ap.add_argument("--tile-cols", type=int, default=0)
    ap.add_argument("--chunk", type=int, default=0)
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--quantity", default="density", choices=["density", "unit", "density2"],
                    help="projected per-tetrahedron value: rho, 1 or rho^2")
    ap.add_argument("--method", default="tessellation", choices=["tessellation", "centroids", "hybrid"],
                    help="exact projection of the tessellation, the centroid splats, or (perspective "
                         "workloads) exact within --lod-radius of the camera and billboards beyond")
    ap.add_argument("--lod-radius", type=float, default=0.25,
                    help="the hybrid's sphere around the camera (box units)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only copy 1 GiB device-to-device twice (scale reference for HBM byte counters)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="about how long the oracle's CPU-baseline sample runs")
    return ap.parse_args()


def host_cores():
    """(threads to use, description): the CPUs this process may run on,
    capped by the cgroup's CPU quota when one is set."""
    import platform
    nproc = os.cpu_count() or 1
    try:
        allowed = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        allowed = nproc
    quota = None
    try:
        with open("/sys/fs/cgroup/cpu.max") as fh:
            q, period = fh.read().split()[:2]
            if q != "max":
                quota = max(1, int(int(q) // int(period)))
    except (OSError, ValueError):
        pass
    threads = min(allowed, quota) if quota else allowed
    model = platform.processor() or ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return threads, {"nproc": nproc, "affinity": allowed, "cgroup_quota_cores": quota, "model": model}


def cpu_baseline(xyz, w, view, full_fragments: float):
    """The FP64 oracle on a bounded sample of the same workload (test harness code).

    The oracle's region mode (a first pass sets up every tetrahedron, then
    exact per-pixel ray clipping of the crop's pixels, FP64, OpenMP over row
    bands) on square crops at the image centre, on all the host cores this
    process may use.  Two crops give the fixed cost of the first pass and the
    cost per fragment; the larger is sized for about args.cpu_seconds of
    clipping.  The full image's time is the fixed cost plus its fragments at
    that rate."""
    import oracle
    threads, host = host_cores()
    dims = (w.n,) * 3

    def run(side):
        x0 = max(0, w.width // 2 - side // 2)
        y0 = max(0, w.height // 2 - side // 2)
        crop = (x0, y0, min(side, w.width), min(side, w.height))
        t0 = time.perf_counter()
        _, st = oracle.project_region(*xyz, dims, view, crop=crop, nthreads=threads)
        return time.perf_counter() - t0, st["fragments"], crop

    ta, fa, _ = run(32)
    tb, fb, _ = run(64)
    rate = (fb - fa) / max(tb - ta, 1e-3)          # fragments per second, marginal
    side = 64
    while 2 * side <= min(w.width, w.height) and full_fragments * (2 * side) ** 2 / (w.width * w.height) <= \
            rate * args.cpu_seconds:
        side *= 2
    if side > 64:
        tb, fb, _ = run(side)
        rate = (fb - fa) / max(tb - ta, 1e-3)
    fixed = max(ta - fa / rate, 0.0)
    full_s = fixed + full_fragments / rate
    return {
        "value": w.tets / full_s,
        "unit": "tets/s",
        "cores": threads,
        "kind": "oracle",
        "sample": (f"FP64 oracle, region mode, {threads} threads: centre crops 32^2 ({fa:.3e} fragments, "
                   f"{ta:.1f} s) and {side}^2 ({fb:.3e} fragments, {tb:.1f} s) of the {w.width}x{w.height} "
                   f"image of the same lattice; fixed cost (setup of all {w.tets} tetrahedra) {fixed:.1f} s, "
                   f"then {rate:.3e} fragments/s; the full image ({full_fragments:.3e} fragments) would take "
                   f"{full_s:.0f} s"),
        "fragments_per_s": rate,
        "ns_per_fragment_per_core": threads / rate * 1e9,
        "fixed_s": fixed,
        "full_image_s": full_s,
        "seconds": ta + tb,
        "host": host,
    }


def run_batched(args, w, tess, W, torch):
    """Many snapshots x views in one tess_project_batch call (captured graph)."""
    dev = torch.device("cuda:0")
    lats = []
    for D in w.growth:
        xyz = W.zeldovich(w.n, w.kmax, D)
        lats.append(tess.build(*[torch.from_numpy(a).to(dev) for a in xyz], (w.n,) * 3,
                               precision=args.precision))
    views = W.workload_views(w)
    out = torch.empty((len(lats), len(views), w.height, w.width), dtype=torch.float32, device=dev)
    t0 = time.perf_counter()
    _, st0 = tess.project_batch(lats, views, out=out, stats=True)  # autotune + graph capture
    first_s = time.perf_counter() - t0
    for _ in range(args.warmup):
        tess.project_batch(lats, views, out=out)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    dev_ms = 0.0
    for _ in range(args.steps):
        _, st = tess.project_batch(lats, views, out=out, stats=True)
        dev_ms += st["ms"] / args.steps
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t_start) * 1e3 / args.steps
    n_img = len(lats) * len(views)
    kinks = st0["kinks"]
    achieved = OPS_PER_KINK * kinks / (dev_ms * 1e-3)
    result = {
        "metric": "tets/s over all images of a batch",
        "value": w.tets * n_img / (ms * 1e-3),
        "unit": "tets/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded Zel'dovich lattices, kmax %d, D %s)" % (w.kmax, list(w.growth)),
        "config": {"workload": w.name, "lattice": w.n, "snapshots": len(lats), "views": len(views),
                   "images": n_img, "image": [w.width, w.height],
                   "tile": [st["tile_rows"], st["tile_cols"]], "chunk": st["chunk"]},
        "images_per_s": n_img / (ms * 1e-3),
        "fragments": st0["fragments"],
        "fragments_per_s": st0["fragments"] / (ms * 1e-3),
        "spans": st0["spans"],
        "kinks": kinks,
        "bin_pairs": st0["bin_pairs"],
        "graph_ms": dev_ms,
        "first_call_s": first_s,
        "roofline": {"kernel": "whole batch graph", "bound": "alu", "achieved": achieved / 1e12,
                     "peak": PEAK_VALU_OPS / 1e12, "unit": "Tops/s", "frac": achieved / PEAK_VALU_OPS,
                     "traffic": None, "ops_per_launch": OPS_PER_KINK * kinks, "ops_per_kink": OPS_PER_KINK},
    }
    print(json.dumps(result), flush=True)


def run_resample(args, w, tess, W, torch):
    """Resampling to a grid: one lattice, a stack of depth slabs of z-views
    (one tess_project_batch call); the slabs must add up to the unclipped
    projection."""
    dev = torch.device("cuda:0")
    xyz = W.zeldovich(w.n, w.kmax, w.growth[0])
    lat = tess.build(*[torch.from_numpy(a).to(dev) for a in xyz], (w.n,) * 3, precision=args.precision)
    views = W.slab_views(w.width, w.n)
    out = torch.empty((1, len(views), w.height, w.width), dtype=torch.float32, device=dev)
    _, st0 = tess.project_batch([lat], views, out=out, stats=True)
    for _ in range(args.warmup):
        tess.project_batch([lat], views, out=out)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        tess.project_batch([lat], views, out=out)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t_start) * 1e3 / args.steps
    full = tess.project(lat, W.z_view(w.width)).double()
    total = out[0].double().sum(dim=0)
    add_err = float((total - full).abs().max() / full.abs().max())
    cells = w.n * w.width * w.height
    result = {
        "metric": "grid cells/s resampling %d^3 -> %d^3 by depth slabs" % (w.n, w.width),
        "value": cells / (ms * 1e-3),
        "unit": "cells/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded Zel'dovich lattice, kmax %d, D %g)" % (w.kmax, w.growth[0]),
        "config": {"workload": w.name, "lattice": w.n, "slabs": len(views), "image": [w.width, w.height],
                   "tile": [st0["tile_rows"], st0["tile_cols"]]},
        "tets_per_s_per_slab": w.tets * len(views) / (ms * 1e-3),
        "fragments": st0["fragments"],
        "slabs_sum_vs_projection_max_rel": add_err,
    }
    print(json.dumps(result), flush=True)


def spectral_upsample(xyz, n, r):
    """Zero-padded FFT upsampling of a periodic lattice's displacements by r
    (the non-learned control: exact for a field band-limited below n/2)."""
    import numpy as np
    import workloads as W
    q = W.lattice_q(n)
    out = []
    m = n * r
    for c in range(3):
        s = (xyz[c].astype(np.float64) - q[:, c])
        s -= np.ceil(s - 0.5)                      # minimal image, unit box
        S = np.fft.fftn(s.reshape(n, n, n))
        P = np.zeros((m, m, m), dtype=np.complex128)
        h = n // 2
        idx = np.r_[0:h, m - h:m]
        src = np.r_[0:h, n - h:n]
        P[np.ix_(idx, idx, idx)] = S[np.ix_(src, src, src)]
        fine = np.real(np.fft.ifftn(P)) * r ** 3
        shape = [1, 1, 1]
        shape[2 - c] = m
        qf = (np.arange(m) / m).reshape(shape)
        out.append(np.ascontiguousarray(W.wrap_to_f32(qf + fine, 1.0).ravel()))
    return out


def run_learned(args, w, tess, W, torch):
    """L1 against the high-resolution reference vs time: plain lattices M^3
    of the same analytic field, and the 64^3 lattice refined r-fold with the
    network (trained once; inference from the trained weights)."""
    import numpy as np
    dev = torch.device("cuda:0")
    view = W.z_view(w.width, w.height)
    wr = W.LEARNED_REF

    def timed_render(xyz, n):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        d = [torch.from_numpy(a).to(dev) for a in xyz]
        lat = tess.build(*d, (n,) * 3)
        img = tess.project(lat, view)
        torch.cuda.synchronize()
        return img.double(), time.perf_counter() - t0

    ref, _ = timed_render(W.zeldovich(wr.n, wr.kmax, wr.growth[0]), wr.n)
    l1 = lambda img: float((img - ref).abs().sum() / ref.abs().sum())
    plain = []
    for m in (64, 96, 128, 160, 192, 256):
        xyz = W.zeldovich(m, w.kmax, w.growth[0])
        timed_render(xyz, m)  # warm
        img, t = timed_render(xyz, m)
        plain.append({"M": m, "tets": 6 * m ** 3, "l1": l1(img), "s": t})
    coarse_xyz = W.zeldovich(w.n, w.kmax, w.growth[0])
    coarse = tess.build(*[torch.from_numpy(a).to(dev) for a in coarse_xyz], (w.n,) * 3)
    _, rep, weights = tess.refine(coarse, r=2, mode="mlp", want_weights=True)
    learned = []
    for r in (1, 2, 3, 4):
        for rep_i in range(2):  # second pass timed
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            d = [torch.from_numpy(a).to(dev) for a in coarse_xyz]
            lat = tess.build(*d, (w.n,) * 3)
            fine, frep = tess.refine(lat, r=r, mode="mlp", steps=0, weights_in=weights)
            img = tess.project(fine, view)
            torch.cuda.synchronize()
            t = time.perf_counter() - t0
            del fine
        learned.append({"r": r, "tets": 6 * (w.n * r) ** 3, "l1": l1(img.double()), "s": t,
                        "infer_ms": frep["infer_ms"]})
    spec = spectral_upsample(coarse_xyz, w.n, 4)
    img, t = timed_render(spec, w.n * 4)
    e_learned = learned[-1]["l1"]
    plain_at = [p for p in plain if p["l1"] <= e_learned]
    result = {
        "metric": "L1 vs the 256^3 reference at 2048^2: learned refinement and plain lattices",
        "value": e_learned,
        "unit": "relative L1 (learned r=4)",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 1,
        "ms_per_step": learned[-1]["s"] * 1e3,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 raster, bf16 network",
        "data": "synthetic (seeded Zel'dovich lattices, kmax %d, D %g)" % (w.kmax, w.growth[0]),
        "config": {"workload": w.name, "coarse": w.n, "reference": wr.n, "image": [w.width, w.height]},
        "plain": plain,
        "learned": learned,
        "training": {"steps": 10000, "batch": 8192, "loss_first": rep["loss_first"],
                     "loss_last": rep["loss_last"], "train_ms": rep["train_ms"]},
        "spectral_control": {"r": 4, "l1": l1(img), "s": t},
        "gain_over_plain_64": plain[0]["l1"] / e_learned,
        "plain_lattice_at_equal_l1": plain_at[0] if plain_at else None,
    }
    print(json.dumps(result), flush=True)


def copy_probe(torch):
    """Kernels of known traffic: what FETCH_SIZE / WRITE_SIZE read for them
    scales the raster's counters to bytes.  A device copy (1 GiB read, 1 GiB
    written; the runtime's copy kernel) and a sum over the same 1 GiB (plain
    vector loads, as the raster's)."""
    a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(2):
        b.copy_(a)
    s = 0.0
    for _ in range(2):
        s += float(a.sum())
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": a.numel() * 4, "copies": 2, "sums": 2, "sum": s}), flush=True)


def raster_traffic(workload, tile, block):
    """HBM bytes per raster launch from the committed counter passes, or None
    for another workload or launch shape, or when the raster's sources changed
    since they were taken."""
    import hashlib
    if workload != TRAFFIC["workload"] or list(tile) != TRAFFIC["tile"] or block != TRAFFIC["block"]:
        return None
    h = hashlib.sha256()
    for f in TRAFFIC["sources"]:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest() != TRAFFIC["sha256"]:
        return None
    return TRAFFIC["fetch_kib"] * 1024 * TRAFFIC["fetch_scale"] + TRAFFIC["write_kib"] * 1024 * TRAFFIC["write_scale"]


def main():
    global args
    args = parse()
    if args.copy_probe:
        import torch
        copy_probe(torch)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported "
              "(the path is measured on one GPU's share of the work)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    import paper_1208_3206_amd as tess
    import workloads as W

    w = W.ALL[args.workload]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if len(w.growth) > 1 or w.n_views > 1:
        run_batched(args, w, tess, W, torch)
        return
    if w is W.LEARNED:
        run_learned(args, w, tess, W, torch)
        return
    if w is W.RESAMPLE:
        run_resample(args, w, tess, W, torch)
        return
    t0 = time.perf_counter()
    xyz = W.zeldovich(w.n, w.kmax, w.growth[0])
    gen_s = time.perf_counter() - t0
    d = [torch.from_numpy(a).to(dev) for a in xyz]
    view = dict(W.workload_views(w)[0], quantity=args.quantity, method=args.method)
    if args.method == "hybrid":
        view["lod_radius"] = args.lod_radius
    lat = tess.build(*d, (w.n,) * 3, precision=args.precision)
    out = torch.empty((w.height, w.width), dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream()

    tune = tess.make_tune(args.tile_rows, args.tile_cols, args.chunk, args.block)
    # the first call counts fragments (untimed); the timed calls take the
    # kernel times with HIP events on the stream and skip the count
    torch.cuda.synchronize()
    free_before = torch.cuda.mem_get_info()[0]
    _, st0 = tess.project(lat, view, out=out, tune=tune, stats=True)
    frags, spans, kinks = st0["fragments"], st0["spans"], st0["kinks"]
    timed_tune = tess.make_tune(args.tile_rows, args.tile_cols, args.chunk, args.block, counts=False)
    for _ in range(args.warmup):
        tess.project(lat, view, out=out, tune=timed_tune)
    torch.cuda.synchronize()

    per_step = []
    kernel = {"setup_ms": 0.0, "bin_ms": 0.0, "raster_ms": 0.0, "finalize_ms": 0.0}
    t_start = time.perf_counter()
    for _ in range(args.steps):
        _, st = tess.project(lat, view, out=out, tune=timed_tune, stats=True)
        per_step.append(st["ms"])
        for k in kernel:
            kernel[k] += st[k] / args.steps
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    ms = wall * 1e3 / args.steps
    # device memory the library's workspace took (its buffers only grow)
    workspace_gb = (free_before - torch.cuda.mem_get_info()[0]) / 1e9
    img = out.double()
    checksum = float(img.mean().item())

    persp = view.get("projection") == "perspective"
    ops_per_unit = OPS_PER_RAY_PIXEL if persp else OPS_PER_KINK
    ops = ops_per_unit * kinks
    lds_bytes = 16 * frags if persp else LDS_BYTES_PER_KINK * kinks  # one FP64 add per covered pixel
    raster_s = kernel["raster_ms"] * 1e-3
    achieved = ops / raster_s
    result = {
        "metric": "tets/s and fragments/s at %d^3->%d^2" % (w.n, w.width) if w.width == w.height
                  else "tets/s and fragments/s at %d^3->%dx%d" % (w.n, w.width, w.height),
        "value": w.tets / (ms * 1e-3),
        "unit": "tets/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded Zel'dovich lattice, kmax %d, D %g)" % (w.kmax, w.growth[0]),
        "config": {"workload": w.name, "lattice": w.n, "tets": w.tets, "image": [w.width, w.height],
                   "view": ("perspective, camera at (%g, %g, %g) looking along +z, 90 degrees" % w.camera
                            if persp else "z-projection, periodic"),
                   "determinant": args.precision,
                   "quantity": args.quantity, "method": args.method,
                   **({"lod_radius": args.lod_radius} if args.method == "hybrid" else {}),
                   "tile": [st["tile_rows"], st["tile_cols"]], "chunk": st["chunk"],
                   "block": st["block"]},
        "fragments": frags,
        "fragments_per_s": frags / (ms * 1e-3),
        "spans": spans,
        "kinks": kinks,
        "kernel_ms": kernel,
        "workspace_gb": workspace_gb,
        "own_records": st0.get("own_records"),
        "fp64_dets": st["fp64_dets"],
        "bin_pairs": st["bin_pairs"],
        "work_items": st["work_items"],
        "image_mean": checksum,
        "lds_bytes_per_s_raster": lds_bytes / raster_s,
        "lds_frac_raster": lds_bytes / raster_s / PEAK_LDS_BYTES,
        "roofline": {
            "kernel": "k_raster",
            "bound": "alu",
            "achieved": achieved / 1e12,
            "peak": PEAK_VALU_OPS / 1e12,
            "unit": "Tops/s",
            "frac": achieved / PEAK_VALU_OPS,
            "traffic": raster_traffic(w.name, (st["tile_rows"], st["tile_cols"]), st["block"]),
            "ops_per_launch": ops,
            "ops_per_kink": ops_per_unit,
            "unit_of_work": "pixel evaluated (perspective)" if persp else "kink",
        },
        "fragment_equivalent": {
            "ops_per_fragment": OPS_PER_FRAGMENT,
            "achieved": OPS_PER_FRAGMENT * frags / raster_s / 1e12,
            "unit": "Tops/s",
            "x_peak": OPS_PER_FRAGMENT * frags / raster_s / PEAK_VALU_OPS,
        },
    }
    # the oracle's region mode draws the exact projection (orthographic
    # centroid splats have no region mode)
    if not args.no_cpu_baseline and not (args.method == "centroids" and not persp):
        result["cpu_baseline"] = cpu_baseline(xyz, w, view, float(frags))
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
