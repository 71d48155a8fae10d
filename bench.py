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
# add, multiply, min and max issue at one lane-operation per lane per clock
# (the same rate as unpacked FP32), so that is the ceiling of its arithmetic.
PEAK_VALU_OPS = 256 * 4 * 16 * 2.4e9          # 3.93e13 lane-ops/s
# Algorithmic FP64 operations of one span (one tetrahedron on one pixel row
# of one tile): 4 line offsets (FMA), 4 zero crossings + 2 clamps, 6 pair
# crossings (subtract, multiply), 12 min/max for the pieces' ends, and per
# break point (3.5 on average: the pieces holding a sample, plus the end)
# step, slope change, floor, fraction and the two entries (8).
OPS_PER_SPAN = 4 + 6 + 12 + 12 + 28
# Its LDS traffic: two FP64 read-modify-writes per break point.
LDS_BYTES_PER_SPAN = 3.5 * 2 * 16
PEAK_LDS_BYTES = 256 * 128 * 2.4e9            # 128 B/clk/CU: 78.6 TB/s


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
    ap.add_argument("--cpu-crop", type=int, default=48,
                    help="edge (pixels) of the centred crop the oracle renders for the CPU baseline")
    return ap.parse_args()


def cpu_baseline(xyz, w, view, full_fragments: float):
    """The FP64 oracle on a bounded sample of the same workload (test harness code).

    Two oracle runs: one pixel (the per-tetrahedron setup of all tetrahedra,
    which a full image pays once) and a centred crop (setup plus the clip work
    of the crop's fragments).  Full-image time = setup + (crop - setup) scaled
    by the fragment ratio."""
    import numpy as np
    import oracle
    threads = oracle.default_threads()
    c = w.width // 2
    e = int(args.cpu_crop)
    crop = (c - e // 2, c - e // 2, e, e)
    t0 = time.perf_counter()
    oracle.project_pixels(*xyz, (w.n,) * 3, view, np.array([c]), np.array([c]), nthreads=threads)
    t_setup = time.perf_counter() - t0
    t0 = time.perf_counter()
    _, st = oracle.project_region(*xyz, (w.n,) * 3, view, crop=crop, nthreads=threads)
    t_crop = time.perf_counter() - t0
    frac = st["fragments"] / max(full_fragments, 1.0)
    t_frag = max(t_crop - t_setup, 1e-9)
    t_full = t_setup + t_frag / max(frac, 1e-30)
    return {
        "value": w.tets / t_full,
        "unit": "tets/s",
        "cores": threads,
        "kind": "oracle",
        "sample": (f"FP64 oracle: per-tet setup of all {w.tets} tets ({t_setup:.1f} s) and the "
                   f"{e}x{e} crop at ({crop[0]},{crop[1]}) of the same image ({st['fragments']:.3e} "
                   f"fragments, {t_crop:.1f} s); full image = setup + crop clip time scaled by "
                   f"fragment count ({t_full:.0f} s)"),
        "fragments_per_s": st["fragments"] / t_frag,
        "seconds": t_setup + t_crop,
    }


def main():
    global args
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported "
              "(this build shows one GPU's share of the work)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    import paper_1208_3206_amd as tess
    import workloads as W

    w = W.ALL[args.workload]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    t0 = time.perf_counter()
    xyz = W.zeldovich(w.n, w.kmax, w.growth[0])
    gen_s = time.perf_counter() - t0
    d = [torch.from_numpy(a).to(dev) for a in xyz]
    view = W.workload_views(w)[0]
    lat = tess.build(*d, (w.n,) * 3, precision=args.precision)
    out = torch.empty((w.height, w.width), dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream()

    tune = tess.make_tune(args.tile_rows, args.tile_cols, args.chunk, args.block)
    _, st0 = tess.project(lat, view, out=out, tune=tune, stats=True)
    frags, spans = st0["fragments"], st0["spans"]
    for _ in range(args.warmup):
        tess.project(lat, view, out=out, tune=tune)
    torch.cuda.synchronize()

    per_step = []
    kernel = {"setup_ms": 0.0, "bin_ms": 0.0, "raster_ms": 0.0, "finalize_ms": 0.0}
    t_start = time.perf_counter()
    for _ in range(args.steps):
        _, st = tess.project(lat, view, out=out, tune=tune, stats=True)
        per_step.append(st["ms"])
        for k in kernel:
            kernel[k] += st[k] / args.steps
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    ms = wall * 1e3 / args.steps
    img = out.double()
    checksum = float(img.mean().item())

    ops = OPS_PER_SPAN * spans
    raster_s = kernel["raster_ms"] * 1e-3
    achieved = ops / raster_s
    result = {
        "metric": "tets/s and fragments/s at 256^3->2048^2",
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
        "data": "synthetic (seeded Zel'dovich lattice, kmax 64, D 8)",
        "config": {"workload": w.name, "lattice": w.n, "tets": w.tets, "image": [w.width, w.height],
                   "view": "z-projection, periodic", "determinant": args.precision,
                   "tile": [st["tile_rows"], st["tile_cols"]], "chunk": st["chunk"],
                   "block": st["block"]},
        "fragments": frags,
        "fragments_per_s": frags / (ms * 1e-3),
        "spans": spans,
        "kernel_ms": kernel,
        "fp64_dets": st["fp64_dets"],
        "bin_pairs": st["bin_pairs"],
        "work_items": st["work_items"],
        "image_mean": checksum,
        "lds_bytes_per_s_raster": LDS_BYTES_PER_SPAN * spans / raster_s,
        "lds_frac_raster": LDS_BYTES_PER_SPAN * spans / raster_s / PEAK_LDS_BYTES,
        "roofline": {
            "kernel": "k_raster",
            "bound": "alu",
            "achieved": achieved / 1e12,
            "peak": PEAK_VALU_OPS / 1e12,
            "unit": "Tops/s",
            "frac": achieved / PEAK_VALU_OPS,
            "traffic": None,
            "ops_per_launch": ops,
            "ops_per_span": OPS_PER_SPAN,
        },
    }
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(xyz, w, view, float(frags))
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
