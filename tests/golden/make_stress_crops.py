"""Writes the oracle's stress-config crops to tests/golden/stress_crops.npz.

Expected values for the GPU parity tests of the stress workload (256^3
lattice, modes 1..64, D = 8; z-projection with periodic wrap):
  * crop_2048: pixels [768, 1280)^2 of the 2048^2 image;
  * crop_4096: pixels [1792, 2304)^2 of the 4096^2 image;
  * strip_2048: rows [1024, 1040) of the 2048^2 image at full width, so that
    every row's running sums cross the periodic seam.
Each is the FP64 oracle's region mode (calls only oracle/ and the input
generator, never the GPU library).  The file also holds a fingerprint of
the FP32 input positions, which the tests check before comparing.

Command (about 40 minutes on 8 host cores):
    python tests/golden/make_stress_crops.py [--threads N]
"""
import argparse
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
import workloads as W  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "stress_crops.npz")

# name -> (image side, crop (x0, y0, w, h))
CROPS = {
    "crop_2048": (2048, (768, 768, 512, 512)),
    "crop_4096": (4096, (1792, 1792, 512, 512)),
    "strip_2048": (2048, (0, 1024, 2048, 16)),
}


def fingerprint(xyz) -> np.ndarray:
    """Sum, sum of squares and a strided sample of each coordinate array."""
    rows = []
    for a in xyz:
        a64 = a.astype(np.float64)
        rows.append(np.concatenate([[a64.sum(), (a64 * a64).sum()], a64[:: max(1, a.size // 61)][:61]]))
    return np.stack(rows)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    args = ap.parse_args()
    w = W.STRESS
    xyz = W.zeldovich(w.n, w.kmax, w.growth[0])
    out = {"fingerprint": fingerprint(xyz)}
    for name, (side, crop) in CROPS.items():
        t0 = time.time()
        img, st = O.project_region(*xyz, (w.n,) * 3, W.z_view(side), crop=crop, nthreads=args.threads)
        dt = time.time() - t0
        print(f"{name}: side {side} crop {crop}: {dt:.0f} s, {st['fragments']:.4g} fragments, "
              f"{args.threads} threads", flush=True)
        out[name] = img
        out[name + "_crop"] = np.array(crop, dtype=np.int64)
        out[name + "_side"] = np.array(side, dtype=np.int64)
        out[name + "_fragments"] = np.array(st["fragments"], dtype=np.int64)
        out[name + "_seconds"] = np.array(dt)
    out["threads"] = np.array(args.threads, dtype=np.int64)
    np.savez_compressed(OUT, **out)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
