"""Writes the oracle's samples of the batched workload to tests/golden/batched_samples.npz.

Expected values for the GPU parity test of the batched workload (128^3
lattice, modes 1..32, snapshots D = 1..8, 64 seeded random rotations, 512^2
windows of side 2): a fixed 16-image subset -- view 0 of every snapshot and
views 1..8 of the last snapshot (D = 8) -- each at 256 seeded random pixels,
computed by the FP64 oracle's pixel-sample mode (calls only oracle/ and the
input generator, never the GPU library).  The file also holds a fingerprint
of every snapshot's FP32 positions, which the test checks first.

Command (a few minutes on 8 host cores):
    python tests/golden/make_batched_samples.py [--threads N]
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

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "batched_samples.npz")
SAMPLES = 256
SAMPLE_SEED = 77


def subset(n_snaps: int):
    """(snapshot, view) pairs of the fixed subset."""
    return [(i, 0) for i in range(n_snaps)] + [(n_snaps - 1, v) for v in range(1, 9)]


def sample_pixels(w: int, h: int):
    rng = np.random.default_rng(SAMPLE_SEED)
    return rng.integers(0, w, SAMPLES).astype(np.int32), rng.integers(0, h, SAMPLES).astype(np.int32)


def fingerprint(xyz) -> np.ndarray:
    rows = []
    for a in xyz:
        a64 = a.astype(np.float64)
        rows.append(np.concatenate([[a64.sum(), (a64 * a64).sum()], a64[:: max(1, a.size // 61)][:61]]))
    return np.stack(rows)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    args = ap.parse_args()
    w = W.BATCHED
    views = W.workload_views(w)
    psi = W.displacement_grid(w.n, w.kmax)
    snaps = [W.zeldovich(w.n, w.kmax, D, psi=psi) for D in w.growth]
    pairs = subset(len(snaps))
    px, py = sample_pixels(w.width, w.height)
    values = np.empty((len(pairs), SAMPLES))
    t0 = time.time()
    for k, (i, v) in enumerate(pairs):
        vals, _ = O.project_pixels(*snaps[i], (w.n,) * 3, views[v], px, py, nthreads=args.threads)
        values[k] = vals
        print(f"image (snapshot {i}, view {v}): mean of samples {vals.mean():.4f}, {time.time() - t0:.0f} s",
              flush=True)
    np.savez_compressed(OUT, pairs=np.array(pairs, dtype=np.int64), px=px, py=py, values=values,
                        fingerprints=np.stack([fingerprint(s) for s in snaps]))
    print("wrote", OUT)


if __name__ == "__main__":
    main()
