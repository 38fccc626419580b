"""Writes bumps1025_oracle_samples.npz: the oracle's FMM solution of the 1025^3 Gaussian-bumps
workload (32 bumps, seed 4, FP32 speeds, centre exit) at a seeded sample of nodes, with the
sha256 of the speed field it was computed on.

The full oracle solve takes about 25 minutes and 45 GB of host memory, so it runs once, here,
and the GPU test compares the device's FP64 solution with these values at the same nodes (and
checks first that it solved the same speeds, by the hash).  Samples: 32768 nodes drawn
uniformly (seed 1306), the three axis lines through the exit and the main diagonal.

    python tests/golden/make_bumps1025_oracle_samples.py
"""
import hashlib
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1306_4743_amd import workloads as W  # noqa: E402

N, SEED = 1025, 4
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "bumps1025_oracle_samples.npz")


def sample_nodes(n: int) -> np.ndarray:
    """Flat indices ([k][j][i] order) of the sampled nodes, sorted and unique."""
    rng = np.random.default_rng(1306)
    pick = rng.integers(0, n ** 3, size=32768, dtype=np.int64)
    c = (n - 1) // 2
    t = np.arange(n, dtype=np.int64)
    lines = [c * n * n + c * n + t,          # along x through the exit
             c * n * n + t * n + c,          # along y
             t * n * n + c * n + c,          # along z
             t * n * n + t * n + t]          # main diagonal
    return np.unique(np.concatenate([pick] + lines))


def main():
    t0 = time.perf_counter()
    p = W.bumps(N, seed=SEED)
    sha = hashlib.sha256(np.ascontiguousarray(p.F).tobytes()).hexdigest()
    print(f"speeds built in {time.perf_counter() - t0:.0f} s, sha256 {sha}", flush=True)
    t0 = time.perf_counter()
    U = oracle.fmm(p.F, p.h, p.src, p.q, progress=1 << 27)
    print(f"oracle FMM {N}^3: {time.perf_counter() - t0:.0f} s", flush=True)
    idx = sample_nodes(N)
    vals = U.reshape(-1)[idx].copy()
    del U
    np.savez(OUT, n=np.int64(N), seed=np.int64(SEED), f_sha256=np.array(sha), idx=idx, u=vals)
    print(f"wrote {OUT}: {idx.size} samples", flush=True)


if __name__ == "__main__":
    main()
