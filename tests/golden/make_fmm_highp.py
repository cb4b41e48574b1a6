"""Writes the oracle FMM products at high Chebyshev orders (p = 20 ... 32)
that the GPU parity tests compare against.

The oracle's level-by-level bbFMM (eqs. 3.6-3.11) costs O(p^5) per cell in
its transfer passes, minutes per product at these orders, which is too slow
to run inside a GPU test.  This script runs it once on the CPU and stores
each product in ``fmm_highp_<name>.npz``.  It calls only ``oracle`` and the
seeded input generators of ``workloads``; nothing here comes from the HIP
path.

Each file holds the expected product ``y`` (element-major [t_s, t_n]) and
the case's parameters, plus a checksum of the geometry and the input vector
so that a test notices when the generators have changed.

Usage (from the repository root): python tests/golden/make_fmm_highp.py [name ...]
The cases run in parallel processes, one per case.
"""
from __future__ import annotations

import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

# name: (fracture seed, fractures, elements per fracture, leaf, p, vector seed)
#   random2000: 11 levels, 872 V pairs; p = 20 is the benchmark order and
#               p = 24 the largest order the multipole transfer kernel runs
#               with four leaf slots per block
#   random400:  9 levels; p = 28 and 32 take the two-slot path
CASES = {
    "random2000_p20": (31, 25, 80, 16, 20, 12),
    "random2000_p24": (31, 25, 80, 16, 24, 12),
    "random400_p28": (32, 20, 20, 8, 28, 13),
    "random400_p32": (32, 20, 20, 8, 32, 13),
}


def checksum(wl, D):
    return np.array([np.sum(wl.x1), np.sum(wl.y1), np.sum(wl.x2), np.sum(wl.y2), np.sum(D)])


def case_inputs(name):
    import workloads as W
    seed, nf, ne, leaf, p, vseed = CASES[name]
    wl = W.random_fractures(seed, nf, ne)
    D = W.random_vector(vseed, wl.n)
    return wl, D, leaf, p


def path_of(name):
    return os.path.join(HERE, f"fmm_highp_{name}.npz")


def run(name):
    import oracle as O
    wl, D, leaf, p = case_inputs(name)
    g = O.Geometry.of(wl)
    T = O.Tree(g, leaf=leaf)
    t0 = time.time()
    y = T.fmm(D, p)
    np.savez(path_of(name), y=y, leaf=np.int64(leaf), p=np.int64(p), checksum=checksum(wl, D),
             levels=np.int64(T.level.max() + 1))
    return name, time.time() - t0


if __name__ == "__main__":
    names = sys.argv[1:] or list(CASES)
    with ProcessPoolExecutor(len(names)) as ex:
        for name, dt in ex.map(run, names):
            print(f"{name}: {dt:.0f} s -> {path_of(name)}", flush=True)
