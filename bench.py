#!/usr/bin/env python3
"""Benchmark: FMM-DDM matrix-vector products per second at N = 20000.

Workload (C2): 200 random pressurized fractures x 100 constant elements
(N = 20000) in a 100 m box, seed 2; FP64 black-box FMM with leaf 32 and
p = 20 Chebyshev nodes per dimension.  One step = one FMM product y = A D
with the tree, lists and M2L operators already built (built once, timed
separately).  Inputs are resident in device memory.

Also reported on the same line: the exact products on the same GPU (stored
dense FP64 matrix, and on-the-fly), the FMM error against the exact product,
the roofline of the dominant FMM kernel (timed with HIP events on the
library's stream, inside the timed region) and the CPU oracle on the host.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {  # MI355X published peaks
    "hbm_GBps": 8000.0,
    "fp64_mfma_TFLOPs": 78.6,
    "fp64_vector_TFLOPs": 78.6,
}
# Algorithmic flop count of one near-field element pair (constant-element
# stress, rotation to the global frame, accumulation): +,-,* count 1, a
# fused multiply-add 2, a division 1.
FLOP_PER_PAIR = 78


def phase_work(info, p, tree, rank, svd):
    """Algorithmic work of each kernel of one FMM product:
    (bound, amount, unit, peak).  Flops count +,-,* as 1 and a fused
    multiply-add as 2; bytes are the compulsory HBM traffic."""
    n = info["n"]
    M = 3 * p * p
    lev, leaf = tree["level"], tree["isleaf"]
    internal = int(((lev >= 2) & (leaf == 0)).sum())
    nleaf, nfar, nV = info["nleaf"], info["nfar"], info["nV"]
    hbm, mfma, alu = PEAK["hbm_GBps"], PEAK["fp64_mfma_TFLOPs"], PEAK["fp64_vector_TFLOPs"]
    slots = 4 if p <= 24 else 2
    work = {
        # D in, sorted D and charges out, permutation, orientation
        "prep": ("hbm", 76.0 * n, "GB/s", hbm),
        # eq. 3.6: the per-element anterpolation matrices streamed once, the
        # charges, the leaf weights written
        "p2m": ("hbm", 8.0 * p * p * n + 24.0 * n + 8.0 * M * nleaf, "GB/s", hbm),
        # eq. 3.7 per (ancestor, leaf) pair: the two p x p composite
        # transfers applied to 3 components (12 p^3), plus forming them
        # (2p barycentric interpolants of about 6p flops)
        "m2m": ("alu", (12.0 * p ** 3 + 12.0 * p * p) * info["m2m_pairs"], "TFLOP/s", alu),
        # item partials read once, the weights of internal cells written once
        "m2m_sum": ("hbm", 8.0 * M * (-(-info["m2m_pairs"] // slots) + internal), "GB/s", hbm),
        # eqs. 3.9-3.11: every (midpoint, ancestor) pair evaluates that
        # ancestor's field there: two barycentric interpolants (about 6p
        # each) and the 3-component p x p contraction (6p^2 + 6p)
        "l2p": ("alu", (6.0 * p * p + 18.0 * p) * info["l2p_pairs"], "TFLOP/s", alu),
        "p2p": ("alu", float(FLOP_PER_PAIR) * info["near_pairs"], "TFLOP/s", alu),
        # far and near stress in, geometry and permutation, tractions out
        "final": ("hbm", 80.0 * n, "GB/s", hbm),
    }
    if svd:
        # projections in and out of the rank-r space, one per far cell, and
        # the r x r operator product per interaction pair (eq. 3.8)
        work["compress"] = ("mfma", 2.0 * rank * M * nfar, "TFLOP/s", mfma)
        work["compress_sum"] = ("hbm", 8.0 * rank * nfar * 5, "GB/s", hbm)
        work["m2l"] = ("mfma", 2.0 * rank * rank * nV, "TFLOP/s", mfma)
        work["m2l_sum"] = ("hbm", 8.0 * rank * (nV + nfar), "GB/s", hbm)
        work["decompress"] = ("mfma", 2.0 * rank * M * nfar, "TFLOP/s", mfma)
    else:
        work["m2l"] = ("mfma", 2.0 * M * M * nV, "TFLOP/s", mfma)
        work["m2l_sum"] = ("hbm", 8.0 * M * (nV + nfar), "GB/s", hbm)
    return work


def kernel_name(phase, p):
    """The library kernel behind each profiled launch."""
    return {"prep": "k_prep", "p2m": "k_p2m", "m2m": f"k_m2m<{p}>", "m2m_sum": "k_m2m_sum",
            "compress": "k_ggemm<32, 32> (projection)", "compress_sum": "k_reduce_split",
            "m2l": "k_ggemm<64, 32> (pair products)", "m2l_sum": "k_sum_pairs",
            "decompress": "k_ggemm<64, 32> (back-projection)", "l2p": f"k_l2p<{p}>", "p2p": "k_p2p",
            "final": "k_final"}[phase]


def kernel_source_hash():
    h = hashlib.sha256()
    for f in sorted(os.listdir(os.path.join(ROOT, "paper_1812_05087_amd", "csrc"))):
        with open(os.path.join(ROOT, "paper_1812_05087_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_for(phase):
    """HBM bytes per launch from the committed rocprofv3 counter summary,
    or None when absent or taken on different kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic_c2.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("source_hash") != kernel_source_hash():
        return None
    return d.get("phases", {}).get(phase, {}).get("bytes_per_launch")


def cpu_baseline(wl, D, seconds):
    """The oracle's exact on-the-fly product of the whole workload on all
    host cores, repeated for about `seconds` of wall time."""
    import oracle as O
    g = O.Geometry.of(wl)
    O.direct_matvec_rows(g, D, [0])  # load the library
    reps, t0 = 0, time.perf_counter()
    while True:
        O.direct_matvec(g, D)
        reps += 1
        dt = time.perf_counter() - t0
        if dt >= seconds:
            break
    return {"value": reps / dt, "unit": "matvecs/s", "cores": O.num_threads(), "kind": "oracle",
            "sample": f"oracle exact on-the-fly product of the full workload (N={g.n}), "
                      f"{reps} products in {dt:.1f} s wall"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--p", type=int, default=20)
    ap.add_argument("--leaf", type=int, default=32)
    ap.add_argument("--exact-steps", type=int, default=20)
    ap.add_argument("--m2l", choices=["svd", "dense"], default="svd")
    ap.add_argument("--m2l-tol", type=float, default=1e-12)
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-dense", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build runs one instance per GPU and has no "
              "multi-GPU path; run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1812_05087_amd as F
    import workloads as W

    torch.cuda.set_device(0)
    wl = W.c2()
    n = wl.n
    t0 = time.perf_counter()
    svd = args.m2l == "svd"
    prob = F.Problem(wl.x1, wl.y1, wl.x2, wl.y2, E=wl.E, nu=wl.nu, leaf=args.leaf, p=args.p,
                     m2l=F.FMDDM_M2L_SVD if svd else F.FMDDM_M2L_DENSE, m2l_tol=args.m2l_tol)
    torch.cuda.synchronize()
    tree_ms = (time.perf_counter() - t0) * 1e3
    info = prob.info
    Dh = W.random_vector(5, n)
    D = prob.vec(Dh)
    out = prob.vec()
    t0 = time.perf_counter()
    prob.apply(D, F.FMDDM_APPLY_FMM, out)  # first product builds operators and buffers
    torch.cuda.synchronize()
    setup_ms = (time.perf_counter() - t0) * 1e3
    for _ in range(args.warmup):
        prob.apply(D, F.FMDDM_APPLY_FMM, out)
    # which phase dominates
    F.fmddm_profile(prob.ctx, (1 << len(F.PHASES)) - 1)
    for _ in range(5):
        prob.apply(D, F.FMDDM_APPLY_FMM, out)
    ph = F.fmddm_profile_read(prob.ctx)
    phase_ms = {k: v[0] / max(v[1], 1) for k, v in ph.items()}
    dom = max(phase_ms, key=phase_ms.get)
    # timed region: K products, the dominant phase bracketed by HIP events
    F.fmddm_profile(prob.ctx, 1 << F.PHASES.index(dom))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        prob.apply(D, F.FMDDM_APPLY_FMM, out)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    dom_tot, dom_cnt = F.fmddm_profile_read(prob.ctx)[dom]
    F.fmddm_profile(prob.ctx, 0)
    dom_ms = dom_tot / max(dom_cnt, 1)
    value = args.steps / elapsed
    y_fmm = out.cpu().numpy()

    # exact products on the same GPU
    exact = {}
    modes = [("direct", F.FMDDM_APPLY_DIRECT)] + ([] if args.no_dense else [("dense", F.FMDDM_APPLY_DENSE)])
    y_ref = None
    for name, mode in modes:
        o = prob.vec()
        prob.apply(D, mode, o)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.exact_steps):
            prob.apply(D, mode, o)
        torch.cuda.synchronize()
        exact[name] = args.exact_steps / (time.perf_counter() - t1)
        if y_ref is None:
            y_ref = o.cpu().numpy()
    err = float(np.linalg.norm(y_fmm - y_ref) / np.linalg.norm(y_ref))

    info = F.fmddm_tree_get_info(prob.ctx, prob.tree)
    tree = F.fmddm_tree_export(prob.ctx, prob.tree)
    work = phase_work(info, args.p, tree, info["m2l_rank"], svd)
    scale = {"GB/s": 1e9, "TFLOP/s": 1e12}
    phases = {}
    for ph, (bound, amount, unit, peak) in work.items():
        ms = phase_ms.get(ph, 0.0)
        if ms <= 0:
            continue
        ach = amount / (ms * 1e-3) / scale[unit] if ms > 0 else None
        phases[ph] = {"ms": ms, "bound": bound, "work": amount, "achieved": ach, "unit": unit,
                      "frac": ach / peak if ach else None}
    bound, amount, unit, peak = work[dom]
    achieved = amount / (dom_ms * 1e-3) / scale[unit]
    roof = {"bound": bound, "kernel": kernel_name(dom, args.p), "achieved": achieved, "peak": peak, "unit": unit,
            "frac": achieved / peak, "traffic": traffic_for(dom), "avg_launch_ms": dom_ms}

    line = {
        "metric": "FMM-DDM matvecs/s at N=20k vs dense; served solves/s + p99 latency",
        "value": value,
        "unit": "matvecs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "C2: 200 random pressurized fractures x 100 elements, N=20000, "
                               "seed 2, FP64 FMM leaf 32 p=20",
                   "N": n, "leaf": args.leaf, "p": args.p, "m2l": args.m2l,
                   "m2l_tol": args.m2l_tol if svd else None, "m2l_rank": info["m2l_rank"]},
        "vs_dense": {
            "dense_matvecs_per_s": exact.get("dense"),
            "direct_matvecs_per_s": exact.get("direct"),
            "fmm_over_dense": value / exact["dense"] if "dense" in exact else None,
            "fmm_over_direct": value / exact["direct"],
            "fmm_rel_err_vs_exact": err,
        },
        "phases": phases,
        "tree_build_ms": tree_ms,
        "first_product_setup_ms": setup_ms,
        "tree": {k: info[k] for k in ("ncell", "nleaf", "nlevel", "nV", "nfar", "near_pairs",
                                      "l2p_pairs", "m2m_pairs")},
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(wl, Dh, args.cpu_seconds)
    prob.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
