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

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {  # MI355X published peaks
    "hbm_GBps": 8000.0,
    "fp64_mfma_TFLOPs": 78.6,
    "fp64_vector_TFLOPs": 78.6,
    "fp32_vector_TFLOPs": 157.3,   # packed; the kernels here issue non-packed FP32 (half of it)
    "fp32_mfma_TFLOPs": 157.3,
    "bf16_mfma_TFLOPs": 2500.0,    # dense
}
# Algorithmic flop count of one near-field element pair (constant-element
# stress, rotation to the global frame, accumulation): +,-,* count 1, a
# fused multiply-add 2, a division 1.
FLOP_PER_PAIR = 78


def phase_work(info, p, tree, rank, svd):
    """Algorithmic work of each kernel of one FMM product:
    (bound, amount, unit, peak, executed).  `amount` is the method's own
    count (the per-unit figures of the bbFMM steps, eqs. 3.6-3.11);
    `executed` is what the kernel computes where its restructuring differs
    (None where it is the same).  Flops count +,-,* as 1 and a fused
    multiply-add as 2; bytes are the compulsory HBM traffic."""
    n = info["n"]
    c = 3                      # charge / field components per node
    M = c * p * p
    nleaf, nfar, nV = info["nleaf"], info["nfar"], info["nV"]
    hbm, mfma, alu = PEAK["hbm_GBps"], PEAK["fp64_mfma_TFLOPs"], PEAK["fp64_vector_TFLOPs"]
    # child-to-parent transfers of the upward pass (cells whose parent has
    # an expansion); the downward pass has the same number of L2L transfers
    transfers = info["m2m_pairs"]
    lev, leaf = tree["level"], tree["isleaf"]
    parents = int(((lev >= 2) & (leaf == 0)).sum())
    work = {
        # D in, sorted D and charges out, permutation, orientation
        "prep": ("hbm", 76.0 * n, "GB/s", hbm, None),
        # eq. 3.6: the per-element anterpolation matrices streamed once, the
        # charges, the leaf weights written
        "p2m": ("hbm", 8.0 * p * p * n + 24.0 * n + 8.0 * M * nleaf, "GB/s", hbm, None),
        # eq. 3.7: two p x p passes over c components per child transfer,
        # 4 p^3 c; the kernel shares the y pass of children with equal y side
        # (a p^3 c x pass per child and two 2 p^3 c y passes per parent)
        "m2m": ("alu", 4.0 * p ** 3 * c * transfers, "TFLOP/s", alu,
                2.0 * p ** 3 * c * transfers + 4.0 * p ** 3 * c * parents),
        # eqs. 3.9-3.11: an L2L transfer per child (4 p^3 c) and the p^2-node
        # interpolation at every midpoint (2 p^2 c); the kernel evaluates
        # every ancestor's field at the midpoint directly: two barycentric
        # interpolants (about 6p each) and the c-component p x p contraction
        "l2p": ("alu", 4.0 * p ** 3 * c * transfers + 2.0 * p * p * c * n, "TFLOP/s", alu,
                (6.0 * p * p + 18.0 * p) * info["l2p_pairs"]),
        "p2p": ("alu", float(FLOP_PER_PAIR) * info["near_pairs"], "TFLOP/s", alu, None),
        # far and near stress in, geometry and permutation, tractions out
        "final": ("hbm", 80.0 * n, "GB/s", hbm, None),
    }
    if svd:
        # projections in and out of the rank-r space, one per far cell, and
        # the r x r operator product per interaction pair (eq. 3.8)
        work["compress"] = ("mfma", 2.0 * rank * M * nfar, "TFLOP/s", mfma, None)
        work["compress_sum"] = ("hbm", 8.0 * rank * nfar * 5, "GB/s", hbm, None)
        work["m2l"] = ("mfma", 2.0 * rank * rank * nV, "TFLOP/s", mfma, None)
        work["m2l_sum"] = ("hbm", 8.0 * rank * (nV + nfar), "GB/s", hbm, None)
        work["decompress"] = ("mfma", 2.0 * rank * M * nfar, "TFLOP/s", mfma, None)
    else:
        work["m2l"] = ("mfma", 2.0 * M * M * nV, "TFLOP/s", mfma, None)
        work["m2l_sum"] = ("hbm", 8.0 * M * (nV + nfar), "GB/s", hbm, None)
    return work


def kernel_name(phase, p):
    """The library kernel behind each profiled launch."""
    return {"prep": "k_prep", "p2m": "k_p2m", "m2m": f"k_m2m<{p}, 3>",
            "compress": "k_ggemm<32, 32, *> (projection)", "compress_sum": "k_reduce_split<double>",
            "m2l": "k_ggemm<64, 32, *> (pair products)", "m2l_sum": "k_sum_pairs<double, double>",
            "decompress": "k_ggemm<64, 32, *> (back-projection)", "l2p": f"k_l2p<{p}, 3>",
            "p2p": "k_p2p<double>", "final": "k_final"}[phase]


# the sources of the FMM product's kernels (the ones the traffic file covers)
TRAFFIC_SOURCES = ("fmm.hip", "elem.h")


def kernel_source_hash():
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, "paper_1812_05087_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_for(phase):
    """HBM bytes per product from the committed rocprofv3 counter summary,
    or None when absent or taken on different kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic_c2.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("source_hash") != kernel_source_hash():
        return None
    ph = d.get("phases", {}).get(phase, {})
    # per product, like the roofline's work and time (the upward pass is
    # several launches per product)
    return ph.get("bytes_per_product", ph.get("bytes_per_launch"))


# direct_below: the exact on-the-fly product beats the FMM's chain of
# launches below about 3000 elements on MI355X (0.048 vs 0.074 ms at 2000,
# 0.093 vs 0.078 ms at 4000)
# coarse_aggregates: a 128-aggregate coarse level keeps the coarse LU per
# request small (33.7 vs 26.1 solves/s batched with 1024 aggregates on
# MI355X; block-Jacobi alone 29.2)
SERVE_PARAMS = dict(p=10, leaf=32, m2l=1, m2l_tol=1e-10, restart=50, maxit=20000, use_graphs=0, direct_below=3000,
                    coarse_aggregates=128)


# the poroelastic medium of the horizontal-well example (Section 5.2.1,
# Table 2; drained E, nu of the well example), 60 s steps
SERVE_PORO = dict(E=20e9, nu=0.2, nu_u=0.35, alpha=0.8, perm=1e-18, visc=1e-3, dt=60.0, p0=48.26e6)
# the left-hand side's M2L of a poroelastic request: 1 compressed (bases
# shared per cell size over the requests), 0 dense
SERVE_PORO_M2L = 1


FAILED = {}  # request index -> status of the last serve_run's failed requests


def serve_run(F, wls, reqs, slots, arrivals, precond=2, precision=0, poro=False, failed=FAILED):
    """Serve the requests with `slots` admission slots; request i is
    submitted at arrivals[i] seconds.  Returns (makespan s, latencies s).
    poro: requests are poroelastic time marches (steps of 60 s)."""
    extra = dict(E=SERVE_PORO["E"], nu=SERVE_PORO["nu"]) if poro else {}
    prm = F.fmddm_default_params(**SERVE_PARAMS, **extra, precond=precond, precision=precision)
    srv = F.fmddm_server_create(prm, slots)
    if poro:
        m = SERVE_PORO
        F.fmddm_server_set_poro(srv, m["nu_u"], m["alpha"], m["perm"], m["visc"], m["dt"], m["p0"],
                                m2l=SERVE_PORO_M2L)
    try:
        warm = F.fmddm_server_submit(srv, wls[0].x1, wls[0].y1, wls[0].x2, wls[0].y2, wls[0].pressure,
                                     wls[0].SH, wls[0].Sh, 1, 1e-6)
        while F.fmddm_server_poll(srv, warm)[0]["state"] < F.FMDDM_REQ_DONE:
            F.fmddm_server_step(srv)
        order = sorted(range(len(reqs)), key=lambda i: arrivals[i])
        tickets, pend, done = {}, 0, {}
        failed.clear()
        t0 = time.perf_counter()
        while len(done) < len(reqs):
            now = time.perf_counter() - t0
            while pend < len(order) and arrivals[order[pend]] <= now:
                i = order[pend]
                w = wls[i]
                tickets[i] = F.fmddm_server_submit(srv, w.x1, w.y1, w.x2, w.y2, w.pressure, w.SH, w.Sh,
                                                   reqs[i].steps, 1e-6)
                pend += 1
            active, queued = F.fmddm_server_step(srv)
            if active + queued == len(tickets) - len(done):
                continue  # nothing finished in this step
            for i, t in tickets.items():
                if i not in done:
                    r = F.fmddm_server_poll(srv, t)[0]
                    if r["state"] >= F.FMDDM_REQ_DONE:
                        if r["state"] != F.FMDDM_REQ_DONE:
                            failed[i] = r["status"]
                            print(f"serving: request {i} (N={wls[i].n}, {reqs[i].steps} steps) failed, "
                                  f"status {r['status']}", file=sys.stderr, flush=True)
                        done[i] = r
        t_first = min(r["t_submit"] for r in done.values())
        span = max(r["t_done"] for r in done.values()) - t_first
        lat = np.array([r["t_done"] - r["t_submit"] for r in done.values()])
        iters = int(sum(r["iters"] for r in done.values()))
        return span, lat, iters
    finally:
        F.fmddm_server_destroy(srv)


def serving_leg(F, W, count, slots, load, poro=True, alone_sample=128):
    """Serving of the seed-5 request stream (random fractures at C2's
    density, N log-uniform in [1e3, 5e4], 1-10 steps, tol 1e-6), GMRES with
    the two-level preconditioner (block-Jacobi plus a 128-aggregate coarse
    level).  poro: every request is a poroelastic time march of its steps
    (60 s each, the well example's medium) with the history sum; else
    elastic load steps (a pressure ramp).  Measured: the one-at-a-time
    service rate (on the first `alone_sample` requests), the batched
    saturation rate (all `count` arriving at once), and a Poisson stream at
    `load` x the batched saturation rate served batched and one at a time
    (solves/s, p50/p99 latency).  At most 100 elastic requests, also the
    batched saturation rates with block-Jacobi alone, without
    preconditioning (the paper's plain GMRES) and with FP32 products."""
    reqs = W.serving_stream(5, count)
    wls = [r.workload() for r in reqs]
    zero = [0.0] * count
    def note(what, k, span):
        print(f"serving: {what} done, {k / span:.1f} solves/s", file=sys.stderr, flush=True)

    k1 = min(alone_sample, count)
    span1, _, _ = serve_run(F, wls[:k1], reqs[:k1], 1, zero[:k1], poro=poro)
    note("one at a time", k1, span1)
    rate1 = k1 / span1
    spanb, _, iters = serve_run(F, wls, reqs, slots, zero, poro=poro)
    failures = {"batched": dict(FAILED)}
    note("batched", count, spanb)
    rateb = count / spanb
    lam = load * rateb
    arr = [r.arrival_units / lam for r in reqs]
    spans, lat, _ = serve_run(F, wls, reqs, slots, arr, poro=poro)
    failures["poisson_batched"] = dict(FAILED)
    note("Poisson batched", count, spans)
    span_o, lat_o, _ = serve_run(F, wls, reqs, 1, arr, poro=poro)
    failures["poisson_one_at_a_time"] = dict(FAILED)
    note("Poisson one at a time", count, span_o)
    pct = lambda a, q: float(np.percentile(a, q))
    comp = {}
    if count <= 100 and not poro:  # the comparison runs (plain GMRES is ~7x slower)
        span_np, _, iters_np = serve_run(F, wls, reqs, slots, zero, precond=0)
        span_32, _, iters_32 = serve_run(F, wls, reqs, slots, zero, precision=F.FMDDM_PREC_FP32)
        span_bj, _, iters_bj = serve_run(F, wls, reqs, slots, zero, precond=F.FMDDM_PRECOND_BLOCK)
        comp = {
            "unpreconditioned": {"batched_saturated_solves_per_s": count / span_np,
                                 "gmres_products_total": iters_np},
            "block_jacobi": {"batched_saturated_solves_per_s": count / span_bj, "gmres_products_total": iters_bj},
            "fp32_products": {"batched_saturated_solves_per_s": count / span_32,
                              "gmres_products_total": iters_32,
                              "note": "Arnoldi on FP32-P2P/FP32-M2L products, residuals and stopping test FP64"},
        }
    return {
        "requests": count, "slots": slots, "elements_total": int(sum(w.n for w in wls)),
        "gmres_products_total": iters,
        "params": {"p": SERVE_PARAMS["p"], "leaf": SERVE_PARAMS["leaf"], "m2l": "svd 1e-10", "tol": 1e-6,
                   "poro_lhs_m2l": ("compressed per cell size, shared by the slots (power-of-two root squares)"
                                    if poro and SERVE_PORO_M2L else "dense"),
                   "restart": SERVE_PARAMS["restart"],
                   "precond": f"two-level: block-Jacobi ({21 if poro else 32}-element groups) + coarse level of "
                              f"{SERVE_PARAMS['coarse_aggregates']} aggregates",
                   "graphs": bool(SERVE_PARAMS["use_graphs"]),
                   "exact_product_at_or_below_elements": None if poro else SERVE_PARAMS["direct_below"]},
        **comp,
        "one_at_a_time_solves_per_s": rate1, "one_at_a_time_sample": k1,
        "batched_saturated_solves_per_s": rateb,
        "poisson_rate_per_s": lam, "poisson_load": f"{load} x the batched saturation rate",
        "served": {"solves_per_s": count / spans, "p50_s": pct(lat, 50), "p99_s": pct(lat, 99)},
        "one_at_a_time_same_stream": {"solves_per_s": count / span_o, "p50_s": pct(lat_o, 50),
                                      "p99_s": pct(lat_o, 99)},
        "failed_requests": {k: {str(i): st for i, st in v.items()} for k, v in failures.items()},
        "kind": ("poroelastic time marches (60 s steps, history sum, FMM on product and history; "
                 "medium of the well example: E 20 GPa, nu 0.2, nu_u 0.35, alpha 0.8, k 1e-18 m^2, "
                 "mu 1e-3 Pa s, p0 48.26 MPa)" if poro else "elastic quasi-static load steps (pressure ramp)"),
        "note": f"the first {count} requests of the seed-5 stream",
    }


def history_run(F, W, elems, steps, mode, p, near_cache=0, m2l=0):
    """One left-hand-side product and the history sum of step `steps` on the
    horizontal-well cluster (5 fractures of `elems` 0.2 m elements, 10 m
    apart; Biot constants of the well example, 60 s steps), timed after a
    first pass that builds the multipole operators and, with the near-field
    cache (near_cache >= 0), integrates every time level's near blocks once;
    that first pass is timed too."""
    import torch
    wl = W.well_cluster(n_frac=5, elems=elems, half_length=0.1 * elems, spacing=10.0)
    prob = F.Problem(wl.x1, wl.y1, wl.x2, wl.y2, E=20e9, nu=0.2, p=p, leaf=32)
    try:
        F.fmddm_poro_set(prob.ctx, 0.35, 0.8, 1e-18, 1e-3, 60.0, 48.26e6, mode=mode, near_cache_bytes=near_cache,
                         m2l=m2l)
        n3 = 3 * prob.n
        rng = np.random.default_rng(3)
        scale = np.tile([1e-4, 1e-4, 1e-10], prob.n)
        hist = torch.as_tensor(np.concatenate([rng.standard_normal(n3) * scale
                                               for _ in range(steps - 1)])).cuda()
        D = hist[:n3].clone()
        out = torch.zeros(n3, dtype=torch.float64, device="cuda")
        rhs = torch.zeros(n3, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        F.fmddm_poro_apply(prob.ctx, prob.tree, 0, D, out)        # builds operators
        F.fmddm_add_history(prob.ctx, prob.tree, steps, hist, rhs)
        torch.cuda.synchronize()
        t_first = time.perf_counter() - t0
        t0 = time.perf_counter()
        F.fmddm_poro_apply(prob.ctx, prob.tree, 0, D, out)
        torch.cuda.synchronize()
        t_lhs = time.perf_counter() - t0
        t0 = time.perf_counter()
        F.fmddm_add_history(prob.ctx, prob.tree, steps, hist, rhs)
        torch.cuda.synchronize()
        t_hist = time.perf_counter() - t0
        return prob.n, t_lhs, t_hist, out.cpu().numpy(), rhs.cpu().numpy(), t_first
    finally:
        prob.close()


def history_leg(F, W, elems, steps, p=16):
    """Poroelastic time marching (the left-hand-side product and the history
    sum over earlier steps): multipole form at the full well-cluster size,
    and multipole against exact evaluation at a tenth of it."""
    small = max(elems // 10, 40)
    out = {"dt_s": 60.0, "history_of_step": steps, "time_levels": steps, "p": p}
    n, tl, th, o_c, r_c, tf = history_run(F, W, elems, steps, F.FMDDM_APPLY_FMM, p)
    _, tl0, th0, o_0, r_0, tf0 = history_run(F, W, elems, steps, F.FMDDM_APPLY_FMM, p, near_cache=-1)
    out["fmm_full"] = {"workload": f"well cluster 5 x {elems} elements (N={n})", "lhs_product_ms": tl * 1e3,
                       "history_ms": th * 1e3, "lag_applications_per_s": (steps - 1) / th,
                       "first_pass_ms": tf * 1e3,
                       "near_on_the_fly": {"lhs_product_ms": tl0 * 1e3, "history_ms": th0 * 1e3,
                                           "first_pass_ms": tf0 * 1e3}}
    n2, tl2, th2, o_f, r_f, _ = history_run(F, W, small, steps, F.FMDDM_APPLY_FMM, p)
    _, tl3, th3, o_e, r_e, _ = history_run(F, W, small, steps, F.FMDDM_APPLY_DIRECT, p)
    rel = lambda a, b: float(max(np.abs(a[k::3] - b[k::3]).max() / max(np.abs(b[k::3]).max(), 1e-300)
                                 for k in range(3)))
    out["small"] = {"workload": f"well cluster 5 x {small} elements (N={n2})",
                    "fmm": {"lhs_product_ms": tl2 * 1e3, "history_ms": th2 * 1e3},
                    "exact": {"lhs_product_ms": tl3 * 1e3, "history_ms": th3 * 1e3},
                    "fmm_err_vs_exact": {"lhs": rel(o_f, o_e), "history": rel(r_f, r_e)}}
    out["fmm_full"]["stored_vs_on_the_fly"] = {"lhs": rel(o_c, o_0), "history": rel(r_c, r_0)}
    _, tlc, _, o_s, _, tfc = history_run(F, W, elems, steps, F.FMDDM_APPLY_FMM, p, m2l=F.FMDDM_M2L_SVD)
    out["fmm_full"]["lhs_m2l_compressed"] = {
        "lhs_product_ms": tlc * 1e3, "first_pass_ms": tfc * 1e3, "diff_vs_uncompressed": rel(o_s, o_c),
        "note": "left-hand side M2L compressed per cell size (m2l_tol 1e-10); the first pass includes the "
                "range finder and the compressed operators"}
    return out


def precision_leg(F, W, steps, tune, leaf, p, solve_tol=1e-8, target_err=1e-6, solves=True):
    """Mixed precision at N=200000 (2000 random fractures x 100 elements,
    seed 4): autotuned leaf and p for the FP64 product, then products and
    solves at FP64, FP32 and BF16-M2L on that configuration (two-level
    preconditioned GMRES; the FP64 solve also unpreconditioned and with
    block-Jacobi alone).  Errors of each
    product against the FP64 FMM product and the exact product (on-the-fly
    FP64 on the GPU); each solve reaches tol on the FP64 FMM residual, and
    its exact-operator residual and distance to the FP64 solve are stated."""
    import torch
    wl = W.c4()
    n = wl.n
    out = {"workload": "2000 random pressurized fractures x 100 elements, N=200000, seed 4", "N": n,
           "solve_tol": solve_tol}
    common = dict(E=wl.E, nu=wl.nu, m2l=F.FMDDM_M2L_SVD, m2l_tol=1e-10, restart=50, maxit=30000)
    if tune:
        base = F.fmddm_default_params(**common)
        t0 = time.perf_counter()
        st, best, log = F.fmddm_autotune(base, wl.x1, wl.y1, wl.x2, wl.y2, leaves=(16, 32, 64, 128),
                                         ps=tuple(range(8, 25, 2)), target_err=target_err, reps=5)
        out["autotune"] = {"seconds": time.perf_counter() - t0, "target_err": target_err, "status": st,
                           "leaf": best.leaf, "p": best.p, "m2l_tiles": best.m2l_tiles, "tried": log}
        leaf, p, tiles = best.leaf, best.p, best.m2l_tiles
    else:
        tiles = 0
    out["leaf"], out["p"], out["m2l_tiles"] = leaf, p, tiles
    common["m2l_tiles"] = tiles
    D = None
    res = {}
    y = {}
    x = {}
    b = None
    ref = None
    for name, prec in [("fp64", F.FMDDM_PREC_FP64), ("fp32", F.FMDDM_PREC_FP32), ("bf16", F.FMDDM_PREC_BF16)]:
        prob = F.Problem(wl.x1, wl.y1, wl.x2, wl.y2, leaf=leaf, p=p, precision=prec, tol=solve_tol,
                         precond=F.FMDDM_PRECOND_TWO_LEVEL, **common)
        if D is None:
            D = prob.vec(W.random_vector(9, n))
            b = prob.rhs(wl.pressure, wl.SH, wl.Sh)
        o = prob.vec()
        prob.apply(D, F.FMDDM_APPLY_FMM, o)
        for _ in range(3):
            prob.apply(D, F.FMDDM_APPLY_FMM, o)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            prob.apply(D, F.FMDDM_APPLY_FMM, o)
        torch.cuda.synchronize()
        r = {"matvecs_per_s": steps / (time.perf_counter() - t0)}
        # per-kernel times (HIP events on each kernel's stream)
        F.fmddm_profile(prob.ctx, (1 << len(F.PHASES)) - 1)
        for _ in range(3):
            prob.apply(D, F.FMDDM_APPLY_FMM, o)
        ph = F.fmddm_profile_read(prob.ctx)
        F.fmddm_profile(prob.ctx, 0)
        r["phase_ms"] = {k: v[0] / 3 for k, v in ph.items() if v[1] > 0}   # per product
        # the near field and the M2L pair products against the peak of the
        # arithmetic they run in (work by the method's own count)
        ti = F.fmddm_tree_get_info(prob.ctx, prob.tree)
        rk = ti["m2l_rank"]
        alu_peak = PEAK["fp64_vector_TFLOPs"] if name == "fp64" else PEAK["fp32_vector_TFLOPs"]
        mf_peak = {"fp64": PEAK["fp64_mfma_TFLOPs"], "fp32": PEAK["fp32_mfma_TFLOPs"],
                   "bf16": PEAK["bf16_mfma_TFLOPs"]}[name]
        rl = {}
        for ph_name, flop, peak, what in (
                ("p2p", float(FLOP_PER_PAIR) * ti["near_pairs"], alu_peak,
                 "FP64 vector" if name == "fp64" else "FP32 vector (published, packed)"),
                ("m2l", 2.0 * rk * rk * ti["nV"], mf_peak, f"{name.upper()} MFMA")):
            ms = r["phase_ms"].get(ph_name, 0.0)
            if ms > 0:
                tf = flop / (ms * 1e-3) / 1e12
                rl[ph_name] = {"achieved_TFLOPs": tf, "peak_TFLOPs": peak, "frac": tf / peak, "peak_kind": what,
                               "work_flop": flop, "ms": ms}
        r["roofline"] = rl
        y[name] = o.cpu().numpy()
        if not solves:              # products only (profiling runs)
            prob.close()
            res[name] = r
            continue
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        xs, info = prob.solve(b)
        torch.cuda.synchronize()
        r["solve_s"] = time.perf_counter() - t0
        r["solve"] = info
        x[name] = xs
        if name == "fp64":
            ref = prob            # kept for the exact products below
            # the paper's unpreconditioned GMRES on the same FP64 product
            prob0 = F.Problem(wl.x1, wl.y1, wl.x2, wl.y2, leaf=leaf, p=p, tol=solve_tol, **common)
            prob0.apply(D, F.FMDDM_APPLY_FMM, o)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, info0 = prob0.solve(b)
            torch.cuda.synchronize()
            out["fp64_unpreconditioned_solve"] = {"solve_s": time.perf_counter() - t0, "solve": info0}
            prob0.close()
            # the same with block-Jacobi alone (set-up timed apart)
            prob2 = F.Problem(wl.x1, wl.y1, wl.x2, wl.y2, leaf=leaf, p=p, tol=solve_tol,
                              precond=F.FMDDM_PRECOND_BLOCK, **common)
            prob2.apply(D, F.FMDDM_APPLY_FMM, o)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            x2, info2 = prob2.solve(b)
            torch.cuda.synchronize()
            t_first = time.perf_counter() - t0
            t0 = time.perf_counter()
            x2, info2 = prob2.solve(b)
            torch.cuda.synchronize()
            out["fp64_block_jacobi_solve"] = {"solve_s": time.perf_counter() - t0, "first_solve_s": t_first,
                                              "solve": info2}
            x["fp64_block_jacobi"] = x2
            prob2.close()
        else:
            prob.close()
        res[name] = r
    if not solves:
        out["precisions"] = res
        return out
    # exact (on-the-fly FP64) products on the GPU
    ex = ref.apply(D, F.FMDDM_APPLY_DIRECT)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ref.apply(D, F.FMDDM_APPLY_DIRECT, ex)
    torch.cuda.synchronize()
    out["direct_matvecs_per_s"] = 1.0 / (time.perf_counter() - t0)
    ex = ex.cpu().numpy()
    rel = lambda a, c: float(np.abs(a - c).max() / np.abs(c).max())
    bn = float(torch.linalg.norm(b))
    for name in res:
        res[name]["product_err_vs_fp64_fmm"] = rel(y[name], y["fp64"])
        res[name]["product_err_vs_exact"] = rel(y[name], ex)
        ax = ref.apply(x[name], F.FMDDM_APPLY_DIRECT)
        res[name]["solution_exact_residual"] = float(torch.linalg.norm(b - ax)) / bn
        res[name]["solution_diff_vs_fp64_solve"] = float(torch.linalg.norm(x[name] - x["fp64"]) /
                                                         torch.linalg.norm(x["fp64"]))
        res[name]["matvecs_over_fp64"] = res[name]["matvecs_per_s"] / res["fp64"]["matvecs_per_s"]
        res[name]["solve_speedup_over_fp64"] = res["fp64"]["solve_s"] / res[name]["solve_s"]
    if "fp64_block_jacobi" in x:
        tl = out["fp64_block_jacobi_solve"]
        ax = ref.apply(x["fp64_block_jacobi"], F.FMDDM_APPLY_DIRECT)
        tl["solution_exact_residual"] = float(torch.linalg.norm(b - ax)) / bn
        tl["solution_diff_vs_fp64_solve"] = float(torch.linalg.norm(x["fp64_block_jacobi"] - x["fp64"]) /
                                                  torch.linalg.norm(x["fp64"]))
    ref.close()
    out["precisions"] = res
    return out


def march_run(F, W, elems, steps, p, restart, precond, coarse, tol, keep=(), mode=None, m2l=1):
    """One poroelastic time march (the horizontal-well example's shape,
    Section 5.2.1): 5 fractures of `elems` 0.2 m elements 10 m apart,
    `steps` steps of 60 s, every step's history sum and GMRES solve (the
    given tolerance, restart and preconditioner: 2 two-level, 1
    block-Jacobi) on the multipole operators.  Returns the timings and the
    DDs (caller order, [D_s, D_n, D_q] per element) after the steps in
    `keep`."""
    import torch
    wl = W.well_cluster(n_frac=5, elems=elems, half_length=0.1 * elems, spacing=10.0)
    n3 = 3 * wl.n
    prob = F.Problem(wl.x1, wl.y1, wl.x2, wl.y2, E=20e9, nu=0.2, p=p, leaf=32, m2l=1, m2l_tol=1e-10, tol=tol,
                     restart=restart, maxit=40000, precond=precond, coarse_aggregates=coarse)
    F.fmddm_poro_set(prob.ctx, 0.35, 0.8, 1e-18, 1e-3, 60.0, 48.26e6,
                     mode=F.FMDDM_APPLY_FMM if mode is None else mode, m2l=m2l)
    b0 = torch.zeros(n3, dtype=torch.float64, device="cuda")
    F.fmddm_poro_rhs(prob.ctx, prob.tree, torch.as_tensor(wl.pressure).cuda(), wl.SH, wl.Sh, b0)
    hist = torch.zeros(steps * n3, dtype=torch.float64, device="cuda")
    D = torch.zeros(n3, dtype=torch.float64, device="cuda")
    t_setup = 0.0
    if mode == F.FMDDM_APPLY_DENSE:  # assemble the dense left-hand side outside the timed march
        tmp = torch.zeros(n3, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        F.fmddm_poro_apply(prob.ctx, prob.tree, 0, D, tmp)
        torch.cuda.synchronize()
        t_setup = time.perf_counter() - t0
    th = tsv = 0.0
    its, worst, per_step, kept, step_s = 0, 0.0, [], {}, []
    torch.cuda.synchronize()
    t_all = time.perf_counter()
    for h in range(1, steps + 1):
        t0 = time.perf_counter()
        rhs = b0.clone()
        F.fmddm_add_history(prob.ctx, prob.tree, h, hist[: (h - 1) * n3] if h > 1 else None, rhs)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        st, info = F.fmddm_poro_solve(prob.ctx, prob.tree, rhs, D)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        if st != F.FMDDM_OK:
            raise RuntimeError(f"march step {h}: {info}")
        hist[(h - 1) * n3: h * n3] = D
        th += t1 - t0
        tsv += t2 - t1
        its += info["iters"]
        per_step.append(info["iters"])
        step_s.append(t2 - t0)
        worst = max(worst, info["relres"])
        if h in keep:
            kept[h] = D.cpu().numpy().reshape(-1, 3).copy()
        if wl.n > 5000:
            print(f"march (tol {tol:g}) step {h}: {info['iters']} products, {t2 - t0:.2f} s", file=sys.stderr,
                  flush=True)
    total = time.perf_counter() - t_all
    Dm = D.cpu().numpy().reshape(-1, 3)
    tinfo = F.fmddm_tree_get_info(prob.ctx, prob.tree)
    rank = tinfo["poro_m2l_rank"]
    prob.close()
    return {"total_s": total, "history_s": th, "solve_s": tsv, "gmres_products": its, "per_step": per_step,
            "max_step_relres": worst, "last": Dm, "kept": kept, "n": wl.n, "setup_s": t_setup, "step_s": step_s,
            "lhs_m2l_rank": rank,
            "tree": {k: tinfo[k] for k in ("ncell", "nleaf", "nlevel", "nV", "near_pairs")}}


def middle_ratio(Dm, elems):
    """max |D_s| on the middle fracture over max |D_n| of the cluster (the
    stack is symmetric about it, so its shear is zero, Section 5.2.1)."""
    mid = Dm[2 * elems: 3 * elems]
    return float(np.abs(mid[:, 0]).max() / np.abs(Dm[:, 1]).max())


def march_leg(F, W, elems, steps, p=16, restart=100, precond=2, coarse=0, ref_tol=1e-10, ref_steps=10, low_p=10):
    """The full C3 march at GMRES tol 1e-6 (the paper's), timed, and its
    accuracy: the first ref_steps steps again at ref_tol (the solver's
    error at this tolerance), and the same steps with p = low_p against
    that reference (the interpolation error of a lower order: on the long
    parallel fractures the solution amplifies the operator's error on
    smooth DDs, 1.1e-5 at p = 10 against 7e-9 at p = 16).  Per unknown
    kind (D_s, D_n, D_q): the largest difference over the largest
    reference value; and the middle fracture's shear over the opening,
    zero by symmetry (Section 5.2.1)."""
    keep = tuple(sorted({1, min(ref_steps, steps), steps}))
    red = march_run(F, W, 40, 10, p, restart, precond, coarse, 1e-6, m2l=0)
    run = march_run(F, W, elems, steps, p, restart, precond, coarse, 1e-6, keep)
    out = {"workload": f"well cluster 5 x {elems} elements (N={run['n']}), {steps} steps of 60 s", "p": p,
           "lhs_m2l": f"compressed per cell size (m2l_tol 1e-10), largest rank {run['lhs_m2l_rank']} of {4 * p * p}",
           "tree": run["tree"],
           "restart": restart, "precond": {1: "block-Jacobi", 2: "two-level"}[precond], "tol": 1e-6,
           "gmres_products_per_step": run["per_step"], "total_s": run["total_s"], "history_s": run["history_s"],
           "solve_s": run["solve_s"], "gmres_products": run["gmres_products"],
           "max_step_relres": run["max_step_relres"],
           "middle_fracture_max_shear_over_opening": middle_ratio(run["last"], elems),
           "reduced": {"workload": "5 x 40 elements (N=200), 10 steps (the oracle's C3 run; cpu_baseline "
                                   "c3_reduced_march)", "total_s": red["total_s"], "gmres_products": red["gmres_products"]}}

    def diff(a, r):
        return {name: float(np.abs(a[:, k] - r[:, k]).max() / np.abs(r[:, k]).max())
                for k, name in enumerate(("D_s", "D_n", "D_q"))}

    if ref_tol and ref_steps:
        rs = min(ref_steps, steps)
        k2 = tuple(sorted({1, rs}))
        ref = march_run(F, W, elems, rs, p, restart, precond, coarse, ref_tol, k2, m2l=0)
        acc = {f"step_{h}": diff(run["kept"][h], ref["kept"][h]) for h in k2}
        out["accuracy_vs_reference"] = {
            "reference": f"the same march (p = {p}, uncompressed M2L) at GMRES tol {ref_tol:g}, {rs} steps",
            "reference_total_s": ref["total_s"], "reference_gmres_products": ref["gmres_products"],
            "max_diff_over_max_ref": acc,
            f"middle_fracture_max_shear_over_opening_step_{rs}": middle_ratio(run["kept"][rs], elems),
            f"reference_middle_fracture_max_shear_over_opening_step_{rs}": middle_ratio(ref["kept"][rs], elems)}
        unc = march_run(F, W, elems, rs, p, restart, precond, coarse, 1e-6, k2, m2l=0)
        out["uncompressed_lhs_m2l_first_steps"] = {
            "steps": rs, "total_s": unc["total_s"], "solve_s": unc["solve_s"], "gmres_products": unc["gmres_products"],
            "compressed": {"total_s": float(sum(run["step_s"][:rs])), "gmres_products": sum(run["per_step"][:rs])}}
        # the history-only variant (Section 2: the earlier method applied
        # the FMM to the history sum only): dense exact left-hand side,
        # multipole history, same steps and tolerance
        ho = march_run(F, W, elems, rs, p, restart, precond, coarse, 1e-6, k2, mode=F.FMDDM_APPLY_DENSE)
        fmm_first = sum(run["per_step"][:rs])
        out["history_only"] = {
            "steps": rs, "dense_lhs_assembly_s": ho["setup_s"], "total_s": ho["total_s"],
            "history_s": ho["history_s"], "solve_s": ho["solve_s"], "gmres_products": ho["gmres_products"],
            "fmm_on_both_first_steps": {"gmres_products": fmm_first, "seconds": float(sum(run["step_s"][:rs]))},
            "max_diff_over_max_ref": {f"step_{h}": diff(ho["kept"][h], ref["kept"][h]) for h in k2},
            "note": "left-hand side F(dt) a stored dense 3N x 3N matrix of exact element integrals "
                    "(FMDDM_APPLY_DENSE), history sum by FMM; the reference is the FMM-on-both march"}
        if low_p:
            low = march_run(F, W, elems, rs, low_p, restart, precond, coarse, 1e-6, k2)
            out["lower_order"] = {
                "p": low_p, "total_s": low["total_s"], "gmres_products": low["gmres_products"],
                "max_diff_over_max_ref": {f"step_{h}": diff(low["kept"][h], ref["kept"][h]) for h in k2},
                f"middle_fracture_max_shear_over_opening_step_{rs}": middle_ratio(low["kept"][rs], elems)}
    return out


def p_sweep_leg(F, W, ps, reps=50):
    """Accuracy against time over the number of Chebyshev nodes per dimension
    (the paper compares 3 and 6, Section 5.2): the C2 product (SVD M2L at
    1e-12, leaf 32) against the exact on-the-fly product, and the C3
    left-hand side (well cluster, FMM on both the product and the history)
    at N = 2000 against its exact evaluation, timed at N = 20 000."""
    import torch

    def timed(apply, reps):
        apply()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            apply()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps * 1e3

    out = {"c2": [], "c3_lhs": []}
    wl = W.c2()
    ref = None
    for p in ps:
        prob = F.Problem(wl.x1, wl.y1, wl.x2, wl.y2, E=wl.E, nu=wl.nu, leaf=32, p=p, m2l=F.FMDDM_M2L_SVD,
                         m2l_tol=1e-12)
        D = prob.vec(W.random_vector(5, wl.n))
        o = prob.vec()
        if ref is None:
            r = prob.vec()
            prob.apply(D, F.FMDDM_APPLY_DIRECT, r)
            ref = r.cpu().numpy()
        ms = timed(lambda: prob.apply(D, F.FMDDM_APPLY_FMM, o), reps)
        y = o.cpu().numpy()
        out["c2"].append({"p": p, "ms_per_product": ms,
                          "rel_err_vs_exact": float(np.linalg.norm(y - ref) / np.linalg.norm(ref))})
        prob.close()
    rel = lambda a, b: float(max(np.abs(a[k::3] - b[k::3]).max() / max(np.abs(b[k::3]).max(), 1e-300)
                                 for k in range(3)))
    for p in [q for q in ps if q <= 16]:
        _, _, _, o_f, _, _ = history_run(F, W, 400, 2, F.FMDDM_APPLY_FMM, p)
        if p == ps[0]:
            _, _, _, o_e, _, _ = history_run(F, W, 400, 2, F.FMDDM_APPLY_DIRECT, p)
        _, tl, _, _, _, _ = history_run(F, W, 4000, 2, F.FMDDM_APPLY_FMM, p)
        out["c3_lhs"].append({"p": p, "lhs_ms_N20000": tl * 1e3, "rel_err_vs_exact_N2000": rel(o_f, o_e)})
    return out


def n_sweep_leg(F, W, ns, reps=5):
    """Time per product against N (the shape of the paper's one-step timing
    figures, Section 5.1: the conventional method grows as N^2, the
    multipole one as N): random fractures at C2's density (100 elements
    each, box scaled with sqrt(N)), the exact on-the-fly product and the
    FMM product (leaf 32, p = 20, SVD M2L at 1e-12) on the GPU, with the
    log-log slopes fitted over the sizes."""
    import torch

    def timed(apply, k):
        apply()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(k):
            apply()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / k * 1e3

    rows = []
    for n in ns:
        nf = max(1, n // 100)
        wl = W.random_fractures(100 + nf, nf, 100, box=100.0 * np.sqrt(nf / 200.0))
        prob = F.Problem(wl.x1, wl.y1, wl.x2, wl.y2, E=wl.E, nu=wl.nu, leaf=32, p=20, m2l=F.FMDDM_M2L_SVD,
                         m2l_tol=1e-12)
        try:
            D = prob.vec(W.random_vector(5, wl.n))
            o = prob.vec()
            fmm = timed(lambda: prob.apply(D, F.FMDDM_APPLY_FMM, o), max(reps, 20))
            direct = timed(lambda: prob.apply(D, F.FMDDM_APPLY_DIRECT, o), reps if wl.n <= 50000 else 2)
            rows.append({"N": wl.n, "fmm_ms": fmm, "direct_ms": direct})
            print(f"n-sweep: N={wl.n} fmm {fmm:.3f} ms direct {direct:.3f} ms", file=sys.stderr, flush=True)
        finally:
            prob.close()
    x = np.log([r["N"] for r in rows])
    big = x >= np.log(5000)  # the asymptotic range: below it both are launch-latency bound
    slope = lambda key: float(np.polyfit(x[big], np.log([r[key] for r in rows])[big], 1)[0])
    return {"workload": "random fractures at C2's density, 100 elements each", "rows": rows,
            "slope_fmm": slope("fmm_ms"), "slope_direct": slope("direct_ms"),
            "fit_range": "N >= 5000"}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(wl, D, seconds, fmm_p=6, others=True):
    """The oracle on the host: its exact on-the-fly product of the whole
    workload on all host cores, repeated for about `seconds` of wall time
    (the reported value); the same product on one thread over 1000 rows
    (scaled to whole products); and the oracle's level-by-level FMM at
    p = fmm_p (the paper's six Chebyshev nodes, Section 5.2) on one
    thread; with `others`, 1000 exact rows of the N = 200 000 workload and
    the whole poroelastic march at 5 x 40 elements, 10 steps (C3 reduced),
    on all host cores."""
    import oracle as O
    g = O.Geometry.of(wl)
    O.direct_matvec_rows(g, D, [0])  # load the library
    cores = O.num_threads()
    reps, times, t0 = 0, [], time.perf_counter()
    while True:
        t1 = time.perf_counter()
        O.direct_matvec(g, D)
        times.append(time.perf_counter() - t1)
        reps += 1
        dt = time.perf_counter() - t0
        if dt >= seconds:
            break
    prev = O.set_num_threads(1)
    try:
        rows = min(1000, g.n)
        t1 = time.perf_counter()
        O.direct_matvec(g, D, rows=(0, rows))
        t_rows = time.perf_counter() - t1
        T = O.Tree(g, leaf=32)
        t1 = time.perf_counter()
        T.fmm(D, fmm_p)
        t_fmm = time.perf_counter() - t1
    finally:
        O.set_num_threads(prev)
    ms = np.array(times) * 1e3
    extra = {}
    if others:
        import workloads as W
        # N = 200 000 (C4): exact rows on all host cores, scaled to products
        w4 = W.c4()
        g4 = O.Geometry.of(w4)
        D4 = W.random_vector(9, g4.n)
        rows4 = np.random.default_rng(1).choice(g4.n, 1000, replace=False)
        O.direct_matvec_rows(g4, D4, rows4[:2])
        t1 = time.perf_counter()
        O.direct_matvec_rows(g4, D4, rows4)
        t4 = time.perf_counter() - t1
        extra["c4_exact_rows"] = {"rows": len(rows4), "seconds": t4, "threads": cores,
                                  "exact_matvecs_per_s_scaled": len(rows4) / g4.n / t4,
                                  "sample": f"1000 random rows of the N = {g4.n} exact product"}
        # C3 at reduced size: the whole poroelastic march, 5 x 40 elements,
        # 10 steps of 60 s (dense exact operators and LU per step)
        wl3 = W.well_cluster(n_frac=5, elems=40, half_length=4.0, spacing=10.0)
        g3 = O.Geometry.of(wl3)
        po = O.Poro(E=20e9, nu=0.2, nuu=0.35, alpha=0.8, perm=1e-18, visc=1e-3)
        t1 = time.perf_counter()
        O.poro_march(g3, po, 60.0, 10, wl3.pressure, 48.26e6, wl3.SH, wl3.Sh)
        t3 = time.perf_counter() - t1
        extra["c3_reduced_march"] = {"n": g3.n, "steps": 10, "seconds": t3, "threads": cores,
                                     "sample": "oracle poroelastic march, well cluster 5 x 40 elements, 10 steps"}
    return {"value": reps / dt, "unit": "matvecs/s", "cores": cores, "kind": "oracle", **extra,
            "cpu_model": cpu_model(),
            "sample": f"oracle exact on-the-fly product of the full workload (N={g.n}) on {cores} threads, "
                      f"{reps} products in {dt:.1f} s wall",
            "product_ms_median": float(np.median(ms)), "product_ms_p90": float(np.percentile(ms, 90)),
            "single_thread_exact_matvecs_per_s": rows / g.n / t_rows,
            "single_thread_exact_sample": f"{rows} of {g.n} rows in {t_rows:.2f} s, scaled to whole products",
            "oracle_fmm_single_thread": {"p": fmm_p, "leaf": 32, "seconds_per_product": t_fmm,
                                         "note": "level-by-level bbFMM with dense M2L, plain C"}}


def c1_leg(F, W, reps=200, solve_reps=5, cpu=True):
    """C1, the pressurized Griffith crack (N = 256; Section 2.1, eq. 2.6):
    microseconds per product (stored dense matrix, on-the-fly exact, FMM at
    the library's default p = 20 and leaf 32), GMRES(50) to 1e-10 from zero
    on each (median of `solve_reps` solves), the opening's relative L2
    error against Sneddon's ellipse and K_I by eq. 2.6 against
    p sqrt(pi a); with `cpu`, the oracle's dense assembly and GMRES(50)
    solve on one thread and on all host cores."""
    import torch
    wl = W.c1()
    n, pr, a = wl.n, wl.meta["p"], wl.meta.get("a", 1.0)
    prob = F.Problem(wl.x1, wl.y1, wl.x2, wl.y2, E=wl.E, nu=wl.nu, tol=1e-10, restart=50)
    out = {"workload": f"Griffith crack, a = {a} m, N = {n}, p = {pr / 1e6:.0f} MPa, E = {wl.E / 1e9:.0f} GPa, "
                       f"nu = {wl.nu}", "gmres": "restart 50, tol 1e-10, x0 = 0"}
    try:
        D = prob.vec(W.random_vector(1, n))
        o = prob.vec()
        b = prob.rhs(wl.pressure, 0.0, 0.0)
        xm = 0.5 * (wl.x1 + wl.x2)
        w_exact = 4.0 * (1.0 - wl.nu ** 2) * pr / wl.E * np.sqrt(np.maximum(a * a - xm * xm, 0.0))
        K_exact = pr * np.sqrt(np.pi * a)
        for name, mode in (("dense", F.FMDDM_APPLY_DENSE), ("direct", F.FMDDM_APPLY_DIRECT),
                           ("fmm", F.FMDDM_APPLY_FMM)):
            prob.apply(D, mode, o)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                prob.apply(D, mode, o)
            torch.cuda.synchronize()
            us = (time.perf_counter() - t0) / reps * 1e6
            prob.solve(b, mode)
            ts = []
            for _ in range(solve_reps):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                x, info = prob.solve(b, mode)
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
            xn = x.cpu().numpy()
            KI, KII = F.fmddm_sif(prob.ctx, prob.tree, x, n - 1)
            out[name] = {"us_per_product": us, "solve_ms_median": float(np.median(ts)) * 1e3,
                         "gmres_iters": info["iters"], "relres": info["relres"],
                         "sneddon_rel_l2": float(np.linalg.norm(xn[1::2] - w_exact) / np.linalg.norm(w_exact)),
                         "KI_over_exact": KI / K_exact}
    finally:
        prob.close()
    if cpu:
        import oracle as O
        g = O.Geometry.of(wl)
        bo = O.rhs(g, wl.pressure, 0.0, 0.0)
        res = {}
        for label, th in (("1_thread", 1), ("all_cores", 0)):
            prev = O.set_num_threads(th)
            try:
                cores = O.num_threads()
                ta, tsv = [], []
                for _ in range(3):
                    t0 = time.perf_counter()
                    A = O.dense_matrix(g)
                    t1 = time.perf_counter()
                    xo, info = O.gmres_dense(A, bo, restart=50, tol=1e-10)
                    t2 = time.perf_counter()
                    ta.append(t1 - t0)
                    tsv.append(t2 - t1)
            finally:
                O.set_num_threads(prev)
            res[label] = {"threads": cores, "assembly_ms_median": float(np.median(ta)) * 1e3,
                          "solve_ms_median": float(np.median(tsv)) * 1e3, "gmres_iters": info["iters"]}
        res["cpu_model"] = cpu_model()
        out["oracle_cpu"] = res
    return out


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
    ap.add_argument("--c1-reps", type=int, default=200,
                    help="products timed per mode on the Griffith crack, C1 (0 skips the leg)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-dense", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=1024)
    ap.add_argument("--serve-kind", choices=["poro", "elastic"], default="poro")
    ap.add_argument("--serve-slots", type=int, default=8)
    ap.add_argument("--serve-load", type=float, default=0.75)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only copy 256 MiB device-to-device 5 times (reference for HBM byte counters)")
    ap.add_argument("--history-elems", type=int, default=4000)
    ap.add_argument("--history-steps", type=int, default=10)
    ap.add_argument("--march-elems", type=int, default=4000)
    ap.add_argument("--march-steps", type=int, default=50,
                    help="poroelastic time steps of the full-march leg (0 skips it)")
    ap.add_argument("--march-restart", type=int, default=100)
    ap.add_argument("--march-precond", type=int, default=2, choices=[1, 2])
    ap.add_argument("--march-p", type=int, default=16)
    ap.add_argument("--march-ref-tol", type=float, default=1e-10,
                    help="GMRES tol of the reference march the C3 accuracy is measured against (0: none)")
    ap.add_argument("--p-sweep", type=str, default="3,6,10,16,20",
                    help="comma-separated Chebyshev orders for the accuracy/time sweep ('' skips it)")
    ap.add_argument("--n-sweep", type=str, default="1000,2000,5000,10000,20000,50000,100000,200000",
                    help="comma-separated element counts for the time-per-product sweep ('' skips it)")
    ap.add_argument("--precision-steps", type=int, default=20,
                    help="products timed per precision at N=200000 (0 skips the mixed-precision leg)")
    ap.add_argument("--precision-no-tune", action="store_true")
    ap.add_argument("--precision-no-solve", action="store_true", help="products only (profiling runs)")
    ap.add_argument("--precision-leaf", type=int, default=64)
    ap.add_argument("--precision-p", type=int, default=10)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library runs one instance per GPU and has no "
              "multi-GPU path; run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1812_05087_amd as F
    import workloads as W

    torch.cuda.set_device(0)
    if args.calibrate_copy:
        nbytes = 256 << 20
        src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "launches": 5}), flush=True)
        return
    # measured roofline denominators (FMA loop, MFMA loop, stream copy)
    peaks = F.fmddm_measure_peaks()
    measured = {"alu": peaks["fp64_vector_tflops"], "mfma": peaks["fp64_mfma_tflops"],
                "hbm": peaks["copy_gbps"]}
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
    # per product (a phase may take more than one launch, on different streams)
    phase_ms = {k: v[0] / 5 for k, v in ph.items()}
    phase_launches = {k: v[1] / 5 for k, v in ph.items()}
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
    dom_ms = dom_tot / args.steps          # kernel time per product
    value = args.steps / elapsed
    y_fmm = out.cpu().numpy()
    # distribution of single products: HIP events on the stream the
    # product runs on (the near field's side stream joins back into it)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(min(args.steps, 200))]
    for e0, e1 in evs:
        e0.record()
        prob.apply(D, F.FMDDM_APPLY_FMM, out)
        e1.record()
    torch.cuda.synchronize()
    one = np.array([e0.elapsed_time(e1) for e0, e1 in evs])

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
    for ph, (bound, amount, unit, peak, executed) in work.items():
        ms = phase_ms.get(ph, 0.0)
        if ms <= 0:
            continue
        ach = amount / (ms * 1e-3) / scale[unit] if ms > 0 else None
        phases[ph] = {"ms": ms, "launches": phase_launches.get(ph), "bound": bound, "work": amount,
                      "achieved": ach, "unit": unit, "frac": ach / peak if ach else None,
                      "frac_measured": ach / measured[bound] if ach else None}
        if executed is not None:
            phases[ph]["work_executed"] = executed
    bound, amount, unit, peak, executed = work[dom]
    # launches of the dominant kernel per product (the upward pass is one
    # launch per schedule step)
    dom_launches = info["m2m_launches"] if dom == "m2m" else 1
    achieved = amount / (dom_ms * 1e-3) / scale[unit]
    roof = {"bound": bound, "kernel": kernel_name(dom, args.p), "achieved": achieved, "peak": peak, "unit": unit,
            "frac": achieved / peak, "traffic": traffic_for(dom), "work": amount,
            "work_basis": "per product: the bbFMM step's own per-unit count (eqs. 3.6-3.11) x units",
            "work_executed": executed, "ms_per_product": dom_ms,
            "launches_per_product": dom_launches,
            "avg_launch_ms": dom_ms / dom_launches, "peak_measured": measured[bound],
            "frac_measured": achieved / measured[bound]}

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
        "product_ms_median": float(np.median(one)), "product_ms_p90": float(np.percentile(one, 90)),
        "phases": phases,
        "tree_build_ms": tree_ms,
        "first_product_setup_ms": setup_ms,
        "tree": {k: info[k] for k in ("ncell", "nleaf", "nlevel", "nV", "nfar", "near_pairs",
                                      "l2p_pairs", "m2m_pairs")},
        "roofline": roof,
        "measured_peaks": {"fp64_vector_TFLOP/s": peaks["fp64_vector_tflops"],
                           "fp64_mfma_TFLOP/s": peaks["fp64_mfma_tflops"], "copy_GB/s": peaks["copy_gbps"],
                           "kernels": "FP64 FMA loop, FP64 16x16x4 MFMA loop, 1 GiB device copy"},
    }
    prob.close()
    if args.c1_reps > 0:
        line["c1"] = c1_leg(F, W, args.c1_reps, cpu=not args.no_cpu_baseline)
    if args.serve_requests > 0:
        line["serving"] = serving_leg(F, W, args.serve_requests, args.serve_slots, args.serve_load,
                                      poro=args.serve_kind == "poro")
    if args.history_elems > 0:
        line["history"] = history_leg(F, W, args.history_elems, args.history_steps)
    if args.p_sweep:
        line["p_sweep"] = p_sweep_leg(F, W, [int(q) for q in args.p_sweep.split(",")])
    if args.n_sweep:
        line["n_sweep"] = n_sweep_leg(F, W, [int(q) for q in args.n_sweep.split(",")])
    if args.march_steps > 0:
        line["march"] = march_leg(F, W, args.march_elems, args.march_steps, p=args.march_p,
                                  restart=args.march_restart, precond=args.march_precond, ref_tol=args.march_ref_tol)
    if args.precision_steps > 0:
        line["mixed_precision"] = precision_leg(F, W, args.precision_steps, not args.precision_no_tune,
                                                args.precision_leaf, args.precision_p,
                                                solves=not args.precision_no_solve)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(wl, Dh, args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
