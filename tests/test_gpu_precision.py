"""Reduced-precision FMM products and the mixed-precision solve on the GPU,
through the C ABI.

Precisions (fmddm_precision): FP32 runs the near field (P2P) in FP32 and
the M2L products on FP32 MFMA; BF16 keeps the FP32 near field and rounds the
M2L operators and weights to bf16 (FP32 sums).  Everything else stays FP64.

Bars (max norm, relative to the largest entry of the compared outputs):
  - FP32 near field.  Per pair the element formulas lose about u32 * (r/a)
    to cancellation (differences of the two end-point terms, u32 = 6e-8),
    r/a up to a few hundred inside a near list, on terms that decay like
    (a/r)^2 against the largest (self) term: 2e-6 (measured 2e-7).
  - The far field alone (two clusters 80 m apart, sources in one, outputs
    read in the other, so every interaction goes through M2L).  A sum
    y = sum_k a_k x_k of rounded operands errs by at most 2 u sum_k |a_k x_k|,
    i.e. 2 u rho relative to y with rho = sum |a_k x_k| / |y| the sum's
    cancellation; three such products are chained (projection, translation,
    expansion).  FP32 (u = 2^-24): 1e-5 leaves rho ~ 30 per product.  BF16
    (8 significand bits, u = 2^-8, both operands rounded: 2u = 7.8e-3 per
    product at rho = 1, 2.3e-2 for the three in the worst case).  Rounding
    errors of many terms add like a random walk, far below that bound:
    measured 6.4e-3 (SVD) and 3.9e-3 (uncompressed), and the kernels are
    deterministic, so the bar 1.2e-2 (2x the larger) holds them with room
    for other inputs.  A wrong lane layout or a dropped pass gives O(1).
  - Iterative refinement stops on the FP64 FMM residual <= tol; the
    solutions then agree with the FP64 solve to about cond(A) * tol
    (bar 1e-7 at tol 1e-8; measured 3e-9) and with the oracle's LU solve to
    that plus the FMM's own error.
Each reduced-precision product is also compared with the oracle's exact
product, and the error is printed.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_1812_05087_amd as F  # noqa: E402

PRECS = {"fp32": F.FMDDM_PREC_FP32, "bf16": F.FMDDM_PREC_BF16}
NEAR_BAR = 2e-6                          # FP32 near field, whole product
FAR_BAR = {"fp32": 1e-5, "bf16": 1.2e-2}  # far field alone


def rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def product(wl, prec, D, **kw):
    prob = F.Problem(wl.x1, wl.y1, wl.x2, wl.y2, E=wl.E, nu=wl.nu, precision=prec, **kw)
    try:
        y = prob.apply(prob.vec(D), F.FMDDM_APPLY_FMM).cpu().numpy()
        info = F.fmddm_tree_get_info(prob.ctx, prob.tree)
    finally:
        prob.close()
    return y, info


@pytest.mark.parametrize("m2l", [F.FMDDM_M2L_SVD, F.FMDDM_M2L_DENSE])
def test_reduced_precision_products(m2l):
    wl = W.random_fractures(21, n_frac=40, elems=50)
    g = O.Geometry.of(wl)
    D = W.random_vector(4, g.n)
    exact = O.direct_matvec(g, D)
    kw = dict(p=12, leaf=32, m2l=m2l, m2l_tol=1e-10)
    y64, info = product(wl, F.FMDDM_PREC_FP64, D, **kw)
    assert info["nV"] > 0
    e64 = rel(y64, exact)
    assert e64 <= 1e-6, e64
    for name, prec in PRECS.items():
        y, _ = product(wl, prec, D, **kw)
        e_fmm, e_ex = rel(y, y64), rel(y, exact)
        print(f"m2l={m2l} {name}: vs FP64 FMM {e_fmm:.2e}, vs exact (oracle) {e_ex:.2e} (FP64 FMM {e64:.2e})")
        assert e_fmm <= NEAR_BAR + (FAR_BAR[name] if name == "bf16" else 0.0), (name, e_fmm)
        assert e_ex <= NEAR_BAR + (FAR_BAR[name] if name == "bf16" else 0.0) + e64, (name, e_ex)


def two_clusters():
    a = W.random_fractures(31, n_frac=15, elems=40, box=10.0)
    b = W.random_fractures(32, n_frac=15, elems=40, box=10.0)
    cat = lambda u, v, sh: np.concatenate([u, v + sh])
    return (cat(a.x1, b.x1, 85.0), cat(a.y1, b.y1, 85.0), cat(a.x2, b.x2, 85.0), cat(a.y2, b.y2, 85.0),
            a.n, a.E, a.nu)


@pytest.mark.parametrize("m2l", [F.FMDDM_M2L_SVD, F.FMDDM_M2L_DENSE])
def test_far_field_alone(m2l):
    x1, y1, x2, y2, na, E, nu = two_clusters()
    g = O.Geometry(x1, y1, x2, y2, E, nu)
    D = W.random_vector(8, g.n)
    D[2 * na:] = 0.0                     # sources in the first cluster only
    rows = np.arange(na, g.n)            # outputs in the second
    exact = O.direct_matvec_rows(g, D, rows).reshape(-1)
    out = {}
    for name, prec in [("fp64", F.FMDDM_PREC_FP64)] + list(PRECS.items()):
        prob = F.Problem(x1, y1, x2, y2, E=E, nu=nu, precision=prec, p=12, leaf=32, m2l=m2l, m2l_tol=1e-10)
        try:
            out[name] = prob.apply(prob.vec(D)).cpu().numpy()[2 * na:]
        finally:
            prob.close()
    e64 = rel(out["fp64"], exact)
    assert e64 <= 1e-6, e64
    for name in PRECS:
        e_fmm, e_ex = rel(out[name], out["fp64"]), rel(out[name], exact)
        print(f"far field alone, m2l={m2l} {name}: vs FP64 FMM {e_fmm:.2e}, vs exact (oracle) {e_ex:.2e}")
        assert e_fmm <= FAR_BAR[name], (name, e_fmm)
        assert e_ex <= FAR_BAR[name] + e64, (name, e_ex)


def test_fp32_near_field_alone():
    """One leaf holds every element: the product is the near field alone, so
    the FP32 P2P is compared with the oracle's exact product directly."""
    wl = W.random_fractures(5, n_frac=6, elems=20, box=10.0)
    g = O.Geometry.of(wl)
    D = W.random_vector(6, g.n)
    exact = O.direct_matvec(g, D)
    for name, prec in PRECS.items():
        y, info = product(wl, prec, D, p=8, leaf=256)
        assert info["nV"] == 0 and info["nleaf"] == 1
        e = rel(y, exact)
        print(f"near field only, {name}: {e:.2e}")
        assert e <= NEAR_BAR, (name, e)


def test_mixed_precision_solve():
    wl = W.random_fractures(22, n_frac=20, elems=100)
    g = O.Geometry.of(wl)
    b = O.rhs(g, wl.pressure, wl.SH, wl.Sh)
    x_lu = O.lu_solve(O.dense_matrix(g), b)
    kw = dict(p=12, leaf=32, m2l=F.FMDDM_M2L_SVD, m2l_tol=1e-10, restart=50, maxit=5000)
    ref = F.Problem(wl.x1, wl.y1, wl.x2, wl.y2, E=wl.E, nu=wl.nu, **kw)   # FP64 products
    bd = ref.vec(b)
    sols = {}
    try:
        for name, prec, tol in [("fp64", F.FMDDM_PREC_FP64, 1e-10), ("fp32", F.FMDDM_PREC_FP32, 1e-8),
                                ("bf16", F.FMDDM_PREC_BF16, 1e-8)]:
            prob = F.Problem(wl.x1, wl.y1, wl.x2, wl.y2, E=wl.E, nu=wl.nu, precision=prec, tol=tol, **kw)
            try:
                x, info = prob.solve(bd)
            finally:
                prob.close()
            # the FP64 FMM residual of the returned solution, recomputed
            rr = float(torch.linalg.norm(bd - ref.apply(x)) / torch.linalg.norm(bd))
            assert info["status"] == F.FMDDM_OK and info["converged"], (name, info)
            assert info["relres"] <= tol and rr <= 1.01 * tol, (name, info, rr)
            if prec != F.FMDDM_PREC_FP64:
                assert info["refinements"] >= 2, info
            sols[name] = x.cpu().numpy()
            e_lu = float(np.linalg.norm(sols[name] - x_lu) / np.linalg.norm(x_lu))
            print(f"{name}: {info}, FP64 FMM residual {rr:.2e}, vs oracle LU {e_lu:.2e}")
            assert e_lu <= 1e-6, (name, e_lu)
    finally:
        ref.close()
    for name in ("fp32", "bf16"):
        e = float(np.linalg.norm(sols[name] - sols["fp64"]) / np.linalg.norm(sols["fp64"]))
        print(f"{name} vs FP64 solve: {e:.2e}")
        assert e <= 1e-7, (name, e)


def test_precision_errors():
    wl = W.random_fractures(5, n_frac=4, elems=10, box=10.0)
    with pytest.raises(F.FmddmError):
        F.fmddm_create(F.fmddm_default_params(precision=3))
    prob = F.Problem(wl.x1, wl.y1, wl.x2, wl.y2, precision=F.FMDDM_PREC_FP32)
    try:
        with pytest.raises(F.FmddmError):
            F.fmddm_poro_set(prob.ctx, 0.35, 0.8, 1e-18, 1e-3, 60.0)
    finally:
        prob.close()


def test_autotune_picks_fastest_accurate_configuration():
    wl = W.random_fractures(23, n_frac=30, elems=100)
    base = F.fmddm_default_params(E=wl.E, nu=wl.nu, m2l=F.FMDDM_M2L_SVD, m2l_tol=1e-10)
    st, best, log = F.fmddm_autotune(base, wl.x1, wl.y1, wl.x2, wl.y2, leaves=(16, 32, 64), ps=(10, 4, 6, 8),
                                     target_err=1e-6, reps=3)
    print("autotune", st, best.leaf, best.p, best.m2l_tiles, log)
    assert st == F.FMDDM_OK
    # the last four entries time the M2L tile sets on the chosen configuration
    tiles, log = log[-4:], log[:-4]
    assert [e["m2l_tiles"] for e in tiles] == [0, 1, 2, 3]
    assert all((e["leaf"], e["p"]) == (best.leaf, best.p) and e["ms"] > 0 for e in tiles)
    assert best.m2l_tiles == min(tiles, key=lambda e: e["ms"])["m2l_tiles"]
    timed = [e for e in log if e["ms"] > 0]
    assert timed and all(e["err"] <= 1e-6 for e in timed)
    assert all(e["err"] > 1e-6 for e in log if e["ms"] < 0)
    fastest = min(timed, key=lambda e: e["ms"])
    assert (best.leaf, best.p) == (fastest["leaf"], fastest["p"])
    # per leaf, p ascends and stops at the first that meets the target
    for lf in (16, 32, 64):
        ps = [e["p"] for e in log if e["leaf"] == lf]
        assert ps == sorted(ps) and ps[0] == 4
        assert [e["ms"] > 0 for e in log if e["leaf"] == lf] == [False] * (len(ps) - 1) + [True]
    # the rest of the parameters are kept
    assert best.m2l == F.FMDDM_M2L_SVD and best.m2l_tol == 1e-10 and best.E == wl.E
    # an unreachable target: ENOTCONV with the most accurate configuration
    st2, best2, log2 = F.fmddm_autotune(base, wl.x1, wl.y1, wl.x2, wl.y2, leaves=(32,), ps=(4, 6),
                                        target_err=1e-30, reps=1)
    assert st2 == F.FMDDM_ENOTCONV and len(log2) == 2   # no tile stage without a configuration
    assert best2.p == min(log2, key=lambda e: e["err"])["p"]


@pytest.mark.parametrize("leaf,p", [(64, 10), (32, 8)])
def test_full_size_sampled_rows(leaf, p):
    """N = 200000 (2000 random fractures x 100 elements, seed 4), the
    configurations of the mixed-precision benchmark: each precision's
    product against the oracle's exact product on 400 sampled outputs."""
    wl = W.c4()
    g = O.Geometry.of(wl)
    D = W.random_vector(9, g.n)
    rows = np.random.default_rng(1).choice(g.n, 400, replace=False)
    exact = O.direct_matvec_rows(g, D, rows).reshape(-1)
    idx = np.stack([2 * rows, 2 * rows + 1], 1).reshape(-1)
    ys = {}
    for name, prec in [("fp64", F.FMDDM_PREC_FP64)] + list(PRECS.items()):
        prob = F.Problem(wl.x1, wl.y1, wl.x2, wl.y2, E=wl.E, nu=wl.nu, precision=prec, p=p, leaf=leaf,
                         m2l=F.FMDDM_M2L_SVD, m2l_tol=1e-10)
        try:
            ys[name] = prob.apply(prob.vec(D)).cpu().numpy()[idx]
        finally:
            prob.close()
    e64 = rel(ys["fp64"], exact)
    print(f"N=200000 leaf={leaf} p={p}: fp64 vs oracle {e64:.2e}")
    assert e64 <= 1e-6, e64
    for name in PRECS:
        e = rel(ys[name], exact)
        print(f"  {name} vs oracle {e:.2e}, vs FP64 FMM {rel(ys[name], ys['fp64']):.2e}")
        assert e <= NEAR_BAR + (FAR_BAR[name] if name == "bf16" else 0.0) + e64, (name, e)


@pytest.mark.parametrize("m2l", [F.FMDDM_M2L_SVD, F.FMDDM_M2L_DENSE])
def test_m2l_tile_sets_agree(m2l):
    """The M2L tile sets change split-K depth and tile heights, i.e. only the
    order of the sums: every set gives the product of set 0 to rounding (set 0
    is the one the oracle parity tests cover), in FP64 and FP32."""
    wl = W.random_fractures(24, n_frac=40, elems=50)
    D = W.random_vector(4, wl.n)
    for prec, bar in [(F.FMDDM_PREC_FP64, 1e-13), (F.FMDDM_PREC_FP32, 1e-6)]:
        ys = [product(wl, prec, D, p=12, leaf=32, m2l=m2l, m2l_tol=1e-10, m2l_tiles=ts)[0] for ts in range(4)]
        for ts in range(1, 4):
            e = rel(ys[ts], ys[0])
            assert e <= bar, (prec, ts, e)
