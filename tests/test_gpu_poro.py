"""GPU parity of the poroelastic path (Section 2, eqs. 2.1-2.5) against the
oracle, through the C ABI.

Both sides evaluate the same element integrals by their own quadrature,
each converged to about 1e-12 relative (pinned for the oracle in
test_oracle_poro), so products agree to 1e-10 of the largest entry of each
response kind (tractions, pressure).  Time marching over several steps with
GMRES at tolerance 1e-12 agrees with the oracle's Gaussian elimination to
1e-8 relative.
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

MED = dict(E=20e9, nu=0.2, nuu=0.35, alpha=0.8, perm=1e-18, visc=1e-3)
DT = 60.0
P0 = 48.26e6


def make(wl, **kw):
    prob = F.Problem(wl.x1, wl.y1, wl.x2, wl.y2, E=MED["E"], nu=MED["nu"], **kw)
    F.fmddm_poro_set(prob.ctx, MED["nuu"], MED["alpha"], MED["perm"], MED["visc"], DT, P0)
    return prob


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def cmp(gpu, ref):
    """max error per response kind, relative to that kind's largest entry"""
    out = []
    for k in range(3):
        r = ref[k::3]
        out.append(float(np.abs(gpu[k::3] - r).max() / max(np.abs(r).max(), 1e-300)))
    return max(out)


def geometries():
    wl1 = W.well_cluster(n_frac=3, elems=20, half_length=2.0, spacing=1.0)
    wl2 = W.random_fractures(41, n_frac=6, elems=9, box=6.0, lmin=0.5, lmax=2.0)
    return [wl1, wl2]


def test_poro_apply_matches_oracle():
    po = O.Poro(**MED)
    for wl in geometries():
        prob = make(wl)
        g = O.Geometry.of(wl)
        rng = np.random.default_rng(7)
        D = rng.standard_normal(3 * g.n) * np.tile([1e-3, 1e-3, 1e-9], g.n)
        Dd = dev(D)
        for lag in (0, 1, 4):
            out = torch.zeros(3 * g.n, dtype=torch.float64, device="cuda")
            F.fmddm_poro_apply(prob.ctx, prob.tree, lag, Dd, out)
            ref = O.poro_matrix(g, po, DT, lag) @ D
            e = cmp(out.cpu().numpy(), ref)
            assert e <= 1e-10, (wl.name, lag, e)
        prob.close()


def test_history_matches_oracle():
    po = O.Poro(**MED)
    wl = geometries()[1]
    g = O.Geometry.of(wl)
    prob = make(wl)
    rng = np.random.default_rng(11)
    h = 6
    Dh = [rng.standard_normal(3 * g.n) * np.tile([1e-3, 1e-3, 1e-9], g.n) for _ in range(h - 1)]
    b = rng.standard_normal(3 * g.n) * 1e6
    rhs = dev(b)
    F.fmddm_add_history(prob.ctx, prob.tree, h, dev(np.concatenate(Dh)), rhs)
    ref = b.copy()
    for k in range(1, h):
        ref -= O.poro_matrix(g, po, DT, h - k) @ Dh[k - 1]
    got = rhs.cpu().numpy()
    e = cmp(got - b, ref - b)
    assert e <= 1e-10, e
    # h = 1 leaves the right-hand side unchanged
    r1 = dev(b)
    F.fmddm_add_history(prob.ctx, prob.tree, 1, None, r1)
    assert np.array_equal(r1.cpu().numpy(), b)
    prob.close()


def test_time_marching_matches_oracle():
    po = O.Poro(**MED)
    wl = W.well_cluster(n_frac=3, elems=12, half_length=2.0, spacing=1.0)
    g = O.Geometry.of(wl)
    steps = 5
    ref, _, _ = O.poro_march(g, po, DT, steps, wl.pressure, P0, wl.SH, wl.Sh)
    prob = make(wl, tol=1e-12, restart=60)
    n3 = 3 * g.n
    b0 = torch.zeros(n3, dtype=torch.float64, device="cuda")
    F.fmddm_poro_rhs(prob.ctx, prob.tree, dev(wl.pressure), wl.SH, wl.Sh, b0)
    assert cmp(b0.cpu().numpy(), O.poro_rhs(g, wl.pressure, P0, wl.SH, wl.Sh)) <= 1e-14
    hist = torch.zeros(steps * n3, dtype=torch.float64, device="cuda")
    D = torch.zeros(n3, dtype=torch.float64, device="cuda")
    for h in range(1, steps + 1):
        rhs = b0.clone()
        F.fmddm_add_history(prob.ctx, prob.tree, h, hist[: (h - 1) * n3] if h > 1 else None, rhs)
        st, info = F.fmddm_poro_solve(prob.ctx, prob.tree, rhs, D)
        assert st == F.FMDDM_OK and info["converged"], info
        hist[(h - 1) * n3: h * n3] = D
        e = float(np.linalg.norm(D.cpu().numpy() - ref[h - 1]) / np.linalg.norm(ref[h - 1]))
        assert e <= 1e-8, (h, e)
    # the symmetric stack: no shear DD on the middle fracture
    Dm = D.cpu().numpy().reshape(-1, 3)
    assert np.abs(Dm[12:24, 0]).max() <= 1e-8 * np.abs(Dm[:, 1]).max()
    prob.close()


def test_poro_errors():
    wl = geometries()[0]
    prob = F.Problem(wl.x1, wl.y1, wl.x2, wl.y2, E=MED["E"], nu=MED["nu"])
    n3 = 3 * prob.n
    D = torch.zeros(n3, dtype=torch.float64, device="cuda")
    out = torch.zeros(n3, dtype=torch.float64, device="cuda")
    with pytest.raises(F.FmddmError):
        F.fmddm_poro_apply(prob.ctx, prob.tree, 0, D, out)   # medium not set
    with pytest.raises(F.FmddmError):
        F.fmddm_poro_set(prob.ctx, 0.1, 0.8, 1e-18, 1e-3, 60.0)   # nu_u < nu
    F.fmddm_poro_set(prob.ctx, 0.35, 0.8, 1e-18, 1e-3, 60.0)
    with pytest.raises(F.FmddmError):
        F.fmddm_poro_apply(prob.ctx, prob.tree, 0, D, D)     # aliasing
    prob.close()


def test_poro_fmm_matches_exact():
    """The multipole form (Chebyshev p = 12, the transient kernel's M2L per
    level and time level) against the exact products on a well cluster whose
    cells (metres) are far wider than the diffusion lengths (< 0.2 m): the
    far field is then a smooth function on well-separated cells and p = 12
    interpolates it to ~1e-8; the bar is 1e-6 of the largest entry of each
    response kind."""
    wl = W.well_cluster(n_frac=5, elems=200, half_length=20.0, spacing=10.0)
    n3 = 3 * wl.n
    rng = np.random.default_rng(5)
    scale = np.tile([1e-4, 1e-4, 1e-10], wl.n)
    D = dev(rng.standard_normal(n3) * scale)
    hist = dev(np.concatenate([rng.standard_normal(n3) * scale for _ in range(5)]))
    res = {}
    for mode in (F.FMDDM_APPLY_DIRECT, F.FMDDM_APPLY_FMM):
        prob = F.Problem(wl.x1, wl.y1, wl.x2, wl.y2, E=MED["E"], nu=MED["nu"], p=12, leaf=32)
        F.fmddm_poro_set(prob.ctx, MED["nuu"], MED["alpha"], MED["perm"], MED["visc"], DT, P0, mode=mode)
        outs = []
        for lag in (0, 2):
            o = torch.zeros(n3, dtype=torch.float64, device="cuda")
            F.fmddm_poro_apply(prob.ctx, prob.tree, lag, D, o)
            outs.append(o.cpu().numpy())
        r = torch.zeros(n3, dtype=torch.float64, device="cuda")
        F.fmddm_add_history(prob.ctx, prob.tree, 6, hist, r)
        outs.append(r.cpu().numpy())
        res[mode] = outs
        info = F.fmddm_tree_get_info(prob.ctx, prob.tree)
        prob.close()
    assert info["nV"] > 0
    for k, (a, b) in enumerate(zip(res[F.FMDDM_APPLY_FMM], res[F.FMDDM_APPLY_DIRECT])):
        e = cmp(a, b)
        print("poro fmm vs exact", k, e)
        assert e <= 1e-6, (k, e)


def test_poro_fmm_time_marching():
    """Three time steps solved with GMRES on the multipole operator (and its
    history) agree with the same steps on the exact operator: both solve
    to 1e-11, and the operators differ by ~1e-9, so the DDs agree to 1e-6."""
    wl = W.well_cluster(n_frac=5, elems=160, half_length=16.0, spacing=10.0)
    n3 = 3 * wl.n
    sols = {}
    for mode in (F.FMDDM_APPLY_DIRECT, F.FMDDM_APPLY_FMM):
        prob = F.Problem(wl.x1, wl.y1, wl.x2, wl.y2, E=MED["E"], nu=MED["nu"], p=12, leaf=32, tol=1e-11,
                         restart=80)
        F.fmddm_poro_set(prob.ctx, MED["nuu"], MED["alpha"], MED["perm"], MED["visc"], DT, P0, mode=mode)
        b0 = torch.zeros(n3, dtype=torch.float64, device="cuda")
        F.fmddm_poro_rhs(prob.ctx, prob.tree, dev(wl.pressure), wl.SH, wl.Sh, b0)
        hist = torch.zeros(3 * n3, dtype=torch.float64, device="cuda")
        D = torch.zeros(n3, dtype=torch.float64, device="cuda")
        for h in range(1, 4):
            rhs = b0.clone()
            F.fmddm_add_history(prob.ctx, prob.tree, h, hist[: (h - 1) * n3] if h > 1 else None, rhs)
            st, info = F.fmddm_poro_solve(prob.ctx, prob.tree, rhs, D)
            assert st == F.FMDDM_OK, info
            hist[(h - 1) * n3: h * n3] = D
        sols[mode] = hist.cpu().numpy().reshape(3, -1)
        prob.close()
    for h in range(3):
        a, b = sols[F.FMDDM_APPLY_FMM][h], sols[F.FMDDM_APPLY_DIRECT][h]
        e = cmp(a, b)
        print("poro fmm marching step", h + 1, e)
        assert e <= 1e-6, (h, e)


@pytest.mark.parametrize("mode", [F.FMDDM_APPLY_DIRECT, F.FMDDM_APPLY_FMM])
def test_poro_block_jacobi(mode):
    """Block-Jacobi preconditioning of the poroelastic left-hand side (groups
    of at most 21 elements, 3 unknowns each), alone and with the coarse
    level (undrained long elements over aggregates): same solution as plain
    GMRES (all to 1e-11), in at most half the products."""
    wl = W.well_cluster(n_frac=3, elems=60, half_length=6.0, spacing=2.0)
    n3 = 3 * wl.n
    res = {}
    for pc in (F.FMDDM_PRECOND_NONE, F.FMDDM_PRECOND_BLOCK, F.FMDDM_PRECOND_TWO_LEVEL):
        prob = F.Problem(wl.x1, wl.y1, wl.x2, wl.y2, E=MED["E"], nu=MED["nu"], p=8, leaf=16, tol=1e-11,
                         restart=50, maxit=20000, precond=pc)
        F.fmddm_poro_set(prob.ctx, MED["nuu"], MED["alpha"], MED["perm"], MED["visc"], DT, P0, mode=mode)
        b0 = torch.zeros(n3, dtype=torch.float64, device="cuda")
        F.fmddm_poro_rhs(prob.ctx, prob.tree, dev(wl.pressure), wl.SH, wl.Sh, b0)
        hist = torch.zeros(2 * n3, dtype=torch.float64, device="cuda")
        D = torch.zeros(n3, dtype=torch.float64, device="cuda")
        its = []
        for h in (1, 2):
            rhs = b0.clone()
            F.fmddm_add_history(prob.ctx, prob.tree, h, hist[:n3] if h > 1 else None, rhs)
            st, info = F.fmddm_poro_solve(prob.ctx, prob.tree, rhs, D)
            assert st == F.FMDDM_OK and info["converged"], (pc, h, info)
            hist[(h - 1) * n3: h * n3] = D
            its.append(info["iters"])
        res[pc] = (hist.cpu().numpy(), its)
        print(f"mode {mode} precond {pc}: iterations {its}")
        prob.close()
    for h in range(2):
        b = res[F.FMDDM_PRECOND_NONE][0][h * n3:(h + 1) * n3]
        for pc in (F.FMDDM_PRECOND_BLOCK, F.FMDDM_PRECOND_TWO_LEVEL):
            a = res[pc][0][h * n3:(h + 1) * n3]
            assert cmp(a, b) <= 1e-7, (pc, h, cmp(a, b))
            assert 2 * res[pc][1][h] <= res[F.FMDDM_PRECOND_NONE][1][h], res


@pytest.mark.parametrize("p,m2l,nrow", [(10, 0, 20), (16, 1, 40)])
def test_poro_full_size_sampled_rows(p, m2l, nrow):
    """N = 20000 (five fractures of 4000 0.2 m elements, 10 m apart) in the
    serving configuration (p = 10, leaf 32) and the march's (p = 16, the
    left-hand side's M2L compressed per cell size; the 4-level history's
    far field in two terms): the left-hand-side product and the history
    sum against the oracle's exact rows for 20 / 40 sampled receivers; bar
    1e-6 of the largest entry of each response kind, as for the smaller
    multipole test."""
    wl = W.well_cluster(n_frac=5, elems=4000, half_length=400.0, spacing=10.0)
    g = O.Geometry.of(wl)
    po = O.Poro(**MED)
    rows = np.random.default_rng(2).choice(g.n, nrow, replace=False)
    idx = np.stack([3 * rows, 3 * rows + 1, 3 * rows + 2], 1).reshape(-1)
    rng = np.random.default_rng(5)
    scale = np.tile([1e-4, 1e-4, 1e-10], g.n)
    D = rng.standard_normal(3 * g.n) * scale
    h = 4
    Dh = [rng.standard_normal(3 * g.n) * scale for _ in range(h - 1)]
    b = rng.standard_normal(3 * g.n) * 1e6
    prob = F.Problem(wl.x1, wl.y1, wl.x2, wl.y2, E=MED["E"], nu=MED["nu"], p=p, leaf=32, m2l_tol=1e-10)
    try:
        F.fmddm_poro_set(prob.ctx, MED["nuu"], MED["alpha"], MED["perm"], MED["visc"], DT, P0,
                         mode=F.FMDDM_APPLY_FMM, m2l=m2l)
        out = torch.zeros(3 * g.n, dtype=torch.float64, device="cuda")
        F.fmddm_poro_apply(prob.ctx, prob.tree, 0, dev(D), out)
        rhs = dev(b)
        F.fmddm_add_history(prob.ctx, prob.tree, h, dev(np.concatenate(Dh)), rhs)
        y0 = out.cpu().numpy()[idx]
        yh = rhs.cpu().numpy()[idx]
        assert (F.fmddm_tree_get_info(prob.ctx, prob.tree)["poro_m2l_rank"] > 0) == (m2l == 1)
    finally:
        prob.close()
    ref0 = O.poro_matrix_rows(g, po, DT, 0, rows) @ D
    refh = b[idx].copy()
    for k in range(1, h):
        refh -= O.poro_matrix_rows(g, po, DT, h - k, rows) @ Dh[k - 1]
    e0, eh = cmp(y0, ref0), cmp(yh - b[idx], refh - b[idx])
    print(f"N=20000 poro FMM (p = {p}, m2l {m2l}) vs oracle rows: lhs {e0:.2e}, history {eh:.2e}")
    assert e0 <= 1e-6 and eh <= 1e-6, (e0, eh)


def test_poro_near_cache():
    """The resident near-field blocks (each time level integrated once, then
    block-sparse products) against on-the-fly integration at every product:
    the same element integrals summed in another order, so the products
    agree to 1e-12 of the largest entry of each response kind.  Budgets: no
    cache, two levels (the lag-4 product and the 6-level history mix stored
    and integrated levels) and the default.  A second call on the stored
    blocks repeats the first bit for bit, and a new medium (another Biot
    coefficient) rebuilds both the blocks and the multipole operators."""
    wl = W.well_cluster(n_frac=5, elems=200, half_length=20.0, spacing=10.0)
    n3 = 3 * wl.n
    rng = np.random.default_rng(11)
    scale = np.tile([1e-4, 1e-4, 1e-10], wl.n)
    D = dev(rng.standard_normal(n3) * scale)
    hist = dev(np.concatenate([rng.standard_normal(n3) * scale for _ in range(5)]))

    def products(prob):
        outs = []
        for lag in (0, 2, 4):
            o = torch.zeros(n3, dtype=torch.float64, device="cuda")
            F.fmddm_poro_apply(prob.ctx, prob.tree, lag, D, o)
            outs.append(o.cpu().numpy())
        r = torch.zeros(n3, dtype=torch.float64, device="cuda")
        F.fmddm_add_history(prob.ctx, prob.tree, 6, hist, r)
        outs.append(r.cpu().numpy())
        return outs

    def problem(budget, alpha=MED["alpha"]):
        prob = F.Problem(wl.x1, wl.y1, wl.x2, wl.y2, E=MED["E"], nu=MED["nu"], p=12, leaf=32)
        F.fmddm_poro_set(prob.ctx, MED["nuu"], alpha, MED["perm"], MED["visc"], DT, P0,
                         mode=F.FMDDM_APPLY_FMM, near_cache_bytes=budget)
        return prob

    prob = problem(-1)
    ref = products(prob)
    pairs = F.fmddm_tree_get_info(prob.ctx, prob.tree)["near_pairs"]
    prob.close()
    assert pairs > 0
    for budget in (2 * 96 * pairs, 0):
        prob = problem(budget)
        try:
            first = products(prob)
            again = products(prob)
            for k, (a, b) in enumerate(zip(first, ref)):
                e = cmp(a, b)
                print(f"near cache budget {budget}: product {k} vs on the fly {e:.2e}")
                assert e <= 1e-12, (budget, k, e)
            for a, b in zip(again, first):
                assert np.array_equal(a, b)
            if budget == 0:
                F.fmddm_poro_set(prob.ctx, MED["nuu"], 0.6, MED["perm"], MED["visc"], DT, P0,
                                 mode=F.FMDDM_APPLY_FMM)
                changed = products(prob)
        finally:
            prob.close()
    prob = problem(-1, alpha=0.6)
    ref2 = products(prob)
    prob.close()
    for k, (a, b) in enumerate(zip(changed, ref2)):
        e = cmp(a, b)
        print(f"new medium: product {k} vs on the fly {e:.2e}")
        assert e <= 1e-12, (k, e)


def test_poro_full_size_smooth_dds():
    """N = 20000 well cluster, left-hand-side product of a smooth,
    solution-like set of DDs (elliptic openings, antisymmetric shear) against
    the oracle's exact rows for 29 receivers.  Smooth DDs weigh the far
    field, where the interpolation error of the transient kernel lives:
    measured 1.1e-5 at p = 10, 1.1e-6 at p = 12 and 7.3e-9 at p = 16 (the
    order the full march uses), which the bars follow with some margin."""
    wl = W.well_cluster(n_frac=5, elems=4000, half_length=400.0, spacing=10.0)
    g = O.Geometry.of(wl)
    po = O.Poro(**MED)
    xm = 0.5 * (wl.x1 + wl.x2)
    ell = np.sqrt(np.maximum(1 - (xm / 400.0) ** 2, 0))
    D = np.zeros((g.n, 3))
    D[:, 0] = 1e-4 * (xm / 400.0) * ell * np.sign(0.5 * (wl.y1 + wl.y2) + 1e-9)
    D[:, 1] = 1e-3 * ell
    D[:, 2] = 1e-9 * ell
    D = D.reshape(-1)
    rows = np.concatenate([np.random.default_rng(2).choice(g.n, 24, replace=False), [10, 2000, 8000, 10000, 12000]])
    idx = np.stack([3 * rows, 3 * rows + 1, 3 * rows + 2], 1).reshape(-1)
    ref = O.poro_matrix_rows(g, po, DT, 0, rows) @ D
    for p, bar in ((10, 5e-5), (16, 1e-7)):
        prob = F.Problem(wl.x1, wl.y1, wl.x2, wl.y2, E=MED["E"], nu=MED["nu"], p=p, leaf=32)
        try:
            F.fmddm_poro_set(prob.ctx, MED["nuu"], MED["alpha"], MED["perm"], MED["visc"], DT, P0,
                             mode=F.FMDDM_APPLY_FMM)
            out = torch.zeros(3 * g.n, dtype=torch.float64, device="cuda")
            F.fmddm_poro_apply(prob.ctx, prob.tree, 0, dev(D), out)
            y = out.cpu().numpy()[idx]
        finally:
            prob.close()
        e = cmp(y, ref)
        print(f"N=20000 smooth DDs, p = {p}: {e:.2e}")
        assert e <= bar, (p, e)


def test_poro_history_only_variant():
    """FMDDM_APPLY_DENSE, the history-only variant: the left-hand side as a
    stored dense matrix of exact element integrals (agrees with the exact
    on-the-fly product and the oracle), the history sum through the FMM
    (bitwise the FMM mode's), and a 3-step march against the oracle's."""
    # 3 n odd: the dense product's rows are not 16-byte aligned
    wl = W.well_cluster(n_frac=3, elems=41, half_length=4.0, spacing=1.0)
    g = O.Geometry.of(wl)
    po = O.Poro(**MED)
    n3 = 3 * g.n
    assert n3 % 2 == 1
    rng = np.random.default_rng(7)
    scale = np.tile([1e-4, 1e-4, 1e-10], g.n)
    D = rng.standard_normal(n3) * scale
    hist = np.concatenate([rng.standard_normal(n3) * scale for _ in range(3)])
    res = {}
    for mode in (F.FMDDM_APPLY_DIRECT, F.FMDDM_APPLY_FMM, F.FMDDM_APPLY_DENSE):
        prob = F.Problem(wl.x1, wl.y1, wl.x2, wl.y2, E=MED["E"], nu=MED["nu"], p=12, leaf=16, tol=1e-12,
                         restart=80)
        try:
            F.fmddm_poro_set(prob.ctx, MED["nuu"], MED["alpha"], MED["perm"], MED["visc"], DT, P0, mode=mode)
            out = torch.zeros(n3, dtype=torch.float64, device="cuda")
            F.fmddm_poro_apply(prob.ctx, prob.tree, 0, dev(D), out)
            rhs = torch.zeros(n3, dtype=torch.float64, device="cuda")
            F.fmddm_add_history(prob.ctx, prob.tree, 4, dev(hist), rhs)
            res[mode] = (out.cpu().numpy(), rhs.cpu().numpy())
            if mode == F.FMDDM_APPLY_DENSE:
                b0 = torch.zeros(n3, dtype=torch.float64, device="cuda")
                F.fmddm_poro_rhs(prob.ctx, prob.tree, dev(wl.pressure), wl.SH, wl.Sh, b0)
                Dh = torch.zeros(3 * n3, dtype=torch.float64, device="cuda")
                x = torch.zeros(n3, dtype=torch.float64, device="cuda")
                marched = []
                for h in range(1, 4):
                    r = b0.clone()
                    F.fmddm_add_history(prob.ctx, prob.tree, h, Dh[: (h - 1) * n3] if h > 1 else None, r)
                    st, info = F.fmddm_poro_solve(prob.ctx, prob.tree, r, x)
                    assert st == F.FMDDM_OK, info
                    Dh[(h - 1) * n3: h * n3] = x
                    marched.append(x.cpu().numpy().copy())
        finally:
            prob.close()
    assert cmp(res[F.FMDDM_APPLY_DENSE][0], res[F.FMDDM_APPLY_DIRECT][0]) <= 1e-10
    assert cmp(res[F.FMDDM_APPLY_DENSE][0], O.poro_matrix(g, po, DT, 0) @ D) <= 1e-10
    assert np.array_equal(res[F.FMDDM_APPLY_DENSE][1], res[F.FMDDM_APPLY_FMM][1])
    ref, _, _ = O.poro_march(g, po, DT, 3, wl.pressure, P0, wl.SH, wl.Sh)
    for h in range(3):
        e = float(np.linalg.norm(marched[h] - ref[h]) / np.linalg.norm(ref[h]))
        print(f"history-only march step {h + 1}: {e:.2e}")
        assert e <= 1e-6, (h, e)


@pytest.mark.parametrize("p", [10, 16])
def test_poro_lhs_compressed_m2l(p):
    """The left-hand side's M2L compressed per cell size (poro m2l = SVD,
    m2l_tol 1e-12) against the uncompressed operators and the exact
    products, on a 5 x 200-element well cluster (four V-list levels).  The
    truncation drops singular values below 1e-12 of the largest, and the
    compressed product sums 27 translations of projected weights, so it
    stays within ~1e-10 of the uncompressed one (bar 1e-9); against the
    exact product the uncompressed bar holds (1e-6).  Not bitwise equal to
    the uncompressed product, so the compressed path ran."""
    wl = W.well_cluster(n_frac=5, elems=200, half_length=20.0, spacing=10.0)
    n3 = 3 * wl.n
    rng = np.random.default_rng(6)
    scale = np.tile([1e-4, 1e-4, 1e-10], wl.n)
    D = dev(rng.standard_normal(n3) * scale)
    res = {}
    for mode, m2l in ((F.FMDDM_APPLY_DIRECT, 0), (F.FMDDM_APPLY_FMM, 0), (F.FMDDM_APPLY_FMM, 1)):
        prob = F.Problem(wl.x1, wl.y1, wl.x2, wl.y2, E=MED["E"], nu=MED["nu"], p=p, leaf=32, m2l_tol=1e-12)
        try:
            F.fmddm_poro_set(prob.ctx, MED["nuu"], MED["alpha"], MED["perm"], MED["visc"], DT, P0, mode=mode,
                             m2l=m2l)
            o = torch.zeros(n3, dtype=torch.float64, device="cuda")
            F.fmddm_poro_apply(prob.ctx, prob.tree, 0, D, o)
            o2 = torch.zeros(n3, dtype=torch.float64, device="cuda")
            F.fmddm_poro_apply(prob.ctx, prob.tree, 0, D, o2)  # the stored compressed operators
            assert torch.equal(o, o2)
            res[(mode, m2l)] = o.cpu().numpy()
            info = F.fmddm_tree_get_info(prob.ctx, prob.tree)
            if mode == F.FMDDM_APPLY_FMM:
                rank = info["poro_m2l_rank"]
                assert (rank > 0) == (m2l == 1), rank
                assert rank < 3 * 4 * p * p // 4
        finally:
            prob.close()
    assert info["nV"] > 0
    exact, dense, comp = res[(F.FMDDM_APPLY_DIRECT, 0)], res[(F.FMDDM_APPLY_FMM, 0)], res[(F.FMDDM_APPLY_FMM, 1)]
    e_cd, e_ce, e_de = cmp(comp, dense), cmp(comp, exact), cmp(dense, exact)
    print(f"p = {p}: rank {rank} of {4 * p * p}; compressed vs uncompressed {e_cd:.2e}, vs exact {e_ce:.2e} "
          f"(uncompressed vs exact {e_de:.2e})")
    assert not np.array_equal(comp, dense)
    assert e_cd <= 1e-9, e_cd
    assert e_ce <= 1e-6, e_ce


def test_poro_history_far_field_two_terms():
    """History sums and lag products with the far field in two multipole
    terms (the transient kernel affine in t outside the diffusion length)
    against one term per time level (exact_far_levels = 1) and the exact
    products, on the 5 x 200-element well cluster (cells of metres, a
    diffusion length below 0.2 m after 9 steps).  The two forms differ by
    e^-z terms with z >= 50 and by the rounding of the extrapolation
    F(dt) + (j - 1)(F(2 dt) - F(dt)), a few ulp times the number of levels:
    bar 1e-12 of each kind's largest entry.  With a permeability 1e5 times
    larger the check refuses the two-term form, and the results are bitwise
    the per-level ones."""
    wl = W.well_cluster(n_frac=5, elems=200, half_length=20.0, spacing=10.0)
    n3 = 3 * wl.n
    rng = np.random.default_rng(8)
    scale = np.tile([1e-4, 1e-4, 1e-10], wl.n)
    D = dev(rng.standard_normal(n3) * scale)
    hist = dev(np.concatenate([rng.standard_normal(n3) * scale for _ in range(8)]))
    for perm, affine in ((MED["perm"], True), (1e5 * MED["perm"], False)):
        res = {}
        for mode, exact in ((F.FMDDM_APPLY_DIRECT, 0), (F.FMDDM_APPLY_FMM, 0), (F.FMDDM_APPLY_FMM, 1)):
            prob = F.Problem(wl.x1, wl.y1, wl.x2, wl.y2, E=MED["E"], nu=MED["nu"], p=12, leaf=32)
            try:
                F.fmddm_poro_set(prob.ctx, MED["nuu"], MED["alpha"], perm, MED["visc"], DT, P0, mode=mode,
                                 exact_far_levels=exact)
                o = torch.zeros(n3, dtype=torch.float64, device="cuda")
                F.fmddm_poro_apply(prob.ctx, prob.tree, 6, D, o)
                r = torch.zeros(n3, dtype=torch.float64, device="cuda")
                F.fmddm_add_history(prob.ctx, prob.tree, 9, hist, r)
                res[(mode, exact)] = (o.cpu().numpy(), r.cpu().numpy())
            finally:
                prob.close()
        two, per, ex = res[(F.FMDDM_APPLY_FMM, 0)], res[(F.FMDDM_APPLY_FMM, 1)], res[(F.FMDDM_APPLY_DIRECT, 0)]
        for k, name in enumerate(("lag 6", "history of step 9")):
            e_tp, e_te, e_pe = cmp(two[k], per[k]), cmp(two[k], ex[k]), cmp(per[k], ex[k])
            print(f"perm {perm:g}, {name}: two-term vs per-level {e_tp:.2e}, vs exact {e_te:.2e} "
                  f"(per-level vs exact {e_pe:.2e})")
            assert e_te <= 1e-6, (name, e_te)
            if affine:
                assert e_tp <= 1e-12, (name, e_tp)
                assert not np.array_equal(two[k], per[k])
            else:
                assert np.array_equal(two[k], per[k])


@pytest.mark.parametrize("far_levels", [0, 1])
def test_poro_graph_replays_match_plain_launches(far_levels):
    """Poroelastic steps with captured GMRES steps (use_graphs = 1) equal the
    same steps launched plainly, bit for bit, in the same numbers of
    products: four steps with the history sum (with one far-field term per
    time level the history's operators grow with the step, reallocating
    buffers the left-hand side reads), then a new Biot coefficient (every
    operator and preconditioner block rebuilt) and two more steps.
    Two-level preconditioning, restart 10 (several cycles per solve), the
    left-hand side's M2L compressed."""
    wl = W.well_cluster(n_frac=3, elems=60, half_length=6.0, spacing=2.0)
    n3 = 3 * wl.n
    out = {}
    for graphs in (0, 1):
        prob = F.Problem(wl.x1, wl.y1, wl.x2, wl.y2, E=MED["E"], nu=MED["nu"], p=10, leaf=16, tol=1e-10,
                         restart=10, maxit=20000, precond=F.FMDDM_PRECOND_TWO_LEVEL, use_graphs=graphs)

        def medium(alpha):
            F.fmddm_poro_set(prob.ctx, MED["nuu"], alpha, MED["perm"], MED["visc"], DT, P0, mode=F.FMDDM_APPLY_FMM,
                             m2l=F.FMDDM_M2L_SVD, exact_far_levels=far_levels)
            b = torch.zeros(n3, dtype=torch.float64, device="cuda")
            F.fmddm_poro_rhs(prob.ctx, prob.tree, dev(wl.pressure), wl.SH, wl.Sh, b)
            return b

        b0 = medium(MED["alpha"])
        hist = torch.zeros(6 * n3, dtype=torch.float64, device="cuda")
        D = torch.zeros(n3, dtype=torch.float64, device="cuda")
        iters = []
        for h in range(1, 7):
            if h == 5:
                b0 = medium(0.6)
            rhs = b0.clone()
            F.fmddm_add_history(prob.ctx, prob.tree, h, hist[: (h - 1) * n3] if h > 1 else None, rhs)
            st, info = F.fmddm_poro_solve(prob.ctx, prob.tree, rhs, D)
            assert st == F.FMDDM_OK and info["converged"], info
            hist[(h - 1) * n3: h * n3] = D
            iters.append(info["iters"])
        out[graphs] = (hist.cpu().numpy(), iters)
        prob.close()
    print("products per step, plain / captured:", out[0][1], out[1][1])
    assert out[0][1] == out[1][1] and min(out[0][1]) > 10
    assert np.array_equal(out[0][0], out[1][0]), float(np.max(np.abs(out[0][0] - out[1][0])))
