"""Pins of the CPU oracle against facts that do not come from the oracle.

Every check here is anchored outside the oracle's own formulas: closed-form
crack solutions (Sneddon opening, K_I = p sqrt(pi a)), exact identities of
the constant element (self coefficient, splitting, rigid motions), limits
(element -> point kernel far away), textbook properties of Chebyshev and
Gauss-Legendre rules, brute-force definitions of the tree and lists, and an
FMM run with a polynomial kernel, for which the interpolation is exact and
the FMM must equal the dense product up to rounding.
"""
import json
import os

import numpy as np
import pytest

import oracle as O
import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")


@pytest.fixture(scope="module", autouse=True)
def _build():
    O.build(force=False)


def sneddon(x, a, p, E, nu):
    return 4.0 * (1.0 - nu ** 2) * p / E * np.sqrt(np.maximum(a * a - x * x, 0.0))


# ---------------------------------------------------------------- crack pins
@pytest.mark.parametrize("n", [200, 256])
def test_sneddon_opening_and_KI(n):
    """Pressurized Griffith crack: opening within 1% (rel. L2) of Sneddon's
    closed form, and K_I from the tip element by eq. 2.6 within 1% of
    p sqrt(pi a)."""
    wl = W.griffith(n)
    g = O.Geometry.of(wl)
    A = O.dense_matrix(g)
    b = O.rhs(g, wl.pressure, 0.0, 0.0)
    x = O.lu_solve(A, b)
    a, p = wl.meta["a"], wl.meta["p"]
    w = sneddon(g.cx, a, p, g.E, g.nu)
    err = np.linalg.norm(x[1::2] - w) / np.linalg.norm(w)
    assert err < 0.01, err
    assert np.abs(x[0::2]).max() < 1e-12 * np.abs(x[1::2]).max()
    gold = json.load(open(GOLD))["sif_eq_2_6"]["factor"]
    KI, KII = O.sif(g.E, g.nu, g.a[-1], x[-2], x[-1])
    KI_exact = p * np.sqrt(np.pi * a)
    assert abs(KI / KI_exact - 1.0) < 0.01
    assert abs(KII) < 1e-9 * KI
    # the factor in eq. 2.6 is the paper's
    f = gold * g.E / (4 * (1 - g.nu ** 2)) * np.sqrt(np.pi / (2 * g.a[-1]))
    assert KI == pytest.approx(f * x[-1], rel=1e-15)


def test_shear_crack_same_profile():
    """Uniform remote shear on a straight crack: the sliding profile is the
    Sneddon profile with tau in place of p."""
    wl = W.griffith(256)
    g = O.Geometry.of(wl)
    A = O.dense_matrix(g)
    tau = 5e6
    b = np.zeros(2 * g.n)
    b[0::2] = -tau
    x = O.lu_solve(A, b)
    w = sneddon(g.cx, 1.0, tau, g.E, g.nu)
    err = np.linalg.norm(x[0::2] - w) / np.linalg.norm(w)
    assert err < 0.01
    assert np.abs(x[1::2]).max() < 1e-12 * np.abs(x[0::2]).max()


@pytest.mark.parametrize("beta_deg", [0.0, 30.0, 75.0])
def test_inclined_crack_far_field(beta_deg):
    """Inclined crack under compressive far field plus internal pressure:
    opening follows Sneddon with the net pressure p - sigma_n(inf) and
    sliding follows Sneddon with the resolved shear stress.  Pins the
    right-hand side (far-field resolution, Section 4)."""
    n, a, pf, SH, Sh = 256, 1.0, 50e6, 40e6, 30e6
    be = np.deg2rad(beta_deg)
    t = np.linspace(-a, a, n + 1)
    x1, x2 = t[:-1] * np.cos(be), t[1:] * np.cos(be)
    y1, y2 = t[:-1] * np.sin(be), t[1:] * np.sin(be)
    g = O.Geometry(x1, y1, x2, y2, 20e9, 0.25)
    b = O.rhs(g, np.full(n, pf), SH, Sh)
    x = O.lu_solve(O.dense_matrix(g), b)
    s = np.linspace(-a, a, n + 1)
    mid = 0.5 * (s[1:] + s[:-1])
    sn_inf = SH * np.sin(be) ** 2 + Sh * np.cos(be) ** 2      # compression
    tau_inf = (SH - Sh) * np.sin(be) * np.cos(be)
    wn = sneddon(mid, a, pf - sn_inf, g.E, g.nu)
    assert np.linalg.norm(x[1::2] - wn) / np.linalg.norm(wn) < 0.01
    if beta_deg != 0.0:
        ws = sneddon(mid, a, tau_inf, g.E, g.nu)
        # positive resolved shear (upper material dragged along +s) makes
        # the + face slide along +s once the crack is cut: D_s > 0
        assert np.linalg.norm(x[0::2] - ws) / np.linalg.norm(ws) < 0.01


def test_self_coefficient_exact():
    """Element on itself: normal and shear self-coefficients equal
    -G / (pi (1 - nu) a), cross terms vanish (constant DD element)."""
    g = O.Geometry(np.array([-0.3]), np.array([0.1]), np.array([0.5]), np.array([0.7]),
                   20e9, 0.25)
    A = O.dense_matrix(g)
    ref = -g.G / (np.pi * (1 - g.nu) * g.a[0])
    assert A[0, 0] == pytest.approx(ref, rel=1e-13)
    assert A[1, 1] == pytest.approx(ref, rel=1e-13)
    assert abs(A[0, 1]) < 1e-12 * abs(ref)
    assert abs(A[1, 0]) < 1e-12 * abs(ref)


def test_rigid_motion_invariance():
    """Rotating and translating the whole geometry leaves the
    shear/normal influence matrix unchanged."""
    wl = W.random_fractures(11, 6, 8)
    g = O.Geometry.of(wl)
    A = O.dense_matrix(g)
    th = 0.7
    c, s = np.cos(th), np.sin(th)

    def rot(x, y):
        return c * x - s * y + 3.3, s * x + c * y - 1.2

    x1, y1 = rot(wl.x1, wl.y1)
    x2, y2 = rot(wl.x2, wl.y2)
    g2 = O.Geometry(x1, y1, x2, y2, wl.E, wl.nu)
    A2 = O.dense_matrix(g2)
    assert np.max(np.abs(A2 - A)) < 1e-9 * np.max(np.abs(A))


def test_element_split_identity():
    """An element equals the sum of its two halves carrying the same DD."""
    rng = np.random.default_rng(3)
    G, nu = 8e9, 0.25
    for _ in range(20):
        b = rng.uniform(0, np.pi)
        cb, sb = np.cos(b), np.sin(b)
        a = rng.uniform(0.01, 0.5)
        cx, cy = rng.uniform(-1, 1, 2)
        X, Y = rng.uniform(-2, 2, 2)
        Ds, Dn = rng.standard_normal(2)
        whole = O.elem_stress(X, Y, cx, cy, cb, sb, a, G, nu, Ds, Dn)
        h1 = O.elem_stress(X, Y, cx - 0.5 * a * cb, cy - 0.5 * a * sb, cb, sb, 0.5 * a, G, nu, Ds, Dn)
        h2 = O.elem_stress(X, Y, cx + 0.5 * a * cb, cy + 0.5 * a * sb, cb, sb, 0.5 * a, G, nu, Ds, Dn)
        assert np.allclose(h1 + h2, whole, rtol=1e-9, atol=1e-9 * np.abs(whole).max())


def test_point_kernel_is_far_field_limit():
    """Far from a short element, its stress divided by its length tends to
    the point kernel applied to the charge, with O((a/r)^2) error."""
    rng = np.random.default_rng(5)
    G, nu = 8e9, 0.25
    for _ in range(10):
        b = rng.uniform(0, np.pi)
        cb, sb = np.cos(b), np.sin(b)
        Ds, Dn = rng.standard_normal(2)
        ang = rng.uniform(0, 2 * np.pi)
        X, Y = np.cos(ang), np.sin(ang)
        K = O.point_kernel(X, Y, G, nu)
        q = O.charge(cb, sb, Ds, Dn)
        errs = []
        for a in (1e-2, 1e-3):
            s = O.elem_stress(X, Y, 0.0, 0.0, cb, sb, a, G, nu, Ds, Dn) / (2 * a)
            errs.append(np.abs(s - K @ q).max() / np.abs(K @ q).max())
        assert errs[1] < 2e-5
        assert errs[1] < errs[0] / 50.0     # quadratic decay


def test_point_kernel_rotation_covariance_and_homogeneity():
    """Rotating source orientation and offset together rotates the stress;
    the kernel is homogeneous of degree -2."""
    rng = np.random.default_rng(6)
    G, nu = 8e9, 0.25
    for _ in range(10):
        b, th = rng.uniform(0, 2 * np.pi, 2)
        Ds, Dn = rng.standard_normal(2)
        x, y = rng.standard_normal(2)
        s0 = O.point_kernel(x, y, G, nu) @ O.charge(np.cos(b), np.sin(b), Ds, Dn)
        c, s = np.cos(th), np.sin(th)
        R = np.array([[c, -s], [s, c]])
        xr, yr = R @ np.array([x, y])
        s1 = O.point_kernel(xr, yr, G, nu) @ O.charge(np.cos(b + th), np.sin(b + th), Ds, Dn)
        S0 = np.array([[s0[0], s0[2]], [s0[2], s0[1]]])
        S1 = R @ S0 @ R.T
        assert np.allclose([S1[0, 0], S1[1, 1], S1[0, 1]], s1, rtol=1e-10,
                           atol=1e-10 * np.abs(s1).max())
        s2 = O.point_kernel(3 * x, 3 * y, G, nu) @ O.charge(np.cos(b), np.sin(b), Ds, Dn)
        assert np.allclose(s2 * 9, s0, rtol=1e-12, atol=1e-12 * np.abs(s0).max())


# ------------------------------------------------------- quadrature / interp
@pytest.mark.parametrize("n", [1, 2, 5, 8, 20])
def test_gauss_legendre_exactness(n):
    t, w = O.gauss_legendre(n)
    for k in range(2 * n):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert np.dot(w, t ** k) == pytest.approx(exact, abs=1e-14)


@pytest.mark.parametrize("p", [3, 6, 12, 20])
def test_chebyshev_interpolant(p):
    """S_p(xbar_l, xbar_m) = delta_lm, sum_l S_p(xbar_l, x) = 1, and
    polynomials of degree < p are reproduced (inside and slightly outside
    [-1, 1])."""
    xb = O.cheb_nodes(p)
    assert np.allclose(np.sort(xb), np.sort(np.cos((2 * np.arange(1, p + 1) - 1) * np.pi / (2 * p))))
    S = np.array([[O.cheb_S(p, l, xb[m]) for m in range(p)] for l in range(p)])
    assert np.allclose(S, np.eye(p), atol=1e-13)
    rng = np.random.default_rng(p)
    coef = rng.standard_normal(p)
    for x in (-1.2, -0.3, 0.77, 1.1):
        Sx = np.array([O.cheb_S(p, l, x) for l in range(p)])
        # rounding is amplified outside [-1, 1] by the growth of T_{p-1}
        growth = np.cosh((p - 1) * np.arccosh(max(abs(x), 1.0)))
        assert Sx.sum() == pytest.approx(1.0, abs=1e-14 * p * growth)
        f = np.polynomial.polynomial.polyval(xb, coef)
        assert np.dot(Sx, f) == pytest.approx(np.polynomial.polynomial.polyval(x, coef),
                                              rel=1e-12 * growth, abs=1e-12 * growth)


# ------------------------------------------------------------- tree / lists
def _tree_case(seed=7, nf=25, el=30, leaf=16):
    wl = W.random_fractures(seed, nf, el)
    g = O.Geometry.of(wl)
    return g, O.Tree(g, leaf=leaf)


def test_tree_invariants():
    g, T = _tree_case()
    x0, y0, L = T.root
    assert x0 == g.cx.min() and y0 == g.cy.min()
    assert L == max(np.ptp(g.cx), np.ptp(g.cy))
    # cells ordered by (level, key)
    order = np.lexsort((T.ix, T.iy, T.level))  # noqa: F841 (ordering checked below)
    lv = T.level
    assert np.all(np.diff(lv) >= 0)
    assert np.sort(T.perm).tolist() == list(range(g.n))
    leafs = np.where(T.isleaf == 1)[0]
    assert (T.pend[leafs] - T.pbeg[leafs]).sum() == g.n
    for c in range(T.ncell):
        side = L / 2.0 ** T.level[c]
        bx0, by0 = x0 + T.ix[c] * side, y0 + T.iy[c] * side
        pts = T.perm[T.pbeg[c]:T.pend[c]]
        assert len(pts) > 0                             # no zero cells stored
        # every point of the cell lies in the cell's closed square
        assert np.all(g.cx[pts] >= bx0 - 1e-12 * L) and np.all(g.cx[pts] <= bx0 + side + 1e-12 * L)
        assert np.all(g.cy[pts] >= by0 - 1e-12 * L) and np.all(g.cy[pts] <= by0 + side + 1e-12 * L)
        if T.isleaf[c]:
            n_c = len(pts)
            child_side = side / 2
            amax = g.a[pts].max()
            # a leaf is either small enough or not allowed to split
            assert n_c <= 16 or child_side < O.KAPPA * amax or T.level[c] >= O.MAX_LEVEL
        else:
            kids = [k for k in T.child[c] if k >= 0]
            assert sum(T.pend[k] - T.pbeg[k] for k in kids) == T.pend[c] - T.pbeg[c]
            for d in range(4):
                k = T.child[c, d]
                if k < 0:
                    continue
                # paper's child order: left to right, then bottom to top
                assert T.ix[k] == 2 * T.ix[c] + (d & 1)
                assert T.iy[k] == 2 * T.iy[c] + (d >> 1)
                assert T.parent[k] == c and T.level[k] == T.level[c] + 1
    # within a level, cells are in Morton (Z) order of their coordinates
    for l in range(lv.max() + 1):
        cs = np.where(lv == l)[0]
        keys = []
        for c in cs:
            k = 0
            for b in range(l):
                k |= ((int(T.ix[c]) >> b) & 1) << (2 * b)
                k |= ((int(T.iy[c]) >> b) & 1) << (2 * b + 1)
            keys.append(k)
        assert keys == sorted(keys)


def _adj(T, c, d):
    lm = max(T.level[c], T.level[d])
    sc, sd = 1 << (lm - T.level[c]), 1 << (lm - T.level[d])
    cx0, cy0 = int(T.ix[c]) * sc, int(T.iy[c]) * sc
    dx0, dy0 = int(T.ix[d]) * sd, int(T.iy[d]) * sd
    return cx0 <= dx0 + sd and dx0 <= cx0 + sc and cy0 <= dy0 + sd and dy0 <= cy0 + sc


def _ancestors(T, c):
    out = []
    while c >= 0:
        out.append(c)
        c = T.parent[c]
    return out


def test_lists_cover_every_pair_exactly_once():
    """For every (target leaf, source leaf) pair, exactly one of: the source
    is in U(target); the source lies under a W(target) cell; the source is in
    X of an ancestor-or-self of the target; or an ancestor-or-self pair
    (A of target, B of source) has B in V(A).  This is what makes the FMM
    sum every interaction exactly once."""
    g, T = _tree_case(seed=9, nf=30, el=25, leaf=8)
    L = T.lists

    def lst(name, c):
        off, idx = L[name]
        return set(idx[off[c]:off[c + 1]].tolist())

    leaves = np.where(T.isleaf == 1)[0]
    anc = {c: _ancestors(T, c) for c in range(T.ncell)}
    for t in leaves:
        Ut, Wt = lst("U", t), lst("W", t)
        Xs = set()
        for a in anc[t]:
            Xs |= lst("X", a)
        Vsets = {a: lst("V", a) for a in anc[t]}
        for s in leaves:
            cnt = int(s in Ut)
            cnt += sum(1 for w in Wt if w in anc[s])
            cnt += int(s in Xs)
            cnt += sum(1 for a in anc[t] for b in anc[s] if b in Vsets[a])
            assert cnt == 1, (t, s, cnt)


def test_list_structure():
    g, T = _tree_case(seed=9, nf=30, el=25, leaf=8)
    L = T.lists

    def lst(name, c):
        off, idx = L[name]
        return idx[off[c]:off[c + 1]].tolist()

    for c in range(T.ncell):
        for name in "UVWX":
            v = lst(name, c)
            assert v == sorted(v)
        for a in lst("U", c):
            assert c in lst("U", a) and _adj(T, a, c)
        for a in lst("V", c):
            assert c in lst("V", a)
            assert T.level[a] == T.level[c] and not _adj(T, a, c)
            assert _adj(T, T.parent[a], T.parent[c])
        for a in lst("W", c):
            assert c in lst("X", a)
            assert T.isleaf[c] and not _adj(T, a, c) and _adj(T, T.parent[a], c)
        if T.isleaf[c]:
            assert c in lst("U", c)


# ----------------------------------------------------------------- FMM pins
def test_fmm_polynomial_kernel_is_exact():
    """With a kernel of degree < p in every coordinate, each far-field step
    (leaf weights, M2M, M2L, L2L, L2P) is exact, so the FMM must reproduce
    the dense product to rounding for any tree: checks the whole pass
    structure and the list coverage at once."""
    g, T = _tree_case(seed=13, nf=20, el=20, leaf=6)
    D = W.random_vector(2, g.n)
    yd = O.dense_matrix_poly(g) @ D
    for p in (4, 6):
        yf = T.fmm(D, p, kernel=1)
        assert np.linalg.norm(yf - yd) / np.linalg.norm(yd) < 1e-12


def test_fmm_elastic_converges_geometrically():
    """Elastic kernel: FMM error against the dense product decays
    geometrically with the number of Chebyshev nodes."""
    g, T = _tree_case(seed=7, nf=20, el=30, leaf=16)
    D = W.random_vector(1, g.n)
    yd = O.dense_matrix(g) @ D
    errs = []
    for p in (4, 6, 8, 10):
        yf = T.fmm(D, p)
        errs.append(np.linalg.norm(yf - yd) / np.linalg.norm(yd))
    for a, b in zip(errs, errs[1:]):
        assert b < a / 3
    assert errs[-1] < 1e-8


def test_gmres_matches_direct_solve():
    """GMRES on the dense operator reproduces the Gaussian-elimination
    solution (unique, the system is nonsingular) within cond * tol."""
    wl = W.random_fractures(21, 8, 20)
    g = O.Geometry.of(wl)
    A = O.dense_matrix(g)
    b = O.rhs(g, wl.pressure, wl.SH, wl.Sh)
    xl = O.lu_solve(A, b)
    assert np.linalg.norm(A @ xl - b) / np.linalg.norm(b) < 1e-12
    xg, info = O.gmres_dense(A, b, restart=50, tol=1e-12)
    assert info["converged"]
    assert np.linalg.norm(xg - xl) / np.linalg.norm(xl) < 1e-8
    xd, info2 = O.gmres_direct(g, b, restart=50, tol=1e-12)
    assert info2["converged"]
    assert np.linalg.norm(xd - xl) / np.linalg.norm(xl) < 1e-8


def test_well_cluster_paper_observations():
    """Five parallel fractures under the paper's Table 2 loads (scaled-down
    discretisation): by symmetry the middle fracture has no shear DD at its
    centre, and the outer fractures open more than the inner ones (stress
    shadow), as the paper reports for its horizontal-well example."""
    gold = json.load(open(GOLD))["well_table_2"]
    wl = W.well_cluster(n_frac=5, elems=40, half_length=gold["half_length_m"],
                        spacing=gold["spacing_m"], p_inj=gold["p_inj_MPa"] * 1e6,
                        SH=gold["SH_MPa"] * 1e6, Sh=gold["Sh_MPa"] * 1e6, E=15e9 * 2.5, nu=0.25)
    g = O.Geometry.of(wl)
    A = O.dense_matrix(g)
    x = O.lu_solve(A, O.rhs(g, wl.pressure, wl.SH, wl.Sh))
    Dn = x[1::2].reshape(5, 40)
    Ds = x[0::2].reshape(5, 40)
    assert Dn[2, 20] > 0 and Dn[0, 20] > 0 and Dn[4, 20] > 0
    assert abs(Ds[2, 19] + Ds[2, 20]) < 1e-10 * Dn[2, 20]     # antisymmetric about centre
    assert abs(Ds[2, 20]) < 1e-3 * Dn[2, 20]
    assert Dn[0, 20] > Dn[2, 20] and Dn[4, 20] > Dn[2, 20]
    assert np.allclose(Dn[0], Dn[4], rtol=1e-9)               # mirror symmetry


def _split_tie_kappa(g):
    """kappa at which the long element of W.split_tie() ties the split test
    of its level-2 cell exactly: children of side 2 >= kappa * amax."""
    amax = g.a.max()
    kappa = 2.0 / amax
    assert kappa * amax == 2.0
    return kappa


def test_tree_split_at_a_tie():
    """Section 3.1 split rule with the size reading (children at least kappa
    times the largest half-length): a tie splits (>=).  One unit in the last
    place more on the half-length stops the split one level earlier, so the
    tree depends on the half-length's rounding (the GPU builds the same tree
    bit for bit, test_gpu_parity)."""
    wl = W.split_tie()
    g = O.Geometry.of(wl)
    dx, dy = wl.x2[0] - wl.x1[0], wl.y2[0] - wl.y1[0]
    assert g.a[0] == 0.5 * np.sqrt(dx * dx + dy * dy)           # separately rounded
    assert 0.5 * np.hypot(dx, dy) == np.nextafter(g.a[0], 1.0)  # one ulp above
    kappa = _split_tie_kappa(g)
    box = wl.meta["root_box"]

    def leaf_level_of_long_element(gg):
        T = O.Tree(gg, leaf=4, kappa=kappa, box=box, lists=False)
        pos = int(np.where(T.perm == 0)[0][0])
        leafs = np.where((T.isleaf == 1) & (T.pbeg <= pos) & (T.pend > pos))[0]
        assert len(leafs) == 1
        return int(T.level[leafs[0]])

    assert leaf_level_of_long_element(g) == 3
    g.a = g.a.copy()
    g.a[0] = np.nextafter(g.a[0], 1.0)
    assert leaf_level_of_long_element(g) == 2
