"""Pins of the oracle's poroelastic influence (Section 2, eqs. 2.1-2.5).

The paper cites rather than states the poroelastic fundamental solutions, so
the oracle derives them; these tests fix them by what the mathematics and
physics determine independently of the derivation:
  - E1 against the library routine (scipy.special.exp1);
  - t -> 0+: the undrained elastic field (Poisson ratio nu_u, closed form of
    the elastic point kernel) and Skempton's pressure p = -B (1 + nu_u)
    (sxx + syy) / 3;
  - t -> infinity: the drained elastic field, p -> 0;
  - at any t > 0: equilibrium (div sigma = 0) and pressure diffusion
    (dp/dt = c lap p) by finite differences;
  - fluid source: volume balance S * integral(p) dA = Q t;
  - element integrals: quadrature convergence, the two-halves identity, the
    point-source far-field limit;
  - time marching: telescoping of the history coefficients;
  - the symmetric well cluster: zero shear DD on the middle fracture;
  - the transient stress potential at intermediate times, which equilibrium
    cannot see: the trace identity sxx + syy = -2 G eta p (fixes its
    Laplacian, hence the radial factor of the DD part), boundedness of the
    transient at the source, and the Biot reciprocal theorem between a DD's
    pressure and a fluid source's stress (fixes the source's potential),
    for points and for a symmetric element pair.  A 1 % error planted in
    either radial factor fails these and none of the others.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W

special = pytest.importorskip("scipy.special")
integrate = pytest.importorskip("scipy.integrate")


@pytest.fixture(scope="module")
def po():
    # Section 5.2.1 / Table 1 style constants of the well example
    return O.Poro(E=20e9, nu=0.2, nuu=0.35, alpha=0.8, perm=1e-18, visc=1e-3)


def elastic(x, y, G, nu, q):
    K = np.zeros(9)
    O.lib().ora_point_kernel(x, y, G, nu, O._p(K))
    return K.reshape(3, 3) @ q


def test_E1_matches_library():
    # series below 1.5, continued fraction above; the fraction's evaluation
    # accumulates rounding over up to a few hundred terms (measured <= 1e-14)
    for z in np.concatenate([np.geomspace(1e-10, 1.49, 25), [1.5, 1.5 + 1e-12],
                             np.geomspace(1.51, 600, 40)]):
        ref = special.exp1(z)
        assert abs(O.E1(z) - ref) <= 2e-14 * abs(ref), z


def test_constants_are_consistent(po):
    # c = kappa / S equals the closed form 2 kappa G (1-nu)(nu_u-nu) / (alpha^2 (1-2nu)^2 (1-nu_u))
    c2 = 2 * po.kappa * po.G * (1 - po.nu) * (po.nuu - po.nu) / (
        po.alpha ** 2 * (1 - 2 * po.nu) ** 2 * (1 - po.nuu))
    assert abs(po.c - c2) < 1e-12 * c2
    assert abs(po.c - 1.3354700854700853e-05) < 1e-15


CHARGES = [np.array([1.0, 1.0, 0.0]), np.array([1.0, -1.0, 0.0]), np.array([0.0, 0.0, 1.0]),
           np.array([0.3, -0.7, 0.45])]
POINTS = [(0.8, 0.35), (-0.2, 1.3), (2.5, -0.1)]


@pytest.mark.parametrize("q", CHARGES)
def test_undrained_limit(po, q):
    for x, y in POINTS:
        r2 = x * x + y * y
        t = r2 / (4 * po.c) / 800.0          # z = 800: exp(-z) underflows
        s = O.poro_point(po, x, y, t, q)
        su = elastic(x, y, po.G, po.nuu, q)
        # the deviatoric part approaches the undrained field like 1/z
        tol = 4.0 / 800.0
        assert np.abs(s[:3] - su).max() <= tol * np.abs(su).max()
        t = r2 / (4 * po.c) / 1e9
        s = O.poro_point(po, x, y, t, q)
        assert np.abs(s[:3] - su).max() <= 1e-8 * np.abs(su).max()
        pu = -po.B * (1 + po.nuu) / 3 * (su[0] + su[1])
        assert abs(s[3] - pu) <= 1e-12 * max(abs(pu), np.abs(su).max() * po.B)


@pytest.mark.parametrize("q", CHARGES)
def test_drained_limit(po, q):
    for x, y in POINTS:
        r2 = x * x + y * y
        t = r2 / (4 * po.c) * 1e8            # z = 1e-8
        s = O.poro_point(po, x, y, t, q)
        sd = elastic(x, y, po.G, po.nu, q)
        assert np.abs(s[:3] - sd).max() <= 1e-6 * np.abs(sd).max()
        su = elastic(x, y, po.G, po.nuu, q)
        assert abs(s[3]) <= 1e-6 * po.B * np.abs(su).max()


@pytest.mark.parametrize("zt", [0.2, 1.5, 14.0])
def test_equilibrium_and_diffusion(po, zt):
    q = np.array([0.3, -0.7, 0.45])
    x, y = 0.8, 0.35
    t = (x * x + y * y) / (4 * po.c * zt)
    f = lambda X, Y, T: O.poro_point(po, X, Y, T, q, qf=2e-9)
    h = 1e-4
    s0 = f(x, y, t)
    dsxx = (f(x + h, y, t)[0] - f(x - h, y, t)[0]) / (2 * h)
    dsxy_y = (f(x, y + h, t)[2] - f(x, y - h, t)[2]) / (2 * h)
    dsxy_x = (f(x + h, y, t)[2] - f(x - h, y, t)[2]) / (2 * h)
    dsyy = (f(x, y + h, t)[1] - f(x, y - h, t)[1]) / (2 * h)
    scale = np.abs(s0[:3]).max() / np.hypot(x, y)
    assert abs(dsxx + dsxy_y) < 1e-6 * scale
    assert abs(dsxy_x + dsyy) < 1e-6 * scale
    # second-order differences: the error falls like hx^2 / ell^2 (ell the
    # diffusion length), largest at early times (large z)
    hx, ht = 5e-4, 2e-4 * t
    pt = (f(x, y, t + ht)[3] - f(x, y, t - ht)[3]) / (2 * ht)
    lap = (f(x + hx, y, t)[3] + f(x - hx, y, t)[3] + f(x, y + hx, t)[3] + f(x, y - hx, t)[3]
           - 4 * s0[3]) / hx ** 2
    tol = 1e-5 if zt < 5 else 1e-3
    assert abs(pt - po.c * lap) < tol * max(abs(pt), abs(po.c * lap))


def test_fluid_source_volume_balance_and_start(po):
    t = 3600.0
    # S * integral of p over the plane = injected volume Q t (Q = 1)
    ell = np.sqrt(4 * po.c * t)
    f = lambda r: O.poro_point(po, r, 0.0, t, np.zeros(3), qf=1.0, transient=True)[3] * 2 * np.pi * r
    tot = 0.0
    edges = np.concatenate([[0.0], np.geomspace(1e-9, 40 * ell, 200)])
    for a, b in zip(edges[:-1], edges[1:]):
        tot += integrate.quad(f, a, b, epsabs=0, epsrel=1e-12)[0]
    assert abs(po.S * tot - t) < 1e-8 * t
    # just after the source starts (diffusion length << r) the pressure has
    # not arrived and the stress is that of the injected volume alone, a
    # center of dilatation growing linearly in t
    s1 = O.poro_point(po, 0.5, 0.2, 1e-6, np.zeros(3), qf=1.0, transient=True)
    s2 = O.poro_point(po, 0.5, 0.2, 2e-6, np.zeros(3), qf=1.0, transient=True)
    assert s1[3] == 0.0 and s2[3] == 0.0
    assert np.abs(s2[:3] - 2 * s1[:3]).max() <= 1e-12 * np.abs(s2[:3]).max()
    assert abs(s1[0] + s1[1]) <= 1e-12 * np.abs(s1[:3]).max()   # trace-free


def test_element_quadrature_converges(po):
    dt = 60.0
    for (X, Y) in [(0.0, 0.0), (0.05, 0.0), (0.05, 0.01), (0.3, 0.2), (2.0, 1.0)]:
        for t1, t0 in [(dt, 0.0), (5 * dt, 4 * dt)]:
            a = O.poro_elem_transient(po, X, Y, 0.0, 0.0, 1.0, 0.0, 0.1, 1e-3, 2e-3, 1e-9, t1, t0)
            b = O.poro_elem_transient(po, X, Y, 0.0, 0.0, 1.0, 0.0, 0.1, 1e-3, 2e-3, 1e-9, t1, t0, 24, 12)
            assert np.abs(a - b).max() <= 3e-12 * np.abs(b).max(), (X, Y, t1)


def test_element_halves_and_far_field(po):
    cb, sb = np.cos(0.4), np.sin(0.4)
    a, t = 0.2, 600.0
    X, Y = 0.13, 0.31
    whole = O.poro_elem_transient(po, X, Y, 0.0, 0.0, cb, sb, a, 1e-3, -2e-3, 3e-9, t)
    h1 = O.poro_elem_transient(po, X, Y, -a / 2 * cb, -a / 2 * sb, cb, sb, a / 2, 1e-3, -2e-3, 3e-9, t)
    h2 = O.poro_elem_transient(po, X, Y, a / 2 * cb, a / 2 * sb, cb, sb, a / 2, 1e-3, -2e-3, 3e-9, t)
    assert np.abs(whole - (h1 + h2)).max() <= 1e-11 * np.abs(whole).max()
    # far away the element acts as a point source of strength 2a
    X, Y = 40.0, 25.0
    el = O.poro_elem_transient(po, X, Y, 0.0, 0.0, cb, sb, 0.01, 1e-3, -2e-3, 3e-9, 1e7)
    q = np.zeros(3)
    O.lib().ora_charge(cb, sb, 1e-3, -2e-3, O._p(q))
    pt = 0.02 * O.poro_point(po, X, Y, 1e7, q, qf=3e-9, transient=True)
    assert np.abs(el - pt).max() <= 1e-6 * np.abs(pt).max()


def test_history_coefficients_telescope(po):
    """A DD held constant over h intervals: F(dt) D + sum_{m=1}^{h-1} K_m D
    equals the continuous response F(h dt) D."""
    wl = W.well_cluster(n_frac=2, elems=6, half_length=1.0, spacing=0.5)
    g = O.Geometry.of(wl)
    dt, h = 60.0, 7
    rng = np.random.default_rng(3)
    D = rng.standard_normal(3 * g.n) * np.tile([1e-3, 1e-3, 1e-9], g.n)
    acc = O.poro_matrix(g, po, dt, 0) @ D
    for m in range(1, h):
        acc += O.poro_matrix(g, po, dt, m) @ D
    full = O.poro_matrix(g, po, h * dt, 0) @ D
    assert np.abs(acc - full).max() <= 1e-9 * np.abs(full).max()


def test_well_cluster_symmetry(po):
    """Three parallel fractures, symmetric about the middle one: its shear
    DD vanishes and the outer two mirror each other (Section 5.2.1)."""
    wl = W.well_cluster(n_frac=3, elems=10, half_length=2.0, spacing=1.0)
    g = O.Geometry.of(wl)
    Ds, _, _ = O.poro_march(g, po, 60.0, 4, wl.pressure, 48.26e6, wl.SH, wl.Sh)
    D = Ds[-1].reshape(-1, 3)
    mid = D[10:20]
    assert np.abs(mid[:, 0]).max() <= 1e-9 * np.abs(D[:, 1]).max()
    top, bot = D[20:30], D[0:10]
    assert np.allclose(top[:, 1], bot[:, 1], rtol=1e-9, atol=1e-12 * np.abs(D[:, 1]).max())
    assert np.allclose(top[:, 0], -bot[:, 0], rtol=1e-9, atol=1e-12 * np.abs(D[:, 1]).max())
    # fluid leaks off into the formation while the fracture pressure exceeds p0
    assert (D[:, 2] > 0).all()


def test_matrix_rows_are_rows_of_the_matrix(po):
    """The sampled-row evaluation (used for full-size GPU parity) is the
    same matrix restricted to the chosen receivers."""
    wl = W.well_cluster(n_frac=2, elems=7, half_length=1.0, spacing=0.5)
    g = O.Geometry.of(wl)
    rows = np.array([0, 5, 13])
    for m in (0, 2):
        A = O.poro_matrix(g, po, 60.0, m)
        R = O.poro_matrix_rows(g, po, 60.0, m, rows)
        idx = np.stack([3 * rows, 3 * rows + 1, 3 * rows + 2], 1).reshape(-1)
        assert np.array_equal(R, A[idx])


# --------------------------------------------------------------------------
# Pins of the transient stress potential at intermediate times.  The stress
# of the transient part is 2G (grad grad phi - I lap phi) for some potential
# phi, which is divergence-free for any phi, so equilibrium alone cannot see
# an error in phi; these three relations can.
# --------------------------------------------------------------------------
Z_MID = [0.05, 0.2, 1.5, 5.0, 14.0]


@pytest.mark.parametrize("z", Z_MID)
def test_transient_trace_is_minus_2G_eta_p(po, z):
    """Biot plane strain: the irrotational transient displacement carries a
    volumetric strain alpha p / (lambda + 2G) = eta p, so the in-plane trace
    of the transient stress is 2 (lambda + G) eta p - 2 alpha p
    = -2 G eta p.  Holds at every z for displacement discontinuities and
    for fluid sources alike."""
    x, y = 0.8, 0.35
    t = (x * x + y * y) / (4 * po.c * z)
    for q, qf in [(c, 0.0) for c in CHARGES] + [(np.zeros(3), 1.0), (CHARGES[3], 2e-9)]:
        s = O.poro_point(po, x, y, t, q, qf=qf, transient=True)
        scale = max(np.abs(s[:3]).max(), 2 * po.G * po.eta * abs(s[3]))
        assert abs(s[0] + s[1] + 2 * po.G * po.eta * s[3]) <= 1e-12 * scale, (z, q, qf)


def test_transient_bounded_at_the_source(po):
    """At a fixed time the transient part of a displacement discontinuity
    (total minus drained) stays finite as the receiver approaches the
    source: the singular part is the drained elastic field alone.  The
    values converge as r -> 0."""
    t = 600.0
    ell = np.sqrt(4 * po.c * t)
    for q in CHARGES:
        prev, rprev = None, None
        for rr in [1e-3, 1e-4, 1e-5, 1e-6]:
            s = O.poro_point(po, 0.6 * rr * ell, 0.8 * rr * ell, t, q, transient=True)
            assert np.all(np.isfinite(s))
            if prev is not None:
                # z = rr^2 and the approach is O(z): the step from rprev to rr
                # changes the values by O(rprev^2)
                assert np.abs(s - prev).max() <= 10 * rprev * rprev * np.abs(s).max(), (q, rr)
            prev, rprev = s, rr
        # and the limit is of the size of the field one diffusion length away
        far = O.poro_point(po, 0.6 * ell, 0.8 * ell, t, q, transient=True)
        assert np.abs(prev).max() <= 100 * np.abs(far).max()


@pytest.mark.parametrize("z", Z_MID)
def test_reciprocity_dd_pressure_vs_source_stress(po, z):
    """Reciprocal theorem of Biot poroelasticity in the Laplace domain:
    sigma1 : e2 + p1 zeta2 is symmetric in the two states (e the matrix
    strain, zeta the fluid content), and for an infinite plane it gives,
    for a point DD (eigenstrain charges q) held at y and a unit fluid source
    rate held at x,
        integral_0^t p_DD(x - y, tau) d tau = -sigma_src(y - x, t) : q.
    This ties the fluid source's stress (its potential) to the DD's
    pressure, which the diffusion and limit pins fix."""
    x, y = 0.8, 0.35
    t = (x * x + y * y) / (4 * po.c * z)
    for q in CHARGES:
        P = lambda tau: O.poro_point(po, x, y, tau, q, transient=True)[3]
        lhs = integrate.quad(P, 0.0, t, epsabs=0, epsrel=1e-12, limit=200)[0]
        f = O.poro_point(po, -x, -y, t, np.zeros(3), qf=1.0, transient=True)
        rhs = -(f[0] * q[0] + f[1] * q[1] + f[2] * q[2])
        scale = np.abs(f[:3]).max() * np.abs(q).max()
        assert abs(lhs - rhs) <= 1e-9 * scale, (z, q, lhs, rhs)


def test_reciprocity_symmetric_element_pair(po):
    """The same reciprocity for two equal parallel elements (receiver at one
    midpoint, source integrated over the other): with D_n = 1 on element 2
    and a unit fluid source on element 1, the time integral of the pressure
    at midpoint 1 equals minus the normal-charge stress at midpoint 2; and
    the DD-to-stress and source-to-pressure blocks are symmetric."""
    a, t = 0.1, 1800.0
    cb, sb = np.cos(0.3), np.sin(0.3)
    for d in [(0.35, 0.12), (0.0, 0.25), (0.7, 0.0)]:
        x1, y1 = 0.0, 0.0
        x2, y2 = d
        q = np.zeros(3)
        O.lib().ora_charge(cb, sb, 0.0, 1.0, O._p(q))     # charges of D_n = 1
        P = lambda tau: O.poro_elem_transient(po, x1, y1, x2, y2, cb, sb, a, 0.0, 1.0, 0.0, tau)[3]
        lhs = integrate.quad(P, 0.0, t, epsabs=0, epsrel=1e-11, limit=200)[0]
        f = O.poro_elem_transient(po, x2, y2, x1, y1, cb, sb, a, 0.0, 0.0, 1.0, t)
        rhs = -(f[0] * q[0] + f[1] * q[1] + f[2] * q[2])
        assert abs(lhs - rhs) <= 1e-8 * np.abs(f[:3]).max(), (d, lhs, rhs)
        for Ds, Dn, Dq in [(1e-3, 0.0, 0.0), (0.0, 1e-3, 0.0), (0.0, 0.0, 1e-9)]:
            s12 = O.poro_elem_transient(po, x1, y1, x2, y2, cb, sb, a, Ds, Dn, Dq, t)
            s21 = O.poro_elem_transient(po, x2, y2, x1, y1, cb, sb, a, Ds, Dn, Dq, t)
            assert np.abs(s12 - s21).max() <= 1e-11 * np.abs(s12).max(), (d, Ds, Dn, Dq)
