"""GMRES with each Arnoldi step replayed as a captured HIP graph, against
the same solves with plain launches, through the C ABI.

The kernels are deterministic (fixed-order sums, no atomics), so replays
must reproduce the eager launches bit for bit: every step graph is
replayed in every restart cycle, with the eager residual products and host
synchronisations between the replays, and across solves with different
right-hand sides on the same tree, with plain products interleaved.  Any
replay that computed something else would change the iterates and so the
returned solution.
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_1812_05087_amd as F  # noqa: E402


def solves(wl, graphs, mode, **kw):
    prob = F.Problem(wl.x1, wl.y1, wl.x2, wl.y2, E=wl.E, nu=wl.nu, use_graphs=graphs, **kw)
    out = []
    try:
        b1 = prob.rhs(wl.pressure, wl.SH, wl.Sh)
        b2 = prob.rhs(0.5 * wl.pressure, 0.0, 0.0)
        for b in (b1, b2, b1):
            x, info = prob.solve(b, mode)
            # a plain product between the solves
            y = prob.apply(x, mode)
            out.append((x.cpu().numpy(), info["iters"], info["status"], y.cpu().numpy()))
    finally:
        prob.close()
    return out


@pytest.mark.parametrize("mode,prec", [(F.FMDDM_APPLY_FMM, F.FMDDM_PREC_FP64),
                                       (F.FMDDM_APPLY_FMM, F.FMDDM_PREC_FP32),
                                       (F.FMDDM_APPLY_DIRECT, F.FMDDM_PREC_FP64)])
def test_graph_replays_match_plain_launches(mode, prec):
    wl = W.random_fractures(41, n_frac=25, elems=40)
    kw = dict(p=10, leaf=32, m2l=F.FMDDM_M2L_SVD, m2l_tol=1e-10, restart=20, tol=1e-9, maxit=3000,
              precision=prec)
    eager = solves(wl, 0, mode, **kw)
    graph = solves(wl, 1, mode, **kw)
    for k, ((xe, ie, se, ye), (xg, ig, sg, yg)) in enumerate(zip(eager, graph)):
        assert se == sg == F.FMDDM_OK, (k, se, sg)
        assert ie == ig and ie > 20, (k, ie, ig)   # several restart cycles
        assert np.array_equal(xe, xg), (k, float(np.abs(xe - xg).max()))
        assert np.array_equal(ye, yg), k
    # the third solve repeats the first on the replayed graphs
    assert np.array_equal(graph[0][0], graph[2][0])


@pytest.mark.parametrize("mode", [F.FMDDM_APPLY_FMM, F.FMDDM_APPLY_DENSE])
def test_block_jacobi_preconditioning(mode):
    """Right block-Jacobi preconditioning changes the iteration count, not
    the solution: both solves meet the tolerance on the same operator and
    agree with the oracle's LU solve to cond * tol plus the FMM error."""
    import oracle as O
    wl = W.random_fractures(42, n_frac=30, elems=60, box=40.0)
    g = O.Geometry.of(wl)
    b = O.rhs(g, wl.pressure, wl.SH, wl.Sh)
    x_lu = O.lu_solve(O.dense_matrix(g), b)
    kw = dict(p=12, leaf=32, m2l=F.FMDDM_M2L_SVD, m2l_tol=1e-10, restart=50, tol=1e-10, maxit=20000)
    res = {}
    for pc in (F.FMDDM_PRECOND_NONE, F.FMDDM_PRECOND_BLOCK, F.FMDDM_PRECOND_TWO_LEVEL):
        prob = F.Problem(wl.x1, wl.y1, wl.x2, wl.y2, E=wl.E, nu=wl.nu, precond=pc, **kw)
        try:
            x, info = prob.solve(prob.vec(b), mode)
        finally:
            prob.close()
        assert info["status"] == F.FMDDM_OK and info["relres"] <= 1e-10, (pc, info)
        e = float(np.linalg.norm(x.cpu().numpy() - x_lu) / np.linalg.norm(x_lu))
        print(f"mode {mode} precond {pc}: {info['iters']} iterations, vs oracle LU {e:.2e}")
        assert e <= (1e-7 if mode == F.FMDDM_APPLY_DENSE else 1e-6), (pc, e)
        res[pc] = (x.cpu().numpy(), info["iters"])
    assert res[F.FMDDM_PRECOND_BLOCK][1] * 2 <= res[F.FMDDM_PRECOND_NONE][1], res
    assert res[F.FMDDM_PRECOND_TWO_LEVEL][1] <= res[F.FMDDM_PRECOND_BLOCK][1], res
    for pc in (F.FMDDM_PRECOND_BLOCK, F.FMDDM_PRECOND_TWO_LEVEL):
        d = np.linalg.norm(res[0][0] - res[pc][0]) / np.linalg.norm(res[0][0])
        assert d <= 1e-7, (pc, d)


def test_two_level_on_long_fractures():
    """Five parallel fractures of 800 elements, 10 m apart (the well-cluster
    shape), on the exact operator (stored dense): the coarse level
    (aggregates of 16 collinear elements as long elements) carries the
    long-wavelength modes that block-Jacobi leaves to GMRES.  Both solves
    (to 1e-11) agree with the oracle's LU solve to cond x 1e-11 (bar 1e-8),
    the two-level one in at most half the products."""
    import oracle as O
    wl = W.well_cluster(n_frac=5, elems=800, half_length=80.0, spacing=10.0)
    g = O.Geometry.of(wl)
    b = O.rhs(g, wl.pressure, wl.SH, wl.Sh)
    x_lu = O.lu_solve(O.dense_matrix(g), b)
    kw = dict(p=8, leaf=32, restart=100, tol=1e-11, maxit=20000)
    res = {}
    for pc in (F.FMDDM_PRECOND_BLOCK, F.FMDDM_PRECOND_TWO_LEVEL):
        prob = F.Problem(wl.x1, wl.y1, wl.x2, wl.y2, E=wl.E, nu=wl.nu, precond=pc, **kw)
        try:
            x, info = prob.solve(prob.vec(b), F.FMDDM_APPLY_DENSE)
        finally:
            prob.close()
        assert info["status"] == F.FMDDM_OK and info["relres"] <= 1e-11, (pc, info)
        xs = x.cpu().numpy()
        e = float(np.linalg.norm(xs - x_lu) / np.linalg.norm(x_lu))
        print(f"long fractures, precond {pc}: {info['iters']} iterations, vs oracle LU {e:.2e}")
        assert e <= 1e-8, (pc, e)
        res[pc] = info["iters"]
    assert 2 * res[F.FMDDM_PRECOND_TWO_LEVEL] <= res[F.FMDDM_PRECOND_BLOCK], res


def test_two_level_left_out_without_collinear_runs():
    """2100 one-element fractures form 2100 aggregates, above the coarse
    level's cap (2048): the two-level solve is then the block-Jacobi one,
    bit for bit, instead of inverting a 4200 x 4200 coarse matrix."""
    wl = W.random_fractures(44, n_frac=2100, elems=1, box=200.0, lmin=0.5, lmax=1.0)
    kw = dict(p=8, leaf=32, m2l=F.FMDDM_M2L_SVD, m2l_tol=1e-10, restart=30, tol=1e-10, maxit=3000)
    res = {}
    for pc in (F.FMDDM_PRECOND_BLOCK, F.FMDDM_PRECOND_TWO_LEVEL):
        prob = F.Problem(wl.x1, wl.y1, wl.x2, wl.y2, E=wl.E, nu=wl.nu, precond=pc, **kw)
        try:
            b = prob.rhs(wl.pressure, wl.SH, wl.Sh)
            x, info = prob.solve(b)
        finally:
            prob.close()
        assert info["status"] == F.FMDDM_OK, (pc, info)
        res[pc] = (x.cpu().numpy(), info["iters"])
    a, c = res[F.FMDDM_PRECOND_TWO_LEVEL], res[F.FMDDM_PRECOND_BLOCK]
    assert a[1] == c[1] and np.array_equal(a[0], c[0])


@pytest.mark.parametrize("pc", [F.FMDDM_PRECOND_BLOCK, F.FMDDM_PRECOND_TWO_LEVEL])
def test_preconditioned_graph_replays_match_plain_launches(pc):
    wl = W.random_fractures(43, n_frac=25, elems=40)
    kw = dict(p=10, leaf=32, m2l=F.FMDDM_M2L_SVD, m2l_tol=1e-10, restart=10, tol=1e-10, maxit=3000,
              precond=pc)
    eager = solves(wl, 0, F.FMDDM_APPLY_FMM, **kw)
    graph = solves(wl, 1, F.FMDDM_APPLY_FMM, **kw)
    for k, ((xe, ie, se, ye), (xg, ig, sg, yg)) in enumerate(zip(eager, graph)):
        assert se == sg == F.FMDDM_OK and ie == ig and ie > 10, (k, se, sg, ie, ig)
        assert np.array_equal(xe, xg) and np.array_equal(ye, yg), k
