"""Serving engine on the GPU (through the C ABI): continuous batching of
fracture solves of different sizes.

Bars:
  - a request's DDs are the same alone and in a mix of concurrently running
    requests: bitwise (per-request buffers, deterministic kernels);
  - a served solution satisfies the oracle's exact system (direct product,
    same right-hand side) to the requested tolerance plus the FMM error;
  - admission never lets the admitted requests' estimated footprints exceed
    the budget; a request larger than the budget fails with ENOMEM;
  - the footprint estimate covers the device memory a request allocates;
  - a request that cannot converge within maxit fails with ENOTCONV.
"""
import time

import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_1812_05087_amd as F  # noqa: E402

P_SERVE = dict(p=10, leaf=32, m2l=1, m2l_tol=1e-10, restart=50, maxit=5000)


def submit(srv, req, tol=1e-6):
    wl = req.workload()
    return F.fmddm_server_submit(srv, wl.x1, wl.y1, wl.x2, wl.y2, wl.pressure, wl.SH, wl.Sh,
                                 req.steps, tol), wl


def drain(srv, tickets, limit_s=120.0, watch=None):
    """Step the engine until every ticket is finished; returns {ticket: result}."""
    t0 = time.time()
    while True:
        F.fmddm_server_step(srv)
        if watch is not None:
            watch()
        res = {t: F.fmddm_server_poll(srv, t)[0] for t in tickets}
        if all(r["state"] >= F.FMDDM_REQ_DONE for r in res.values()):
            return res
        assert time.time() - t0 < limit_s, "serving loop did not finish"


@pytest.mark.parametrize("pc", [F.FMDDM_PRECOND_NONE, F.FMDDM_PRECOND_TWO_LEVEL])
def test_alone_equals_mix_bitwise(pc):
    reqs = W.serving_stream(seed=7, count=10, nmin=500, nmax=6000, steps_max=3)
    prm = F.fmddm_default_params(**P_SERVE, precond=pc, coarse_aggregates=128)
    srv = F.fmddm_server_create(prm, 5)
    try:
        mix = {}
        tickets = []
        for r in reqs:
            t, wl = submit(srv, r)
            tickets.append(t)
            mix[t] = wl.n
        res = drain(srv, tickets)
        assert all(v["state"] == F.FMDDM_REQ_DONE for v in res.values()), res
        D_mix = {t: F.fmddm_server_poll(srv, t, mix[t])[1] for t in tickets}
        # the same requests again, one at a time on the same server
        for k, r in enumerate(reqs[::3]):
            t, wl = submit(srv, r)
            res1 = drain(srv, [t])[t]
            assert res1["state"] == F.FMDDM_REQ_DONE
            D1 = F.fmddm_server_poll(srv, t, wl.n)[1]
            D0 = D_mix[tickets[3 * k]]
            assert np.array_equal(D1, D0), float(np.max(np.abs(D1 - D0)))
            assert res1["iters"] == res[tickets[3 * k]]["iters"]
    finally:
        F.fmddm_server_destroy(srv)


@pytest.mark.parametrize("pc", [F.FMDDM_PRECOND_NONE, F.FMDDM_PRECOND_TWO_LEVEL])
def test_served_solution_satisfies_exact_system(pc):
    req = W.serving_stream(seed=11, count=1, nmin=600, nmax=600, steps_max=1)[0]
    req.steps = 3
    prm = F.fmddm_default_params(**P_SERVE, precond=pc, coarse_aggregates=128)
    srv = F.fmddm_server_create(prm, 2)
    try:
        tol = 1e-9
        t, wl = submit(srv, req, tol=tol)
        r = drain(srv, [t])[t]
        assert r["state"] == F.FMDDM_REQ_DONE and r["steps_done"] == 3
        D = F.fmddm_server_poll(srv, t, wl.n)[1]
    finally:
        F.fmddm_server_destroy(srv)
    g = O.Geometry.of(wl)
    b = O.rhs(g, wl.pressure, wl.SH, wl.Sh)
    res = O.direct_matvec(g, D) - b
    # requested tolerance plus the FMM error at p = 10 (well below 1e-6)
    assert np.linalg.norm(res) / np.linalg.norm(b) < 1e-6
    D_lu = O.lu_solve(O.dense_matrix(g), b)
    assert np.linalg.norm(D - D_lu) / np.linalg.norm(D_lu) < 1e-4


def test_admission_respects_budget():
    reqs = W.serving_stream(seed=13, count=4, nmin=3000, nmax=4000, steps_max=2)
    prm = F.fmddm_default_params(**P_SERVE)
    probe = F.fmddm_server_create(prm, 1)
    big = max(F.fmddm_server_footprint(probe, r.n) for r in reqs)
    F.fmddm_server_destroy(probe)
    budget = int(1.2 * big)  # room for one request at a time
    srv = F.fmddm_server_create(prm, 4, budget)
    try:
        tickets = [submit(srv, r)[0] for r in reqs]
        # a request that can never fit
        huge = W.serving_stream(seed=17, count=1, nmin=40000, nmax=40000)[0]
        assert F.fmddm_server_footprint(srv, huge.n) > budget
        t_huge = submit(srv, huge)[0]
        peak = [0]

        def watch():
            run = [F.fmddm_server_poll(srv, t)[0] for t in tickets]
            charged = sum(r["device_bytes"] for r in run if r["state"] == F.FMDDM_REQ_RUNNING)
            assert charged <= budget
            peak[0] = max(peak[0], sum(r["state"] == F.FMDDM_REQ_RUNNING for r in run))

        res = drain(srv, tickets + [t_huge], watch=watch)
        assert all(res[t]["state"] == F.FMDDM_REQ_DONE for t in tickets)
        assert res[t_huge]["state"] == F.FMDDM_REQ_FAILED and res[t_huge]["status"] == F.FMDDM_ENOMEM
        assert peak[0] == 1
    finally:
        F.fmddm_server_destroy(srv)


@pytest.mark.parametrize("pc", [F.FMDDM_PRECOND_NONE, F.FMDDM_PRECOND_TWO_LEVEL])
def test_footprint_estimate_covers_allocation(pc):
    prm = F.fmddm_default_params(**P_SERVE, precond=pc, coarse_aggregates=128)
    for seed, n in [(19, 1000), (23, 8000), (29, 30000)]:
        srv = F.fmddm_server_create(prm, 1)
        try:
            req = W.serving_stream(seed=seed, count=1, nmin=n, nmax=n, steps_max=1)[0]
            before = F.fmddm_memory_in_use()
            t, wl = submit(srv, req)
            peak = [0]

            def watch():  # the set-up runs on a host thread: watch the whole request
                peak[0] = max(peak[0], F.fmddm_memory_in_use() - before)

            drain(srv, [t], watch=watch)
            est = F.fmddm_server_footprint(srv, wl.n)
            assert 0 < peak[0] <= est, (wl.n, peak[0], est)
        finally:
            F.fmddm_server_destroy(srv)


def test_not_converged_request_fails_cleanly():
    prm = F.fmddm_default_params(**dict(P_SERVE, maxit=3))
    srv = F.fmddm_server_create(prm, 2)
    try:
        req = W.serving_stream(seed=31, count=1, nmin=800, nmax=800, steps_max=1)[0]
        t, _ = submit(srv, req, tol=1e-12)
        r = drain(srv, [t])[t]
        assert r["state"] == F.FMDDM_REQ_FAILED and r["status"] == F.FMDDM_ENOTCONV
        assert r["iters"] == 3
        # the slot is usable again
        t2, _ = submit(srv, req, tol=0.9)
        assert drain(srv, [t2])[t2]["state"] >= F.FMDDM_REQ_DONE
        assert F.fmddm_server_step(srv) == (0, 0)
    finally:
        F.fmddm_server_destroy(srv)


@pytest.mark.parametrize("prec", [F.FMDDM_PREC_FP32, F.FMDDM_PREC_BF16])
def test_served_mixed_precision_meets_tolerance(prec):
    """A server with reduced-precision products: each step's Arnoldi runs on
    them, residuals on the FP64 product, so the served DDs satisfy the
    oracle's exact system to the requested tolerance plus the FMM error,
    and agree with the FP64 server's."""
    req = W.serving_stream(seed=37, count=1, nmin=1500, nmax=1500, steps_max=1)[0]
    req.steps = 2
    out = {}
    for p in (F.FMDDM_PREC_FP64, prec):
        prm = F.fmddm_default_params(**P_SERVE, precision=p, precond=F.FMDDM_PRECOND_BLOCK)
        srv = F.fmddm_server_create(prm, 2)
        try:
            t, wl = submit(srv, req, tol=1e-8)
            r = drain(srv, [t])[t]
            assert r["state"] == F.FMDDM_REQ_DONE and r["relres"] <= 1e-8, r
            out[p] = F.fmddm_server_poll(srv, t, wl.n)[1]
        finally:
            F.fmddm_server_destroy(srv)
    g = O.Geometry.of(wl)
    b = O.rhs(g, wl.pressure, wl.SH, wl.Sh)
    res = np.linalg.norm(O.direct_matvec(g, out[prec]) - b) / np.linalg.norm(b)
    d = np.linalg.norm(out[prec] - out[F.FMDDM_PREC_FP64]) / np.linalg.norm(out[F.FMDDM_PREC_FP64])
    print(f"precision {prec}: exact residual {res:.2e}, vs FP64 server {d:.2e}")
    assert res <= 1e-6 and d <= 1e-6, (res, d)


def test_small_requests_on_exact_product():
    """Requests at or below direct_below elements are solved with the exact
    on-the-fly product: the served DDs satisfy the oracle's exact system to
    the requested tolerance itself (no FMM error), beside FMM requests."""
    reqs = W.serving_stream(seed=41, count=3, nmin=600, nmax=3000, steps_max=1)
    prm = F.fmddm_default_params(**P_SERVE, precond=F.FMDDM_PRECOND_BLOCK, direct_below=1500)
    srv = F.fmddm_server_create(prm, 3)
    try:
        subs = [submit(srv, r, tol=1e-9) for r in reqs]
        res = drain(srv, [t for t, _ in subs])
        for (t, wl) in subs:
            r = res[t]
            assert r["state"] == F.FMDDM_REQ_DONE and r["relres"] <= 1e-9, r
            D = F.fmddm_server_poll(srv, t, wl.n)[1]
            g = O.Geometry.of(wl)
            b = O.rhs(g, wl.pressure, wl.SH, wl.Sh)
            e = np.linalg.norm(O.direct_matvec(g, D) - b) / np.linalg.norm(b)
            bar = 1.01e-9 if wl.n <= 1500 else 1e-6   # exact product vs FMM
            print(f"n={wl.n}: exact residual {e:.2e}")
            assert e <= bar, (wl.n, e)
        assert any(wl.n <= 1500 for _, wl in subs) and any(wl.n > 1500 for _, wl in subs)
    finally:
        F.fmddm_server_destroy(srv)


# ------------------------------------------------------- poroelastic requests
MED = dict(nu_u=0.35, alpha=0.8, perm=1e-18, visc=1e-3, dt=60.0, p0=48.26e6)


def poro_server(slots, pc=F.FMDDM_PRECOND_TWO_LEVEL, m2l=F.FMDDM_M2L_DENSE, **kw):
    prm = F.fmddm_default_params(**dict(P_SERVE, E=20e9, nu=0.2, precond=pc, coarse_aggregates=128, **kw))
    srv = F.fmddm_server_create(prm, slots)
    F.fmddm_server_set_poro(srv, MED["nu_u"], MED["alpha"], MED["perm"], MED["visc"], MED["dt"], MED["p0"],
                            m2l=m2l)
    return srv


@pytest.mark.parametrize("m2l", [F.FMDDM_M2L_DENSE, F.FMDDM_M2L_SVD])
def test_poro_alone_equals_mix_bitwise(m2l):
    """Poroelastic time marches (1-3 steps of 60 s with the history sum):
    each request's DDs are the same alone and in the mix; with the
    compressed left-hand side too, whose operators the slots share per cell
    size (built by whichever request needs a size first)."""
    reqs = W.serving_stream(seed=43, count=6, nmin=500, nmax=3000, steps_max=3)
    srv = poro_server(4, m2l=m2l)
    try:
        tickets, sizes = [], {}
        for r in reqs:
            t, wl = submit(srv, r)
            tickets.append(t)
            sizes[t] = wl.n
        res = drain(srv, tickets, limit_s=300)
        assert all(v["state"] == F.FMDDM_REQ_DONE for v in res.values()), res
        for k in (0, 3, 5):
            t, wl = submit(srv, reqs[k])
            r1 = drain(srv, [t], limit_s=120)[t]
            assert r1["state"] == F.FMDDM_REQ_DONE and r1["steps_done"] == reqs[k].steps
            D1 = F.fmddm_server_poll(srv, t, wl.n, 3)[1]
            D0 = F.fmddm_server_poll(srv, tickets[k], sizes[tickets[k]], 3)[1]
            assert np.array_equal(D1, D0), float(np.max(np.abs(D1 - D0)))
            assert r1["iters"] == res[tickets[k]]["iters"]
    finally:
        F.fmddm_server_destroy(srv)


@pytest.mark.parametrize("m2l", [F.FMDDM_M2L_DENSE, F.FMDDM_M2L_SVD])
def test_poro_served_march_matches_oracle(m2l):
    """A served poroelastic request (3 steps) against the oracle's march on
    the exact operator (Gaussian elimination per step): GMRES at 1e-10 on
    the multipole operators (p = 10, ~1e-8 from the exact ones; compressed
    left-hand side at m2l_tol 1e-10 on a power-of-two root square) agrees to
    1e-5 of the largest entry of each unknown kind."""
    wl = W.random_fractures(47, n_frac=6, elems=20, box=20.0)
    po = O.Poro(E=20e9, nu=0.2, nuu=MED["nu_u"], alpha=MED["alpha"], perm=MED["perm"], visc=MED["visc"])
    g = O.Geometry(wl.x1, wl.y1, wl.x2, wl.y2, 20e9, 0.2)
    steps = 3
    ref, _, _ = O.poro_march(g, po, MED["dt"], steps, wl.pressure, MED["p0"], wl.SH, wl.Sh)
    srv = poro_server(2, m2l=m2l)
    try:
        t = F.fmddm_server_submit(srv, wl.x1, wl.y1, wl.x2, wl.y2, wl.pressure, wl.SH, wl.Sh, steps, 1e-10)
        r = drain(srv, [t], limit_s=120)[t]
        assert r["state"] == F.FMDDM_REQ_DONE and r["steps_done"] == steps, r
        D = F.fmddm_server_poll(srv, t, wl.n, 3)[1]
    finally:
        F.fmddm_server_destroy(srv)
    R = ref[steps - 1]
    for k in range(3):
        e = float(np.abs(D[k::3] - R[k::3]).max() / np.abs(R[k::3]).max())
        print(f"unknown {k}: {e:.2e}")
        assert e <= 1e-5, (k, e)


@pytest.mark.parametrize("m2l", [F.FMDDM_M2L_DENSE, F.FMDDM_M2L_SVD])
def test_poro_footprint_covers_allocation(m2l):
    for seed, n, steps in [(53, 1000, 3), (59, 8000, 10)]:
        srv = poro_server(1, m2l=m2l)
        try:
            req = W.serving_stream(seed=seed, count=1, nmin=n, nmax=n, steps_max=1)[0]
            req.steps = steps
            before = F.fmddm_memory_in_use()
            t, wl = submit(srv, req)
            peak = [0]

            def watch():  # set-up (operators, near blocks of all steps) and every step
                peak[0] = max(peak[0], F.fmddm_memory_in_use() - before)

            drain(srv, [t], limit_s=120, watch=watch)
            est = F.fmddm_server_poll(srv, t)[0]["device_bytes"]
            print(f"poro footprint n={wl.n} steps={steps}: peak {peak[0] / 2**20:.0f} MiB, estimate {est / 2**20:.0f} MiB")
            assert 0 < peak[0] <= est, (wl.n, peak[0], est)
        finally:
            F.fmddm_server_destroy(srv)


def test_poro_set_refused_while_busy():
    srv = poro_server(1)
    try:
        req = W.serving_stream(seed=61, count=1, nmin=600, nmax=600, steps_max=1)[0]
        t, _ = submit(srv, req)
        with pytest.raises(F.FmddmError):
            F.fmddm_server_set_poro(srv, MED["nu_u"], MED["alpha"], MED["perm"], MED["visc"], 30.0, MED["p0"])
        drain(srv, [t], limit_s=60)
        F.fmddm_server_set_poro(srv, MED["nu_u"], MED["alpha"], MED["perm"], MED["visc"], 30.0, MED["p0"])
    finally:
        F.fmddm_server_destroy(srv)
