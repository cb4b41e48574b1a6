"""The allocation-free FMM product (fmddm_apply_static) through the C ABI:
bit for bit the product of fmddm_apply's FMM mode, on two calls in a row
(the second on a smaller tree, which reuses the same static workspace),
and its refusals: a tree without set-up, a product larger than the
workspace, a reduced-precision context."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_1812_05087_amd as F  # noqa: E402


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def check_case(wl, seed, **kw):
    prob = F.Problem(wl.x1, wl.y1, wl.x2, wl.y2, E=wl.E, nu=wl.nu, **kw)
    try:
        D = prob.vec(W.random_vector(seed, wl.n))
        y = prob.apply(D, F.FMDDM_APPLY_FMM).cpu().numpy()       # builds schedules and operators
        out = torch.full_like(D, np.nan)
        F.fmddm_apply_static(prob.ctx, prob.tree, D, out)
        ys = out.cpu().numpy()
        assert np.all(np.isfinite(ys))
        assert rel(ys, y) <= 1e-12
        assert np.array_equal(ys, y)                              # same kernels, same order
        # a second product on the same tree, a different vector
        D2 = prob.vec(W.random_vector(seed + 1, wl.n))
        y2 = prob.apply(D2, F.FMDDM_APPLY_FMM).cpu().numpy()
        F.fmddm_apply_static(prob.ctx, prob.tree, D2, out)
        assert np.array_equal(out.cpu().numpy(), y2)
    finally:
        prob.close()


def test_static_product_equals_apply_then_smaller():
    # C2 at the benchmark configuration (p = 20, SVD M2L), then a smaller
    # tree (600 elements, dense M2L, p = 8) in the workspace the first left
    check_case(W.c2(), 5, leaf=32, p=20, m2l=F.FMDDM_M2L_SVD, m2l_tol=1e-12)
    check_case(W.random_fractures(7, 20, 30), 3, leaf=16, p=8)


def test_static_product_refusals():
    wl = W.random_fractures(7, 20, 30)
    prob = F.Problem(wl.x1, wl.y1, wl.x2, wl.y2, E=wl.E, nu=wl.nu, leaf=16, p=8)
    D = prob.vec(W.random_vector(3, wl.n))
    out = prob.vec()
    with pytest.raises(F.FmddmError) as e:        # no product has run on the tree yet
        F.fmddm_apply_static(prob.ctx, prob.tree, D, out)
    assert e.value.status == F.FMDDM_EINVAL
    with pytest.raises(F.FmddmError) as e:        # aliasing
        F.fmddm_apply_static(prob.ctx, prob.tree, D, D)
    assert e.value.status == F.FMDDM_EINVAL
    prob.close()
    # intermediates larger than the workspace: N = 200 000 at p = 10
    wl = W.c4()
    prob = F.Problem(wl.x1, wl.y1, wl.x2, wl.y2, E=wl.E, nu=wl.nu, leaf=64, p=10, m2l=F.FMDDM_M2L_SVD,
                     m2l_tol=1e-10)
    D = prob.vec(W.random_vector(9, wl.n))
    out = prob.vec()
    prob.apply(D, F.FMDDM_APPLY_FMM, out)
    with pytest.raises(F.FmddmError) as e:
        F.fmddm_apply_static(prob.ctx, prob.tree, D, out)
    assert e.value.status == F.FMDDM_EINVAL and "workspace" in str(e.value)
    prob.close()
    # reduced precision
    wl = W.random_fractures(7, 20, 30)
    prob = F.Problem(wl.x1, wl.y1, wl.x2, wl.y2, E=wl.E, nu=wl.nu, leaf=16, p=8, m2l=F.FMDDM_M2L_SVD,
                     precision=F.FMDDM_PREC_FP32)
    D = prob.vec(W.random_vector(3, wl.n))
    out = prob.vec()
    prob.apply(D, F.FMDDM_APPLY_FMM, out)
    with pytest.raises(F.FmddmError) as e:
        F.fmddm_apply_static(prob.ctx, prob.tree, D, out)
    assert e.value.status == F.FMDDM_EUNSUPPORTED
    prob.close()
