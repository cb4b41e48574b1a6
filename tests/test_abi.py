"""CPU-side checks of the C-ABI library: it loads, exports every function
declared in include/fmddm.h, and validates arguments before touching a
device.  No compute calls (there is no GPU here)."""
import ctypes as C
import os
import re

import pytest

import paper_1812_05087_amd as F

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fmddm.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fmddm_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    if not os.path.exists(F.LIB_PATH):
        pytest.skip("library not built")
    lib = C.CDLL(F.LIB_PATH)
    names = declared_functions()
    assert len(names) >= 13
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(F.EXPORTED) == names


def test_struct_layouts_match_header():
    """The ctypes mirrors of the public structs have the sizes the C
    compiler gives them (computed from the header by gcc)."""
    import subprocess
    import tempfile
    src = '#include "fmddm.h"\n#include <stdio.h>\nint main(){printf("%zu %zu %zu %zu %zu %zu %zu\\n",' \
          'sizeof(fmddm_params),sizeof(fmddm_tree_info),sizeof(fmddm_solve_info),' \
          'sizeof(fmddm_request),sizeof(fmddm_result),sizeof(fmddm_poro_params),' \
          'sizeof(fmddm_tune_entry));printf("%zu\\n",sizeof(fmddm_peaks));return 0;}\n'
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "s.c")
        open(c, "w").write(src)
        exe = os.path.join(d, "s")
        subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe])
        sizes = list(map(int, subprocess.check_output([exe]).split()))
    assert sizes == [C.sizeof(F.Params), C.sizeof(F.TreeInfo), C.sizeof(F.SolveInfo),
                     C.sizeof(F.Request), C.sizeof(F.Result), C.sizeof(F.PoroParams),
                     C.sizeof(F.TuneEntry), C.sizeof(F.Peaks)]


def test_default_params_and_validation_without_device():
    if not os.path.exists(F.LIB_PATH):
        pytest.skip("library not built")
    p = F.fmddm_default_params()
    assert (p.leaf, p.p, p.max_level, p.restart, p.use_graphs, p.precond, p.precision) == (32, 20, 24, 50, 0, 0, 0)
    assert p.E == 20e9 and p.nu == 0.25 and p.kappa == 8.0 and p.tol == 1e-10
    lib = F.lib()
    out = C.c_void_p()
    for field, bad in [("p", 0), ("p", 33), ("leaf", 0), ("nu", 0.5), ("E", -1.0),
                       ("max_level", 31), ("restart", 0), ("tol", -1.0), ("precision", 3),
                       ("precision", -1), ("use_graphs", 2), ("precond", 3), ("precond", -1), ("coarse_aggregates", -1), ("coarse_aggregates", 4096)]:
        q = F.fmddm_default_params(**{field: bad})
        assert lib.fmddm_create(C.byref(q), None, C.byref(out)) == F.FMDDM_EINVAL, field
        assert not out.value
    assert lib.fmddm_create(None, None, C.byref(out)) == F.FMDDM_EINVAL
    # null-handle calls are rejected, not crashed
    assert lib.fmddm_apply(None, None, 0, None, None) == F.FMDDM_EINVAL
    assert lib.fmddm_solve(None, None, 0, None, None, None) == F.FMDDM_EINVAL
    assert lib.fmddm_build_tree(None, 1, None, None, None, None, 0, C.byref(out)) == F.FMDDM_EINVAL
    lib.fmddm_destroy(None)
    lib.fmddm_tree_free(None)
    # server entry points: invalid arguments are rejected before any device work
    p = F.fmddm_default_params()
    for slots, budget in [(0, 0), (65, 0), (4, -1)]:
        assert lib.fmddm_server_create(C.byref(p), slots, budget, C.byref(out)) == F.FMDDM_EINVAL
        assert not out.value
    t = C.c_int64()
    a = C.c_int()
    assert lib.fmddm_server_submit(None, None, C.byref(t)) == F.FMDDM_EINVAL
    assert lib.fmddm_server_step(None, C.byref(a), C.byref(a)) == F.FMDDM_EINVAL
    assert lib.fmddm_server_poll(None, 1, None, None) == F.FMDDM_EINVAL
    assert lib.fmddm_server_release(None, 1) == F.FMDDM_EINVAL
    assert lib.fmddm_server_footprint(None, 100) == 0
    lib.fmddm_server_destroy(None)
    assert lib.fmddm_poro_set(None, None) == F.FMDDM_EINVAL
    assert lib.fmddm_poro_apply(None, None, 0, None, None) == F.FMDDM_EINVAL
    assert lib.fmddm_add_history(None, None, 2, None, None) == F.FMDDM_EINVAL
    assert lib.fmddm_poro_rhs(None, None, None, 0.0, 0.0, None) == F.FMDDM_EINVAL
    assert lib.fmddm_poro_solve(None, None, None, None, None) == F.FMDDM_EINVAL
    # autotuner: argument checks come first
    best = F.Params()
    x = (C.c_double * 4)(0.0, 1.0, 2.0, 3.0)
    lv = (C.c_int32 * 2)(16, 32)
    pv = (C.c_int32 * 2)(8, 10)
    args = [C.byref(p), 2, x, x, x, x, lv, 2, pv, 2, 1e-6, 3, C.byref(best), None, 0, None]
    for i, bad in [(0, None), (2, None), (6, None), (7, 0), (9, 0), (10, 0.0), (11, 0), (12, None),
                   (14, 4)]:
        a2 = list(args)
        a2[i] = bad
        assert lib.fmddm_autotune(*a2) == F.FMDDM_EINVAL, i
    assert lib.fmddm_measure_peaks(None) == F.FMDDM_EINVAL
    bad_p = (C.c_int32 * 2)(8, 33)
    a2 = list(args)
    a2[8] = bad_p
    assert lib.fmddm_autotune(*a2) == F.FMDDM_EINVAL


def test_binding_refuses_host_tensors():
    torch = pytest.importorskip("torch")
    with pytest.raises(TypeError):
        F._ptr(torch.zeros(4, dtype=torch.float64))
