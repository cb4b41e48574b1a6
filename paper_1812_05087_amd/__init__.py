"""Python binding of the fmddm C ABI (include/fmddm.h).

Argument marshalling only: every step of the FMM/DDM path runs in the HIP
library ``libfmddm.so`` built from ``csrc/``.  PyTorch provides device memory
and the stream.  There is no CPU fallback: importing works without a GPU,
but any call needs the built library and a device, and fails loudly
otherwise.

Functions carry the C names (``fmddm_create``, ``fmddm_build_tree``,
``fmddm_apply``, ``fmddm_rhs``, ``fmddm_solve``, ``fmddm_sif``, ...).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfmddm.so")

FMDDM_OK, FMDDM_ENOTCONV = 0, 1
FMDDM_EINVAL, FMDDM_ENOMEM, FMDDM_EDEVICE, FMDDM_EGEOM, FMDDM_EUNSUPPORTED = -1, -2, -3, -4, -5
FMDDM_APPLY_FMM, FMDDM_APPLY_DIRECT, FMDDM_APPLY_DENSE = 0, 1, 2
FMDDM_M2L_DENSE, FMDDM_M2L_SVD = 0, 1
FMDDM_PREC_FP64, FMDDM_PREC_FP32, FMDDM_PREC_BF16 = 0, 1, 2
FMDDM_PRECOND_NONE, FMDDM_PRECOND_BLOCK, FMDDM_PRECOND_TWO_LEVEL = 0, 1, 2
LIST_U, LIST_V, LIST_W, LIST_X = 0, 1, 2, 3

EXPORTED = [
    "fmddm_default_params", "fmddm_create", "fmddm_destroy", "fmddm_last_error",
    "fmddm_build_tree", "fmddm_tree_free", "fmddm_tree_get_info", "fmddm_tree_export",
    "fmddm_tree_export_list", "fmddm_apply", "fmddm_apply_static", "fmddm_rhs", "fmddm_solve", "fmddm_sif",
    "fmddm_profile", "fmddm_profile_read",
    "fmddm_server_create", "fmddm_server_set_poro", "fmddm_server_destroy", "fmddm_server_last_error", "fmddm_server_footprint",
    "fmddm_server_submit", "fmddm_server_step", "fmddm_server_poll", "fmddm_server_release",
    "fmddm_memory_in_use", "fmddm_memory_cached", "fmddm_trim_cache",
    "fmddm_poro_set", "fmddm_poro_apply", "fmddm_add_history", "fmddm_poro_rhs", "fmddm_poro_solve",
    "fmddm_autotune", "fmddm_measure_peaks",
]
FMDDM_REQ_QUEUED, FMDDM_REQ_RUNNING, FMDDM_REQ_DONE, FMDDM_REQ_FAILED = 0, 1, 2, 3
PHASES = ["prep", "p2m", "m2m", "m2m_sum", "compress", "compress_sum", "m2l", "m2l_sum", "decompress",
          "l2p", "p2p", "final"]


class FmddmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"fmddm status {status}: {msg}")
        self.status = status


class Params(C.Structure):
    _fields_ = [
        ("E", C.c_double), ("nu", C.c_double),
        ("leaf", C.c_int), ("p", C.c_int), ("max_level", C.c_int),
        ("kappa", C.c_double), ("m2l", C.c_int), ("m2l_tol", C.c_double),
        ("use_root_box", C.c_int), ("root_x0", C.c_double), ("root_y0", C.c_double),
        ("root_L", C.c_double), ("restart", C.c_int), ("maxit", C.c_int), ("tol", C.c_double),
        ("precision", C.c_int), ("use_graphs", C.c_int), ("precond", C.c_int), ("m2l_tiles", C.c_int),
        ("direct_below", C.c_int64), ("coarse_aggregates", C.c_int32),
    ]


class TreeInfo(C.Structure):
    _fields_ = [
        ("n", C.c_int64), ("ncell", C.c_int64), ("nleaf", C.c_int64), ("nlevel", C.c_int32),
        ("nU", C.c_int64), ("nV", C.c_int64), ("nW", C.c_int64), ("nX", C.c_int64),
        ("near_pairs", C.c_int64), ("l2p_pairs", C.c_int64), ("m2m_pairs", C.c_int64),
        ("nfar", C.c_int64),
        ("m2l_rank", C.c_int64),
        ("root_x0", C.c_double), ("root_y0", C.c_double), ("root_L", C.c_double),
        ("device_bytes", C.c_int64), ("m2m_launches", C.c_int64), ("m2m_cut", C.c_int32),
        ("poro_m2l_rank", C.c_int32),
    ]


class Request(C.Structure):
    _fields_ = [("n", C.c_int64), ("x1", C.c_void_p), ("y1", C.c_void_p), ("x2", C.c_void_p),
                ("y2", C.c_void_p), ("pf", C.c_void_p), ("SH", C.c_double), ("Sh", C.c_double),
                ("steps", C.c_int32), ("tol", C.c_double)]


class Result(C.Structure):
    _fields_ = [("state", C.c_int32), ("status", C.c_int32), ("steps_done", C.c_int32),
                ("iters", C.c_int32), ("relres", C.c_double), ("t_submit", C.c_double),
                ("t_admit", C.c_double), ("t_done", C.c_double), ("device_bytes", C.c_int64)]


class PoroParams(C.Structure):
    _fields_ = [("nu_u", C.c_double), ("alpha", C.c_double), ("perm", C.c_double), ("visc", C.c_double),
                ("dt", C.c_double), ("p0", C.c_double), ("mode", C.c_int32), ("near_cache_bytes", C.c_int64),
                ("m2l", C.c_int32), ("exact_far_levels", C.c_int32)]


class Peaks(C.Structure):
    _fields_ = [("fp64_vector_tflops", C.c_double), ("fp64_mfma_tflops", C.c_double), ("copy_gbps", C.c_double)]


class TuneEntry(C.Structure):
    _fields_ = [("leaf", C.c_int32), ("p", C.c_int32), ("ms", C.c_double), ("err", C.c_double),
                ("m2l_tiles", C.c_int32)]


class SolveInfo(C.Structure):
    _fields_ = [("iters", C.c_int32), ("restarts", C.c_int32), ("relres", C.c_double),
                ("converged", C.c_int32), ("refinements", C.c_int32)]


_lib = None
_vp = C.c_void_p
_d = C.POINTER(C.c_double)


def lib():
    """Load libfmddm.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run paper_1812_05087_amd/build.py "
                               "(or __graft_entry__.build()) first; there is no fallback")
        # PyTorch's HIP runtime is loaded first, so that the library binds
        # to the same one (a second runtime in the process would leave
        # torch without devices)
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        L.fmddm_default_params.argtypes = [C.POINTER(Params)]
        L.fmddm_default_params.restype = None
        L.fmddm_create.argtypes = [C.POINTER(Params), _vp, C.POINTER(_vp)]
        L.fmddm_destroy.argtypes = [_vp]
        L.fmddm_destroy.restype = None
        L.fmddm_last_error.argtypes = [_vp]
        L.fmddm_last_error.restype = C.c_char_p
        L.fmddm_build_tree.argtypes = [_vp, C.c_int64, _vp, _vp, _vp, _vp, C.c_int, C.POINTER(_vp)]
        L.fmddm_tree_free.argtypes = [_vp]
        L.fmddm_tree_free.restype = None
        L.fmddm_tree_get_info.argtypes = [_vp, _vp, C.POINTER(TreeInfo)]
        L.fmddm_tree_export.argtypes = [_vp, _vp] + [_vp] * 11
        L.fmddm_tree_export_list.argtypes = [_vp, _vp, C.c_int, _vp, _vp]
        L.fmddm_apply.argtypes = [_vp, _vp, C.c_int, _vp, _vp]
        L.fmddm_apply_static.argtypes = [_vp, _vp, _vp, _vp]
        L.fmddm_rhs.argtypes = [_vp, _vp, _vp, C.c_double, C.c_double, _vp]
        L.fmddm_solve.argtypes = [_vp, _vp, C.c_int, _vp, _vp, C.POINTER(SolveInfo)]
        L.fmddm_sif.argtypes = [_vp, _vp, _vp, C.c_int64, _d, _d]
        L.fmddm_profile.argtypes = [_vp, C.c_uint]
        L.fmddm_profile_read.argtypes = [_vp, _d, C.POINTER(C.c_int64)]
        L.fmddm_server_create.argtypes = [C.POINTER(Params), C.c_int, C.c_int64, C.POINTER(_vp)]
        L.fmddm_server_destroy.argtypes = [_vp]
        L.fmddm_server_destroy.restype = None
        L.fmddm_server_last_error.argtypes = [_vp]
        L.fmddm_server_last_error.restype = C.c_char_p
        L.fmddm_server_footprint.argtypes = [_vp, C.c_int64]
        L.fmddm_server_footprint.restype = C.c_int64
        L.fmddm_server_submit.argtypes = [_vp, C.POINTER(Request), C.POINTER(C.c_int64)]
        L.fmddm_server_step.argtypes = [_vp, C.POINTER(C.c_int), C.POINTER(C.c_int)]
        L.fmddm_server_poll.argtypes = [_vp, C.c_int64, C.POINTER(Result), _vp]
        L.fmddm_server_release.argtypes = [_vp, C.c_int64]
        for name in ("fmddm_memory_in_use", "fmddm_memory_cached", "fmddm_trim_cache"):
            getattr(L, name).argtypes = []
        L.fmddm_poro_set.argtypes = [_vp, C.POINTER(PoroParams)]
        L.fmddm_server_set_poro.argtypes = [_vp, C.POINTER(PoroParams)]
        L.fmddm_poro_apply.argtypes = [_vp, _vp, C.c_int, _vp, _vp]
        L.fmddm_add_history.argtypes = [_vp, _vp, C.c_int, _vp, _vp]
        L.fmddm_poro_rhs.argtypes = [_vp, _vp, _vp, C.c_double, C.c_double, _vp]
        L.fmddm_poro_solve.argtypes = [_vp, _vp, _vp, _vp, C.POINTER(SolveInfo)]
        L.fmddm_measure_peaks.argtypes = [C.POINTER(Peaks)]
        L.fmddm_autotune.argtypes = [C.POINTER(Params), C.c_int64, _vp, _vp, _vp, _vp, _vp, C.c_int32, _vp,
                                     C.c_int32, C.c_double, C.c_int32, C.POINTER(Params), _vp, C.c_int32,
                                     C.POINTER(C.c_int32)]
        for name in EXPORTED:
            f = getattr(L, name)
            if name not in ("fmddm_default_params", "fmddm_destroy", "fmddm_tree_free",
                            "fmddm_last_error", "fmddm_server_destroy", "fmddm_server_last_error",
                            "fmddm_server_footprint", "fmddm_memory_in_use", "fmddm_memory_cached",
                            "fmddm_trim_cache"):
                f.restype = C.c_int
        for name in ("fmddm_memory_in_use", "fmddm_memory_cached", "fmddm_trim_cache"):
            getattr(L, name).restype = C.c_int64
        _lib = L
    return _lib


def _check(st, ctx=None):
    if st < 0:
        msg = lib().fmddm_last_error(ctx).decode() if ctx else ""
        raise FmddmError(st, msg)
    return st


def _ptr(t):
    """Device pointer of a contiguous CUDA/HIP float64 tensor."""
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a device (cuda) tensor")
    if t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError("expected a contiguous float64 tensor")
    return C.c_void_p(t.data_ptr())


# ----------------------------------------------------------- C-ABI wrappers
def fmddm_default_params(**kw) -> Params:
    p = Params()
    lib().fmddm_default_params(C.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise AttributeError(k)
        setattr(p, k, v)
    return p


def fmddm_create(params: Params, stream=None):
    """stream: a torch.cuda.Stream, a raw hipStream_t int, or None (the
    current torch stream)."""
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    raw = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
    out = C.c_void_p()
    _check(lib().fmddm_create(C.byref(params), C.c_void_p(raw), C.byref(out)))
    return out


def fmddm_destroy(ctx):
    lib().fmddm_destroy(ctx)


def fmddm_last_error(ctx) -> str:
    return lib().fmddm_last_error(ctx).decode()


def fmddm_build_tree(ctx, x1, y1, x2, y2):
    """Endpoints as numpy arrays (host) or float64 device tensors."""
    out = C.c_void_p()
    if isinstance(x1, np.ndarray):
        arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (x1, y1, x2, y2)]
        ptrs = [C.c_void_p(a.ctypes.data) for a in arrs]
        n, dev = arrs[0].shape[0], 0
    else:
        ptrs = [_ptr(a) for a in (x1, y1, x2, y2)]
        n, dev = x1.shape[0], 1
    _check(lib().fmddm_build_tree(ctx, n, *ptrs, dev, C.byref(out)), ctx)
    return out


def fmddm_tree_free(tree):
    lib().fmddm_tree_free(tree)


def fmddm_tree_get_info(ctx, tree) -> dict:
    info = TreeInfo()
    _check(lib().fmddm_tree_get_info(ctx, tree, C.byref(info)), ctx)
    return {k: getattr(info, k) for k, _ in TreeInfo._fields_}


def fmddm_tree_export(ctx, tree) -> dict:
    info = fmddm_tree_get_info(ctx, tree)
    n, nc = info["n"], info["ncell"]
    out = {
        "perm": np.zeros(n, np.int64), "key": np.zeros(n, np.uint64),
        "level": np.zeros(nc, np.int32), "ix": np.zeros(nc, np.uint32), "iy": np.zeros(nc, np.uint32),
        "parent": np.zeros(nc, np.int32), "child": np.zeros((nc, 4), np.int32),
        "pbeg": np.zeros(nc, np.int64), "pend": np.zeros(nc, np.int64),
        "isleaf": np.zeros(nc, np.int32), "root": np.zeros(3),
    }
    order = ["perm", "key", "level", "ix", "iy", "parent", "child", "pbeg", "pend", "isleaf", "root"]
    _check(lib().fmddm_tree_export(ctx, tree, *[C.c_void_p(out[k].ctypes.data) for k in order]), ctx)
    return out


def fmddm_tree_export_list(ctx, tree, which):
    info = fmddm_tree_get_info(ctx, tree)
    nc = info["ncell"]
    off = np.zeros(nc + 1, np.int64)
    _check(lib().fmddm_tree_export_list(ctx, tree, which, C.c_void_p(off.ctypes.data), None), ctx)
    idx = np.zeros(max(int(off[-1]), 1), np.int32)
    _check(lib().fmddm_tree_export_list(ctx, tree, which, C.c_void_p(off.ctypes.data),
                                        C.c_void_p(idx.ctypes.data)), ctx)
    return off, idx[:int(off[-1])]


def fmddm_apply(ctx, tree, mode, D, out):
    return _check(lib().fmddm_apply(ctx, tree, mode, _ptr(D), _ptr(out)), ctx)


def fmddm_apply_static(ctx, tree, D, out):
    """The FMM product in the library's static device workspace (allocates
    nothing); the tree must have run one fmddm_apply FMM product."""
    _check(lib().fmddm_apply_static(ctx, tree, _ptr(D), _ptr(out)), ctx)


def fmddm_rhs(ctx, tree, pf, SH, Sh, rhs):
    return _check(lib().fmddm_rhs(ctx, tree, _ptr(pf), float(SH), float(Sh), _ptr(rhs)), ctx)


def fmddm_solve(ctx, tree, mode, rhs, D):
    info = SolveInfo()
    st = _check(lib().fmddm_solve(ctx, tree, mode, _ptr(rhs), _ptr(D), C.byref(info)), ctx)
    return st, {"iters": info.iters, "restarts": info.restarts, "relres": info.relres,
                "converged": bool(info.converged), "refinements": info.refinements}


def fmddm_autotune(params: Params, x1, y1, x2, y2, leaves=(16, 32, 64, 128), ps=tuple(range(8, 25, 2)),
                   target_err=1e-6, reps=10):
    """Returns (status, best Params, [TuneEntry as dict, ...])."""
    x1, y1, x2, y2 = (np.ascontiguousarray(v, dtype=np.float64) for v in (x1, y1, x2, y2))
    lv = (C.c_int32 * len(leaves))(*leaves)
    pv = (C.c_int32 * len(ps))(*ps)
    cap = len(leaves) * len(ps) + 4
    log = (TuneEntry * cap)()
    nlog = C.c_int32()
    best = Params()
    dp = lambda a: a.ctypes.data_as(C.c_void_p)
    st = lib().fmddm_autotune(C.byref(params), int(x1.shape[0]), dp(x1), dp(y1), dp(x2), dp(y2), lv,
                              len(leaves), pv, len(ps), float(target_err), int(reps), C.byref(best), log,
                              cap, C.byref(nlog))
    if st < 0:
        raise FmddmError(st, "autotune failed")
    return st, best, [{k: getattr(log[i], k) for k, _ in TuneEntry._fields_} for i in range(nlog.value)]


def fmddm_measure_peaks():
    p = Peaks()
    st = lib().fmddm_measure_peaks(C.byref(p))
    if st < 0:
        raise FmddmError(st, "peak measurement failed")
    return {k: getattr(p, k) for k, _ in Peaks._fields_}


def fmddm_sif(ctx, tree, D, elem):
    KI, KII = C.c_double(), C.c_double()
    _check(lib().fmddm_sif(ctx, tree, _ptr(D), int(elem), C.byref(KI), C.byref(KII)), ctx)
    return KI.value, KII.value


def fmddm_profile(ctx, mask):
    return _check(lib().fmddm_profile(ctx, int(mask)), ctx)


def fmddm_profile_read(ctx):
    """{phase: (total_ms, launches)} since the previous read."""
    ms = (C.c_double * len(PHASES))()
    cnt = (C.c_int64 * len(PHASES))()
    _check(lib().fmddm_profile_read(ctx, ms, cnt), ctx)
    return {PHASES[i]: (ms[i], cnt[i]) for i in range(len(PHASES))}


# --------------------------------------------------------------- convenience
class Problem:
    """A context plus a tree over one geometry, with device buffers."""

    def __init__(self, x1, y1, x2, y2, device="cuda:0", **params):
        import torch
        self.device = torch.device(device)
        torch.cuda.set_device(self.device)
        self.params = fmddm_default_params(**params)
        self.ctx = fmddm_create(self.params)
        self.tree = fmddm_build_tree(self.ctx, np.asarray(x1), np.asarray(y1),
                                     np.asarray(x2), np.asarray(y2))
        self.info = fmddm_tree_get_info(self.ctx, self.tree)
        self.n = self.info["n"]

    def vec(self, data=None):
        import torch
        if data is None:
            return torch.zeros(2 * self.n, dtype=torch.float64, device=self.device)
        return torch.as_tensor(np.ascontiguousarray(data, dtype=np.float64)).to(self.device)

    def apply(self, D, mode=FMDDM_APPLY_FMM, out=None):
        out = self.vec() if out is None else out
        fmddm_apply(self.ctx, self.tree, mode, D, out)
        return out

    def rhs(self, pf, SH, Sh):
        import torch
        pf = torch.as_tensor(np.ascontiguousarray(pf, dtype=np.float64)).to(self.device)
        out = self.vec()
        fmddm_rhs(self.ctx, self.tree, pf, SH, Sh, out)
        return out

    def solve(self, rhs, mode=FMDDM_APPLY_FMM, x0=None):
        x = self.vec() if x0 is None else x0.clone()
        st, info = fmddm_solve(self.ctx, self.tree, mode, rhs, x)
        info["status"] = st
        return x, info

    def close(self):
        if getattr(self, "tree", None):
            fmddm_tree_free(self.tree)
            self.tree = None
        if getattr(self, "ctx", None):
            fmddm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------ serving
def _scheck(st, srv):
    if st < 0:
        raise FmddmError(st, lib().fmddm_server_last_error(srv).decode())
    return st


def fmddm_server_create(params: Params, max_slots: int, hbm_budget: int = 0):
    out = _vp()
    st = lib().fmddm_server_create(C.byref(params), int(max_slots), int(hbm_budget), C.byref(out))
    if st < 0:
        raise FmddmError(st, "server creation failed")
    return out


def fmddm_server_destroy(srv):
    lib().fmddm_server_destroy(srv)


def fmddm_server_footprint(srv, n: int) -> int:
    return int(lib().fmddm_server_footprint(srv, int(n)))


def fmddm_server_submit(srv, x1, y1, x2, y2, pf, SH, Sh, steps, tol) -> int:
    arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (x1, y1, x2, y2, pf)]
    n = arrs[0].size
    if any(a.size != n for a in arrs):
        raise ValueError("geometry and pressure arrays must have the same length")
    r = Request(n, *[a.ctypes.data for a in arrs], float(SH), float(Sh), int(steps), float(tol))
    t = C.c_int64()
    _scheck(lib().fmddm_server_submit(srv, C.byref(r), C.byref(t)), srv)
    return t.value


def fmddm_server_step(srv):
    a, q = C.c_int(), C.c_int()
    _scheck(lib().fmddm_server_step(srv, C.byref(a), C.byref(q)), srv)
    return a.value, q.value


def fmddm_server_poll(srv, ticket: int, n: int = 0, comps: int = 2):
    """(result dict, D or None); D (host, comps x n: 2 on elastic servers,
    3 on poroelastic ones) once the request is done."""
    r = Result()
    D = np.empty(comps * n) if n else None
    _scheck(lib().fmddm_server_poll(srv, int(ticket), C.byref(r),
                                    C.c_void_p(D.ctypes.data) if D is not None else None), srv)
    res = {k: getattr(r, k) for k, _ in Result._fields_}
    return res, (D if res["state"] == FMDDM_REQ_DONE else None)


def fmddm_server_set_poro(srv, nu_u, alpha, perm, visc, dt, p0=0.0, near_cache_bytes=0, m2l=0):
    """Poroelastic medium for every later request (time marches with the
    multipole form, FMDDM_APPLY_FMM)."""
    pp = PoroParams(float(nu_u), float(alpha), float(perm), float(visc), float(dt), float(p0), FMDDM_APPLY_FMM,
                    int(near_cache_bytes), int(m2l), 0)
    _scheck(lib().fmddm_server_set_poro(srv, C.byref(pp)), srv)


def fmddm_server_release(srv, ticket: int):
    _scheck(lib().fmddm_server_release(srv, int(ticket)), srv)


def fmddm_memory_in_use() -> int:
    return int(lib().fmddm_memory_in_use())


def fmddm_memory_cached() -> int:
    return int(lib().fmddm_memory_cached())


def fmddm_trim_cache() -> int:
    return int(lib().fmddm_trim_cache())


# ------------------------------------------------------------ poroelastic
def fmddm_poro_set(ctx, nu_u, alpha, perm, visc, dt, p0=0.0, mode=1, near_cache_bytes=0, m2l=0,
                   exact_far_levels=0):
    """mode: FMDDM_APPLY_DIRECT (1, exact), FMDDM_APPLY_FMM (0) or
    FMDDM_APPLY_DENSE (2, history-only).  near_cache_bytes: FMM near-field
    cache budget (0 default, < 0 none).  m2l: FMDDM_M2L_DENSE (0) or
    FMDDM_M2L_SVD (1, the left-hand side's M2L compressed per cell size).
    exact_far_levels: 1 keeps one far-field term per time level in history
    sums (0: two terms where the far field is affine in time)."""
    pp = PoroParams(float(nu_u), float(alpha), float(perm), float(visc), float(dt), float(p0), int(mode),
                    int(near_cache_bytes), int(m2l), int(exact_far_levels))
    _check(lib().fmddm_poro_set(ctx, C.byref(pp)), ctx)


def fmddm_poro_apply(ctx, tree, lag, D, out):
    _check(lib().fmddm_poro_apply(ctx, tree, int(lag), _ptr(D), _ptr(out)), ctx)


def fmddm_add_history(ctx, tree, h, Dhist, rhs):
    """rhs -= sum_{k=1}^{h-1} K_{h-k} D^k; Dhist: device tensor holding
    D^1..D^{h-1} consecutively (or None when h == 1)."""
    dh = _ptr(Dhist) if Dhist is not None else None
    _check(lib().fmddm_add_history(ctx, tree, int(h), dh, _ptr(rhs)), ctx)


def fmddm_poro_rhs(ctx, tree, pf, SH, Sh, rhs):
    _check(lib().fmddm_poro_rhs(ctx, tree, _ptr(pf), float(SH), float(Sh), _ptr(rhs)), ctx)


def fmddm_poro_solve(ctx, tree, rhs, D):
    info = SolveInfo()
    st = _check(lib().fmddm_poro_solve(ctx, tree, _ptr(rhs), _ptr(D), C.byref(info)), ctx)
    return st, {k: getattr(info, k) for k, _ in SolveInfo._fields_}
