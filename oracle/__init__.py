"""Oracle: plain FP64 CPU reference for the fast-multipole DDM.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  The product
library (``paper_1812_05087_amd``) never imports, links or calls it, and the
two share no code; the only common module is ``workloads`` (seeded inputs).

The arithmetic lives in ``fmddm_oracle.c`` (plain C, no FMA contraction);
this file only marshals numpy arrays through ctypes.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fmddm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

LIST_U, LIST_V, LIST_W, LIST_X = 0, 1, 2, 3
KAPPA = 8.0          # children at least KAPPA element half-lengths wide
MAX_LEVEL = 24       # default level cap of the tree


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, no FMA contraction)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math",
               "-fopenmp", "-fPIC", "-shared", _SRC, "-o", _LIB + ".tmp", "-lm"]
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None
_d = C.POINTER(C.c_double)
_i64 = C.POINTER(C.c_int64)
_i32 = C.POINTER(C.c_int32)
_u32 = C.POINTER(C.c_uint32)
_u64 = C.POINTER(C.c_uint64)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = C.CDLL(_LIB)
        L.ora_elem_stress.argtypes = [C.c_double] * 11 + [_d]
        L.ora_point_kernel.argtypes = [C.c_double] * 4 + [_d]
        L.ora_charge.argtypes = [C.c_double] * 4 + [_d]
        L.ora_traction.argtypes = [C.c_double, C.c_double, _d, _d, _d]
        L.ora_gauss_legendre.argtypes = [C.c_int, _d, _d]
        L.ora_cheb_nodes.argtypes = [C.c_int, _d]
        L.ora_cheb_S.argtypes = [C.c_int, C.c_int, C.c_double]
        L.ora_cheb_S.restype = C.c_double
        L.ora_dense_matrix.argtypes = [C.c_int64] + [_d] * 5 + [C.c_double] * 2 + [_d]
        L.ora_dense_matrix_poly.argtypes = [C.c_int64] + [_d] * 5 + [_d]
        L.ora_dense_matvec.argtypes = [C.c_int64, _d, _d, _d]
        L.ora_direct_matvec.argtypes = [C.c_int64] + [_d] * 5 + [C.c_double] * 2 + [_d, _d]
        L.ora_direct_matvec_rows.argtypes = ([C.c_int64] + [_d] * 5 + [C.c_double] * 2
                                             + [_d, _d, C.c_int64, C.c_int64])
        L.ora_direct_matvec_idx.argtypes = ([C.c_int64] + [_d] * 5 + [C.c_double] * 2
                                            + [_d, C.c_int64, _i64, _d])
        L.ora_lu_solve.argtypes = [C.c_int64, _d, _d, _d]
        L.ora_gmres_dense.argtypes = [C.c_int64, _d, _d, _d, C.c_int, C.c_double, C.c_int,
                                      C.POINTER(C.c_int), _d]
        L.ora_gmres_direct.argtypes = ([C.c_int64] + [_d] * 5 + [C.c_double] * 2 +
                                       [_d, _d, C.c_int, C.c_double, C.c_int,
                                        C.POINTER(C.c_int), _d])
        L.ora_rhs.argtypes = [C.c_int64, _d, _d, _d, C.c_double, C.c_double, _d]
        L.ora_sif.argtypes = [C.c_double] * 5 + [_d, _d]
        L.ora_tree_build.argtypes = ([C.c_int64, _d, _d, _d, C.c_int, C.c_int, C.c_double,
                                      C.c_int, C.c_double, C.c_double, C.c_double])
        L.ora_tree_build.restype = C.c_void_p
        L.ora_tree_ncell.argtypes = [C.c_void_p]
        L.ora_tree_ncell.restype = C.c_int64
        L.ora_tree_export.argtypes = [C.c_void_p, _i64, _u64, _i32, _u32, _u32, _i32, _i32,
                                      _i64, _i64, _i32, _d]
        L.ora_tree_free.argtypes = [C.c_void_p]
        L.ora_lists_build.argtypes = [C.c_void_p]
        L.ora_list_size.argtypes = [C.c_void_p, C.c_int]
        L.ora_list_size.restype = C.c_int64
        L.ora_list_export.argtypes = [C.c_void_p, C.c_int, _i64, _i32]
        L.ora_fmm_apply.argtypes = ([C.c_void_p] + [_d] * 5 + [C.c_double] * 2 +
                                    [C.c_int, C.c_int, _d, _d])
        L.ora_fmm_apply.restype = C.c_int
        L.ora_set_num_threads.argtypes = [C.c_int]
        L.ora_poro_consts.argtypes = [C.c_double] * 6 + [_d]
        L.ora_E1.argtypes = [C.c_double]
        L.ora_E1.restype = C.c_double
        L.ora_poro_point_transient.argtypes = [_d] + [C.c_double] * 3 + [_d, C.c_double, _d]
        L.ora_poro_point.argtypes = [_d] + [C.c_double] * 3 + [_d, C.c_double, _d]
        L.ora_poro_elem_transient.argtypes = ([_d] + [C.c_double] * 12 + [C.c_int, C.c_int, _d])
        L.ora_poro_matrix.argtypes = ([C.c_int64] + [_d] * 5 + [_d, C.c_double, C.c_int,
                                                               C.c_int, C.c_int, _d])
        L.ora_poro_matrix_rows.argtypes = ([C.c_int64] + [_d] * 5 + [_d, C.c_double, C.c_int, C.c_int, C.c_int,
                                                                    C.c_int64, _i64, _d])
        _lib = L
    return _lib


def _p(arr, ty=_d):
    return arr.ctypes.data_as(ty)


def _f64(x):
    return np.ascontiguousarray(x, dtype=np.float64)


# --------------------------------------------------------------------------
# geometry
# --------------------------------------------------------------------------
class Geometry:
    """Element midpoints, orientation and half-lengths from endpoints."""

    def __init__(self, x1, y1, x2, y2, E=20e9, nu=0.25):
        x1, y1, x2, y2 = map(_f64, (x1, y1, x2, y2))
        self.cx = _f64(0.5 * (x1 + x2))
        self.cy = _f64(0.5 * (y1 + y2))
        dx, dy = x2 - x1, y2 - y1
        # separately rounded squares, sum and square root (the device path
        # computes the half-length, which decides tree splits, the same way)
        ln = np.sqrt(dx * dx + dy * dy)
        self.cb = _f64(dx / ln)
        self.sb = _f64(dy / ln)
        self.a = _f64(0.5 * ln)
        self.E, self.nu = float(E), float(nu)
        self.G = self.E / (2.0 * (1.0 + self.nu))
        self.n = int(self.cx.shape[0])

    @classmethod
    def of(cls, wl):
        return cls(wl.x1, wl.y1, wl.x2, wl.y2, wl.E, wl.nu)

    def args(self):
        return (_p(self.cx), _p(self.cy), _p(self.cb), _p(self.sb), _p(self.a))


# --------------------------------------------------------------------------
# kernels
# --------------------------------------------------------------------------
def elem_stress(X, Y, cx, cy, cb, sb, a, G, nu, Ds, Dn):
    out = np.zeros(3)
    lib().ora_elem_stress(X, Y, cx, cy, cb, sb, a, G, nu, Ds, Dn, _p(out))
    return out


def point_kernel(x, y, G, nu):
    out = np.zeros(9)
    lib().ora_point_kernel(x, y, G, nu, _p(out))
    return out.reshape(3, 3)


def charge(cb, sb, Ds, Dn):
    out = np.zeros(3)
    lib().ora_charge(cb, sb, Ds, Dn, _p(out))
    return out


def traction(cb, sb, sg):
    sg = _f64(sg)
    ts, tn = C.c_double(), C.c_double()
    lib().ora_traction(cb, sb, _p(sg), C.byref(ts), C.byref(tn))
    return ts.value, tn.value


def gauss_legendre(n):
    t, w = np.zeros(n), np.zeros(n)
    lib().ora_gauss_legendre(n, _p(t), _p(w))
    return t, w


def cheb_nodes(p):
    x = np.zeros(p)
    lib().ora_cheb_nodes(p, _p(x))
    return x


def cheb_S(p, l, x):
    return lib().ora_cheb_S(p, l, float(x))


# --------------------------------------------------------------------------
# dense operator, direct product, solvers
# --------------------------------------------------------------------------
def dense_matrix(g: Geometry):
    A = np.zeros((2 * g.n, 2 * g.n))
    lib().ora_dense_matrix(g.n, *g.args(), g.G, g.nu, _p(A))
    return A


def dense_matrix_poly(g: Geometry):
    A = np.zeros((2 * g.n, 2 * g.n))
    lib().ora_dense_matrix_poly(g.n, *g.args(), _p(A))
    return A


def dense_matvec(A, x):
    A = _f64(A)
    x = _f64(x)
    y = np.zeros(A.shape[0])
    lib().ora_dense_matvec(A.shape[0], _p(A), _p(x), _p(y))
    return y


def direct_matvec(g: Geometry, D, rows=None):
    D = _f64(D)
    out = np.zeros(2 * g.n)
    if rows is None:
        lib().ora_direct_matvec(g.n, *g.args(), g.G, g.nu, _p(D), _p(out))
    else:
        lib().ora_direct_matvec_rows(g.n, *g.args(), g.G, g.nu, _p(D), _p(out),
                                     int(rows[0]), int(rows[1]))
    return out


def direct_matvec_rows(g: Geometry, D, idx):
    """Rows of the exact product for receivers idx: array [len(idx), 2]."""
    D = _f64(D)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    out = np.zeros(2 * len(idx))
    lib().ora_direct_matvec_idx(g.n, *g.args(), g.G, g.nu, _p(D), len(idx), _p(idx, _i64), _p(out))
    return out.reshape(-1, 2)


def lu_solve(A, b):
    A = _f64(A)
    b = _f64(b)
    x = np.zeros_like(b)
    rc = lib().ora_lu_solve(A.shape[0], _p(A), _p(b), _p(x))
    if rc != 0:
        raise RuntimeError(f"oracle LU failed: {rc}")
    return x


def gmres_dense(A, b, restart=50, tol=1e-10, maxit=10000, x0=None):
    A = _f64(A)
    b = _f64(b)
    x = np.zeros_like(b) if x0 is None else _f64(x0).copy()
    it, rr = C.c_int(), C.c_double()
    rc = lib().ora_gmres_dense(A.shape[0], _p(A), _p(b), _p(x), restart, tol, maxit,
                               C.byref(it), C.byref(rr))
    return x, {"converged": rc == 0, "iters": it.value, "relres": rr.value}


def gmres_direct(g: Geometry, b, restart=50, tol=1e-10, maxit=10000):
    b = _f64(b)
    x = np.zeros_like(b)
    it, rr = C.c_int(), C.c_double()
    rc = lib().ora_gmres_direct(g.n, *g.args(), g.G, g.nu, _p(b), _p(x), restart, tol,
                                maxit, C.byref(it), C.byref(rr))
    return x, {"converged": rc == 0, "iters": it.value, "relres": rr.value}


def rhs(g: Geometry, pressure, SH, Sh):
    pressure = _f64(pressure)
    out = np.zeros(2 * g.n)
    lib().ora_rhs(g.n, _p(g.cb), _p(g.sb), _p(pressure), SH, Sh, _p(out))
    return out


def sif(E, nu, a, Ds, Dn):
    KI, KII = C.c_double(), C.c_double()
    lib().ora_sif(E, nu, a, Ds, Dn, C.byref(KI), C.byref(KII))
    return KI.value, KII.value


# --------------------------------------------------------------------------
# tree, lists, FMM
# --------------------------------------------------------------------------
class Tree:
    """Oracle quad-tree and U/V/W/X lists (exported as numpy arrays)."""

    def __init__(self, g: Geometry, leaf=32, cap=MAX_LEVEL, kappa=KAPPA, box=None,
                 lists=True):
        self.g = g
        use_box = box is not None
        bx0, by0, bL = box if use_box else (0.0, 0.0, 0.0)
        h = lib().ora_tree_build(g.n, _p(g.cx), _p(g.cy), _p(g.a), leaf, cap, kappa,
                                 int(use_box), bx0, by0, bL)
        if not h:
            raise ValueError("oracle tree build rejected the input")
        self._h = C.c_void_p(h)
        nc = lib().ora_tree_ncell(self._h)
        n = g.n
        self.ncell = nc
        self.perm = np.zeros(n, np.int64)
        self.key = np.zeros(n, np.uint64)
        self.level = np.zeros(nc, np.int32)
        self.ix = np.zeros(nc, np.uint32)
        self.iy = np.zeros(nc, np.uint32)
        self.parent = np.zeros(nc, np.int32)
        self.child = np.zeros((nc, 4), np.int32)
        self.pbeg = np.zeros(nc, np.int64)
        self.pend = np.zeros(nc, np.int64)
        self.isleaf = np.zeros(nc, np.int32)
        self.root = np.zeros(3)
        lib().ora_tree_export(self._h, _p(self.perm, _i64), _p(self.key, _u64),
                              _p(self.level, _i32), _p(self.ix, _u32), _p(self.iy, _u32),
                              _p(self.parent, _i32), _p(self.child, _i32),
                              _p(self.pbeg, _i64), _p(self.pend, _i64),
                              _p(self.isleaf, _i32), _p(self.root))
        self.lists = {}
        if lists:
            lib().ora_lists_build(self._h)
            for w, name in enumerate("UVWX"):
                sz = lib().ora_list_size(self._h, w)
                off = np.zeros(nc + 1, np.int64)
                idx = np.zeros(max(sz, 1), np.int32)
                lib().ora_list_export(self._h, w, _p(off, _i64), _p(idx, _i32))
                self.lists[name] = (off, idx[:sz])

    def __del__(self):
        try:
            if getattr(self, "_h", None):
                lib().ora_tree_free(self._h)
                self._h = None
        except Exception:
            pass

    def fmm(self, D, p, kernel=0):
        if not self.lists:
            raise ValueError("tree built without lists")
        D = _f64(D)
        out = np.zeros(2 * self.g.n)
        g = self.g
        rc = lib().ora_fmm_apply(self._h, *g.args(), g.G, g.nu, p, kernel, _p(D), _p(out))
        if rc != 0:
            raise RuntimeError("oracle FMM failed")
        return out


def num_threads() -> int:
    """Host threads the oracle's parallel loops use."""
    return int(lib().ora_num_threads())


def set_num_threads(n: int) -> int:
    """Use n threads in the parallel loops (n <= 0: one per processor);
    returns the previous count.  Timing only: the loops parallelise over
    independent rows, so results do not depend on it."""
    prev = num_threads()
    lib().ora_set_num_threads(int(n))
    return prev


# --------------------------------------------------------------------------
# poroelastic influence (Section 2, eqs. 2.1-2.5)
# --------------------------------------------------------------------------
class Poro:
    """Material constants of the fully coupled (Biot) medium: drained E, nu,
    undrained nu_u, Biot alpha, permeability and fluid viscosity."""

    def __init__(self, E=20e9, nu=0.2, nuu=0.35, alpha=0.8, perm=1e-18, visc=1e-3):
        self.P = np.zeros(10)
        lib().ora_poro_consts(E, nu, nuu, alpha, perm, visc, _p(self.P))
        self.E, self.nu, self.nuu, self.alpha = E, nu, nuu, alpha
        (self.G, _, _, _, self.kappa, self.M, self.S, self.c, self.eta, self.B) = self.P


def E1(z):
    return lib().ora_E1(float(z))


def poro_point(po: Poro, x, y, t, q, qf=0.0, transient=False):
    """(sxx, syy, sxy, p) of a point DD with charges q and a fluid source qf,
    both held from t = 0; transient=True drops the drained elastic part."""
    out = np.zeros(4)
    qq = _f64(q)
    f = lib().ora_poro_point_transient if transient else lib().ora_poro_point
    f(_p(po.P), float(x), float(y), float(t), _p(qq), float(qf), _p(out))
    return out


def poro_elem_transient(po: Poro, X, Y, cx, cy, cb, sb, a, Ds, Dn, Dq, t1, t0=0.0, nq=12, np_min=4):
    out = np.zeros(4)
    lib().ora_poro_elem_transient(_p(po.P), X, Y, cx, cy, cb, sb, a, Ds, Dn, Dq, t1, t0, nq, np_min,
                                  _p(out))
    return out


def poro_matrix(g: Geometry, po: Poro, dt, m, nq=12, np_min=4):
    """Time-marching coefficient matrix (3n x 3n): m = 0 gives F(dt), m >= 1
    gives F((m+1)dt) - F(m dt); rows (shear, normal, pressure) per receiver,
    columns (Ds, Dn, Dq) per element."""
    A = np.zeros((3 * g.n, 3 * g.n))
    lib().ora_poro_matrix(g.n, _p(g.cx), _p(g.cy), _p(g.cb), _p(g.sb), _p(g.a), _p(po.P),
                          float(dt), int(m), int(nq), int(np_min), _p(A))
    return A


def poro_matrix_rows(g: Geometry, po: Poro, dt, m, rows, nq=12, np_min=4):
    """Rows of poro_matrix for the receivers `rows`: array [3 len(rows), 3n]
    (shear, normal, pressure per receiver)."""
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    R = np.zeros((3 * len(rows), 3 * g.n))
    lib().ora_poro_matrix_rows(g.n, _p(g.cx), _p(g.cy), _p(g.cb), _p(g.sb), _p(g.a), _p(po.P),
                               float(dt), int(m), int(nq), int(np_min), len(rows), _p(rows, _i64), _p(R))
    return R


def poro_rhs(g: Geometry, pf, p0, SH, Sh):
    """Right-hand side of one time step without history (Section 4): the
    induced tractions cancel the fluid pressure and the far field, the
    induced pore pressure at the faces equals pf - p0."""
    b2 = rhs(g, pf, SH, Sh)
    b = np.zeros(3 * g.n)
    b[0::3] = b2[0::2]
    b[1::3] = b2[1::2]
    b[2::3] = np.asarray(pf, dtype=np.float64) - p0
    return b


def poro_march(g: Geometry, po: Poro, dt, steps, pf, p0, SH, Sh, nq=12, np_min=4):
    """Time marching of eqs. 2.3-2.5 with dense matrices and Gaussian
    elimination: D^h solves K_0 D^h = b - sum_{k<h} K_{h-k} D^k.  Returns the
    list of D^h (3n each) and the history contributions."""
    K = [poro_matrix(g, po, dt, m, nq, np_min) for m in range(steps)]
    b = poro_rhs(g, pf, p0, SH, Sh)
    Ds, hist = [], []
    for h in range(1, steps + 1):
        hs = np.zeros(3 * g.n)
        for k in range(1, h):
            hs += K[h - k] @ Ds[k - 1]
        hist.append(hs)
        Ds.append(lu_solve(K[0], b - hs))
    return Ds, hist, K
