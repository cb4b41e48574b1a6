"""Seeded synthetic inputs shared by the oracle tests and the GPU path.

This module only produces geometry and loads (element endpoints, per-element
fluid pressure, far-field stresses, material constants).  It contains none of
the method's arithmetic: no influence coefficients, no tree, no expansions,
no right-hand-side resolution.  Both the oracle (``oracle/``) and the HIP
path read the same arrays from here.

The paper's own workloads cannot be reproduced (its fracture geometries exist
only in figures that are not available), so these are stand-ins with the same
structure: a single pressurized Griffith crack (closed-form check), random
pressurized fractures of mixed orientation in a square box (the paper's
Section 5.2.2 example, with orientations drawn uniformly instead of three
fixed angles), and parallel transverse fractures of a horizontal well
(Section 5.2.1).

Random numbers: numpy's PCG64 with an explicit seed.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Workload:
    """Element endpoints plus loads.  Lengths in m, stresses/pressures in Pa."""

    name: str
    x1: np.ndarray
    y1: np.ndarray
    x2: np.ndarray
    y2: np.ndarray
    pressure: np.ndarray          # fluid pressure acting on each element face
    frac_id: np.ndarray           # fracture each element belongs to
    E: float = 20e9
    nu: float = 0.25
    SH: float = 0.0               # compression-positive far field along x
    Sh: float = 0.0               # compression-positive far field along y
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.x1.shape[0])

    @property
    def G(self) -> float:
        return self.E / (2.0 * (1.0 + self.nu))


def _discretise(xa, ya, xb, yb, m):
    """Split the segment (xa,ya)-(xb,yb) into m equal elements."""
    t = np.arange(m + 1, dtype=np.float64) / m
    xs = xa + (xb - xa) * t
    ys = ya + (yb - ya) * t
    return xs[:-1], ys[:-1], xs[1:], ys[1:]


def griffith(n: int = 256, a: float = 1.0, p: float = 10e6,
             E: float = 20e9, nu: float = 0.25) -> Workload:
    """Straight crack on the x-axis from -a to a, n equal elements,
    uniform internal pressure p, no far field (plane strain)."""
    x1, y1, x2, y2 = _discretise(-a, 0.0, a, 0.0, n)
    return Workload("griffith", x1, y1, x2, y2,
                    pressure=np.full(n, p), frac_id=np.zeros(n, np.int32),
                    E=E, nu=nu, meta={"a": a, "p": p})


def _seg_dist(p0, p1, q0, q1):
    """Minimum distance between segment p0-p1 and each segment q0[k]-q1[k]
    (q arrays shaped [k,2]).  Zero when they cross."""
    def cross(ax, ay, bx, by):
        return ax * by - ay * bx

    d = p1 - p0
    e = q1 - q0
    # proper intersection test
    r0 = cross(d[0], d[1], q0[:, 0] - p0[0], q0[:, 1] - p0[1])
    r1 = cross(d[0], d[1], q1[:, 0] - p0[0], q1[:, 1] - p0[1])
    s0 = cross(e[:, 0], e[:, 1], p0[0] - q0[:, 0], p0[1] - q0[:, 1])
    s1 = cross(e[:, 0], e[:, 1], p1[0] - q0[:, 0], p1[1] - q0[:, 1])
    crossing = (r0 * r1 <= 0) & (s0 * s1 <= 0)

    def pt_seg(px, py, ax, ay, bx, by):
        vx, vy = bx - ax, by - ay
        ll = vx * vx + vy * vy
        t = np.clip(((px - ax) * vx + (py - ay) * vy) / np.where(ll > 0, ll, 1.0), 0.0, 1.0)
        cx, cy = ax + t * vx, ay + t * vy
        return np.hypot(px - cx, py - cy)

    dd = np.minimum.reduce([
        pt_seg(p0[0], p0[1], q0[:, 0], q0[:, 1], q1[:, 0], q1[:, 1]),
        pt_seg(p1[0], p1[1], q0[:, 0], q0[:, 1], q1[:, 0], q1[:, 1]),
        pt_seg(q0[:, 0], q0[:, 1], p0[0], p0[1], p1[0], p1[1]),
        pt_seg(q1[:, 0], q1[:, 1], p0[0], p0[1], p1[0], p1[1]),
    ])
    return np.where(crossing, 0.0, dd)


def random_fractures(seed: int, n_frac: int = 200, elems: int = 100,
                     box: float = 100.0, lmin: float = 1.0, lmax: float = 5.0,
                     pmin: float = 5e6, pmax: float = 15e6,
                     SH: float = 40e6, Sh: float = 30e6,
                     E: float = 20e9, nu: float = 0.25,
                     gap_factor: float = 2.0) -> Workload:
    """Random pressurized fractures in a box.

    Centres uniform in [0,box]^2, orientation uniform in [0,pi), length
    uniform in [lmin,lmax], pressure uniform in [pmin,pmax] per fracture.
    A candidate is rejected when it crosses, or comes closer than
    gap_factor x (its element length, or the larger neighbour's) to, any
    accepted fracture.  Each fracture is split into `elems` equal elements.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    P0 = np.zeros((0, 2))
    P1 = np.zeros((0, 2))
    elen = np.zeros(0)
    lens, press = [], []
    while P0.shape[0] < n_frac:
        c = rng.uniform(0.0, box, size=2)
        th = rng.uniform(0.0, np.pi)
        L = rng.uniform(lmin, lmax)
        pf = rng.uniform(pmin, pmax)
        u = np.array([np.cos(th), np.sin(th)])
        p0 = c - 0.5 * L * u
        p1 = c + 0.5 * L * u
        if P0.shape[0]:
            dist = _seg_dist(p0, p1, P0, P1)
            need = gap_factor * np.maximum(elen, L / elems)
            if np.any(dist < need):
                continue
        P0 = np.vstack([P0, p0])
        P1 = np.vstack([P1, p1])
        elen = np.append(elen, L / elems)
        lens.append(L)
        press.append(pf)
    xs1, ys1, xs2, ys2, pr, fid = [], [], [], [], [], []
    for k in range(n_frac):
        a, b, c_, d = _discretise(P0[k, 0], P0[k, 1], P1[k, 0], P1[k, 1], elems)
        xs1.append(a); ys1.append(b); xs2.append(c_); ys2.append(d)
        pr.append(np.full(elems, press[k]))
        fid.append(np.full(elems, k, np.int32))
    return Workload(f"random{seed}", np.concatenate(xs1), np.concatenate(ys1),
                    np.concatenate(xs2), np.concatenate(ys2),
                    pressure=np.concatenate(pr), frac_id=np.concatenate(fid),
                    E=E, nu=nu, SH=SH, Sh=Sh,
                    meta={"seed": seed, "n_frac": n_frac, "elems": elems,
                          "box": box, "frac_len": np.array(lens)})


def well_cluster(n_frac: int = 5, elems: int = 4000, half_length: float = 400.0,
                 spacing: float = 10.0, p_inj: float = 58e6,
                 SH: float = 58.60e6, Sh: float = 55.15e6,
                 E: float = 20e9, nu: float = 0.2) -> Workload:
    """Parallel transverse fractures of a horizontal well (paper Section 5.2.1,
    Table 2 loads): fractures along x, centred at x=0, at y = k*spacing
    symmetric about 0."""
    ys = (np.arange(n_frac) - (n_frac - 1) / 2.0) * spacing
    xs1, ys1, xs2, ys2, fid = [], [], [], [], []
    for k, y in enumerate(ys):
        a, b, c_, d = _discretise(-half_length, y, half_length, y, elems)
        xs1.append(a); ys1.append(b); xs2.append(c_); ys2.append(d)
        fid.append(np.full(elems, k, np.int32))
    n = n_frac * elems
    return Workload("well", np.concatenate(xs1), np.concatenate(ys1),
                    np.concatenate(xs2), np.concatenate(ys2),
                    pressure=np.full(n, p_inj), frac_id=np.concatenate(fid),
                    E=E, nu=nu, SH=SH, Sh=Sh,
                    meta={"half_length": half_length, "spacing": spacing})


def split_tie() -> Workload:
    """Nine elements in the root square [0, 16)^2 (pass it as the user root
    box): one long element from (2, 2) to (2.7896393349678577,
    2.8656608821898697) and eight short horizontal ones (length 0.02)
    centred at (2.1 + 0.2 k, 3.5).  The long element's squared length is
    not a double; rounding its two squares and their sum separately gives a
    length one unit in the last place below the value a fused multiply-add
    or a correctly rounded hypot gives."""
    cxs = 2.1 + 0.2 * np.arange(8)
    x1 = np.concatenate([[2.0], cxs - 0.01])
    x2 = np.concatenate([[2.7896393349678577], cxs + 0.01])
    y1 = np.concatenate([[2.0], np.full(8, 3.5)])
    y2 = np.concatenate([[2.8656608821898697], np.full(8, 3.5)])
    n = x1.shape[0]
    return Workload("split_tie", x1, y1, x2, y2, np.zeros(n), np.zeros(n, np.int64),
                    meta={"root_box": (0.0, 0.0, 16.0)})


def random_vector(seed: int, n: int, scale: float = 1e-3) -> np.ndarray:
    """Seeded displacement-discontinuity vector, element-major [Ds, Dn]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal(2 * n) * scale


def c1() -> Workload:
    """Griffith crack, N=256, a=1 m, p=10 MPa, E=20 GPa, nu=0.25."""
    return griffith(256)


def c2() -> Workload:
    """200 random fractures x 100 elements (N=20000), seed 2."""
    return random_fractures(2, 200, 100)


def c4() -> Workload:
    """2000 random fractures x 100 elements (N=200000), seed 4."""
    return random_fractures(4, 2000, 100)


@dataclass
class ServingRequest:
    """One request of a serving stream: a random-fracture problem (as in
    random_fractures) with n_frac fractures of `elems` elements in a box
    scaled to keep the fracture density of the 200-fracture, 100 m case,
    `steps` load steps, and an arrival time in units of the mean
    inter-arrival gap (multiply by 1/rate)."""

    index: int
    seed: int
    n_frac: int
    elems: int
    box: float
    steps: int
    arrival_units: float

    @property
    def n(self) -> int:
        return self.n_frac * self.elems

    def workload(self) -> Workload:
        return random_fractures(self.seed, self.n_frac, self.elems, box=self.box)


def serving_stream(seed: int = 5, count: int = 1024, nmin: int = 1000, nmax: int = 50000,
                   steps_max: int = 10, elems: int = 100) -> list:
    """Poisson-arrival request stream: N log-uniform in [nmin, nmax] rounded
    to whole fractures of `elems` elements, steps uniform in 1..steps_max,
    exponential inter-arrival gaps of unit mean.  Geometry is generated on
    demand (ServingRequest.workload) from a per-request seed."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out, t = [], 0.0
    for i in range(count):
        n = float(np.exp(rng.uniform(np.log(nmin), np.log(nmax))))
        n_frac = max(1, int(round(n / elems)))
        steps = int(rng.integers(1, steps_max + 1))
        t += float(rng.exponential(1.0))
        box = 100.0 * float(np.sqrt(n_frac / 200.0))
        out.append(ServingRequest(i, seed * 100003 + i, n_frac, elems, box, steps, t))
    return out
