"""Plain CPU oracle of the self-propelled Voronoi (SPV) step.

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package; the product
path (the HIP library and its binding) never does.  The oracle shares no code
with the HIP library: it is the serial C file ``spv_oracle.c`` (full periodic
Bowyer-Watson retriangulation every step, exact predicates, dual-number
forces, Philox noise) plus this ctypes wrapper.

Paper: Sussman, "cellGPU: massively parallel simulations of dynamic vertex
models", arXiv:1702.02939 -- Eq. (1) energy, Eq. (3) equation of motion,
Sec. II.A rotational noise, Sec. II.C.1 Voronoi geometry, Sec. II.C.3
empty-circumcircle validity, App. B force sign F = -dE/dr.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "spv_oracle.c")
_SRC_AVM = os.path.join(_HERE, "avm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK, EINVAL, ENOMEM, EPRECOND, ECAPACITY, EFAIL = 0, -1, -2, -4, -5, -8


def build(force: bool = True) -> str:
    """Compile spv_oracle.c with gcc into liboracle.so (next to the source)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fPIC", "-shared",
                               "-o", tmp, _SRC, _SRC_AVM, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


class _Params(ctypes.Structure):
    _fields_ = [("KA", ctypes.c_double), ("KP", ctypes.c_double), ("mu", ctypes.c_double),
                ("v0", ctypes.c_double), ("Dr", ctypes.c_double), ("dt", ctypes.c_double),
                ("seed", ctypes.c_uint64)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = ctypes.CDLL(_LIB)
        P = ctypes.POINTER
        d, i64, i32 = ctypes.c_double, ctypes.c_int64, ctypes.c_int32
        L.orc_grid_q.restype = ctypes.c_int
        L.orc_grid_q.argtypes = [d]
        L.orc_quantize.restype = None
        L.orc_quantize.argtypes = [i64, P(d), d, ctypes.c_int, P(d)]
        for f in ("orc_orient",):
            getattr(L, f).restype = ctypes.c_int
            getattr(L, f).argtypes = [P(i64)] * 3
        L.orc_incircle.restype = ctypes.c_int
        L.orc_incircle.argtypes = [P(i64)] * 4
        L.orc_incircle_sos.restype = ctypes.c_int
        L.orc_incircle_sos.argtypes = [P(i64)] * 5
        L.orc_exact_calls.restype = i64
        L.orc_triangulate.restype = ctypes.c_int
        L.orc_triangulate.argtypes = [i64, P(d), P(d), d, d, ctypes.c_int, P(i32), P(i32), i64, P(i64), P(d)]
        L.orc_geometry.restype = ctypes.c_int
        L.orc_geometry.argtypes = [i64, P(d), P(d), d, d, P(i32), P(i32), P(d), P(d)]
        L.orc_forces.restype = ctypes.c_int
        L.orc_forces.argtypes = [i64, P(d), P(d), d, d, P(i32), P(i32), P(d), P(d), d, d, P(d), P(d)]
        L.orc_observables.restype = None
        L.orc_observables.argtypes = [i64, P(d), P(d), P(d), P(d), d, d, P(d), P(d), P(d)]
        L.orc_philox4x64.restype = None
        L.orc_philox4x64.argtypes = [P(ctypes.c_uint64)] * 3
        L.orc_normal.restype = d
        L.orc_normal.argtypes = [ctypes.c_uint64] * 3
        L.orc_theta0.restype = d
        L.orc_theta0.argtypes = [ctypes.c_uint64] * 2
        L.orc_run.restype = ctypes.c_int
        L.orc_run.argtypes = [i64, P(d), P(d), P(d), d, d, ctypes.c_int, P(d), P(d), P(_Params),
                              ctypes.c_uint64, i64, P(d), P(d), P(d), P(d), P(i32), P(i32), i64]
        _lib = L
    return _lib


def _p(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what}: oracle status {code}")
        self.code = code


# ---------------------------------------------------------------- grid
def grid_q(Lmax: float) -> int:
    """Grid exponent q: positions are multiples of 2^-q, max(Lx,Ly) <= 2^(51-q)."""
    return int(lib().orc_grid_q(float(Lmax)))


def prepare(x, y, Lx, Ly):
    """Quantise raw positions and box onto the grid.  Returns (x, y, Lx, Ly, q)."""
    q = grid_q(max(Lx, Ly))
    xq, yq = _f64(x).copy(), _f64(y).copy()
    Lxq, Lyq = ctypes.c_double(), ctypes.c_double()
    lib().orc_quantize(len(xq), _p(xq, ctypes.c_double), float(Lx), q, ctypes.byref(Lxq))
    lib().orc_quantize(len(yq), _p(yq, ctypes.c_double), float(Ly), q, ctypes.byref(Lyq))
    return xq, yq, Lxq.value, Lyq.value, q


# ---------------------------------------------------------------- predicates
def orient(a, b, c) -> int:
    """Sign of the orientation of integer points a, b, c (> 0: counter-clockwise)."""
    A, B, C = (np.asarray(v, dtype=np.int64) for v in (a, b, c))
    return int(lib().orc_orient(_p(A, ctypes.c_int64), _p(B, ctypes.c_int64), _p(C, ctypes.c_int64)))


def incircle(a, b, c, d) -> int:
    """Sign of the in-circle determinant (> 0: d strictly inside circle abc, abc CCW)."""
    A, B, C, D = (np.asarray(v, dtype=np.int64) for v in (a, b, c, d))
    return int(lib().orc_incircle(*(_p(v, ctypes.c_int64) for v in (A, B, C, D))))


def incircle_sos(a, b, c, d, ranks) -> int:
    A, B, C, D = (np.asarray(v, dtype=np.int64) for v in (a, b, c, d))
    R = np.asarray(ranks, dtype=np.int64)
    return int(lib().orc_incircle_sos(*(_p(v, ctypes.c_int64) for v in (A, B, C, D, R))))


def exact_calls() -> int:
    return int(lib().orc_exact_calls())


# ---------------------------------------------------------------- triangulation
def triangulate(x, y, Lx, Ly, q):
    """Periodic Delaunay triangulation of grid positions.

    Returns (ring_off[N+1], ring, ntri, max_circumradius); the neighbours of
    cell i are ring[ring_off[i]:ring_off[i+1]], counter-clockwise, starting at
    the smallest tag."""
    x, y = _f64(x), _f64(y)
    n = len(x)
    cap = 32 * n + 64
    off = np.zeros(n + 1, dtype=np.int32)
    ring = np.zeros(cap, dtype=np.int32)
    ntri = ctypes.c_int64()
    mcr = ctypes.c_double()
    rc = lib().orc_triangulate(n, _p(x, ctypes.c_double), _p(y, ctypes.c_double), float(Lx), float(Ly), int(q),
                               _p(off, ctypes.c_int32), _p(ring, ctypes.c_int32), cap, ctypes.byref(ntri),
                               ctypes.byref(mcr))
    if rc != OK:
        raise OracleError(rc, "triangulate")
    return off, ring[: off[-1]].copy(), int(ntri.value), float(mcr.value)


def rings_as_lists(off, ring):
    return [ring[off[i]:off[i + 1]].tolist() for i in range(len(off) - 1)]


def geometry(x, y, Lx, Ly, off, ring):
    """Voronoi area and perimeter of every cell."""
    x, y = _f64(x), _f64(y)
    n = len(x)
    A = np.zeros(n)
    P = np.zeros(n)
    lib().orc_geometry(n, _p(x, ctypes.c_double), _p(y, ctypes.c_double), float(Lx), float(Ly),
                       _p(off, ctypes.c_int32), _p(ring, ctypes.c_int32), _p(A, ctypes.c_double),
                       _p(P, ctypes.c_double))
    return A, P


def forces(x, y, Lx, Ly, off, ring, A0, P0, KA=1.0, KP=1.0):
    """F_i = -dE/dr_i for Eq. (1) with the given topology (dual numbers)."""
    x, y = _f64(x), _f64(y)
    n = len(x)
    A0 = _f64(np.broadcast_to(A0, (n,)))
    P0 = _f64(np.broadcast_to(P0, (n,)))
    fx = np.zeros(n)
    fy = np.zeros(n)
    rc = lib().orc_forces(n, _p(x, ctypes.c_double), _p(y, ctypes.c_double), float(Lx), float(Ly),
                          _p(off, ctypes.c_int32), _p(ring, ctypes.c_int32), _p(A0, ctypes.c_double),
                          _p(P0, ctypes.c_double), float(KA), float(KP), _p(fx, ctypes.c_double),
                          _p(fy, ctypes.c_double))
    if rc != OK:
        raise OracleError(rc, "forces")
    return fx, fy


def energy(A, P, A0, P0, KA=1.0, KP=1.0) -> float:
    """Eq. (1)."""
    A, P = _f64(A), _f64(P)
    n = len(A)
    A0 = _f64(np.broadcast_to(A0, (n,)))
    P0 = _f64(np.broadcast_to(P0, (n,)))
    E, qb, sa = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    lib().orc_observables(n, _p(A, ctypes.c_double), _p(P, ctypes.c_double), _p(A0, ctypes.c_double),
                          _p(P0, ctypes.c_double), float(KA), float(KP), ctypes.byref(E), ctypes.byref(qb),
                          ctypes.byref(sa))
    return E.value, qb.value, sa.value


# ---------------------------------------------------------------- noise
def philox4x64(ctr, key):
    c = np.asarray(ctr, dtype=np.uint64)
    k = np.asarray(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    lib().orc_philox4x64(_p(c, ctypes.c_uint64), _p(k, ctypes.c_uint64), _p(out, ctypes.c_uint64))
    return out


def normal(seed, step, tag) -> float:
    return float(lib().orc_normal(int(seed), int(step), int(tag)))


def theta0(seed, n):
    return np.array([lib().orc_theta0(int(seed), t) for t in range(n)])


# ---------------------------------------------------------------- whole steps
def run(x, y, theta, Lx, Ly, q, A0, P0, *, KA=1.0, KP=1.0, mu=1.0, v0=0.0, Dr=0.0, dt=0.01, seed=0,
        step0=0, nsteps=1, want_forces=False, want_rings=False):
    """Run nsteps oracle steps on copies of (x, y, theta).

    Returns a dict with x, y, theta after the run, E and qbar of the state at
    the start of every step plus the final one (nsteps+1 entries), and
    optionally the forces and the topology of the final state."""
    x, y, th = _f64(x).copy(), _f64(y).copy(), _f64(theta).copy()
    n = len(x)
    A0 = _f64(np.broadcast_to(A0, (n,)))
    P0 = _f64(np.broadcast_to(P0, (n,)))
    prm = _Params(KA, KP, mu, v0, Dr, dt, seed)
    E = np.zeros(nsteps + 1)
    Q = np.zeros(nsteps + 1)
    fx = np.zeros(n) if want_forces else None
    fy = np.zeros(n) if want_forces else None
    cap = 32 * n + 64
    off = np.zeros(n + 1, dtype=np.int32) if want_rings else None
    ring = np.zeros(cap, dtype=np.int32) if want_rings else None
    nullD = ctypes.POINTER(ctypes.c_double)()
    nullI = ctypes.POINTER(ctypes.c_int32)()
    rc = lib().orc_run(n, _p(x, ctypes.c_double), _p(y, ctypes.c_double), _p(th, ctypes.c_double), float(Lx),
                       float(Ly), int(q), _p(A0, ctypes.c_double), _p(P0, ctypes.c_double), ctypes.byref(prm),
                       int(step0), int(nsteps), _p(E, ctypes.c_double), _p(Q, ctypes.c_double),
                       _p(fx, ctypes.c_double) if want_forces else nullD,
                       _p(fy, ctypes.c_double) if want_forces else nullD,
                       _p(off, ctypes.c_int32) if want_rings else nullI,
                       _p(ring, ctypes.c_int32) if want_rings else nullI, cap)
    if rc != OK:
        raise OracleError(rc, "run")
    out = {"x": x, "y": y, "theta": th, "E": E, "qbar": Q}
    if want_forces:
        out["fx"], out["fy"] = fx, fy
    if want_rings:
        out["ring_off"], out["ring"] = off, ring[: off[-1]].copy()
    return out


# ---------------------------------------------------------------- active vertex model
class _AvmParams(ctypes.Structure):
    _fields_ = [("KA", ctypes.c_double), ("KP", ctypes.c_double), ("mu", ctypes.c_double),
                ("v0", ctypes.c_double), ("Dr", ctypes.c_double), ("dt", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("l_t1", ctypes.c_double), ("l_new", ctypes.c_double)]


def _avm_lib():
    L = lib()
    if not getattr(L, "_avm_ready", False):
        P = ctypes.POINTER
        d, i64, i32 = ctypes.c_double, ctypes.c_int64, ctypes.c_int32
        L.orc_avm_geometry.restype = ctypes.c_int
        L.orc_avm_geometry.argtypes = [i64, P(d), P(d), d, d, P(i32), P(i32), P(d), P(d)]
        L.orc_avm_forces.restype = ctypes.c_int
        L.orc_avm_forces.argtypes = [i64, i64, P(d), P(d), d, d, P(i32), P(i32), P(d), P(d), d, d, P(d), P(d)]
        L.orc_avm_run.restype = ctypes.c_int
        L.orc_avm_run.argtypes = [i64, i64, P(d), P(d), P(d), d, d, ctypes.c_int, P(i32), P(i32), i64, P(d), P(d),
                                  P(_AvmParams), ctypes.c_uint64, i64, P(d), P(d), P(i64)]
        L._avm_ready = True
    return L


def voronoi_network(x, y, Lx, Ly, q):
    """The active vertex model's polygon network of the Voronoi tessellation
    of cells at (x, y) (grid-exact): one vertex per Delaunay triangle at its
    circumcentre, cell i's vertex list counter-clockwise in the order of its
    ring (from its smallest-tag neighbour).  Vertices are numbered by first
    appearance, cells visited in tag order (so a triangle is first met at its
    smallest-tag corner, whose frame gives its position), positions wrapped
    into the box and put on the grid 2^-q.  Returns vx, vy, cell_off, cell_vtx."""
    x, y = _f64(x), _f64(y)
    off, ring, ntri, _ = triangulate(x, y, Lx, Ly, q)
    n = len(x)
    s = 2.0 ** q
    ids, vx, vy = {}, [], []
    cv = np.zeros(off[-1], dtype=np.int32)
    for i in range(n):
        js = ring[off[i]:off[i + 1]]
        k = len(js)
        for m in range(k):
            a, b = int(js[m]), int(js[(m + 1) % k])
            tri = (i, a, b)
            r = tri.index(min(tri))
            key = tri[r:] + tri[:r]
            if key not in ids:
                bx = x[a] - x[i]
                bx -= Lx * round(bx / Lx)
                by = y[a] - y[i]
                by -= Ly * round(by / Ly)
                cx = x[b] - x[i]
                cx -= Lx * round(cx / Lx)
                cy = y[b] - y[i]
                cy -= Ly * round(cy / Ly)
                d = 2.0 * (bx * cy - by * cx)
                ux = (cy * (bx * bx + by * by) - by * (cx * cx + cy * cy)) / d
                uy = (bx * (cx * cx + cy * cy) - cx * (bx * bx + by * by)) / d
                X = np.rint((x[i] + ux) * s) % np.rint(Lx * s)
                Y = np.rint((y[i] + uy) * s) % np.rint(Ly * s)
                ids[key] = len(vx)
                vx.append(X / s)
                vy.append(Y / s)
            cv[off[i] + m] = ids[key]
    return np.array(vx), np.array(vy), off.astype(np.int32), cv


def avm_geometry(vx, vy, Lx, Ly, cell_off, cell_vtx):
    vx, vy = _f64(vx), _f64(vy)
    off = np.ascontiguousarray(cell_off, dtype=np.int32)
    cv = np.ascontiguousarray(cell_vtx, dtype=np.int32)
    nc = len(off) - 1
    A, P = np.zeros(nc), np.zeros(nc)
    rc = _avm_lib().orc_avm_geometry(nc, _p(vx, ctypes.c_double), _p(vy, ctypes.c_double), float(Lx), float(Ly),
                                     _p(off, ctypes.c_int32), _p(cv, ctypes.c_int32), _p(A, ctypes.c_double),
                                     _p(P, ctypes.c_double))
    if rc != OK:
        raise OracleError(rc, "avm_geometry")
    return A, P


def avm_forces(vx, vy, Lx, Ly, cell_off, cell_vtx, A0, P0, KA=1.0, KP=1.0):
    """F_v = -dE/dh_v of Eq. (1) over the polygon cells (dual numbers)."""
    vx, vy = _f64(vx), _f64(vy)
    off = np.ascontiguousarray(cell_off, dtype=np.int32)
    cv = np.ascontiguousarray(cell_vtx, dtype=np.int32)
    nc, nv = len(off) - 1, len(vx)
    A0 = _f64(np.broadcast_to(A0, (nc,)))
    P0 = _f64(np.broadcast_to(P0, (nc,)))
    fx, fy = np.zeros(nv), np.zeros(nv)
    rc = _avm_lib().orc_avm_forces(nc, nv, _p(vx, ctypes.c_double), _p(vy, ctypes.c_double), float(Lx), float(Ly),
                                   _p(off, ctypes.c_int32), _p(cv, ctypes.c_int32), _p(A0, ctypes.c_double),
                                   _p(P0, ctypes.c_double), float(KA), float(KP), _p(fx, ctypes.c_double),
                                   _p(fy, ctypes.c_double))
    if rc != OK:
        raise OracleError(rc, "avm_forces")
    return fx, fy


def avm_run(vx, vy, theta, Lx, Ly, q, cell_off, cell_vtx, A0, P0, *, KA=1.0, KP=1.0, mu=1.0, v0=0.0, Dr=0.0,
            dt=0.01, seed=0, l_t1=0.04, l_new=0.06, step0=0, nsteps=1):
    """nsteps of the active vertex model (Eq. 4, T1 rounds) on copies of the
    state; returns vx, vy, theta, cell_off, cell_vtx, E and qbar (nsteps + 1
    entries) and the T1 transitions and rounds."""
    vx, vy, th = _f64(vx).copy(), _f64(vy).copy(), _f64(theta).copy()
    off = np.array(cell_off, dtype=np.int32)
    nc, nv = len(off) - 1, len(vx)
    cap = 3 * nv + 64 * 8
    cv = np.zeros(cap, dtype=np.int32)
    cv[: off[-1]] = np.asarray(cell_vtx, dtype=np.int32)[: off[-1]]
    A0 = _f64(np.broadcast_to(A0, (nc,)))
    P0 = _f64(np.broadcast_to(P0, (nc,)))
    prm = _AvmParams(KA, KP, mu, v0, Dr, dt, seed, l_t1, l_new)
    E, Q = np.zeros(nsteps + 1), np.zeros(nsteps + 1)
    cnt = np.zeros(2, dtype=np.int64)
    rc = _avm_lib().orc_avm_run(nc, nv, _p(vx, ctypes.c_double), _p(vy, ctypes.c_double), _p(th, ctypes.c_double),
                                float(Lx), float(Ly), int(q), _p(off, ctypes.c_int32), _p(cv, ctypes.c_int32), cap,
                                _p(A0, ctypes.c_double), _p(P0, ctypes.c_double), ctypes.byref(prm), int(step0),
                                int(nsteps), _p(E, ctypes.c_double), _p(Q, ctypes.c_double),
                                _p(cnt, ctypes.c_int64))
    if rc != OK:
        raise OracleError(rc, "avm_run")
    return {"vx": vx, "vy": vy, "theta": th, "cell_off": off, "cell_vtx": cv[: off[-1]].copy(), "E": E, "qbar": Q,
            "t1": int(cnt[0]), "t1_rounds": int(cnt[1])}


def canonical_cells(cell_off, cell_vtx):
    """Each cell's vertex list rotated to start at its smallest vertex index
    (the comparison form of two networks)."""
    out = []
    for c in range(len(cell_off) - 1):
        v = list(cell_vtx[cell_off[c]:cell_off[c + 1]])
        r = v.index(min(v))
        out.append(tuple(v[r:] + v[:r]))
    return out
