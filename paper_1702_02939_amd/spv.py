"""ctypes binding of libspv.so (the C-ABI declared in include/spv.h).

Argument marshalling only: every step of the model runs in the library's HIP
kernels.  The functions keep the C names (spv_create, spv_step, ...); the
`System` class is a convenience wrapper used by the tests and the benchmark.
Arrays may be numpy arrays (host) or torch tensors (host or device); the
handle's stream is torch's current stream on the current device unless one is
given.  There is no CPU fallback: importing this module fails if the library
is missing.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libspv.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python __graft_entry__.py` (hipcc, gfx950)")

_lib = ctypes.CDLL(LIB_PATH)

SPV_OK, SPV_EINVAL, SPV_ENOMEM, SPV_EHIP, SPV_EPRECOND, SPV_ECAPACITY, SPV_ENONFINITE, SPV_EREPAIR = (
    0, -1, -2, -3, -4, -5, -6, -7)
SPV_FP64, SPV_MIXED = 0, 1
STATUS_NAMES = {0: "SPV_OK", -1: "SPV_EINVAL", -2: "SPV_ENOMEM", -3: "SPV_EHIP", -4: "SPV_EPRECOND",
                -5: "SPV_ECAPACITY", -6: "SPV_ENONFINITE", -7: "SPV_EREPAIR"}

# kernel classes for spv_kernel_time
K_FORCE, K_GEOM, K_REPAIR, K_RETEST, K_TAIL, K_LIST, K_COMPACT, K_RESORT, K_HOST = range(9)
KERNEL_CLASSES = {"force_update": K_FORCE, "geometry_test": K_GEOM, "repair": K_REPAIR, "retest": K_RETEST,
                  "tail": K_TAIL, "cell_list": K_LIST, "compact": K_COMPACT, "resort": K_RESORT,
                  "host_rounds": K_HOST}


class Params(ctypes.Structure):
    _fields_ = [("KA", ctypes.c_double), ("KP", ctypes.c_double), ("mu", ctypes.c_double),
                ("v0", ctypes.c_double), ("Dr", ctypes.c_double), ("dt", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("precision", ctypes.c_int32), ("resort_every", ctypes.c_int32),
                ("kcap", ctypes.c_int32), ("repair_rounds", ctypes.c_int32), ("device_rounds", ctypes.c_int32),
                ("no_graphs", ctypes.c_int32), ("repair_cells", ctypes.c_int32), ("autotune", ctypes.c_int32),
                ("tail_items", ctypes.c_int32), ("full_rounds", ctypes.c_int32), ("bin_order", ctypes.c_int32),
                ("force_mode", ctypes.c_int32), ("bin_factor", ctypes.c_double), ("dense", ctypes.c_int32),
                ("repair_mode", ctypes.c_int32)]

    def __init__(self, KA=1.0, KP=1.0, mu=1.0, v0=0.0, Dr=1.0, dt=0.01, seed=0, precision=SPV_FP64,
                 resort_every=0, kcap=0, repair_rounds=0, device_rounds=0, no_graphs=0, repair_cells=0,
                 autotune=0, tail_items=0, full_rounds=0, bin_order=0, force_mode=0, bin_factor=0.0, dense=0,
                 repair_mode=0):
        super().__init__(KA, KP, mu, v0, Dr, dt, seed, precision, resort_every, kcap, repair_rounds,
                         device_rounds, no_graphs, repair_cells, autotune, tail_items, full_rounds, bin_order,
                         force_mode, bin_factor, dense, repair_mode)


class AvmParams(ctypes.Structure):
    _fields_ = [("KA", ctypes.c_double), ("KP", ctypes.c_double), ("mu", ctypes.c_double),
                ("v0", ctypes.c_double), ("Dr", ctypes.c_double), ("dt", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("t1_length", ctypes.c_double), ("t1_new_length", ctypes.c_double),
                ("resort_every", ctypes.c_int32), ("bin_order", ctypes.c_int32)]

    def __init__(self, KA=1.0, KP=1.0, mu=1.0, v0=0.0, Dr=1.0, dt=0.01, seed=0, t1_length=0.04,
                 t1_new_length=0.0, resort_every=0, bin_order=0):
        super().__init__(KA, KP, mu, v0, Dr, dt, seed, t1_length, t1_new_length, resort_every, bin_order)


class Tuning(ctypes.Structure):
    _fields_ = [("resort_every", ctypes.c_int32), ("device_rounds", ctypes.c_int32),
                ("repair_cells", ctypes.c_int32), ("tail_items", ctypes.c_int32), ("full_rounds", ctypes.c_int32),
                ("force_mode", ctypes.c_int32), ("source", ctypes.c_int32),
                ("bin_factor", ctypes.c_double),
                ("ms_per_step", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_P = ctypes.c_void_p
_d = ctypes.c_double
_i64 = ctypes.c_int64
_i32 = ctypes.c_int32
_H = ctypes.c_void_p

_SIGS = {
    "spv_create": [ctypes.POINTER(_H), _i64, _P, _P, _d, _d, _P, _P, _d, _P, ctypes.POINTER(Params), _P],
    "spv_batch_create": [ctypes.POINTER(_H), _i32, _P, _P, _P, _P, _P, _P, _P, _P, _P, ctypes.POINTER(Params), _P],
    "spv_step": [_H, _i64],
    "spv_get_tuning": [_H, ctypes.POINTER(Tuning)],
    "spv_save_state": [_H, _P, _i64, ctypes.POINTER(_i64)],
    "spv_load_state": [_H, _P, _i64],
    "spv_get_size": [_H, ctypes.POINTER(_i32), ctypes.POINTER(_i64)],
    "spv_get_kcap": [_H, ctypes.POINTER(_i32)],
    "spv_get_system_range": [_H, _i32, ctypes.POINTER(_i64), ctypes.POINTER(_i64)],
    "spv_get_box": [_H, ctypes.POINTER(_d), ctypes.POINTER(_d), ctypes.POINTER(_i32)],
    "spv_get_system_box": [_H, _i32, ctypes.POINTER(_d), ctypes.POINTER(_d), ctypes.POINTER(_i32)],
    "spv_get_system_observables": [_H, _i32, ctypes.POINTER(_d), ctypes.POINTER(_d), ctypes.POINTER(_d)],
    "spv_get_positions": [_H, _P, _P],
    "spv_get_directors": [_H, _P],
    "spv_get_forces": [_H, _P, _P],
    "spv_get_geometry": [_H, _P, _P],
    "spv_get_neighbors": [_H, _P, _P, _i64, ctypes.POINTER(_i64)],
    "spv_debug_set_ring": [_H, _i64, _i32, _P],
    "spv_get_observables": [_H, ctypes.POINTER(_d), ctypes.POINTER(_d), ctypes.POINTER(_d), _P],
    "spv_set_timing": [_H, _i32],
    "spv_kernel_time": [_H, _i32, ctypes.POINTER(_d), ctypes.POINTER(_i64)],
    "spv_traj_forward": [_H, _i64, _i64, ctypes.POINTER(_d)],
    "spv_traj_backward": [_H, _d, _P],
    "spv_force_tangent": [_H, _P, _P, _P, _P],
    "spv_force_tangent_static": [_H, _P, _P, _P, _P],
    "spv_destroy": [_H],
    "spv_avm_create": [ctypes.POINTER(_H), _i64, _i64, _P, _P, _P, _P, _d, _d, _P, _P, _d, _P, _P, _P],
    "spv_avm_step": [_H, _i64],
    "spv_avm_get_vertices": [_H, _P, _P],
    "spv_avm_get_forces": [_H, _P, _P],
    "spv_avm_get_directors": [_H, _P],
    "spv_avm_get_geometry": [_H, _P, _P],
    "spv_avm_get_cells": [_H, _P, _P, _i64, ctypes.POINTER(_i64)],
    "spv_avm_get_observables": [_H, ctypes.POINTER(_d), ctypes.POINTER(_d), _P],
    "spv_avm_destroy": [_H],
    "spv_voronoi_network": [_H, _P, _P, _P, _P],
}
for _name, _args in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = ctypes.c_int
_lib.spv_last_error.restype = ctypes.c_char_p
_lib.spv_last_error.argtypes = []


class SPVError(RuntimeError):
    def __init__(self, status, where):
        msg = _lib.spv_last_error().decode(errors="replace")
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _check(status, where):
    if status != SPV_OK:
        raise SPVError(status, where)


def _ptr(a):
    """Raw pointer of a contiguous float64/int32 numpy array or torch tensor."""
    if a is None:
        return None
    if hasattr(a, "data_ptr"):
        assert a.is_contiguous()
        return ctypes.c_void_p(a.data_ptr())
    assert a.flags["C_CONTIGUOUS"]
    return ctypes.c_void_p(a.ctypes.data)


def _f64(a):
    if a is None:
        return None
    if hasattr(a, "data_ptr"):
        import torch
        return a.to(torch.float64).contiguous()
    return np.ascontiguousarray(a, dtype=np.float64)


def _current_stream():
    try:
        import torch
        if torch.cuda.is_available():
            return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    except ImportError:
        pass
    return ctypes.c_void_p(0)


# ------------------------------------------------------------------ C names
def spv_create(N, x, y, Lx, Ly, A0=None, P0=None, p0=3.8, theta0=None, params=None, stream=None):
    params = params if params is not None else Params()
    h = _H()
    keep = [_f64(x), _f64(y), _f64(A0), _f64(P0), _f64(theta0)]
    st = _lib.spv_create(ctypes.byref(h), int(N), _ptr(keep[0]), _ptr(keep[1]), float(Lx), float(Ly),
                         _ptr(keep[2]), _ptr(keep[3]), float(p0), _ptr(keep[4]), ctypes.byref(params),
                         stream if stream is not None else _current_stream())
    _check(st, "spv_create")
    return h


def spv_batch_create(N_s, L_s, x, y, p0_s, v0_s=None, seed_s=None, P0=None, params=None, stream=None):
    """S independent systems (square boxes of side L_s) stepped together."""
    params = params if params is not None else Params()
    S = len(N_s)
    N_s = np.ascontiguousarray(N_s, dtype=np.int64)
    L_s = np.ascontiguousarray(L_s, dtype=np.float64)
    keep = [N_s, L_s, _f64(x), _f64(y), _f64(P0), _f64(p0_s), _f64(v0_s),
            None if seed_s is None else np.ascontiguousarray(seed_s, dtype=np.uint64)]
    h = _H()
    st = _lib.spv_batch_create(ctypes.byref(h), S, _ptr(keep[0]), _ptr(keep[1]), _ptr(keep[1]), _ptr(keep[2]),
                               _ptr(keep[3]), _ptr(keep[4]), _ptr(keep[5]), _ptr(keep[6]), _ptr(keep[7]),
                               ctypes.byref(params), stream if stream is not None else _current_stream())
    _check(st, "spv_batch_create")
    return h


def spv_get_size(h):
    S, N = _i32(), _i64()
    _check(_lib.spv_get_size(h, ctypes.byref(S), ctypes.byref(N)), "spv_get_size")
    return S.value, N.value


def spv_get_kcap(h):
    k = _i32()
    _check(_lib.spv_get_kcap(h, ctypes.byref(k)), "spv_get_kcap")
    return k.value


def spv_get_system_range(h, s):
    a, n = _i64(), _i64()
    _check(_lib.spv_get_system_range(h, int(s), ctypes.byref(a), ctypes.byref(n)), "spv_get_system_range")
    return a.value, n.value


def spv_get_system_box(h, s):
    Lx, Ly, q = _d(), _d(), _i32()
    _check(_lib.spv_get_system_box(h, int(s), ctypes.byref(Lx), ctypes.byref(Ly), ctypes.byref(q)),
           "spv_get_system_box")
    return Lx.value, Ly.value, q.value


def spv_get_system_observables(h, s):
    E, q, a = _d(), _d(), _d()
    _check(_lib.spv_get_system_observables(h, int(s), ctypes.byref(E), ctypes.byref(q), ctypes.byref(a)),
           "spv_get_system_observables")
    return E.value, q.value, a.value


def spv_step(h, nsteps):
    _check(_lib.spv_step(h, int(nsteps)), "spv_step")


def spv_get_box(h):
    Lx, Ly, q = _d(), _d(), _i32()
    _check(_lib.spv_get_box(h, ctypes.byref(Lx), ctypes.byref(Ly), ctypes.byref(q)), "spv_get_box")
    return Lx.value, Ly.value, q.value


def spv_get_positions(h, x, y):
    _check(_lib.spv_get_positions(h, _ptr(x), _ptr(y)), "spv_get_positions")


def spv_get_directors(h, th):
    _check(_lib.spv_get_directors(h, _ptr(th)), "spv_get_directors")


def spv_get_forces(h, fx, fy):
    _check(_lib.spv_get_forces(h, _ptr(fx), _ptr(fy)), "spv_get_forces")


def spv_get_geometry(h, A, P):
    _check(_lib.spv_get_geometry(h, _ptr(A), _ptr(P)), "spv_get_geometry")


def spv_get_neighbors(h, N):
    off = np.zeros(N + 1, dtype=np.int32)
    need = _i64()
    st = _lib.spv_get_neighbors(h, _ptr(off), None, 0, ctypes.byref(need))
    if st not in (SPV_OK, SPV_ECAPACITY):
        _check(st, "spv_get_neighbors")
    nbr = np.zeros(max(int(need.value), 1), dtype=np.int32)
    _check(_lib.spv_get_neighbors(h, _ptr(off), _ptr(nbr), int(need.value), ctypes.byref(need)),
           "spv_get_neighbors")
    return off, nbr[: int(need.value)]


def spv_debug_set_ring(h, cell, nbr):
    nbr = np.ascontiguousarray(nbr, dtype=np.int32)
    _check(_lib.spv_debug_set_ring(h, int(cell), len(nbr), _ptr(nbr)), "spv_debug_set_ring")


def spv_get_observables(h):
    E, q, a = _d(), _d(), _d()
    cnt = np.zeros(13, dtype=np.int64)
    _check(_lib.spv_get_observables(h, ctypes.byref(E), ctypes.byref(q), ctypes.byref(a), _ptr(cnt)),
           "spv_get_observables")
    return E.value, q.value, a.value, cnt


def spv_save_state(h):
    """The handle's state as a uint8 array (host)."""
    need = _i64()
    st = _lib.spv_save_state(h, None, 0, ctypes.byref(need))
    if st != SPV_ECAPACITY:
        _check(st, "spv_save_state")
    buf = np.zeros(int(need.value), dtype=np.uint8)
    _check(_lib.spv_save_state(h, _ptr(buf), int(need.value), ctypes.byref(need)), "spv_save_state")
    return buf


def spv_load_state(h, buf):
    buf = np.ascontiguousarray(buf, dtype=np.uint8)
    _check(_lib.spv_load_state(h, _ptr(buf), int(buf.size)), "spv_load_state")


def spv_get_tuning(h):
    t = Tuning()
    _check(_lib.spv_get_tuning(h, ctypes.byref(t)), "spv_get_tuning")
    return t.as_dict()


def spv_set_timing(h, enable):
    _check(_lib.spv_set_timing(h, int(bool(enable))), "spv_set_timing")


def spv_kernel_time(h, which):
    ms, n = _d(), _i64()
    _check(_lib.spv_kernel_time(h, int(which), ctypes.byref(ms), ctypes.byref(n)), "spv_kernel_time")
    return ms.value, n.value


def spv_traj_forward(h, T, ckpt_every):
    Q = _d()
    _check(_lib.spv_traj_forward(h, int(T), int(ckpt_every), ctypes.byref(Q)), "spv_traj_forward")
    return Q.value


def spv_traj_backward(h, dQ, out):
    _check(_lib.spv_traj_backward(h, float(dQ), _ptr(out)), "spv_traj_backward")


def spv_force_tangent(h, vx, vy, fx, fy):
    keep = [_f64(vx), _f64(vy)]
    _check(_lib.spv_force_tangent(h, _ptr(keep[0]), _ptr(keep[1]), _ptr(fx), _ptr(fy)), "spv_force_tangent")


def spv_force_tangent_static(h, vx, vy, fx, fy):
    """No-allocation variant: all four arrays are device tensors (float64,
    contiguous); the result is written on the handle's stream."""
    _check(_lib.spv_force_tangent_static(h, _ptr(vx), _ptr(vy), _ptr(fx), _ptr(fy)), "spv_force_tangent_static")


def spv_destroy(h):
    _check(_lib.spv_destroy(h), "spv_destroy")


# ------------------------------------------------------------------ convenience
class System:
    """One SPV system (or a batch, see `System.batch`) on the current HIP
    device (see include/spv.h)."""

    def __init__(self, x, y, Lx, Ly, *, p0=3.8, A0=None, P0=None, theta0=None, params=None, stream=None,
                 _handle=None):
        self.params = params if params is not None else Params()
        if _handle is not None:
            self.h = _handle
            self.N = spv_get_size(self.h)[1]
            return
        self.N = len(x)
        self.h = spv_create(self.N, x, y, Lx, Ly, A0=A0, P0=P0, p0=p0, theta0=theta0, params=self.params,
                            stream=stream)

    @classmethod
    def batch(cls, N_s, L_s, x, y, p0_s, v0_s=None, seed_s=None, P0=None, params=None, stream=None):
        params = params if params is not None else Params()
        h = spv_batch_create(N_s, L_s, x, y, p0_s, v0_s=v0_s, seed_s=seed_s, P0=P0, params=params, stream=stream)
        return cls(None, None, None, None, params=params, _handle=h)

    def size(self):
        return spv_get_size(self.h)

    def kcap(self):
        return spv_get_kcap(self.h)

    def system_range(self, s):
        return spv_get_system_range(self.h, s)

    def system_box(self, s):
        return spv_get_system_box(self.h, s)

    def system_observables(self, s):
        return spv_get_system_observables(self.h, s)

    def step(self, n=1):
        spv_step(self.h, n)

    def box(self):
        return spv_get_box(self.h)

    def positions(self):
        x, y = np.zeros(self.N), np.zeros(self.N)
        spv_get_positions(self.h, x, y)
        return x, y

    def directors(self):
        th = np.zeros(self.N)
        spv_get_directors(self.h, th)
        return th

    def forces(self):
        fx, fy = np.zeros(self.N), np.zeros(self.N)
        spv_get_forces(self.h, fx, fy)
        return fx, fy

    def geometry(self):
        A, P = np.zeros(self.N), np.zeros(self.N)
        spv_get_geometry(self.h, A, P)
        return A, P

    def neighbors(self):
        return spv_get_neighbors(self.h, self.N)

    def debug_set_ring(self, cell, nbr):
        """Overwrite one cell's ring (fault injection for tests)."""
        spv_debug_set_ring(self.h, cell, nbr)

    def observables(self):
        return spv_get_observables(self.h)

    def tuning(self):
        return spv_get_tuning(self.h)

    def save_state(self):
        return spv_save_state(self.h)

    def load_state(self, buf):
        spv_load_state(self.h, buf)

    def traj_forward(self, T, ckpt_every):
        return spv_traj_forward(self.h, T, ckpt_every)

    def traj_backward(self, dQ=1.0, out=None):
        """dQ * dQ/dp0 (tag order) into `out` (a float64 numpy array or
        device tensor of N entries; a new numpy array when None)."""
        g = np.zeros(self.N) if out is None else out
        spv_traj_backward(self.h, dQ, g)
        return g

    def force_tangent(self, vx, vy):
        fx, fy = np.zeros(self.N), np.zeros(self.N)
        spv_force_tangent(self.h, vx, vy, fx, fy)
        return fx, fy

    def close(self):
        if self.h:
            spv_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------ active vertex model
def spv_avm_create(Nc, Nv, vx, vy, cell_off, cell_vtx, Lx, Ly, A0=None, P0=None, p0=3.8, theta0=None, params=None,
                   stream=None):
    params = params if params is not None else AvmParams()
    keep = [_f64(vx), _f64(vy), np.ascontiguousarray(cell_off, dtype=np.int32),
            np.ascontiguousarray(cell_vtx, dtype=np.int32), _f64(A0), _f64(P0), _f64(theta0)]
    h = _H()
    st = _lib.spv_avm_create(ctypes.byref(h), int(Nc), int(Nv), _ptr(keep[0]), _ptr(keep[1]), _ptr(keep[2]),
                             _ptr(keep[3]), float(Lx), float(Ly), _ptr(keep[4]), _ptr(keep[5]), float(p0),
                             _ptr(keep[6]), ctypes.byref(params), stream if stream is not None else _current_stream())
    _check(st, "spv_avm_create")
    return h


def spv_avm_step(h, n):
    _check(_lib.spv_avm_step(h, int(n)), "spv_avm_step")


def spv_avm_get_vertices(h, vx, vy):
    _check(_lib.spv_avm_get_vertices(h, _ptr(vx), _ptr(vy)), "spv_avm_get_vertices")


def spv_avm_get_forces(h, fx, fy):
    _check(_lib.spv_avm_get_forces(h, _ptr(fx), _ptr(fy)), "spv_avm_get_forces")


def spv_avm_get_directors(h, theta):
    _check(_lib.spv_avm_get_directors(h, _ptr(theta)), "spv_avm_get_directors")


def spv_avm_get_geometry(h, A, P):
    _check(_lib.spv_avm_get_geometry(h, _ptr(A), _ptr(P)), "spv_avm_get_geometry")


def spv_avm_get_cells(h, Nc, Nv):
    off = np.zeros(Nc + 1, dtype=np.int32)
    cv = np.zeros(3 * Nv, dtype=np.int32)
    need = _i64()
    _check(_lib.spv_avm_get_cells(h, _ptr(off), _ptr(cv), len(cv), ctypes.byref(need)), "spv_avm_get_cells")
    return off, cv[: int(need.value)]


def spv_avm_get_observables(h):
    E, q = _d(), _d()
    cnt = np.zeros(6, dtype=np.int64)
    _check(_lib.spv_avm_get_observables(h, ctypes.byref(E), ctypes.byref(q), _ptr(cnt)), "spv_avm_get_observables")
    return E.value, q.value, cnt


def spv_avm_destroy(h):
    _check(_lib.spv_avm_destroy(h), "spv_avm_destroy")


def spv_voronoi_network(h, N):
    vx, vy = np.zeros(2 * N), np.zeros(2 * N)
    off = np.zeros(N + 1, dtype=np.int32)
    cv = np.zeros(6 * N, dtype=np.int32)
    _check(_lib.spv_voronoi_network(h, _ptr(vx), _ptr(vy), _ptr(off), _ptr(cv)), "spv_voronoi_network")
    return vx, vy, off, cv


class AVM:
    """An active vertex model on the current HIP device (see include/spv.h)."""

    def __init__(self, vx, vy, cell_off, cell_vtx, Lx, Ly, A0=None, P0=None, p0=3.8, theta0=None, params=None):
        self.Nc, self.Nv = len(cell_off) - 1, len(vx)
        self.h = spv_avm_create(self.Nc, self.Nv, vx, vy, cell_off, cell_vtx, Lx, Ly, A0, P0, p0, theta0, params)

    @classmethod
    def from_voronoi(cls, system, A0=None, P0=None, p0=3.8, theta0=None, params=None):
        vx, vy, off, cv = spv_voronoi_network(system.h, system.N)
        Lx, Ly, _ = system.box()
        return cls(vx, vy, off, cv, Lx, Ly, A0, P0, p0, theta0, params)

    def step(self, n):
        spv_avm_step(self.h, n)

    def vertices(self):
        x, y = np.zeros(self.Nv), np.zeros(self.Nv)
        spv_avm_get_vertices(self.h, x, y)
        return x, y

    def forces(self):
        x, y = np.zeros(self.Nv), np.zeros(self.Nv)
        spv_avm_get_forces(self.h, x, y)
        return x, y

    def directors(self):
        t = np.zeros(self.Nc)
        spv_avm_get_directors(self.h, t)
        return t

    def geometry(self):
        A, P = np.zeros(self.Nc), np.zeros(self.Nc)
        spv_avm_get_geometry(self.h, A, P)
        return A, P

    def cells(self):
        return spv_avm_get_cells(self.h, self.Nc, self.Nv)

    def observables(self):
        return spv_avm_get_observables(self.h)

    def close(self):
        if self.h:
            spv_avm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
