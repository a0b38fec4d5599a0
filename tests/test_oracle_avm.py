"""Pins of the oracle's active vertex model (Eq. 1 over polygon cells, App. A
vertex forces, Eq. 4 motion, Sec. II.D T1 transitions), each against
something other than the oracle itself: central finite differences of the
energy, the regular honeycomb's closed forms and zero force, exact motion
without forces, a T1 built by hand, torus invariants, gradient flow, and
the Voronoi construction's equidistance."""
import math

import numpy as np
import pytest

import oracle
from paper_1702_02939_amd import inputs


def _network(n, seed, jitter=0.0):
    L = math.sqrt(n)
    x, y = inputs.uniform_positions(n, L, L, seed)
    xq, yq, Lx, Ly, q = oracle.prepare(x, y, L, L)
    vx, vy, off, cv = oracle.voronoi_network(xq, yq, Lx, Ly, q)
    if jitter:
        rng = np.random.default_rng(seed + 1)
        vx = (vx + jitter * rng.standard_normal(len(vx))) % Lx
        vy = (vy + jitter * rng.standard_normal(len(vy))) % Ly
    return vx, vy, off, cv, Lx, Ly, q, (xq, yq)


def _energy(vx, vy, Lx, Ly, off, cv, A0, P0, KA=1.0, KP=1.0):
    A, P = oracle.avm_geometry(vx, vy, Lx, Ly, off, cv)
    return float(np.sum(KA * (A - A0) ** 2 + KP * (P - P0) ** 2))


def _check_network(vx, off, cv):
    nc, nv = len(off) - 1, len(vx)
    assert nv == 2 * nc and off[-1] == 3 * nv  # torus: V = 2F, each vertex in three cells
    counts = np.bincount(cv, minlength=nv)
    assert np.all(counts == 3)
    directed = set()
    for c in range(nc):
        v = cv[off[c]:off[c + 1]]
        for m in range(len(v)):
            e = (int(v[m]), int(v[(m + 1) % len(v)]))
            assert e not in directed  # every directed edge once (consistent orientation)
            directed.add(e)
    for a, b in directed:
        assert (b, a) in directed  # every edge shared by two cells, in opposite directions


def test_forces_match_finite_differences():
    vx, vy, off, cv, Lx, Ly, _, _ = _network(120, 201, jitter=0.05)
    rng = np.random.default_rng(7)
    A0 = rng.uniform(0.8, 1.2, len(off) - 1)
    P0 = rng.uniform(3.5, 4.0, len(off) - 1)
    fx, fy = oracle.avm_forces(vx, vy, Lx, Ly, off, cv, A0, P0, KA=1.3, KP=0.7)
    h = 1e-6
    scale = max(np.abs(fx).max(), np.abs(fy).max())
    for v in rng.choice(len(vx), 25, replace=False):
        for f, arr in ((fx, vx), (fy, vy)):
            p, m = arr.copy(), arr.copy()
            p[v] += h
            m[v] -= h
            args = (vx, vy) if arr is vx else (vx, vy)
            if arr is vx:
                ep = _energy(p, vy, Lx, Ly, off, cv, A0, P0, 1.3, 0.7)
                em = _energy(m, vy, Lx, Ly, off, cv, A0, P0, 1.3, 0.7)
            else:
                ep = _energy(vx, p, Lx, Ly, off, cv, A0, P0, 1.3, 0.7)
                em = _energy(vx, m, Lx, Ly, off, cv, A0, P0, 1.3, 0.7)
            del args
            fd = -(ep - em) / (2 * h)
            assert abs(f[v] - fd) < 1e-7 * scale, (v, f[v], fd)
    # translation invariance
    assert abs(fx.sum()) < 1e-10 * scale * len(vx) and abs(fy.sum()) < 1e-10 * scale * len(vx)


def test_regular_honeycomb_closed_form_and_zero_force():
    a = 1.3
    x, y, Lx, Ly = inputs.hex_lattice(8, 10, a)
    xq, yq, Lx, Ly, q = oracle.prepare(x, y, Lx, Ly)
    vx, vy, off, cv = oracle.voronoi_network(xq, yq, Lx, Ly, q)
    _check_network(vx, off, cv)
    A, P = oracle.avm_geometry(vx, vy, Lx, Ly, off, cv)
    np.testing.assert_allclose(A, math.sqrt(3) / 2 * a * a, rtol=1e-12)
    np.testing.assert_allclose(P, 2 * math.sqrt(3) * a, rtol=1e-12)
    assert np.all(np.diff(off) == 6)
    for A0, P0 in ((1.0, 3.8), (2.5, 5.0)):
        fx, fy = oracle.avm_forces(vx, vy, Lx, Ly, off, cv, A0, P0)
        assert np.abs(fx).max() < 1e-10 and np.abs(fy).max() < 1e-10


def test_voronoi_vertices_are_circumcentres():
    vx, vy, off, cv, Lx, Ly, q, (xq, yq) = _network(150, 202)
    _check_network(vx, off, cv)
    A, _ = oracle.avm_geometry(vx, vy, Lx, Ly, off, cv)
    assert abs(A.sum() - Lx * Ly) < 1e-9 * Lx * Ly
    dist = {}
    for c in range(len(off) - 1):
        for v in cv[off[c]:off[c + 1]]:
            dx = (vx[v] - xq[c] + Lx / 2) % Lx - Lx / 2
            dy = (vy[v] - yq[c] + Ly / 2) % Ly - Ly / 2
            dist.setdefault(int(v), []).append(math.hypot(dx, dy))
    for v, d in dist.items():
        assert len(d) == 3 and max(d) - min(d) < 1e-9


def test_motion_without_forces_is_the_mean_director():
    vx, vy, off, cv, Lx, Ly, q, _ = _network(100, 203)
    th = np.full(len(off) - 1, 0.3)
    out = oracle.avm_run(vx, vy, th, Lx, Ly, q, off, cv, 1.0, 3.8, KA=0.0, KP=0.0, v0=0.5, Dr=0.0, dt=0.01,
                         l_t1=1e-9, l_new=2e-9, nsteps=1)
    dx = (out["vx"] - vx + Lx / 2) % Lx - Lx / 2
    dy = (out["vy"] - vy + Ly / 2) % Ly - Ly / 2
    grid = 2.0 ** -q
    assert np.abs(dx - 0.005 * math.cos(0.3)).max() <= grid and np.abs(dy - 0.005 * math.sin(0.3)).max() <= grid
    np.testing.assert_array_equal(out["theta"], th)


def test_single_t1_by_hand():
    # a honeycomb with one edge shrunk below the threshold (its two vertices
    # moved towards the midpoint); no motion (mu = v0 = 0)
    x, y, Lx, Ly = inputs.hex_lattice(6, 6, 1.0)
    xq, yq, Lx, Ly, q = oracle.prepare(x, y, Lx, Ly)
    vx, vy, off, cv = oracle.voronoi_network(xq, yq, Lx, Ly, q)
    v1, v2 = int(cv[off[7]]), int(cv[off[7] + 1])  # an edge of cell 7
    mx = vx[v1] + 0.5 * ((vx[v2] - vx[v1] + Lx / 2) % Lx - Lx / 2)
    my = vy[v1] + 0.5 * ((vy[v2] - vy[v1] + Ly / 2) % Ly - Ly / 2)
    ex = (vx[v2] - vx[v1] + Lx / 2) % Lx - Lx / 2
    ey = (vy[v2] - vy[v1] + Ly / 2) % Ly - Ly / 2
    s = 0.01 / math.hypot(ex, ey)
    vx, vy = vx.copy(), vy.copy()
    vx[v1], vy[v1] = (mx - s * ex) % Lx, (my - s * ey) % Ly
    vx[v2], vy[v2] = (mx + s * ex) % Lx, (my + s * ey) % Ly
    scale = 2.0 ** q
    vx, vy = np.rint(vx * scale) / scale, np.rint(vy * scale) / scale
    before = oracle.canonical_cells(off, cv)
    cells_with = lambda cl, v: {c for c, t in enumerate(cl) if v in t}  # noqa: E731
    shared = cells_with(before, v1) & cells_with(before, v2)
    ends = (cells_with(before, v1) | cells_with(before, v2)) - shared
    assert len(shared) == 2 and len(ends) == 2
    out = oracle.avm_run(vx, vy, np.zeros(len(off) - 1), Lx, Ly, q, off, cv, 1.0, 3.8, mu=0.0, v0=0.0, Dr=0.0,
                         l_t1=0.05, l_new=0.2, nsteps=1)
    assert out["t1"] == 1
    after = oracle.canonical_cells(out["cell_off"], out["cell_vtx"])
    for c in shared:
        assert len(after[c]) == len(before[c]) - 1
    for c in ends:
        assert len(after[c]) == len(before[c]) + 1 and v1 in after[c] and v2 in after[c]
    _check_network(out["vx"], out["cell_off"], out["cell_vtx"])
    nx = (out["vx"][v2] - out["vx"][v1] + Lx / 2) % Lx - Lx / 2
    ny = (out["vy"][v2] - out["vy"][v1] + Ly / 2) % Ly - Ly / 2
    grid = 2.0 ** -q
    assert abs(math.hypot(nx, ny) - 0.2) < 4 * grid       # the new length
    assert abs(nx * ex + ny * ey) < 1e-10                # perpendicular to the old edge
    nmx = (out["vx"][v1] + 0.5 * nx) % Lx
    nmy = (out["vy"][v1] + 0.5 * ny) % Ly
    assert abs((nmx - mx + Lx / 2) % Lx - Lx / 2) < 4 * grid and abs((nmy - my + Ly / 2) % Ly - Ly / 2) < 4 * grid
    A, _ = oracle.avm_geometry(out["vx"], out["vy"], Lx, Ly, out["cell_off"], out["cell_vtx"])
    assert abs(A.sum() - Lx * Ly) < 1e-9 * Lx * Ly


def test_dynamics_keep_a_valid_network():
    vx, vy, off, cv, Lx, Ly, q, _ = _network(300, 204)
    out = oracle.avm_run(vx, vy, oracle.theta0(5, len(off) - 1), Lx, Ly, q, off, cv, 1.0, 3.9, v0=0.2, Dr=1.0,
                         dt=0.01, seed=5, l_t1=0.04, l_new=0.06, nsteps=150)
    assert out["t1"] > 0
    _check_network(out["vx"], out["cell_off"], out["cell_vtx"])
    A, _ = oracle.avm_geometry(out["vx"], out["vy"], Lx, Ly, out["cell_off"], out["cell_vtx"])
    assert abs(A.sum() - Lx * Ly) < 1e-9 * Lx * Ly and np.all(A > 0)


def test_gradient_flow_decreases_energy():
    vx, vy, off, cv, Lx, Ly, q, _ = _network(200, 205, jitter=0.02)
    out = oracle.avm_run(vx, vy, np.zeros(len(off) - 1), Lx, Ly, q, off, cv, 1.0, 3.7, v0=0.0, Dr=0.0, dt=0.005,
                         l_t1=1e-9, l_new=2e-9, nsteps=60)
    assert out["t1"] == 0
    assert np.all(np.diff(out["E"]) <= 1e-12 * out["E"][0])
