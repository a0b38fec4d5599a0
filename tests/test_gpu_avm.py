"""The active vertex model's HIP path (through the C-ABI) against the oracle.

Bar: cell lists (topology after T1 rounds) bit-exact in canonical form;
areas and perimeters within 1e-12 relative; forces within 1e-10 of
max(max|F|, K_P P0); vertex positions after one step from a common state
within 1e-12 (both sides round onto the same grid; one grid unit apart at
most where the two force evaluations round differently); directors within
1e-12 (libm and device sincos / log differ in the last bits)."""
import math

import numpy as np
import pytest

import oracle
from paper_1702_02939_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def spv():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    from paper_1702_02939_amd import spv as mod
    return mod


def _network(n, seed, jitter=0.0):
    L = math.sqrt(n)
    x, y = inputs.uniform_positions(n, L, L, seed)
    xq, yq, Lx, Ly, q = oracle.prepare(x, y, L, L)
    vx, vy, off, cv = oracle.voronoi_network(xq, yq, Lx, Ly, q)
    if jitter:
        rng = np.random.default_rng(seed + 1)
        vx = (vx + jitter * rng.standard_normal(len(vx))) % Lx
        vy = (vy + jitter * rng.standard_normal(len(vy))) % Ly
        s = 2.0 ** q
        vx, vy = np.rint(vx * s) % np.rint(Lx * s) / s, np.rint(vy * s) % np.rint(Ly * s) / s
    return vx, vy, off, cv, Lx, Ly, q, (xq, yq)


def _canon(off, cv):
    return oracle.canonical_cells(off, cv)


def test_geometry_and_forces_match_oracle(spv):
    vx, vy, off, cv, Lx, Ly, q, _ = _network(2000, 301, jitter=0.03)
    rng = np.random.default_rng(3)
    nc = len(off) - 1
    A0 = rng.uniform(0.8, 1.2, nc)
    P0 = rng.uniform(3.5, 4.0, nc)
    a = spv.AVM(vx, vy, off, cv, Lx, Ly, A0=A0, P0=P0, params=spv.AvmParams(KA=1.3, KP=0.7))
    gx, gy = a.vertices()
    assert np.array_equal(gx, vx) and np.array_equal(gy, vy)
    A, P = oracle.avm_geometry(vx, vy, Lx, Ly, off, cv)
    gA, gP = a.geometry()
    np.testing.assert_allclose(gA, A, rtol=1e-12)
    np.testing.assert_allclose(gP, P, rtol=1e-12)
    fx, fy = oracle.avm_forces(vx, vy, Lx, Ly, off, cv, A0, P0, 1.3, 0.7)
    gfx, gfy = a.forces()
    scale = max(np.abs(fx).max(), np.abs(fy).max(), 0.7 * P0.max())
    err = max(np.abs(gfx - fx).max(), np.abs(gfy - fy).max())
    assert err <= 1e-10 * scale, err / scale
    goff, gcv = a.cells()
    assert _canon(goff, gcv) == _canon(off, cv)
    a.close()


def test_honeycomb_zero_force(spv):
    x, y, Lx, Ly = inputs.hex_lattice(10, 12, 1.1)
    xq, yq, Lx, Ly, q = oracle.prepare(x, y, Lx, Ly)
    vx, vy, off, cv = oracle.voronoi_network(xq, yq, Lx, Ly, q)
    a = spv.AVM(vx, vy, off, cv, Lx, Ly, p0=3.9)
    fx, fy = a.forces()
    assert np.abs(fx).max() < 1e-10 and np.abs(fy).max() < 1e-10
    a.close()


def _compare_state(a, ref, Lx, Ly, q, tol_pos=1e-12):
    gx, gy = a.vertices()
    grid = 2.0 ** -q
    dx = np.abs((gx - ref["vx"] + Lx / 2) % Lx - Lx / 2)
    dy = np.abs((gy - ref["vy"] + Ly / 2) % Ly - Ly / 2)
    assert max(dx.max(), dy.max()) <= max(tol_pos, grid), (dx.max(), dy.max())
    np.testing.assert_allclose(a.directors(), ref["theta"], rtol=0, atol=1e-12)
    goff, gcv = a.cells()
    assert _canon(goff, gcv) == _canon(ref["cell_off"], ref["cell_vtx"])


@pytest.mark.parametrize("n,p0,v0", [(400, 3.8, 0.1), (1500, 3.95, 0.3)])
def test_steps_match_oracle(spv, n, p0, v0):
    """Several steps with T1 transitions from a common start (topology
    exact, positions at the grid), then one step from the device's state
    after 60 steps (the oracle continuing with the same noise counter)."""
    vx, vy, off, cv, Lx, Ly, q, _ = _network(n, 302 + n)
    th = oracle.theta0(11, n)
    prm = dict(KA=1.0, KP=1.0, mu=1.0, v0=v0, Dr=1.0, dt=0.01, seed=11)
    a = spv.AVM(vx, vy, off, cv, Lx, Ly, p0=p0, theta0=th,
                params=spv.AvmParams(t1_length=0.04, t1_new_length=0.06, **prm))
    a.step(5)
    ref = oracle.avm_run(vx, vy, th, Lx, Ly, q, off, cv, 1.0, p0, l_t1=0.04, l_new=0.06, nsteps=5, **prm)
    _compare_state(a, ref, Lx, Ly, q)
    a.step(55)
    E, qbar, cnt = a.observables()
    assert cnt[0] == 60 and cnt[1] > 0, cnt  # transitions happened
    assert cnt[4] > 0 and cnt[5] >= 1, cnt   # captured batches replayed; sorted at creation
    gx, gy = a.vertices()
    goff, gcv = a.cells()
    gth = a.directors()
    ref = oracle.avm_run(gx, gy, gth, Lx, Ly, q, goff, gcv, 1.0, p0, l_t1=0.04, l_new=0.06, step0=60, nsteps=1,
                         **prm)
    a.step(1)
    _compare_state(a, ref, Lx, Ly, q)
    E2, q2, _ = a.observables()
    assert abs(E2 - ref["E"][-1]) < 1e-9 * abs(ref["E"][-1]) and abs(q2 - ref["qbar"][-1]) < 1e-12 * q2
    a.close()


def test_many_t1_rounds_use_host_rounds(spv):
    """A large threshold makes many edges qualify at once, so that steps need
    more T1 rounds than the device runs (counted) and the host finishes them;
    the topology still equals the oracle's."""
    n = 600
    vx, vy, off, cv, Lx, Ly, q, _ = _network(n, 303)
    th = oracle.theta0(12, n)
    prm = dict(KA=1.0, KP=1.0, mu=1.0, v0=0.05, Dr=1.0, dt=0.01, seed=12)
    a = spv.AVM(vx, vy, off, cv, Lx, Ly, p0=3.8, theta0=th,
                params=spv.AvmParams(t1_length=0.15, t1_new_length=0.2, **prm))
    a.step(3)
    _, _, cnt = a.observables()
    ref = oracle.avm_run(vx, vy, th, Lx, Ly, q, off, cv, 1.0, 3.8, l_t1=0.15, l_new=0.2, nsteps=3, **prm)
    assert cnt[1] == ref["t1"] and cnt[3] > 0, (cnt, ref["t1"], ref["t1_rounds"])
    _compare_state(a, ref, Lx, Ly, q)
    a.close()


def test_voronoi_network_matches_oracle(spv):
    n = 1000
    L = math.sqrt(n)
    x, y = inputs.uniform_positions(n, L, L, 304)
    s = spv.System(x, y, L, L)
    gx, gy = s.positions()
    Lx, Ly, q = s.box()
    vx, vy, off, cv = oracle.voronoi_network(gx, gy, Lx, Ly, q)
    a = spv.AVM.from_voronoi(s, p0=3.8)
    s.close()
    goff, gcv = a.cells()
    assert np.array_equal(goff, off) and np.array_equal(gcv, cv)
    hx, hy = a.vertices()
    grid = 2.0 ** -q
    assert np.abs(hx - vx).max() <= grid and np.abs(hy - vy).max() <= grid
    a.close()


def test_invalid_networks_rejected(spv):
    vx, vy, off, cv, Lx, Ly, q, _ = _network(50, 305)
    bad = cv.copy()
    bad[0], bad[1] = bad[1], bad[0]  # one cell's orientation broken
    with pytest.raises(spv.SPVError) as ei:
        spv.AVM(vx, vy, off, bad, Lx, Ly)
    assert ei.value.status == spv.SPV_EINVAL
    with pytest.raises(spv.SPVError) as ei:
        spv.AVM(vx[:-2], vy[:-2], off, cv, Lx, Ly)
    assert ei.value.status == spv.SPV_EINVAL


@pytest.mark.parametrize("resort_every,bin_order", [(16, 0), (8, 1), (1, 0)])
def test_memory_order_is_invisible(spv, resort_every, bin_order):
    """Re-sorting vertices and cells (any interval, Hilbert or row-major
    bins) changes no result: positions, directors and topology after 120
    steps with transitions are bitwise those of a run that keeps the
    caller's order; the network comes in randomly relabelled, so that the
    memory order after the first sort differs from the labels."""
    vx, vy, off, cv, Lx, Ly, q, _ = _network(1200, 310)
    rng = np.random.default_rng(5)
    nc, nv = len(off) - 1, len(vx)
    cp, vp = rng.permutation(nc), rng.permutation(nv)  # new label of old cell / vertex
    rows = [cv[off[c]:off[c + 1]] for c in np.argsort(cp)]
    off2 = np.concatenate([[0], np.cumsum([len(r) for r in rows])]).astype(np.int32)
    cv2 = vp[np.concatenate(rows)].astype(np.int32)
    vx2, vy2 = vx[np.argsort(vp)], vy[np.argsort(vp)]
    prm = dict(KA=1.0, KP=1.0, mu=1.0, v0=0.3, Dr=1.0, dt=0.01, seed=21, t1_length=0.04, t1_new_length=0.06)
    out = []
    for re, bo in ((-1, 0), (resort_every, bin_order)):
        a = spv.AVM(vx2, vy2, off2, cv2, Lx, Ly, p0=3.95, params=spv.AvmParams(resort_every=re, bin_order=bo, **prm))
        a.step(120)
        _, _, cnt = a.observables()
        out.append((a.vertices(), a.directors(), a.cells(), cnt))
        a.close()
    (v1, t1, c1, n1), (v2, t2, c2, n2) = out
    assert n1[1] > 0 and n1[1] == n2[1] and n1[2] == n2[2], (n1, n2)
    assert n1[5] == 0 and n2[5] >= 120 // resort_every, (n1, n2)
    assert np.array_equal(v1[0], v2[0]) and np.array_equal(v1[1], v2[1])
    assert np.array_equal(t1, t2)
    assert np.array_equal(c1[0], c2[0]) and np.array_equal(c1[1], c2[1])


def test_error_paths(spv):
    """Bad parameters are refused at creation; an update that overflows is
    SPV_ENONFINITE and stays the handle's answer (its stored vertices are
    the last finite ones)."""
    vx, vy, off, cv, Lx, Ly, q, _ = _network(300, 306)
    for bad in (dict(resort_every=-2), dict(bin_order=2), dict(t1_length=0.0), dict(t1_length=0.1, t1_new_length=0.05),
                dict(dt=0.0)):
        with pytest.raises(spv.SPVError) as ei:
            spv.AVM(vx, vy, off, cv, Lx, Ly, params=spv.AvmParams(**bad))
        assert ei.value.status == spv.SPV_EINVAL, bad
    a = spv.AVM(vx, vy, off, cv, Lx, Ly, params=spv.AvmParams(v0=1.0, dt=1e300))
    with pytest.raises(spv.SPVError) as ei:
        a.step(1)
    assert ei.value.status == spv.SPV_ENONFINITE
    with pytest.raises(spv.SPVError) as ei:
        a.step(1)
    assert ei.value.status == spv.SPV_ENONFINITE
    gx, gy = a.vertices()
    assert np.isfinite(gx).all() and np.isfinite(gy).all()
    a.close()


@pytest.mark.parametrize("name", ["avm_n100k", "avm_n1m"])
def test_benchmark_workloads_one_step_from_device_state(spv, name):
    """The benchmark's active vertex model workloads in its launch
    configuration (the Voronoi network of the random points built by the
    library, Hilbert re-sort, batches replayed from graphs, the adaptive
    device rounds), 104 steps in as the benchmark times them; then one step
    from the device's state on both sides: topology exact, vertices within a
    grid unit, directors within 1e-12, E and q-bar."""
    w = inputs.WORKLOADS[name]
    n, L = w["N"], w["L"]
    x, y = inputs.uniform_positions(n, L, L, w["seed"])
    s = spv.System(x, y, L, L)
    Lx, Ly, q = s.box()
    vx, vy, off, cv = spv.spv_voronoi_network(s.h, s.N)
    s.close()
    prm = dict(KA=1.0, KP=1.0, mu=w["mu"], v0=w["v0"], Dr=w["Dr"], dt=w["dt"], seed=w["seed"])
    a = spv.AVM(vx, vy, off, cv, Lx, Ly, p0=w["p0"],
                params=spv.AvmParams(t1_length=w["t1"], t1_new_length=w["t1_new"], **prm))
    a.step(104)
    _, _, cnt = a.observables()
    assert cnt[0] == 104 and cnt[1] > 0 and cnt[4] > 0 and cnt[5] >= 1, cnt
    gx, gy = a.vertices()
    goff, gcv = a.cells()
    gth = a.directors()
    ref = oracle.avm_run(gx, gy, gth, Lx, Ly, q, goff, gcv, 1.0, w["p0"], l_t1=w["t1"], l_new=w["t1_new"], step0=104,
                         nsteps=1, **prm)
    a.step(1)
    _compare_state(a, ref, Lx, Ly, q)
    E, qb, _ = a.observables()
    assert abs(E - ref["E"][-1]) < 1e-9 * abs(ref["E"][-1]) and abs(qb - ref["qbar"][-1]) < 1e-12 * qb
    a.close()
