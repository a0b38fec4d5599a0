"""Parity of the HIP path (through the C-ABI) with the CPU oracle.

Bar: neighbour rings bit-exact (same CCW order, same start); FP64 forces
within 1e-10 * max(max|F_oracle|, K_P P0) (per system); areas and perimeters
within 1e-12 relative; one-step positions within 1e-12; trajectory energy and
mean shape index within 1e-6 over short runs (they diverge chaotically later).
"""
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


def _compare_topology(sysm, x, y):
    Lx, Ly, q = sysm.box()
    off, ring, ntri, _ = oracle.triangulate(x, y, Lx, Ly, q)
    goff, gring = sysm.neighbors()
    assert ntri == 2 * len(x)
    assert np.array_equal(goff, off), "degrees differ"
    assert np.array_equal(gring, ring), "rings differ"
    return off, ring


def _compare_forces(sysm, x, y, off, ring, A0, P0, KA=1.0, KP=1.0):
    Lx, Ly, q = sysm.box()
    fx, fy = oracle.forces(x, y, Lx, Ly, off, ring, A0, P0, KA, KP)
    gfx, gfy = sysm.forces()
    scale = max(np.abs(np.concatenate([fx, fy])).max(), KP * np.max(P0))
    err = max(np.abs(gfx - fx).max(), np.abs(gfy - fy).max())
    assert err <= 1e-10 * scale, f"max |dF| = {err:.3e} (scale {scale:.3e})"
    A, P = oracle.geometry(x, y, Lx, Ly, off, ring)
    gA, gP = sysm.geometry()
    np.testing.assert_allclose(gA, A, rtol=1e-12, atol=0)
    np.testing.assert_allclose(gP, P, rtol=1e-12, atol=0)
    return err


def _random_case(n, seed, L=None):
    L = float(math.sqrt(n)) if L is None else L
    x, y = inputs.uniform_positions(n, L, L, seed)
    return x, y, L, L


CREATE_CASES = [
    ("uniform_256", lambda: _random_case(256, inputs.BASE_SEED + 1, 16.0)),
    ("uniform_1000", lambda: _random_case(1000, 31)),
    ("uniform_4099", lambda: _random_case(4099, 32)),
    ("uniform_20011", lambda: _random_case(20011, 33)),
    ("hex_12x12", lambda: inputs.hex_lattice(12, 12, 1.0)),
    ("square_10x10", lambda: inputs.square_lattice(10, 1.0)),
    ("rect_box_3000", lambda: (*inputs.uniform_positions(3000, 100.0, 30.0, 34), 100.0, 30.0)),
]


@pytest.mark.parametrize("name,make", CREATE_CASES, ids=[c[0] for c in CREATE_CASES])
def test_create_topology_and_forces(spv, name, make):
    x, y, Lx, Ly = make()
    n = len(x)
    sysm = spv.System(x, y, Lx, Ly, p0=3.8, params=spv.Params(v0=0.05, seed=1))
    gx, gy = sysm.positions()
    xq, yq, _, _, _ = oracle.prepare(x, y, Lx, Ly)
    assert np.array_equal(gx, xq) and np.array_equal(gy, yq), "grid quantisation differs"
    off, ring = _compare_topology(sysm, gx, gy)
    if name.startswith("square"):
        # exactly at T1 points the perimeter gradient is undefined: geometry only
        Lxq, Lyq, _ = sysm.box()
        A, P = oracle.geometry(gx, gy, Lxq, Lyq, off, ring)
        gA, gP = sysm.geometry()
        np.testing.assert_allclose(gA, A, rtol=1e-12)
        np.testing.assert_allclose(gP, P, rtol=1e-12)
    else:
        _compare_forces(sysm, gx, gy, off, ring, 1.0, 3.8)
    E, qbar, sumA, cnt = sysm.observables()
    Lxq, Lyq, _ = sysm.box()
    assert abs(sumA - Lxq * Lyq) < 1e-9 * Lxq * Lyq
    assert cnt[7] == 0
    sysm.close()


def test_hex_lattice_zero_force(spv):
    x, y, Lx, Ly = inputs.hex_lattice(16, 16, 1.0)
    sysm = spv.System(x, y, Lx, Ly, p0=3.0, params=spv.Params())
    fx, fy = sysm.forces()
    assert np.abs(fx).max() < 1e-10 and np.abs(fy).max() < 1e-10
    A, P = sysm.geometry()
    np.testing.assert_allclose(A, math.sqrt(3) / 2, rtol=1e-12)
    np.testing.assert_allclose(P, 2 * math.sqrt(3), rtol=1e-12)
    sysm.close()


def test_per_cell_targets_and_moduli(spv):
    n = 2000
    x, y, Lx, Ly = _random_case(n, 41)
    rng = np.random.default_rng(5)
    A0 = rng.uniform(0.8, 1.2, n)
    P0 = rng.uniform(3.4, 4.2, n)
    prm = spv.Params(KA=1.7, KP=0.6)
    sysm = spv.System(x, y, Lx, Ly, A0=A0, P0=P0, params=prm)
    gx, gy = sysm.positions()
    off, ring = _compare_topology(sysm, gx, gy)
    _compare_forces(sysm, gx, gy, off, ring, A0, P0, 1.7, 0.6)
    sysm.close()


def test_one_step_parity(spv):
    n = 1024
    x, y, Lx, Ly = _random_case(n, 42)
    th0 = np.random.default_rng(6).uniform(0, 2 * math.pi, n)
    mu, v0, Dr, dt, seed = 1.0, 0.1, 1.0, 0.01, 99
    sysm = spv.System(x, y, Lx, Ly, p0=3.9, theta0=th0, params=spv.Params(mu=mu, v0=v0, Dr=Dr, dt=dt, seed=seed))
    Lxq, Lyq, q = sysm.box()
    xq, yq, _, _, _ = oracle.prepare(x, y, Lx, Ly)
    out = oracle.run(xq, yq, th0, Lxq, Lyq, q, 1.0, 3.9, mu=mu, v0=v0, Dr=Dr, dt=dt, seed=seed, nsteps=1,
                     want_rings=True, want_forces=True)
    sysm.step(1)
    gx, gy = sysm.positions()
    dx = (gx - out["x"] + Lxq / 2) % Lxq - Lxq / 2
    dy = (gy - out["y"] + Lyq / 2) % Lyq - Lyq / 2
    assert np.abs(dx).max() <= 1e-12 and np.abs(dy).max() <= 1e-12
    np.testing.assert_allclose(sysm.directors(), out["theta"], rtol=0, atol=1e-12)
    # topology and forces at the new state, evaluated by the oracle on the GPU positions
    off, ring = _compare_topology(sysm, gx, gy)
    _compare_forces(sysm, gx, gy, off, ring, 1.0, 3.9)
    sysm.close()


def test_default_directors_match_counter_rule(spv):
    n = 500
    x, y, Lx, Ly = _random_case(n, 43)
    sysm = spv.System(x, y, Lx, Ly, params=spv.Params(seed=1234))
    np.testing.assert_allclose(sysm.directors(), oracle.theta0(1234, n), rtol=0, atol=1e-14)
    sysm.close()


@pytest.mark.parametrize("n,p0,v0,steps,every", [(256, 3.8, 0.05, 300, 50), (4096, 3.9, 0.1, 200, 40)])
def test_repair_keeps_exact_topology(spv, n, p0, v0, steps, every):
    """After every block of steps the device topology equals the oracle's
    from-scratch triangulation of the device positions, and forces agree."""
    L = 16.0 if n == 256 else math.sqrt(n)
    x, y = inputs.uniform_positions(n, L, L, inputs.BASE_SEED + 1 if n == 256 else 44)
    sysm = spv.System(x, y, L, L, p0=p0, params=spv.Params(v0=v0, Dr=1.0, dt=0.01, seed=3, resort_every=25))
    done = 0
    while done < steps:
        sysm.step(every)
        done += every
        gx, gy = sysm.positions()
        off, ring = _compare_topology(sysm, gx, gy)
        _compare_forces(sysm, gx, gy, off, ring, 1.0, p0)
    E, qbar, sumA, cnt = sysm.observables()
    assert cnt[0] == steps and cnt[1] > 0 and cnt[7] == 0
    sysm.close()


def test_trajectory_energy_and_shape_index(spv):
    """spv_n256 workload: E and qbar per step against the oracle to 1e-6."""
    w = inputs.WORKLOADS["spv_n256"]
    n, L, T = w["N"], w["L"], 150
    x, y = inputs.uniform_positions(n, L, L, w["seed"])
    th0 = oracle.theta0(w["seed"], n)
    prm = spv.Params(mu=w["mu"], v0=w["v0"], Dr=w["Dr"], dt=w["dt"], seed=w["seed"])
    sysm = spv.System(x, y, L, L, p0=w["p0"], theta0=th0, params=prm)
    Lxq, Lyq, q = sysm.box()
    xq, yq, _, _, _ = oracle.prepare(x, y, L, L)
    out = oracle.run(xq, yq, th0, Lxq, Lyq, q, 1.0, w["p0"], mu=w["mu"], v0=w["v0"], Dr=w["Dr"], dt=w["dt"],
                     seed=w["seed"], nsteps=T)
    Eg, Qg = [], []
    for t in range(T + 1):
        E, qbar, _, _ = sysm.observables()
        Eg.append(E)
        Qg.append(qbar)
        if t < T:
            sysm.step(1)
    Eg, Qg = np.array(Eg), np.array(Qg)
    np.testing.assert_allclose(Eg, out["E"], rtol=1e-6)
    np.testing.assert_allclose(Qg, out["qbar"], rtol=1e-6)
    sysm.close()


def test_determinism(spv):
    n = 3000
    x, y, Lx, Ly = _random_case(n, 45)
    res = []
    for _ in range(2):
        s = spv.System(x, y, Lx, Ly, p0=3.9, params=spv.Params(v0=0.1, seed=11, resort_every=10))
        s.step(60)
        res.append((*s.positions(), s.directors(), s.observables()[0]))
        s.close()
    for a, b in zip(res[0], res[1]):
        assert np.array_equal(np.asarray(a), np.asarray(b))


def test_large_system_sampled(spv):
    """spv_n100k workload size: full topology and force comparison after steps."""
    w = inputs.WORKLOADS["spv_n100k"]
    n, L = w["N"], w["L"]
    x, y = inputs.uniform_positions(n, L, L, w["seed"])
    sysm = spv.System(x, y, L, L, p0=w["p0"], params=spv.Params(v0=w["v0"], Dr=w["Dr"], dt=w["dt"],
                                                                  seed=w["seed"]))
    gx, gy = sysm.positions()
    off, ring = _compare_topology(sysm, gx, gy)
    sysm.step(30)
    gx, gy = sysm.positions()
    off, ring = _compare_topology(sysm, gx, gy)
    _compare_forces(sysm, gx, gy, off, ring, 1.0, w["p0"])
    sysm.close()


def test_precondition_error(spv):
    x = np.array([1.0, 2.0, 1.5, 7.0, 3.0])
    y = np.array([1.0, 1.0, 2.0, 7.0, 5.0])
    with pytest.raises(spv.SPVError) as ei:
        spv.System(x, y, 10.0, 10.0)
    assert ei.value.status == spv.SPV_EPRECOND


def test_invalid_inputs(spv):
    x, y, Lx, Ly = _random_case(100, 46)
    x2 = x.copy()
    x2[3] = Lx + 1.0
    with pytest.raises(spv.SPVError) as ei:
        spv.System(x2, y, Lx, Ly)
    assert ei.value.status == spv.SPV_EINVAL
    x3, y3 = x.copy(), y.copy()
    x3[5], y3[5] = x3[9], y3[9]
    with pytest.raises(spv.SPVError) as ei:
        spv.System(x3, y3, Lx, Ly)
    assert ei.value.status == spv.SPV_EINVAL
    for bad in (float("nan"), float("inf"), -0.5):
        x4 = x.copy()
        x4[7] = bad
        with pytest.raises(spv.SPVError) as ei:
            spv.System(x4, y, Lx, Ly)
        assert ei.value.status == spv.SPV_EINVAL


def test_device_pointer_inputs_and_outputs(spv):
    import torch
    n = 700
    x, y, Lx, Ly = _random_case(n, 47)
    tx = torch.tensor(x, dtype=torch.float64, device="cuda")
    ty = torch.tensor(y, dtype=torch.float64, device="cuda")
    s = spv.System(tx, ty, Lx, Ly)
    ox = torch.empty(n, dtype=torch.float64, device="cuda")
    oy = torch.empty(n, dtype=torch.float64, device="cuda")
    spv.spv_get_positions(s.h, ox, oy)
    hx, hy = s.positions()
    assert np.array_equal(ox.cpu().numpy(), hx) and np.array_equal(oy.cpu().numpy(), hy)
    s.close()


# ---------------------------------------------------------------- launch paths, batches, precision

def _run(spv, x, y, L, steps_seq, counters=False, **kw):
    s = spv.System(x, y, L, L, p0=3.9, params=spv.Params(v0=0.1, seed=21, **kw))
    for k in steps_seq:
        s.step(k)
    out = (*s.positions(), s.directors(), *s.neighbors())
    cnt = s.observables()[3]
    s.close()
    return (out, cnt) if counters else out


def test_graph_and_eager_paths_bitwise_equal(spv):
    """A long enough run leaves the fast-moving start, so whole re-sort
    periods replay as captured graphs (counted); the trajectory is bitwise
    that of all-eager launches and of other step-count splits."""
    n = 2000
    x, y, L, _ = _random_case(n, 51)
    a, ca = _run(spv, x, y, L, [301], counters=True, resort_every=8)      # graph periods + eager steps
    b, cb = _run(spv, x, y, L, [301], counters=True, resort_every=8, no_graphs=1)
    c = _run(spv, x, y, L, [1, 2, 3, 31, 264], resort_every=8)            # mixed boundaries
    assert ca[8] > 0, "no re-sort period was replayed as a graph"
    assert cb[8] == 0
    for u, v, w in zip(a, b, c):
        assert np.array_equal(u, v) and np.array_equal(u, w)
    Lx = Ly = L
    gx, gy = a[0], a[1]
    s = spv.System(gx, gy, Lx, Ly, p0=3.9)
    Lq, _, q = s.box()
    s.close()
    off, ring, _, _ = oracle.triangulate(gx, gy, Lq, Lq, q)
    assert np.array_equal(a[3], off) and np.array_equal(a[4], ring)


def test_dense_rounds_bitwise_equal(spv):
    """Dense first rounds (flag and touched bytes scanned by the whole grid)
    and worklist rounds give the same trajectory bit for bit: from the random
    start, where a large share of the cells fails every step, on into the
    quiet phase; and the topology is the oracle's."""
    n = 3000
    x, y, L, _ = _random_case(n, 53)
    a, ca = _run(spv, x, y, L, [90], counters=True, resort_every=8, dense=1)  # never
    b, cb = _run(spv, x, y, L, [90], counters=True, resort_every=8, dense=2)  # every step, graphs too
    c, cc = _run(spv, x, y, L, [90], counters=True, resort_every=8)           # while cells move fast
    assert ca[9] == 0 and cb[9] == 90 and cc[9] > 0
    for u, v, w in zip(a, b, c):
        assert np.array_equal(u, v) and np.array_equal(u, w)
    s = spv.System(a[0], a[1], L, L, p0=3.9)
    Lq, _, q = s.box()
    s.close()
    off, ring, _, _ = oracle.triangulate(a[0], a[1], Lq, Lq, q)
    assert np.array_equal(a[3], off) and np.array_equal(a[4], ring)


def test_dense_repair_hands_crowded_cells_on(spv):
    """A crowded start (300 cells in a disk of radius 1.2 inside a uniform
    system) gives repairs with more candidates than a dense repair holds;
    those go to the worklist rounds and the host rounds, and the result is
    still bitwise the worklist path's and the oracle's triangulation."""
    n = 2000
    L = math.sqrt(n)
    x, y = inputs.uniform_positions(n, L, L, 54)
    rng = np.random.default_rng(55)
    r = 1.2 * np.sqrt(rng.uniform(0.0, 1.0, 300))
    t = rng.uniform(0.0, 2.0 * math.pi, 300)
    x[:300] = 0.5 * L + r * np.cos(t)
    y[:300] = 0.5 * L + r * np.sin(t)
    a = _run(spv, x, y, L, [12], resort_every=8, dense=1)
    b, cb = _run(spv, x, y, L, [12], counters=True, resort_every=8, dense=2)
    for u, v in zip(a, b):
        assert np.array_equal(u, v)
    s = spv.System(b[0], b[1], L, L, p0=3.9)
    Lq, _, q = s.box()
    s.close()
    off, ring, _, _ = oracle.triangulate(b[0], b[1], Lq, Lq, q)
    assert np.array_equal(b[3], off) and np.array_equal(b[4], ring)


def test_host_recovery_rounds_bitwise_equal(spv):
    """One device round per step forces the host to finish most repairs; the
    result must not depend on where the rounds run."""
    n = 3000
    x, y, L, _ = _random_case(n, 52)
    a = _run(spv, x, y, L, [48], resort_every=16)
    b = _run(spv, x, y, L, [48], resort_every=16, device_rounds=1)
    for u, v in zip(a, b):
        assert np.array_equal(u, v)


def _batch_inputs(S, seed):
    rng = np.random.default_rng(seed)
    N_s = [64, 300, 1000, 257, 4096][:S]
    L_s = [math.sqrt(nn) for nn in N_s]
    xs, ys = [], []
    for k, nn in enumerate(N_s):
        x, y = inputs.uniform_positions(nn, L_s[k], L_s[k], seed + 1 + k)
        xs.append(x)
        ys.append(y)
    p0_s = rng.uniform(3.6, 4.0, S)
    v0_s = rng.uniform(0.01, 0.2, S)
    seed_s = np.arange(S, dtype=np.uint64) + 1000
    return N_s, L_s, xs, ys, p0_s, v0_s, seed_s


def test_batch_equals_systems_run_alone(spv):
    S = 5
    N_s, L_s, xs, ys, p0_s, v0_s, seed_s = _batch_inputs(S, 60)
    steps = 40
    b = spv.System.batch(N_s, L_s, np.concatenate(xs), np.concatenate(ys), p0_s, v0_s=v0_s, seed_s=seed_s,
                         params=spv.Params(Dr=1.0, dt=0.01, resort_every=8))
    b.step(steps)
    bx, by = b.positions()
    boff, bnb = b.neighbors()
    for k in range(S):
        first, nn = b.system_range(k)
        assert nn == N_s[k]
        s = spv.System(xs[k], ys[k], L_s[k], L_s[k], p0=p0_s[k],
                       params=spv.Params(v0=v0_s[k], seed=int(seed_s[k]), Dr=1.0, dt=0.01, resort_every=8))
        s.step(steps)
        sx, sy = s.positions()
        assert np.array_equal(bx[first:first + nn], sx) and np.array_equal(by[first:first + nn], sy)
        soff, snb = s.neighbors()
        ring_b = bnb[boff[first]:boff[first + nn]] - first
        assert np.array_equal(ring_b, snb)
        Eb, qb, ab = b.system_observables(k)
        Es, qs, as_, _ = s.observables()
        assert abs(Eb - Es) <= 1e-12 * max(1.0, abs(Es)) and abs(ab - as_) <= 1e-9 * as_
        # and each system's topology is its exact Delaunay triangulation
        Lx, Ly, q = b.system_box(k)
        off, ring, _, _ = oracle.triangulate(sx, sy, Lx, Ly, q)
        assert np.array_equal(soff, off) and np.array_equal(snb, ring)
        s.close()
    b.close()


def test_mixed_precision_forces_and_topology(spv):
    """FP32 geometry/forces: topology stays exact (FP64 predicates); the force
    error against the FP64 oracle is reported and bounded."""
    n = 20000
    x, y, L, _ = _random_case(n, 61)
    s = spv.System(x, y, L, L, p0=3.9, params=spv.Params(v0=0.1, seed=5, precision=spv.SPV_MIXED))
    s.step(50)
    gx, gy = s.positions()
    Lx, Ly, q = s.box()
    off, ring = _compare_topology(s, gx, gy)
    fx, fy = oracle.forces(gx, gy, Lx, Ly, off, ring, 1.0, 3.9)
    gfx, gfy = s.forces()
    F = np.hypot(fx, fy)
    dF = np.hypot(gfx - fx, gfy - fy)
    scale = max(F.max(), 3.9)
    rel = dF.max() / scale
    rms = np.sqrt((dF ** 2).mean()) / scale
    l2 = np.sqrt((dF ** 2).sum() / (F ** 2).sum())
    print(f"mixed precision: max|dF|/scale = {rel:.3e}, rms|dF|/scale = {rms:.3e}, |dF|_2/|F|_2 = {l2:.3e}, "
          f"p99.9 = {np.quantile(dF, 0.999) / scale:.3e}")
    assert rel < 2e-5 and rms < 5e-6
    A, P = oracle.geometry(gx, gy, Lx, Ly, off, ring)
    gA, gP = s.geometry()
    assert np.abs(gA - A).max() < 1e-5 and np.abs(gP - P).max() < 1e-5
    s.close()


def test_stiff_start_wraps_jumps_longer_than_the_box(spv):
    """A random start whose first step moves a cell by more than a box length
    (largest force about 7e3 after step 1 at dt = 0.01, N = 1200): positions
    wrap modulo the box in grid units, as the oracle's integer wrap does, the
    drift bound counts the whole jump, and the run goes on; E and qbar follow
    the oracle step by step."""
    n = 1200
    L = math.sqrt(n)
    x, y = inputs.uniform_positions(n, L, L, 92)
    th0 = oracle.theta0(7, n)
    sysm = spv.System(x, y, L, L, p0=3.9, theta0=th0, params=spv.Params(v0=0.15, Dr=1.0, dt=0.01, seed=7))
    Lxq, Lyq, q = sysm.box()
    xq, yq, _, _, _ = oracle.prepare(x, y, L, L)
    T = 4
    out = oracle.run(xq, yq, th0, Lxq, Lyq, q, 1.0, 3.9, v0=0.15, Dr=1.0, dt=0.01, seed=7, nsteps=T)
    for t in range(T + 1):
        E, qbar, _, _ = sysm.observables()
        assert abs(E - out["E"][t]) <= 1e-6 * abs(out["E"][t]), (t, E, out["E"][t])
        assert abs(qbar - out["qbar"][t]) <= 1e-6 * abs(out["qbar"][t]), (t, qbar, out["qbar"][t])
        if t < T:
            sysm.step(1)
    gx, gy = sysm.positions()
    assert gx.min() >= 0 and gx.max() < Lxq and gy.min() >= 0 and gy.max() < Lyq
    sysm.close()


# ---------------------------------------------------------------- error paths

def test_repair_budget_exhausted_is_an_error(spv):
    """repair_rounds = device_rounds = 1 from a random start: the first step
    needs more rounds than allowed.  The kernels end normally (the tail halts
    the step), the host returns SPV_EREPAIR, and the handle keeps returning
    it."""
    x, y, L, _ = _random_case(2000, 81)
    s = spv.System(x, y, L, L, p0=3.9, params=spv.Params(v0=0.1, seed=1, repair_rounds=1, device_rounds=1))
    with pytest.raises(spv.SPVError) as ei:
        s.step(5)
    assert ei.value.status == spv.SPV_EREPAIR
    with pytest.raises(spv.SPVError) as ei:
        s.step(1)
    assert ei.value.status == spv.SPV_EREPAIR
    s.close()


def test_overflowing_update_is_a_nonfinite_error(spv):
    """A time step so large that the Eq. 3 update overflows: SPV_ENONFINITE
    from the device error word (the stored positions stay finite)."""
    x, y, L, _ = _random_case(500, 82)
    s = spv.System(x, y, L, L, p0=3.9, params=spv.Params(v0=1.0, seed=1, dt=1e300))
    with pytest.raises(spv.SPVError) as ei:
        s.step(1)
    assert ei.value.status == spv.SPV_ENONFINITE
    gx, gy = s.positions()
    assert np.isfinite(gx).all() and np.isfinite(gy).all()
    s.close()


# ---------------------------------------------------------------- hybrid comparison mode

def test_hybrid_mode_bitwise_equal_to_device_repair(spv):
    """repair_mode = 1 (the paper's split: the device tests, the host
    rebuilds failed rings each step, the device re-tests) follows bitwise the
    trajectory of the device repair, from the random start (thousands of
    host repairs in the first steps) on; rings equal the oracle's."""
    n = 3000
    x, y, L, _ = _random_case(n, 57)
    a, ca = _run(spv, x, y, L, [40], counters=True, resort_every=8)
    b, cb = _run(spv, x, y, L, [7, 33], counters=True, resort_every=8, repair_mode=1)
    for u, v in zip(a, b):
        assert np.array_equal(u, v)
    assert cb[1] == ca[1] and cb[8] == 0  # the same repairs, no graphs
    s = spv.System(b[0], b[1], L, L, p0=3.9)
    Lq, _, q = s.box()
    s.close()
    off, ring, _, _ = oracle.triangulate(b[0], b[1], Lq, Lq, q)
    assert np.array_equal(b[3], off) and np.array_equal(b[4], ring)


def test_hybrid_mode_batch(spv):
    S = 4
    N_s, L_s, xs, ys, p0_s, v0_s, seed_s = _batch_inputs(S, 62)
    out = []
    for mode in (0, 1):
        b = spv.System.batch(N_s, L_s, np.concatenate(xs), np.concatenate(ys), p0_s, v0_s=v0_s, seed_s=seed_s,
                             params=spv.Params(Dr=1.0, dt=0.01, resort_every=8, repair_mode=mode))
        b.step(30)
        out.append((*b.positions(), *b.neighbors()))
        b.close()
    for u, v in zip(*out):
        assert np.array_equal(u, v)


def test_never_resort_bitwise_equal(spv):
    """resort_every = -1: the memory order of creation is kept and every
    step's repairs search a cell list of the step's positions; graph periods
    still replay (without a re-sort).  The trajectory is bitwise that of the
    re-sorting default, with the same Hilbert or row-major bins."""
    n = 3000
    x, y, L, _ = _random_case(n, 58)
    for order in (0, 1):
        a, ca = _run(spv, x, y, L, [600], counters=True, bin_order=order)
        b, cb = _run(spv, x, y, L, [3, 597], counters=True, resort_every=-1, bin_order=order)
        for u, v in zip(a, b):
            assert np.array_equal(u, v)
        assert cb[5] == 0 and cb[8] > 0 and ca[5] > 0


@pytest.mark.parametrize("repair_mode", [0, 1])
def test_corrupted_ring_is_detected_and_repaired(spv, repair_mode):
    """A ring overwritten through the fault-injection hook (one neighbour
    dropped, two swapped, one replaced by a second-shell cell) fails the
    next step's test and is rebuilt by the repair (device rounds inside
    replayed graph periods, or the hybrid host repair): the topology equals
    the oracle's triangulation of the positions again, forces within the
    bound.  Invalid rings are rejected with the topology unchanged."""
    n = 2000
    x, y, L, _ = _random_case(n, 63)
    s = spv.System(x, y, L, L, p0=3.9, params=spv.Params(v0=0.1, Dr=1.0, seed=5, resort_every=8,
                                                           repair_mode=repair_mode))
    s.step(301)
    off, ring = s.neighbors()
    rng = np.random.default_rng(9)
    cells = [int(c) for c in rng.choice(n, 40, replace=False) if off[c + 1] - off[c] >= 5][:3]
    assert len(cells) == 3
    a, b, c = cells
    ra, rb, rc = (list(ring[off[t]:off[t + 1]]) for t in (a, b, c))
    second = [int(v) for v in ring[off[rc[0]]:off[rc[0] + 1]] if v != c and v not in rc]
    bad = {a: ra[:2] + ra[3:], b: [rb[1], rb[0]] + rb[2:], c: [second[0]] + rc[1:]}
    cnt0 = s.observables()[3]
    for t, r in bad.items():
        s.debug_set_ring(t, r)
    goff, gring = s.neighbors()
    for t, r in bad.items():
        assert list(gring[goff[t]:goff[t + 1]]) == r
    s.step(1)  # the next step's test and repair fix all three rings
    gx, gy = s.positions()
    _compare_topology(s, gx, gy)
    cnt = s.observables()[3]
    assert cnt[1] >= cnt0[1] + 3 and cnt[7] == 0
    for t, r in bad.items():
        s.debug_set_ring(t, r)
    s.step(16)  # corrupted again, now with re-sort periods replayed as graphs
    gx, gy = s.positions()
    o2, r2 = _compare_topology(s, gx, gy)
    _compare_forces(s, gx, gy, o2, r2, 1.0, 3.9)
    cnt = s.observables()[3]
    assert cnt[7] == 0
    if repair_mode == 0:
        assert cnt[8] > cnt0[8], "no graph period replayed after the corruption"
    t = int(rng.integers(n))
    r = list(r2[o2[t]:o2[t + 1]])
    kcap = 16
    for wrong in ([r[0], r[1]], (r * 3)[:kcap + 1], [t] + r[1:], [r[0]] + r[:-1], [n] + r[1:], [-1] + r[1:]):
        with pytest.raises(spv.SPVError) as ei:
            s.debug_set_ring(t, wrong)
        assert ei.value.status == spv.SPV_EINVAL
    with pytest.raises(spv.SPVError):
        s.debug_set_ring(n, r)
    o3, r3 = s.neighbors()
    assert np.array_equal(o3, o2) and np.array_equal(r3, r2)
    s.close()


def test_corrupted_ring_in_a_batch(spv):
    """The fault-injection hook on a batch: a ring of the third system (a
    global index) with one neighbour dropped is rebuilt by the next step;
    every system's rings equal the oracle's triangulation of its positions,
    and a ring naming a cell of another system is rejected."""
    S = 4
    N_s, L_s, xs, ys, p0_s, v0_s, seed_s = _batch_inputs(S, 64)
    b = spv.System.batch(N_s, L_s, np.concatenate(xs), np.concatenate(ys), p0_s, v0_s=v0_s, seed_s=seed_s,
                         params=spv.Params(Dr=1.0, dt=0.01, resort_every=8))
    b.step(40)
    off, ring = b.neighbors()
    first, n2 = b.system_range(2)
    t = first + int(np.argmax(np.diff(off)[first:first + n2]))
    r = list(ring[off[t]:off[t + 1]])
    assert len(r) >= 5
    b.debug_set_ring(t, r[:1] + r[2:])
    other = b.system_range(1)[0]
    with pytest.raises(spv.SPVError) as ei:
        b.debug_set_ring(t, [other] + r[1:])
    assert ei.value.status == spv.SPV_EINVAL
    b.step(1)
    gx, gy = b.positions()
    off, ring = b.neighbors()
    for k in range(S):
        f, nk = b.system_range(k)
        Lx, Ly, q = b.system_box(k)
        o, rr, _, _ = oracle.triangulate(gx[f:f + nk], gy[f:f + nk], Lx, Ly, q)
        go = off[f:f + nk + 1] - off[f]
        assert np.array_equal(go, o)
        assert np.array_equal(ring[off[f]:off[f + nk]] - f, rr)
    b.close()
