"""Scheduling knobs and the autotuner, through the C-ABI: every knob setting
gives bitwise the same trajectory (positions, directors, rings) as the
defaults, and a tuned handle starts from the caller's input, not from the
tuner's trial state.  The trajectory itself is pinned to the oracle by the
parity tests; here equality with the untuned handle is the bar."""
import json
import math
import os

import numpy as np
import pytest

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


def _run(spv, x, y, L, steps, **kw):
    s = spv.System(x, y, L, L, p0=3.9, params=spv.Params(v0=0.1, seed=23, **kw))
    tun = s.tuning()
    s.step(steps)
    out = (*s.positions(), s.directors(), *s.neighbors())
    s.close()
    return out, tun


KNOB_CASES = [
    dict(bin_factor=2.0),
    dict(bin_factor=0.5),
    dict(bin_factor=1.5, repair_cells=16),
    dict(repair_cells=1024, device_rounds=3),
    dict(resort_every=64, repair_cells=8),
    dict(device_rounds=1),                    # every later round on the host
    dict(tail_items=1),                       # the tail hands most rounds to the host
    dict(device_rounds=16, tail_items=4096),  # the tail takes everything
    dict(full_rounds=2),                      # two full-grid rounds before the tail
    dict(full_rounds=4, device_rounds=3),     # full-grid rounds capped by the device rounds
    dict(bin_order=1),                        # row-major bins instead of the Hilbert order
    dict(force_mode=1),                       # force kernel with kcap/4 lanes per cell
    dict(force_mode=2),                       # force kernel with one thread per (cell, slot) item
]


@pytest.mark.parametrize("kw", KNOB_CASES, ids=[",".join(f"{k}={v}" for k, v in c.items()) for c in KNOB_CASES])
def test_knobs_do_not_change_results(spv, kw):
    n = 3000
    L = math.sqrt(n)
    x, y = inputs.uniform_positions(n, L, L, 71)
    ref, t0 = _run(spv, x, y, L, 70)
    got, t1 = _run(spv, x, y, L, 70, **kw)
    assert t0["source"] == 0 and t1["source"] == 0
    for k, v in kw.items():
        if k in t1:
            assert t1[k] == v
    for u, v in zip(ref, got):
        assert np.array_equal(u, v)


def test_autotune_trials_cache_and_results(spv, tmp_path, monkeypatch):
    n = 4000
    L = math.sqrt(n)
    x, y = inputs.uniform_positions(n, L, L, 72)
    cache = tmp_path / "tune.json"
    monkeypatch.setenv("SPV_TUNE_CACHE", str(cache))
    ref, t0 = _run(spv, x, y, L, 50)
    tuned, t2 = _run(spv, x, y, L, 50, autotune=2)
    assert t2["source"] == 2 and t2["ms_per_step"] > 0.0
    assert t2["bin_factor"] in (1.0, 1.5, 2.0)
    assert t2["repair_cells"] in (16, 64, 256) and t2["device_rounds"] in (2, 4, 8)
    assert t2["tail_items"] in (16, 64, 256) and t2["full_rounds"] in (1, 2) and t2["force_mode"] in (1, 2)
    assert t2["resort_every"] in (16, 32, 64)
    for u, v in zip(ref, tuned):
        assert np.array_equal(u, v)
    data = json.loads(cache.read_text())
    assert len(data) == 1
    (key, entry), = data.items()
    assert "/fp64/kc16/n2^12/s2^0" in key
    assert entry["resort_every"] == t2["resort_every"] and entry["bin_factor"] == t2["bin_factor"]
    # a second handle of the same size class reads the cache, runs no trial
    cached, t1 = _run(spv, x, y, L, 50, autotune=1)
    assert t1["source"] == 1
    knobs = ("resort_every", "device_rounds", "repair_cells", "tail_items", "full_rounds", "force_mode", "bin_factor")
    assert {k: t1[k] for k in knobs} == {k: t2[k] for k in knobs}
    for u, v in zip(ref, cached):
        assert np.array_equal(u, v)


def test_autotune_batch(spv, monkeypatch):
    monkeypatch.delenv("SPV_TUNE_CACHE", raising=False)
    N_s = [64, 500, 1200, 300]
    L_s = [math.sqrt(v) for v in N_s]
    xs, ys = zip(*[inputs.uniform_positions(v, L_s[k], L_s[k], 80 + k) for k, v in enumerate(N_s)])
    p0_s = np.array([3.7, 3.8, 3.9, 4.0])
    v0_s = np.array([0.05, 0.1, 0.15, 0.2])
    seed_s = np.array([5, 6, 7, 8], dtype=np.uint64)
    outs = []
    for tune in (0, 2):
        b = spv.System.batch(N_s, L_s, np.concatenate(xs), np.concatenate(ys), p0_s, v0_s=v0_s, seed_s=seed_s,
                             params=spv.Params(precision=spv.SPV_MIXED, autotune=tune))
        assert b.tuning()["source"] == tune
        b.step(40)
        outs.append((*b.positions(), *b.neighbors()))
        b.close()
    for u, v in zip(*outs):
        assert np.array_equal(u, v)



@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_force_layouts_agree_batched_and_kcap32(spv, precision):
    """Both kernel layouts (lanes per cell, one thread per (cell, slot) item)
    give bitwise the same trajectories for a batch of uneven systems and for
    a single system with ring capacity 32, in both precisions."""
    prec = spv.SPV_FP64 if precision == "fp64" else spv.SPV_MIXED
    N_s = [64, 500, 1200, 300, 2000]
    L_s = [math.sqrt(v) for v in N_s]
    xs, ys = zip(*[inputs.uniform_positions(v, L_s[k], L_s[k], 90 + k) for k, v in enumerate(N_s)])
    p0_s = np.array([3.7, 3.8, 3.9, 4.0, 3.85])
    v0_s = np.array([0.05, 0.1, 0.15, 0.2, 0.1])
    seed_s = np.array([5, 6, 7, 8, 9], dtype=np.uint64)
    outs = []
    for mode in (1, 2):
        b = spv.System.batch(N_s, L_s, np.concatenate(xs), np.concatenate(ys), p0_s, v0_s=v0_s, seed_s=seed_s,
                             params=spv.Params(precision=prec, force_mode=mode))
        assert b.tuning()["force_mode"] == mode
        b.step(60)
        outs.append((*b.positions(), b.directors(), *b.neighbors(), *b.forces()))
        b.close()
    for u, v in zip(*outs):
        assert np.array_equal(u, v)
    n = 3000
    L = math.sqrt(n)
    x, y = inputs.uniform_positions(n, L, L, 93)
    outs = []
    for mode in (1, 2):
        s = spv.System(x, y, L, L, p0=3.9, params=spv.Params(v0=0.1, seed=31, kcap=32, precision=prec,
                                                               force_mode=mode))
        assert s.tuning()["force_mode"] == mode
        s.step(60)
        outs.append((*s.positions(), s.directors(), *s.neighbors(), *s.forces()))
        s.close()
    for u, v in zip(*outs):
        assert np.array_equal(u, v)
