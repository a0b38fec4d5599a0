"""Host logic of the hybrid comparison mode: the library's host repair
(spv_host_repair.hpp: exact gift-wrapping over a certified disk, the device
repair's tie-break), run on every cell from scratch, reproduces the oracle's
periodic Delaunay triangulation ring for ring (same counter-clockwise order,
same start).  Built for the host only; no GPU involved."""
import math
import os
import subprocess

import numpy as np
import pytest

import oracle
from paper_1702_02939_amd import inputs

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def tool(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("hostrepair") / "host_repair_check")
    subprocess.run([os.environ.get("HIPCC", "/opt/rocm/bin/hipcc"), "-std=c++20", "-O2", "--offload-host-only",
                    "-o", exe, os.path.join(HERE, "host_repair_check.cpp")], check=True, capture_output=True)

    def run(x, y, Lx, Ly, q):
        text = f"{len(x)} {float(Lx)!r} {float(Ly)!r} {int(q)}\n" + "".join(
            f"{float(a)!r} {float(b)!r}\n" for a, b in zip(x, y))
        out = subprocess.run([exe], input=text, check=True, capture_output=True, text=True).stdout
        return out.splitlines()
    return run


def _check(tool, x, y, Lx, Ly):
    xq, yq, Lx, Ly, q = oracle.prepare(x, y, Lx, Ly)
    off, ring, ntri, _ = oracle.triangulate(xq, yq, Lx, Ly, q)
    lines = tool(xq, yq, Lx, Ly, q)
    assert len(lines) == len(xq)
    for i, line in enumerate(lines):
        f = line.split()
        assert f[0] != "err", f"cell {i}: {line}"
        k = int(f[0])
        assert k == off[i + 1] - off[i], f"cell {i}: degree"
        assert [int(v) for v in f[1:]] == list(ring[off[i]:off[i + 1]]), f"cell {i}: ring"


@pytest.mark.parametrize("n,seed", [(300, 101), (1200, 102)])
def test_uniform(tool, n, seed):
    L = math.sqrt(n)
    x, y = inputs.uniform_positions(n, L, L, seed)
    _check(tool, x, y, L, L)


def test_rectangular_box(tool):
    x, y = inputs.uniform_positions(900, 60.0, 15.0, 103)
    _check(tool, x, y, 60.0, 15.0)


def test_lattices_with_cocircular_ties(tool):
    # the exact square lattice (every empty circle has four cells on it: the
    # tag tie-break decides) and the hexagonal lattice
    x, y, Lx, Ly = inputs.square_lattice(12, 1.0)
    _check(tool, x, y, Lx, Ly)
    x, y, Lx, Ly = inputs.hex_lattice(10, 10, 1.0)
    _check(tool, x, y, Lx, Ly)


def test_clustered(tool):
    # dense clusters inside a sparse background: candidate sets from a few to
    # a few hundred, radius doublings
    rng = np.random.default_rng(104)
    L = 30.0
    x, y = inputs.uniform_positions(500, L, L, 105)
    r = 0.8 * np.sqrt(rng.uniform(0, 1, 150))
    t = rng.uniform(0, 2 * math.pi, 150)
    x[:150] = 10.0 + r * np.cos(t)
    y[:150] = 20.0 + r * np.sin(t)
    _check(tool, x, y, L, L)
