"""Seeded synthetic inputs for the SPV workloads.

Only random numbers and lattice coordinates live here -- none of the model's
arithmetic (no quantisation, no geometry, no dynamics) -- so that the HIP
path and the CPU oracle can both be fed from it.

The workloads follow the paper's regimes (Sussman, arXiv:1702.02939, Sec. III:
solid P0 = 3.8 and fluid P0 = 3.9 / 4.0 at unit preferred area); positions are
uniform random in a periodic square box of side sqrt(N) (density 1).
"""
from __future__ import annotations

import math

import numpy as np

BASE_SEED = 20170209

# name -> workload description (sizes and parameters)
WORKLOADS = {
    "spv_n256": dict(N=256, L=16.0, p0=3.8, v0=0.05, Dr=1.0, mu=1.0, dt=0.01, steps=1000, seed=BASE_SEED + 1),
    "spv_n100k": dict(N=100_000, L=math.sqrt(100_000), p0=3.9, v0=0.1, Dr=1.0, mu=1.0, dt=0.01, steps=10_000,
                      seed=BASE_SEED + 2),
    "spv_n4096_adjoint": dict(N=4096, L=64.0, p0=3.8, p0_sigma=0.05, v0=0.05, Dr=1.0, mu=1.0, dt=0.01, steps=200,
                              ckpt=20, seed=BASE_SEED + 4),
    "spv_n1m": dict(N=1_000_000, L=1000.0, p0=3.85, v0=0.1, Dr=1.0, mu=1.0, dt=0.01, steps=2000,
                    seed=BASE_SEED + 5),
    # active vertex model: the Voronoi network of N uniform-random points
    # (2N vertices), T1 threshold 0.04 and new edge 0.06 (in units of the
    # mean cell side sqrt(A0) = 1)
    "avm_n100k": dict(N=100_000, L=math.sqrt(100_000), p0=3.8, v0=0.1, Dr=1.0, mu=1.0, dt=0.01, t1=0.04,
                      t1_new=0.06, steps=2000, seed=BASE_SEED + 6),
    "avm_n1m": dict(N=1_000_000, L=1000.0, p0=3.8, v0=0.1, Dr=1.0, mu=1.0, dt=0.01, t1=0.04, t1_new=0.06,
                    steps=400, seed=BASE_SEED + 7),
}


def uniform_positions(n: int, Lx: float, Ly: float, seed: int):
    """n points uniform in [0,Lx) x [0,Ly) from numpy's default generator."""
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.0, Lx, n)
    y = rng.uniform(0.0, Ly, n)
    return x, y


def hex_lattice(nx: int, ny: int, a: float = 1.0, offset=(0.1, 0.1)):
    """Triangular lattice of spacing a (hexagonal Voronoi cells), nx x ny
    sites, ny even, in a periodic box nx*a by ny*a*sqrt(3)/2."""
    assert ny % 2 == 0
    h = a * math.sqrt(3.0) / 2.0
    xs, ys = [], []
    for r in range(ny):
        for c in range(nx):
            xs.append(offset[0] + c * a + (0.5 * a if r % 2 else 0.0))
            ys.append(offset[1] + r * h)
    return np.array(xs), np.array(ys), nx * a, ny * h


def square_lattice(n: int, a: float = 1.0, offset=(0.25, 0.25)):
    """n x n square lattice (every Delaunay quad is cocircular)."""
    xs, ys = np.meshgrid(np.arange(n) * a + offset[0], np.arange(n) * a + offset[1])
    return xs.ravel().copy(), ys.ravel().copy(), n * a, n * a


def batch_systems(S: int = 256, seed: int = BASE_SEED + 3, nmin: int = 64, nmax: int = 4096):
    """Independent systems of uneven size: N_s ~ U{nmin..nmax}, L_s = sqrt(N_s),
    p0 ~ U[3.6, 4.0], v0 ~ U[0.01, 0.2]; positions seeded per system."""
    rng = np.random.default_rng(seed)
    N = rng.integers(nmin, nmax + 1, size=S)
    p0 = rng.uniform(3.6, 4.0, size=S)
    v0 = rng.uniform(0.01, 0.2, size=S)
    systems = []
    for s in range(S):
        L = math.sqrt(int(N[s]))
        x, y = uniform_positions(int(N[s]), L, L, seed + 1 + s)
        systems.append(dict(N=int(N[s]), L=L, p0=float(p0[s]), v0=float(v0[s]), x=x, y=y, seed=seed + 1 + s))
    return systems


def per_cell_p0(n: int, mean: float, sigma: float, seed: int):
    """Per-cell target shape index ~ N(mean, sigma)."""
    return np.random.default_rng(seed).normal(mean, sigma, n)
