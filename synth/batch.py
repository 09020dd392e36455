"""Batched-stream workload: many independent rotations of uneven size (input recipe only).

Rotation i draws, from PCG64(1000*40 + 7): pulses N in {900, 1800, 3600}, fast-time samples
M in {256, 512, 1024}, range rows in {256, 512, 1024}, K in {32, 64} with window W = 4K;
rotation radius 0.3 m; the grid covers [0.5, min(15, 0.9 * M * bin)] m; the scene has 50..300
Rayleigh scatterers (uniform range over the grid, uniform azimuth), no clutter, nominal angles.
Its scene / noise / support seeds are those of workload id 400 + i.
"""
from __future__ import annotations

import concurrent.futures as cf
import dataclasses

import numpy as np

from .configs import PolarGrid, SceneSpec, SparseSpec, Workload, bin_size_m, radar
from .scene import Inputs, make_inputs


def batch_workloads(n: int = 64, seed: int = 40) -> list[Workload]:
    rng = np.random.Generator(np.random.PCG64(1000 * seed + 7))
    out = []
    for i in range(n):
        n_p = int(rng.choice([900, 1800, 3600]))
        m = int(rng.choice([256, 512, 1024]))
        rg = int(rng.choice([256, 512, 1024]))
        k = int(rng.choice([32, 64]))
        n_sc = int(rng.integers(50, 301))
        g = radar(n_p, m, 0.3)
        r1 = min(15.0, 0.9 * m * bin_size_m(g))
        grid = PolarGrid(rg, n_p, 0.5, (r1 - 0.5) / (rg - 1))
        out.append(Workload(f"batch{i}", 400 + i, g, grid, SceneSpec(n_sc, "rayleigh", 0.5, r1),
                            SparseSpec(k, 4 * k, shared_support=False)))
    return out


def make_batch_inputs(ws: list[Workload], threads: int = 8) -> list[Inputs]:
    """Inputs of every rotation (generated in parallel threads; numpy releases the GIL)."""
    with cf.ThreadPoolExecutor(max_workers=threads) as ex:
        return list(ex.map(make_inputs, ws))


def scaled_batch(n: int = 6, seed: int = 41) -> list[Workload]:
    """A small heterogeneous batch (for parity cases): shapes from the same menus, cut down."""
    rng = np.random.Generator(np.random.PCG64(1000 * seed + 7))
    out = []
    menu = [(120, 64, 16, 8), (256, 128, 40, 16), (360, 256, 24, 32), (512, 512, 8, 32), (200, 1024, 12, 16),
            (96, 2048, 6, 8)]
    for i in range(n):
        n_p, m, rg, k = menu[i % len(menu)]
        g = radar(n_p, m, 0.3)
        r1 = min(6.0, 0.9 * m * bin_size_m(g))
        grid = PolarGrid(rg, n_p, 0.5, (r1 - 0.5) / (rg - 1))
        n_sc = int(rng.integers(3, 12))
        out.append(Workload(f"sbatch{i}", 500 + i, g, grid, SceneSpec(n_sc, "rayleigh", 0.5, r1, noise_power=1e-3),
                            SparseSpec(k, 4 * k, shared_support=False)))
    return out
