"""Workload definitions for the rotating-SAR imaging path (plain data, no method arithmetic).

Each workload fixes the radar (chirp, sampling, rotation), the polar output grid, the scene
recipe and the sparse-aperture recipe.  Five workloads are defined:

  small      N=360 pulses, M=L=256, r=0.25 m, 128x360 grid aligned to FFT bins 13..140,
             3 unit scatterers, 20 dB SNR, K=32 of a 64-pulse window (support shared by rows).
  rotation   N=3600, M=L=512, r=0.3 m, 1024x3600 grid over [0.5, 15] m, 200 Rayleigh
             scatterers + complex white clutter 30 dB down, angle jitter N(0, 0.05 deg),
             K=64 of 256 per range row.
  precision  the `rotation` scene model at N=7200, M=L=1024, 2048x7200 grid; used with
             FP16/BF16 range-compressed storage and FP16 weights.
  batch      64 rotations of uneven size (see synth.batch).
  calib      `rotation` sizes with LINEAR interpolation for gradient-based calibration.
  testbed    the paper's radar (Table II chirp, N=800, M=L=225, r=0.145 m) and its 9.8756 m
             square image area on a 0.04 m Cartesian lattice (247 x 247 targets), 155 polar
             weight rows one FFT bin apart, K=157 of a 400-pulse window.

Radar common to all but `testbed`: f_c = 77 GHz, B = 4 GHz swept over the M samples, F_s = 10 MHz,
K_s = B*F_s/M, T_Start = 0, c = 299 792 458 m/s.  With L = M one FFT bin is c/(2B) m.
"""
from __future__ import annotations

import dataclasses
import math
from dataclasses import dataclass, field

C_LIGHT = 299_792_458.0
FC_HZ = 77e9
BANDWIDTH_HZ = 4e9
FS_HZ = 10e6


@dataclass(frozen=True)
class Geometry:
    """Radar and rotation parameters (paper Table I/II notation: N, M, L, r, f_c, K, F_s, T_Start)."""
    n_pulses: int
    n_fast: int
    n_fft: int
    radius_m: float
    fc_hz: float
    slope_hz_s: float
    fs_hz: float
    t_start_s: float = 0.0
    c_m_s: float = C_LIGHT
    phi0_rad: float = 0.0


@dataclass(frozen=True)
class PolarGrid:
    """Polar output grid: R_r = r0 + r*dr, phi_a = phi0 + 2*pi*a/n_az."""
    n_range: int
    n_az: int
    r0_m: float
    dr_m: float

    def ranges(self):
        return [self.r0_m + i * self.dr_m for i in range(self.n_range)]


@dataclass(frozen=True)
class SceneSpec:
    n_scatterers: int
    amplitude: str               # "unit" or "rayleigh" (CN(0,1))
    r_min_m: float
    r_max_m: float
    noise_power: float = 0.0     # complex white noise per raw sample, CN(0, noise_power)
    jitter_sigma_rad: float = 0.0


@dataclass(frozen=True)
class SparseSpec:
    k: int                       # taps kept per range row
    window: int                  # W: offsets drawn from [-W/2, W/2)
    shared_support: bool         # one support for every range row
    taylor_nbar: int = 4
    taylor_sll_db: float = 30.0


@dataclass(frozen=True)
class Workload:
    name: str
    cfg_id: int                  # seeds are PCG64(1000*cfg_id + j)
    geometry: Geometry
    grid: PolarGrid
    scene: SceneSpec
    sparse: SparseSpec
    interp: str = "nearest"      # "nearest" or "linear"
    extra: dict = field(default_factory=dict)

    def replace(self, **kw):
        return dataclasses.replace(self, **kw)


def radar(n_pulses: int, n_fast: int, radius_m: float, n_fft: int | None = None) -> Geometry:
    return Geometry(n_pulses=n_pulses, n_fast=n_fast, n_fft=n_fft or n_fast, radius_m=radius_m,
                    fc_hz=FC_HZ, slope_hz_s=BANDWIDTH_HZ * FS_HZ / n_fast, fs_hz=FS_HZ)


def bin_size_m(geom: Geometry) -> float:
    """Range spanned by one FFT bin for this radar (input recipe: used to place grids)."""
    return geom.c_m_s * geom.fs_hz / (2.0 * geom.slope_hz_s * geom.n_fft)


def band_for(geom: Geometry, grid: PolarGrid) -> tuple[int, int]:
    """FFT rows [l_lo, l_lo+l_count) that cover every slant range the grid can reach.

    The nearest slant range of a pixel at R is R - r, the farthest visible one is below R;
    two extra rows leave room for linear interpolation.
    """
    b = bin_size_m(geom)
    r_lo = max(grid.r0_m - geom.radius_m, 0.0)
    r_hi = grid.r0_m + (grid.n_range - 1) * grid.dr_m
    lo = max(int(math.floor(r_lo / b)) - 1, 0)
    hi = min(int(math.ceil(r_hi / b)) + 2, geom.n_fft)
    return lo, hi - lo


def small() -> Workload:
    g = radar(360, 256, 0.25)
    b = bin_size_m(g)
    grid = PolarGrid(n_range=128, n_az=360, r0_m=13 * b, dr_m=b)
    return Workload("small", 1, g, grid,
                    SceneSpec(3, "unit", 1.0, 5.0, noise_power=1e-2, jitter_sigma_rad=0.0),
                    SparseSpec(32, 64, shared_support=True))


def rotation() -> Workload:
    g = radar(3600, 512, 0.3)
    grid = PolarGrid(n_range=1024, n_az=3600, r0_m=0.5, dr_m=(15.0 - 0.5) / 1023)
    return Workload("rotation", 2, g, grid,
                    SceneSpec(200, "rayleigh", 0.5, 15.0, noise_power=1e-3,
                              jitter_sigma_rad=math.radians(0.05)),
                    SparseSpec(64, 256, shared_support=False))


def precision() -> Workload:
    g = radar(7200, 1024, 0.3)
    grid = PolarGrid(n_range=2048, n_az=7200, r0_m=0.5, dr_m=(15.0 - 0.5) / 2047)
    return Workload("precision", 3, g, grid,
                    SceneSpec(200, "rayleigh", 0.5, 15.0, noise_power=1e-3,
                              jitter_sigma_rad=math.radians(0.05)),
                    SparseSpec(64, 256, shared_support=False))


def calib() -> Workload:
    return rotation().replace(name="calib", cfg_id=5, interp="linear")


def scaled(w: Workload, n_pulses: int, n_fast: int, n_range: int, k: int | None = None,
           window: int | None = None, name: str | None = None) -> Workload:
    """Same scene recipe on a smaller radar/grid (for parity cases the oracle finishes quickly)."""
    g = dataclasses.replace(radar(n_pulses, n_fast, w.geometry.radius_m))
    r_hi = w.grid.r0_m + (w.grid.n_range - 1) * w.grid.dr_m
    r_hi = min(r_hi, 0.9 * n_fast * bin_size_m(g))
    grid = PolarGrid(n_range=n_range, n_az=n_pulses, r0_m=w.grid.r0_m,
                     dr_m=(r_hi - w.grid.r0_m) / max(n_range - 1, 1))
    sc = dataclasses.replace(w.scene, r_max_m=min(w.scene.r_max_m, r_hi))
    sp = dataclasses.replace(w.sparse, k=k or w.sparse.k, window=window or w.sparse.window)
    return w.replace(name=name or f"{w.name}_{n_pulses}x{n_fast}x{n_range}", geometry=g,
                     grid=grid, scene=sc, sparse=sp)


# The paper's radar (Sec. IV-B, Table II): chirp from 60 GHz with slope K = 6.8e13 Hz/s, sampled
# at F_s = 4.5 MHz from T_Start = 7 us, M = L = 225 samples, r = 0.145 m, N = 800 pulses per
# rotation.  One FFT bin spans c F_s / (2 K L) = 0.04409 m, so the 225 bins reach 9.8756 m: the
# side of the testbed's square image area (Sec. IV-F).
PAPER_FC_HZ = 60e9
PAPER_SLOPE_HZ_S = 6.8e13
PAPER_FS_HZ = 4.5e6
PAPER_T_START_S = 7e-6
PAPER_AREA_M = 9.8756
PAPER_CELL_M = 0.04
# the wheel encoder's angle spread (Sec. IV-B), read in degrees
PAPER_SIGMA_RAD = math.radians(0.086)


def paper_radar(n_pulses: int = 800) -> Geometry:
    return Geometry(n_pulses=n_pulses, n_fast=225, n_fft=225, radius_m=0.145, fc_hz=PAPER_FC_HZ,
                    slope_hz_s=PAPER_SLOPE_HZ_S, fs_hz=PAPER_FS_HZ, t_start_s=PAPER_T_START_S)


@dataclass(frozen=True)
class CartLattice:
    """Cartesian targets x0 + i dx, y0 + j dy (i < nx, j < ny), row-major [ny][nx]."""
    nx: int
    ny: int
    x0_m: float
    y0_m: float
    dx_m: float
    dy_m: float

    def positions(self):
        import numpy as np
        xs = (self.x0_m + np.arange(self.nx) * self.dx_m)[None, :].repeat(self.ny, 0)
        ys = (self.y0_m + np.arange(self.ny) * self.dy_m)[:, None].repeat(self.nx, 1)
        return xs.ravel(), ys.ravel()


def paper_lattice() -> CartLattice:
    """The testbed's image area (Sec. IV-F): a 9.8756 m square centred on the rotation centre,
    cut into 0.04 m cells; the targets are the 247 x 247 cell centres."""
    n = int(math.ceil(PAPER_AREA_M / PAPER_CELL_M))
    x0 = -PAPER_AREA_M / 2 + PAPER_CELL_M / 2
    return CartLattice(n, n, x0, x0, PAPER_CELL_M, PAPER_CELL_M)


def testbed() -> Workload:
    """The paper's radar and image area: polar weight rows one FFT bin apart from 0.2 m out to
    the area's corners (7.0 m), 20 Rayleigh scatterers inside the area plus white noise, the
    encoder's angle jitter, K = 157 taps (Table IV's robust count) of a 400-pulse window."""
    g = paper_radar(800)
    b = bin_size_m(g)
    r_hi = math.hypot(PAPER_AREA_M / 2, PAPER_AREA_M / 2)
    n_rows = int(math.ceil((r_hi - 0.2) / b)) + 1
    grid = PolarGrid(n_range=n_rows, n_az=800, r0_m=0.2, dr_m=b)
    return Workload("testbed", 6, g, grid,
                    SceneSpec(20, "rayleigh", 0.5, PAPER_AREA_M / 2, noise_power=1e-3,
                              jitter_sigma_rad=PAPER_SIGMA_RAD),
                    SparseSpec(157, 400, shared_support=False))


WORKLOADS = {"small": small, "rotation": rotation, "precision": precision, "calib": calib, "testbed": testbed}
