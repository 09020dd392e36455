"""Seeded synthetic inputs: scatterer scenes, pulse angles, raw IF cubes, windows, sparse sets.

These are the inputs of the imaging path; both the FP64 oracle and the HIP path consume the
same arrays.  The raw cube follows the paper's deramped, sampled IF model (Sec. II-B, eq. 10,
residual video phase dropped as the paper does) with the cosine antenna pattern (eq. 8) at
the true, possibly jittered, pulse angles (eq. 37).  The weights follow the recipe "K of a
W-pulse window": a seeded random support (the paper's random phase-centre selection idea,
Sec. IV-C) with phase-matched, Taylor-tapered coefficients normalised to unit norm (the
unit-norm constraint C3 of eq. 20).  They stand in for the offline FPP-SCA design.

Seeds: numpy Generator(PCG64(1000*cfg_id + j)), j = 1 scene, 2 noise, 3 jitter, 4 support.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import scipy.signal.windows as sw

from .configs import Geometry, PolarGrid, Workload, band_for

SEED_SCENE, SEED_NOISE, SEED_JITTER, SEED_SUPPORT = 1, 2, 3, 4


def rng_for(cfg_id: int, j: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(1000 * cfg_id + j))


@dataclass
class Scene:
    r_m: np.ndarray          # [S] scatterer range from the rotation centre
    phi_rad: np.ndarray      # [S] scatterer azimuth
    amp: np.ndarray          # [S] complex reflectivity


@dataclass
class Inputs:
    """Everything one imaging call consumes, as host arrays."""
    workload: Workload
    scene: Scene
    angles: np.ndarray       # [N] float64 true pulse angles (nominal + jitter)
    raw: np.ndarray          # [N, M] complex64 raw IF cube, pulse-major
    window: np.ndarray       # [M] float32 fast-time window
    offsets: np.ndarray      # [Rg, K] int32 in [-W/2, W/2)
    weights: np.ndarray      # [Rg, K] complex128
    l_lo: int
    l_count: int


def make_scene(w: Workload) -> Scene:
    rng = rng_for(w.cfg_id, SEED_SCENE)
    s = w.scene
    r = rng.uniform(s.r_min_m, s.r_max_m, s.n_scatterers)
    phi = rng.uniform(0.0, 2.0 * math.pi, s.n_scatterers)
    if s.amplitude == "unit":
        amp = np.ones(s.n_scatterers, dtype=np.complex128)
    else:
        amp = (rng.standard_normal(s.n_scatterers) + 1j * rng.standard_normal(s.n_scatterers)) / math.sqrt(2)
    return Scene(r, phi, amp)


def nominal_angles(geom: Geometry) -> np.ndarray:
    return geom.phi0_rad + 2.0 * math.pi * np.arange(geom.n_pulses) / geom.n_pulses


def jitter_draws(seed: int, window: int, n_samples: int, sigma_rad: float) -> np.ndarray:
    """Monte-Carlo angle errors for the Delta_R estimate (eq. 37): [window, n_samples] float64,
    independent N(0, sigma^2) per phase centre and draw, draw-minor (the device layout)."""
    return np.random.Generator(np.random.PCG64(seed)).normal(0.0, sigma_rad, (window, n_samples))


def make_angles(w: Workload) -> np.ndarray:
    """True pulse angles: nominal 2*pi*n/N plus N(0, sigma^2) jitter (eq. 37)."""
    a = nominal_angles(w.geometry)
    if w.scene.jitter_sigma_rad > 0:
        a = a + rng_for(w.cfg_id, SEED_JITTER).normal(0.0, w.scene.jitter_sigma_rad, a.shape)
    return a


def hann(m: int) -> np.ndarray:
    """Symmetric Hann window h[m] = 1/2 - 1/2 cos(2 pi m/(M-1))."""
    return (0.5 - 0.5 * np.cos(2.0 * math.pi * np.arange(m) / (m - 1))).astype(np.float32)


def simulate_raw(geom: Geometry, scene: Scene, angles: np.ndarray, noise_power: float = 0.0,
                 rng: np.random.Generator | None = None, chunk: int = 256) -> np.ndarray:
    """Raw deramped IF samples y[n, m] for point scatterers (eq. 10 with alpha_n of eq. 15).

    phase(m) = 2 pi [tau K (m t_s + T_Start) + f_c tau], tau = 2 R_n / c, amplitude
    amp * cos(theta_n) inside the +-90 deg antenna field of view, 0 outside.  The m axis is
    split as m = 32*m1 + m2 so the exponentials factor into two short tables per
    (pulse, scatterer) and the sum over scatterers is a batched matrix product.
    """
    n_p, m = geom.n_pulses, geom.n_fast
    out = np.zeros((n_p, m), dtype=np.complex64)
    blk = 32 if m % 32 == 0 else 1
    m1 = np.arange(m // blk, dtype=np.float64) * blk
    m2 = np.arange(blk, dtype=np.float64)
    r = geom.radius_m
    two_pi = 2.0 * math.pi
    for n0 in range(0, n_p, chunk):
        ang = angles[n0:n0 + chunk][:, None]                       # [n,1]
        d = ang - scene.phi_rad[None, :]                            # [n,S]
        rn = np.sqrt(scene.r_m ** 2 + r * r - 2.0 * r * scene.r_m * np.cos(d))
        cos_theta = (scene.r_m * np.cos(d) - r) / rn
        alpha = scene.amp[None, :] * np.maximum(cos_theta, 0.0)
        tau = 2.0 * rn / geom.c_m_s
        f_beat = tau * geom.slope_hz_s                              # Hz
        w_s = two_pi * f_beat / geom.fs_hz                          # rad / sample
        ph0 = np.mod(two_pi * tau * (geom.slope_hz_s * geom.t_start_s + geom.fc_hz), two_pi)
        u = alpha[:, :, None] * np.exp(1j * (ph0[:, :, None] + w_s[:, :, None] * m1[None, None, :]))
        v = np.exp(1j * (w_s[:, :, None] * m2[None, None, :]))
        y = np.matmul(u.transpose(0, 2, 1), v)                      # [n, M/blk, blk]
        out[n0:n0 + chunk] = y.reshape(y.shape[0], m).astype(np.complex64)
    if noise_power > 0:
        rng = rng or np.random.default_rng(0)
        nz = (rng.standard_normal((n_p, m)) + 1j * rng.standard_normal((n_p, m))) * math.sqrt(noise_power / 2)
        out += nz.astype(np.complex64)
    return out


def taylor_taper(w: int, nbar: int, sll_db: float) -> np.ndarray:
    return sw.taylor(w, nbar=nbar, sll=sll_db, norm=True)


def make_support(w: Workload) -> np.ndarray:
    """Offsets [Rg, K] int32: a seeded random K-subset of [-W/2, W/2), sorted per row."""
    rng = rng_for(w.cfg_id, SEED_SUPPORT)
    k, win, rg = w.sparse.k, w.sparse.window, w.grid.n_range
    if w.sparse.shared_support:
        row = np.sort(rng.choice(win, k, replace=False)) - win // 2
        return np.tile(row.astype(np.int32), (rg, 1))
    out = np.empty((rg, k), dtype=np.int32)
    for i in range(rg):
        out[i] = np.sort(rng.choice(win, k, replace=False)) - win // 2
    return out


def phase_matched_weights(geom: Geometry, grid: PolarGrid, offsets: np.ndarray,
                          taper: np.ndarray) -> np.ndarray:
    """w[r,k] = t(o_k + W/2) exp(+j 2 k_w R(o_k)) / ||.||, R(o) the nominal slant range to a
    point at (phi_a, R_r) from the pulse o steps away (phase of the steering vector, eq. 16).
    The FP64 phase is reduced modulo 2 pi before the exponential."""
    kw = 2.0 * math.pi * (geom.slope_hz_s * geom.t_start_s + geom.fc_hz) / geom.c_m_s
    rr = np.array(grid.ranges())[:, None]
    d = offsets.astype(np.float64) * (2.0 * math.pi / geom.n_pulses)
    rn = np.sqrt(rr ** 2 + geom.radius_m ** 2 - 2.0 * rr * geom.radius_m * np.cos(d))
    ph = np.mod(2.0 * kw * rn, 2.0 * math.pi)
    win = taper.shape[0]
    t = taper[offsets + win // 2]
    w = t * np.exp(1j * ph)
    return w / np.linalg.norm(w, axis=1, keepdims=True)


def make_inputs(w: Workload, with_raw: bool = True) -> Inputs:
    g = w.geometry
    scene = make_scene(w)
    angles = make_angles(w)
    raw = (simulate_raw(g, scene, angles, w.scene.noise_power, rng_for(w.cfg_id, SEED_NOISE))
           if with_raw else np.zeros((g.n_pulses, g.n_fast), np.complex64))
    offsets = make_support(w)
    weights = phase_matched_weights(g, w.grid, offsets,
                                    taylor_taper(w.sparse.window, w.sparse.taylor_nbar, w.sparse.taylor_sll_db))
    lo, cnt = band_for(g, w.grid)
    return Inputs(w, scene, angles, raw, hann(g.n_fast), offsets, weights, lo, cnt)


def random_complex(shape, seed: int, scale: float = 1.0, dtype=np.complex64) -> np.ndarray:
    """Plain CN(0, scale^2) array (for linearity/adjoint cases that need arbitrary data)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return ((rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) * (scale / math.sqrt(2))).astype(dtype)
