"""GPU tests of Algorithm 2 on a Cartesian lattice against the FP64 oracle (relative L2 <= 1e-4
for complex64 data, <= 1e-2 for FP16 storage)."""
import dataclasses
from types import SimpleNamespace

import numpy as np
import pytest

import oracle
import synth
from gpu_common import custom_workload, inputs, log, need_gpu, oracle_band, rel_l2, to_dev, torch

pytestmark = pytest.mark.gpu

TOL = 1e-4


def lattice(nx, ny, x0, y0, dx, dy):
    c = SimpleNamespace(nx=nx, ny=ny, x0_m=x0, y0_m=y0, dx_m=dx, dy_m=dy)
    xs = (x0 + np.arange(nx) * dx)[None, :].repeat(ny, 0)
    ys = (y0 + np.arange(ny) * dy)[:, None].repeat(nx, 1)
    return c, xs.ravel(), ys.ravel()


@pytest.mark.parametrize("interp", ["nearest", "linear"])
def test_cartesian_small(interp):
    rs = need_gpu()
    w, x = inputs("small")
    g, grid = w.geometry, w.grid
    r1 = grid.r0_m + (grid.n_range - 1) * grid.dr_m
    # ragged, covers the annulus; the origin is offset so that no target sits exactly halfway
    # between two weight rows or two pulse angles (a tie that floating rounding decides)
    c, xs, ys = lattice(97, 83, -r1 - 0.01234, -r1 * 0.9 + 0.00567, 2 * r1 / 96, 1.8 * r1 / 82)
    rc = rs.range_compress(g, to_dev(x.raw), to_dev(x.window), x.l_lo, x.l_count, halo=w.sparse.window // 2)
    log(f"cartesian small {interp}")
    img = rs.sparse_filter_cartesian(g, grid, c, rc, to_dev(x.offsets), to_dev(x.weights.astype(np.complex64)),
                                     w.sparse.window, interp=interp).cpu().numpy()
    ref = oracle.sparse_filter_cartesian(oracle_band("small"), x.l_lo, g, grid, xs, ys, x.offsets, x.weights,
                                         interp).reshape(c.ny, c.nx)
    assert rel_l2(img, ref) <= TOL
    assert np.count_nonzero(img) < img.size          # the centre and the corners are outside the rows


def test_cartesian_axes_match_polar():
    """Targets on the positive x axis at the rows' radii are polar pixels (azimuth bin 0)."""
    rs = need_gpu()
    w, x = inputs("small")
    g, grid = w.geometry, w.grid
    rc = rs.range_compress(g, to_dev(x.raw), to_dev(x.window), x.l_lo, x.l_count, halo=w.sparse.window // 2)
    off, wts = to_dev(x.offsets), to_dev(x.weights.astype(np.complex64))
    c = SimpleNamespace(nx=grid.n_range, ny=1, x0_m=grid.r0_m, y0_m=0.0, dx_m=grid.dr_m, dy_m=1.0)
    log("cartesian axes")
    cart = rs.sparse_filter_cartesian(g, grid, c, rc, off, wts, w.sparse.window).cpu().numpy()[0]
    polar = rs.sparse_filter(g, grid, rc, off, wts, w.sparse.window).cpu().numpy()[:, 0]
    assert rel_l2(cart, polar) <= 1e-6


def test_cartesian_f16():
    rs = need_gpu()
    w, x = inputs("small")
    g, grid = w.geometry, w.grid
    r1 = grid.r0_m + (grid.n_range - 1) * grid.dr_m
    c, xs, ys = lattice(64, 64, -r1 - 0.00917, -r1 + 0.00431, 2 * r1 / 63, 2 * r1 / 63)
    rc = rs.range_compress(g, to_dev(x.raw), to_dev(x.window), x.l_lo, x.l_count, halo=w.sparse.window // 2,
                           dtype="f16", scale=2.0 ** -4)
    log("cartesian f16")
    img = rs.sparse_filter_cartesian(g, grid, c, rc, to_dev(x.offsets), to_dev(x.weights.astype(np.complex64)),
                                     w.sparse.window).cpu().numpy()
    ref = oracle.sparse_filter_cartesian(oracle_band("small"), x.l_lo, g, grid, xs, ys, x.offsets,
                                         x.weights).reshape(64, 64)
    assert rel_l2(img, ref) <= 1e-2


def test_cartesian_paper_radar():
    """The paper's radar (N = 800, M = L = 225, r = 0.145 m, 60 GHz, T_Start = 7 us) on a 0.04 m
    Cartesian lattice, with weights designed for 24 polar rows over [0.5, 2.5] m."""
    rs = need_gpu()
    w = custom_workload("paper_radar", 77, 800, 225, 24, 0.5, 2.5, 32, 64, radius=0.145)
    g = dataclasses.replace(w.geometry, fc_hz=60e9, t_start_s=7e-6)
    w = dataclasses.replace(w, geometry=g)
    x = synth.make_inputs(w)
    yb = oracle.range_compress(x.raw, x.window, g.n_fft)[:, x.l_lo:x.l_lo + x.l_count]
    rc = rs.range_compress(g, to_dev(x.raw), to_dev(x.window), x.l_lo, x.l_count, halo=32)
    c, xs, ys = lattice(126, 126, -2.5 + 0.0013, -2.5 + 0.0029, 0.04, 0.04)
    log("cartesian paper radar")
    img = rs.sparse_filter_cartesian(g, w.grid, c, rc, to_dev(x.offsets), to_dev(x.weights.astype(np.complex64)),
                                     w.sparse.window, interp="linear").cpu().numpy()
    ref = oracle.sparse_filter_cartesian(yb, x.l_lo, g, w.grid, xs, ys, x.offsets, x.weights,
                                         "linear").reshape(126, 126)
    assert rel_l2(img, ref) <= TOL


def polar_positions(grid, n_az):
    """Targets of a polar grid with n_az azimuth bins: R_i, phi0 + 2 pi a / n_az (phi0 = 0)."""
    r = grid.r0_m + np.arange(grid.n_range) * grid.dr_m
    phi = 2 * np.pi * np.arange(n_az) / n_az
    return (r[:, None] * np.cos(phi)[None, :]).ravel(), (r[:, None] * np.sin(phi)[None, :]).ravel()


@pytest.mark.parametrize("interp,n_az", [("nearest", 500), ("linear", 500), ("nearest", 250)])
def test_polar_az_other_than_pulses(interp, n_az):
    """A = 500 and 250 azimuth bins for N = 360 pulses (a N / A never falls halfway between two
    pulses, so the central phase centre has no tie), against Algorithm 2 at those targets."""
    rs = need_gpu()
    w, x = inputs("small")
    g = w.geometry
    grid = dataclasses.replace(w.grid, n_az=n_az)
    rc = rs.range_compress(g, to_dev(x.raw), to_dev(x.window), x.l_lo, x.l_count, halo=w.sparse.window // 2)
    log(f"polar A={n_az} {interp}")
    img = rs.sparse_filter_polar(g, grid, rc, to_dev(x.offsets), to_dev(x.weights.astype(np.complex64)),
                                 w.sparse.window, interp=interp).cpu().numpy()
    xs, ys = polar_positions(grid, n_az)
    ref = oracle.sparse_filter_cartesian(oracle_band("small"), x.l_lo, g, w.grid, xs, ys, x.offsets, x.weights,
                                         interp).reshape(grid.n_range, n_az)
    assert img.shape == (grid.n_range, n_az)
    assert rel_l2(img, ref) <= TOL


def test_polar_az_equal_pulses_is_plain_filter():
    rs = need_gpu()
    w, x = inputs("small")
    rc = rs.range_compress(w.geometry, to_dev(x.raw), to_dev(x.window), x.l_lo, x.l_count, halo=w.sparse.window // 2)
    off, wts = to_dev(x.offsets), to_dev(x.weights.astype(np.complex64))
    log("polar A=N")
    a = rs.sparse_filter_polar(w.geometry, w.grid, rc, off, wts, w.sparse.window).cpu().numpy()
    b = rs.sparse_filter(w.geometry, w.grid, rc, off, wts, w.sparse.window).cpu().numpy()
    assert rel_l2(a, b) <= 1e-6


def test_polar_az_f16():
    rs = need_gpu()
    w, x = inputs("small")
    g = w.geometry
    grid = dataclasses.replace(w.grid, n_az=500)
    rc = rs.range_compress(g, to_dev(x.raw), to_dev(x.window), x.l_lo, x.l_count, halo=w.sparse.window // 2,
                           dtype="f16", scale=2.0 ** -4)
    log("polar A=500 f16")
    img = rs.sparse_filter_polar(g, grid, rc, to_dev(x.offsets), to_dev(x.weights.astype(np.complex64)),
                                 w.sparse.window).cpu().numpy()
    xs, ys = polar_positions(grid, 500)
    ref = oracle.sparse_filter_cartesian(oracle_band("small"), x.l_lo, g, w.grid, xs, ys, x.offsets, x.weights,
                                         "nearest").reshape(grid.n_range, 500)
    assert rel_l2(img, ref) <= 1e-2


def test_polar_az_rotation_sampled():
    """Rotation workload (N = 3600, 1024 rows, K = 64 of 256) on A = 4801 azimuth bins (odd A:
    a N / A is never halfway between two pulses), complex64 data; 300 sampled pixels against
    Algorithm 2 at those targets."""
    rs = need_gpu()
    w, x = inputs("rotation")
    g = w.geometry
    grid = dataclasses.replace(w.grid, n_az=4801)
    rc = rs.range_compress(g, to_dev(x.raw), to_dev(x.window), x.l_lo, x.l_count, halo=w.sparse.window // 2)
    log("polar A=4801 rotation")
    img = rs.sparse_filter_polar(g, grid, rc, to_dev(x.offsets), to_dev(x.weights.astype(np.complex64)),
                                 w.sparse.window).cpu().numpy()
    rng = np.random.default_rng(9)
    rows = rng.integers(0, grid.n_range, 300)
    azs = rng.integers(0, 4801, 300)
    r = grid.r0_m + rows * grid.dr_m
    phi = 2 * np.pi * azs / 4801
    ref = oracle.sparse_filter_cartesian(oracle_band("rotation"), x.l_lo, g, w.grid, r * np.cos(phi),
                                         r * np.sin(phi), x.offsets, x.weights)
    assert rel_l2(img[rows, azs], ref) <= TOL


@pytest.mark.parametrize("interp,jitter", [("nearest", False), ("linear", False), ("nearest", True)])
def test_bp_cartesian_small(interp, jitter):
    """Back-projection on a ragged lattice over the small workload's annulus (origin offset off
    ties), nominal or jittered pulse angles, against the oracle."""
    rs = need_gpu()
    w = synth.small()
    if jitter:
        w = dataclasses.replace(w, scene=dataclasses.replace(w.scene, jitter_sigma_rad=np.deg2rad(0.05)))
    x = synth.make_inputs(w)
    g, grid = w.geometry, w.grid
    r1 = grid.r0_m + (grid.n_range - 1) * grid.dr_m
    c, xs, ys = lattice(97, 83, -r1 - 0.01234, -r1 * 0.9 + 0.00567, 2 * r1 / 96, 1.8 * r1 / 82)
    rc = rs.range_compress(g, to_dev(x.raw), to_dev(x.window), x.l_lo, x.l_count, halo=w.sparse.window // 2)
    log(f"bp cartesian {interp} jitter={jitter}")
    img = rs.bp_cartesian(g, c, rc, angles=to_dev(x.angles) if jitter else None, interp=interp).cpu().numpy()
    yb = oracle.range_compress(x.raw, x.window, g.n_fft)[:, x.l_lo:x.l_lo + x.l_count]
    ref = oracle.bp_cartesian_at(yb, x.l_lo, g, xs, ys, pulse_angles=x.angles if jitter else None,
                                 interp=interp).reshape(c.ny, c.nx)
    assert rel_l2(img, ref) <= TOL


@pytest.mark.parametrize("interp", ["nearest", "linear"])
@pytest.mark.parametrize("jitter", [False, True])
def test_bp_cartesian_pulses_past_the_lds_table(interp, jitter):
    """N = 4000 pulses: more than the per-pulse (cos, sin) table holds in LDS, so every
    cos(phi - theta_n) is evaluated directly; against the oracle."""
    rs = need_gpu()
    w = custom_workload("bp_cart_big_n", 91, 4000, 64, 6, 0.5, 1.5, 16, 32)
    if jitter:
        w = dataclasses.replace(w, scene=dataclasses.replace(w.scene, jitter_sigma_rad=np.deg2rad(0.05)))
    x = synth.make_inputs(w)
    g, grid = w.geometry, w.grid
    r1 = grid.r0_m + (grid.n_range - 1) * grid.dr_m
    c, xs, ys = lattice(17, 13, -r1 - 0.01234, -r1 * 0.9 + 0.00567, 2 * r1 / 16, 1.8 * r1 / 12)
    rc = rs.range_compress(g, to_dev(x.raw), to_dev(x.window), x.l_lo, x.l_count, halo=w.sparse.window // 2)
    log(f"bp cartesian N = 4000 {interp} jitter={jitter}")
    img = rs.bp_cartesian(g, c, rc, angles=to_dev(x.angles) if jitter else None, interp=interp).cpu().numpy()
    yb = oracle.range_compress(x.raw, x.window, g.n_fft)[:, x.l_lo:x.l_lo + x.l_count]
    ref = oracle.bp_cartesian_at(yb, x.l_lo, g, xs, ys, pulse_angles=x.angles if jitter else None,
                                 interp=interp).reshape(c.ny, c.nx)
    assert rel_l2(img, ref) <= TOL


def test_bp_cartesian_axis_matches_polar_bpa():
    """Targets on the positive x axis at the rows' radii are polar pixels of azimuth bin 0."""
    rs = need_gpu()
    w, x = inputs("small")
    g, grid = w.geometry, w.grid
    rc = rs.range_compress(g, to_dev(x.raw), to_dev(x.window), x.l_lo, x.l_count, halo=w.sparse.window // 2)
    c = SimpleNamespace(nx=grid.n_range, ny=1, x0_m=grid.r0_m, y0_m=0.0, dx_m=grid.dr_m, dy_m=1.0)
    log("bp cartesian axis")
    cart = rs.bp_cartesian(g, c, rc).cpu().numpy()[0]
    polar = rs.bp_full(g, grid, rc).cpu().numpy()[:, 0]
    assert rel_l2(cart, polar) <= 1e-5


@pytest.mark.parametrize("dtype,scale", [("f16", 2.0 ** -4), ("bf16", 1.0)])
def test_bp_cartesian_reduced_precision(dtype, scale):
    """Back-projection on the lattice from FP16 / BF16 storage (float32 accumulation)."""
    rs = need_gpu()
    w, x = inputs("small")
    g, grid = w.geometry, w.grid
    r1 = grid.r0_m + (grid.n_range - 1) * grid.dr_m
    c, xs, ys = lattice(64, 64, -r1 - 0.00917, -r1 + 0.00431, 2 * r1 / 63, 2 * r1 / 63)
    rc = rs.range_compress(g, to_dev(x.raw), to_dev(x.window), x.l_lo, x.l_count, halo=w.sparse.window // 2,
                           dtype=dtype, scale=scale)
    log(f"bp cartesian {dtype}")
    img = rs.bp_cartesian(g, c, rc).cpu().numpy()
    ref = oracle.bp_cartesian_at(oracle_band("small"), x.l_lo, g, xs, ys).reshape(64, 64)
    assert rel_l2(img, ref) <= 1e-2


@pytest.mark.parametrize("interp", ["nearest", "linear"])
def test_cartesian_window_wider_than_the_lds_table(interp):
    """A 4400-pulse window (N = 5000): wider than the kernel's table of the offsets' cosines, so
    the target-to-pulse angle takes its cosine directly; against the oracle."""
    rs = need_gpu()
    w = custom_workload("cart_wide", 83, 5000, 64, 8, 1.0, 2.0, 8, 4400, radius=0.25)
    x = synth.make_inputs(w)
    g = w.geometry
    yb = oracle.range_compress(x.raw, x.window, g.n_fft)[:, x.l_lo:x.l_lo + x.l_count]
    rc = rs.range_compress(g, to_dev(x.raw), to_dev(x.window), x.l_lo, x.l_count, halo=16)
    c, xs, ys = lattice(24, 20, -2.0 + 0.00731, -2.0 + 0.00419, 4.0 / 23, 4.0 / 19)
    log(f"cartesian, window 4400 of 5000, {interp}")
    img = rs.sparse_filter_cartesian(g, w.grid, c, rc, to_dev(x.offsets), to_dev(x.weights.astype(np.complex64)),
                                     w.sparse.window, interp=interp).cpu().numpy()
    ref = oracle.sparse_filter_cartesian(yb, x.l_lo, g, w.grid, xs, ys, x.offsets, x.weights,
                                         interp).reshape(20, 24)
    assert rel_l2(img, ref) <= TOL
