"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics (CPU only).

Each test checks the oracle against something other than itself: a value the paper prints,
a closed form derived independently (Cartesian geometry and the physical beat frequency
rather than the law-of-cosines/eq. 40 code paths the oracle uses), a brute-force sum on tiny
inputs, an invariant, or a library special case.
"""
import dataclasses
import json
import math
import os

import numpy as np
import pytest

import oracle
import synth
from oracle import metrics

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# --------------------------------------------------------------------------- helpers
def cart_range(geom, pulse_angle, r_t, phi_t):
    """Distance between the phase centre at pulse_angle and the point (r_t, phi_t), in x/y."""
    px, py = geom.radius_m * np.cos(pulse_angle), geom.radius_m * np.sin(pulse_angle)
    tx, ty = r_t * np.cos(phi_t), r_t * np.sin(phi_t)
    return np.hypot(tx - px, ty - py)


def beat_bin(geom, rng_m):
    """Fractional FFT bin of a target at slant range rng_m: beat frequency 2 R K / c over F_s/L."""
    return (2.0 * rng_m * geom.slope_hz_s / geom.c_m_s) / geom.fs_hz * geom.n_fft


def carrier_phase(geom, rng_m):
    """2 pi tau (K T_Start + f_c), tau = 2R/c (the constant part of eq. 10's phase)."""
    return 2.0 * math.pi * (2.0 * rng_m / geom.c_m_s) * (geom.slope_hz_s * geom.t_start_s + geom.fc_hz)


def boresight_cos(geom, pulse_angle, r_t, phi_t):
    """cos(theta): projection of the unit vector radar->target on the outward bore-sight."""
    px, py = geom.radius_m * np.cos(pulse_angle), geom.radius_m * np.sin(pulse_angle)
    tx, ty = r_t * np.cos(phi_t), r_t * np.sin(phi_t)
    d = np.hypot(tx - px, ty - py)
    return ((tx - px) * np.cos(pulse_angle) + (ty - py) * np.sin(pulse_angle)) / d


def dirichlet(x, m):
    """sum_{m'<m} exp(j 2 pi x m') in closed form."""
    x = np.asarray(x, dtype=np.float64)
    z = np.exp(2j * np.pi * x)
    near = np.abs(1 - z) < 1e-14
    return np.where(near, m, (1 - z ** m) / np.where(near, 1, 1 - z))


def small_geom(n=64, m=64, r=0.25, t_start=0.0):
    g = synth.radar(n, m, r)
    import dataclasses
    return dataclasses.replace(g, t_start_s=t_start)


# --------------------------------------------------------------------------- P1
def test_visibility_worked_example():
    """381 effective phase centres for (pi/2, 2 m), r = 0.145 m, N = 800 (Sec. IV-D.1)."""
    with open(os.path.join(GOLDEN, "visibility_worked_example.json")) as f:
        gold = json.load(f)
    r, n, rt = gold["radius_m"], gold["n_pulses"], gold["target_range_m"]
    lo, hi = oracle.visible_index_range(rt, r, n)
    assert hi - lo + 1 == gold["effective_phase_centres"]
    # the back-projection's own visibility rule must select exactly those pulses
    g = synth.Geometry(n, 225, 225, r, 60e9, 6.8e13, 4.5e6)
    grid = synth.PolarGrid(1, n, rt, 0.0)
    vis, _, alpha = oracle.bp_terms(g, grid, 0, gold["target_azimuth_rad"],
                                    2 * np.pi * np.arange(n) / n)
    idx = np.nonzero(vis[0])[0]
    assert len(idx) == gold["effective_phase_centres"]
    assert idx[0] == lo and idx[-1] == hi
    # alpha is the cosine antenna pattern of eq. 8 at the bore-sight angle
    ang = 2 * np.pi * idx / n
    np.testing.assert_allclose(alpha[0, idx], boresight_cos(g, ang, rt, np.pi / 2), rtol=1e-12)


# --------------------------------------------------------------------------- P2, P3
@pytest.mark.parametrize("window", ["rect", "hann"])
@pytest.mark.parametrize("m,l", [(64, 64), (48, 64), (256, 512)])
def test_range_compress_tone_closed_form(window, m, l):
    nu = np.array([0.1234567, 0.31, -0.2])[:, None]                   # cycles per sample
    mm = np.arange(m)
    raw = np.exp(2j * np.pi * nu * mm)
    h = None if window == "rect" else 0.5 - 0.5 * np.cos(2 * np.pi * mm / (m - 1))
    y = oracle.range_compress(raw, h, l)
    x = nu - np.arange(l)[None, :] / l
    if window == "rect":
        ref = dirichlet(x, m)
    else:  # h = 1/2 - 1/4 e^{+j2pi m/(M-1)} - 1/4 e^{-j2pi m/(M-1)}
        s = 1.0 / (m - 1)
        ref = 0.5 * dirichlet(x, m) - 0.25 * dirichlet(x + s, m) - 0.25 * dirichlet(x - s, m)
    np.testing.assert_allclose(y, ref, rtol=0, atol=1e-9 * m)


def test_range_compress_direct_sum_and_parseval():
    raw = synth.random_complex((3, 12), seed=11).astype(np.complex128)
    h = synth.hann(12)
    np.testing.assert_allclose(oracle.range_compress(raw, h, 16),
                               oracle.range_compress_direct(raw, h, 16), atol=1e-12)
    y = oracle.range_compress(raw, None, 12)
    np.testing.assert_allclose(np.sum(np.abs(y) ** 2, axis=1), 12 * np.sum(np.abs(raw) ** 2, axis=1),
                               rtol=1e-12)


def test_peak_bin_matches_beat_frequency():
    """argmax |Y_1D| of a simulated target equals round(beta R) (eq. 40)."""
    g = synth.radar(8, 512, 0.3)
    beta = oracle.bins_per_metre(g)
    rng = np.random.default_rng(5)
    for r_t in rng.uniform(1.0, 15.0, 20):
        sc = synth.Scene(np.array([r_t]), np.array([0.0]), np.array([1.0 + 0j]))
        raw = synth.simulate_raw(g, sc, np.zeros(g.n_pulses))
        y = oracle.range_compress(raw[:1], None, g.n_fft)
        rn = r_t - g.radius_m
        assert np.argmax(np.abs(y[0])) == int(np.floor(beta * rn + 0.5))
        assert abs(beta * rn - beat_bin(g, rn)) < 1e-9


# --------------------------------------------------------------------------- P4
def _bin_exact_scene(g, grid, offsets, row, a0, l_lo, l_count, dtype=np.complex128):
    """Y_1D with a unit response e^{j2kR} at exactly the bin of a point at pixel (row, a0)."""
    yb = np.zeros((g.n_pulses, l_count), dtype=dtype)
    r_t = grid.r0_m + row * grid.dr_m
    phi_t = g.phi0_rad + 2 * np.pi * a0 / grid.n_az
    for o in offsets[row]:
        n = (a0 + int(o)) % g.n_pulses
        ang = g.phi0_rad + 2 * np.pi * n / g.n_pulses
        rn = cart_range(g, ang, r_t, phi_t)
        lb = int(np.floor(beat_bin(g, rn) + 0.5)) - l_lo
        assert 0 <= lb < l_count
        yb[n, lb] = np.exp(1j * carrier_phase(g, rn))
    return yb


@pytest.mark.parametrize("t_start", [0.0, 3e-6])
def test_sum_abs_weights_closed_form(t_start):
    """Phase-matched weights on a bin-exact unit scatterer give I = sum_k |w_k| at its pixel and
    strictly less everywhere else (triangle inequality)."""
    g = small_geom(180, 128, 0.25, t_start)
    w = synth.Workload("p4", 41, g, synth.PolarGrid(6, 180, 1.3, 0.11),
                       synth.SceneSpec(0, "unit", 1, 2), synth.SparseSpec(24, 64, False))
    offs = synth.make_support(w)
    wts = synth.phase_matched_weights(g, w.grid, offs, synth.taylor_taper(64, 4, 30))
    l_lo, l_count = synth.band_for(g, w.grid)
    row, a0 = 3, 17
    yb = _bin_exact_scene(g, w.grid, offs, row, a0, l_lo, l_count)
    img = oracle.sparse_filter(yb, l_lo, g, w.grid, offs, wts)
    peak = np.sum(np.abs(wts[row]))
    assert abs(img[row, a0] - peak) < 1e-9 * peak
    others = np.abs(img).copy()
    others[row, a0] = 0
    assert others.max() < peak * (1 - 1e-6)


# --------------------------------------------------------------------------- P4, corrected
def _recorded_point(g, grid, offsets, row, a0, l_lo, l_count, delta=None, psi=None, spread=False):
    """Band of a unit point at pixel (row, a0) as recorded by phase centres that really sat at
    phi0 + 2 pi n / N + delta_n (positions in x/y), with a per-pulse phase error e^{+j psi_n} in
    the data: value e^{+j carrier phase} at the bin of the true beat frequency (NEAREST), or at
    both bins around it (spread, so LINEAR reads the same value)."""
    n_p = g.n_pulses
    delta = np.zeros(n_p) if delta is None else delta
    psi = np.zeros(n_p) if psi is None else psi
    yb = np.zeros((n_p, l_count), dtype=np.complex128)
    r_t = grid.r0_m + row * grid.dr_m
    phi_t = g.phi0_rad + 2 * np.pi * a0 / grid.n_az
    for o in offsets[row]:
        n = (a0 + int(o)) % n_p
        ang = g.phi0_rad + 2 * np.pi * n / n_p + delta[n]
        rn = cart_range(g, ang, r_t, phi_t)
        u = beat_bin(g, rn)
        assert abs(u - np.floor(u) - 0.5) > 1e-6          # no rounding tie
        val = np.exp(1j * (carrier_phase(g, rn) + psi[n]))
        if spread:
            lb = int(np.floor(u)) - l_lo
            yb[n, lb] = yb[n, lb + 1] = val
        else:
            yb[n, int(np.floor(u + 0.5)) - l_lo] = val
    return yb


def _p4_case(seed):
    g = small_geom(180, 128, 0.25)
    w = synth.Workload("p4c", 48, g, synth.PolarGrid(6, 180, 1.3, 0.11),
                       synth.SceneSpec(0, "unit", 1, 2), synth.SparseSpec(24, 64, False))
    offs = synth.make_support(w)
    wts = synth.phase_matched_weights(g, w.grid, offs, synth.taylor_taper(64, 4, 30))
    l_lo, l_count = synth.band_for(g, w.grid)
    rng = np.random.default_rng(seed)
    return g, w.grid, offs, wts, l_lo, l_count, rng


@pytest.mark.parametrize("interp", ["nearest", "linear"])
def test_corrected_filter_angle_error_physical(interp):
    """Data recorded at true angles 2 pi n / N + delta_n (eq. 37), with the bin and the carrier
    phase of the true x/y range: the corrected filter given dphi = delta refocuses the point to
    sum_k |w_k| exactly (weights matched to the nominal geometry); dphi = -delta, or no
    correction, does not.  This fixes the sign convention of delta relative to the offsets."""
    g, grid, offs, wts, l_lo, l_count, rng = _p4_case(61)
    row, a0 = 3, 17
    delta = rng.normal(0, 3e-3, g.n_pulses)
    yb = _recorded_point(g, grid, offs, row, a0, l_lo, l_count, delta=delta, spread=interp == "linear")
    peak = np.sum(np.abs(wts[row]))
    at = lambda d, p=None: oracle.sparse_filter_at(yb, l_lo, g, grid, offs, wts, [row], [a0], d, p, interp)[0]
    got = at(delta)
    assert abs(got - peak) < 1e-9 * peak
    assert abs(at(-delta)) < 0.9 * peak
    assert abs(at(np.zeros(g.n_pulses))) < 0.9 * peak
    assert abs(oracle.sparse_filter_at(yb, l_lo, g, grid, offs, wts, [row], [a0], interp=interp)[0]) < 0.9 * peak


def test_corrected_filter_phase_error_physical():
    """Data carrying a per-pulse phase error e^{+j psi_n}: the corrected filter given dpsi = psi
    refocuses the point to sum_k |w_k|; dpsi = -psi does not."""
    g, grid, offs, wts, l_lo, l_count, rng = _p4_case(62)
    row, a0 = 2, 100
    psi = rng.uniform(-np.pi, np.pi, g.n_pulses)
    yb = _recorded_point(g, grid, offs, row, a0, l_lo, l_count, psi=psi)
    peak = np.sum(np.abs(wts[row]))
    at = lambda p: oracle.sparse_filter_at(yb, l_lo, g, grid, offs, wts, [row], [a0], None, p)[0]
    assert abs(at(psi) - peak) < 1e-9 * peak
    assert abs(at(-psi)) < 0.9 * peak


@pytest.mark.parametrize("which", ["delta", "psi"])
def test_calibration_gradient_points_to_truth(which):
    """L = -|I(pixel)|^2 of the recorded point: its gradient vanishes at the true errors (the
    refocused maximum) and, one pulse's estimate moved by eps from the truth, has the sign of
    eps, so a gradient step moves the estimate back (LINEAR, derivatives of the corrected
    model)."""
    g, grid, offs, wts, l_lo, l_count, rng = _p4_case(63)
    row, a0 = 4, 60
    true = rng.normal(0, 3e-3, g.n_pulses) if which == "delta" else rng.uniform(-1, 1, g.n_pulses)
    kw = {which: true}
    yb = _recorded_point(g, grid, offs, row, a0, l_lo, l_count, spread=True, **kw)
    sub = synth.PolarGrid(grid.n_range, grid.n_az, grid.r0_m, grid.dr_m)

    def grad(est):
        dphi, dpsi = (est, None) if which == "delta" else (None, est)
        img = oracle.sparse_filter(yb, l_lo, g, sub, offs, wts, dphi, dpsi, "linear", rows=range(grid.n_range))
        gimg = np.zeros_like(img)
        gimg[row, a0] = -2.0 * img[row, a0]           # dL/dRe I + j dL/dIm I of L = -|I|^2
        _, gd, gp = oracle.sparse_filter_grad(yb, l_lo, g, sub, offs, wts, gimg,
                                              dphi if dphi is not None else np.zeros(g.n_pulses),
                                              dpsi if dpsi is not None else np.zeros(g.n_pulses), "linear")
        return gd if which == "delta" else gp

    at_truth = grad(true)
    pulses = (a0 + offs[row][[2, 9, 20]]) % g.n_pulses
    scale = np.sum(np.abs(wts[row])) ** 2
    assert np.max(np.abs(at_truth)) < 1e-9 * scale * (1e3 if which == "delta" else 1)
    eps = 2e-4 if which == "delta" else 0.05
    for n, sgn in zip(pulses, (1, -1, 1)):
        est = true.copy()
        est[n] += sgn * eps
        gn = grad(est)[n]
        assert np.sign(gn) == sgn and abs(gn) > 1e-6 * scale, (n, sgn, gn)


# --------------------------------------------------------------------------- LINEAR closed form
def _quadratic_band(g, l_lo, l_count, rng):
    """Y[n, l] = c0_n + c1_n l + c2_n l^2 in the absolute bin index l, complex coefficients."""
    c = rng.normal(size=(3, g.n_pulses)) + 1j * rng.normal(size=(3, g.n_pulses))
    c[2] *= 1e-2
    l = np.arange(l_lo, l_lo + l_count, dtype=np.float64)
    return c[0][:, None] + c[1][:, None] * l[None, :] + c[2][:, None] * l[None, :] ** 2, c


def _quadratic_read(c, n, u, interp):
    """What a sampler must return on the quadratic band at fractional bin u: NEAREST reads
    l = floor(u + 1/2); LINEAR is the chord between floor(u) and floor(u) + 1, which lies
    f (1 - f) (f = u - floor(u)) above the parabola l^2 (half its second difference, 2)."""
    if interp == "nearest":
        l = np.floor(u + 0.5)
        return c[0][n] + c[1][n] * l + c[2][n] * l * l
    f = u - np.floor(u)
    return c[0][n] + c[1][n] * u + c[2][n] * (u * u + f * (1.0 - f))


@pytest.mark.parametrize("interp", ["nearest", "linear"])
@pytest.mark.parametrize("corrected", [False, True])
def test_sparse_filter_quadratic_band_closed_form(interp, corrected):
    """The sparse filter on a band quadratic in the bin index equals
    sum_k conj(w_k) rot_k Q_n(u_k), u_k the beat bin of the x/y range from the phase centre
    (at its jittered angle when corrected) and rot_k = e^{-j 2k (R^ - R_nom)} e^{-j psi_n}.
    An extrapolating LINEAR index (ceil), swapped weights or a wrong bin fail it."""
    g, grid, offs, _, l_lo, l_count, rng = _p4_case(64 + corrected)
    yb, c = _quadratic_band(g, l_lo, l_count, rng)
    wts = rng.normal(size=offs.shape) + 1j * rng.normal(size=offs.shape)
    delta = rng.normal(0, 3e-3, g.n_pulses) if corrected else None
    psi = rng.uniform(-1, 1, g.n_pulses) if corrected else None
    k = oracle.wavenumber(g)
    rows, azs = rng.integers(0, grid.n_range, 12), rng.integers(0, grid.n_az, 12)
    got = oracle.sparse_filter_at(yb, l_lo, g, grid, offs, wts, rows, azs, delta, psi, interp)
    for i, (row, a) in enumerate(zip(rows, azs)):
        r_t, phi_t = grid.r0_m + row * grid.dr_m, g.phi0_rad + 2 * np.pi * a / grid.n_az
        want = 0j
        for kk, o in enumerate(offs[row]):
            n = (a + int(o)) % g.n_pulses
            nominal = g.phi0_rad + 2 * np.pi * n / g.n_pulses
            r_nom = cart_range(g, nominal, r_t, phi_t)
            r_hat = cart_range(g, nominal + (delta[n] if corrected else 0.0), r_t, phi_t)
            u = beat_bin(g, r_hat)
            assert l_lo + 1 <= u < l_lo + l_count - 2
            rot = np.exp(-2j * k * (r_hat - r_nom) - 1j * psi[n]) if corrected else 1.0
            want += np.conj(wts[row, kk]) * rot * _quadratic_read(c, n, u, interp)
        assert abs(got[i] - want) <= 1e-9 * abs(want), (row, a, got[i], want)


@pytest.mark.parametrize("interp", ["nearest", "linear"])
def test_bp_quadratic_band_closed_form(interp):
    """Back-projection on the quadratic band with jittered pulse angles equals
    sum over visible n of cos(theta_n) e^{-j 2k R_n} Q_n(u_n), with R_n, the bore-sight cosine
    and u_n from x/y positions."""
    g, grid, _, _, l_lo, l_count, rng = _p4_case(66)
    yb, c = _quadratic_band(g, l_lo, l_count, rng)
    ang = synth.nominal_angles(g) + rng.normal(0, 3e-3, g.n_pulses)
    k = oracle.wavenumber(g)
    rows, azs = rng.integers(0, grid.n_range, 6), rng.integers(0, grid.n_az, 6)
    got = oracle.bp_full_at(yb, l_lo, g, grid, rows, azs, pulse_angles=ang, interp=interp)
    for i, (row, a) in enumerate(zip(rows, azs)):
        r_t, phi_t = grid.r0_m + row * grid.dr_m, g.phi0_rad + 2 * np.pi * a / grid.n_az
        rn = cart_range(g, ang, r_t, phi_t)
        cb = boresight_cos(g, ang, r_t, phi_t)
        vis = cb > 0
        u = beat_bin(g, rn[vis])
        n = np.nonzero(vis)[0]
        want = np.sum(cb[vis] * np.exp(-2j * k * rn[vis]) * _quadratic_read(c, n, u, interp))
        assert abs(got[i] - want) <= 1e-9 * abs(want), (row, a)


# --------------------------------------------------------------------------- P5
def test_raw_domain_closed_form():
    """O1 then O2 on a simulated scatterer equals sum_k conj(w_k) alpha_k e^{j2kR_k} H(u_k - l_k)
    with H(x) = sum_m h[m] exp(j 2 pi x m / L) (eq. 39 at the selected bins)."""
    g = small_geom(360, 256, 0.25, 2e-6)
    grid = synth.PolarGrid(4, 360, 2.0, 0.05)
    wl = synth.Workload("p5", 42, g, grid, synth.SceneSpec(0, "unit", 1, 2), synth.SparseSpec(32, 64, False))
    offs = synth.make_support(wl)
    wts = synth.phase_matched_weights(g, grid, offs, synth.taylor_taper(64, 4, 30))
    row, a0 = 2, 100
    r_t, phi_t = grid.r0_m + row * grid.dr_m, 2 * np.pi * a0 / 360
    raw = synth.simulate_raw(g, synth.Scene(np.array([r_t]), np.array([phi_t]), np.array([1 + 0j])),
                             2 * np.pi * np.arange(360) / 360)
    h = synth.hann(g.n_fast).astype(np.float64)
    l_lo, l_count = synth.band_for(g, grid)
    y = oracle.range_compress(raw, h, g.n_fft)[:, l_lo:l_lo + l_count]
    got = oracle.sparse_filter_at(y, l_lo, g, grid, offs, wts, [row], [a0])[0]
    mm = np.arange(g.n_fast)
    ref = 0j
    for kk, o in enumerate(offs[row]):
        ang = 2 * np.pi * ((a0 + o) % 360) / 360
        rn = cart_range(g, ang, r_t, phi_t)
        u = beat_bin(g, rn)
        lsel = np.floor(u + 0.5)
        al = max(boresight_cos(g, ang, r_t, phi_t), 0.0)
        hx = np.sum(h * np.exp(2j * np.pi * (u - lsel) * mm / g.n_fft))
        ref += np.conj(wts[row, kk]) * al * np.exp(1j * carrier_phase(g, rn)) * hx
    # raw is stored in complex64: allow its rounding
    assert abs(got - ref) < 2e-6 * abs(ref)


# --------------------------------------------------------------------------- P6
def test_rotation_invariance():
    """Shifting the pulses one angular step circularly shifts the image one azimuth bin."""
    w = synth.small()
    x = synth.make_inputs(w)
    g, grid = w.geometry, w.grid
    y = oracle.range_compress(x.raw, x.window, g.n_fft)[:, x.l_lo:x.l_lo + x.l_count]
    rows = [0, 40, 127]
    i0 = oracle.sparse_filter(y, x.l_lo, g, grid, x.offsets, x.weights, rows=rows)
    i1 = oracle.sparse_filter(np.roll(y, 1, axis=0), x.l_lo, g, grid, x.offsets, x.weights, rows=rows)
    np.testing.assert_allclose(i1, np.roll(i0, 1, axis=1), rtol=0, atol=1e-12 * np.abs(i0).max())
    # back-projection with jittered angles: pulse n of the shifted set sits one step further on
    ang = synth.nominal_angles(g) + np.random.default_rng(3).normal(0, 1e-3, g.n_pulses)
    b0 = oracle.bp_full(y, x.l_lo, g, grid, ang, rows=rows)
    ang1 = np.roll(ang, 1) + 2 * np.pi / g.n_pulses
    b1 = oracle.bp_full(np.roll(y, 1, axis=0), x.l_lo, g, grid, ang1, rows=rows)
    np.testing.assert_allclose(b1, np.roll(b0, 1, axis=1), rtol=0, atol=1e-10 * np.abs(b0).max())


# --------------------------------------------------------------------------- P7
def test_bpa_equals_dense_sparse_filter():
    """With nominal angles, BPA equals the sparse filter whose support is every visible pulse and
    whose weights are the steering vector alpha e^{+j2kR} (eq. 16): two separately coded sums."""
    g = small_geom(64, 64, 0.3)
    grid = synth.PolarGrid(8, 64, 0.35, 0.2)
    l_lo, l_count = synth.band_for(g, grid)
    yb = synth.random_complex((64, l_count), seed=7).astype(np.complex128)
    n = g.n_pulses
    vis_sets = []
    for row in range(grid.n_range):
        r_t = grid.r0_m + row * grid.dr_m
        o = np.arange(-n // 2, n // 2)
        c = boresight_cos(g, 2 * np.pi * o / n, r_t, 0.0)
        vis_sets.append(o[c > 0])
    kmax = max(len(v) for v in vis_sets)
    offs = np.zeros((grid.n_range, kmax), np.int32)
    wts = np.zeros((grid.n_range, kmax), np.complex128)
    for row, v in enumerate(vis_sets):
        r_t = grid.r0_m + row * grid.dr_m
        pad = [o for o in range(-n // 2, n // 2) if o not in set(v.tolist())][:kmax - len(v)]
        offs[row] = np.concatenate([v, pad]).astype(np.int32)
        ang = 2 * np.pi * v / n
        rn = cart_range(g, ang, r_t, 0.0)
        wts[row, :len(v)] = boresight_cos(g, ang, r_t, 0.0) * np.exp(1j * carrier_phase(g, rn))
    for interp in ("nearest", "linear"):
        a = oracle.sparse_filter(yb, l_lo, g, grid, offs, wts, interp=interp)
        b = oracle.bp_full(yb, l_lo, g, grid, None, interp=interp)
        assert np.abs(a - b).max() < 1e-11 * np.abs(b).max()


# --------------------------------------------------------------------------- P8
def test_time_domain_bpa_brute_force():
    """Literal eq.-14 double sum (fast-time ramp at the selected bin) on tiny random data equals
    range FFT + BPA (eqs. 38, 43)."""
    g = small_geom(16, 16, 0.3)
    grid = synth.PolarGrid(3, 16, 0.9, 0.45)
    raw = synth.random_complex((16, 16), seed=21).astype(np.complex128)
    y = oracle.range_compress(raw, None, 16)
    got = oracle.bp_full(y, 0, g, grid)
    ref = np.zeros_like(got)
    for row in range(3):
        r_t = grid.r0_m + row * grid.dr_m
        for a in range(16):
            phi_t = 2 * np.pi * a / 16
            acc = 0j
            for n in range(16):
                ang = 2 * np.pi * n / 16
                cth = boresight_cos(g, ang, r_t, phi_t)
                if cth <= 0:
                    continue
                rn = cart_range(g, ang, r_t, phi_t)
                lsel = math.floor(beat_bin(g, rn) + 0.5)
                if not 0 <= lsel < 16:
                    continue
                for m in range(16):
                    acc += cth * np.exp(-2j * np.pi * lsel * m / 16) * np.exp(-1j * carrier_phase(g, rn)) * raw[n, m]
            ref[row, a] = acc
    np.testing.assert_allclose(got, ref, atol=1e-10 * np.abs(ref).max())


def test_time_domain_bpa_equals_fft_bpa_on_bins():
    """Radius -> 0 and range rows on FFT-bin centres: every tau_n K t_s lands on a bin, so the
    conventional BPA equals range FFT + BPA (NEAREST) for any window."""
    import dataclasses
    g0 = small_geom(32, 32, 1e-9)
    beta = oracle.bins_per_metre(g0)
    grid = synth.PolarGrid(4, 32, 6.0 / beta, 1.0 / beta)            # rows at bins 6..9
    raw = synth.random_complex((32, 32), seed=23).astype(np.complex128)
    win = synth.hann(32)
    yb = oracle.range_compress(raw, win, 32)
    rows = np.repeat(np.arange(4), 8)
    azs = np.tile(np.arange(0, 32, 4), 4)
    td = oracle.bp_time_domain_at(raw, win, g0, grid, rows, azs)
    ff = oracle.bp_full_at(yb, 0, g0, grid, rows, azs)
    np.testing.assert_allclose(td, ff, atol=1e-6 * np.abs(ff).max())
    assert dataclasses.is_dataclass(g0)


def test_time_domain_bpa_zero_padding_limit():
    """With r > 0 the beat frequencies fall between bins; range FFTs zero-padded to 1024 M bins
    read the nearest of a grid 1024 times finer, and FFT+BPA converges to the conventional
    BPA (phase error of the nearest-bin ramp over M samples <= pi M / L')."""
    import dataclasses
    g = small_geom(16, 16, 0.05)
    grid = synth.PolarGrid(3, 16, 0.2, 0.1)     # slant ranges within the 16-bin unambiguous range
    raw = synth.random_complex((16, 16), seed=24).astype(np.complex128)
    win = synth.hann(16)
    lp = 16 * 1024
    gp = dataclasses.replace(g, n_fft=lp)
    yb = oracle.range_compress(raw, win, lp)
    rows = np.repeat(np.arange(3), 16)
    azs = np.tile(np.arange(16), 3)
    td = oracle.bp_time_domain_at(raw, win, g, grid, rows, azs)
    ff = oracle.bp_full_at(yb, 0, gp, grid, rows, azs)
    assert metrics.rel_l2(ff, td) <= 2e-3
    # at the plain FFT length the nearest-bin reading is visibly different
    ff16 = oracle.bp_full_at(oracle.range_compress(raw, win, 16), 0, g, grid, rows, azs)
    assert metrics.rel_l2(ff16, td) > 1e-2


def _sas_case(n, m, r, r0, dr, rows, k, w, seed):
    g = small_geom(n, m, r)
    grid = synth.PolarGrid(rows, n, r0, dr)
    wl = synth.Workload("tdsas", seed, g, grid, synth.SceneSpec(0, "unit", 1, 2), synth.SparseSpec(k, w, False))
    offs = synth.make_support(wl)
    wts = synth.random_complex((rows, k), seed + 1).astype(np.complex128)
    raw = synth.random_complex((n, m), seed + 2).astype(np.complex128)
    return g, grid, offs, wts, raw


def test_time_domain_sas_equals_fft_sas_on_bins():
    """Radius -> 0 and range rows on bin centres: the sparse filter on raw samples equals range
    FFT + sparse filter (NEAREST) for any window."""
    g0 = small_geom(32, 32, 1e-9)
    beta = oracle.bins_per_metre(g0)
    g, grid, offs, wts, raw = _sas_case(32, 32, 1e-9, 6.0 / beta, 1.0 / beta, 4, 5, 8, 61)
    win = synth.hann(32)
    rows = np.repeat(np.arange(4), 32)
    azs = np.tile(np.arange(32), 4)
    td = oracle.sas_time_domain_at(raw, win, g, grid, offs, wts, rows, azs)
    ff = oracle.sparse_filter(oracle.range_compress(raw, win, 32), 0, g, grid, offs, wts).ravel()
    np.testing.assert_allclose(td, ff, atol=1e-6 * np.abs(ff).max())


def test_time_domain_sas_zero_padding_limit():
    """r > 0: FFT + sparse filter on range FFTs zero-padded to 1024 M bins converges to the
    sparse filter on raw samples; at the plain length the nearest-bin reading differs."""
    import dataclasses
    g, grid, offs, wts, raw = _sas_case(16, 16, 0.05, 0.2, 0.1, 3, 5, 8, 71)
    win = synth.hann(16)
    rows = np.repeat(np.arange(3), 16)
    azs = np.tile(np.arange(16), 3)
    td = oracle.sas_time_domain_at(raw, win, g, grid, offs, wts, rows, azs)
    lp = 16 * 1024
    gp = dataclasses.replace(g, n_fft=lp)
    ff = oracle.sparse_filter(oracle.range_compress(raw, win, lp), 0, gp, grid, offs, wts).ravel()
    assert metrics.rel_l2(ff, td) <= 2e-3
    ff16 = oracle.sparse_filter(oracle.range_compress(raw, win, 16), 0, g, grid, offs, wts).ravel()
    assert metrics.rel_l2(ff16, td) > 1e-2


@pytest.mark.parametrize("interp", ["nearest", "linear"])
def test_cartesian_on_polar_pixels(interp):
    """Cartesian targets on the four axes at the grid rows' radii coincide with polar pixels
    (phi on a pulse, R on a row): the Cartesian filter equals the polar one there."""
    w = synth.small()
    x = synth.make_inputs(w)
    g, grid = w.geometry, w.grid
    y = oracle.range_compress(x.raw, x.window, g.n_fft)[:, x.l_lo:x.l_lo + x.l_count]
    polar = oracle.sparse_filter(y, x.l_lo, g, grid, x.offsets, x.weights, interp=interp)
    radii = grid.r0_m + np.arange(grid.n_range) * grid.dr_m
    n = g.n_pulses
    for q, (cx, cy) in enumerate(((1, 0), (0, 1), (-1, 0), (0, -1))):
        got = oracle.sparse_filter_cartesian(y, x.l_lo, g, grid, cx * radii, cy * radii, x.offsets, x.weights, interp)
        np.testing.assert_allclose(got, polar[:, q * n // 4], atol=1e-9 * np.abs(polar).max())


def test_cartesian_rotation_invariance():
    """Rotating the targets by j pulse steps and the data by j pulses leaves the Cartesian image
    unchanged; the targets here sit between pulse angles (centre-pulse residual != 0)."""
    w = synth.small()
    x = synth.make_inputs(w)
    g, grid = w.geometry, w.grid
    y = oracle.range_compress(x.raw, x.window, g.n_fft)[:, x.l_lo:x.l_lo + x.l_count]
    rng = np.random.default_rng(3)
    rt = grid.r0_m + rng.uniform(0, grid.n_range - 1, 40) * grid.dr_m
    phi = rng.uniform(0, 2 * np.pi, 40)
    j = 7
    base = oracle.sparse_filter_cartesian(y, x.l_lo, g, grid, rt * np.cos(phi), rt * np.sin(phi), x.offsets,
                                          x.weights, "linear")
    rot = phi + j * 2 * np.pi / g.n_pulses
    moved = oracle.sparse_filter_cartesian(np.roll(y, j, axis=0), x.l_lo, g, grid, rt * np.cos(rot), rt * np.sin(rot),
                                           x.offsets, x.weights, "linear")
    np.testing.assert_allclose(moved, base, atol=1e-9 * np.abs(base).max())
    assert np.count_nonzero(np.abs(base) > 1e-6) > 30


def _steering_xy(geom, rr, phi_t, d):
    """eq. 16 element from explicit x/y positions: the phase centre at angle phi_t + d on the
    circle (bore-sight radial), the target at (rr, phi_t)."""
    k = oracle.wavenumber(geom)
    ang = phi_t + d
    dist = cart_range(geom, ang, rr, phi_t)
    return np.maximum(boresight_cos(geom, ang, rr, phi_t), 0.0) * np.exp(1j * 2 * k * dist)


def test_delta_r_cartesian_positions():
    """||a^ - a|| with both steering vectors built from perturbed and nominal x/y positions of the
    W phase centres (77 GHz, metres of range)."""
    g = small_geom(360, 64, 0.3)
    grid = synth.PolarGrid(5, 360, 0.6, 3.1)
    rng = np.random.default_rng(11)
    deltas = rng.normal(0, 2e-3, (50, 64))
    got = oracle.delta_r_samples(g, grid, 64, deltas)
    d0 = np.arange(-32, 32) * 2 * np.pi / 360
    for row in range(5):
        rr = grid.r0_m + row * grid.dr_m
        phi_t = 0.7
        want = np.linalg.norm(_steering_xy(g, rr, phi_t, d0[None, :] + deltas) - _steering_xy(g, rr, phi_t, d0)[None, :],
                              axis=1)
        np.testing.assert_allclose(got[row], want, rtol=1e-9)


def test_delta_r_cancellation_free_form():
    """The form the device evaluates, |alpha^ e^{j psi} - alpha|^2 = (alpha^ - alpha)^2
    + 4 alpha alpha^ sin^2(psi/2) with psi = 2k (R^2^ - R^2)/(R^ + R) and R^2^ - R^2 =
    4 R r sin((D + D^)/2) sin((D^ - D)/2), equals the oracle's direct difference of complex
    exponentials to 1e-9 at 77 GHz over 0.5-15 m."""
    g = small_geom(3600, 64, 0.3)
    grid = synth.PolarGrid(4, 3600, 0.5, 4.8)
    k = oracle.wavenumber(g)
    r = g.radius_m
    rng = np.random.default_rng(13)
    deltas = rng.normal(0, np.deg2rad(0.05), (40, 256))
    got = oracle.delta_r_samples(g, grid, 256, deltas)
    d0 = np.arange(-128, 128) * 2 * np.pi / 3600
    for row in range(4):
        rr = grid.r0_m + row * grid.dr_m
        d1 = d0[None, :] + deltas
        rn = np.sqrt(rr * rr + r * r - 2 * rr * r * np.cos(d0))
        rh = np.sqrt(rr * rr + r * r - 2 * rr * r * np.cos(d1))
        al = np.maximum(rr * np.cos(d0) - r, 0) / rn
        alh = np.maximum(rr * np.cos(d1) - r, 0) / rh
        psi = 2 * k * 4 * rr * r * np.sin((d0[None, :] + d1) / 2) * np.sin(deltas / 2) / (rh + rn[None, :])
        want = np.sqrt(np.sum((alh - al[None, :]) ** 2 + 4 * al[None, :] * alh * np.sin(psi / 2) ** 2, axis=1))
        np.testing.assert_allclose(got[row], want, rtol=1e-9)


def test_delta_r_small_sigma_linearisation():
    """Small sigma: E[Delta^2] -> sigma^2 sum_n |da_n/dphi|^2, the derivative taken by central
    differences of the directly evaluated steering vector."""
    g = small_geom(360, 64, 0.25)
    grid = synth.PolarGrid(3, 360, 1.0, 0.5)
    k = oracle.wavenumber(g)
    sigma = 1e-6
    rng = np.random.default_rng(12)
    deltas = rng.normal(0, sigma, (20000, 64))
    got = np.mean(oracle.delta_r_samples(g, grid, 64, deltas) ** 2, axis=1)
    d0 = np.arange(-32, 32) * 2 * np.pi / 360
    h = 1e-7
    for row in range(3):
        rr = grid.r0_m + row * grid.dr_m
        da = (_steering_xy(g, rr, 0.3, d0 + h) - _steering_xy(g, rr, 0.3, d0 - h)) / (2 * h)
        want = sigma ** 2 * np.sum(np.abs(da) ** 2)
        assert abs(got[row] - want) <= 0.03 * want, (row, got[row], want)


def test_delta_r_quantile():
    samples = np.array([[5.0, 1.0, 3.0, 2.0, 4.0]])
    assert oracle.delta_r(samples, 0.99)[0] == 5.0
    assert oracle.delta_r(samples, 0.6)[0] == 3.0      # ceil(0.6 * 5) = 3rd smallest


def _cartesian_steering(geom, rr, phi, offsets, k):
    """Tap elements from explicit positions: phase centre of tap o on the circle at angle
    o 2 pi / N, boresight radial; target at angle phi, range rr."""
    th = offsets * 2 * np.pi / geom.n_pulses
    px, py = geom.radius_m * np.cos(th), geom.radius_m * np.sin(th)
    tx, ty = rr * np.cos(phi), rr * np.sin(phi)
    dx, dy = tx - px, ty - py
    dist = np.hypot(dx, dy)
    cos_b = (dx * np.cos(th) + dy * np.sin(th)) / dist
    return np.maximum(cos_b, 0.0) * np.exp(1j * 2 * k * dist)


@pytest.mark.parametrize("jitter", [False, True])
def test_bp_cartesian_on_polar_pixels(jitter):
    """Back-projection for Cartesian targets placed on polar pixels equals the polar BPA there
    (nominal and jittered pulse angles, both interpolations)."""
    w = synth.small()
    if jitter:
        w = dataclasses.replace(w, scene=dataclasses.replace(w.scene, jitter_sigma_rad=np.deg2rad(0.05)))
    x = synth.make_inputs(w)
    g, grid = w.geometry, w.grid
    yb = oracle.range_compress(x.raw, x.window, g.n_fft)[:, x.l_lo:x.l_lo + x.l_count]
    ang = x.angles if jitter else None
    rng = np.random.default_rng(35)
    rows, azs = rng.integers(0, grid.n_range, 40), rng.integers(0, grid.n_az, 40)
    r = grid.r0_m + rows * grid.dr_m
    phi = g.phi0_rad + 2 * np.pi * azs / grid.n_az
    for interp in ("nearest", "linear"):
        want = oracle.bp_full_at(yb, x.l_lo, g, grid, rows, azs, pulse_angles=ang, interp=interp)
        got = oracle.bp_cartesian_at(yb, x.l_lo, g, r * np.cos(phi), r * np.sin(phi), pulse_angles=ang,
                                     interp=interp)
        np.testing.assert_allclose(got, want, rtol=1e-9, atol=1e-9 * np.abs(want).max())


def test_beampattern_matched_weights_cartesian():
    """Weights matched to the main-lobe steering vector built from explicit Cartesian positions:
    |w^H a(0)| = ||a(0)|| (Cauchy-Schwarz equality) and every other direction is <= it."""
    g = small_geom(360, 64, 0.25)
    grid = synth.PolarGrid(3, 360, 0.8, 0.9)
    k = oracle.wavenumber(g)
    rng = np.random.default_rng(31)
    offs = np.stack([np.sort(rng.choice(np.arange(-32, 32), 24, replace=False)) for _ in range(3)]).astype(np.int32)
    w = np.zeros((3, 24), complex)
    for i in range(3):
        rr = grid.r0_m + i * grid.dr_m
        a0 = _cartesian_steering(g, rr, 0.0, offs[i], k)
        w[i] = a0 / np.linalg.norm(a0)
    ang = np.concatenate([[0.0], np.linspace(-0.3, 0.3, 61)])
    pat = oracle.beampattern(g, grid, offs, w, 64, ang)
    for i in range(3):
        rr = grid.r0_m + i * grid.dr_m
        np.testing.assert_allclose(pat[i, 0], np.linalg.norm(_cartesian_steering(g, rr, 0.0, offs[i], k)), rtol=1e-12)
        for j, phi in enumerate(ang):
            want = abs(np.vdot(w[i], _cartesian_steering(g, rr, phi, offs[i], k)))
            np.testing.assert_allclose(pat[i, j], want, rtol=1e-9, atol=1e-12)
        assert pat[i, 1:].max() <= pat[i, 0] * (1 + 1e-12)


def test_beampattern_main_lobe_is_filter_response():
    """A unit scatterer at pixel (row, a0) whose data at each tap's bin is alpha e^{+j 2kR} (the
    carrier phase of the data model, amplitude the cosine pattern from Cartesian positions):
    the sparse filter's output there has the magnitude of the beampattern's main lobe, for
    arbitrary complex weights (so the steering vector's sign and conjugation are fixed)."""
    g = small_geom(180, 128, 0.25)
    w = synth.Workload("p14", 47, g, synth.PolarGrid(6, 180, 1.3, 0.11),
                       synth.SceneSpec(0, "unit", 1, 2), synth.SparseSpec(24, 64, False))
    offs = synth.make_support(w)
    rng = np.random.default_rng(34)
    wts = rng.normal(size=offs.shape) + 1j * rng.normal(size=offs.shape)
    l_lo, l_count = synth.band_for(g, w.grid)
    row, a0 = 3, 17
    yb = _bin_exact_scene(g, w.grid, offs, row, a0, l_lo, l_count)
    r_t = w.grid.r0_m + row * w.grid.dr_m
    phi_t = 2 * np.pi * a0 / 180
    for o in offs[row]:
        n = (a0 + int(o)) % 180
        ang = 2 * np.pi * n / 180
        px, py = g.radius_m * np.cos(ang), g.radius_m * np.sin(ang)
        dx, dy = r_t * np.cos(phi_t) - px, r_t * np.sin(phi_t) - py
        yb[n] *= (dx * np.cos(ang) + dy * np.sin(ang)) / np.hypot(dx, dy)
    img = oracle.sparse_filter_at(yb, l_lo, g, w.grid, offs, wts, np.array([row]), np.array([a0]))[0]
    sub = synth.PolarGrid(1, 180, r_t, 0.11)
    pat = oracle.beampattern(g, sub, offs[row:row + 1], wts[row:row + 1], 64, np.array([0.0]))[0, 0]
    np.testing.assert_allclose(abs(img), pat, rtol=1e-9)


def test_beampattern_offset_shift_invariance():
    """Shifting every offset by one pulse and the direction by one pulse step leaves D_k, hence
    the pattern, unchanged; taps shifted out of the window drop out."""
    g = small_geom(360, 64, 0.25)
    grid = synth.PolarGrid(2, 360, 1.0, 0.5)
    rng = np.random.default_rng(32)
    offs = np.stack([np.sort(rng.choice(np.arange(-30, 30), 16, replace=False)) for _ in range(2)]).astype(np.int32)
    w = rng.normal(size=(2, 16)) + 1j * rng.normal(size=(2, 16))
    ang = np.linspace(-0.2, 0.2, 41)
    a = oracle.beampattern(g, grid, offs, w, 64, ang)
    b = oracle.beampattern(g, grid, offs + 1, w, 64, ang + 2 * np.pi / 360)
    np.testing.assert_allclose(a, b, rtol=1e-9)
    offs2 = offs.copy()
    offs2[:, 0] = 40                      # outside [-32, 32): contributes nothing
    w2 = w.copy()
    w2[:, 0] = 0
    np.testing.assert_allclose(oracle.beampattern(g, grid, offs2, w, 64, ang),
                               oracle.beampattern(g, grid, offs, w2, 64, ang), rtol=1e-12)


def test_robust_summary_bounds_random_errors():
    """For unit-norm w and errors of norm <= Delta_R, |w^H (a + e)|^2 stays within the bounds the
    summary's ratio is built from, and the bound is reached by e along a (equality case)."""
    rng = np.random.default_rng(33)
    n = 40
    w = rng.normal(size=n) + 1j * rng.normal(size=n)
    w /= np.linalg.norm(w)
    am = rng.normal(size=n) + 1j * rng.normal(size=n)
    as_ = 0.2 * (rng.normal(size=n) + 1j * rng.normal(size=n))
    dr = 0.3
    main, side = abs(np.vdot(w, am)), abs(np.vdot(w, as_))
    ratio = oracle.robust_summary(np.array([main]), np.array([side]), np.array([dr]))[0]
    worst_m, worst_s = np.inf, 0.0
    for _ in range(2000):
        e = rng.normal(size=n) + 1j * rng.normal(size=n)
        e *= dr * rng.uniform() ** (1 / (2 * n)) / np.linalg.norm(e)
        worst_m = min(worst_m, abs(np.vdot(w, am + e)) ** 2)
        worst_s = max(worst_s, abs(np.vdot(w, as_ + e)) ** 2)
    assert worst_m >= (main - dr) ** 2 - 1e-12 and worst_s <= (side + dr) ** 2 + 1e-12
    assert worst_s / worst_m <= ratio
    e_eq = -dr * w * np.exp(1j * np.angle(np.vdot(w, am)))     # aligned with w, against w^H a_m
    np.testing.assert_allclose(abs(np.vdot(w, am + e_eq)), main - dr, rtol=1e-12)
    assert np.isinf(oracle.robust_summary(np.array([0.1]), np.array([0.0]), np.array([0.2]))[0])


# --------------------------------------------------------------------------- P9
def test_linearity():
    w = synth.small()
    x = synth.make_inputs(w)
    g, grid = w.geometry, w.grid
    y1 = synth.random_complex((g.n_pulses, x.l_count), 1).astype(np.complex128)
    y2 = synth.random_complex((g.n_pulses, x.l_count), 2).astype(np.complex128)
    rows = [5, 60]
    f = lambda y, wt: oracle.sparse_filter(y, x.l_lo, g, grid, x.offsets, wt, rows=rows)
    a, b = 0.3 - 1.2j, 2.0 + 0.5j
    np.testing.assert_allclose(f(a * y1 + b * y2, x.weights), a * f(y1, x.weights) + b * f(y2, x.weights), atol=1e-10)
    w2 = synth.random_complex(x.weights.shape, 3).astype(np.complex128)
    np.testing.assert_allclose(f(y1, a * x.weights + w2), np.conj(a) * f(y1, x.weights) + f(y1, w2), atol=1e-10)


# --------------------------------------------------------------------------- P10
def _calib_case():
    g = small_geom(96, 64, 0.25)
    grid = synth.PolarGrid(6, 96, 0.8, 0.07)
    wl = synth.Workload("p10", 43, g, grid, synth.SceneSpec(0, "unit", 1, 2), synth.SparseSpec(12, 32, False))
    offs = synth.make_support(wl)
    wts = synth.phase_matched_weights(g, grid, offs, synth.taylor_taper(32, 4, 30))
    l_lo, l_count = synth.band_for(g, grid)
    yb = synth.random_complex((96, l_count), 9).astype(np.complex128)
    rng = np.random.default_rng(4)
    dphi = rng.normal(0, 2e-3, 96)
    dpsi = rng.normal(0, 0.1, 96)
    return g, grid, offs, wts, l_lo, yb, dphi, dpsi


@pytest.mark.parametrize("interp", ["nearest", "linear"])
def test_adjoint_dot_product_weights(interp):
    g, grid, offs, wts, l_lo, yb, dphi, dpsi = _calib_case()
    gimg = synth.random_complex((grid.n_range, grid.n_az), 12).astype(np.complex128)
    dw = synth.random_complex(wts.shape, 13).astype(np.complex128)
    gw, _, _ = oracle.sparse_filter_grad(yb, l_lo, g, grid, offs, wts, gimg, dphi, dpsi, interp)
    img_dw = oracle.sparse_filter(yb, l_lo, g, grid, offs, dw, dphi, dpsi, interp)
    lhs = np.real(np.sum(np.conj(gimg) * img_dw))
    rhs = np.real(np.sum(np.conj(dw) * gw))
    assert abs(lhs - rhs) < 1e-12 * (abs(lhs) + 1)


@pytest.mark.parametrize("interp", ["nearest", "linear"])
@pytest.mark.parametrize("corrected", [False, True])
def test_adjoint_band_identity(interp, corrected):
    """<g, A Y> = <A^H g, Y> as complex numbers, A = sparse_filter as a linear map of the band."""
    g, grid, offs, wts, l_lo, yb, dphi, dpsi = _calib_case()
    if not corrected:
        dphi = dpsi = None
    gimg = synth.random_complex((grid.n_range, grid.n_az), 14).astype(np.complex128)
    img = oracle.sparse_filter(yb, l_lo, g, grid, offs, wts, dphi, dpsi, interp)
    gy = oracle.sparse_filter_adjoint_band(yb.shape[1], l_lo, g, grid, offs, wts, gimg, dphi, dpsi, interp)
    lhs = np.sum(np.conj(gimg) * img)
    rhs = np.sum(np.conj(gy) * yb)
    assert abs(lhs - rhs) < 1e-12 * (abs(lhs) + 1)


@pytest.mark.parametrize("interp", ["nearest", "linear"])
def test_adjoint_band_identity_narrow_band(interp):
    """The identity with a band narrower than the bins the taps read (those taps contribute
    nothing to either side)."""
    w = synth.small()
    x = synth.make_inputs(w)
    g, grid = w.geometry, w.grid
    lo, cnt = x.l_lo + 20, 15
    yb = synth.random_complex((g.n_pulses, cnt), 31).astype(np.complex128)
    gimg = synth.random_complex((grid.n_range, grid.n_az), 32).astype(np.complex128)
    img = oracle.sparse_filter(yb, lo, g, grid, x.offsets, x.weights, interp=interp)
    gy = oracle.sparse_filter_adjoint_band(cnt, lo, g, grid, x.offsets, x.weights, gimg, interp=interp)
    assert np.count_nonzero(img) < img.size            # some rows read nothing
    lhs = np.sum(np.conj(gimg) * img)
    rhs = np.sum(np.conj(gy) * yb)
    assert abs(lhs - rhs) < 1e-12 * (abs(lhs) + 1)


@pytest.mark.parametrize("interp", ["nearest", "linear"])
def test_adjoint_band_brute_force(interp):
    """Tiny case: the matrix of sparse_filter built column by column from unit band inputs;
    the adjoint equals conj(A)^T g."""
    geom = small_geom(16, 32, 0.25)
    grid = synth.PolarGrid(3, 16, 0.9, 0.11)
    wl = synth.Workload("adj", 44, geom, grid, synth.SceneSpec(0, "unit", 1, 2), synth.SparseSpec(5, 8, False))
    offs = synth.make_support(wl)
    wts = synth.random_complex((grid.n_range, 5), 21).astype(np.complex128)
    l_lo, l_count = synth.band_for(geom, grid)
    cols = []
    for n in range(16):
        for l in range(l_count):
            e = np.zeros((16, l_count), dtype=np.complex128)
            e[n, l] = 1.0
            cols.append(oracle.sparse_filter(e, l_lo, geom, grid, offs, wts, interp=interp).ravel())
    a = np.stack(cols, axis=1)                      # [pixels, N * l_count]
    gimg = synth.random_complex((grid.n_range, grid.n_az), 22).astype(np.complex128)
    want = (np.conj(a).T @ gimg.ravel()).reshape(16, l_count)
    got = oracle.sparse_filter_adjoint_band(l_count, l_lo, geom, grid, offs, wts, gimg, interp=interp)
    np.testing.assert_allclose(got, want, atol=1e-12)
    assert np.count_nonzero(np.abs(want) > 1e-9) > 10   # the case is not degenerate


def test_adjoint_finite_differences_linear():
    """Central differences (h = 1e-4) of L = Re<g, I> in delta, psi and w against the adjoint."""
    g, grid, offs, wts, l_lo, yb, dphi, dpsi = _calib_case()
    gimg = synth.random_complex((grid.n_range, grid.n_az), 14).astype(np.complex128)
    f = lambda w_, d_, p_: np.real(np.sum(np.conj(gimg) *
                                          oracle.sparse_filter(yb, l_lo, g, grid, offs, w_, d_, p_, "linear")))
    gw, gd, gp = oracle.sparse_filter_grad(yb, l_lo, g, grid, offs, wts, gimg, dphi, dpsi, "linear")
    h = 1e-4
    fd_d, fd_p, an_d, an_p = [], [], [], []
    for n in [0, 7, 33, 50, 95]:
        e = np.zeros(96); e[n] = h
        fd_d.append((f(wts, dphi + e, dpsi) - f(wts, dphi - e, dpsi)) / (2 * h)); an_d.append(gd[n])
        fd_p.append((f(wts, dphi, dpsi + e) - f(wts, dphi, dpsi - e)) / (2 * h)); an_p.append(gp[n])
    fd_d, an_d, fd_p, an_p = map(np.array, (fd_d, an_d, fd_p, an_p))
    assert np.linalg.norm(fd_d - an_d) <= 1e-3 * np.linalg.norm(an_d)
    assert np.linalg.norm(fd_p - an_p) <= 1e-3 * np.linalg.norm(an_p)
    for (row, kk) in [(0, 0), (3, 5), (5, 11)]:
        for unit in (1.0, 1j):
            e = np.zeros_like(wts); e[row, kk] = h * unit
            fd = (f(wts + e, dphi, dpsi) - f(wts - e, dphi, dpsi)) / (2 * h)
            an = gw[row, kk].real if unit == 1.0 else gw[row, kk].imag
            assert abs(fd - an) <= 1e-6 * (abs(an) + 1e-3)


def test_calibration_loss_gradient_chain():
    """Entropy + sidelobe loss: analytic dL/dI pulled back through the adjoint matches central
    differences of the full loss in delta and w."""
    g, grid, offs, wts, l_lo, yb, dphi, dpsi = _calib_case()
    mask = metrics.box_mask((grid.n_range, grid.n_az), [2, 4], [10, 70])
    loss = lambda w_, d_: metrics.calib_loss(
        oracle.sparse_filter(yb, l_lo, g, grid, offs, w_, d_, dpsi, "linear"), mask)[0]
    _, gimg = metrics.calib_loss(oracle.sparse_filter(yb, l_lo, g, grid, offs, wts, dphi, dpsi, "linear"), mask)
    gw, gd, _ = oracle.sparse_filter_grad(yb, l_lo, g, grid, offs, wts, gimg, dphi, dpsi, "linear")
    h = 1e-4
    fd, an = [], []
    for n in [3, 40, 77]:
        def cd(step):
            e = np.zeros(96); e[n] = step
            return (loss(wts, dphi + e) - loss(wts, dphi - e)) / (2 * step)
        # central differences at h and h/2 combined (Richardson) to cancel the O(h^2) term:
        # at 77 GHz a 1e-4 rad step already turns the phase by 2 k r h ~ 0.08 rad
        fd.append((4 * cd(h / 2) - cd(h)) / 3); an.append(gd[n])
    assert np.linalg.norm(np.array(fd) - an) <= 1e-3 * np.linalg.norm(an)
    e = np.zeros_like(wts); e[2, 3] = h
    fdw = (loss(wts + e, dphi) - loss(wts - e, dphi)) / (2 * h)
    assert abs(fdw - gw[2, 3].real) <= 1e-3 * abs(gw[2, 3].real) + 1e-9


# --------------------------------------------------------------------------- P11
def test_point_target_focus():
    """A simulated point focuses on its own pixel (BPA and sparse filter)."""
    g = synth.radar(3600, 512, 0.3)
    # place row 200 so the nearest slant range R - r sits on a bin centre (u = 206): the taps'
    # fractional bins then stay within [0, 0.2] and the residual phase of Remark 1 stays small
    # (at half-bin offsets NEAREST selection splits the taps between two bins and defocuses)
    row, a0 = 200, 1234
    r_row = 206.0 / oracle.bins_per_metre(g) + g.radius_m
    grid = synth.PolarGrid(400, 3600, r_row - row * 0.0375, 0.0375)
    r_t, phi_t = grid.r0_m + row * grid.dr_m, 2 * np.pi * a0 / 3600
    raw = synth.simulate_raw(g, synth.Scene(np.array([r_t]), np.array([phi_t]), np.array([1 + 0j])),
                             synth.nominal_angles(g))
    l_lo, l_count = synth.band_for(g, grid)
    y = oracle.range_compress(raw, synth.hann(512), 512)[:, l_lo:l_lo + l_count]
    wl = synth.Workload("p11", 44, g, grid, synth.SceneSpec(0, "unit", 1, 2), synth.SparseSpec(64, 256, False))
    offs = synth.make_support(wl)
    wts = synth.phase_matched_weights(g, grid, offs, synth.taylor_taper(256, 4, 30))
    rr, aa = np.meshgrid(np.arange(row - 3, row + 4), np.arange(a0 - 3, a0 + 4), indexing="ij")
    rr, aa = rr.ravel(), aa.ravel()
    for img in (oracle.bp_full_at(y, l_lo, g, grid, rr, aa),
                oracle.sparse_filter_at(y, l_lo, g, grid, offs, wts, rr, aa)):
        i = np.argmax(np.abs(img))
        assert (rr[i], aa[i]) == (row, a0)


# --------------------------------------------------------------------------- metrics
@pytest.mark.parametrize("m", [16, 64, 250])
def test_pisr_rect_aperture_closed_form(m):
    """Rectangular aperture of M (even) samples, transformed with 2M points (a circular cut):
    even bins are nulls, odd bin j has |X|^2 = csc^2(pi j / 2M), and the odd-bin sum is M^2, so
    with the main lobe {-2..2} (out to the first nulls) PISR = M^2 / (M^2 - 2 csc^2(pi / 2M))."""
    cut = np.fft.fft(np.ones(m), 2 * m)
    want = 10 * np.log10(m * m / (m * m - 2 / np.sin(np.pi / (2 * m)) ** 2))
    got = metrics.pisr_db(cut[None, :], [0], [0], m - 1)[0]
    assert got == pytest.approx(want, abs=1e-9)
    assert 7.0 < got < 7.5            # tends to -10 log10(1 - 8 / pi^2) = 7.24 dB


def test_entropy_closed_forms():
    assert metrics.image_entropy(np.ones((4, 8))) == pytest.approx(math.log(32), abs=1e-12)
    z = np.zeros((5, 5), complex); z[2, 3] = 3 - 4j
    assert metrics.image_entropy(z) == 0.0


def test_pslr_rect_sinc():
    """A rectangular-aperture response has its first sidelobe at -13.26 dB."""
    m = 64
    cut = dirichlet(np.arange(-512, 512) / (16 * m), m)          # 16x oversampled Dirichlet
    img = np.roll(cut, 512)[None, :]
    val, lobes, peaks = metrics.pslr_db(img, [0], [0], half_window=200, return_lobes=True)
    assert val[0] == pytest.approx(-13.26, abs=0.05)
    # first nulls of a 16x oversampled length-64 aperture: 16 bins either side of the peak
    assert lobes[0] == (16, 16) and peaks[0] == (0, 0)
    again = metrics.pslr_db(img * 3.0, [0], [0], 200, lobes=lobes, peaks=peaks)
    assert again[0] == pytest.approx(val[0], abs=1e-9)


def test_calib_loss_gradient_fd():
    rng = np.random.default_rng(2)
    img = rng.standard_normal((4, 6)) + 1j * rng.standard_normal((4, 6))
    mask = metrics.box_mask(img.shape, [1], [2], half=1)
    l0, g = metrics.calib_loss(img, mask)
    h = 1e-6
    for (i, j) in [(0, 0), (1, 2), (3, 5)]:
        for unit in (1, 1j):
            e = np.zeros_like(img); e[i, j] = h * unit
            fd = (metrics.calib_loss(img + e, mask)[0] - metrics.calib_loss(img - e, mask)[0]) / (2 * h)
            an = g[i, j].real if unit == 1 else g[i, j].imag
            assert fd == pytest.approx(an, rel=1e-5, abs=1e-8)


# --------------------------------------------------------------------------- generator
def test_generator_deterministic():
    a = synth.make_inputs(synth.small())
    b = synth.make_inputs(synth.small())
    assert a.raw.tobytes() == b.raw.tobytes()
    assert a.offsets.tobytes() == b.offsets.tobytes()
    assert a.weights.tobytes() == b.weights.tobytes()
    assert np.all(a.offsets >= -32) and np.all(a.offsets < 32)
    assert np.allclose(np.linalg.norm(a.weights, axis=1), 1.0)
