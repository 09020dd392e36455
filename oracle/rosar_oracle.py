"""Plain FP64 CPU oracle of the rotating-SAR imaging path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or execute this
module: only the test suite, the smoke check and the CPU-baseline leg of the benchmark do.
It shares no code with the HIP implementation.

Everything is numpy in float64 / complex128, written as the plain definitions of the paper's
equations, vectorised over one axis at most (azimuth for whole images, pulses or taps for
single pixels).  Notation follows the paper: N pulses per rotation, M fast-time samples,
L FFT points, r rotation radius, f_c carrier, K chirp slope (called `slope` here to keep K for
the tap count), F_s sampling rate, T_Start sampling start, k the wavenumber.

Readings of the paper taken here (each also an explicit argument of the HIP entry points):
  * The weight vector is applied conjugated, I = w^H y (eq. 43); the BPA coefficient applied
    to pulse n is alpha_n exp(-j 2 k R_n), i.e. BPA's w is the steering vector of eq. 16.
  * `round` in eq. 40 is floor(u + 1/2) (u >= 0), evaluated in float64.
  * FFT rows outside the computed band [l_lo, l_lo + l_count) read as 0.
  * Pulse indices wrap modulo N (the track is a closed circle, Sec. II-A).
  * Output azimuth bins coincide with the pulse grid (A = N), so Algorithm 2's centre pulse
    of pixel a is pulse a and a tap at offset o reads pulse (a + o) mod N.
  * Outside the +-90 deg field of view alpha = 0 (eqs. 3-5, 8): alpha = max(R cos D - r, 0)/R_n.
  * The residual Dirichlet phase after the range FFT (Remark 1) is not corrected.
  * Per-pulse angle errors delta_n (data taken at phi_n + delta_n, eq. 37) and phase errors
    psi_n enter the corrected sparse filter as s <- s exp(-j 2k (R^ - R_nom)) exp(-j psi_n).
  * Delta_R (eq. 37): the steering vector spans the sparse set's W-element window; the angle
    draws are inputs shared by every range row; the q point of the empirical CDF is the sample
    of rank ceil(q S) - 1 in ascending order.
"""
from __future__ import annotations

import math

import numpy as np

TWO_PI = 2.0 * math.pi


# ----------------------------------------------------------------------------- constants
def wavenumber(geom) -> float:
    """k = 2 pi (K T_Start + f_c) / c  (Sec. II-B after eq. 12, and Sec. III-D after eq. 38)."""
    return TWO_PI * (geom.slope_hz_s * geom.t_start_s + geom.fc_hz) / geom.c_m_s


def bins_per_metre(geom) -> float:
    """beta such that the peak bin of a target at slant range R is round(beta R) (eq. 40):
    beta = 2 K t_s L / c with t_s = 1/F_s."""
    return 2.0 * geom.slope_hz_s * geom.n_fft / (geom.fs_hz * geom.c_m_s)


def slant_range(r_t, r, dphi):
    """Distance from a phase centre on the circle of radius r to a point at range r_t whose
    azimuth differs by dphi (eq. 2)."""
    return np.sqrt(r_t * r_t + r * r - 2.0 * r * r_t * np.cos(dphi))


def visible_index_range(r_t: float, r: float, n: int) -> tuple[int, int]:
    """[N_min, N_max] of the phase centres that see a target at (pi/2, R_t) (eqs. 4-5)."""
    phi_v = math.acos(r / r_t)
    step = TWO_PI / n
    return math.ceil((math.pi / 2 - phi_v) / step), math.floor((math.pi / 2 + phi_v) / step)


# ----------------------------------------------------------------------- range compression
def range_compress(raw: np.ndarray, window: np.ndarray | None, n_fft: int) -> np.ndarray:
    """Y[n, l] = sum_m h[m] y[n, m] exp(-j 2 pi l m / L), l = 0..L-1 (eq. 38), zero-padded when
    L > M.  The window h is the input array (rectangular if None).  Uses the library FFT."""
    y = raw.astype(np.complex128)
    if window is not None:
        y = y * window.astype(np.float64)[None, :]
    return np.fft.fft(y, n=n_fft, axis=1)


def range_compress_direct(raw: np.ndarray, window: np.ndarray | None, n_fft: int) -> np.ndarray:
    """Literal DFT sum of eq. 38 (tiny sizes only)."""
    n_p, m = raw.shape
    h = np.ones(m) if window is None else window.astype(np.float64)
    out = np.zeros((n_p, n_fft), dtype=np.complex128)
    for n in range(n_p):
        for l in range(n_fft):
            acc = 0j
            for mm in range(m):
                acc += h[mm] * complex(raw[n, mm]) * complex(math.cos(-TWO_PI * l * mm / n_fft),
                                                             math.sin(-TWO_PI * l * mm / n_fft))
            out[n, l] = acc
    return out


# ----------------------------------------------------------------------------- sampling
def _band(yb: np.ndarray, n: np.ndarray, l: np.ndarray) -> np.ndarray:
    """Y_1D[n, l] read from the computed band; rows outside it read as 0."""
    ok = (l >= 0) & (l < yb.shape[1])
    lc = np.where(ok, l, 0)
    return np.where(ok, yb[n, lc], 0.0)


def sample(yb: np.ndarray, l_lo: int, n: np.ndarray, u: np.ndarray, interp: str):
    """Range-compressed sample of pulse n at fractional bin u, and its derivative d/du.
    nearest: Y[n, round(u)] (eq. 40 with round = floor(u + 1/2)); derivative 0.
    linear:  (1-f) Y[n, i] + f Y[n, i+1], i = floor(u), f = u - i."""
    if interp == "nearest":
        l = np.floor(u + 0.5).astype(np.int64) - l_lo
        return _band(yb, n, l), np.zeros(np.shape(u), dtype=np.complex128)
    if interp == "linear":
        fl = np.floor(u)
        f = u - fl
        i = fl.astype(np.int64) - l_lo
        y0 = _band(yb, n, i)
        y1 = _band(yb, n, i + 1)
        return (1.0 - f) * y0 + f * y1, y1 - y0
    raise ValueError(interp)


# ----------------------------------------------------------------------- sparse filter (FFT+SAS)
def _row_taps(geom, grid, row: int, o: int, n: np.ndarray, dphi, dpsi, yb, l_lo, interp):
    """Sample s and its partial derivatives for range row `row`, tap offset o, pulses n."""
    r = geom.radius_m
    rr = grid.r0_m + row * grid.dr_m
    beta = bins_per_metre(geom)
    k = wavenumber(geom)
    d0 = o * TWO_PI / geom.n_pulses
    dl = np.zeros(n.shape) if dphi is None else dphi[n].astype(np.float64)
    d = d0 + dl
    r_hat = slant_range(rr, r, d)
    s, dsdu = sample(yb, l_lo, n, beta * r_hat, interp)
    corrected = dphi is not None or dpsi is not None
    if corrected:
        r_nom = slant_range(rr, r, d0)
        ps = np.zeros(n.shape) if dpsi is None else dpsi[n].astype(np.float64)
        rot = np.exp(-1j * 2.0 * k * (r_hat - r_nom)) * np.exp(-1j * ps)
    else:
        rot = np.ones(n.shape, dtype=np.complex128)
    drdd = rr * r * np.sin(d) / r_hat
    ds_ddelta = rot * (beta * dsdu - 1j * 2.0 * k * s) * drdd
    return s * rot, ds_ddelta


def sparse_filter(yb: np.ndarray, l_lo: int, geom, grid, offsets: np.ndarray, weights: np.ndarray,
                  dphi=None, dpsi=None, interp: str = "nearest", rows=None) -> np.ndarray:
    """Sparse-aperture azimuth filter over range-compressed data (Algorithm 2 with eq. 43):
        I[r, a] = sum_k conj(w[r, k]) s[r, a, k],
        s = Y_1D[n, u(R^)],  n = (a + o_k) mod N,  R^ = R(o_k 2 pi/N + delta_n)  (eq. 2),
    u = beta R^ (eq. 40), with the delta/psi correction when either is given.
    yb: [N, l_count] rows [l_lo, l_lo + l_count) of Y_1D.  Returns [n_rows, A] complex128."""
    n_p = geom.n_pulses
    assert grid.n_az == n_p
    rows = range(grid.n_range) if rows is None else rows
    a = np.arange(grid.n_az)
    out = np.zeros((len(rows), grid.n_az), dtype=np.complex128)
    for i, row in enumerate(rows):
        for kk in range(offsets.shape[1]):
            o = int(offsets[row, kk])
            n = (a + o) % n_p
            s, _ = _row_taps(geom, grid, row, o, n, dphi, dpsi, yb, l_lo, interp)
            out[i] += np.conj(weights[row, kk]) * s
    return out


def steering_vector(geom, rr: float, d):
    """Element a_n of the steering vector (eq. 16) of a target at range rr seen from a phase
    centre whose angle differs from the target's by d: cos(theta'_n) exp(+j 2 k R_n), with R_n
    from eq. 2 and cos(theta'_n) = max(R cos D - r, 0) / R_n (the field-of-view reading)."""
    k = wavenumber(geom)
    r = geom.radius_m
    rn = slant_range(rr, r, d)
    return np.maximum(rr * np.cos(d) - r, 0.0) / rn * np.exp(1j * 2.0 * k * rn)


def delta_r_samples(geom, grid, window: int, deltas: np.ndarray) -> np.ndarray:
    """Monte-Carlo samples of Delta^_R = ||a^(phi; R) - a(phi; R)|| (Sec. III-C parameter
    settings, eq. 37), straight from the definition: a is the steering vector (eq. 16) of the W
    phase centres around the target direction, D_n = o 2 pi / N for offsets o in [-W/2, W/2);
    a^ is the same vector with each angle perturbed by the given draw,
    D^_n = D_n + deltas[s, o + W/2].  Both vectors are evaluated as complex exponentials in
    float64 and subtracted.  Returns [n_range, S]."""
    o = np.arange(-(window // 2), window // 2)
    d0 = o * TWO_PI / geom.n_pulses
    out = np.zeros((grid.n_range, deltas.shape[0]))
    for row in range(grid.n_range):
        rr = grid.r0_m + row * grid.dr_m
        a = steering_vector(geom, rr, d0)
        a_hat = steering_vector(geom, rr, d0[None, :] + deltas)
        out[row] = np.linalg.norm(a_hat - a[None, :], axis=1)
    return out


def delta_r(samples: np.ndarray, q: float = 0.99) -> np.ndarray:
    """Delta_R per row: the smallest sample whose empirical CDF reaches q (the 99 % point of the
    Monte-Carlo distribution, Sec. III-C), i.e. sorted[ceil(q S) - 1]."""
    s = np.sort(samples, axis=1)
    idx = int(np.ceil(q * samples.shape[1])) - 1
    return s[:, idx]


def beampattern(geom, grid, offsets: np.ndarray, weights: np.ndarray, window: int,
                angles: np.ndarray) -> np.ndarray:
    """|w^H a(phi; R)| of each range row's sparse weights (Sec. III-A, eq. 16 and C1/C2 of
    eq. 20): a target at angle phi from a pixel's direction is seen by tap k (pulse a + o_k) at
    D_k = phi - o_k 2 pi / N, with a_k = alpha(D_k) exp(+j 2 k R(D_k)) (eq. 16's sign, the data's
    carrier phase; the filter applies conj(w)), R from eq. 2 and alpha
    = max(R cos D - r, 0) / R(D) as in BPA.  Taps outside [-W/2, W/2) contribute nothing (the
    filter's rule).  Returns [n_range, len(angles)]."""
    k = wavenumber(geom)
    r = geom.radius_m
    step = TWO_PI / geom.n_pulses
    out = np.zeros((grid.n_range, len(angles)))
    half = window // 2
    for row in range(grid.n_range):
        rr = grid.r0_m + row * grid.dr_m
        o = offsets[row].astype(np.int64)
        keep = (o >= -half) & (o < half)
        d = angles[:, None] - o[None, keep] * step                     # [A, K']
        rn = slant_range(rr, r, d)
        al = np.maximum(rr * np.cos(d) - r, 0.0) / rn
        a = al * np.exp(1j * 2.0 * k * rn)
        out[row] = np.abs(a @ np.conj(weights[row, keep]))
    return out


def robust_summary(main: np.ndarray, side_max: np.ndarray, delta_r: np.ndarray) -> np.ndarray:
    """Worst case over array errors of norm <= Delta_R for a unit-norm w (the Cauchy-Schwarz and
    triangle bounds of Sec. III-A): main-lobe gain >= (|w^H a_m| - Delta_R)^2, side-lobe response
    <= (|w^H a_s| + Delta_R)^2.  Returns their ratio per row (+inf when |w^H a_m| <= Delta_R);
    a design meets C2 relative to C1 when it is <= eta."""
    lo = main - delta_r
    hi = side_max + delta_r
    with np.errstate(divide="ignore"):
        return np.where(lo > 0, hi * hi / np.where(lo > 0, lo * lo, 1.0), np.inf)


def sparse_filter_cartesian(yb: np.ndarray, l_lo: int, geom, grid, xs: np.ndarray, ys: np.ndarray,
                            offsets: np.ndarray, weights: np.ndarray, interp: str = "nearest") -> np.ndarray:
    """Algorithm 2 for targets at Cartesian positions (xs[i], ys[i]) (FFT+SAS form, eq. 43):
    R_t = |(x, y)|, phi_t = atan2(y, x); the weights are those of the polar grid row nearest to
    R_t (pixels farther than half a row spacing outside the rows read nothing); the central
    phase centre is n_c = round((phi_t - phi0) / phi_Delta); tap k reads pulse
    n = (n_c + o_k) mod N at the bin of the slant range from that pulse to the target (eq. 2,
    eq. 40):  I = sum_k conj(w[row, k]) Y_1D[n, u(R(phi_t - phi_n))]."""
    n_p = geom.n_pulses
    step = TWO_PI / n_p
    rt = np.hypot(xs, ys)
    phi = np.arctan2(ys, xs)
    nc = np.floor((phi - geom.phi0_rad) / step + 0.5).astype(np.int64)
    row = np.floor((rt - grid.r0_m) / grid.dr_m + 0.5).astype(np.int64)
    inside = (row >= 0) & (row < grid.n_range)
    rowc = np.where(inside, row, 0)
    beta = bins_per_metre(geom)
    out = np.zeros(len(xs), dtype=np.complex128)
    for kk in range(offsets.shape[1]):
        o = offsets[rowc, kk].astype(np.int64)
        nn = nc + o
        d = phi - (geom.phi0_rad + nn * step)
        u = beta * slant_range(rt, geom.radius_m, d)
        s, _ = sample(yb, l_lo, nn % n_p, u, interp)
        out += np.where(inside, np.conj(weights[rowc, kk]) * s, 0.0)
    return out


def sparse_filter_at(yb, l_lo, geom, grid, offsets, weights, rows, azs, dphi=None, dpsi=None,
                     interp="nearest") -> np.ndarray:
    """The same sum as sparse_filter, evaluated pixel by pixel at (rows[i], azs[i])."""
    out = np.zeros(len(rows), dtype=np.complex128)
    for i, (row, a) in enumerate(zip(rows, azs)):
        acc = 0j
        for kk in range(offsets.shape[1]):
            o = int(offsets[row, kk])
            n = np.array([(a + o) % geom.n_pulses])
            s, _ = _row_taps(geom, grid, row, o, n, dphi, dpsi, yb, l_lo, interp)
            acc += np.conj(weights[row, kk]) * s[0]
        out[i] = acc
    return out


def sparse_filter_adjoint_band(l_count: int, l_lo: int, geom, grid, offsets, weights, grad_image, dphi=None,
                               dpsi=None, interp: str = "nearest") -> np.ndarray:
    """Adjoint of sparse_filter with respect to the range-compressed band: sparse_filter is
    linear in Y, I[r, a] = sum_k conj(w[r, k]) rot c_l Y_1D[n, l] over the bins l the sample of
    tap k reads with interpolation weights c_l (eq. 40; 1 for NEAREST, 1 - f and f for LINEAR),
    n = (a + o_k) mod N, rot the delta/psi correction (1 without).  For a real loss with
    g = dL/dRe(I) + j dL/dIm(I) the gradient with respect to Y is
        grad_Y[n, l] = sum over (r, a, k) reading (n, l) of w[r, k] conj(rot) c_l g[r, a],
    i.e. A^H g for the linear map A.  Bins outside the band get nothing.  Returns
    [N, l_count] complex128 in the layout of the band argument of sparse_filter."""
    n_p = geom.n_pulses
    r = geom.radius_m
    beta = bins_per_metre(geom)
    k = wavenumber(geom)
    a = np.arange(grid.n_az)
    out = np.zeros((n_p, l_count), dtype=np.complex128)
    for row in range(grid.n_range):
        rr = grid.r0_m + row * grid.dr_m
        g = grad_image[row].astype(np.complex128)
        for kk in range(offsets.shape[1]):
            o = int(offsets[row, kk])
            n = (a + o) % n_p
            d0 = o * TWO_PI / n_p
            d = d0 + (np.zeros(n.shape) if dphi is None else dphi[n].astype(np.float64))
            r_hat = slant_range(rr, r, d)
            u = beta * r_hat
            rot = np.ones(n.shape, dtype=np.complex128)
            if dphi is not None or dpsi is not None:
                ps = np.zeros(n.shape) if dpsi is None else dpsi[n].astype(np.float64)
                rot = np.exp(-1j * 2.0 * k * (r_hat - slant_range(rr, r, d0))) * np.exp(-1j * ps)
            if interp == "nearest":
                parts = [(np.floor(u + 0.5).astype(np.int64) - l_lo, np.ones(n.shape))]
            elif interp == "linear":
                fl = np.floor(u)
                f = u - fl
                i = fl.astype(np.int64) - l_lo
                parts = [(i, 1.0 - f), (i + 1, f)]
            else:
                raise ValueError(interp)
            contrib = weights[row, kk] * np.conj(rot) * g
            for l, c in parts:
                ok = (l >= 0) & (l < l_count)
                # n is a permutation of 0..N-1 for a fixed tap, so the fancy-index add is exact
                out[n[ok], l[ok]] += c[ok] * contrib[ok]
    return out


# ----------------------------------------------------------------------- full-aperture BPA
def bp_terms(geom, grid, row: int, phi_a, pulse_angles):
    """Visibility, slant range and pattern weight of every (pixel, pulse) pair of one range row:
    D = phi_a - phi^_n, v = R cos D - r, visible iff v > 0 (eqs. 4-5),
    R_n from eq. 2, alpha = v / R_n = cos(theta_n) (eqs. 3, 8, 15)."""
    r = geom.radius_m
    rr = grid.r0_m + row * grid.dr_m
    d = np.subtract.outer(np.atleast_1d(phi_a), pulse_angles)
    v = rr * np.cos(d) - r
    rn = slant_range(rr, r, d)
    vis = v > 0
    alpha = np.where(vis, v / rn, 0.0)
    return vis, rn, alpha


def _angles(geom, pulse_angles):
    if pulse_angles is None:
        return geom.phi0_rad + TWO_PI * np.arange(geom.n_pulses) / geom.n_pulses
    return np.asarray(pulse_angles, dtype=np.float64)


def bp_full(yb, l_lo, geom, grid, pulse_angles=None, interp="nearest", rows=None) -> np.ndarray:
    """Full-aperture back-projection over range-compressed data ("FFT+BPA", eq. 43 with the BPA
    weights): I[r, a] = sum over visible n of alpha_n exp(-j 2 k R_n) Y_1D[n, u(R_n)],
    phi_a = phi0 + 2 pi a / A, pulses at their given angles phi^_n."""
    ang = _angles(geom, pulse_angles)
    beta = bins_per_metre(geom)
    k = wavenumber(geom)
    rows = range(grid.n_range) if rows is None else rows
    phi_a = geom.phi0_rad + TWO_PI * np.arange(grid.n_az) / grid.n_az
    n_idx = np.arange(geom.n_pulses)
    out = np.zeros((len(rows), grid.n_az), dtype=np.complex128)
    for i, row in enumerate(rows):
        vis, rn, alpha = bp_terms(geom, grid, row, phi_a, ang)          # [A, N]
        s, _ = sample(yb, l_lo, np.broadcast_to(n_idx, rn.shape), beta * rn, interp)
        term = alpha * np.exp(-1j * 2.0 * k * rn) * s
        out[i] = np.where(vis, term, 0.0).sum(axis=1)
    return out


def bp_cartesian_at(yb, l_lo, geom, xs, ys, pulse_angles=None, interp="nearest") -> np.ndarray:
    """Full-aperture back-projection for targets at Cartesian positions (xs[i], ys[i]) (eq. 43
    with the BPA weights, as bp_full for a polar pixel): R_t = |(x, y)|, phi_t = atan2(y, x),
    D = phi_t - phi^_n, visible iff R_t cos D - r > 0 (eqs. 4-5), and
    I = sum over visible n of alpha_n exp(-j 2 k R_n) Y_1D[n, u(R_n)]."""
    ang = _angles(geom, pulse_angles)
    beta = bins_per_metre(geom)
    k = wavenumber(geom)
    r = geom.radius_m
    n_idx = np.arange(geom.n_pulses)
    out = np.zeros(len(xs), dtype=np.complex128)
    for i, (x, y) in enumerate(zip(xs, ys)):
        rt, phi = math.hypot(x, y), math.atan2(y, x)
        d = phi - ang
        v = rt * np.cos(d) - r
        rn = slant_range(rt, r, d)
        s, _ = sample(yb, l_lo, n_idx, beta * rn, interp)
        out[i] = np.where(v > 0, v / rn * np.exp(-1j * 2.0 * k * rn) * s, 0.0).sum()
    return out


def bp_full_at(yb, l_lo, geom, grid, rows, azs, pulse_angles=None, interp="nearest") -> np.ndarray:
    """bp_full evaluated pixel by pixel at (rows[i], azs[i])."""
    ang = _angles(geom, pulse_angles)
    beta = bins_per_metre(geom)
    k = wavenumber(geom)
    n_idx = np.arange(geom.n_pulses)
    out = np.zeros(len(rows), dtype=np.complex128)
    for i, (row, a) in enumerate(zip(rows, azs)):
        phi_a = geom.phi0_rad + TWO_PI * a / grid.n_az
        vis, rn, alpha = bp_terms(geom, grid, row, phi_a, ang)
        s, _ = sample(yb, l_lo, n_idx, beta * rn[0], interp)
        out[i] = np.where(vis[0], alpha[0] * np.exp(-1j * 2.0 * k * rn[0]) * s, 0.0).sum()
    return out


# ----------------------------------------------------------------------- adjoint
def sas_time_domain_at(raw, window, geom, grid, offsets, weights, rows, azs) -> np.ndarray:
    """Sparse-aperture filter on the raw samples (the W_SA compensation of Sec. II-C followed by
    the weights, before range compression), pixel by pixel at (rows[i], azs[i]):
        I = sum_k conj(w[r, k]) sum_m h[m] y[n_k, m] exp(-j 2 pi tau_k K m t_s),
    n_k = (a + o_k) mod N, tau_k = 2 R(o_k 2 pi / N) / c (eq. 2), h the range window.  The
    weights carry the carrier phase and the pattern; the ramp uses the exact beat frequency,
    where FFT+SAS reads the nearest FFT bin (eq. 40)."""
    n_p, m_s = raw.shape
    h = np.ones(m_s) if window is None else np.asarray(window, dtype=np.float64)
    hy = raw.astype(np.complex128) * h[None, :]
    m = np.arange(m_s)
    out = np.zeros(len(rows), dtype=np.complex128)
    for i, (row, a) in enumerate(zip(rows, azs)):
        rr = grid.r0_m + row * grid.dr_m
        o = offsets[row].astype(np.int64)
        n = (a + o) % n_p
        r_hat = slant_range(rr, geom.radius_m, o * TWO_PI / n_p)
        f = 2.0 * r_hat / geom.c_m_s * geom.slope_hz_s / geom.fs_hz
        d = np.sum(np.exp(-2j * np.pi * np.outer(f, m)) * hy[n], axis=1)
        out[i] = np.sum(np.conj(weights[row]) * d)
    return out


def bp_time_domain_at(raw, window, geom, grid, rows, azs, pulse_angles=None) -> np.ndarray:
    """Conventional time-domain BPA (the W_BP Hadamard sum of Sec. II-C, before range
    compression), pixel by pixel at (rows[i], azs[i]):
        I = sum over visible n of alpha_n exp(-j 2 k R_n) sum_m h[m] y[n, m] exp(-j 2 pi tau_n K m t_s)
    with tau_n = 2 R_n / c, t_s = 1 / F_s, visibility and alpha as in bp_full (eqs. 3-5, 8,
    15), h the range window (rect if None).  The fast-time ramp uses the exact beat frequency,
    where FFT+BPA reads the nearest FFT bin."""
    n_p, m_s = raw.shape
    h = np.ones(m_s) if window is None else np.asarray(window, dtype=np.float64)
    hy = raw.astype(np.complex128) * h[None, :]
    k = wavenumber(geom)
    angles = _angles(geom, pulse_angles)
    m = np.arange(m_s)
    out = np.zeros(len(rows), dtype=np.complex128)
    for i, (row, a) in enumerate(zip(rows, azs)):
        phi_a = geom.phi0_rad + TWO_PI * a / grid.n_az
        vis, rn, alpha = bp_terms(geom, grid, row, phi_a, angles)
        vis, rn, alpha = vis[0], rn[0], alpha[0]
        nv = np.nonzero(vis)[0]
        tau = 2.0 * rn[nv] / geom.c_m_s
        ramp = np.exp(-2j * np.pi * np.outer(tau * geom.slope_hz_s / geom.fs_hz, m))   # [visible, M]
        d = np.sum(ramp * hy[nv], axis=1)
        out[i] = np.sum(alpha[nv] * np.exp(-2j * k * rn[nv]) * d)
    return out


def sparse_filter_grad(yb, l_lo, geom, grid, offsets, weights, grad_image, dphi=None, dpsi=None,
                       interp="linear"):
    """Exact derivatives of sparse_filter for a real loss, in the convention
    g = dL/dRe(I) + j dL/dIm(I) (the same convention is returned for the complex weights):
        grad_w[r, k]  = sum_a conj(g[r, a]) s[r, a, k]
        grad_delta[n] = sum_{r,k} Re(conj(g) conj(w) ds/ddelta_n)
        grad_psi[n]   = sum_{r,k} Im(conj(g) conj(w) s)
    with a = (n - o_k) mod N, ds/ddelta = rot (beta dY/du - j 2k Y) R_r r sin(D)/R^.
    The derivatives are those of the corrected model (delta = psi = 0 when not given)."""
    n_p = geom.n_pulses
    dphi = np.zeros(n_p) if dphi is None else dphi
    dpsi = np.zeros(n_p) if dpsi is None else dpsi
    a = np.arange(grid.n_az)
    gw = np.zeros(weights.shape, dtype=np.complex128)
    gd = np.zeros(n_p)
    gp = np.zeros(n_p)
    for row in range(grid.n_range):
        g = grad_image[row].astype(np.complex128)
        for kk in range(offsets.shape[1]):
            o = int(offsets[row, kk])
            n = (a + o) % n_p
            s, dsd = _row_taps(geom, grid, row, o, n, dphi, dpsi, yb, l_lo, interp)
            gw[row, kk] = np.sum(np.conj(g) * s)
            z = np.conj(g) * np.conj(weights[row, kk])
            gd[n] += np.real(z * dsd)       # n is a permutation of 0..N-1 for fixed o
            gp[n] += np.imag(z * s)
    return gw, gd, gp
