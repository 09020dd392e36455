"""Image-quality metrics and the calibration loss, FP64 (TEST INFRASTRUCTURE ONLY).

Image entropy follows eq. 45 (Sec. IV-C); the main-lobe width rule follows the half main-lobe
definition of Sec. IV-C.  NMSE, relative L2, PSLR and the sidelobe-energy term are not defined in
the paper; the definitions used here are stated in each docstring.
"""
from __future__ import annotations

import numpy as np


def nmse(img: np.ndarray, ref: np.ndarray) -> float:
    """||img - ref||^2 / ||ref||^2."""
    ref = ref.astype(np.complex128)
    return float(np.sum(np.abs(img.astype(np.complex128) - ref) ** 2) / np.sum(np.abs(ref) ** 2))


def rel_l2(img, ref) -> float:
    return float(np.sqrt(nmse(img, ref)))


def image_entropy(img: np.ndarray) -> float:
    """E_I = -sum d ln d, d = |I|^2 / sum |I|^2 (eq. 45), with 0 ln 0 = 0."""
    p = np.abs(img.astype(np.complex128)) ** 2
    d = p / p.sum()
    nz = d > 0
    return float(-np.sum(d[nz] * np.log(d[nz])))


def scatterer_pixels(grid, geom, r_m, phi_rad):
    """Nominal pixel (row, az) of each scatterer on the polar grid."""
    rows = np.rint((np.asarray(r_m) - grid.r0_m) / grid.dr_m).astype(np.int64)
    az = np.rint((np.asarray(phi_rad) - geom.phi0_rad) / (2 * np.pi / grid.n_az)).astype(np.int64) % grid.n_az
    return rows, az


def box_mask(shape, rows, azs, half: int = 3) -> np.ndarray:
    """True inside the +-half Chebyshev box (range clipped, azimuth circular) of each pixel."""
    m = np.zeros(shape, dtype=bool)
    n_r, n_a = shape
    for r0, a0 in zip(rows, azs):
        if r0 < -half or r0 >= n_r + half:
            continue
        rr = np.arange(max(r0 - half, 0), min(r0 + half + 1, n_r))
        aa = (a0 + np.arange(-half, half + 1)) % n_a
        m[np.ix_(rr, aa)] = True
    return m


def calib_loss(img: np.ndarray, mask: np.ndarray):
    """Calibration loss L = E_I + SLE / E, SLE = energy outside the scatterer boxes, E = total
    energy.  Returns (L, g) with g = dL/dRe(I) + j dL/dIm(I)."""
    img = img.astype(np.complex128)
    p = np.abs(img) ** 2
    e = p.sum()
    nz = p > 0
    lp = np.where(nz, np.log(np.where(nz, p, 1.0)), 0.0)
    s = np.sum(p * lp)
    ent = -s / e + np.log(e)
    sle = p[~mask].sum()
    loss = ent + sle / e
    dldp = np.where(nz, -lp / e + s / e ** 2, 0.0) + (~mask) / e - sle / e ** 2
    return float(loss), 2.0 * dldp * img


def pslr_db(img: np.ndarray, rows, azs, half_window: int, exclude: np.ndarray | None = None,
            search: int = 3, lobes=None, return_lobes: bool = False, peaks=None):
    """Peak sidelobe ratio (dB) on the circular azimuth cut through each scatterer's peak.

    Peak: max |I| within +-search bins of the nominal pixel.  Main lobe: from the peak out to
    the nearest local minimum on each side (the half main-lobe rule of Sec. IV-C), unless
    `lobes` gives the extents (lo, hi) to use; `peaks` likewise fixes the peak pixels (pr, pa).
    Taking both from a reference image compares two images over the same pixels.  Sidelobe:
    max |I|^2 within +-half_window bins of the peak outside the main lobe and outside `exclude`
    (boxes of other scatterers).  Returns one value per scatterer (nan where undefined), and
    with return_lobes also the extents and the peak pixels."""
    n_r, n_a = img.shape
    mag = np.abs(img.astype(np.complex128)) ** 2
    out = np.full(len(rows), np.nan)
    ext, pks = [], []
    for i, (r0, a0) in enumerate(zip(rows, azs)):
        if r0 < 0 or r0 >= n_r:
            ext.append((0, 0))
            pks.append((-1, -1))
            continue
        if peaks is not None:
            pr, pa = peaks[i]
        else:
            rr = np.arange(max(r0 - search, 0), min(r0 + search + 1, n_r))
            aa = (a0 + np.arange(-search, search + 1)) % n_a
            sub = mag[np.ix_(rr, aa)]
            ir, ia = np.unravel_index(np.argmax(sub), sub.shape)
            pr, pa = int(rr[ir]), int(aa[ia])
        pks.append((pr, pa))
        cut = mag[pr]
        if lobes is not None:
            lo, hi = lobes[i]
        else:
            lo = 0
            while lo < half_window and cut[(pa - lo - 1) % n_a] < cut[(pa - lo) % n_a]:
                lo += 1
            hi = 0
            while hi < half_window and cut[(pa + hi + 1) % n_a] < cut[(pa + hi) % n_a]:
                hi += 1
        ext.append((lo, hi))
        side = []
        for d in range(-half_window, half_window + 1):
            if -lo <= d <= hi:
                continue
            a = (pa + d) % n_a
            if exclude is not None and exclude[pr, a]:
                continue
            side.append(cut[a])
        if side and cut[pa] > 0:
            out[i] = 10 * np.log10(max(side) / cut[pa])
    return (out, ext, pks) if return_lobes else out


def pisr_db(img: np.ndarray, rows, azs, half_window: int, exclude: np.ndarray | None = None,
            search: int = 3, lobes=None, peaks=None):
    """Peak-to-integral sidelobe ratio (eq. 44) in dB, |I(phi_m, R)|^2 / sum_s |I(phi_s, R)|^2, on
    the circular azimuth cut through each scatterer's peak.  The peak and the main lobe are those
    of pslr_db (same `search`, `lobes`, `peaks`); the side-lobe directions phi_s are the bins
    within +-half_window of the peak outside the main lobe and outside `exclude`.  Higher is
    better.  One value per scatterer (nan where undefined)."""
    _, ext, pks = pslr_db(img, rows, azs, half_window, exclude, search, lobes, True, peaks)
    n_a = img.shape[1]
    mag = np.abs(img.astype(np.complex128)) ** 2
    out = np.full(len(rows), np.nan)
    for i, ((lo, hi), (pr, pa)) in enumerate(zip(ext, pks)):
        if pr < 0:
            continue
        side = 0.0
        for d in range(-half_window, half_window + 1):
            a = (pa + d) % n_a
            if -lo <= d <= hi or (exclude is not None and exclude[pr, a]):
                continue
            side += mag[pr, a]
        if side > 0 and mag[pr, pa] > 0:
            out[i] = 10 * np.log10(mag[pr, pa] / side)
    return out

