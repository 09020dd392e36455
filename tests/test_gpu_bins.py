"""GPU tests of the integer decisions of the path: the bin each NEAREST sample reads (eq. 40's
rounding of beta R, eq. 2) must be the oracle's, bit for bit, on the rotation workload's
geometry with jittered pulse angles.

The band encodes its own bin index, Y[n, l] = l (absolute bin, real), so |output| / |weight|
(or / alpha for back-projection) reveals exactly which bin a kernel read.  Mismatches are
allowed only where the oracle's own u lies within 1e-10 of a rounding boundary (where float64
evaluations that differ in the last bit may disagree); there should be none.

Also here: the corrected forward at the full rotation size with nonzero angle errors, on
sampled pixels."""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import assert_image, dev, inputs, log, need_gpu, oracle_band, to_dev, torch

pytestmark = pytest.mark.gpu

TIE = 1e-10


def index_band(rs, g, l_lo, l_count, halo, only_pulse=None):
    """Band rows [l_lo, l_lo + l_count) holding their absolute bin index (real), stored with
    halo copies; all pulses, or one."""
    n = g.n_pulses
    col = np.arange(l_lo, l_lo + l_count, dtype=np.float32)[:, None]
    yt = np.repeat(col, n, axis=1).astype(np.complex64)
    if only_pulse is not None:
        mask = np.zeros(n, dtype=np.float32)
        mask[only_pulse] = 1.0
        yt = yt * mask[None, :]
    full = np.concatenate([yt[:, n - halo:], yt, yt[:, :halo]], axis=1) if halo else yt
    rc = rs.empty_rc(n, l_lo, l_count, halo=halo, device=dev())
    rc.data.copy_(to_dev(np.ascontiguousarray(full)))
    return rc


def jitter_f32(w, x):
    """Per-pulse angle errors of the workload as the float32 the corrected filter takes."""
    d = x.angles - synth.nominal_angles(w.geometry)
    return d.astype(np.float32)


def plain_u(g, rr, d):
    """beta R(d) of eq. 2 / eq. 40 in float64, the oracle's expression (tie classification)."""
    return oracle.bins_per_metre(g) * oracle.slant_range(rr, g.radius_m, d)


def check_bins(got_bin, ref_bin, u_ref, what):
    """Every decoded bin equals the oracle's; mismatches only at rounding ties of the oracle's u."""
    bad = got_bin != ref_bin
    if not bad.any():
        return
    t = np.abs((u_ref[bad] + 0.5) - np.floor(u_ref[bad] + 0.5))
    near = np.minimum(t, 1 - t) < TIE
    assert near.all(), (what, int(bad.sum()), "mismatching bins, of which", int((~near).sum()),
                        "away from a rounding tie; first:", np.argwhere(bad)[:5].tolist())
    assert bad.sum() <= 2, (what, "too many ties", int(bad.sum()))


def test_corrected_forward_nearest_bins_rotation():
    """Corrected forward (NEAREST) with the rotation workload's jitter and random phase errors,
    K = 1 per row at a random offset of the W = 256 window, unit weight: |I| = the bin read
    (|rotation| = 1 to float32 rounding).  Four draws of the offsets: 14.7 M decisions."""
    rs = need_gpu()
    w, x = inputs("rotation")
    g, grid = w.geometry, w.grid
    n = g.n_pulses
    halo = w.sparse.window // 2
    rc = index_band(rs, g, x.l_lo, x.l_count, halo)
    dphi = jitter_f32(w, x)
    dpsi = np.random.default_rng(5).uniform(-np.pi, np.pi, n).astype(np.float32)
    wts = torch.ones((grid.n_range, 1), dtype=torch.complex64, device=dev())
    a = np.arange(n)
    for draw in range(4):
        offs = np.random.default_rng(100 + draw).integers(-halo, halo, (grid.n_range, 1)).astype(np.int32)
        log(f"corrected forward bins: draw {draw}")
        img = rs.sparse_filter(g, grid, rc, to_dev(offs), wts, w.sparse.window, dphi=to_dev(dphi), dpsi=to_dev(dpsi),
                               interp="nearest").cpu().numpy()
        got = np.rint(np.abs(img)).astype(np.int64)
        # the oracle's bin: floor(beta R^ + 1/2), R^ at angle o 2 pi / N + delta_n (eq. 2, eq. 37)
        ref = np.zeros_like(got)
        uref = np.zeros(got.shape)
        d64 = dphi.astype(np.float64)
        for r in range(grid.n_range):
            o = int(offs[r, 0])
            pn = (a + o) % n
            u = plain_u(g, grid.r0_m + r * grid.dr_m, o * oracle.rosar_oracle.TWO_PI / n + d64[pn])
            lb = np.floor(u + 0.5).astype(np.int64)
            ref[r] = np.where((lb >= x.l_lo) & (lb < x.l_lo + x.l_count), lb, 0)
            uref[r] = u
        check_bins(got, ref, uref, f"corrected forward draw {draw}")
        # the oracle's own image agrees on a sample of rows (its bins are the ones above)
        if draw == 0:
            yb = np.repeat(np.arange(x.l_lo, x.l_lo + x.l_count, dtype=np.float64)[None, :], n, axis=0)
            rows = [0, 511, grid.n_range - 1]
            sub = oracle.sparse_filter(yb.astype(np.complex128), x.l_lo, g, grid, offs, np.ones((grid.n_range, 1)),
                                       d64, dpsi.astype(np.float64), "nearest", rows=rows)
            assert np.array_equal(np.rint(np.abs(sub)).astype(np.int64), ref[rows])


def test_bp_nearest_bins_rotation():
    """Back-projection (NEAREST) with the rotation workload's true angles on a band that is zero
    except for one pulse, whose rows hold their bin index: |I| / alpha = the bin read for every
    pixel that pulse sees.  Four pulses: about 7 M decisions."""
    rs = need_gpu()
    w, x = inputs("rotation")
    g, grid = w.geometry, w.grid
    n = g.n_pulses
    beta = oracle.bins_per_metre(g)
    ang = to_dev(x.angles)
    phi_a = g.phi0_rad + oracle.rosar_oracle.TWO_PI * np.arange(grid.n_az) / grid.n_az
    for n0 in (0, 901, 1800, 3599):
        rc = index_band(rs, g, x.l_lo, x.l_count, 0, only_pulse=n0)
        log(f"bp bins: pulse {n0}")
        img = np.abs(rs.bp_full(g, grid, rc, angles=ang).cpu().numpy())
        got = np.zeros(img.shape, dtype=np.int64)
        ref = np.zeros(img.shape, dtype=np.int64)
        uref = np.zeros(img.shape)
        keep = np.zeros(img.shape, dtype=bool)
        for r in range(grid.n_range):
            vis, rn, alpha = oracle.bp_terms(g, grid, r, phi_a, x.angles[n0:n0 + 1])
            u = beta * rn[:, 0]
            lb = np.floor(u + 0.5).astype(np.int64)
            inband = (lb >= x.l_lo) & (lb < x.l_lo + x.l_count)
            ok = vis[:, 0] & (alpha[:, 0] > 0.05)
            keep[r] = ok
            ref[r] = np.where(inband, lb, 0)
            uref[r] = u
            got[r] = np.where(ok, np.rint(img[r] / np.where(ok, alpha[:, 0], 1.0)), 0).astype(np.int64)
            # pixels the pulse cannot see get nothing (up to float32 alpha at the field-of-view edge)
            assert np.all(img[r][~vis[:, 0]] < 1.0), (n0, r)
        assert keep.sum() > 1_000_000
        check_bins(got[keep], ref[keep], uref[keep], f"bp pulse {n0}")


def test_adjoint_nearest_bins_rotation():
    """Adjoint (NEAREST): a gradient image that is one-hot per row at a random pixel and K = 1
    give grad_w[r] = s[r, a_r] of the index band, |grad_w| = the bin read.  Eight draws."""
    rs = need_gpu()
    w, x = inputs("rotation")
    g, grid = w.geometry, w.grid
    n = g.n_pulses
    halo = w.sparse.window // 2
    rc = index_band(rs, g, x.l_lo, x.l_count, halo)
    dphi = jitter_f32(w, x)
    d64 = dphi.astype(np.float64)
    dpsi = torch.zeros(n, dtype=torch.float32, device=dev())
    wts = torch.ones((grid.n_range, 1), dtype=torch.complex64, device=dev())
    rows = np.arange(grid.n_range)
    for draw in range(8):
        rng = np.random.default_rng(200 + draw)
        offs = rng.integers(-halo, halo, (grid.n_range, 1)).astype(np.int32)
        a_r = rng.integers(0, n, grid.n_range)
        gimg = np.zeros((grid.n_range, n), dtype=np.complex64)
        gimg[rows, a_r] = 1.0
        log(f"adjoint bins: draw {draw}")
        gw, _, _ = rs.sparse_filter_backward(g, grid, rc, to_dev(offs), wts, w.sparse.window, to_dev(gimg),
                                             to_dev(dphi), dpsi, "nearest", need_phi=True, need_psi=True)
        got = np.rint(np.abs(gw.cpu().numpy()[:, 0])).astype(np.int64)
        o = offs[:, 0].astype(np.int64)
        pn = (a_r + o) % n
        rr = grid.r0_m + rows * grid.dr_m
        u = plain_u(g, rr, o * oracle.rosar_oracle.TWO_PI / n + d64[pn])
        lb = np.floor(u + 0.5).astype(np.int64)
        ref = np.where((lb >= x.l_lo) & (lb < x.l_lo + x.l_count), lb, 0)
        check_bins(got, ref, u, f"adjoint draw {draw}")


@pytest.mark.parametrize("interp", ["nearest", "linear"])
def test_corrected_forward_rotation_sampled(interp):
    """Corrected forward at the full rotation size with the workload's own angle errors
    (float32) and random phase errors, on real range-compressed data: 400 sampled pixels
    (grid corners and the azimuth wrap included) against the oracle, per pixel."""
    rs = need_gpu()
    w, x = inputs("rotation")
    g, grid = w.geometry, w.grid
    n = g.n_pulses
    dphi = jitter_f32(w, x)
    dpsi = np.random.default_rng(6).normal(0, 0.3, n).astype(np.float32)
    rc = rs.range_compress(g, to_dev(x.raw), to_dev(x.window), x.l_lo, x.l_count, halo=w.sparse.window // 2)
    log(f"corrected forward rotation sampled {interp}")
    img = rs.sparse_filter(g, grid, rc, to_dev(x.offsets), to_dev(x.weights.astype(np.complex64)), w.sparse.window,
                           dphi=to_dev(dphi), dpsi=to_dev(dpsi), interp=interp).cpu().numpy()
    rng = np.random.default_rng(7)
    rows = rng.integers(0, grid.n_range, 400)
    azs = rng.integers(0, grid.n_az, 400)
    rows[:4] = [0, 0, grid.n_range - 1, grid.n_range - 1]
    azs[:4] = [0, grid.n_az - 1, 0, grid.n_az - 1]
    ref = oracle.sparse_filter_at(oracle_band("rotation"), x.l_lo, g, grid, x.offsets, x.weights, rows, azs,
                                  dphi.astype(np.float64), dpsi.astype(np.float64), interp)
    assert_image(img[rows, azs], ref, 1e-4, interp)
    # the correction matters here: the uncorrected oracle is far from this image
    plain = oracle.sparse_filter_at(oracle_band("rotation"), x.l_lo, g, grid, x.offsets, x.weights, rows, azs,
                                    interp=interp)
    assert np.linalg.norm(plain - ref) > 0.1 * np.linalg.norm(ref)
