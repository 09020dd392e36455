"""GPU parity: every kernel of the imaging path against the FP64 oracle, through the C ABI.

Bar (stated per test): relative L2 <= 1e-4 for complex64 storage with FP32 arithmetic,
<= 1e-2 for FP16/BF16 storage, <= 1e-3 for gradients; bit-exact where the arithmetic is
identical by construction (launch shapes, rotation shift, halo copies)."""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import assert_image, custom_workload, dev, inputs, log, need_gpu, oracle_band, rel_l2, to_dev, torch

pytestmark = pytest.mark.gpu

TOL = 1e-4


def upload(w, x, halo=None, dtype="c64", scale=1.0, rs=None):
    g = w.geometry
    halo = w.sparse.window // 2 if halo is None else halo
    rc = rs.range_compress(g, to_dev(x.raw), to_dev(x.window), x.l_lo, x.l_count, halo=halo, dtype=dtype,
                           scale=scale)
    return rc, to_dev(x.offsets), to_dev(x.weights.astype(np.complex64))


def rc_from_band(rs, w, yb, l_lo, halo):
    """Upload an oracle band (rounded to complex64) as range-compressed input."""
    n = w.geometry.n_pulses
    rc = rs.empty_rc(n, l_lo, yb.shape[1], halo=halo, device=dev())
    yt = np.ascontiguousarray(yb.T.astype(np.complex64))              # [l_count, N]
    full = np.concatenate([yt[:, n - halo:], yt, yt[:, :halo]], axis=1) if halo else yt
    rc.data.copy_(to_dev(full))
    return rc


# ------------------------------------------------------------------ range compression
@pytest.mark.parametrize("dtype", ["c64", "f16", "bf16"])
def test_range_compress_small(dtype):
    rs = need_gpu()
    w, x = inputs("small")
    log(f"range_compress small dtype={dtype}")
    scale = 2.0 ** -4 if dtype == "f16" else 1.0
    rc, _, _ = upload(w, x, halo=32, dtype=dtype, scale=scale, rs=rs)
    torch.cuda.synchronize()
    got = rc.pulses(w.geometry.n_pulses).cpu().numpy().T                # [N, l_count]
    ref = oracle_band("small")
    tol = 1e-5 if dtype == "c64" else 5e-3
    assert rel_l2(got, ref) <= tol
    # halo columns are exact copies of the wrapped pulses
    d = rc.data.cpu()
    n = w.geometry.n_pulses
    assert torch.equal(d[:, :32], d[:, n:n + 32]) and torch.equal(d[:, n + 32:n + 64], d[:, 32:64])


@pytest.mark.parametrize("n,m,l", [(100, 200, 256), (70, 64, 64), (64, 2048, 2048), (129, 1000, 1024),
                                   # mixed-radix path: the paper's M = L = 225, other 2^a 3^b 5^c, 4096
                                   (800, 225, 225), (37, 90, 100), (40, 3000, 4096), (20, 7000, 7200)])
def test_range_compress_shapes(n, m, l):
    """Zero padding (M < L), the smallest and largest FFT, ragged pulse counts, and lengths of
    the mixed-radix path; odd and even halos."""
    rs = need_gpu()
    log(f"range_compress N={n} M={m} L={l}")
    g = synth.Geometry(n, m, l, 0.25, 77e9, 4e9 * 1e7 / m, 1e7)
    raw = synth.random_complex((n, m), seed=n + m)
    win = synth.hann(m)
    l_lo, l_cnt = 3, l - 7
    ref = oracle.range_compress(raw, win, l)[:, l_lo:l_lo + l_cnt]
    # an odd halo takes the element-wise band store; an even one (with even N) the paired store
    for halo in (5, 6):
        rc = rs.range_compress(g, to_dev(raw), to_dev(win), l_lo, l_cnt, halo=halo)
        torch.cuda.synchronize()
        assert rel_l2(rc.pulses(n).cpu().numpy().T, ref) <= 1e-5, halo
        d = rc.data.cpu()
        assert torch.equal(d[:, :halo], d[:, n:n + halo]) and torch.equal(d[:, n + halo:], d[:, halo:2 * halo])
    rc2 = rs.range_compress(g, to_dev(raw), None, 0, l, halo=0)
    torch.cuda.synchronize()
    assert rel_l2(rc2.pulses(n).cpu().numpy().T, oracle.range_compress(raw, None, l)) <= 1e-5


@pytest.mark.parametrize("name", ["rotation", "precision"])
@pytest.mark.parametrize("dtype", ["c64", "f16"])
def test_range_compress_full_size(name, dtype):
    """The rotation (3600 x 512) and precision (7200 x 1024) workloads at full size: every band
    element against the FP64 oracle's windowed FFT (whole-pulse loads and paired band stores),
    and the halo columns as exact copies of the wrapped pulses."""
    rs = need_gpu()
    w = getattr(synth, name)()
    x = synth.make_inputs(w)
    g = w.geometry
    n, halo = g.n_pulses, w.sparse.window // 2
    scale = 2.0 ** -6 if dtype == "f16" else 1.0
    log(f"range_compress full size {name} {dtype}")
    rc = rs.range_compress(g, to_dev(x.raw), to_dev(x.window), x.l_lo, x.l_count, halo=halo, dtype=dtype,
                           scale=scale)
    torch.cuda.synchronize()
    got = rc.pulses(n).cpu().numpy().T                                   # [N, l_count]
    ref = oracle.range_compress(x.raw, x.window, g.n_fft)[:, x.l_lo:x.l_lo + x.l_count]
    tol = 1e-5 if dtype == "c64" else 2e-3
    assert rel_l2(got, ref) <= tol
    assert np.abs(got - ref).max() <= 10 * tol * np.abs(ref).max()
    d = rc.data.cpu()
    assert torch.equal(d[:, :halo], d[:, n:n + halo]) and torch.equal(d[:, n + halo:], d[:, halo:2 * halo])


def test_range_compress_mixed_f16():
    """Mixed-radix path with FP16 storage and a power-of-two scale."""
    rs = need_gpu()
    n, m, l = 64, 225, 225
    g = synth.Geometry(n, m, l, 0.145, 60e9, 4e9 * 1e7 / m, 1e7)
    raw = synth.random_complex((n, m), seed=5)
    win = synth.hann(m)
    log("range_compress mixed f16")
    rc = rs.range_compress(g, to_dev(raw), to_dev(win), 10, 150, halo=8, dtype="f16", scale=2.0 ** -4)
    torch.cuda.synchronize()
    got = rc.pulses(n).cpu().numpy().T
    ref = oracle.range_compress(raw, win, l)[:, 10:160]
    assert rel_l2(got, ref) <= 1e-3


def test_paper_radar_end_to_end():
    """The paper's radar (N = 800, M = L = 225 through the mixed-radix range FFT, r = 0.145 m,
    60 GHz, T_Start = 7 us) on a polar grid: range compression + sparse filter (both
    interpolations) and BPA against the FP64 oracle."""
    import dataclasses
    rs = need_gpu()
    w = custom_workload("paper_radar", 77, 800, 225, 24, 0.5, 2.5, 32, 64, radius=0.145)
    g = dataclasses.replace(w.geometry, fc_hz=60e9, t_start_s=7e-6)
    w = dataclasses.replace(w, geometry=g)
    x = synth.make_inputs(w)
    yb = oracle.range_compress(x.raw, x.window, g.n_fft)[:, x.l_lo:x.l_lo + x.l_count]
    rc = rs.range_compress(g, to_dev(x.raw), to_dev(x.window), x.l_lo, x.l_count, halo=32)
    torch.cuda.synchronize()
    assert rel_l2(rc.pulses(g.n_pulses).cpu().numpy().T, yb) <= 1e-5
    off, wts = to_dev(x.offsets), to_dev(x.weights.astype(np.complex64))
    for interp in ("nearest", "linear"):
        log(f"paper radar sparse filter {interp}")
        img = rs.sparse_filter(g, w.grid, rc, off, wts, w.sparse.window, interp=interp).cpu().numpy()
        ref = oracle.sparse_filter(yb, x.l_lo, g, w.grid, x.offsets, x.weights, interp=interp)
        assert_image(img, ref, TOL, interp)
    log("paper radar BPA")
    bpa = rs.bp_full(g, w.grid, rc).cpu().numpy()
    assert_image(bpa, oracle.bp_full(yb, x.l_lo, g, w.grid), TOL)


# ------------------------------------------------------------------ sparse filter
def test_sparse_filter_small_end_to_end():
    rs = need_gpu()
    w, x = inputs("small")
    log("sparse_filter small end to end")
    rc, off, wts = upload(w, x, rs=rs)
    img = rs.sparse_filter(w.geometry, w.grid, rc, off, wts, w.sparse.window)
    torch.cuda.synchronize()
    ref = oracle.sparse_filter(oracle_band("small"), x.l_lo, w.geometry, w.grid, x.offsets, x.weights)
    assert_image(img.cpu().numpy(), ref, TOL)


SHAPES = [(v, p, nw) for v in (1, 2) for p in (1, 2, 4, 8) for nw in (1, 2, 4, 8) if not (p == 8 and nw == 8)]


def test_sparse_filter_launch_shapes_bit_identical():
    """Every launch shape runs the same per-pixel FMA sequence: identical bits, oracle parity."""
    rs = need_gpu()
    w, x = inputs("small")
    yb = oracle_band("small")
    rc = rc_from_band(rs, w, yb, x.l_lo, 32)
    off, wts = to_dev(x.offsets), to_dev(x.weights.astype(np.complex64))
    ref = oracle.sparse_filter(yb, x.l_lo, w.geometry, w.grid, x.offsets, x.weights)
    first = None
    for t in SHAPES:
        log(f"sparse_filter tile={t}")
        img = rs.sparse_filter(w.geometry, w.grid, rc, off, wts, w.sparse.window, tile=t).cpu()
        assert_image(img.numpy(), ref, TOL, t)
        if first is None:
            first = img
        assert torch.equal(img, first), t


@pytest.mark.parametrize("interp", ["nearest", "linear"])
def test_sparse_filter_halo_and_wrap(interp):
    """halo = 0 (explicit modulo-N wrap) and halo = W/2 (direct reads) agree with the oracle."""
    rs = need_gpu()
    w, x = inputs("small")
    yb = oracle_band("small")
    ref = oracle.sparse_filter(yb, x.l_lo, w.geometry, w.grid, x.offsets, x.weights, interp=interp)
    off, wts = to_dev(x.offsets), to_dev(x.weights.astype(np.complex64))
    outs = []
    for halo in (0, 7, 32):
        log(f"sparse_filter halo={halo} interp={interp}")
        rc = rc_from_band(rs, w, yb, x.l_lo, halo)
        img = rs.sparse_filter(w.geometry, w.grid, rc, off, wts, w.sparse.window, interp=interp).cpu().numpy()
        assert_image(img, ref, TOL, halo)
        outs.append(img)
    np.testing.assert_allclose(outs[0], outs[2], rtol=0, atol=1e-6 * np.abs(ref).max())


EDGE = [
    # name, N, M, rows, r0, r1, K, W
    ("ragged_n_k5", 100, 128, 9, 0.6, 2.5, 5, 16),
    ("k100_gt_wave", 300, 256, 6, 0.8, 4.0, 100, 128),
    ("k1", 64, 64, 3, 0.5, 1.2, 1, 2),
    ("w_equals_n", 96, 64, 4, 0.5, 1.0, 40, 96),
    ("many_rows", 128, 64, 300, 0.4, 1.4, 12, 32),
]


@pytest.mark.parametrize("case", EDGE, ids=[c[0] for c in EDGE])
@pytest.mark.parametrize("interp", ["nearest", "linear"])
def test_sparse_filter_edge_cases(case, interp):
    rs = need_gpu()
    name, n, m, rg, r0, r1, k, win = case
    w = custom_workload(name, 60 + len(name), n, m, rg, r0, r1, k, win)
    x = synth.make_inputs(w)
    log(f"sparse_filter edge {name} interp={interp}")
    yb = oracle.range_compress(x.raw, x.window, m)[:, x.l_lo:x.l_lo + x.l_count]
    ref = oracle.sparse_filter(yb, x.l_lo, w.geometry, w.grid, x.offsets, x.weights, interp=interp)
    rc = rs.range_compress(w.geometry, to_dev(x.raw), to_dev(x.window), x.l_lo, x.l_count, halo=win // 2)
    img = rs.sparse_filter(w.geometry, w.grid, rc, to_dev(x.offsets), to_dev(x.weights.astype(np.complex64)),
                           win, interp=interp).cpu().numpy()
    assert_image(img, ref, TOL)


def test_sparse_filter_narrow_band():
    """Taps whose bin falls outside the stored band read zero, as in the oracle."""
    rs = need_gpu()
    w, x = inputs("small")
    y = oracle.range_compress(x.raw, x.window, w.geometry.n_fft)
    lo, cnt = 40, 30
    yb = y[:, lo:lo + cnt]
    log("sparse_filter narrow band")
    ref = oracle.sparse_filter(yb, lo, w.geometry, w.grid, x.offsets, x.weights)
    rc = rs.range_compress(w.geometry, to_dev(x.raw), to_dev(x.window), lo, cnt, halo=32)
    img = rs.sparse_filter(w.geometry, w.grid, rc, to_dev(x.offsets), to_dev(x.weights.astype(np.complex64)),
                           w.sparse.window).cpu().numpy()
    assert_image(img, ref, TOL)
    assert np.count_nonzero(img) < img.size     # rows far outside the band are exactly zero


@pytest.mark.parametrize("interp", ["nearest", "linear"])
@pytest.mark.parametrize("which", ["dphi", "dpsi", "both"])
def test_sparse_filter_corrected(interp, which):
    rs = need_gpu()
    w, x = inputs("small")
    yb = oracle_band("small")
    rng = np.random.default_rng(17)
    n = w.geometry.n_pulses
    dphi = rng.normal(0, 3e-3, n).astype(np.float32) if which in ("dphi", "both") else None
    dpsi = rng.normal(0, 0.3, n).astype(np.float32) if which in ("dpsi", "both") else None
    log(f"sparse_filter corrected {which} {interp}")
    ref = oracle.sparse_filter(yb, x.l_lo, w.geometry, w.grid, x.offsets, x.weights,
                               dphi=None if dphi is None else dphi.astype(np.float64),
                               dpsi=None if dpsi is None else dpsi.astype(np.float64), interp=interp)
    rc = rc_from_band(rs, w, yb, x.l_lo, 32)
    img = rs.sparse_filter(w.geometry, w.grid, rc, to_dev(x.offsets), to_dev(x.weights.astype(np.complex64)),
                           w.sparse.window, dphi=None if dphi is None else to_dev(dphi),
                           dpsi=None if dpsi is None else to_dev(dpsi), interp=interp).cpu().numpy()
    assert_image(img, ref, TOL)


@pytest.mark.parametrize("interp", ["nearest", "linear"])
@pytest.mark.parametrize("halo_half", [False, True])
def test_sparse_filter_corrected_wide_window(interp, halo_half):
    """A window too wide for the corrected kernel's LDS pulse table (tile + W > 4096 columns):
    the per-pulse angle/phase terms come from global memory for every pair.  With halo 0 the
    pulse columns wrap modulo N explicitly."""
    rs = need_gpu()
    n, win = 3200, 3200
    w = custom_workload("wide_window", 71, n, 64, 6, 0.6, 1.5, 16, win)
    x = synth.make_inputs(w)
    rng = np.random.default_rng(23)
    dphi = rng.normal(0, 2e-3, n).astype(np.float32)
    dpsi = rng.normal(0, 0.3, n).astype(np.float32)
    log(f"sparse_filter corrected wide window {interp} halo_half={halo_half}")
    yb = oracle.range_compress(x.raw, x.window, 64)[:, x.l_lo:x.l_lo + x.l_count]
    ref = oracle.sparse_filter(yb, x.l_lo, w.geometry, w.grid, x.offsets, x.weights, dphi=dphi.astype(np.float64),
                               dpsi=dpsi.astype(np.float64), interp=interp)
    rc = rs.range_compress(w.geometry, to_dev(x.raw), to_dev(x.window), x.l_lo, x.l_count,
                           halo=win // 2 if halo_half else 0)
    img = rs.sparse_filter(w.geometry, w.grid, rc, to_dev(x.offsets), to_dev(x.weights.astype(np.complex64)),
                           win, dphi=to_dev(dphi), dpsi=to_dev(dpsi), interp=interp).cpu().numpy()
    assert_image(img, ref, TOL)


PATH_CASES = [
    # name, n, window, rows r0..r1, K, angle-error sigma; the paths these take (checked on the
    # CPU from the kernels' series bound and the rows each range row's taps reach):
    ("staged", 1024, 64, 0.6, 1.4, 32, 2e-3),          # rows 1-3 staged in LDS, row 0 exact
    ("series_global", 2048, 1536, 0.6, 1.4, 32, 1e-3),  # series, tile + W past the staging limit
    ("exact", 1024, 64, 0.6, 1.4, 32, 0.05),           # large errors: the exact correction
    ("near_rows", 1024, 256, 0.27, 0.4, 32, 2e-4),      # series, taps spanning 5-6 bin rows
]


@pytest.mark.parametrize("interp", ["nearest", "linear"])
@pytest.mark.parametrize("case", PATH_CASES, ids=[c[0] for c in PATH_CASES])
def test_corrected_forward_and_adjoint_paths(case, interp):
    """Corrected forward and adjoint against the oracle on shapes that take each path of the
    kernels: staged series rows, series with gathers from global memory (the window too wide to
    stage), the exact correction (errors beyond the series bound) and rows whose taps span many
    bin rows.  The image and the three gradients each meet the bars of the small-workload tests."""
    rs = need_gpu()
    name, n, win, r0, r1, k, sig = case
    w = custom_workload(f"path_{name}", 81 + PATH_CASES.index(case), n, 64, 4, r0, r1, k, win)
    x = synth.make_inputs(w)
    rng = np.random.default_rng(41)
    dphi = rng.normal(0, sig, n).astype(np.float32)
    dpsi = rng.normal(0, 0.3, n).astype(np.float32)
    yb = oracle.range_compress(x.raw, x.window, 64)[:, x.l_lo:x.l_lo + x.l_count]
    rc = rs.range_compress(w.geometry, to_dev(x.raw), to_dev(x.window), x.l_lo, x.l_count, halo=win // 2)
    off, wts = to_dev(x.offsets), to_dev(x.weights.astype(np.complex64))
    log(f"corrected forward path {name} {interp}")
    ref = oracle.sparse_filter(yb, x.l_lo, w.geometry, w.grid, x.offsets, x.weights, dphi=dphi.astype(np.float64),
                               dpsi=dpsi.astype(np.float64), interp=interp)
    img = rs.sparse_filter(w.geometry, w.grid, rc, off, wts, win, dphi=to_dev(dphi), dpsi=to_dev(dpsi),
                           interp=interp).cpu().numpy()
    assert_image(img, ref, TOL, name)
    log(f"adjoint path {name} {interp}")
    gimg = synth.random_complex((w.grid.n_range, n), seed=43)
    gw_r, gd_r, gp_r = oracle.sparse_filter_grad(yb, x.l_lo, w.geometry, w.grid, x.offsets, x.weights,
                                                 gimg.astype(np.complex128), dphi.astype(np.float64),
                                                 dpsi.astype(np.float64), interp)
    gw, gd, gp = rs.sparse_filter_backward(w.geometry, w.grid, rc, off, wts, win, to_dev(gimg), to_dev(dphi),
                                           to_dev(dpsi), interp)
    assert rel_l2(gw.cpu().numpy(), gw_r) <= 1e-3, name
    assert rel_l2(gd.cpu().numpy(), gd_r) <= 1e-3, name
    assert rel_l2(gp.cpu().numpy(), gp_r) <= 1e-3, name


def test_sparse_filter_rotation_invariance_bitwise():
    rs = need_gpu()
    w, x = inputs("small")
    log("sparse_filter rotation invariance")
    rc0, off, wts = upload(w, x, rs=rs)
    i0 = rs.sparse_filter(w.geometry, w.grid, rc0, off, wts, w.sparse.window).cpu()
    x1 = synth.Inputs(**{**x.__dict__, "raw": np.roll(x.raw, 1, axis=0)})
    rc1, _, _ = upload(w, x1, rs=rs)
    i1 = rs.sparse_filter(w.geometry, w.grid, rc1, off, wts, w.sparse.window).cpu()
    assert torch.equal(i1, torch.roll(i0, 1, dims=1))


def test_sparse_filter_rotation_full():
    """Full rotation-size workload (1024 x 3600, K=64 of 256) against the full oracle image."""
    rs = need_gpu()
    w, x = inputs("rotation")
    log("sparse_filter rotation full size")
    rc, off, wts = upload(w, x, rs=rs)
    img = rs.sparse_filter(w.geometry, w.grid, rc, off, wts, w.sparse.window).cpu().numpy()
    ref = oracle.sparse_filter(oracle_band("rotation"), x.l_lo, w.geometry, w.grid, x.offsets, x.weights)
    assert_image(img, ref, TOL)


# ------------------------------------------------------------------ back-projection
@pytest.mark.parametrize("interp", ["nearest", "linear"])
def test_bp_full_small(interp):
    rs = need_gpu()
    w, x = inputs("small")
    log(f"bp_full small {interp}")
    rc, _, _ = upload(w, x, rs=rs)
    img = rs.bp_full(w.geometry, w.grid, rc, interp=interp).cpu().numpy()
    ref = oracle.bp_full(oracle_band("small"), x.l_lo, w.geometry, w.grid, interp=interp)
    assert_image(img, ref, TOL)


def test_bp_full_jittered_angles_small():
    rs = need_gpu()
    w, x = inputs("small")
    ang = synth.nominal_angles(w.geometry) + np.random.default_rng(8).normal(0, 2e-3, w.geometry.n_pulses)
    log("bp_full small jittered")
    rc, _, _ = upload(w, x, rs=rs)
    img = rs.bp_full(w.geometry, w.grid, rc, angles=to_dev(ang)).cpu().numpy()
    ref = oracle.bp_full(oracle_band("small"), x.l_lo, w.geometry, w.grid, pulse_angles=ang)
    assert_image(img, ref, TOL)


def test_bp_full_rotation_sampled():
    """Rotation workload with the true (jittered) angles: sampled pixels vs the oracle."""
    rs = need_gpu()
    w, x = inputs("rotation")
    log("bp_full rotation full size (sampled check)")
    rc, _, _ = upload(w, x, rs=rs)
    img = rs.bp_full(w.geometry, w.grid, rc, angles=to_dev(x.angles)).cpu().numpy()
    rng = np.random.default_rng(99)
    rows = rng.integers(0, w.grid.n_range, 300)
    azs = rng.integers(0, w.grid.n_az, 300)
    # include rows at both ends of the grid and azimuths at the wrap-around
    rows[:4] = [0, 0, w.grid.n_range - 1, w.grid.n_range - 1]
    azs[:4] = [0, w.grid.n_az - 1, 0, w.grid.n_az - 1]
    ref = oracle.bp_full_at(oracle_band("rotation"), x.l_lo, w.geometry, w.grid, rows, azs, pulse_angles=x.angles)
    assert_image(img[rows, azs], ref, TOL)


@pytest.mark.parametrize("interp", ["nearest", "linear"])
def test_bp_full_narrow_band(interp):
    """Bins outside a narrow stored band read zero (the clamped row lies past the band, where the
    buffer range check returns zero), as in the oracle; with jittered angles."""
    rs = need_gpu()
    w, x = inputs("small")
    y = oracle.range_compress(x.raw, x.window, w.geometry.n_fft)
    lo, cnt = 40, 30
    rng = np.random.default_rng(5)
    ang = w.geometry.phi0_rad + 2 * np.pi * np.arange(w.geometry.n_pulses) / w.geometry.n_pulses
    ang = ang + rng.normal(0, np.deg2rad(0.3), ang.size)
    log(f"bp_full narrow band {interp}")
    ref = oracle.bp_full(y[:, lo:lo + cnt], lo, w.geometry, w.grid, pulse_angles=ang, interp=interp)
    rc = rs.range_compress(w.geometry, to_dev(x.raw), to_dev(x.window), lo, cnt, halo=0)
    img = rs.bp_full(w.geometry, w.grid, rc, angles=to_dev(ang), interp=interp).cpu().numpy()
    assert_image(img, ref, TOL)
    assert np.count_nonzero(img) < img.size


def test_bp_full_rows_inside_radius():
    """Rows at or inside the rotation radius see no pulse (R cos D - r <= 0): exactly zero."""
    rs = need_gpu()
    w = custom_workload("inside_radius", 72, 120, 64, 24, 0.07, 1.22, 8, 16)   # no row within 2 cm of r
    x = synth.make_inputs(w)
    yb = oracle.range_compress(x.raw, x.window, 64)[:, x.l_lo:x.l_lo + x.l_count]
    log("bp_full rows inside the radius")
    ref = oracle.bp_full(yb, x.l_lo, w.geometry, w.grid)
    rc = rs.range_compress(w.geometry, to_dev(x.raw), to_dev(x.window), x.l_lo, x.l_count, halo=8)
    img = rs.bp_full(w.geometry, w.grid, rc).cpu().numpy()
    assert_image(img, ref, TOL)
    inside = w.grid.r0_m + np.arange(w.grid.n_range) * w.grid.dr_m <= w.geometry.radius_m
    assert inside.any() and not np.any(img[inside])


def test_bpa_equals_dense_sparse_filter_gpu():
    """GPU BPA equals the GPU sparse filter with every visible pulse and steering weights."""
    rs = need_gpu()
    g = synth.radar(64, 64, 0.3)
    grid = synth.PolarGrid(8, 64, 0.35, 0.2)
    l_lo, l_count = synth.band_for(g, grid)
    yb = synth.random_complex((64, l_count), seed=7).astype(np.complex128)
    n = 64
    vis = []
    for row in range(8):
        rt = grid.r0_m + row * grid.dr_m
        o = np.arange(-n // 2, n // 2)
        vis.append(o[rt * np.cos(2 * np.pi * o / n) - g.radius_m > 0])
    kmax = max(len(v) for v in vis)
    offs = np.zeros((8, kmax), np.int32)
    wts = np.zeros((8, kmax), np.complex128)
    k_w = oracle.wavenumber(g)
    for row, v in enumerate(vis):
        rt = grid.r0_m + row * grid.dr_m
        pad = [o for o in range(-n // 2, n // 2) if o not in set(v.tolist())][:kmax - len(v)]
        offs[row] = np.concatenate([v, pad])
        d = 2 * np.pi * v / n
        rn = np.sqrt(rt ** 2 + g.radius_m ** 2 - 2 * rt * g.radius_m * np.cos(d))
        wts[row, :len(v)] = (rt * np.cos(d) - g.radius_m) / rn * np.exp(2j * k_w * rn)
    log("bpa == dense sparse filter")
    w = synth.Workload("dense", 77, g, grid, synth.SceneSpec(0, "unit", 1, 2), synth.SparseSpec(kmax, n, False))
    rc = rc_from_band(rs, w, yb, l_lo, n // 2)
    a = rs.sparse_filter(g, grid, rc, to_dev(offs), to_dev(wts.astype(np.complex64)), n).cpu().numpy()
    b = rs.bp_full(g, grid, rc).cpu().numpy()
    assert_image(a, b, TOL)
    assert_image(b, oracle.bp_full(yb, l_lo, g, grid), TOL)


# ------------------------------------------------------------------ adjoint
@pytest.mark.parametrize("interp", ["nearest", "linear"])
def test_backward_small(interp):
    rs = need_gpu()
    w, x = inputs("small")
    yb = oracle_band("small")
    n = w.geometry.n_pulses
    rng = np.random.default_rng(23)
    dphi = rng.normal(0, 2e-3, n).astype(np.float32)
    dpsi = rng.normal(0, 0.2, n).astype(np.float32)
    gimg = synth.random_complex((w.grid.n_range, n), seed=31)
    log(f"backward small {interp}")
    gw_r, gd_r, gp_r = oracle.sparse_filter_grad(yb, x.l_lo, w.geometry, w.grid, x.offsets, x.weights,
                                                 gimg.astype(np.complex128), dphi.astype(np.float64),
                                                 dpsi.astype(np.float64), interp)
    rc = rc_from_band(rs, w, yb, x.l_lo, 32)
    gw, gd, gp = rs.sparse_filter_backward(w.geometry, w.grid, rc, to_dev(x.offsets),
                                           to_dev(x.weights.astype(np.complex64)), w.sparse.window, to_dev(gimg),
                                           to_dev(dphi), to_dev(dpsi), interp)
    assert rel_l2(gw.cpu().numpy(), gw_r) <= 1e-3
    assert rel_l2(gd.cpu().numpy(), gd_r) <= 1e-3
    assert rel_l2(gp.cpu().numpy(), gp_r) <= 1e-3
    # deterministic: a second call gives identical bits
    gw2, gd2, gp2 = rs.sparse_filter_backward(w.geometry, w.grid, rc, to_dev(x.offsets),
                                              to_dev(x.weights.astype(np.complex64)), w.sparse.window,
                                              to_dev(gimg), to_dev(dphi), to_dev(dpsi), interp)
    assert torch.equal(gw, gw2) and torch.equal(gd, gd2) and torch.equal(gp, gp2)


@pytest.mark.parametrize("interp", ["nearest", "linear"])
def test_max_taps_forward_corrected_and_adjoint(interp):
    """K = 1024 (the ABI maximum) with W = N: several LDS tap chunks in the corrected forward and
    in the adjoint, a tap table of 1024 entries in the plain filter."""
    rs = need_gpu()
    n = 1024
    w = custom_workload("max_taps", 73, n, 64, 4, 0.6, 1.4, 1024, n)
    x = synth.make_inputs(w)
    yb = oracle.range_compress(x.raw, x.window, 64)[:, x.l_lo:x.l_lo + x.l_count]
    rng = np.random.default_rng(29)
    dphi = rng.normal(0, 2e-3, n).astype(np.float32)
    dpsi = rng.normal(0, 0.2, n).astype(np.float32)
    rc = rs.range_compress(w.geometry, to_dev(x.raw), to_dev(x.window), x.l_lo, x.l_count, halo=n // 2)
    off, wts = to_dev(x.offsets), to_dev(x.weights.astype(np.complex64))
    log(f"max taps plain {interp}")
    ref = oracle.sparse_filter(yb, x.l_lo, w.geometry, w.grid, x.offsets, x.weights, interp=interp)
    img = rs.sparse_filter(w.geometry, w.grid, rc, off, wts, n, interp=interp).cpu().numpy()
    assert_image(img, ref, TOL)
    log(f"max taps corrected {interp}")
    ref = oracle.sparse_filter(yb, x.l_lo, w.geometry, w.grid, x.offsets, x.weights, dphi=dphi.astype(np.float64),
                               dpsi=dpsi.astype(np.float64), interp=interp)
    img = rs.sparse_filter(w.geometry, w.grid, rc, off, wts, n, dphi=to_dev(dphi), dpsi=to_dev(dpsi),
                           interp=interp).cpu().numpy()
    assert_image(img, ref, TOL)
    log(f"max taps adjoint {interp}")
    gimg = synth.random_complex((w.grid.n_range, n), seed=37)
    gw_r, gd_r, gp_r = oracle.sparse_filter_grad(yb, x.l_lo, w.geometry, w.grid, x.offsets, x.weights,
                                                 gimg.astype(np.complex128), dphi.astype(np.float64),
                                                 dpsi.astype(np.float64), interp)
    gw, gd, gp = rs.sparse_filter_backward(w.geometry, w.grid, rc, off, wts, n, to_dev(gimg), to_dev(dphi),
                                           to_dev(dpsi), interp)
    assert rel_l2(gw.cpu().numpy(), gw_r) <= 1e-3
    assert rel_l2(gd.cpu().numpy(), gd_r) <= 1e-3
    assert rel_l2(gp.cpu().numpy(), gp_r) <= 1e-3


def test_calibration_gradient_rotation_subgrid():
    """Calibration workload: loss = entropy + sidelobe energy on a 64 x 360 sub-grid of the
    full-size image, gradients through the autograd Function vs the FP64 oracle gradient."""
    rs = need_gpu()
    w, x = inputs("calib")
    g, grid = w.geometry, w.grid
    n = g.n_pulses
    r_lo, a_lo = 400, 1700
    rows_sub = np.arange(r_lo, r_lo + 64)
    log("calibration gradient (full-size forward/backward)")
    rc, off, wts = upload(w, x, rs=rs)
    wts_p = wts.clone().requires_grad_(True)
    dphi = torch.zeros(n, dtype=torch.float32, device=dev(), requires_grad=True)
    dpsi = torch.zeros(n, dtype=torch.float32, device=dev(), requires_grad=True)
    img = rs.sparse_filter_diff(g, grid, rc, off, wts_p, w.sparse.window, dphi, dpsi, "linear")
    sub = img[r_lo:r_lo + 64, a_lo:a_lo + 360].to(torch.complex128)
    # scatterers inside the sub-grid define the mainlobe boxes
    srow, saz = oracle.metrics.scatterer_pixels(grid, g, x.scene.r_m, x.scene.phi_rad)
    sel = (srow >= r_lo) & (srow < r_lo + 64) & (saz >= a_lo) & (saz < a_lo + 360)
    mask = oracle.metrics.box_mask((64, 360), srow[sel] - r_lo, saz[sel] - a_lo)
    p = sub.abs() ** 2
    e = p.sum()
    d = p / e
    ent = -(torch.where(d > 0, d * torch.log(torch.where(d > 0, d, torch.ones_like(d))), torch.zeros_like(d))).sum()
    loss = ent + p[~torch.from_numpy(mask).to(dev())].sum() / e
    loss.backward()
    # FP64 oracle on the same 64 rows
    yb = oracle_band("calib")
    sub_grid = synth.PolarGrid(64, n, grid.r0_m + r_lo * grid.dr_m, grid.dr_m)
    offs_s, wts_s = x.offsets[rows_sub], x.weights[rows_sub]
    img_o = oracle.sparse_filter(yb, x.l_lo, g, sub_grid, offs_s, wts_s, np.zeros(n), np.zeros(n), "linear")
    gfull = np.zeros_like(img_o)
    _, gsub = oracle.metrics.calib_loss(img_o[:, a_lo:a_lo + 360], mask)
    gfull[:, a_lo:a_lo + 360] = gsub
    gw_r, gd_r, _ = oracle.sparse_filter_grad(yb, x.l_lo, g, sub_grid, offs_s, wts_s, gfull, np.zeros(n),
                                              np.zeros(n), "linear")
    assert rel_l2(wts_p.grad[r_lo:r_lo + 64].cpu().numpy(), gw_r) <= 1e-3
    assert rel_l2(dphi.grad.cpu().numpy(), gd_r) <= 1e-3
    others = torch.cat([wts_p.grad[:r_lo], wts_p.grad[r_lo + 64:]])
    assert float(others.abs().max()) == 0.0


# ------------------------------------------------------------------ reduced precision
@pytest.mark.parametrize("dtype", ["f16", "bf16"])
def test_reduced_precision_small(dtype):
    rs = need_gpu()
    w, x = inputs("small")
    log(f"reduced precision small {dtype}")
    scale = 2.0 ** -4 if dtype == "f16" else 1.0
    rc, off, wts = upload(w, x, dtype=dtype, scale=scale, rs=rs)
    ref = oracle.sparse_filter(oracle_band("small"), x.l_lo, w.geometry, w.grid, x.offsets, x.weights)
    for tile in (None, (1, 4, 4), (2, 8, 2)):
        for wt in (wts, rs.weights_f16(wts)):
            img = rs.sparse_filter(w.geometry, w.grid, rc, off, wt, w.sparse.window, tile=tile).cpu().numpy()
            assert rel_l2(img, ref) <= 1e-2, (tile, wt.dtype)
    bpa = rs.bp_full(w.geometry, w.grid, rc).cpu().numpy()
    assert rel_l2(bpa, oracle.bp_full(oracle_band("small"), x.l_lo, w.geometry, w.grid)) <= 1e-2
