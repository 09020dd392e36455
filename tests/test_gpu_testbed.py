"""GPU tests on the paper's own instance: the radar of Sec. IV-B (Table II: a chirp from 60 GHz
with K = 6.8e13 Hz/s sampled at 4.5 MHz from T_Start = 7 us, M = L = 225, r = 0.145 m, N = 800)
and the testbed's image area of Sec. IV-F (a 9.8756 m square on a 0.04 m lattice, 247 x 247
targets).  Each image is compared with the FP64 oracle over the whole lattice: the mixed-radix
range FFT, Algorithm 2 with K = 157 taps per weight row (both interpolations, and FP16 storage),
and back-projection with the true, jittered pulse angles.  A point target at the paper's
simulated position (pi/2, 2 m) peaks at its own cell in both images."""
import dataclasses

import numpy as np
import pytest

import oracle
import synth
from gpu_common import assert_image, dev, inputs, log, need_gpu, oracle_band, rel_l2, to_dev, torch

pytestmark = pytest.mark.gpu


def _rc(rs, w, x, **kw):
    return rs.range_compress(w.geometry, to_dev(x.raw), to_dev(x.window), x.l_lo, x.l_count,
                             halo=w.sparse.window // 2, **kw)


def test_testbed_range_compress():
    rs = need_gpu()
    w, x = inputs("testbed")
    log("testbed range compression (L = 225)")
    rc = _rc(rs, w, x)
    torch.cuda.synchronize()
    got = rc.pulses(w.geometry.n_pulses).cpu().numpy().T                # [N, l_count]
    assert rel_l2(got, oracle_band("testbed")) <= 1e-5


@pytest.mark.parametrize("interp", ["nearest", "linear"])
def test_testbed_sparse_filter_lattice(interp):
    rs = need_gpu()
    w, x = inputs("testbed")
    lat = synth.paper_lattice()
    xs, ys = lat.positions()
    log(f"testbed Algorithm 2 on the 247 x 247 lattice, {interp}")
    img = rs.sparse_filter_cartesian(w.geometry, w.grid, lat, _rc(rs, w, x), to_dev(x.offsets),
                                     to_dev(x.weights.astype(np.complex64)), w.sparse.window,
                                     interp=interp).cpu().numpy()
    ref = oracle.sparse_filter_cartesian(oracle_band("testbed"), x.l_lo, w.geometry, w.grid, xs, ys, x.offsets,
                                         x.weights, interp).reshape(lat.ny, lat.nx)
    assert_image(img, ref, 1e-4, f"testbed sparse {interp}")


def test_testbed_sparse_filter_lattice_f16():
    rs = need_gpu()
    w, x = inputs("testbed")
    lat = synth.paper_lattice()
    xs, ys = lat.positions()
    log("testbed Algorithm 2, FP16 band")
    img = rs.sparse_filter_cartesian(w.geometry, w.grid, lat, _rc(rs, w, x, dtype="f16", scale=2.0 ** -4),
                                     to_dev(x.offsets), to_dev(x.weights.astype(np.complex64)),
                                     w.sparse.window).cpu().numpy()
    ref = oracle.sparse_filter_cartesian(oracle_band("testbed"), x.l_lo, w.geometry, w.grid, xs, ys, x.offsets,
                                         x.weights).reshape(lat.ny, lat.nx)
    assert rel_l2(img, ref) <= 1e-2


def test_testbed_bp_lattice_true_angles():
    rs = need_gpu()
    w, x = inputs("testbed")
    lat = synth.paper_lattice()
    xs, ys = lat.positions()
    log("testbed back-projection on the 247 x 247 lattice, true angles")
    img = rs.bp_cartesian(w.geometry, lat, _rc(rs, w, x), angles=to_dev(x.angles)).cpu().numpy()
    ref = oracle.bp_cartesian_at(oracle_band("testbed"), x.l_lo, w.geometry, xs, ys,
                                 pulse_angles=x.angles).reshape(lat.ny, lat.nx)
    assert_image(img, ref, 1e-4, "testbed BPA")


def test_testbed_point_target_peaks_at_its_cell():
    """One unit scatterer at (pi/2, 2 m), no noise or jitter: |image| peaks at the lattice cell
    nearest (0, 2) for Algorithm 2 with phase-matched weights and for back-projection."""
    rs = need_gpu()
    w = synth.testbed()
    w = dataclasses.replace(w, name="testbed_point", cfg_id=61,
                            scene=dataclasses.replace(w.scene, n_scatterers=1, noise_power=0.0, jitter_sigma_rad=0.0))
    x = synth.make_inputs(w, with_raw=False)
    scene = synth.Scene(np.array([2.0]), np.array([np.pi / 2]), np.array([1.0 + 0j]))
    raw = synth.simulate_raw(w.geometry, scene, x.angles)
    x = dataclasses.replace(x, raw=raw, scene=scene)
    lat = synth.paper_lattice()
    rc = _rc(rs, w, x)
    want = (int(round((2.0 - lat.y0_m) / lat.dy_m)), int(round((0.0 - lat.x0_m) / lat.dx_m)))
    log("testbed point target")
    sas = rs.sparse_filter_cartesian(w.geometry, w.grid, lat, rc, to_dev(x.offsets),
                                     to_dev(x.weights.astype(np.complex64)), w.sparse.window).abs().cpu().numpy()
    bpa = rs.bp_cartesian(w.geometry, lat, rc).abs().cpu().numpy()
    for name, im in (("sas", sas), ("bpa", bpa)):
        got = np.unravel_index(np.argmax(im), im.shape)
        log(f"  {name}: peak {im.max():.3f} at {got}, want {want}")
        assert got == want, (name, got, want)
