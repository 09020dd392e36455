"""GPU tests of the sparse weights' beampattern and the worst-case robust check against the FP64
oracle (both float64: per element within 1e-9 of the row's largest value; the summary exactly
from the device's own pattern)."""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import inputs, log, need_gpu, to_dev, torch

pytestmark = pytest.mark.gpu

TOL = 1e-9


def _angles(n_side, span):
    return np.concatenate([[0.0], np.linspace(-span, span, n_side)])


def _check_rows(g, grid, offsets, w64, window, ang, pat, rows):
    for r in rows:
        sub = synth.PolarGrid(1, grid.n_az, grid.r0_m + r * grid.dr_m, grid.dr_m)
        ref = oracle.beampattern(g, sub, offsets[r:r + 1], w64[r:r + 1], window, ang)[0]
        err = np.max(np.abs(pat[r] - ref)) / np.max(ref)
        assert err <= TOL, (r, err)


def test_beampattern_small():
    """128 rows, K = 32 of 64, 701 angles (three ragged workgroups), all rows."""
    rs = need_gpu()
    w, x = inputs("small")
    ang = _angles(700, 0.5)
    w64 = x.weights.astype(np.complex64).astype(np.complex128)   # the device's weights
    log("beampattern small")
    pat, summ = rs.beampattern(w.geometry, w.grid, to_dev(x.offsets), to_dev(x.weights.astype(np.complex64)),
                               w.sparse.window, to_dev(ang))
    pat, summ = pat.cpu().numpy(), summ.cpu().numpy()
    ref = oracle.beampattern(w.geometry, w.grid, x.offsets, w64, w.sparse.window, ang)
    err = np.max(np.abs(pat - ref) / np.max(ref, axis=1, keepdims=True))
    assert err <= TOL, err
    np.testing.assert_array_equal(summ[:, 0], pat[:, 0])
    np.testing.assert_array_equal(summ[:, 1], pat[:, 1:].max(axis=1))
    np.testing.assert_allclose(summ[:, 2], oracle.robust_summary(pat[:, 0], pat[:, 1:].max(axis=1),
                                                                 np.zeros(w.grid.n_range)), rtol=1e-14)


def test_beampattern_rotation_with_delta_r():
    """Rotation workload (1024 rows, K = 64 of 256), 2049 angles over the window's span, the
    summary fed by the device's Delta_R; sampled rows against the oracle."""
    rs = need_gpu()
    w, x = inputs("rotation")
    g, grid = w.geometry, w.grid
    ang = _angles(2048, 128 * 2 * np.pi / g.n_pulses)
    draws = to_dev(synth.jitter_draws(41, w.sparse.window, 512, w.scene.jitter_sigma_rad))
    log("beampattern rotation + delta_r")
    dr, _ = rs.delta_r(g, grid, w.sparse.window, draws)
    pat, summ = rs.beampattern(g, grid, to_dev(x.offsets), to_dev(x.weights.astype(np.complex64)), w.sparse.window,
                               to_dev(ang), delta_r=dr)
    pat, summ, dr = pat.cpu().numpy(), summ.cpu().numpy(), dr.cpu().numpy()
    w64 = x.weights.astype(np.complex64).astype(np.complex128)
    _check_rows(g, grid, x.offsets, w64, w.sparse.window, ang, pat, [0, 3, 500, 1023])
    want = oracle.robust_summary(pat[:, 0], pat[:, 1:].max(axis=1), dr)
    fin = np.isfinite(want)
    np.testing.assert_array_equal(np.isfinite(summ[:, 2]), fin)
    np.testing.assert_allclose(summ[fin, 2], want[fin], rtol=1e-14)


def test_beampattern_single_angle_and_window_rule():
    """One angle: no side lobes (max 0).  Offsets outside the window contribute nothing."""
    rs = need_gpu()
    w, x = inputs("small")
    off = x.offsets.copy()
    off[:, 0] = w.sparse.window          # outside [-W/2, W/2)
    wz = x.weights.astype(np.complex64).copy()
    log("beampattern window rule")
    a, sa = rs.beampattern(w.geometry, w.grid, to_dev(off), to_dev(x.weights.astype(np.complex64)), w.sparse.window,
                           to_dev(np.array([0.0, 0.01, -0.02])))
    wz[:, 0] = 0
    b, _ = rs.beampattern(w.geometry, w.grid, to_dev(x.offsets), to_dev(wz), w.sparse.window,
                          to_dev(np.array([0.0, 0.01, -0.02])))
    assert torch.equal(a, b)
    p1, s1 = rs.beampattern(w.geometry, w.grid, to_dev(x.offsets), to_dev(x.weights.astype(np.complex64)),
                            w.sparse.window, to_dev(np.array([0.0])))
    assert float(s1[:, 1].abs().max()) == 0.0
    assert torch.equal(s1[:, 0], p1[:, 0])
