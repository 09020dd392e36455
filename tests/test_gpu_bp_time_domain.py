"""GPU tests of the raw-sample (time-domain) forms: the conventional BPA and the sparse-aperture
filter with the exact beat frequency, against the FP64 oracle: relative L2 <= 1e-4 (complex64
data, float32 accumulation)."""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import custom_workload, inputs, log, need_gpu, rel_l2, to_dev, torch

pytestmark = pytest.mark.gpu

TOL = 1e-4


def test_time_domain_bpa_tiny_full():
    rs = need_gpu()
    w = custom_workload("td_tiny", 90, 64, 64, 3, 0.5, 1.2, 8, 16)
    x = synth.make_inputs(w)
    log("time-domain BPA tiny")
    img = rs.bp_time_domain(w.geometry, w.grid, to_dev(x.raw), to_dev(x.window)).cpu().numpy()
    rows = np.repeat(np.arange(w.grid.n_range), w.grid.n_az)
    azs = np.tile(np.arange(w.grid.n_az), w.grid.n_range)
    ref = oracle.bp_time_domain_at(x.raw, x.window, w.geometry, w.grid, rows, azs).reshape(img.shape)
    assert rel_l2(img, ref) <= TOL


@pytest.mark.parametrize("jitter", [False, True])
def test_time_domain_bpa_small_sampled(jitter):
    rs = need_gpu()
    w, x = inputs("small")
    angles = x.angles if jitter else None
    log(f"time-domain BPA small jitter={jitter}")
    img = rs.bp_time_domain(w.geometry, w.grid, to_dev(x.raw), to_dev(x.window),
                            angles=None if angles is None else to_dev(angles)).cpu().numpy()
    rng = np.random.default_rng(5)
    rows = rng.integers(0, w.grid.n_range, 200)
    azs = rng.integers(0, w.grid.n_az, 200)
    ref = oracle.bp_time_domain_at(x.raw, x.window, w.geometry, w.grid, rows, azs, pulse_angles=angles)
    assert rel_l2(img[rows, azs], ref) <= TOL


def test_time_domain_bpa_rotation_rows():
    """Eight rows of the rotation workload (M = 512, ~1700 visible pulses per pixel), true angles,
    on sampled pixels; the row range argument offsets the output rows."""
    rs = need_gpu()
    w, x = inputs("rotation")
    first, count = 500, 8
    log("time-domain BPA rotation rows")
    img = rs.bp_time_domain(w.geometry, w.grid, to_dev(x.raw), to_dev(x.window), angles=to_dev(x.angles),
                            rows=(first, count)).cpu().numpy()
    assert img.shape == (count, w.grid.n_az)
    rng = np.random.default_rng(6)
    rl = rng.integers(0, count, 30)
    azs = rng.integers(0, w.grid.n_az, 30)
    ref = oracle.bp_time_domain_at(x.raw, x.window, w.geometry, w.grid, rl + first, azs, pulse_angles=x.angles)
    assert rel_l2(img[rl, azs], ref) <= TOL


@pytest.mark.parametrize("name", ["small", "edge"])
def test_time_domain_sas(name):
    rs = need_gpu()
    if name == "small":
        w, x = inputs("small")
    else:
        w = custom_workload("td_sas_edge", 91, 100, 128, 5, 0.6, 2.5, 5, 16)   # ragged N, K = 5
        x = synth.make_inputs(w)
    log(f"time-domain SAS {name}")
    img = rs.sas_time_domain(w.geometry, w.grid, to_dev(x.raw), to_dev(x.offsets),
                             to_dev(x.weights.astype(np.complex64)), w.sparse.window, window=to_dev(x.window)).cpu().numpy()
    rng = np.random.default_rng(8)
    rows = rng.integers(0, w.grid.n_range, 200)
    azs = rng.integers(0, w.grid.n_az, 200)
    ref = oracle.sas_time_domain_at(x.raw, x.window, w.geometry, w.grid, x.offsets, x.weights, rows, azs)
    assert rel_l2(img[rows, azs], ref) <= TOL


def test_time_domain_sas_rotation_rows():
    rs = need_gpu()
    w, x = inputs("rotation")
    first, count = 300, 4
    log("time-domain SAS rotation rows")
    img = rs.sas_time_domain(w.geometry, w.grid, to_dev(x.raw), to_dev(x.offsets),
                             to_dev(x.weights.astype(np.complex64)), w.sparse.window, window=to_dev(x.window),
                             rows=(first, count)).cpu().numpy()
    rng = np.random.default_rng(9)
    rl = rng.integers(0, count, 60)
    azs = rng.integers(0, w.grid.n_az, 60)
    ref = oracle.sas_time_domain_at(x.raw, x.window, w.geometry, w.grid, x.offsets, x.weights, rl + first, azs)
    assert rel_l2(img[rl, azs], ref) <= TOL
