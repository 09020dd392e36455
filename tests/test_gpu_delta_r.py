"""GPU tests of the Delta_R Monte-Carlo (eq. 37): the per-draw error norms against the FP64
oracle (both sides float64, relative 1e-9 per sample), and the selected order statistic bit-exact
against a sort of the device's own samples."""
import dataclasses

import numpy as np
import pytest

import oracle
import synth
from gpu_common import log, need_gpu, to_dev, torch

pytestmark = pytest.mark.gpu

TOL = 1e-9


def _check(rs, g, grid, window, n_s, sigma, seed, q=0.99, rows=None):
    d = synth.jitter_draws(seed, window, n_s, sigma)
    log(f"delta_r N={g.n_pulses} W={window} S={n_s} rows={grid.n_range} sigma={sigma}")
    dr, smp = rs.delta_r(g, grid, window, to_dev(d), quantile=q)
    dr, smp = dr.cpu().numpy(), smp.cpu().numpy()
    k = int(np.ceil(q * n_s)) - 1
    np.testing.assert_array_equal(dr, np.sort(smp, axis=1)[:, k])   # selection: exact
    rows = np.arange(grid.n_range) if rows is None else np.asarray(rows)
    sub = dataclasses.replace(grid, n_range=1)
    for r in rows:
        sub = dataclasses.replace(grid, n_range=1, r0_m=grid.r0_m + r * grid.dr_m)
        ref = oracle.delta_r_samples(g, sub, window, d.T)[0]
        err = np.max(np.abs(smp[r] - ref) / np.maximum(ref, 1e-300))
        assert err <= TOL, (r, err)
        assert abs(dr[r] - oracle.delta_r(ref[None, :], q)[0]) <= TOL * dr[r]
    return dr, smp


def test_delta_r_ragged_tiles():
    """Window over two LDS chunks (320), draws over three workgroups (700), rows over two row
    groups (13): every tail is ragged."""
    rs = need_gpu()
    g = synth.radar(800, 64, 0.145)
    grid = synth.PolarGrid(13, 800, 0.3, 0.25)
    _check(rs, g, grid, 320, 700, np.deg2rad(0.086), 21)


def test_delta_r_rotation_workload():
    """1024 rows x 256-element window x 4096 draws, sigma 0.05 deg: sampled rows against the
    oracle, every row's order statistic against the device samples."""
    rs = need_gpu()
    w = synth.rotation()
    _check(rs, w.geometry, w.grid, w.sparse.window, 4096, np.deg2rad(0.05), 22, rows=[0, 1, 511, 777, 1023])


def test_delta_r_zero_jitter_and_quantiles():
    """No jitter gives a^ = a; q = 1 selects the maximum; one draw is its own quantile."""
    rs = need_gpu()
    g = synth.radar(360, 64, 0.25)
    grid = synth.PolarGrid(9, 360, 0.6, 0.3)
    d = torch.zeros((64, 300), dtype=torch.float64, device="cuda")
    dr, smp = rs.delta_r(g, grid, 64, d)
    assert float(smp.abs().max()) <= 1e-12
    dr, smp = _check(rs, g, grid, 64, 300, 1e-3, 23, q=1.0)
    np.testing.assert_array_equal(dr, smp.max(axis=1))
    dr1, smp1 = _check(rs, g, grid, 64, 1, 1e-3, 24, q=0.5)
    np.testing.assert_array_equal(dr1, smp1[:, 0])


def test_delta_r_grows_with_sigma():
    """Same draws scaled: the error norm of every draw grows with sigma in the small-error regime."""
    rs = need_gpu()
    g = synth.radar(360, 64, 0.25)
    grid = synth.PolarGrid(4, 360, 1.0, 1.0)
    d = to_dev(synth.jitter_draws(25, 32, 512, 1.0))
    lo = rs.delta_r(g, grid, 32, d * 1e-5)[1]
    hi = rs.delta_r(g, grid, 32, d * 2e-5)[1]
    assert bool((hi > lo).all())
    ratio = (hi / lo).cpu().numpy()
    np.testing.assert_allclose(ratio, 2.0, rtol=1e-3)   # linear in sigma to first order


def test_delta_r_graph_replays():
    """Captured in a HIP graph (no memset nodes), every replay equals the eager result bit for
    bit, with eager work and synchronisations between replays; the samples buffer is reused."""
    rs = need_gpu()
    g = synth.radar(800, 64, 0.145)
    grid = synth.PolarGrid(21, 800, 0.3, 0.2)
    d = to_dev(synth.jitter_draws(26, 128, 1000, np.deg2rad(0.086)))
    out = torch.empty(21, dtype=torch.float64, device="cuda")
    smp = torch.empty((21, 1000), dtype=torch.float64, device="cuda")
    log("delta_r graph replays")
    rs.delta_r(g, grid, 128, d, samples=smp, out=out)
    torch.cuda.synchronize()
    ref_out, ref_smp = out.clone(), smp.clone()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(graph, stream=s):
            rs.delta_r(g, grid, 128, d, samples=smp, out=out)
    torch.cuda.current_stream().wait_stream(s)
    for i in range(4):
        out.fill_(-1.0)
        smp.fill_(-1.0)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, ref_out) and torch.equal(smp, ref_smp), i
