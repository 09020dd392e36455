"""GPU tests of the robust sparse-array synthesis (Algorithm 1, FPP-SCA with eq. 36) against the
FP64 oracle, through the C ABI: the per-iteration objective, U' and slacks, and the designed
weights; and the design checked by the GPU beampattern's worst-case summary (C1/C2 of eqs.
31-32 with Delta_R)."""
import dataclasses
import math

import numpy as np
import pytest

import synth
from gpu_common import dev, log, need_gpu, torch
from oracle import fppsca as F

pytestmark = pytest.mark.gpu


def paper_radar(n_pulses):
    g = synth.radar(n_pulses, 225, 0.145)
    return dataclasses.replace(g, fc_hz=60e9, t_start_s=7e-6, slope_hz_s=6.8e13, fs_hz=4.5e6)


def small_case(iters):
    g = paper_radar(160)
    grid = synth.PolarGrid(3, 160, 1.2, 0.3)          # R = 1.2, 1.5, 1.8 m
    p = F.SasParams(iters=iters, d_angle=math.radians(2.0), phi_mw=math.radians(4.0), eta=0.01, u_min=2.0,
                    lam_b=200.0)
    return g, grid, p


def gpu_params(rs, p):
    return rs.sas_params(iters=p.iters, max_newton=p.max_newton, th=p.th, phi_mw=p.phi_mw, d_angle=p.d_angle,
                         lam_b=p.lam_b, eta=p.eta, u_min=p.u_min, b_min=p.b_min, eps=p.eps, mu=p.mu, tau0=p.tau0,
                         newton_tol=p.newton_tol, ls_alpha=p.ls_alpha, ls_beta=p.ls_beta, ls_min=p.ls_min)


def test_sas_design_matches_oracle_per_iteration():
    rs = need_gpu()
    g, grid, p = small_case(6)
    deltas = np.array([0.03, 0.02, 0.015])
    log("sas design: 3 rows x 6 iterations")
    d = rs.sas_design(g, grid, torch.from_numpy(deltas).to(dev()), gpu_params(rs, p))
    torch.cuda.synchronize()
    hist = d.history.cpu().numpy()
    offs, wts, cnt = d.offsets.cpu().numpy(), d.weights.cpu().numpy(), d.count.cpu().numpy()
    for row in range(grid.n_range):
        rr = grid.r0_m + row * grid.dr_m
        ref = F.design_bin(g, rr, deltas[row], p)
        for it, h in enumerate(ref.history):
            got = hist[row, it]
            log(f"  row {row} it {it}: J {got[0]:.9f} / {h['J']:.9f}, U' {got[1]:.9f} / {h['U']:.9f}, "
                f"newton {int(got[5])} / {h['newton']}")
            assert abs(got[0] - h["J"]) <= 1e-5 * abs(h["J"]), (row, it, got[0], h["J"])
            assert abs(got[1] - h["U"]) <= 1e-5 * abs(h["U"]), (row, it, got[1], h["U"])
            for j, key in ((2, "b"), (3, "b1"), (4, "b2")):
                assert abs(got[j] - h[key]) <= 1e-6 + 1e-4 * abs(h[key]), (row, it, key, got[j], h[key])
        # designed taps: the oracle's nonzero candidates, in order, as complex64
        keep = np.abs(ref.w) > 0
        assert cnt[row] == np.count_nonzero(keep), (row, cnt[row], np.count_nonzero(keep))
        np.testing.assert_array_equal(offs[row, :cnt[row]], ref.offsets[keep])
        np.testing.assert_allclose(wts[row, :cnt[row]], ref.w[keep], atol=2e-5)
        assert np.all(wts[row, cnt[row]:] == 0)


def test_sas_design_meets_worst_case_with_gpu_beampattern():
    """32 iterations: the C1 and C2 slacks vanish, and the GPU beampattern's worst-case ratio
    (side + Delta_R)^2 / (main - Delta_R)^2 of each row's design is at most eta, as eqs. 31-32
    require of the sub-problem's solution (the kernel runs with Th = 0 and returns every
    candidate's weight).  The thresholding of Sec. III-C (|w_k| < Th set to zero) then moves
    each pattern value by at most eps = sum of the removed |w_k| (|a_k| <= 1), so the sparse
    set's ratio stays within ((side + Delta_R + eps) / (main - Delta_R - eps))^2."""
    rs = need_gpu()
    g, grid, p = small_case(32)
    p_all = dataclasses.replace(p, th=0.0)
    deltas = torch.tensor([0.03, 0.02, 0.015], dtype=torch.float64, device=dev())
    log("sas design: 3 rows x 32 iterations, then the beampattern check")
    d = rs.sas_design(g, grid, deltas, gpu_params(rs, p_all))
    torch.cuda.synchronize()
    hist = d.history.cpu().numpy()
    assert np.all(hist[:, -1, 3] < 1e-8) and np.all(hist[:, -1, 4] < 1e-8), hist[:, -1]
    cnt = d.count.cpu().numpy()
    for row in range(grid.n_range):
        rr = grid.r0_m + row * grid.dr_m
        assert cnt[row] == len(F.candidates(g, rr))            # Th = 0 keeps every candidate
        sub = synth.PolarGrid(1, g.n_pulses, rr, 0.1)
        ph = F.sidelobe_angles(F.candidates(g, rr), g.n_pulses, p.phi_mw, p.d_angle)
        a = torch.from_numpy(np.concatenate([[0.0], ph])).to(dev())
        dr = deltas[row:row + 1].contiguous()
        off = d.offsets[row:row + 1, :cnt[row]].contiguous()
        w = d.weights[row:row + 1, :cnt[row]].contiguous()
        _, summ = rs.beampattern(g, sub, off, w, g.n_pulses, a, delta_r=dr)
        main, side, ratio = summ.cpu().numpy()[0]
        u2 = hist[row, -1, 1] ** 2
        log(f"  row {row}: main {main:.5f} side {side:.5f} ratio {ratio:.4e} eta {p.eta}")
        assert ratio <= p.eta * (1 + 1e-3), (row, ratio)
        assert (main - deltas[row].item()) ** 2 >= u2 * (1 - 1e-3)
        # the paper's thresholding
        keep = (w.abs() >= p.th)[0]
        eps = float(w[0, ~keep].abs().sum())
        _, summ_t = rs.beampattern(g, sub, off[:, keep].contiguous(), w[:, keep].contiguous(), g.n_pulses, a,
                                   delta_r=dr)
        ratio_t = summ_t.cpu().numpy()[0][2]
        dl = deltas[row].item()
        bound = ((side + dl + eps) / (main - dl - eps)) ** 2
        log(f"    thresholded at {p.th}: {int(keep.sum())} of {cnt[row]} kept, ratio {ratio_t:.4e} <= {bound:.4e}")
        assert 0 < keep.sum() < cnt[row]
        assert ratio_t <= bound * (1 + 1e-9), (row, ratio_t, bound)


def test_sas_design_rows_without_candidates_and_ragged_rows():
    """A grid whose first row lies inside the radius (no phase centre sees it, eqs. 4-5) next to
    rows with different candidate counts: the first row gets count 0, zero taps and a zero
    history; the others match the oracle per iteration."""
    rs = need_gpu()
    g, _, p = small_case(2)
    grid = synth.PolarGrid(3, 160, 0.1, 0.85)          # R = 0.1 (< r = 0.145), 0.95, 1.8 m
    deltas = np.array([0.05, 0.03, 0.015])
    log("sas design: a row inside the radius and two ragged rows, 2 iterations")
    d = rs.sas_design(g, grid, torch.from_numpy(deltas).to(dev()), gpu_params(rs, p))
    torch.cuda.synchronize()
    hist, cnt = d.history.cpu().numpy(), d.count.cpu().numpy()
    assert cnt[0] == 0 and np.all(hist[0] == 0)
    assert np.all(d.weights[0].cpu().numpy() == 0) and np.all(d.offsets[0].cpu().numpy() == 0)
    for row in (1, 2):
        rr = grid.r0_m + row * grid.dr_m
        ref = F.design_bin(g, rr, deltas[row], p)
        for it, h in enumerate(ref.history):
            assert abs(hist[row, it, 0] - h["J"]) <= 1e-5 * abs(h["J"]), (row, it)
            assert abs(hist[row, it, 1] - h["U"]) <= 1e-5 * abs(h["U"]), (row, it)
        assert cnt[row] == np.count_nonzero(np.abs(ref.w) > 0)
