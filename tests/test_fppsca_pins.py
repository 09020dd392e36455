"""Pins of the FP64 oracle of the robust sparse-array synthesis (Algorithm 1, eq. 36), CPU only.

Each check is independent of the oracle's own barrier code:
  * the convex sub-problem's optimum against scipy's SLSQP on a tiny instance, with the
    constraints retyped here from eqs. 33-35 in their original (not linearised) places;
  * the first-order bounds of eqs. 33-35 are upper bounds of the concave terms, tight at the
    linearisation point;
  * FPP-SCA's objective never increases (the previous iterate is feasible for the next
    sub-problem);
  * the design meets the worst-case main-lobe and side-lobe constraints of eqs. 31-32 once its
    slacks vanish, as measured by the (separately pinned) beampattern oracle.

Parity unpinned: Table IV's nonzero counts (141 non-robust, 157 robust) and U' (8.21, 8.38)
for the paper's radar at R = 2 m need the paper's exact side-lobe grid and solver tolerances;
they are approximate targets only.
"""
import dataclasses
import math

import numpy as np
import pytest
from scipy.optimize import minimize

import oracle
import synth
from oracle import fppsca as F


def paper_radar(n_pulses=800):
    """The paper's radar (Table II): r = 0.145 m, 60-64 GHz chirp K = 6.8e13 Hz/s sampled at
    4.5 MHz from T_Start = 7 us, M = L = 225, with N pulses per rotation."""
    g = synth.radar(n_pulses, 225, 0.145)
    return dataclasses.replace(g, fc_hz=60e9, t_start_s=7e-6, slope_hz_s=6.8e13, fs_hz=4.5e6)


def tiny_subproblem(seed=0, n=4, s=5, delta=0.05):
    rng = np.random.default_rng(seed)
    a_m = rng.normal(size=n) + 1j * rng.normal(size=n)
    a_s = 0.3 * (rng.normal(size=(s, n)) + 1j * rng.normal(size=(s, n)))
    w_i = rng.normal(size=n) + 1j * rng.normal(size=n)
    w_i /= np.linalg.norm(w_i)
    u_i = abs(np.vdot(w_i, a_m)) * 0.8
    return F.SubProblem(a_m, a_s, w_i, u_i, delta, 0.05, math.sqrt(0.5), 5.0)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_subproblem_optimum_matches_slsqp(seed):
    """eq. 36 solved by the oracle's barrier method: feasible for the paper's inequalities as
    retyped here (epigraph t_k >= |w_k| in squared form), and at least as good as what SLSQP
    finds from six starts (equal, with the same w, where SLSQP reaches the optimum)."""
    sp = tiny_subproblem(seed)
    p = F.SasParams(eps=1e-9, newton_tol=1e-12)
    x, info = F.solve_subproblem(sp, p)
    n = sp.n
    a_m, a_s, w_i, u_i, d = sp.a_m, sp.a_s, sp.w_i, sp.u_i, sp.delta
    eta, lam = sp.eta, sp.lam_b

    def wv(v):
        return v[:n] + 1j * v[n:2 * n]

    def cons(v):
        w, t, u, b, b1, b2 = wv(v), v[2 * n:3 * n], v[3 * n], v[3 * n + 1], v[3 * n + 2], v[3 * n + 3]
        lin_c1 = abs(np.vdot(a_m, w_i)) ** 2 + 2 * np.real(np.conj(np.vdot(a_m, w_i)) * np.vdot(a_m, w - w_i))
        lin_c2 = (math.sqrt(eta) * u_i - d) ** 2 + 2 * (eta * u_i - math.sqrt(eta) * d) * (u - u_i)
        lin_c4 = np.vdot(w_i, w_i).real + 2 * np.real(np.vdot(w_i, w - w_i))
        out = [lin_c1 + b1 - (u + d) ** 2,                                  # C1 (eq. 33)
               1 + b - np.vdot(w, w).real,                                     # C3
               lin_c4 - 1 + b,                                              # C4 (eq. 35)
               u - sp.u_min, b, b1, b2]
        out += [lin_c2 + b2 - abs(np.vdot(a, w)) ** 2 for a in a_s]         # C2 (eq. 34)
        out += list(t * t - np.abs(w) ** 2) + list(t)
        return np.array(out)

    f = lambda v: np.sum(v[2 * n:3 * n]) + lam * np.sum(v[3 * n + 1:3 * n + 4])
    best = None
    rng = np.random.default_rng(100 + seed)
    for trial in range(6):
        v0 = x + 0.05 * rng.normal(size=x.shape) if trial else x.copy()
        v0[2 * n:3 * n] = np.abs(wv(v0)) + 0.1
        r = minimize(f, v0, method="SLSQP", constraints=[{"type": "ineq", "fun": cons}],
                     options={"ftol": 1e-13, "maxiter": 2000})
        if r.success and np.all(cons(r.x) > -1e-8) and (best is None or r.fun < best.fun):
            best = r
    assert best is not None
    # the oracle's point satisfies every inequality as written here, and no SLSQP run (from
    # the oracle's point or perturbations of it) finds a feasible point with a lower objective;
    # SLSQP itself can stall above the optimum where the cones |w_k| <= t_k meet at w_k = 0
    assert np.all(cons(x) > -1e-9), cons(x).min()
    got = F.objective(sp, x)
    assert got <= best.fun + 1e-7 * max(1.0, abs(best.fun)), (got, best.fun)
    if abs(got - best.fun) <= 1e-6 * max(1.0, abs(best.fun)):
        np.testing.assert_allclose(wv(x), wv(best.x), atol=2e-4)


def test_linearisations_are_upper_bounds():
    """eqs. 33-35: each first-order bound of a concave term lies above it, and touches it at
    the linearisation point."""
    sp = tiny_subproblem(3, n=6, s=4)
    g, c1, alpha, beta, c4 = sp.lin()
    rng = np.random.default_rng(7)
    for _ in range(50):
        w = rng.normal(size=6) + 1j * rng.normal(size=6)
        u = rng.uniform(0, 10)
        assert -abs(np.vdot(sp.a_m, w)) ** 2 <= c1 - 2 * np.vdot(g, w).real + 1e-12
        assert -(math.sqrt(sp.eta) * u - sp.delta) ** 2 <= alpha * u + beta + 1e-12
        assert -np.vdot(w, w).real <= (c4 - 1) - 2 * np.vdot(sp.w_i, w).real + 1e-12
    w, u = sp.w_i, sp.u_i
    assert abs(-abs(np.vdot(sp.a_m, w)) ** 2 - (c1 - 2 * np.vdot(g, w).real)) < 1e-12
    assert abs(-(math.sqrt(sp.eta) * u - sp.delta) ** 2 - (alpha * u + beta)) < 1e-12


def _small_design(delta, iters, n_pulses=160, rr=1.5, lam_b=200.0):
    g = paper_radar(n_pulses)
    p = F.SasParams(iters=iters, d_angle=math.radians(2.0), phi_mw=math.radians(4.0), eta=0.01, u_min=2.0,
                    lam_b=lam_b)
    return g, p, F.design_bin(g, rr, delta, p)


def test_sca_objective_never_increases():
    """FPP-SCA: the previous iterate is feasible for the next sub-problem, so J^(i) is
    non-increasing (up to the sub-problem's duality-gap tolerance)."""
    _, p, res = _small_design(0.02, 10)
    js = [h["J"] for h in res.history]
    for a, b in zip(js, js[1:]):
        assert b <= a + 1e-5, js
    assert js[-1] < js[0]


def test_design_meets_worst_case_constraints():
    """After 32 iterations the slacks of C1 and C2 have vanished (the norm slack b, which only
    relaxes ||w|| = 1, is below 1e-4), and the design satisfies the worst-case forms of C1 and C2
    (eqs. 31-32) as the beampattern oracle measures them: (|w^H a_m| - Delta_R)^2 >= U and
    (|w^H a_s| + Delta_R)^2 <= eta U on the side-lobe grid, i.e. the robust ratio <= eta; ||w|| = 1
    (C3) to the slack; and the l1 objective made it sparse."""
    delta = 0.02
    g, p, res = _small_design(delta, 32)
    last = res.history[-1]
    assert last["b1"] < 1e-8 and last["b2"] < 1e-8 and last["b"] < 1e-4, last
    rr = 1.5
    n = g.n_pulses
    offs = res.offsets.astype(np.int32)[None, :]
    w = res.w[None, :]
    grid = synth.PolarGrid(1, n, rr, 0.1)
    phi_s = F.sidelobe_angles(res.offsets, n, p.phi_mw, p.d_angle)
    pat = oracle.beampattern(g, grid, offs, w, n, np.concatenate([[0.0], phi_s]))[0]
    main, side = pat[0], pat[1:].max()
    u_design = res.u_prime ** 2
    assert (main - delta) ** 2 >= u_design * (1 - 1e-4)
    assert (side + delta) ** 2 <= p.eta * u_design * (1 + 1e-3)
    ratio = oracle.robust_summary(np.array([main]), np.array([side]), np.array([delta]))[0]
    assert ratio <= p.eta * (1 + 1e-3)
    assert abs(np.linalg.norm(res.w) - 1) < 1e-3          # thresholding removes only |w_k| < Th
    assert 0 < np.count_nonzero(res.w) < len(res.offsets)


def test_candidates_follow_visibility():
    """Candidates of a bin are the phase centres of eqs. 4-5: the paper's 381 for R = 2 m."""
    g = paper_radar()
    assert len(F.candidates(g, 2.0)) == 381
    lo, hi = oracle.visible_index_range(2.0, g.radius_m, g.n_pulses)
    assert len(F.candidates(g, 2.0)) == hi - lo + 1
