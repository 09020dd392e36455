"""Plain FP64 CPU oracle of the offline robust sparse-array synthesis: Algorithm 1 of the paper
(FPP-SCA), solving the convex sub-problem of eq. 36 at every iteration.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or execute this
module: only the test suite and the benchmark's CPU-baseline leg do.  It shares no code with
the HIP implementation.

What is computed (Sec. III-A/B):
  * Per range bin R, the candidate phase centres are the pulses that see a target at the
    bin's azimuth (eqs. 4-5): offsets o with R cos(o 2 pi / N) > r.  The steering vector of a
    direction phi (radians from the target's azimuth) has the elements
    a_k(phi) = cos(theta'_k) exp(+j 2 k R(phi - D_k)), D_k = o_k 2 pi / N (eq. 16), with the
    cosine pattern taken as max(R cos D - r, 0) / R(D) as for back-projection.
  * The main lobe is phi_m = 0; the side-lobe directions phi_s are spaced by the sampled angle
    interval over [D_min, -phi_MW] and [phi_MW, D_max] (D_min, D_max the extreme candidates).
  * Iteration i solves eq. 36: the l1 norm plus lambda_b (b + b1 + b2) subject to the
    linearised C1 (eq. 33), C2 (eq. 34), C3, the linearised C4 (eq. 35), C5, and b, b1, b2 >= 0,
    around (w_(i-1), U'_(i-1)).
  * The convex sub-problem is solved by the barrier method (an interior-point method for convex
    inequality-constrained problems): minimise tau f0 + phi(x) by damped Newton steps with a
    backtracking line search, for tau multiplied by mu after each centring, until the duality
    gap bound m / tau is below eps.  |w_k| <= t_k enters as a second-order cone with the barrier
    -log(t_k^2 - |w_k|^2).  Variables x = [Re w, Im w, t, U', b, b1, b2].

Readings (where the paper is silent or inconsistent):
  * U'_(0): the paper writes |w_(0)^H a(phi; R)|^2 but defines U' = sqrt(U); we take
    U'_(0) = |w_(0)^H a(phi_m; R)|, the value consistent with U' = sqrt(U).
  * b, b1, b2 > 0 are taken as b, b1, b2 >= 0 (the closure; the barrier keeps them positive).
  * The final thresholding sets |w_k| < Th to zero (Th absolute, with ||w|| = 1), and a design
    is accepted when b + b1 + b2 < b_min.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

TWO_PI = 2.0 * math.pi


@dataclass
class SasParams:
    """Design parameters of Algorithm 1 (Table V gives ITER = 50, Th = 0.001, phi_MW = 1 deg,
    a 0.5 deg angle interval, lambda_b = 50, eta = 0.0005, U_min = 5)."""
    iters: int = 50
    th: float = 1e-3
    phi_mw: float = math.radians(1.0)
    d_angle: float = math.radians(0.5)
    lam_b: float = 50.0
    eta: float = 0.0005
    u_min: float = 5.0
    b_min: float = 1e-5
    # barrier method: stop when the duality-gap bound m / tau is below eps; a centring stops at
    # a Newton decrement^2 / 2 below newton_tol, after max_newton steps, or when the line search
    # cannot move (step below ls_min: the barrier values agree to rounding)
    eps: float = 1e-6
    mu: float = 8.0
    tau0: float = 1.0
    newton_tol: float = 1e-8
    max_newton: int = 50
    ls_alpha: float = 0.01
    ls_beta: float = 0.5
    ls_min: float = 1e-10


def candidates(geom, rr: float) -> np.ndarray:
    """Offsets o (pulses from the target's azimuth) of the phase centres that see a target at
    range rr (eqs. 4-5): R cos(o 2 pi / N) - r > 0."""
    n = geom.n_pulses
    half = n // 2
    o = np.arange(-half, n - half)
    return o[rr * np.cos(o * TWO_PI / n) - geom.radius_m > 0]


def steering(geom, rr: float, offsets: np.ndarray, phi: np.ndarray, k: float) -> np.ndarray:
    """Steering vectors a(phi; R) as rows [len(phi), n] (eq. 16)."""
    d = np.asarray(phi, dtype=np.float64)[:, None] - offsets[None, :] * (TWO_PI / geom.n_pulses)
    r = geom.radius_m
    rn = np.sqrt(rr * rr + r * r - 2.0 * rr * r * np.cos(d))
    alpha = np.maximum(rr * np.cos(d) - r, 0.0) / rn
    return alpha * np.exp(1j * 2.0 * k * rn)


def sidelobe_angles(offsets: np.ndarray, n_pulses: int, phi_mw: float, d_angle: float) -> np.ndarray:
    """phi_s spaced by d_angle over [D_min, -phi_MW] and [phi_MW, D_max]."""
    d_min = offsets.min() * TWO_PI / n_pulses
    d_max = offsets.max() * TWO_PI / n_pulses
    left = -phi_mw - d_angle * np.arange(int(math.floor((-phi_mw - d_min) / d_angle)) + 1)
    right = phi_mw + d_angle * np.arange(int(math.floor((d_max - phi_mw) / d_angle)) + 1)
    return np.concatenate([left[::-1], right])


# ----------------------------------------------------------------------------- sub-problem
@dataclass
class SubProblem:
    """Data of eq. 36 around (w_i, U'_i): a_m [n], a_s [S, n] (rows a(phi_s)), Delta_R, eta,
    U'_min = sqrt(U_min) and lambda_b."""
    a_m: np.ndarray
    a_s: np.ndarray
    w_i: np.ndarray
    u_i: float
    delta: float
    eta: float
    u_min: float
    lam_b: float

    @property
    def n(self):
        return self.a_m.shape[0]

    def lin(self):
        """Constants of the linearised C1, C2 and C4 (eqs. 33-35)."""
        g = self.a_m * np.vdot(self.a_m, self.w_i)        # a a^H w_i
        c1 = abs(np.vdot(self.a_m, self.w_i)) ** 2         # w_i^H a a^H w_i
        se = math.sqrt(self.eta)
        alpha = 2.0 * (se * self.delta - self.eta * self.u_i)
        beta = self.eta * self.u_i ** 2 - self.delta ** 2
        c4 = 1.0 + np.vdot(self.w_i, self.w_i).real
        return g, c1, alpha, beta, c4


def _unpack(x, n):
    w = x[:n] + 1j * x[n:2 * n]
    return w, x[2 * n:3 * n], x[3 * n], x[3 * n + 1], x[3 * n + 2], x[3 * n + 3]


def constraints(sp: SubProblem, x: np.ndarray) -> dict:
    """Values of every inequality f(x) <= 0 of eq. 36 (and the cones |w_k| - t_k)."""
    n = sp.n
    w, t, u, b, b1, b2 = _unpack(x, n)
    g, c1, alpha, beta, c4 = sp.lin()
    z = sp.a_s.conj() @ w                                  # a(phi_s)^H w
    return {
        "cone": np.abs(w) - t,
        "c1": (u + sp.delta) ** 2 + c1 - 2.0 * np.vdot(g, w).real - b1,
        "c2": np.abs(z) ** 2 + alpha * u + beta - b2,
        "c3": np.vdot(w, w).real - 1.0 - b,
        "c4": c4 - b - 2.0 * np.vdot(sp.w_i, w).real,
        "c5": sp.u_min - u,
        "b": -np.array([b, b1, b2]),
    }


def objective(sp: SubProblem, x: np.ndarray) -> float:
    n = sp.n
    w, t, u, b, b1, b2 = _unpack(x, n)
    return float(np.sum(np.abs(w)) + sp.lam_b * (b + b1 + b2))


def _barrier_terms(sp: SubProblem, x: np.ndarray, tau: float, need_hessian: bool):
    """tau f0 + phi(x), its gradient and (optionally) Hessian, or None outside the domain."""
    n = sp.n
    nv = 3 * n + 4
    iu, ib, ib1, ib2 = 3 * n, 3 * n + 1, 3 * n + 2, 3 * n + 3
    w, t, u, b, b1, b2 = _unpack(x, n)
    g, c1, alpha, beta, c4 = sp.lin()
    val = 0.0
    grad = np.zeros(nv)
    hess = np.zeros((nv, nv)) if need_hessian else None
    # objective: sum t + lambda_b (b + b1 + b2)
    val += tau * (np.sum(t) + sp.lam_b * (b + b1 + b2))
    grad[2 * n:3 * n] += tau
    grad[[ib, ib1, ib2]] += tau * sp.lam_b

    def scalar(f, df, d2f=None):
        nonlocal val
        if not f < 0:
            return False
        val_ = -math.log(-f)
        val += val_
        grad[:] += df / (-f)
        if need_hessian:
            hess[:] += np.outer(df, df) / (f * f)
            if d2f is not None:
                hess[:] += d2f / (-f)
        return True

    # second-order cones |w_k| <= t_k: -log(t^2 - |w|^2)
    uu = t * t - np.abs(w) ** 2
    if np.any(uu <= 0) or np.any(t <= 0):
        return None
    val += -np.sum(np.log(uu))
    wr, wi = w.real, w.imag
    grad[:n] += 2 * wr / uu
    grad[n:2 * n] += 2 * wi / uu
    grad[2 * n:3 * n] += -2 * t / uu
    if need_hessian:
        # per cone: diag(2, 2, -2) / u + du du^T / u^2 with du = (-2 wr, -2 wi, 2 t)
        du = np.stack([-2 * wr, -2 * wi, 2 * t])                        # [3, n]
        ks = np.arange(n)
        blocks = [ks, n + ks, 2 * n + ks]
        for i1 in range(3):
            for i2 in range(3):
                hv = du[i1] * du[i2] / uu ** 2
                if i1 == i2:
                    hv = hv + (2.0 if i1 < 2 else -2.0) / uu
                hess[blocks[i1], blocks[i2]] += hv
    # C1: (U' + Delta)^2 + c1 - 2 Re(g^H w) - b1
    f = (u + sp.delta) ** 2 + c1 - 2.0 * np.vdot(g, w).real - b1
    df = np.zeros(nv)
    df[:n], df[n:2 * n] = -2 * g.real, -2 * g.imag
    df[iu], df[ib1] = 2 * (u + sp.delta), -1.0
    d2 = np.zeros((nv, nv))
    d2[iu, iu] = 2.0
    if not scalar(f, df, d2 if need_hessian else None):
        return None
    # C2_s: |a_s^H w|^2 + alpha U' + beta - b2, all s at once
    a_s = sp.a_s
    z = a_s.conj() @ w                                                  # [S]
    f2 = np.abs(z) ** 2 + alpha * u + beta - b2
    if not np.all(f2 < 0):
        return None
    val += -np.sum(np.log(-f2))
    pm = np.concatenate([a_s.real, a_s.imag], axis=1)                  # rows d Re z_s / d(wr, wi)
    qm = np.concatenate([-a_s.imag, a_s.real], axis=1)                 # rows d Im z_s / d(wr, wi)
    dfw = 2 * (z.real[:, None] * pm + z.imag[:, None] * qm)            # [S, 2n]
    df2 = np.zeros((len(z), nv))
    df2[:, :2 * n] = dfw
    df2[:, iu], df2[:, ib2] = alpha, -1.0
    inv = 1.0 / (-f2)
    grad[:] += df2.T @ inv
    if need_hessian:
        hess[:] += (df2 * (inv * inv)[:, None]).T @ df2
        hess[:2 * n, :2 * n] += 2 * ((pm * inv[:, None]).T @ pm + (qm * inv[:, None]).T @ qm)
    # C3: ||w||^2 - 1 - b
    f = np.vdot(w, w).real - 1.0 - b
    df = np.zeros(nv)
    df[:n], df[n:2 * n], df[ib] = 2 * wr, 2 * wi, -1.0
    d2 = None
    if need_hessian:
        d2 = np.zeros((nv, nv))
        d2[:2 * n, :2 * n] = 2 * np.eye(2 * n)
    if not scalar(f, df, d2):
        return None
    # C4: 1 - b + ||w_i||^2 - 2 Re(w_i^H w)
    f = c4 - b - 2.0 * np.vdot(sp.w_i, w).real
    df = np.zeros(nv)
    df[:n], df[n:2 * n], df[ib] = -2 * sp.w_i.real, -2 * sp.w_i.imag, -1.0
    if not scalar(f, df):
        return None
    # C5: U'_min - U'
    df = np.zeros(nv)
    df[iu] = -1.0
    if not scalar(sp.u_min - u, df):
        return None
    # b, b1, b2 >= 0
    for ix in (ib, ib1, ib2):
        df = np.zeros(nv)
        df[ix] = -1.0
        if not scalar(-x[ix], df):
            return None
    return val, grad, hess


def strictly_feasible_start(sp: SubProblem, w0: np.ndarray, u0: float) -> np.ndarray:
    """A point inside every constraint: w = w0, t = |w0| + 1, U' = max(u0, U'_min + 1), and each
    slack one above the largest violation of the constraints it relaxes."""
    n = sp.n
    x = np.zeros(3 * n + 4)
    x[:n], x[n:2 * n] = w0.real, w0.imag
    x[2 * n:3 * n] = np.abs(w0) + 1.0
    x[3 * n] = u0 if u0 > sp.u_min + 1e-3 else sp.u_min + 1.0
    x[3 * n + 1:3 * n + 4] = 0.0
    c = constraints(sp, x)
    x[3 * n + 1] = max(c["c3"], c["c4"], 0.0) + 1.0
    x[3 * n + 2] = max(c["c1"], 0.0) + 1.0
    x[3 * n + 3] = max(np.max(c["c2"]), 0.0) + 1.0
    return x


def solve_subproblem(sp: SubProblem, p: SasParams, x0: np.ndarray | None = None) -> tuple[np.ndarray, dict]:
    """Barrier method on eq. 36 from a strictly feasible x0 (default: from (w_i, U'_i)).
    Returns the final iterate and {'tau', 'newton_steps', 'gap_bound'}."""
    n = sp.n
    m = 2 * n + sp.a_s.shape[0] + 7                     # barrier degree: cones count 2
    x = strictly_feasible_start(sp, sp.w_i, sp.u_i) if x0 is None else x0.copy()
    tau = p.tau0
    steps = 0
    while True:
        for _ in range(p.max_newton):
            val, grad, hess = _barrier_terms(sp, x, tau, True)
            dx = np.linalg.solve(hess, -grad)
            dec2 = float(-grad @ dx)                        # Newton decrement squared
            if dec2 / 2.0 <= p.newton_tol:
                break
            s = 1.0
            while s >= p.ls_min:
                r = _barrier_terms(sp, x + s * dx, tau, False)
                if r is not None and r[0] <= val + p.ls_alpha * s * float(grad @ dx):
                    break
                s *= p.ls_beta
            if s < p.ls_min:
                break
            x = x + s * dx
            steps += 1
        if m / tau < p.eps:
            break
        tau *= p.mu
    return x, {"tau": tau, "newton_steps": steps, "gap_bound": m / tau}


# ----------------------------------------------------------------------------- Algorithm 1
@dataclass
class SasResult:
    w: np.ndarray                  # [n] complex weights after thresholding
    offsets: np.ndarray            # [n] candidate offsets
    u_prime: float
    slack: float                   # b + b1 + b2 of the last iteration
    accepted: bool                 # slack < b_min
    history: list = field(default_factory=list)   # per iteration: dict(J, U', b, b1, b2, w)


def design_bin(geom, rr: float, delta: float, p: SasParams, record_w: bool = False) -> SasResult:
    """Algorithm 1 for one range bin: candidates and steering vectors of the bin, w_(0) uniform
    with unit norm, U'_(0) = |w_(0)^H a(phi_m)|, then ITER solutions of eq. 36, each
    linearised at the previous one; entries below Th set to zero."""
    k = 2.0 * math.pi * (geom.slope_hz_s * geom.t_start_s + geom.fc_hz) / geom.c_m_s
    offs = candidates(geom, rr)
    n = len(offs)
    a_m = steering(geom, rr, offs, np.array([0.0]), k)[0]
    phi_s = sidelobe_angles(offs, geom.n_pulses, p.phi_mw, p.d_angle)
    a_s = steering(geom, rr, offs, phi_s, k)
    w = np.ones(n, dtype=np.complex128) / math.sqrt(n)
    u = abs(np.vdot(w, a_m))
    hist = []
    x = None
    for _ in range(p.iters):
        sp = SubProblem(a_m, a_s, w, u, delta, p.eta, math.sqrt(p.u_min), p.lam_b)
        x, info = solve_subproblem(sp, p)
        w = x[:n] + 1j * x[n:2 * n]
        u = float(x[3 * n])
        b, b1, b2 = (float(v) for v in x[3 * n + 1:3 * n + 4])
        rec = {"J": objective(sp, x), "U": u, "b": b, "b1": b1, "b2": b2, "newton": info["newton_steps"]}
        if record_w:
            rec["w"] = w.copy()
        hist.append(rec)
    slack = hist[-1]["b"] + hist[-1]["b1"] + hist[-1]["b2"]
    wt = np.where(np.abs(w) < p.th, 0.0, w)
    return SasResult(wt, offs, u, slack, slack < p.b_min, hist)
