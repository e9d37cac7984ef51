"""Reduced-order model of an electric-field-driven droplet on a lubricant-infused surface
(Results, Eqs. 1-7): the drag coefficient from the geometric-mean viscosity and the pillar
spreading factor (Eq. 1), the point-dipole DEP force of a strip electrode (Eqs. 2-4), the
equation of motion (Eq. 5), its quasi-steady transport time (Eqs. 6-7), and fits of the drag
coefficient and the force-balance factor to a trajectory.

This is host-side modelling in numpy/scipy on scalars; it does not touch the lattice.  Units are
whatever the caller uses consistently (lattice units for trajectories of this package's
simulations).
"""
from __future__ import annotations

import math

import numpy as np


def spreading_ratio(gamma_og, gamma_wg, gamma_ow, theta_os, theta_ws):
    """I_os(w) / I_s (text before Eq. 1): the spreading coefficient of lubricant on the pillars
    in the presence of the droplet, I_os(w) = gamma_og cos(theta_os) - gamma_wg cos(theta_ws)
    - gamma_ow, over the reference I_s = -gamma_ow.  Angles in radians; o = lubricant (oil),
    w = droplet (water), g = ambient gas."""
    i_osw = gamma_og * math.cos(theta_os) - gamma_wg * math.cos(theta_ws) - gamma_ow
    return i_osw / (-gamma_ow)


def effective_viscosity(mu_w, mu_o, mu_g):
    """Geometric mean of the three phases' dynamic viscosities (text before Eq. 1)."""
    return (mu_w * mu_o * mu_g) ** (1.0 / 3.0)


def drag_coefficient(c_alpha, ratio, mu_bar, mu_o):
    """Eq. 1b: C_drag = C_alpha (1 + 1.5 ratio^2) mu_bar / mu_o, ratio = I_os(w) / I_s.  The
    relation holds in the paper's mobile regime 0 < ratio < 0.8; above 0.8 the droplet is pinned
    and below 0 the drag no longer depends on the wettability (ratio is then taken as 0)."""
    r = max(ratio, 0.0)
    return c_alpha * (1.0 + 1.5 * r * r) * mu_bar / mu_o


def drag_force_scaled(c_drag, r0, l_c, ca):
    """Eq. 1a: F_drag / (2 gamma_ow R0) = 3.5 pi C_drag (R0 / l_c)^0.5 Ca.  The length l_c is not
    defined in the text; the caller supplies it."""
    return 3.5 * math.pi * c_drag * math.sqrt(r0 / l_c) * ca


def dep_factor(eps_w, r0, sigma_w, sigma_o, reading="clausius-mossotti"):
    """K_e of Eq. 2 for a sphere of radius r0 and permittivity eps_w.  The printed denominator
    is sigma_w - 2 sigma_o; the DC Clausius-Mossotti factor of a dipole has sigma_w + 2 sigma_o.
    reading="clausius-mossotti" (default) takes the latter, reading="printed" the former; for
    sigma_w >> sigma_o (the paper's regime) both tend to 2 pi eps_w r0^3, and the free factor
    Lambda of Eq. 5 absorbs what is left."""
    if reading == "clausius-mossotti":
        den = sigma_w + 2.0 * sigma_o
    elif reading == "printed":
        den = sigma_w - 2.0 * sigma_o
    else:
        raise ValueError(f"unknown reading {reading!r}")
    return 2.0 * math.pi * eps_w * r0 ** 3 * (sigma_w - sigma_o) / den


def strip_constants(phi0, h_e, l_e):
    """Eq. 4: decay rate alpha0 = pi / (2 (h_e + l_e)) of the strip's lowest Laplace mode
    sin(alpha0 y) (grounded at y = 0, insulating at y = h_e + l_e), the integrals J_N (over the
    insulating part 0..l_e of the electrode wall) and J_D (over the electrode part l_e..h_e + l_e)
    of sin^2(alpha0 y), and the amplitude C_ele of the squared field's decay.  alpha0, J_N and
    J_D follow from the mode itself; C_ele comes from a derivation given outside the main text
    and is checked only through its phi0^2 scaling (parity unpinned)."""
    a0 = math.pi / (2.0 * (h_e + l_e))
    s2 = math.sin(2.0 * a0 * l_e) / (4.0 * a0)
    j_n = l_e / 2.0 - s2
    j_d = h_e / 2.0 + s2
    c_ele = 2.0 * a0 * phi0 ** 2 * math.cos(a0 * l_e) ** 2 / (j_d + a0 * j_n) ** 2
    return dict(alpha0=a0, J_N=j_n, J_D=j_d, C_ele=c_ele)


def electric_force(k_e, c_ele, alpha0, s_e):
    """Eq. 3: DEP force K_e C_ele exp(-2 alpha0 S_e) at droplet-electrode distance s_e."""
    return k_e * c_ele * math.exp(-2.0 * alpha0 * s_e)


def _rhs(state, m, drag, drive, alpha0, s0):
    s, v = state
    return np.array([v, (-drag * v + drive * math.exp(-2.0 * alpha0 * (s0 - s))) / m])


def integrate_motion(t_end, m, c_drag, r0, mu_bar, drive, alpha0, s0, v0=0.0, n_steps=20000, t_out=None):
    """Eq. 5, m S'' = -C_drag 2 R0 mu_bar S' + drive exp(-2 alpha0 (S0 - S)) with drive =
    Lambda K_e C_ele, from S(0) = 0, S'(0) = v0, by classical fourth-order Runge-Kutta with
    n_steps equal steps.  Returns (t, S, V) at the step times, or at t_out (sorted, within
    [0, t_end]) by cubic Hermite interpolation of the steps."""
    drag = 2.0 * c_drag * r0 * mu_bar
    h = t_end / n_steps
    ts = np.linspace(0.0, t_end, n_steps + 1)
    y = np.empty((n_steps + 1, 2))
    y[0] = (0.0, v0)
    for i in range(n_steps):
        yi = y[i]
        k1 = _rhs(yi, m, drag, drive, alpha0, s0)
        k2 = _rhs(yi + 0.5 * h * k1, m, drag, drive, alpha0, s0)
        k3 = _rhs(yi + 0.5 * h * k2, m, drag, drive, alpha0, s0)
        k4 = _rhs(yi + h * k3, m, drag, drive, alpha0, s0)
        y[i + 1] = yi + (h / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
    if t_out is None:
        return ts, y[:, 0], y[:, 1]
    t_out = np.asarray(t_out, dtype=np.float64)
    idx = np.clip(np.searchsorted(ts, t_out, side="right") - 1, 0, n_steps - 1)
    u = (t_out - ts[idx]) / h
    s_a, s_b, v_a, v_b = y[idx, 0], y[idx + 1, 0], y[idx, 1], y[idx + 1, 1]
    h00, h10, h01, h11 = 2 * u**3 - 3 * u**2 + 1, u**3 - 2 * u**2 + u, -2 * u**3 + 3 * u**2, u**3 - u**2
    s = h00 * s_a + h10 * h * v_a + h01 * s_b + h11 * h * v_b
    v = v_a + u * (v_b - v_a)
    return t_out, s, v


def transport_time(s_t, m, c_drag, r0, mu_bar, drive, alpha0, s0, inertia=True):
    """Eq. 7: time to travel s_t from rest, from the quasi-steady slope of Eq. 6 (the velocity at
    which drag balances the force, plus the first-order inertial lag 2 alpha0 tau_v with
    tau_v = m / (2 C_drag R0 mu_bar)).  inertia=False drops the second term."""
    cr = r0 * mu_bar * c_drag
    t = cr / (alpha0 * drive) * (math.exp(2.0 * alpha0 * s0) - math.exp(2.0 * alpha0 * (s0 - s_t)))
    if inertia:
        t += alpha0 * m / cr * s_t
    return t


def average_velocity(s_t, *args, **kw):
    """V_avg = S_t / t(S_t) with t from Eq. 7 (same arguments as transport_time)."""
    return s_t / transport_time(s_t, *args, **kw)


def drag_from_deceleration(m, v0, r0, mu_bar, s_max):
    """C_drag,sim = m V0 / (2 R0 mu_bar S_max): the drag coefficient that stops a droplet
    launched at V0 after S_max under linear drag alone (Eq. 5 without the electric term)."""
    return m * v0 / (2.0 * r0 * mu_bar * s_max)


def fit_motion(t, s, m, r0, mu_bar, alpha0, s0, guess=(1.0, 1.0), n_steps=4000):
    """Least-squares fit of (C_drag, drive = Lambda K_e C_ele) of Eq. 5 to a trajectory S(t)
    that starts from rest at t[0] = 0 (S measured from the start).  Both parameters are fitted
    in logarithms, so they stay positive.  Returns dict(c_drag, drive, rms)."""
    from scipy.optimize import least_squares

    t = np.asarray(t, dtype=np.float64)
    s = np.asarray(s, dtype=np.float64)
    scale = max(float(np.max(np.abs(s))), 1e-300)

    def resid(p):
        c, d = math.exp(p[0]), math.exp(p[1])
        _, sm, _ = integrate_motion(float(t[-1]), m, c, r0, mu_bar, d, alpha0, s0, n_steps=n_steps, t_out=t)
        return (sm - s) / scale

    res = least_squares(resid, np.log(np.asarray(guess, dtype=np.float64)), method="lm", xtol=1e-14,
                        ftol=1e-14, gtol=1e-14)
    c, d = (float(math.exp(x)) for x in res.x)
    return dict(c_drag=c, drive=d, rms=float(np.sqrt(np.mean(res.fun ** 2))) * scale)


def overdamped_time(s, v0, alpha0):
    """Eq. 7 without its inertial term: the time to travel s from rest when drag balances the
    electric force at every instant, t(s) = (1 - exp(-2 alpha0 s)) / (2 alpha0 v0), with v0 =
    Lambda K_e C_ele exp(-2 alpha0 S0) / (2 C_drag R0 mu_bar) the balance velocity at the start."""
    s = np.asarray(s, dtype=np.float64)
    return (1.0 - np.exp(-2.0 * alpha0 * s)) / (2.0 * alpha0 * v0)


def fit_overdamped(t, s, alpha0):
    """Least-squares fit of the start velocity v0 of the overdamped transport law (Eq. 7 without
    inertia) to a trajectory S(t) from rest: t_i = g(S_i) / v0 with g(S) = (1 - exp(-2 alpha0 S))
    / (2 alpha0), linear in 1/v0.  Where the viscous relaxation time m / (2 C_drag R0 mu_bar) is
    many orders below the travel time (the lattice-unit workloads), a trajectory fixes only this
    ratio of drive to drag, not C_drag and Lambda separately.  Returns dict(v0, rms_t) with the
    root-mean-square time residual."""
    t = np.asarray(t, dtype=np.float64)
    g = (1.0 - np.exp(-2.0 * alpha0 * np.asarray(s, dtype=np.float64))) / (2.0 * alpha0)
    v0 = float(g @ g / (g @ t))
    return dict(v0=v0, rms_t=float(np.sqrt(np.mean((t - g / v0) ** 2))))


def drag_to_drive(v0, alpha0, s0, r0, mu_bar):
    """C_drag / (Lambda K_e C_ele) from the fitted start velocity v0 of fit_overdamped."""
    return math.exp(-2.0 * alpha0 * s0) / (2.0 * r0 * mu_bar * v0)


# ------------------------------------------------------------------ two-electrode switching (Fig. 5b)
def _leg_time(x_from, x_to, u, alpha0, dist_from, dist_to):
    """Overdamped travel time between two positions under one electrode pulling with velocity
    u exp(-2 alpha0 S_e): (exp(2 alpha0 S_from) - exp(2 alpha0 S_to)) / (2 alpha0 u), S the
    distances to that electrode."""
    return (math.exp(2.0 * alpha0 * dist_from) - math.exp(2.0 * alpha0 * dist_to)) / (2.0 * alpha0 * u)


def two_electrode_switch_times(u, alpha0, half_gap, s_sw, t_sw1=None):
    """The periodic protocol of the Results (Fig. 5b) in the overdamped form of Eq. 5: a droplet
    midway between two electrodes at distance half_gap from each is pulled by electrode 1 until
    its distance to it falls to s_sw (time t_sw1), then by electrode 2 until its distance to that
    one falls to s_sw (time t_sw2).  u is the pull velocity at zero distance (v0 exp(2 alpha0
    S0)).  Given t_sw1 (e.g. advanced or delayed), the first leg stops where the droplet is then;
    returns (t_sw1, t_sw2, position at the first switch), positions measured from the midpoint
    towards electrode 1.  A t_sw1 at or beyond the electrode's arrival time is invalid."""
    t_arrive = math.exp(2.0 * alpha0 * half_gap) / (2.0 * alpha0 * u)
    if t_sw1 is None:
        t_sw1 = _leg_time(0.0, half_gap - s_sw, u, alpha0, half_gap, s_sw)
    if not t_sw1 < t_arrive:
        raise ValueError("the droplet reaches electrode 1 before the switch")
    # position under electrode 1 after t: exp(2 a0 S_e1) = exp(2 a0 half_gap) - 2 a0 u t
    s_e1 = math.log(math.exp(2.0 * alpha0 * half_gap) - 2.0 * alpha0 * u * t_sw1) / (2.0 * alpha0)
    x1 = half_gap - s_e1
    t2 = _leg_time(x1, -(half_gap - s_sw), u, alpha0, half_gap + x1, s_sw)
    return t_sw1, t_sw1 + t2, x1


def two_electrode_position(t, u, alpha0, half_gap, t_sw1):
    """Position at time t of the two-electrode protocol in the overdamped Eq. 5: pulled by
    electrode 1 (distance half_gap ahead at the start) until t_sw1, then by electrode 2 (as far
    behind the start).  Positions from the start, towards electrode 1; no turn-back past the
    electrodes (t_sw1 before the arrival at electrode 1, t before the arrival at electrode 2)."""
    a2 = 2.0 * alpha0
    e1 = math.exp(a2 * half_gap) - a2 * u * min(t, t_sw1)
    if not e1 > 1.0:
        raise ValueError("the droplet reaches electrode 1")
    x = half_gap - math.log(e1) / a2
    if t <= t_sw1:
        return x
    e2 = math.exp(a2 * (half_gap + x)) - a2 * u * (t - t_sw1)
    if not e2 > 1.0:
        raise ValueError("the droplet reaches electrode 2")
    return math.log(e2) / a2 - half_gap


def two_electrode_switch_for_target(u, alpha0, half_gap, T, x_target=0.0, tol=1e-9):
    """The switch time t_sw1 of the two-electrode protocol that puts the droplet at x_target at
    time T (overdamped Eq. 5; x(T) grows with t_sw1, so bisection on [0, T])."""
    f = lambda ts: two_electrode_position(T, u, alpha0, half_gap, ts) - x_target
    lo, hi = 0.0, float(T)
    if not (f(lo) <= 0.0 <= f(hi)):
        raise ValueError("target not reachable with one switch before T")
    while hi - lo > tol * T:
        mid = 0.5 * (lo + hi)
        if f(mid) < 0.0:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


# ------------------------------------------------------------------ long-distance transport (Fig. 5c)
def relay_switch_times(u, alpha0, s0, pitch, s_sw, n_electrodes=3):
    """The long-distance protocol of the Results (Fig. 5c) in the overdamped form of Eq. 5:
    electrodes at a fixed pitch ahead of the droplet, the first at distance s0; each is switched
    off, and the next one on, when the droplet's distance to it falls to s_sw.  u is the pull
    velocity at zero distance.  Returns (switch times, arrival time at s_sw from the last
    electrode), times from the start; the droplet has then travelled s0 - s_sw + (n - 1) pitch."""
    if not (s0 > s_sw and pitch > 0 and s_sw >= 0 and n_electrodes >= 1):
        raise ValueError("need s0 > s_sw >= 0 and pitch > 0")
    t, times = 0.0, []
    dist = s0
    for k in range(n_electrodes):
        t += _leg_time(0.0, dist - s_sw, u, alpha0, dist, s_sw)
        times.append(t)
        dist = s_sw + pitch
    return times[:-1], times[-1]


def relay_position(t, u, alpha0, s0, pitch, s_sw, switch_times):
    """Displacement at times t under the relay protocol with the given switch times (the droplet
    keeps moving towards the last electrode after the last switch), from the overdamped law: under
    an electrode at distance S, exp(2 alpha0 S) falls at the rate 2 alpha0 u."""
    t = np.atleast_1d(np.asarray(t, dtype=np.float64))
    out = np.empty_like(t)
    for i, ti in enumerate(t):
        x, t0, dist0 = 0.0, 0.0, s0   # displacement and electrode distance at the stage start
        for k, ts in enumerate(list(switch_times) + [math.inf]):
            tend = min(ti, ts)
            e = math.exp(2.0 * alpha0 * dist0) - 2.0 * alpha0 * u * (tend - t0)
            d = math.log(e) / (2.0 * alpha0) if e > 1.0 else 0.0   # at the electrode: stays there
            x += dist0 - d
            if ti <= ts:
                break
            t0, dist0 = ts, d + pitch
        out[i] = x
    return out
