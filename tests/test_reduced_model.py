"""Reduced-order droplet-migration model (paper_2608_12868_amd/reduced.py, Results Eqs. 1-7)
pinned to what the mathematics fixes: Young's relations for the spreading factor, the strip's
Laplace mode and its integrals by quadrature, the closed-form decay under linear drag, Eq. 7 as
the exact integral of Eq. 6 and as the transport time of Eq. 5 up to the start-up lag, and the
fit recovering the parameters of a trajectory integrated at another resolution."""
import math

import numpy as np
import pytest
from scipy.integrate import quad

from paper_2608_12868_amd import reduced as rm


def test_spreading_ratio_matches_young_relations():
    # Young on the solid: gamma_os = gamma_sg - gamma_og cos(theta_os), gamma_sw = gamma_sg -
    # gamma_wg cos(theta_ws); droplet on the solid under lubricant: gamma_os - gamma_sw =
    # gamma_ow cos(theta_ws(o)).  The ratio is then 1 + cos(theta_ws(o)), whatever gamma_sg is.
    g_og, g_wg, g_ow = 20.0, 72.0, 40.0
    for th_os, th_ws in ((5.0, 110.0), (30.0, 95.0), (40.0, 120.0)):
        a, b = math.radians(th_os), math.radians(th_ws)
        for g_sg in (30.0, 55.0):
            g_os = g_sg - g_og * math.cos(a)
            g_sw = g_sg - g_wg * math.cos(b)
            cos_wso = (g_os - g_sw) / g_ow
            assert rm.spreading_ratio(g_og, g_wg, g_ow, a, b) == pytest.approx(1.0 + cos_wso, abs=1e-13)


def test_drag_coefficient_special_cases():
    mu = (1.0, 3.0, 0.02)
    mu_bar = rm.effective_viscosity(*mu)
    assert mu_bar == pytest.approx(math.exp(sum(math.log(x) for x in mu) / 3.0), rel=1e-14)
    # a lubricant-dominated case with no pillar-wetting contribution reduces to C_alpha
    assert rm.drag_coefficient(17.1, 0.0, 2.0, 2.0) == pytest.approx(17.1, rel=1e-15)
    # negative spreading factor: drag independent of the wettability
    assert rm.drag_coefficient(17.1, -0.4, 2.0, 2.0) == pytest.approx(17.1, rel=1e-15)
    assert rm.drag_coefficient(10.0, 0.5, 1.0, 2.0) == pytest.approx(10.0 * 1.375 * 0.5, rel=1e-15)


def test_dep_factor_limits_and_readings():
    base = 2.0 * math.pi * 80.0 * 2.0 ** 3
    assert rm.dep_factor(80.0, 2.0, 1.0, 0.0) == pytest.approx(base, rel=1e-15)
    assert rm.dep_factor(80.0, 2.0, 1.0, 0.0, reading="printed") == pytest.approx(base, rel=1e-15)
    cm = rm.dep_factor(80.0, 2.0, 1.0, 0.01)
    pr = rm.dep_factor(80.0, 2.0, 1.0, 0.01, reading="printed")
    assert cm == pytest.approx(base * 0.99 / 1.02, rel=1e-14)
    assert pr == pytest.approx(base * 0.99 / 0.98, rel=1e-14)
    with pytest.raises(ValueError):
        rm.dep_factor(80.0, 2.0, 1.0, 0.01, reading="other")


@pytest.mark.parametrize("h_e,l_e", [(1.0, 3.0), (2.5, 0.5), (4.0, 4.0)])
def test_strip_constants_by_quadrature(h_e, l_e):
    c = rm.strip_constants(1.7, h_e, l_e)
    a0, L = c["alpha0"], h_e + l_e
    # lowest mode of the strip: grounded at y = 0, zero normal derivative at y = L
    assert math.sin(a0 * 0.0) == 0.0 and abs(math.cos(a0 * L)) < 1e-15
    assert c["J_N"] == pytest.approx(quad(lambda y: math.sin(a0 * y) ** 2, 0.0, l_e, epsrel=1e-13)[0], rel=1e-12)
    assert c["J_D"] == pytest.approx(quad(lambda y: math.sin(a0 * y) ** 2, l_e, L, epsrel=1e-13)[0], rel=1e-12)
    assert c["J_N"] + c["J_D"] == pytest.approx(L / 2.0, rel=1e-14)
    # C_ele scales with the square of the electrode potential
    assert rm.strip_constants(3.4, h_e, l_e)["C_ele"] == pytest.approx(4.0 * c["C_ele"], rel=1e-14)
    f1 = rm.electric_force(2.0, c["C_ele"], a0, 5.0)
    f2 = rm.electric_force(2.0, c["C_ele"], a0, 3.0)
    assert f2 / f1 == pytest.approx(math.exp(4.0 * a0), rel=1e-14)


def test_linear_drag_decay_closed_form_and_drag_from_deceleration():
    m, c, r0, mu, v0 = 2.0, 7.0, 1.5, 0.4, 0.3
    drag = 2.0 * c * r0 * mu
    t_end = 40.0 * m / drag
    t, s, v = rm.integrate_motion(t_end, m, c, r0, mu, 0.0, 0.1, 10.0, v0=v0, n_steps=4000)
    s_exact = m * v0 / drag * (1.0 - np.exp(-drag * t / m))
    assert np.max(np.abs(s - s_exact)) <= 1e-9 * s_exact[-1]
    assert np.max(np.abs(v - v0 * np.exp(-drag * t / m))) <= 1e-9 * v0
    assert rm.drag_from_deceleration(m, v0, r0, mu, s[-1]) == pytest.approx(c, rel=1e-12)


def test_eq7_is_the_integral_of_eq6():
    m, c, r0, mu, drive, a0, s0, st = 1.3, 10.0, 1.0, 0.8, 0.7, 0.1, 10.0, 3.0
    slope = lambda x: 2.0 * c * r0 * mu / (drive * math.exp(-2.0 * a0 * (s0 - x))) + a0 * m / (c * r0 * mu)
    t_quad = quad(slope, 0.0, st, epsabs=0.0, epsrel=1e-13)[0]
    assert rm.transport_time(st, m, c, r0, mu, drive, a0, s0) == pytest.approx(t_quad, rel=1e-12)
    assert rm.average_velocity(st, m, c, r0, mu, drive, a0, s0) == pytest.approx(st / t_quad, rel=1e-12)


@pytest.mark.parametrize("c_drag", [5.0, 10.0, 20.0])
def test_eq7_matches_the_motion_up_to_the_start_up_lag(c_drag):
    # tau_v = m / (2 C R0 mu) is far shorter than the travel time: Eq. 7 then misses the time at
    # which Eq. 5 (started from rest) reaches S_t by the velocity's start-up lag, about tau_v,
    # and its inertial term moves it closer than the plain quasi-steady estimate.
    m, r0, mu, drive, a0, s0, st = 1.0, 1.0, 1.0, 1.0, 0.1, 10.0, 3.0
    tau = m / (2.0 * c_drag * r0 * mu)
    t7 = rm.transport_time(st, m, c_drag, r0, mu, drive, a0, s0)
    t7q = rm.transport_time(st, m, c_drag, r0, mu, drive, a0, s0, inertia=False)
    t, s, _ = rm.integrate_motion(1.2 * t7, m, c_drag, r0, mu, drive, a0, s0, n_steps=20000)
    i = int(np.searchsorted(s, st))
    t_ode = t[i - 1] + (st - s[i - 1]) / (s[i] - s[i - 1]) * (t[i] - t[i - 1])
    assert abs(t7 - t_ode) <= 1.5 * tau
    assert abs(t7 - t_ode) < abs(t7q - t_ode)


def test_fit_recovers_parameters_of_a_trajectory():
    m, r0, mu, a0, s0 = 1.0, 1.0, 1.0, 0.1, 10.0
    c_true, d_true = 8.0, 1.6
    t_end = 0.8 * rm.transport_time(3.0, m, c_true, r0, mu, d_true, a0, s0)
    t_obs = np.linspace(0.0, t_end, 41)
    _, s_obs, _ = rm.integrate_motion(t_end, m, c_true, r0, mu, d_true, a0, s0, n_steps=30000, t_out=t_obs)
    rng = np.random.default_rng(3)
    s_noisy = s_obs + 1e-6 * float(s_obs[-1]) * rng.standard_normal(s_obs.size)
    fit = rm.fit_motion(t_obs, s_noisy, m, r0, mu, a0, s0, guess=(3.0, 0.5), n_steps=3000)
    assert fit["c_drag"] == pytest.approx(c_true, rel=1e-3)
    assert fit["drive"] == pytest.approx(d_true, rel=1e-3)
    assert fit["rms"] <= 1e-5 * float(s_obs[-1])


def test_overdamped_transport_fit():
    """The overdamped form of Eq. 7 is the exact solution of Eq. 5 without inertia (dS/dt =
    v0 exp(2 alpha0 S)), and its fit recovers v0 from a noisy trajectory of that law; with the
    inertial lag tau_v 1e-4 of the travel time the full Eq. 5 gives the same times."""
    a0, v0 = 0.025, 8e-5
    s = np.linspace(0.0, 36.0, 60)
    # dS/dt = v0 exp(2 a0 S) -> t(S) = (1 - exp(-2 a0 S)) / (2 a0 v0)
    t = np.array([quad(lambda x: math.exp(-2 * a0 * x) / v0, 0.0, si)[0] for si in s])
    assert np.allclose(rm.overdamped_time(s, v0, a0), t, rtol=1e-12, atol=1e-6)
    rng = np.random.default_rng(5)
    fit = rm.fit_overdamped(t * (1 + 0.01 * rng.standard_normal(t.size)), s, a0)
    assert abs(fit["v0"] / v0 - 1) < 0.01
    # Eq. 5 with drag 2 C R0 mu and drive chosen to have the same start velocity
    m, r0, mu, c = 226.0, 12.0, 1.0 / 6.0, 10.0
    s0 = 48.0
    drive = v0 * 2 * c * r0 * mu * math.exp(2 * a0 * s0)
    ratio = rm.drag_to_drive(v0, a0, s0, r0, mu)
    assert ratio == pytest.approx(c / drive, rel=1e-12)
    t_end = float(t[-1])
    ts, ss, _ = rm.integrate_motion(1.01 * t_end, m, c, r0, mu, drive, a0, s0, n_steps=200000)
    t36 = float(np.interp(36.0, ss, ts))
    assert abs(t36 / t_end - 1) < 1e-3


def test_two_electrode_switch_times_and_sensitivity():
    """The two-electrode protocol (Results, Fig. 5b) in the overdamped Eq. 5: the switch times
    from the closed-form legs agree with a direct integration of dS/dt = +-u exp(-2 alpha0 S_e);
    moving the first switch by +-10 % moves the second by several times more (the force grows
    exponentially towards the first electrode, so the return leg starts from a very different
    place), the sensitivity the paper points out (about 50 % there)."""
    u, a0, half, s_sw = 8.3e-5 * math.exp(2 * 0.02533 * 48.0), 0.02533, 48.0, 24.0
    t1, t2, x1 = rm.two_electrode_switch_times(u, a0, half, s_sw)
    assert x1 == pytest.approx(half - s_sw, rel=1e-12)
    # direct integration (forward Euler in small steps) of the same law
    x, t, dt = 0.0, 0.0, 1.0
    while half - x > s_sw:
        x += dt * u * math.exp(-2 * a0 * (half - x))
        t += dt
    assert t / t1 == pytest.approx(1.0, abs=1e-3)
    while x + half > s_sw:
        x -= dt * u * math.exp(-2 * a0 * (x + half))
        t += dt
    assert t / t2 == pytest.approx(1.0, abs=1e-3)
    late = rm.two_electrode_switch_times(u, a0, half, s_sw, t_sw1=1.1 * t1)
    early = rm.two_electrode_switch_times(u, a0, half, s_sw, t_sw1=0.9 * t1)
    leg = t2 - t1
    d_late = (late[1] - late[0]) / leg - 1
    d_early = (early[1] - early[0]) / leg - 1
    print("second leg", leg, "late switch", d_late, "early switch", d_early)
    assert d_late > 0.1 and d_early < -0.1
    assert abs(late[1] / t2 - 1) > 0.1 and abs(early[1] / t2 - 1) > 0.1
    with pytest.raises(ValueError):
        rm.two_electrode_switch_times(u, a0, half, s_sw, t_sw1=10 * t1)


def test_relay_switch_times_and_positions():
    """The long-distance protocol (Results, Fig. 5c) in the overdamped Eq. 5: electrodes at a
    fixed pitch, each switched off when the droplet is s_sw from it.  The closed-form switch
    times agree with a direct integration of dS/dt = u exp(-2 alpha0 S_e) under the active
    electrode, and the displacement at each switch is s0 - s_sw + k pitch."""
    u, a0, s0, pitch, s_sw = 7.7e-4, 0.02533, 48.0, 24.0, 18.0
    sw, arrive = rm.relay_switch_times(u, a0, s0, pitch, s_sw, 3)
    assert len(sw) == 2 and sw[0] < sw[1] < arrive
    x, t, dt, k, hits = 0.0, 0.0, 1.0, 0, []
    edge = s0
    while k < 3:
        x += dt * u * math.exp(-2 * a0 * (edge - x))
        t += dt
        if edge - x <= s_sw:
            hits.append(t)
            edge += pitch
            k += 1
    for a, b in zip(hits, list(sw) + [arrive]):
        assert a / b == pytest.approx(1.0, abs=1e-3)
    pos = rm.relay_position(list(sw) + [arrive], u, a0, s0, pitch, s_sw, sw)
    assert pos == pytest.approx([s0 - s_sw, s0 - s_sw + pitch, s0 - s_sw + 2 * pitch], abs=1e-9)
    # after the last switch the droplet keeps approaching the last electrode, never past it
    late = rm.relay_position([10 * arrive], u, a0, s0, pitch, s_sw, sw)[0]
    assert s0 - s_sw + 2 * pitch < late <= s0 + 2 * pitch
    with pytest.raises(ValueError):
        rm.relay_switch_times(u, a0, s_sw, pitch, s_sw)


def test_two_electrode_position_and_switch_for_target():
    """The protocol's position in time (overdamped Eq. 5, one switch) against a direct
    integration of dx/dt = +-u exp(-2 alpha0 S_e), and the switch time that returns the
    droplet to its start at T."""
    u, a0, half = 1.37e-3, math.pi / 92.0, 32.0
    t_sw, T = 19000.0, 45000.0
    x, t, dt = 0.0, 0.0, 0.5
    while t < T - 1e-9:
        s = (half - x) if t < t_sw else (half + x)
        x += (1.0 if t < t_sw else -1.0) * dt * u * math.exp(-2 * a0 * s)
        t += dt
        if abs(t - t_sw) < 1e-9:
            assert rm.two_electrode_position(t_sw, u, a0, half, t_sw) == pytest.approx(x, abs=2e-4)
    assert rm.two_electrode_position(T, u, a0, half, t_sw) == pytest.approx(x, abs=2e-4)
    ts = rm.two_electrode_switch_for_target(u, a0, half, T)
    assert abs(rm.two_electrode_position(T, u, a0, half, ts)) <= 1e-6
    assert rm.two_electrode_position(T, u, a0, half, 0.99 * ts) < 0.0 < rm.two_electrode_position(T, u, a0, half, 1.01 * ts)
    with pytest.raises(ValueError):
        rm.two_electrode_switch_for_target(u, a0, half, T, x_target=40.0)
