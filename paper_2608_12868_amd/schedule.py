"""Electrode-voltage schedules designed with the adjoint: the programmable droplet manipulation
that the paper pursues with electrode switching protocols (Results, Fig. 5), posed as reaching a
target droplet position at a given time.

The residual r(V) = x_c(T; V)[axis] - x* of the droplet centroid after T steps is a scalar
function of the piecewise-constant schedule V of one electrode; its gradient J = dr/dV comes
from one checkpointed forward and one adjoint sweep.  Each iteration takes the minimum-norm step
of the linearised residual, r + J dV = 0, over the segments that are not held at a voltage bound
(projected Gauss-Newton), halving it until |r| decreases.  Also: switch times designed with the
adjoint, the relay protocol's schedules (Fig. 5c) and the two-electrode periodic protocol
(Fig. 5b) switched on the droplet's position.  Host-side drivers only: every forward step and
every adjoint step runs in the library.
"""
import math

import numpy as np


def design_schedule(sim, phi0, volts0, t_total, T, K, target, axis=0, electrode=0, bounds=(0.0, 0.08),
                    iters=8, rtol=1e-3, max_halvings=6):
    """Returns (volts, history).  history[k]: residual, |step| and forward/adjoint sweeps of
    iteration k.  Stops when |r| <= rtol * |r_0| or after `iters` iterations."""
    lo, hi = bounds
    v = np.clip(np.asarray(volts0, dtype=np.float64), lo, hi)
    sweeps = {"forward": 0, "adjoint": 0}

    def run(volts):
        sim.set_phase(phi0)
        sim.set_schedule(electrode, volts, t_total)
        sim.forward_checkpointed(T, K)
        sweeps["forward"] += 1
        return float(sim.observables()["centroid"][axis])

    r = run(v) - target
    r0 = abs(r)
    history = [dict(iteration=0, residual=r, step=0.0, **sweeps)]
    gx = np.zeros(3)
    gx[axis] = 1.0
    for k in range(1, iters + 1):
        if abs(r) <= rtol * r0:
            break
        J = sim.adjoint(gx, np.zeros(3), electrode, v.size)  # d x_c[axis] / dV, same forward as r
        sweeps["adjoint"] += 1
        direction = -r * J
        free = ~(((v <= lo) & (direction < 0)) | ((v >= hi) & (direction > 0)))
        Jf = np.where(free, J, 0.0)
        nrm = float(Jf @ Jf)
        if nrm == 0.0:
            break
        dv = -r * Jf / nrm
        t = 1.0
        for _ in range(max_halvings + 1):
            v_new = np.clip(v + t * dv, lo, hi)
            r_new = run(v_new) - target
            if abs(r_new) < abs(r):
                break
            t *= 0.5
        else:
            break   # no decrease along the projected step: the sim holds the last trial's forward
        step = float(np.linalg.norm(v_new - v))
        v, r = v_new, r_new
        history.append(dict(iteration=k, residual=r, step=step, **sweeps))
    return v, history


def switch_schedules(t_sw, volts, n_seg, T):
    """Schedules of two electrodes for one switch at step t_sw (electrode 1 on before, electrode 2
    on after, both at `volts`) over n_seg segments of T / n_seg steps: the segment containing the
    switch holds each electrode at its on-time fraction of the segment (the time average of the
    switched voltage over the segment), so x_c(T) depends continuously on t_sw."""
    width = T / n_seg
    s = min(int(t_sw // width), n_seg - 1)
    frac = (t_sw - s * width) / width
    v1 = np.zeros(n_seg)
    v1[:s] = volts
    v1[s] = volts * frac
    v2 = volts - v1
    return v1, v2, s


def switch_time_gradient(sim, phi0, t_sw, volts, n_seg, T, K, axis=0, electrodes=(0, 1)):
    """x_c(T)[axis] and its derivative with respect to the switch time, from one checkpointed
    forward and the adjoint with respect to each electrode's schedule: d x / d t_sw =
    (dx/dV1[s] - dx/dV2[s]) volts n_seg / T for the switching segment s."""
    e1, e2 = electrodes
    v1, v2, s = switch_schedules(t_sw, volts, n_seg, T)
    sim.set_phase(phi0)
    sim.set_schedule(e1, v1, T)
    sim.set_schedule(e2, v2, T)
    sim.forward_checkpointed(T, K)
    x = float(sim.observables()["centroid"][axis])
    gx = np.zeros(3)
    gx[axis] = 1.0
    g1 = sim.adjoint(gx, np.zeros(3), e1, n_seg)
    g2 = sim.adjoint(gx, np.zeros(3), e2, n_seg)
    return x, (g1[s] - g2[s]) * volts * n_seg / T


def design_switch_time(sim, phi0, t_sw0, target, volts, n_seg, T, K, axis=0, electrodes=(0, 1), iters=6,
                       atol=1e-6, max_halvings=6):
    """Newton iteration on the switch time so that the droplet centroid reaches `target` at step
    T (the two-electrode protocols of the Results, Fig. 5b-c, one switch at a time), each step from
    switch_time_gradient, halved until |x - target| decreases.  Returns (t_sw, history)."""
    t = float(t_sw0)
    x, d = switch_time_gradient(sim, phi0, t, volts, n_seg, T, K, axis, electrodes)
    history = [dict(iteration=0, t_sw=t, residual=x - target, slope=d)]
    for k in range(1, iters + 1):
        r = x - target
        if abs(r) <= atol or d == 0.0:
            break
        step = -r / d
        for _ in range(max_halvings + 1):
            t_new = min(max(t + step, 0.0), T * (1.0 - 1e-9))
            x_new, d_new = switch_time_gradient(sim, phi0, t_new, volts, n_seg, T, K, axis, electrodes)
            if abs(x_new - target) < abs(r):
                break
            step *= 0.5
        else:
            break
        t, x, d = t_new, x_new, d_new
        history.append(dict(iteration=k, t_sw=t, residual=x - target, slope=d))
    return t, history


def relay_schedules(switch_times, volts, n_electrodes, t_total, seg_len):
    """Schedules of the long-distance protocol (Results, Fig. 5c): electrode k holds `volts` from
    switch k - 1 to switch k (the last one to the end) and floats otherwise (NaN: switched off,
    its faces insulate).  Segments of seg_len steps over t_total; a switch takes effect at the
    segment boundary nearest to it.  Returns (list of per-electrode arrays, switch steps used)."""
    n_seg = int(math.ceil(t_total / seg_len))
    edges = [int(round(t / seg_len)) for t in switch_times]
    bounds = [0] + edges + [n_seg]
    out = []
    for k in range(n_electrodes):
        v = np.full(n_seg, np.nan)
        if k < len(bounds) - 1:
            v[bounds[k]:bounds[k + 1]] = volts
        out.append(v)
    return out, [e * seg_len for e in edges]


def periodic_protocol(sim, x0, d, volts, n_switches, electrodes=(0, 1), chunk=250, max_steps=2_000_000, axis=0):
    """The two-electrode periodic motion of the Results (Fig. 5b), switched on the droplet's
    position: electrodes[0] holds `volts` (electrodes[1] floats) until the centroid passes
    x0 + d, then electrodes[1] holds it (electrodes[0] floats) until the centroid passes x0 - d,
    and so on for n_switches switches.  The centroid is read every `chunk` steps; a switch takes
    effect from the next step.  Returns dict(switch_steps, switch_positions, trajectory) with
    positions relative to x0 and the trajectory as (step, position) pairs.  Raises if the state
    turns non-finite or max_steps pass first."""
    if not (d > 0 and n_switches >= 1 and chunk >= 1 and electrodes[0] != electrodes[1]):
        raise ValueError("need d > 0, n_switches >= 1, chunk >= 1 and two distinct electrodes")
    e_a, e_b = electrodes
    on = 0

    def apply():
        sim.set_schedule(e_a, np.array([volts if on == 0 else np.nan]), 1)
        sim.set_schedule(e_b, np.array([volts if on == 1 else np.nan]), 1)

    apply()
    steps, pos, traj = [], [], []
    start = int(sim.observables()["step"])
    while len(steps) < n_switches:
        sim.step(chunk)
        ob = sim.observables(strict=False)
        if ob["status"] != 0:
            raise RuntimeError(f"status {ob['status']} at step {ob['step']}")
        x = float(ob["centroid"][axis]) - x0
        traj.append((int(ob["step"]), x))
        if (on == 0 and x >= d) or (on == 1 and x <= -d):
            steps.append(int(ob["step"]))
            pos.append(x)
            on = 1 - on
            apply()
        if ob["step"] - start >= max_steps:
            raise RuntimeError(f"{len(steps)} of {n_switches} switches after {max_steps} steps")
    return dict(switch_steps=steps, switch_positions=pos, trajectory=traj)
