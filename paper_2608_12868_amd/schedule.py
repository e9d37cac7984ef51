"""Electrode-voltage schedules designed with the adjoint: the programmable droplet manipulation
that the paper pursues with electrode switching protocols (Results, Fig. 5), posed as reaching a
target droplet position at a given time.

The residual r(V) = x_c(T; V)[axis] - x* of the droplet centroid after T steps is a scalar
function of the piecewise-constant schedule V of one electrode; its gradient J = dr/dV comes
from one checkpointed forward and one adjoint sweep.  Each iteration takes the minimum-norm step
of the linearised residual, r + J dV = 0, over the segments that are not held at a voltage bound
(projected Gauss-Newton), halving it until |r| decreases.  Host-side driver only: every forward
step and every adjoint step runs in the library.
"""
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
