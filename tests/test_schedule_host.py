"""Host logic of the adjoint-driven schedule design (paper_2608_12868_amd/schedule.py) against a
stand-in simulation whose centroid responds linearly to the schedule, x(V) = x0 + a . V, with the
exact gradient a: one projected Gauss-Newton step reaches an attainable target when no bound is
active; with bounds active the iterations stay feasible and the residual decreases to the best
the free segments allow."""
import numpy as np

from paper_2608_12868_amd.schedule import design_schedule


class LinearSim:
    def __init__(self, a, x0):
        self.a, self.x0 = np.asarray(a, float), float(x0)
        self.v = None
        self.forward_runs = 0

    def set_phase(self, phi):
        pass

    def set_schedule(self, electrode, volts, t_total):
        self.v = np.array(volts, float)

    def forward_checkpointed(self, T, K):
        self.forward_runs += 1

    def observables(self):
        return {"centroid": np.array([self.x0 + self.a @ self.v, 0.0, 0.0])}

    def adjoint(self, gx, gv, electrode, n_seg):
        return gx[0] * self.a


def test_one_step_without_active_bounds():
    rng = np.random.default_rng(0)
    a = rng.uniform(0.5, 1.5, 8)
    sim = LinearSim(a, 10.0)
    v0 = np.full(8, 0.04)
    target = 10.0 + a @ v0 + 0.01
    v, hist = design_schedule(sim, None, v0, 100, 10, 5, target, bounds=(0.0, 0.08), iters=5)
    assert abs(hist[-1]["residual"]) <= 1e-12
    assert len(hist) == 2 and hist[1]["adjoint"] == 1
    # the minimum-norm step is parallel to the gradient
    d = v - v0
    assert np.allclose(d / np.linalg.norm(d), a / np.linalg.norm(a))


def test_bounds_stay_feasible_and_residual_decreases():
    a = np.array([1.0, 1.0, 1.0, -1.0])
    sim = LinearSim(a, 0.0)
    v0 = np.array([0.08, 0.0, 0.04, 0.0])   # segment 0 at the upper bound, 3 at the lower
    target = a @ v0 + 0.03                   # needs +0.03 from segments that can still move up
    v, hist = design_schedule(sim, None, v0, 100, 10, 5, target, bounds=(0.0, 0.08), iters=6)
    assert np.all(v >= 0.0) and np.all(v <= 0.08)
    res = [abs(h["residual"]) for h in hist]
    assert all(b < a_ for a_, b in zip(res, res[1:]))
    assert res[-1] <= 1e-9
    assert v[0] == 0.08 and v[3] == 0.0       # segments at a bound in the step's direction stay


def test_stops_at_relative_tolerance():
    a = np.ones(4)
    sim = LinearSim(a, 0.0)
    v, hist = design_schedule(sim, None, np.full(4, 0.02), 100, 10, 5, a @ np.full(4, 0.02), iters=5)
    assert len(hist) == 1 and sim.forward_runs == 1   # already on target: no adjoint sweep


class PullSim:
    """Stand-in for the periodic protocol: the centroid moves at speed v towards whichever of
    electrodes 0 (ahead, +x) and 1 (behind) holds a finite voltage; a floating one (NaN) pulls
    nothing."""

    def __init__(self, v):
        self.v, self.x, self.t = float(v), 0.0, 0
        self.volts = {0: np.nan, 1: np.nan}

    def set_schedule(self, electrode, volts, t_total):
        assert len(volts) == 1 and t_total == 1
        self.volts[electrode] = float(volts[0])

    def step(self, n):
        sign = (0.0 if np.isnan(self.volts[0]) else 1.0) - (0.0 if np.isnan(self.volts[1]) else 1.0)
        self.x += sign * self.v * n
        self.t += n

    def observables(self, strict=True):
        return {"step": self.t, "centroid": np.array([self.x, 0.0, 0.0]), "status": 0}


def test_periodic_protocol_switches_on_position():
    from paper_2608_12868_amd.schedule import periodic_protocol
    sim = PullSim(2.0 ** -7)                  # 1 lu per chunk of 128 steps, exactly
    out = periodic_protocol(sim, 0.0, 4.0, 0.7, n_switches=4, chunk=128)
    # a first leg of 4 lu, then legs of 8 lu between the turning points
    assert out["switch_steps"] == [512, 1536, 2560, 3584]
    assert out["switch_positions"] == [4.0, -4.0, 4.0, -4.0]
    # one electrode holds the voltage at a time, the other floats
    assert sim.volts[0] == 0.7 and np.isnan(sim.volts[1])


def test_periodic_protocol_gives_up_after_max_steps():
    import pytest
    from paper_2608_12868_amd.schedule import periodic_protocol
    with pytest.raises(RuntimeError):
        periodic_protocol(PullSim(0.0), 0.0, 1.0, 0.7, n_switches=2, chunk=100, max_steps=1000)


def test_periodic_protocol_rejects_bad_arguments():
    import pytest
    from paper_2608_12868_amd.schedule import periodic_protocol
    for kw in (dict(d=0.0), dict(n_switches=0), dict(chunk=0), dict(electrodes=(1, 1))):
        args = dict(d=1.0, n_switches=2, chunk=100, electrodes=(0, 1))
        args.update(kw)
        with pytest.raises(ValueError):
            periodic_protocol(PullSim(1.0), 0.0, args["d"], 0.7, n_switches=args["n_switches"], chunk=args["chunk"],
                              electrodes=args["electrodes"])
