"""Failure reporting through the C ABI (finite data paths only; every kernel exits normally).

ENONFINITE: a NaN in the initial phase fields propagates through the step; the observables'
FP64 reduction counts non-finite values and the sticky flag is reported.
ENOCONV: a potential solve capped at one iteration with a tolerance it cannot reach in one.
ESTATE: anything that changes the state or the schedule between the checkpointed forward and
the adjoint (the forward generation counter), also through the autograd boundary.
"""
import numpy as np
import pytest
import torch

from inputs import make_case

import gpu_util as gu

pytestmark = pytest.mark.gpu


def _sim(case, precision="fp64", **over):
    from paper_2608_12868_amd import Simulation
    gu.require_gpu()
    return Simulation.from_case(case, precision=precision, **over)


def test_nonfinite_phase_is_reported():
    from paper_2608_12868_amd import _lib as L
    case = make_case("c2s", precision="fp64")
    sim = _sim(case)
    phi = case.phi.copy()
    fluid = np.flatnonzero(case.flags == 0)
    node = int(fluid[len(fluid) // 2])
    phi[0, node] = np.nan
    print("NaN at node", node, "of c2s", case.n, flush=True)
    sim.set_phase(phi)
    sim.step(3)
    ob = sim.observables(strict=False)
    assert ob["status"] == L.ENONFINITE
    assert ob["flags"] & 1
    with pytest.raises(L.EhdlbError):
        sim.observables()
    # a fresh start clears the sticky flag
    sim.set_phase(case.phi)
    sim.step(3)
    ob = sim.observables(strict=False)
    assert ob["status"] == L.OK and ob["flags"] == 0


def test_iteration_cap_is_reported():
    from paper_2608_12868_amd import _lib as L
    case = make_case("c2s", precision="fp64")
    sim = _sim(case, poisson_max_iter=1, poisson_tol=1e-15)
    print("c2s with poisson_max_iter = 1, tol = 1e-15", flush=True)
    sim.step(2)
    ob = sim.observables(strict=False)
    assert ob["status"] == L.ENOCONV
    assert ob["flags"] & 2 and not ob["flags"] & 1
    assert ob["poisson_iters"] == 1 and ob["poisson_residual"] > 1e-15


@pytest.mark.parametrize("change", ["set_schedule", "step", "set_solver_options", "set_phase",
                                    "forward_again"])
def test_adjoint_rejects_changed_forward(change):
    from paper_2608_12868_amd import _lib as L
    case = make_case("c4s", precision="fp64")
    sim = _sim(case)
    T = 12
    sim.set_schedule(0, case.schedule, T)
    print("c4s forward_checkpointed then", change, flush=True)
    sim.forward_checkpointed(T, 5)
    g0 = sim.adjoint([1.0, 0, 0], [0, 0, 0], 0, len(case.schedule))
    # the adjoint itself leaves the forward intact: a second call gives the same gradient
    assert np.array_equal(g0, sim.adjoint([1.0, 0, 0], [0, 0, 0], 0, len(case.schedule)))
    if change == "set_schedule":
        sim.set_schedule(0, case.schedule * 0.5, T)
    elif change == "step":
        sim.step(1)
    elif change == "set_solver_options":
        sim.set_solver_options(warm_start=1)
    elif change == "set_phase":
        sim.set_phase(case.phi)
    else:
        sim.forward_checkpointed(T, 5)
        g1 = sim.adjoint([1.0, 0, 0], [0, 0, 0], 0, len(case.schedule))
        assert np.all(np.isfinite(g1))
        return
    with pytest.raises(L.EhdlbError) as ei:
        sim.adjoint([1.0, 0, 0], [0, 0, 0], 0, len(case.schedule))
    assert ei.value.status == L.ESTATE


def test_autograd_backward_rejects_reused_simulation():
    from paper_2608_12868_amd.autograd import schedule_to_observables
    case = make_case("c4s", precision="fp64")
    sim = _sim(case)
    T = 12
    v1 = torch.tensor(case.schedule, dtype=torch.float64, requires_grad=True)
    xc1, _ = schedule_to_observables(v1, sim, case.phi, T, 5, T)
    v2 = torch.tensor(case.schedule * 0.5, dtype=torch.float64, requires_grad=True)
    xc2, _ = schedule_to_observables(v2, sim, case.phi, T, 5, T)
    xc2[0].backward()                   # the latest forward: fine
    assert v2.grad is not None and torch.all(torch.isfinite(v2.grad))
    with pytest.raises(RuntimeError):
        xc1[0].backward()               # its checkpoints were overwritten by the second forward
