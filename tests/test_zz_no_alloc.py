"""The allocation-free observables entry point (library-held scratch) against ehdlb_observables,
through the C ABI: two calls in a row, the second on a smaller lattice, each equal bit for bit."""
import ctypes as C

import numpy as np
import pytest
import torch

from inputs import make_case

import gpu_util as gu

pytestmark = pytest.mark.gpu


def _device_obs(sim):
    from paper_2608_12868_amd import _lib as L
    out = torch.full((12,), float("nan"), dtype=torch.float64, device=sim.device)
    st = L.lib().ehdlb_observables_device(sim.h, C.c_void_p(out.data_ptr()))
    sim._chk(st)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def test_observables_device_matches_observables():
    from paper_2608_12868_amd import Simulation
    gu.require_gpu()
    # the second call runs on a smaller lattice (36,864 then 8,192 nodes) in the same scratch
    for name, precision, steps in (("c3s", "fp32", 9), ("c2s", "fp64", 5)):
        case = make_case(name, precision=precision)
        print("no-alloc observables", name, case.n, precision, steps, "steps", flush=True)
        sim = Simulation.from_case(case, precision=precision,
                                   poisson_tol=1e-13 if precision == "fp64" else 1e-5)
        sim.step(steps)
        d = _device_obs(sim)
        ref = sim.observables()
        expect = np.concatenate([ref["mass"], ref["centroid"], ref["velocity"],
                                 [ref["total_charge"], ref["sum_phi_drift"], 0.0]])
        print("  device", d, flush=True)
        assert np.array_equal(d, expect)
        del sim


def test_observables_device_rejects_bad_output():
    from paper_2608_12868_amd import Simulation, _lib as L
    gu.require_gpu()
    case = make_case("c1s", precision="fp64")
    sim = Simulation.from_case(case)
    assert L.lib().ehdlb_observables_device(sim.h, None) == L.EINVAL
