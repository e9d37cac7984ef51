"""HIP path against the FP64 oracle, element by element, through the C ABI.

Tolerances: FP64 path <= 1e-10 relative (max-norm over the field, per field);
FP32-deviation path <= 1e-4 relative on the droplet centroid trajectory.
"""
import numpy as np
import pytest

from inputs import make_case

import gpu_util as gu

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-10


def _gpu(case, precision=None, **over):
    from paper_2608_12868_amd import Simulation
    gu.require_gpu()
    return Simulation.from_case(case, precision=precision, **over)


def _compare(sim, o, s, aux, tol, fields=None):
    ref = gu.oracle_fields(o, s, aux)
    errs = {}
    for k, v in ref.items():
        if fields and k not in fields:
            continue
        errs[k] = gu.rel_err(sim.field(k), v)
    print({k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    bad = {k: v for k, v in errs.items() if not v <= tol}
    assert not bad, bad
    return errs


@pytest.mark.parametrize("name,steps", [("c1s", 300), ("c2s", 150), ("c4s", 150)])
def test_fp64_parity_2d(name, steps):
    case = make_case(name, precision="fp64")
    print("case", name, case.n, "steps", steps, flush=True)
    sim = _gpu(case)
    sim.step(steps)
    o, s, aux = gu.oracle_run(case, steps)
    _compare(sim, o, s, aux, FP64_TOL)
    pops = sim.field("pops")
    assert gu.rel_err(pops, gu.oracle_pops(o, s)) <= FP64_TOL


def test_fp64_parity_config1_full():
    """The 128x64 flat-film configuration at its full 1000 steps."""
    case = make_case("c1")
    sim = _gpu(case)
    sim.step(case.steps)
    o, s, aux = gu.oracle_run(case, case.steps)
    _compare(sim, o, s, aux, FP64_TOL)
    ob = sim.observables()
    ref = o.observables(s)
    assert np.allclose(ob["mass"], ref["mass"].numpy(), rtol=1e-12, atol=0)
    assert np.allclose(ob["centroid"], ref["centroid"].numpy(), rtol=1e-12, atol=1e-12)
    assert np.allclose(ob["velocity"], ref["velocity"].numpy(), rtol=1e-9, atol=1e-15)


def test_fp64_parity_3d():
    case = make_case("c3s", precision="fp64")
    sim = _gpu(case)
    steps = 12
    sim.step(steps)
    o, s, aux = gu.oracle_run(case, steps)
    _compare(sim, o, s, aux, FP64_TOL)


def test_fp64_parity_variable_viscosity_and_schedule():
    """Per-phase tau (second-order moments away from equilibrium) and a voltage schedule."""
    case = make_case("c4s", precision="fp64")
    over = dict(tau_flow=(0.8, 1.3, 0.65))
    sim = _gpu(case, **over)
    sim.set_schedule(0, case.schedule, case.t_total)
    steps = 120
    sim.step(steps)
    nseg = len(case.schedule)

    def volts(t):
        import torch
        seg = min(t * nseg // case.t_total, nseg - 1)
        return torch.tensor([case.schedule[seg], 0, 0, 0], dtype=torch.float64)
    o, s, aux = gu.oracle_run(case, steps, params=over, volts_fn=volts)
    _compare(sim, o, s, aux, FP64_TOL)


def test_fp32_centroid_trajectory():
    case = make_case("c2s")
    sim = _gpu(case, precision="fp32", poisson_tol=1e-5)
    from oracle import Oracle
    o = Oracle(case.dim, case.n, case.periodic, case.params, case.flags)
    s = o.init_state(case.phi)
    x0 = o.observables(s)["centroid"].numpy()
    worst = 0.0
    for k in range(6):
        sim.step(50)
        s, _ = o.run(s, 50)
        xg = sim.observables()["centroid"]
        xo = o.observables(s)["centroid"].numpy()
        worst = max(worst, float(np.abs(xg[:2] - xo[:2]).max() / np.abs(xo[:2]).max()))
    print("fp32 centroid rel err", worst, "displacement", xo - x0, flush=True)
    assert worst <= 1e-4


@pytest.mark.parametrize("name,precision,save_at,warm", [("c2s", "fp64", 20, 2), ("c3s", "fp32", 2, 2),
                                                         ("c3s", "fp32", 20, 3), ("c3s", "fp32", 20, 1),
                                                         ("c2s", "fp64", 20, 0), ("c3s", "fp32", 20, 4)])
def test_determinism_and_checkpoint_replay(name, precision, save_at, warm):
    """Two runs agree bit for bit, and so does a replay from a saved state: the potentials that the
    warm starts use (the last four for the projection, t = 2 leaves a partial history) are part
    of the state."""
    case = make_case(name, precision=precision)
    a = _gpu(case, precision)
    a.set_solver_options(warm_start=warm)
    a.step(save_at)
    blob = a.save_state()
    a.step(30)
    pa = a.field("pops")
    b = _gpu(case, precision)
    b.set_solver_options(warm_start=warm)
    b.step(save_at + 30)
    assert np.array_equal(pa, b.field("pops")), "two runs differ"
    b.load_state(blob)
    b.step(30)
    assert np.array_equal(pa, b.field("pops")), "replay from checkpoint differs"
    assert b.observables()["step"] == save_at + 30


def test_mass_conservation_config2_full():
    case = make_case("c2")
    sim = _gpu(case)
    m0 = sim.observables()["mass"]
    sim.step(200)
    ob = sim.observables()
    assert np.all(np.abs(ob["mass"] - m0) / m0 <= 1e-12)
    assert ob["poisson_residual"] <= case.params["poisson_tol"]


# ---------------------------------------------------------------- edge cases
def _droplet_case(n, periodic, radius, volts=0.05, electrode=True):
    """Droplet of phase 1 in phase 3 on a grounded bottom wall, insulating top wall with an
    electrode patch (odd sizes allowed); the field on."""
    from inputs import default_params
    from inputs.presets import ELECTRODE0, GROUND, NEUMANN, FLUID
    import pin_cases as pc
    dim = 3 if n[2] > 1 else 2
    x, y, z = pc.grid(n)
    h = z if dim == 3 else y
    top = n[dim - 1] - 1
    flags = np.zeros(x.size, np.uint8)
    flags[h == 0] = GROUND
    flags[h == top] = NEUMANN
    if electrode:
        patch = (h == top) & (x >= n[0] // 2) & (x < n[0] // 2 + max(4, n[0] // 4))
        flags[patch] = ELECTRODE0
    cx = n[0] / 3.0
    r2 = (x - cx) ** 2 + (h - 0.5) ** 2
    if dim == 3:
        r2 = r2 + (y - n[1] / 2.0) ** 2
    p1 = 0.5 * (1 + np.tanh(2 * (radius - np.sqrt(r2)) / 4.0))
    phi = np.stack([p1, np.zeros_like(p1), 1 - p1])
    phi[:, flags != FLUID] = 0
    params = default_params(dim, ehd=1, electrode_volts=(volts, 0.0, 0.0, 0.0), charge_diffusion=1e-3)
    return dim, n, periodic, params, flags, phi


def _run_pair(dim, n, periodic, params, flags, phi, steps):
    from paper_2608_12868_amd import Simulation
    from oracle import Oracle
    gu.require_gpu()
    sim = Simulation(dim, n, periodic, "fp64", params, flags, phi)
    sim.step(steps)
    o = Oracle(dim, n, periodic, params, flags)
    s = o.init_state(phi)
    aux = None
    for _ in range(steps):
        s, aux = o.step(s)
    return sim, o, s, aux


@pytest.mark.parametrize("n,periodic", [((75, 41, 1), (1, 0, 0)), ((29, 23, 19), (1, 1, 0)),
                                        ((40, 24, 1), (1, 0, 0))])
def test_fp64_parity_ragged_sizes(n, periodic):
    """Odd and non-tile-multiple lattice sizes (partial aggregates and tiles on every multigrid
    level); 40x24 keeps the whole hierarchy in the single-workgroup tail."""
    case = _droplet_case(n, periodic, radius=min(n[0], n[-1] if n[2] > 1 else n[1]) / 3.0)
    print("ragged", n, flush=True)
    sim, o, s, aux = _run_pair(*case, steps=40)
    _compare(sim, o, s, aux, FP64_TOL)


def test_fp64_zero_potential():
    """Field on with every electrode at 0 V and no charge: the Gauss law's right-hand side
    vanishes, the potential is exactly zero and no iteration runs."""
    case = _droplet_case((64, 36, 1), (1, 0, 0), radius=10.0, volts=0.0)
    sim, o, s, aux = _run_pair(*case, steps=20)
    assert np.all(sim.field("pot") == 0.0)
    ob = sim.observables()
    assert ob["poisson_iters"] == 0 and ob["poisson_residual"] == 0.0
    _compare(sim, o, s, aux, FP64_TOL)


@pytest.mark.parametrize("n", [(64, 36, 1), (24, 20, 16)])
def test_fp64_parity_without_droplet(n):
    """The degenerate two-phase state of the ternary model: no droplet (Phi_1 = 0 everywhere), a
    lubricant film under the ambient, the field on (in 3D uniform along y).  Fields against the oracle, and the
    observables against the oracle's: the droplet mass, and a centroid that is undefined (NaN)
    exactly when that mass is zero."""
    import pin_cases as pc
    from oracle import Oracle
    dim, n, periodic, params, flags, _ = _droplet_case(n, (1, 0, 0) if n[2] == 1 else (1, 1, 0), radius=1.0)
    x, y, z = pc.grid(n)
    h = z if dim == 3 else y
    p2 = 0.5 * (1 + np.tanh(2 * (4.5 - h) / 4.0))
    phi = np.stack([np.zeros_like(p2), p2, 1 - p2])
    phi[:, flags != 0] = 0
    print("no droplet", n, flush=True)
    sim, o, s, aux = _run_pair(dim, n, periodic, params, flags, phi, steps=30)
    # in 3D the state is uniform along y, so u_y is rounding noise on both sides: the velocity
    # components are compared against the largest of them
    ref = gu.oracle_fields(o, s, aux)
    uscale = max(np.abs(ref[k]).max() for k in ("ux", "uy", "uz") if k in ref)
    errs = {}
    for k, v in ref.items():
        den = uscale if k in ("ux", "uy", "uz") else max(np.abs(v).max(), 1e-300)
        errs[k] = float(np.abs(sim.field(k) - v).max() / den)
    print({k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    assert max(errs.values()) <= FP64_TOL, errs
    ob = sim.observables(strict=False)
    ref = o.observables(s)
    m1 = float(ref["mass"][0])
    print("droplet mass", ob["mass"][0], m1, "centroid", ob["centroid"], flush=True)
    assert ob["status"] == 0
    assert abs(ob["mass"][0] - m1) <= 1e-12
    if m1 == 0.0:
        assert ob["mass"][0] == 0.0 and np.all(np.isnan(ob["centroid"]))
    else:
        assert np.allclose(ob["centroid"], ref["centroid"].numpy(), rtol=1e-10, atol=1e-10)
    assert np.allclose(ob["mass"][1:], ref["mass"].numpy()[1:], rtol=1e-12)


def test_zero_steps_change_nothing():
    """step(0) leaves the state, the step counter and the forward generation unchanged."""
    case = make_case("c2s", precision="fp64")
    sim = _gpu(case, "fp64")
    sim.step(3)

    def state():
        buf = sim.save_state()
        off = (-buf.data_ptr()) % 256          # save_state writes at the first 256-byte boundary
        return buf[off:off + sim.state_bytes].clone()

    ob0 = sim.observables()
    g0, st0 = sim.generation, state()
    sim.step(0)
    assert sim.generation == g0
    assert bool((state() == st0).all())
    ob1 = sim.observables()
    assert ob1["step"] == ob0["step"] == 3
    assert np.array_equal(ob1["centroid"], ob0["centroid"])


@pytest.mark.parametrize("name,steps,s_high", [("c2s", 120, 1.3), ("c3s", 10, 0.8)])
def test_fp64_parity_higher_moment_rate(name, steps, s_high):
    """The higher raw moments away from rate 1 (s_high: orders >= 2 of the phase fields and the
    charge, >= 3 of the flow), with per-phase viscosities: fields and populations."""
    case = make_case(name, precision="fp64")
    over = dict(s_high=s_high, tau_flow=(0.8, 1.3, 0.65))
    print("case", name, case.n, "steps", steps, "s_high", s_high, flush=True)
    sim = _gpu(case, **over)
    sim.step(steps)
    o, s, aux = gu.oracle_run(case, steps, params=over)
    _compare(sim, o, s, aux, FP64_TOL)
    assert gu.rel_err(sim.field("pops"), gu.oracle_pops(o, s)) <= FP64_TOL


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_read_field_to_device_memory(precision):
    """Every field read into device memory equals the host read-out bit for bit (after an odd
    number of steps, when the velocity and Ohmic source come from the slots the first step
    writes; their solid nodes read as zero)."""
    import torch
    from paper_2608_12868_amd import _lib as L
    case = make_case("c2s", precision=precision)
    sim = _gpu(case, precision=precision, poisson_tol=1e-13 if precision == "fp64" else 1e-5)
    sim.step(7)
    for name in L.FIELDS:
        host = sim.field(name)
        if name != "pops":
            assert np.all(host[case.flags != 0] == 0.0), name
        dev = sim.field(name, device=True)
        torch.cuda.synchronize()
        assert dev.device.type == "cuda" and dev.dtype == torch.float64
        assert np.array_equal(dev.cpu().numpy(), host), name


@pytest.mark.parametrize("name,steps,rho", [("c2s", 100, (5.0, 2.0, 1.0)), ("c3s", 8, (0.5, 0.8, 1.0))])
def test_fp64_parity_variable_density(name, steps, rho):
    """Unequal phase densities (the velocity-based flow with the pressure and viscous
    density-gradient forces) with per-phase viscosities: fields and populations."""
    case = make_case(name, precision="fp64")
    over = dict(rho=rho, tau_flow=(0.8, 1.3, 0.65))
    print("case", name, case.n, "steps", steps, "densities", rho, flush=True)
    sim = _gpu(case, **over)
    sim.step(steps)
    o, s, aux = gu.oracle_run(case, steps, params=over)
    _compare(sim, o, s, aux, FP64_TOL)
    assert gu.rel_err(sim.field("pops"), gu.oracle_pops(o, s)) <= FP64_TOL


def test_paper_regime_densities_and_viscosities():
    """The paper's Table 1 fluids on the 128x64 EHD case: densities 998 : 970 : 1.2 and dynamic
    viscosities 1 : 0.5 : 0.0179 (water, oil, air; kinematic 0.01, 0.0051, 0.149 lu), FP64 against
    the oracle over 40 steps, and 2000 steps of the FP32 path stay finite with every phase's mass
    conserved."""
    case = make_case("c2s", precision="fp64")
    rho = (1.0, 970.0 / 998.0, 1.2 / 998.0)
    nu = (0.01, 0.01 * 0.5 / rho[1], 0.01 * 0.0179 / rho[2])
    over = dict(rho=rho, tau_flow=tuple(0.5 + 3.0 * v for v in nu))
    print("c2s with Table 1 densities", rho, "taus", over["tau_flow"], flush=True)
    sim = _gpu(case, **over)
    sim.step(40)
    o, s, aux = gu.oracle_run(case, 40, params=over)
    _compare(sim, o, s, aux, FP64_TOL)
    sim32 = _gpu(make_case("c2s"), precision="fp32", poisson_tol=1e-5, **over)
    m0 = sim32.observables()["mass"]
    sim32.step(2000)
    ob = sim32.observables()
    print("  FP32 after 2000 steps: mass drift", (ob["mass"] - m0) / m0, "velocity", ob["velocity"], flush=True)
    assert ob["flags"] == 0
    assert np.all(np.abs(ob["mass"] - m0) / m0 <= 2000 * 9 * 2.0 ** -24)


def test_fp64_parity_cloaking_tensions():
    """gamma13 > gamma12 + gamma23 (Upsilon_2 < 0, the lubricant cloaks the droplet)."""
    case = make_case("c2s", precision="fp64")
    over = dict(gamma12=1e-3, gamma13=2.5e-3, gamma23=1e-3)
    sim = _gpu(case, **over)
    sim.step(100)
    o, s, aux = gu.oracle_run(case, 100, params=over)
    _compare(sim, o, s, aux, FP64_TOL)


def _two_electrodes(case, second=None):
    """c2s/c3s geometry with a second electrode on the top wall behind the droplet (flag
    `second`, default electrode 1)."""
    from inputs.presets import ELECTRODE0
    n = case.n
    f = case.flags.copy()
    if case.dim == 2:
        f = f.reshape(n[1], n[0])
        f[n[1] - 1, 2:22] = ELECTRODE0 + 1 if second is None else second
    else:
        f = f.reshape(n[2], n[1], n[0])
        f[n[2] - 1, :, 1:7] = ELECTRODE0 + 1 if second is None else second
    return f.reshape(-1)


@pytest.mark.parametrize("name,steps", [("c2s", 60), ("c3s", 6)])
def test_fp64_parity_floating_electrode(name, steps):
    """An electrode switched off and floating (NaN in its schedule): electrode 1 is on, floating,
    then on again while electrode 0 holds its voltage; fields against the oracle."""
    import torch
    from oracle import Oracle
    case = make_case(name, precision="fp64")
    fl = _two_electrodes(case)
    sched = np.array([0.04, np.nan, 0.06])
    sim = _gpu(case)
    sim.set_geometry(fl)
    sim.set_phase(case.phi)
    sim.set_schedule(1, sched, steps)
    sim.step(steps)
    V = case.params["electrode_volts"][0]
    o = Oracle(case.dim, case.n, case.periodic, case.params, fl)
    s = o.init_state(case.phi)
    aux = None
    for t in range(steps):
        seg = min(t * 3 // steps, 2)
        s, aux = o.step(s, torch.tensor([V, sched[seg], 0.0, 0.0], dtype=torch.float64))
    print("case", name, case.n, "steps", steps, "electrode 1 schedule", sched, flush=True)
    _compare(sim, o, s, aux, FP64_TOL)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_floating_electrode_equals_insulating_wall(precision):
    """A floating electrode and an insulating wall in its place give the same bits."""
    from inputs.presets import NEUMANN
    case = make_case("c2s", precision=precision)
    out = []
    for fl, v1 in ((_two_electrodes(case), np.nan), (_two_electrodes(case, NEUMANN), 0.0)):
        sim = _gpu(case, precision, poisson_tol=1e-13 if precision == "fp64" else 1e-5)
        sim.set_geometry(fl)
        sim.set_phase(case.phi)
        sim.set_schedule(1, np.array([v1]), 1)
        sim.step(40)
        out.append(sim.field("pops"))
    print("c2s", precision, "floating vs insulating: max |diff|", np.abs(out[0] - out[1]).max(), flush=True)
    assert np.array_equal(out[0], out[1])
