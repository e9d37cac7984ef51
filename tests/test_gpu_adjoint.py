"""Hand-written GPU adjoint of the coupled step (checkpoint + recompute) through the C ABI.

Checked against (1) reverse-mode autograd through the FP64 oracle, (2) central finite
differences of the GPU FP64 forward with h = 1e-4, (3) its own invariance to the
checkpoint interval, (4) the torch.autograd boundary.
"""
import numpy as np
import pytest
import torch

from inputs import make_case

import gpu_util as gu

pytestmark = pytest.mark.gpu

GX = np.array([1.0, 0.3, 0.0])      # dL/d(centroid)
GV = np.array([40.0, -25.0, 0.0])   # dL/d(velocity)


def _sim(case, precision="fp64", **over):
    from paper_2608_12868_amd import Simulation
    gu.require_gpu()
    return Simulation.from_case(case, precision=precision, **over)


def _gpu_grad(case, sched, T, t_total, K, precision="fp64", **over):
    sim = _sim(case, precision, **over)
    sim.set_schedule(0, sched, t_total)
    sim.forward_checkpointed(T, K)
    ob = sim.observables()
    g = sim.adjoint(GX, GV, 0, len(sched))
    return g, ob


def _loss(ob):
    return float(GX @ ob["centroid"] + GV @ ob["velocity"])


def test_adjoint_matches_oracle_autograd():
    from oracle import Oracle
    from oracle.adjoint import schedule_gradient
    case = make_case("c4s", precision="fp64")
    sched = case.schedule.copy()
    T = 24
    t_total = 24
    print("case c4s", case.n, "T", T, "segments", len(sched), flush=True)
    g_gpu, ob = _gpu_grad(case, sched, T, t_total, K=7)        # ragged last segment
    o = Oracle(case.dim, case.n, case.periodic, case.params, case.flags)
    g_ref, xc, vc = schedule_gradient(o, case.phi, sched, T, t_total, GX, GV)
    g_ref = g_ref.numpy()
    err = np.abs(g_gpu - g_ref).max() / np.abs(g_ref).max()
    print("adjoint vs oracle autograd", err, g_gpu, g_ref, flush=True)
    assert np.allclose(ob["centroid"], xc.numpy(), rtol=1e-12, atol=1e-12)
    assert err <= 1e-8


def test_adjoint_matches_finite_differences():
    case = make_case("c4s", precision="fp64")
    n_seg = 4
    sched = np.random.default_rng(3).uniform(0.0, 0.08, n_seg)
    T = t_total = 80
    g, ob = _gpu_grad(case, sched, T, t_total, K=20)
    h = 1e-4
    fd = np.zeros(n_seg)
    sim = _sim(case)
    for k in range(n_seg):
        vals = []
        for sgn in (1, -1):
            v = sched.copy()
            v[k] += sgn * h
            sim.set_phase(case.phi)
            sim.set_schedule(0, v, t_total)
            sim.step(T)
            vals.append(_loss(sim.observables()))
        fd[k] = (vals[0] - vals[1]) / (2 * h)
    err = np.abs(g - fd).max() / np.abs(fd).max()
    print("adjoint vs central FD", err, g, fd, flush=True)
    assert err <= 1e-4


def test_adjoint_independent_of_checkpoint_interval():
    case = make_case("c4s", precision="fp64")
    sched = case.schedule.copy()
    T = t_total = 30
    g1, _ = _gpu_grad(case, sched, T, t_total, K=30)
    g2, _ = _gpu_grad(case, sched, T, t_total, K=4)
    assert np.array_equal(g1, g2)


def test_autograd_function_and_fp32():
    from paper_2608_12868_amd.autograd import schedule_to_observables
    case = make_case("c4s")
    T = t_total = 40
    sched = torch.tensor(case.schedule, dtype=torch.float64, requires_grad=True)
    target = 31.0
    grads = {}
    for prec in ("fp64", "fp32"):
        sim = _sim(case, prec, poisson_tol=1e-13 if prec == "fp64" else 1e-5)
        v = sched.detach().clone().requires_grad_(True)
        xc, vc = schedule_to_observables(v, sim, case.phi, T, 10, t_total)
        loss = (xc[0] - target) ** 2
        loss.backward()
        grads[prec] = v.grad.numpy().copy()
        assert np.all(np.isfinite(grads[prec]))
    rel = np.abs(grads["fp32"] - grads["fp64"]).max() / np.abs(grads["fp64"]).max()
    print("fp32 vs fp64 adjoint", rel, flush=True)
    assert rel <= 1e-2


def test_adjoint_checkpoint_invariance_with_extrapolated_warm_start():
    """The potential history used by the extrapolated warm start is part of the saved state:
    the recompute from any checkpoint interval reproduces the same gradient bit for bit."""
    case = make_case("c4s", precision="fp64")
    sched = case.schedule.copy()
    T = t_total = 30
    out = []
    for K in (30, 4):
        sim = _sim(case)
        sim.set_solver_options(warm_start=1)
        sim.set_schedule(0, sched, t_total)
        sim.forward_checkpointed(T, K)
        out.append(sim.adjoint(GX, GV, 0, len(sched)))
    assert np.array_equal(out[0], out[1])


def test_adjoint_higher_moment_rate_matches_oracle_autograd():
    """s_high != 1: the reverse collision with every equilibrium and source term rescaled and the
    direct (1 - s_high) share of the streamed population cotangents."""
    from oracle import Oracle
    from oracle.adjoint import schedule_gradient
    case = make_case("c4s", precision="fp64")
    over = dict(s_high=1.3, tau_flow=(0.8, 1.3, 0.65))
    sched = case.schedule.copy()
    T = t_total = 24
    print("case c4s", case.n, "T", T, "s_high 1.3", flush=True)
    g_gpu, ob = _gpu_grad(case, sched, T, t_total, K=7, **over)
    p = dict(case.params)
    p.update(over)
    o = Oracle(case.dim, case.n, case.periodic, p, case.flags)
    g_ref, xc, vc = schedule_gradient(o, case.phi, sched, T, t_total, GX, GV)
    g_ref = g_ref.numpy()
    err = np.abs(g_gpu - g_ref).max() / np.abs(g_ref).max()
    print("adjoint (s_high 1.3) vs oracle autograd", err, flush=True)
    assert np.allclose(ob["centroid"], xc.numpy(), rtol=1e-12, atol=1e-12)
    assert err <= 1e-8


def test_adjoint_cloaking_tensions_matches_oracle_autograd():
    """Upsilon_2 < 0 (gamma13 > gamma12 + gamma23): the reverse of the chemical potentials."""
    from oracle import Oracle
    from oracle.adjoint import schedule_gradient
    case = make_case("c4s", precision="fp64")
    over = dict(gamma12=1e-3, gamma13=2.5e-3, gamma23=1e-3)
    sched = case.schedule.copy()
    T = t_total = 16
    g_gpu, ob = _gpu_grad(case, sched, T, t_total, K=5, **over)
    p = dict(case.params)
    p.update(over)
    o = Oracle(case.dim, case.n, case.periodic, p, case.flags)
    g_ref, xc, vc = schedule_gradient(o, case.phi, sched, T, t_total, GX, GV)
    err = np.abs(g_gpu - g_ref.numpy()).max() / np.abs(g_ref.numpy()).max()
    print("adjoint (cloaking tensions) vs oracle autograd", err, flush=True)
    assert err <= 1e-8


def test_default_warm_start_differentiates_the_iterated_forward():
    """With the default forward warm start (4), plain steps keep a projected start that meets the
    tolerance, while the checkpointed forward and the adjoint's recompute iterate at least once
    (mode 2): the FP32 gradient equals mode 2's bit for bit, and the plain forward's centroid
    agrees with the checkpointed one to the FP32 solve's tolerance."""
    case = make_case("c4s")
    sched = case.schedule.copy()
    T = t_total = 60
    g, x = {}, {}
    for warm in (4, 2):
        sim = _sim(case, "fp32", poisson_tol=1e-5)
        sim.set_solver_options(warm_start=warm)
        sim.set_schedule(0, sched, t_total)
        sim.forward_checkpointed(T, 10)
        x[warm] = sim.observables()["centroid"]
        g[warm] = sim.adjoint(GX, GV, 0, len(sched))
        if warm == 4:
            sim.set_phase(case.phi)
            sim.solver_stats(reset=True)
            sim.step(T)
            x["plain"] = sim.observables()["centroid"]
            it_plain = sim.solver_stats()["forward"]["iters"]
    print("c4s fp32 T", T, "plain forward iterations", it_plain, "centroids", x, flush=True)
    assert np.array_equal(g[4], g[2])
    assert np.array_equal(x[4], x[2])
    assert np.allclose(x["plain"], x[4], rtol=1e-5, atol=0)


def test_adjoint_with_floating_segment_matches_oracle_autograd():
    """Electrode 1 on, floating (NaN), on: the reverse sweep treats its faces as insulating in
    the floating segment (dL/dV = 0 there) and as Dirichlet elsewhere."""
    from inputs.presets import ELECTRODE0
    from oracle import Oracle
    from oracle.adjoint import schedule_gradient
    case = make_case("c4s", precision="fp64")
    n = case.n
    fl = case.flags.copy().reshape(n[1], n[0])
    fl[n[1] - 1, 2:18] = ELECTRODE0 + 1
    fl = fl.reshape(-1)
    sched = np.array([0.04, np.nan, 0.06])
    T = t_total = 18
    sim = _sim(case)
    sim.set_geometry(fl)
    sim.set_phase(case.phi)
    sim.set_schedule(1, sched, t_total)
    sim.forward_checkpointed(T, 5)
    g = sim.adjoint(GX, GV, 1, len(sched))
    o = Oracle(case.dim, case.n, case.periodic, case.params, fl)
    g_ref, _, _ = schedule_gradient(o, case.phi, sched, T, t_total, GX, GV, electrode=1)
    g_ref = g_ref.numpy()
    err = np.abs(g - g_ref).max() / np.abs(g_ref).max()
    print("adjoint with a floating segment vs oracle autograd", err, g, g_ref, flush=True)
    assert g[1] == 0.0 and g_ref[1] == 0.0
    assert err <= 1e-8


@pytest.mark.parametrize("name,rho,T,K", [("c4s", (5.0, 2.0, 1.0), 24, 7), ("c4s", (0.5, 0.8, 1.0), 24, 5),
                                          ("c3s", (5.0, 2.0, 1.0), 8, 3)])
def test_adjoint_variable_density_matches_oracle_autograd(name, rho, T, K):
    """Unequal phase densities (Eq. 9 with rho(Phi), the velocity-based form): the reverse of the
    acceleration F/rho, of the pressure force -cs2 p* grad rho and of the viscous force from the
    provisional collision's second moments, against the oracle's autograd through the same
    step, in 2D and 3D, with per-phase viscosities."""
    from oracle import Oracle
    from oracle.adjoint import schedule_gradient
    case = make_case(name, precision="fp64")
    over = dict(rho=rho, tau_flow=(0.8, 1.3, 0.65))
    sched = np.array([0.03, 0.08, 0.05]) if name == "c3s" else case.schedule.copy()
    t_total = T
    print("case", name, case.n, "densities", rho, "T", T, "K", K, flush=True)
    sim = _sim(case, **over)
    sim.set_schedule(0, sched, t_total)
    sim.forward_checkpointed(T, K)
    ob = sim.observables()
    g = sim.adjoint(GX, GV, 0, len(sched))
    p = dict(case.params)
    p.update(over)
    o = Oracle(case.dim, case.n, case.periodic, p, case.flags)
    g_ref, xc, vc = schedule_gradient(o, case.phi, sched, T, t_total, GX, GV)
    g_ref = g_ref.numpy()
    err = np.abs(g - g_ref).max() / np.abs(g_ref).max()
    print("adjoint (unequal densities) vs oracle autograd", err, g, g_ref, flush=True)
    assert np.allclose(ob["centroid"], xc.numpy(), rtol=1e-12, atol=1e-12)
    assert err <= 1e-8


def test_adjoint_paper_regime_fluids_matches_oracle_autograd():
    """The paper's Table 1 fluids (densities 998 : 970 : 1.2, dynamic viscosities 1 : 0.5 :
    0.0179, so a density ratio of 830 between droplet and ambient): the variable-density
    adjoint against the oracle's autograd on the 96x48 schedule case."""
    from oracle import Oracle
    from oracle.adjoint import schedule_gradient
    case = make_case("c4s", precision="fp64")
    rho = (1.0, 970.0 / 998.0, 1.2 / 998.0)
    nu = (0.01, 0.01 * 0.5 / rho[1], 0.01 * 0.0179 / rho[2])
    over = dict(rho=rho, tau_flow=tuple(0.5 + 3.0 * v for v in nu))
    sched = case.schedule.copy()
    T = t_total = 24
    print("case c4s, Table 1 fluids", rho, "T", T, flush=True)
    sim = _sim(case, **over)
    sim.set_schedule(0, sched, t_total)
    sim.forward_checkpointed(T, 7)
    g = sim.adjoint(GX, GV, 0, len(sched))
    p = dict(case.params)
    p.update(over)
    o = Oracle(case.dim, case.n, case.periodic, p, case.flags)
    g_ref, _, _ = schedule_gradient(o, case.phi, sched, T, t_total, GX, GV)
    g_ref = g_ref.numpy()
    err = np.abs(g - g_ref).max() / np.abs(g_ref).max()
    print("adjoint (Table 1 fluids) vs oracle autograd", err, flush=True)
    assert err <= 1e-8


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-8), ("fp32", 1e-3)])
def test_adjoint_full_size_2d_matches_stored_oracle_gradient(precision, tol):
    """The 512x256 adjoint workload (its 64-segment schedule spread over T = 16 steps, K = 5 with
    a ragged last segment) against the oracle's autograd gradient stored by
    tests/golden/make_config4_adjoint_oracle.py: the launch configuration of the benchmark's 2D
    adjoint at its full lattice.  Segments that no step uses get exactly zero.  FP64: 8e-12.
    FP32: 2.6e-4 of a gradient whose largest entry is 1.8e-7 after 16 steps from rest."""
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "config4_adjoint_oracle.json")
    with open(path) as f:
        gold = json.load(f)
    case = make_case("c4", precision=precision)
    sched = np.asarray(gold["schedule"])
    sim = _sim(case, precision, **({"poisson_tol": 1e-5} if precision == "fp32" else {}))
    sim.set_schedule(0, sched, gold["t_total"])
    print("c4", precision, case.n, "T", gold["T"], "K 5, segments", len(sched), flush=True)
    sim.forward_checkpointed(gold["T"], 5)
    ob = sim.observables()
    g = sim.adjoint(np.asarray(gold["dL_dcentroid"]), np.asarray(gold["dL_dvelocity"]), 0, len(sched))
    ref = np.asarray(gold["gradient"])
    err = np.abs(g - ref).max() / np.abs(ref).max()
    print(f"  gradient vs oracle autograd: {err:.3e}; centroid "
          f"{np.abs(ob['centroid'] - np.asarray(gold['centroid'])).max():.3e} lu", flush=True)
    assert np.all(g[ref == 0.0] == 0.0)
    assert np.allclose(ob["centroid"], gold["centroid"], rtol=1e-12 if precision == "fp64" else 1e-6, atol=1e-12)
    assert err <= tol
