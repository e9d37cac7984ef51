"""The full-size workloads through the C ABI.

512x256 EHD (2D, pillars, droplet R=40, electrode): the GPU paths against the stored output of
the FP64 oracle (tests/golden/config2_oracle.json, written by make_config2_oracle.py from the
oracle alone): every field at 1000 steps on 4096 sampled nodes (FP64 path, <= 1e-10 of the
field's max-norm) and the droplet centroid every 100 steps over the configured 20000 steps
(FP64 path <= 1e-9 relative; FP32-deviation path <= 1e-4 relative and <= 1e-3 of the
displacement).

256x128x96 3D EHD, the lattice and launch configuration the benchmark times: every field after 2
and 100 steps against the stored output of the FP64 oracle on 4096 sampled fluid nodes, and the
centroid every 10 steps to step 100 (tests/golden/config3_oracle.json, written by
make_config3_oracle.py from the oracle alone); per-component mass over 100 steps; the
FP32-deviation path against the FP64 path over the configured 5000 steps, a length the CPU
oracle cannot run at this size.

384x192x128 3D EHD, the 3D adjoint workload's lattice: every field after 1 and 2 steps on 4096
sampled fluid nodes and the observables against tests/golden/config5_oracle.json (written by
make_config5_oracle.py from the oracle alone).

The 2D adjoint workload (512x256, 64-segment schedule, T = 4000, K = 100): the FP32 gradient
against the FP64 adjoint, and the FP64 adjoint against central differences of the FP64 forward
at two step sizes.
"""
import json
import os

import numpy as np
import pytest

from inputs import make_case

import gpu_util as gu

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = os.path.join(HERE, "golden", "config2_oracle.json")
GOLD3 = os.path.join(HERE, "golden", "config3_oracle.json")
GOLD5 = os.path.join(HERE, "golden", "config5_oracle.json")


def _gold():
    with open(GOLD) as f:
        return json.load(f)


def _sim(case, precision, **over):
    from paper_2608_12868_amd import Simulation
    gu.require_gpu()
    return Simulation.from_case(case, precision=precision, **over)


def test_config2_fp64_fields_at_1000_steps():
    g = _gold()
    assert g["steps_done"] >= 1000 and g["fields_at_1000"]
    case = make_case("c2", precision="fp64")
    # the oracle solves the 2D Gauss law directly (sparse LU); the Ohmic source is a divergence
    # of fluxes whose error relative to its own max-norm is the solve's residual amplified by
    # the conductivity contrast, so the FP64 path solves to 1e-14 here
    sim = _sim(case, "fp64", poisson_tol=1e-14)
    print("c2 fp64 1000 steps", case.n, flush=True)
    sim.step(1000)
    idx = np.asarray(g["sample_nodes"])
    worst = 0.0
    for name, ref in g["fields_at_1000"].items():
        a = sim.field(name)[idx]
        b = np.asarray(ref["sample"])
        err = float(np.abs(a - b).max() / max(ref["max_abs"], 1e-300))
        print(f"  {name}: {err:.3e}", flush=True)
        worst = max(worst, err)
    assert worst <= 1e-10


@pytest.mark.parametrize("precision,tol,disp_tol", [("fp64", 1e-9, 1e-7), ("fp32", 1e-4, 1e-3)])
def test_config2_centroid_trajectory(precision, tol, disp_tol):
    g = _gold()
    traj = g["trajectory"]
    case = make_case("c2", precision=precision)
    over = dict(poisson_tol=1e-14) if precision == "fp64" else dict(poisson_tol=1e-5)
    sim = _sim(case, precision, **over)
    print("c2", precision, "trajectory to step", traj[-1]["step"], flush=True)
    worst = worst_abs = 0.0
    x0 = np.asarray(traj[0]["centroid"])
    disp = 0.0
    t = 0
    for rec in traj:
        sim.step(rec["step"] - t)
        t = rec["step"]
        xc = sim.observables()["centroid"]
        ref = np.asarray(rec["centroid"])
        worst = max(worst, float(np.linalg.norm(xc - ref) / np.linalg.norm(ref)))
        worst_abs = max(worst_abs, float(np.linalg.norm(xc - ref)))
        disp = max(disp, float(np.linalg.norm(ref - x0)))
    print(f"  max relative centroid error {worst:.3e} over {t} steps; absolute {worst_abs:.3e} lu, "
          f"{worst_abs / disp:.3e} of the largest displacement {disp:.3f} lu", flush=True)
    assert worst <= tol
    # the droplet moves ~0.1 lu here, so the error is also bounded against the motion itself
    assert worst_abs <= disp_tol * disp


# FP64: the 1e-10 bar of the FP64 path.  FP32-deviation storage: each stored value carries a
# relative rounding of 2^-24 (6e-8); the phase stencils difference neighbouring values (up to
# ~100x relative amplification near flat regions) and the potential is solved to a 1e-5 relative
# residual, which acts on the electric force; 1e-4 of the max-norm (the FP32 bound used for the
# centroid trajectories) covers both.  The pressure (a deviation ~1e-5 lu after 2 steps), the
# potential, the Ohmic source and the charge density it builds (their error is the solve's
# residual amplified by the conductivity contrast: set by the solver tolerance, not the storage)
# are compared for the FP64 path only.
@pytest.mark.parametrize("precision,tol,names", [
    ("fp64", 1e-10, ("phi1", "phi2", "phi3", "ux", "uy", "uz", "p", "rho_e", "pot", "q")),
    ("fp32", 1e-4, ("phi1", "phi2", "phi3", "ux", "uy", "uz"))])
def test_config3_fields_vs_oracle(precision, tol, names):
    with open(GOLD3) as f:
        g = json.load(f)
    case = make_case("c3", precision=precision)
    sim = _sim(case, precision, poisson_tol=1e-14 if precision == "fp64" else 1e-5)
    records = g.get("fields_at") or {str(g["steps_done"]): g["fields"]}
    idx = np.asarray(g["sample_nodes"])
    worst = 0.0
    t = 0
    for step in sorted(int(k) for k in records):
        print("c3", precision, case.n, step, "steps vs stored oracle fields", flush=True)
        sim.step(step - t)
        t = step
        for name in names:
            ref = records[str(step)][name]
            a = sim.field(name)[idx]
            err = float(np.abs(a - np.asarray(ref["sample"])).max() / max(ref["max_abs"], 1e-300))
            print(f"  {name}: {err:.3e}", flush=True)
            worst = max(worst, err)
    assert worst <= tol


# The same bars at 384x192x128, the lattice of the 3D adjoint workload (its forward at full size).
@pytest.mark.parametrize("precision,tol,names", [
    ("fp64", 1e-10, ("phi1", "phi2", "phi3", "ux", "uy", "uz", "p", "rho_e", "pot", "q")),
    ("fp32", 1e-4, ("phi1", "phi2", "phi3", "ux", "uy", "uz"))])
def test_config5_fields_vs_oracle(precision, tol, names):
    """Every field after each stored step (1 and 2) on 4096 sampled fluid nodes against the stored FP64
    oracle output (tests/golden/config5_oracle.json, written by make_config5_oracle.py from the
    oracle alone), and the droplet mass and centroid at both steps."""
    with open(GOLD5) as f:
        g = json.load(f)
    case = make_case("c5", precision=precision)
    sim = _sim(case, precision, poisson_tol=1e-14 if precision == "fp64" else 1e-5)
    idx = np.asarray(g["sample_nodes"])
    obs = {t["step"]: t for t in g["trajectory"]}
    worst = 0.0
    for step in range(1, g["steps_done"] + 1):
        print("c5", precision, case.n, step, "steps vs stored oracle fields", flush=True)
        sim.step(1)
        rec = g["fields_at"][str(step)]
        for name in names:
            a = sim.field(name)[idx]
            err = float(np.abs(a - np.asarray(rec[name]["sample"])).max() / max(rec[name]["max_abs"], 1e-300))
            print(f"  {name}: {err:.3e}", flush=True)
            worst = max(worst, err)
        ob = sim.observables()
        m_err = float(np.abs(np.asarray(ob["mass"]) - obs[step]["mass"]).max() / max(obs[step]["mass"]))
        c_err = float(np.abs(np.asarray(ob["centroid"]) - obs[step]["centroid"]).max()
                      / np.abs(obs[step]["centroid"]).max())
        print(f"  mass {m_err:.3e}, centroid {c_err:.3e}", flush=True)
        worst = max(worst, m_err, c_err)
    assert worst <= tol


@pytest.mark.parametrize("precision,tol,disp_tol", [("fp64", 1e-10, 1e-7), ("fp32", 1e-4, 1e-3)])
def test_config3_centroid_vs_oracle(precision, tol, disp_tol):
    """The droplet centroid at 256x128x96 every 10 steps over the stored oracle trajectory,
    relative to the position and to the droplet's displacement (3e-4 lu over 100 steps)."""
    with open(GOLD3) as f:
        g = json.load(f)
    traj = g.get("trajectory")
    if not traj or traj[-1]["step"] < 10:
        pytest.skip("no stored 3D oracle trajectory")
    case = make_case("c3", precision=precision)
    sim = _sim(case, precision, poisson_tol=1e-14 if precision == "fp64" else 1e-5)
    print("c3", precision, "centroid vs oracle to step", traj[-1]["step"], flush=True)
    worst = worst_abs = 0.0
    t = 0
    for rec in traj:
        sim.step(rec["step"] - t)
        t = rec["step"]
        ob = sim.observables()
        ref = np.asarray(rec["centroid"])
        worst = max(worst, float(np.linalg.norm(ob["centroid"] - ref) / np.linalg.norm(ref)))
        worst_abs = max(worst_abs, float(np.linalg.norm(ob["centroid"] - ref)))
        assert np.allclose(ob["mass"], rec["mass"], rtol=1e-12 if precision == "fp64" else 1e-5, atol=0)
    disp = float(np.linalg.norm(np.asarray(traj[-1]["centroid"]) - np.asarray(traj[0]["centroid"])))
    print(f"  max relative centroid error {worst:.3e}; absolute {worst_abs:.3e} lu "
          f"(displacement {disp:.4f} lu)", flush=True)
    assert worst <= tol
    assert worst_abs <= disp_tol * disp


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_config3_mass_conservation(precision):
    """Per-component mass over 100 steps at 256x128x96 (the collision conserves each phase's
    zeroth moment and bounce-back returns every population): round-off in FP64; in FP32 each
    node's moment is a sum of 19 rounded values, so the drift per step is at most 19 * 2^-24 of
    the mass, 100 times that over the run."""
    steps = 100
    case = make_case("c3", precision=precision)
    sim = _sim(case, precision, poisson_tol=1e-13 if precision == "fp64" else 1e-5)
    m0 = sim.observables()["mass"]
    print("c3", precision, "mass over", steps, "steps", m0, flush=True)
    sim.step(steps)
    m1 = sim.observables()["mass"]
    drift = float(np.max(np.abs(m1 - m0) / m0))
    print(f"  max relative drift {drift:.3e}", flush=True)
    assert drift <= (1e-12 if precision == "fp64" else steps * 19 * 2.0 ** -24)


def test_config3_fp32_centroid_vs_fp64():
    steps, every = 5000, 250
    tracks = {}
    for precision in ("fp64", "fp32"):
        case = make_case("c3", precision=precision)
        over = dict(poisson_tol=1e-13) if precision == "fp64" else dict(poisson_tol=1e-5)
        sim = _sim(case, precision, **over)
        print("c3", precision, case.n, steps, "steps", flush=True)
        xs = [sim.observables()["centroid"]]
        for _ in range(steps // every):
            sim.step(every)
            xs.append(sim.observables()["centroid"])
        tracks[precision] = np.asarray(xs)
        del sim
    err = np.linalg.norm(tracks["fp32"] - tracks["fp64"], axis=1) / np.linalg.norm(tracks["fp64"], axis=1)
    err_abs = np.linalg.norm(tracks["fp32"] - tracks["fp64"], axis=1)
    disp = np.linalg.norm(tracks["fp64"] - tracks["fp64"][0], axis=1).max()
    print(f"  max relative centroid error {err.max():.3e}; absolute {err_abs.max():.3e} lu, "
          f"{err_abs.max() / disp:.3e} of the largest displacement {disp:.3f} lu", flush=True)
    assert err.max() <= 1e-4
    assert err_abs.max() <= 1e-3 * disp


_C4_FP64 = {}


def _c4_fp64_gradient():
    """The FP64 adjoint gradient of x_c(4000) on the 512x256 schedule workload (K = 100,
    solver tolerance 1e-13), computed once and shared by the tests that compare against it."""
    if "g" not in _C4_FP64:
        case = make_case("c4", precision="fp64")
        sim = _sim(case, "fp64", poisson_tol=1e-13)
        sim.set_schedule(0, case.schedule, case.t_total)
        print("c4 fp64 checkpointed forward + adjoint, T 4000, K 100", flush=True)
        sim.forward_checkpointed(4000, 100)
        _C4_FP64["g"] = sim.adjoint(np.array([1.0, 0.0, 0.0]), np.zeros(3), 0, len(case.schedule))
        del sim
    return _C4_FP64["g"]


@pytest.mark.parametrize("warm", [4, 1])
def test_config4_fp32_gradient_vs_fp64(warm):
    """512x256, 64-segment schedule, T = 4000, K = 100: the FP32 gradient of the centroid agrees
    with the FP64 adjoint to 3e-4 with the default forward warm start (whose checkpointed forward
    takes the projection, then at least one CG iteration) and with the extrapolated one (a start kept without iterating lags the
    exact Gauss law by an error correlated from step to step: ~7e-4 with the projection alone,
    ~4e-3 with the previous potential).  The bar is the FP32 sweep's own rounding: 4000 steps
    amplify single-precision rounding to ~1e-4 of the gradient (two builds of the same
    arithmetic that differ only in where the compiler fuses multiply-adds give 6.1e-5 and
    1.27e-4, and their FP64 gradients differ by 8e-14, the same amplification of FP64 rounding),
    so a bar at 1e-4 would test the compiler's choices rather than the adjoint."""
    T, K = 4000, 100
    g = {"fp64": _c4_fp64_gradient()}
    case = make_case("c4", precision="fp32")
    sim = _sim(case, "fp32", poisson_tol=1e-5)
    if warm != 4:
        sim.set_solver_options(warm_start=warm)
    sim.set_schedule(0, case.schedule, case.t_total)
    print("c4 fp32 warm_start", warm, "T", T, "K", K, flush=True)
    sim.forward_checkpointed(T, K)
    g["fp32"] = sim.adjoint(np.array([1.0, 0.0, 0.0]), np.zeros(3), 0, len(case.schedule))
    del sim
    err = np.abs(g["fp32"] - g["fp64"]).max() / np.abs(g["fp64"]).max()
    print(f"  FP32 (warm_start {warm}) vs FP64 adjoint: {err:.3e}", flush=True)
    assert err <= 3e-4


@pytest.mark.timeout(400)
def test_config4_fp64_adjoint_vs_central_difference_sequence():
    """512x256, 64 segments, T = 4000, K = 100: the FP64 adjoint's directional derivatives of the
    droplet centroid x_c(T) along three seeded unit directions (the benchmark's) against central
    differences of the FP64 forward at h = 8e-3 and 4e-3.  The two quotients agree to 1e-7 of
    the gradient's norm, so no h^2 truncation term is visible at these steps (over h = 8e-3 ...
    1e-3 the quotient moves only by its round-off, which grows as 1/h; the benchmark adds h =
    1e-3 and 1e-4), and the largest h is the most accurate: there the adjoint agrees to <= 1e-4
    relative on every direction, including one whose derivative is ~100x smaller than the
    others, and to <= 1e-6 on the directions that carry the gradient."""
    T = 4000
    case = make_case("c4", precision="fp64")
    g = _c4_fp64_gradient()
    sim = _sim(case, "fp64")
    sched = np.asarray(case.schedule, dtype=np.float64)

    def xc(v):
        sim.set_phase(case.phi)
        sim.set_schedule(0, v, case.t_total)
        sim.step(T)
        return float(sim.observables()["centroid"][0])

    rng = np.random.default_rng(1)
    hs = (8e-3, 4e-3)
    gn = float(np.linalg.norm(g))
    for k in range(3):
        d = rng.standard_normal(len(sched))
        d /= np.linalg.norm(d)
        gd = float(g @ d)
        fd = {}
        for h in hs:
            fd[h] = (xc(sched + h * d) - xc(sched - h * d)) / (2 * h)
            print(f"  direction {k}: g.d {gd:+.12e}, h {h:g}: quotient {fd[h]:+.12e}, relative {abs(fd[h] - gd) / abs(gd):.2e}, "
                  f"absolute {abs(fd[h] - gd):.2e}", flush=True)
        rel = abs(fd[hs[0]] - gd) / abs(gd)
        assert rel <= 1e-4, (k, rel)
        if abs(gd) >= 0.1 * gn:
            assert rel <= 1e-6, (k, rel)
        # the quotients at the two largest steps agree to 1e-7 of the gradient's norm: an h^2
        # truncation term would separate them by three quarters of its value at h = 8e-3
        assert abs(fd[hs[0]] - fd[hs[1]]) <= 1e-7 * gn, k
