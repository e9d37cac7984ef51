"""Benchmark of the ternary EHD lattice-Boltzmann step on one MI355X.

    python bench.py [--steps K] [--warmup W] [--workload c3|c2|c2-fp64|c1] [--adjoint c4,c5|c5full|none]

Prints one JSON line: throughput in MLUPS (million lattice-node updates per
second, all nodes counted; fluid-only MLUPS beside it) of whole steps (moments
and wetting ghosts, potential solve to tolerance, fused collide-stream of all
population families), with inputs resident in HBM; the roofline of the dominant
kernel (the fused collide-stream) from its algorithmic bytes and its HIP-event
time; bandwidth references (device copies and the bare population pattern); the FP64 CPU oracle timed on a bounded
sample of the same physics; and the adjoint leg: the cost of the gradient of
the droplet centroid with respect to a piecewise-constant electrode schedule
relative to the forward run, with its error stated against the FP64 adjoint
and against central finite differences of the FP64 forward.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS & HBM GB/s (ternary EHD LB step); adjoint/forward cost at stated error"
HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    "c3": ("c3", "fp32", "3D D3Q19 ternary EHD LB, 256x128x96, pillars 6x6x10 pitch 12, droplet R=30, "
                         "electrode strip 0.05 lu, FP32-deviation storage, FP64 potential residual"),
    "c2": ("c2", "fp32", "2D D2Q9 ternary EHD LB, 512x256, pillars 8/16/12, droplet R=40, electrode 0.05 lu, "
                         "FP32-deviation storage"),
    "c2-fp64": ("c2", "fp64", "2D D2Q9 ternary EHD LB, 512x256, pillars 8/16/12, droplet R=40, electrode "
                              "0.05 lu, FP64"),
    "c1": ("c1", "fp64", "2D D2Q9 ternary LB, 128x64, 6-cell film, droplet R=20, no field, FP64"),
}


def step_kernel_bytes(dim, ehd, tsize):
    """Algorithmic bytes of one fused collide-stream per fluid node: every population read
    once and written once; phi, phi_prev, rho, rho_prev, u_prev, q_prev, pot read once;
    u, q written once; one flag byte (neighbour values are shared, counted once)."""
    Q = 9 if dim == 2 else 19
    F = 5 if ehd else 4
    pops = 2 * F * Q
    reads = 3 + 3 + dim + (4 if ehd else 0)   # phi, phi_prev, u_prev, (rho, rho_prev, q_prev, pot)
    writes = dim + (1 if ehd else 0)
    return (pops + reads + writes) * tsize + 1


def source_hash():
    """Hash of the fused collide-stream kernel's source (its own header and the lattice tables)."""
    h = hashlib.sha256()
    for n in ("step.h", "lattice.h"):
        with open(os.path.join(ROOT, "paper_2608_12868_amd", "csrc", n), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(workload):
    """HBM bytes per fused-step launch from the committed rocprofv3 counter summary, if it was
    taken on the current kernel source (else None)."""
    p = os.path.join(ROOT, "profiles", f"k_step_{workload}_counters.json")
    if not os.path.exists(p):
        return None
    with open(p) as f:
        d = json.load(f)
    if d.get("source_hash") != source_hash():
        return None
    return d.get("hbm_bytes_per_launch")


def _timed(fn, reps):
    """Mean milliseconds of fn() over reps launches (HIP events on torch's current stream, which
    is also the stream fn queues on), after one untimed launch."""
    import torch
    fn()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def copy_ceiling(dims, q, nfam, nbytes=1 << 30, reps=10):
    """Practical HBM ceilings, read + write counted: a 1 GiB device-to-device copy through torch
    (hipMemcpy; the calibration kernel of the rocprofv3 FETCH_SIZE/WRITE_SIZE counters), the
    library's copy kernels at 16 and 4 bytes per lane, and the fused step's population access
    pattern without its arithmetic on the workload's lattice (nfam families of q populations per
    node, stored by population, each pushed to the node its velocity points to), with plain and
    with non-temporal loads."""
    import ctypes as C
    import torch
    from paper_2608_12868_amd import _lib
    L = _lib.lib()
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    out = {"bytes_per_copy": 2 * nbytes}
    out["memcpy_gbs"] = 2 * nbytes / (_timed(lambda: dst.copy_(src), reps) * 1e-3) / 1e9

    def probe(kind, a, b, nb, d=None):
        dd = (C.c_int32 * 3)(*d) if d else None
        st = L.ehdlb_bandwidth_probe(kind, C.c_void_p(a.data_ptr()), C.c_void_p(b.data_ptr()), nb, dd, q, nfam,
                                     stream)
        if st != 0:
            raise RuntimeError(f"ehdlb_bandwidth_probe({kind}) returned {st}")

    for kind, key in ((0, "copy_16B_per_lane_gbs"), (1, "copy_4B_per_lane_gbs")):
        out[key] = 2 * nbytes / (_timed(lambda: probe(kind, src, dst, nbytes), reps) * 1e-3) / 1e9
    del src, dst
    n_nodes = dims[0] * dims[1] * dims[2]
    pb = nfam * q * n_nodes * 4
    a = torch.ones(pb // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    pat = {"lattice": list(dims), "q": q, "families": nfam, "bytes_per_launch": 2 * pb}
    for kind, key in ((2, "plain_loads"), (3, "nontemporal_loads")):
        ms = _timed(lambda: probe(kind, a, b, pb, dims), reps)
        pat[key] = {"us_per_launch": ms * 1e3, "gbs": 2 * pb / (ms * 1e-3) / 1e9}
    out["population_pattern"] = pat
    del a, b
    torch.cuda.empty_cache()
    return out


# adjoint legs: workload, steps before the window, T, K, central-difference directions, FP64 adjoint,
# every warm start, description
ADJOINT = {
    "c4": ("c4", 0, 4000, 100, 3, True, True,
           "2D D2Q9 ternary EHD LB, 512x256 (pillars, droplet R=40, electrode), FP32-deviation storage, 64-segment "
           "voltage schedule, T=4000, checkpoint every 100 steps"),
    "c5": ("c5", 0, 200, 50, 1, False, False,
           "3D D3Q19 ternary EHD LB, 384x192x128 (pillars pitch 12, droplet R=48, electrode strip), FP32-deviation "
           "storage, the 32-segment schedule, steps 0-200 (of its 2000), checkpoint every 50"),
    "c5late": ("c5", 600, 200, 50, 1, False, False,
               "3D D3Q19 ternary EHD LB, 384x192x128 (pillars pitch 12, droplet R=48, electrode strip), "
               "FP32-deviation storage, the 32-segment schedule, steps 600-800 (of its 2000; the first 600 run "
               "untimed), checkpoint every 50"),
    "c5full": ("c5", 0, 2000, 50, 1, False, True,
               "3D D3Q19 ternary EHD LB, 384x192x128 (pillars pitch 12, droplet R=48, electrode strip), "
               "FP32-deviation storage, 32-segment schedule, T=2000, checkpoint every 50"),
}
# central-difference steps: 1e-4 as the workload names it; the quotient of the FP64 forward shows no
# h^2 term up to 8e-3 and its round-off grows as 1/h, so the largest step is the most accurate
FD_H = (8e-3, 1e-3, 1e-4)


def adjoint_leg(key, seed=1):
    """Cost of dL/dV for L = (x_c(T) - x*)^2 (x* = initial centroid + 5 lu), FP32 path: plain
    forward, checkpointed forward and reverse sweep (recompute included), timed with device
    syncs, with the forward warm start that the default uses for the gradient's forward
    (projected onto the last five potentials, then at least one CG iteration: `warm_projected`,
    which also times the default's plain forward, where a projected start that meets the
    tolerance is kept) and, for the 2D leg, the other three (the projection alone; previous
    potential; extrapolated from the last two); each gradient's error against the FP64 adjoint
    (2D leg) and the directional derivatives against central differences of the FP64 forward at
    each step of FD_H."""
    import numpy as np
    import torch
    from inputs import make_case
    from paper_2608_12868_amd import Simulation
    name, start, T, K, ndir, with_fp64_adjoint, all_modes, desc = ADJOINT[key]
    torch.cuda.empty_cache()
    torch.cuda.reset_peak_memory_stats()
    case = make_case(name)
    runs = {}
    target = None
    modes = ((2, "warm_projected"), (3, "warm_projected_only"), (0, "warm_previous"), (1, "warm_extrapolated"))
    for mode, label in (modes if all_modes else modes[:1]):
        sim = Simulation.from_case(case, precision="fp32", poisson_tol=1e-5)
        sim.set_solver_options(warm_start=mode)
        sim.set_schedule(0, case.schedule, case.t_total)
        sim.step(10)
        sim.set_phase(case.phi)
        if target is None:
            target = sim.observables()["centroid"][0] + 5.0
        sim.step(start)
        sim.solver_stats(reset=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(T)
        torch.cuda.synchronize()
        t_fwd = time.perf_counter() - t0
        st_f = sim.solver_stats(reset=True)
        default_fwd = None
        if mode == 2:
            # the library's default (4): plain steps keep a projected start that meets the
            # tolerance, only the gradient's forward iterates at least once (as mode 2)
            sim.set_solver_options(warm_start=4)
            sim.set_phase(case.phi)
            sim.step(start)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sim.step(T)
            torch.cuda.synchronize()
            default_fwd = time.perf_counter() - t0
            sim.set_solver_options(warm_start=mode)
        sim.set_phase(case.phi)
        sim.step(start)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.forward_checkpointed(T, K)
        torch.cuda.synchronize()
        t_ck = time.perf_counter() - t0
        xT = sim.observables()["centroid"]
        sim.solver_stats(reset=True)
        t0 = time.perf_counter()
        g = sim.adjoint(np.array([2.0 * (xT[0] - target), 0.0, 0.0]), np.zeros(3), 0, len(case.schedule))
        torch.cuda.synchronize()
        t_adj = time.perf_counter() - t0
        st_a = sim.solver_stats()["adjoint"]
        runs[label] = dict(forward_s=t_fwd, checkpointed_forward_s=t_ck, adjoint_s=t_adj,
                           ratio_adjoint_to_forward=t_adj / t_fwd,
                           ratio_gradient_to_forward=(t_ck + t_adj) / t_fwd,
                           forward_mlups=case.N * T / t_fwd / 1e6,
                           potential_iters_per_step={"forward": st_f["forward"]["iters"] / T,
                                                     "adjoint": st_a["iters"] / T},
                           grad=g)
        if default_fwd is not None:
            runs[label].update(default_forward_s=default_fwd, ratio_adjoint_to_default_forward=t_adj / default_fwd)
        ws = sim.adjoint_workspace_bytes(T, K) / 1e9
        del sim
        torch.cuda.empty_cache()
        print(f"adjoint leg {key}: {label} reverse/forward {t_adj / t_fwd:.3f}", file=sys.stderr, flush=True)
    peak32 = torch.cuda.max_memory_allocated() / 1e9

    # FP64: adjoint (when the checkpoints fit) and central differences of the forward
    case64 = make_case(name, precision="fp64")
    s64 = Simulation.from_case(case64, precision="fp64")
    g64 = None
    t64 = {}

    def loss(v):
        # the schedule perturbed from the window's start (the gradient covers the window only)
        s64.set_phase(case64.phi)
        s64.set_schedule(0, case64.schedule, case64.t_total)
        s64.step(start)
        s64.set_schedule(0, v, case64.t_total)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s64.step(T)
        torch.cuda.synchronize()
        t64["forward_s"] = time.perf_counter() - t0
        return float((s64.observables()["centroid"][0] - target) ** 2)

    if with_fp64_adjoint:
        loss(case64.schedule)
        s64.set_phase(case64.phi)
        s64.set_schedule(0, case64.schedule, case64.t_total)
        s64.step(start)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s64.forward_checkpointed(T, K)
        torch.cuda.synchronize()
        t64["checkpointed_forward_s"] = time.perf_counter() - t0
        x64 = s64.observables()["centroid"]
        t0 = time.perf_counter()
        g64 = s64.adjoint(np.array([2.0 * (x64[0] - target), 0.0, 0.0]), np.zeros(3), 0, len(case64.schedule))
        torch.cuda.synchronize()
        t64["adjoint_s"] = time.perf_counter() - t0
        t64["ratio_adjoint_to_forward"] = t64["adjoint_s"] / t64["forward_s"]
        print(f"adjoint leg {key}: fp64 reverse/forward {t64['ratio_adjoint_to_forward']:.3f}", file=sys.stderr,
              flush=True)
        s64.adj_ws = None
        torch.cuda.empty_cache()

    rng = np.random.default_rng(seed)
    fd = []
    for _ in range(ndir):
        d = rng.standard_normal(len(case.schedule))
        d /= np.linalg.norm(d)
        row = {}
        for h in FD_H:
            f = (loss(case64.schedule + h * d) - loss(case64.schedule - h * d)) / (2 * h)
            # relative to the directional derivative, and to the gradient's norm (the first is
            # inflated on directions where the derivative is much smaller than the gradient)
            r_h = {"fd": f}
            for label, r in runs.items():
                r_h[label] = float(r["grad"] @ d)
                r_h[label + "_rel_err"] = abs(r_h[label] - f) / abs(f)
                r_h[label + "_err_over_norm"] = abs(r_h[label] - f) / float(np.linalg.norm(r["grad"]))
            if g64 is not None:
                r_h.update(fp64_adjoint=float(g64 @ d), fp64_rel_err=abs(float(g64 @ d) - f) / abs(f),
                           fp64_err_over_norm=abs(float(g64 @ d) - f) / float(np.linalg.norm(g64)))
            row[f"h={h:g}"] = r_h
        print(f"adjoint leg {key}: central difference {len(fd) + 1}/{ndir} done", file=sys.stderr, flush=True)
        fd.append(row)
    out = {"workload": desc, "dtype": "f32", "start_step": start, "T": T, "K": K, "adjoint_workspace_gb": ws, "peak_hbm_gb": peak32,
           "fd_h": list(FD_H), "fd_directions": fd}

    def worst(key_, h):
        return max(row[f"h={h:g}"][key_] for row in fd)
    for label, r in runs.items():
        g = r.pop("grad")
        for h in FD_H:
            r[f"fd_rel_err_max_h={h:g}"] = worst(label + "_rel_err", h)
            r[f"fd_err_over_norm_max_h={h:g}"] = worst(label + "_err_over_norm", h)
        if g64 is not None:
            r["grad_rel_err_vs_fp64_adjoint"] = float(np.abs(g - g64).max() / np.abs(g64).max())
        out[label] = r
    if g64 is not None:
        for h in FD_H:
            t64[f"fd_rel_err_max_h={h:g}"] = worst("fp64_rel_err", h)
            t64[f"fd_err_over_norm_max_h={h:g}"] = worst("fp64_err_over_norm", h)
        out["fp64"] = t64
    return out


def cpu_baseline(budget_s=12.0):
    """The FP64 oracle, as it stands, on a bounded sample: the 48x32x24 3D lattice with the same
    structure (D3Q19, pillars, lubricant, droplet, electrode, field on)."""
    import torch
    from inputs import make_case
    from oracle import Oracle
    case = make_case("c3s")
    o = Oracle(case.dim, case.n, case.periodic, case.params, case.flags)
    s = o.init_state(case.phi)
    s, _ = o.step(s)          # first step (warm-up, factorisation paths)
    n = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s:
        s, _ = o.step(s)
        n += 1
    dt = time.perf_counter() - t0
    return dict(value=case.N * n / dt / 1e6, unit="MLUPS", cores=torch.get_num_threads(), kind="oracle",
                sample=f"{n} steps of the 48x32x24 D3Q19 EHD lattice (pillars, droplet, electrode), FP64")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="c3", choices=sorted(WORKLOADS))
    ap.add_argument("--spin-up", type=int, default=200,
                    help="steps run before the warm-up (not timed): the state the timed steps start from")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-copy-probe", action="store_true",
                    help="skip the bandwidth references (1 GiB device copies, one of them the "
                         "calibration kernel of the rocprofv3 FETCH_SIZE/WRITE_SIZE counters, and the "
                         "fused step's bare population pattern)")
    ap.add_argument("--adjoint", default="c4,c5,c5late",
                    help="comma-separated adjoint legs: c4 (2D 512x256, T = 4000, every forward warm "
                         "start), c5 (3D 384x192x128, steps 0-200), c5late (3D, steps 600-800), c5full "
                         "(3D at T = 2000: about 250 GB of HBM and two minutes), or none")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the step is built for a single MI355X (multi-GPU slab "
              "decomposition is design-only); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from inputs import make_case
    from paper_2608_12868_amd import Simulation

    name, prec, desc = WORKLOADS[args.workload]
    case = make_case(name, precision=prec)
    over = {}
    if prec == "fp32":
        over["poisson_tol"] = 1e-5
    sim = Simulation.from_case(case, precision=prec, **over)
    # the configured runs are thousands of steps long; their first ~50 steps carry a start-up
    # transient of the potential solve (from rest: about 2 CG iterations per step instead of 1.2),
    # so the state is advanced first and the timed steps are representative of the whole run
    sim.step(args.spin_up)
    sim.step(args.warmup)
    torch.cuda.synchronize()
    sim.solver_stats(reset=True)
    sim.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms3, nt = sim.timing()
    sim.set_timing(False)
    stats = sim.solver_stats(reset=True)["forward"]
    obs = sim.observables()
    wall = t1 - t0
    N = case.N
    nfluid = int(np.count_nonzero(case.flags == 0))
    ehd = bool(case.params["ehd"])
    tsize = 8 if prec == "fp64" else 4
    bpn = step_kernel_bytes(case.dim, ehd, tsize)
    step_ms = ms3[2] / max(nt, 1)
    achieved = bpn * nfluid / (step_ms * 1e-3) / 1e9
    traffic = measured_traffic(args.workload)
    out = {
        "metric": METRIC,
        "value": N * args.steps / wall / 1e6,
        "unit": "MLUPS",
        "fluid_mlups": nfluid * args.steps / wall / 1e6,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": desc, "lattice": list(case.n), "nodes": N, "fluid_nodes": nfluid,
                   "spin_up_steps": args.spin_up, "steps_configured": case.steps},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic},
        "phase_ms_per_step": {"moments_ghosts": ms3[0] / max(nt, 1), "potential_solve": ms3[1] / max(nt, 1),
                              "fused_step": step_ms},
        "fused_step_bytes_per_fluid_node": bpn,
        "potential_iters_per_step": stats["iters"] / max(stats["solves"], 1),
        "potential_iters_last_step": obs["poisson_iters"],
        "potential_residual_last_step": obs["poisson_residual"],
    }
    if not args.no_copy_probe:
        from paper_2608_12868_amd import _lib
        dims = list(case.n)
        q = 9 if case.dim == 2 else 19
        nfam = int(_lib.lib().ehdlb_num_populations(sim.h)) // (q * N)
        cc = copy_ceiling(dims, q, nfam)
        pat = max(cc["population_pattern"][k]["gbs"] for k in ("plain_loads", "nontemporal_loads"))
        cc["fused_step_frac_of"] = {"memcpy": achieved / cc["memcpy_gbs"],
                                    "copy_16B_per_lane": achieved / cc["copy_16B_per_lane_gbs"],
                                    "population_pattern": achieved / pat}
        out["copy_ceiling"] = cc
    del sim
    torch.cuda.empty_cache()
    if args.adjoint != "none":
        legs = [k for k in args.adjoint.split(",") if k]
        for k in legs:
            if k not in ADJOINT:
                ap.error(f"unknown adjoint leg {k}")
        out["adjoint"] = {k: adjoint_leg(k) for k in legs}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
