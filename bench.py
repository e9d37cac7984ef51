"""Benchmark of the ternary EHD lattice-Boltzmann step on one MI355X.

    python bench.py [--steps K] [--warmup W] [--workload c3|c2|c2-fp64|c1]

Prints one JSON line: throughput in MLUPS (million lattice-node updates per
second, all nodes counted) of whole steps (moments and wetting ghosts,
potential solve to tolerance, fused collide-stream of all population
families), with inputs resident in HBM; the roofline of the dominant kernel
(the fused collide-stream) from its algorithmic bytes and its HIP-event time;
and the FP64 CPU oracle timed on a bounded sample of the same physics.
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


def copy_ceiling(nbytes=1 << 30, reps=10):
    """Practical HBM ceiling: a plain device-to-device copy of nbytes (read + write counted),
    timed with HIP events on torch's stream."""
    import torch
    src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    return dict(bytes_per_copy=2 * nbytes, gbs=2 * nbytes / (ms * 1e-3) / 1e9)


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
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="c3", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also time a plain 1 GiB device copy (practical bandwidth ceiling; the "
                         "calibration kernel of the rocprofv3 FETCH_SIZE/WRITE_SIZE counters)")
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
    sim.step(args.warmup)
    torch.cuda.synchronize()
    sim.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms3, nt = sim.timing()
    sim.set_timing(False)
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
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": desc, "lattice": list(case.n), "nodes": N, "fluid_nodes": nfluid},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic},
        "phase_ms_per_step": {"moments_ghosts": ms3[0] / max(nt, 1), "potential_solve": ms3[1] / max(nt, 1),
                              "fused_step": step_ms},
        "fused_step_bytes_per_fluid_node": bpn,
        "potential_iters_last_step": obs["poisson_iters"],
        "potential_residual_last_step": obs["poisson_residual"],
    }
    if args.copy_probe:
        out["copy_ceiling"] = copy_ceiling()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
