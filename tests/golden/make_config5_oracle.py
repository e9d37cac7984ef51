"""Write the FP64 oracle's reference for the 3D 384x192x128 EHD workload (D3Q19, square pillars
6x6x10 at pitch 12, droplet R=48, electrode strip 0.05 lu): every field after 1 and 2 steps (the
first without, the second with the time-derivative terms) on a fixed sample of 4096 fluid nodes,
plus each field's max-norm, and the droplet observables at steps 0, 1 and 2.  Calls only the
oracle and the shared input generator.  About 50 GB of host memory.

    python tests/golden/make_config5_oracle.py [--threads 16] [--out tests/golden/config5_oracle.json]
"""
import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402
import torch  # noqa: E402

from inputs import make_case  # noqa: E402
from oracle import Oracle  # noqa: E402
from oracle import poisson  # noqa: E402

STEPS = 2
NAMES = ("phi1", "phi2", "phi3", "ux", "uy", "uz", "p", "rho_e", "pot", "q")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=16)
    ap.add_argument("--out", default=os.path.join(HERE, "config5_oracle.json"))
    args = ap.parse_args()
    torch.set_num_threads(args.threads)
    poisson.PROGRESS_EVERY = 200
    case = make_case("c5", precision="fp64")
    print("c5", case.n, "oracle set-up", flush=True)
    o = Oracle(case.dim, case.n, case.periodic, case.params, case.flags)
    s = o.init_state(case.phi)
    rng = np.random.default_rng(12868)
    fluid = np.nonzero(case.flags == 0)[0]
    sample = np.sort(rng.choice(fluid, 4096, replace=False))
    t0 = time.time()
    records, traj = {}, []

    def observe(k):
        ob = o.observables(s)
        traj.append(dict(step=k, centroid=ob["centroid"].tolist(), velocity=ob["velocity"].tolist(),
                         mass=ob["mass"].tolist(), charge=float(ob["charge"])))

    observe(0)
    for k in range(1, STEPS + 1):
        s, aux = o.step(s)
        print("step", k, f"{time.time() - t0:.0f}s", flush=True)
        observe(k)
        f = o.fields(s)
        arrays = dict(phi1=f["phi"][0], phi2=f["phi"][1], phi3=f["phi"][2], ux=f["u"][0], uy=f["u"][1],
                      uz=f["u"][2], p=f["p"], rho_e=f["rho_e"], pot=aux["pot"], q=aux["Q"])
        rec = {}
        for name in NAMES:
            a = arrays[name].detach().numpy()
            rec[name] = dict(max_abs=float(np.abs(a).max()), sample=a[sample].tolist())
        records[str(k)] = rec
        out = dict(workload="c5", description=__doc__.split("\n")[0], steps_done=k, sample_nodes=sample.tolist(),
                   fields_at=records, trajectory=traj)
        with open(args.out + ".tmp", "w") as fh:
            json.dump(out, fh)
        os.replace(args.out + ".tmp", args.out)
        print("wrote", args.out, "at step", k, f"{time.time() - t0:.0f}s", flush=True)


if __name__ == "__main__":
    main()
