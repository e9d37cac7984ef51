"""Write the FP64 oracle's reference for the 512x256 EHD workload (2D D2Q9, pillars 8/16/12,
droplet R=40, electrode 0.05 lu): the droplet centroid and velocity every 100 steps over 20000
steps, and every field at 1000 steps on a fixed sample of 4096 nodes plus its per-field
max-norm.  Calls only the oracle and the shared input generator.

    python tests/golden/make_config2_oracle.py [--steps 20000] [--out PATH]

The output is written to PATH (default: config2_oracle.json beside this script) every 1000
steps; a run writing elsewhere leaves the stored reference untouched until it is copied over.
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--threads", type=int, default=6)
    ap.add_argument("--out", default=os.path.join(HERE, "config2_oracle.json"))
    args = ap.parse_args()
    torch.set_num_threads(args.threads)
    case = make_case("c2")
    o = Oracle(case.dim, case.n, case.periodic, case.params, case.flags)
    s = o.init_state(case.phi)
    rng = np.random.default_rng(12868)
    fluid = np.nonzero(case.flags == 0)[0]
    sample = np.sort(rng.choice(fluid, 4096, replace=False))
    traj = []
    fields_1000 = None
    t0 = time.time()
    path = args.out
    for k in range(args.steps + 1):
        if k % 100 == 0:
            ob = o.observables(s)
            traj.append(dict(step=k, centroid=ob["centroid"].tolist(), velocity=ob["velocity"].tolist(),
                             mass=ob["mass"].tolist(), charge=float(ob["charge"])))
            print(k, traj[-1]["centroid"], f"{time.time() - t0:.0f}s", flush=True)
        if k == 1000:
            f = o.fields(s)
            fields_1000 = {}
            for name, arr in (("phi1", f["phi"][0]), ("phi2", f["phi"][1]), ("phi3", f["phi"][2]),
                              ("ux", f["u"][0]), ("uy", f["u"][1]), ("p", f["p"]), ("rho_e", f["rho_e"]),
                              ("pot", aux["pot"]), ("q", aux["Q"])):
                a = arr.detach().numpy()
                fields_1000[name] = dict(max_abs=float(np.abs(a).max()), sample=a[sample].tolist())
        if k % 1000 == 0 or k == args.steps:
            out = dict(workload="c2", description=__doc__.split("\n")[0], steps_done=k,
                       sample_nodes=sample.tolist(), trajectory=traj, fields_at_1000=fields_1000)
            with open(path + ".tmp", "w") as fh:
                json.dump(out, fh)
            os.replace(path + ".tmp", path)
        if k < args.steps:
            s, aux = o.step(s)


if __name__ == "__main__":
    main()
