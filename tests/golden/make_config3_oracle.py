"""Write the FP64 oracle's reference for the 3D 256x128x96 EHD workload (D3Q19, square pillars
6x6x10 at pitch 12, droplet R=30, electrode strip 0.05 lu): every field after 2 steps (the
first without, the second with the time-derivative terms) and after the last step, on a fixed
sample of 4096 fluid nodes, plus each field's max-norm, and the droplet observables every 10
steps.  Calls only the oracle and the shared input generator.

    python tests/golden/make_config3_oracle.py [--steps 100] [--threads 6]
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


def sample_fields(o, s, aux, sample):
    f = o.fields(s)
    fields = {}
    for name, arr in (("phi1", f["phi"][0]), ("phi2", f["phi"][1]), ("phi3", f["phi"][2]), ("ux", f["u"][0]),
                      ("uy", f["u"][1]), ("uz", f["u"][2]), ("p", f["p"]), ("rho_e", f["rho_e"]),
                      ("pot", aux["pot"]), ("q", aux["Q"])):
        a = arr.detach().numpy()
        fields[name] = dict(max_abs=float(np.abs(a).max()), sample=a[sample].tolist())
    return fields


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--threads", type=int, default=6)
    args = ap.parse_args()
    torch.set_num_threads(args.threads)
    case = make_case("c3", precision="fp64")
    o = Oracle(case.dim, case.n, case.periodic, case.params, case.flags)
    s = o.init_state(case.phi)
    rng = np.random.default_rng(12868)
    fluid = np.nonzero(case.flags == 0)[0]
    sample = np.sort(rng.choice(fluid, 4096, replace=False))
    t0 = time.time()
    aux = None
    records = {}
    traj = []
    path = os.path.join(HERE, "config3_oracle.json")

    def observe(k):
        ob = o.observables(s)
        traj.append(dict(step=k, centroid=ob["centroid"].tolist(), velocity=ob["velocity"].tolist(),
                         mass=ob["mass"].tolist(), charge=float(ob["charge"])))

    observe(0)
    for k in range(1, args.steps + 1):
        s, aux = o.step(s)
        print("step", k, f"{time.time() - t0:.0f}s", flush=True)
        if k % 10 == 0 or k == args.steps:
            observe(k)
        if k == 2 or k == args.steps:
            records[str(k)] = sample_fields(o, s, aux, sample)
            out = dict(workload="c3", description=__doc__.split("\n")[0], steps_done=k,
                       sample_nodes=sample.tolist(), fields=records["2"], fields_at=records,
                       trajectory=traj)
            with open(path + ".tmp", "w") as fh:
                json.dump(out, fh)
            os.replace(path + ".tmp", path)
            print("wrote", path, "at step", k, f"{time.time() - t0:.0f}s", flush=True)


if __name__ == "__main__":
    main()
