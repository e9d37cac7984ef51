"""Write the FP64 oracle's schedule gradient for the 2D 512x256 adjoint workload (pillars, droplet
R=40, electrode, its 64-segment voltage schedule) over T = 16 steps with the schedule spread over
those steps (segment k covers steps with floor(64 t / 16) = k, so every fourth segment is
active): dL/dV by reverse-mode autograd through the oracle's steps, for the loss cotangents
dL/dx_c = (1, 0.3, -0.2) and dL/dv_c = (40, -25, 15), with x_c and v_c at T.  Calls only the
oracle and the shared input generator.  About 25 GB of host memory.

    python tests/golden/make_config4_adjoint_oracle.py [--threads 6]
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
from oracle.adjoint import schedule_gradient  # noqa: E402

T = 16
GX = (1.0, 0.3, -0.2)
GV = (40.0, -25.0, 15.0)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=6)
    ap.add_argument("--out", default=os.path.join(HERE, "config4_adjoint_oracle.json"))
    args = ap.parse_args()
    torch.set_num_threads(args.threads)
    case = make_case("c4", precision="fp64")
    sched = np.asarray(case.schedule, dtype=np.float64)
    o = Oracle(case.dim, case.n, case.periodic, case.params, case.flags)
    t0 = time.time()
    g, xc, vc = schedule_gradient(o, case.phi, sched, T, T, np.asarray(GX), np.asarray(GV))
    print("gradient", f"{time.time() - t0:.0f}s", flush=True)
    out = dict(workload="c4", description=__doc__.split("\n")[0], T=T, t_total=T, schedule=sched.tolist(),
               dL_dcentroid=list(GX), dL_dvelocity=list(GV), gradient=g.numpy().tolist(),
               centroid=xc.numpy().tolist(), velocity=vc.numpy().tolist())
    with open(args.out + ".tmp", "w") as fh:
        json.dump(out, fh)
    os.replace(args.out + ".tmp", args.out)
    print("wrote", args.out, flush=True)


if __name__ == "__main__":
    main()
