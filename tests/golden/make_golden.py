"""Write the oracle's SS-DGC estimate at a strided subset of sweep points of a
full-size workload, with the shared seeded inputs:

    python tests/golden/make_golden.py            # 64^3 Anderson (N = 262144, N_v = 80,
                                                  # M = 1000, N_t = 1000, sigma^ = 0.01)
    python tests/golden/make_golden.py 4          # the shifted SPD Anderson lattice
                                                  # (M = 1500, N_t = 1500, sigma^ = 1/150)
    python tests/golden/make_golden.py 3          # the random-graph Laplacian (N = 2^20,
                                                  # N_v = 128, M = 2000, N_t = 2000), 16 points
                                                  # (hours on one host core)

Calls only the oracle (and the input generators).  Run from the repository root.
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import ssm_oracle as O  # noqa: E402
from paper_1504_07690_amd import workloads as WL  # noqa: E402


OUT = {2: "anderson64_fp64_oracle.json", 4: "anderson64_spd_fp64_oracle.json", 3: "er_graph_2p20_fp64_oracle.json"}
NPOINTS = {2: 10, 4: 10, 3: 16}


def main(cfg=2, out=None):
    wl = WL.make_workload(cfg)
    stride = wl.nt // NPOINTS[cfg]
    out = out or OUT[cfg]
    points = np.arange(stride // 2, wl.nt, stride)
    t0 = time.time()
    res = O.ss_dgc(wl.a, wl.w(), wl.t, wl.degree, wl.sigma, wl.lo, wl.hi, points=points)
    rec = {
        "about": "oracle SS-DGC (FP64) on a full-size workload, strided sweep points",
        "workload": wl.name, "n": wl.a.n, "nnz": wl.a.nnz, "nv": wl.nv, "degree": wl.degree, "nt": wl.nt,
        "sigma_hat": wl.sigma_hat, "lo": wl.lo, "hi": wl.hi, "sigma": wl.sigma, "seed": wl.seed,
        "points": points.tolist(), "dos": res["dos"].tolist(), "r1": res["r1"].tolist(),
        "r2": res["r2"].tolist(), "seconds": time.time() - t0,
    }
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), out), "w") as fh:
        json.dump(rec, fh, indent=1)
    print("wrote", out, "in", round(rec["seconds"], 1), "s")


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 2)
