"""Write tests/golden/anderson64_fp64_oracle.json: the oracle's SS-DGC estimate at a
strided subset of sweep points of the 64^3 Anderson workload (N = 262144,
N_v = 80, M = 1000, N_t = 1000, sigma^ = 0.01), with the shared seeded inputs.

Calls only the oracle (and the input generators).  Run from the repository root:
    python tests/golden/make_golden.py
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


def main(stride=100, out="anderson64_fp64_oracle.json"):
    wl = WL.make_workload(2)
    points = np.arange(stride // 2, wl.nt, stride)
    t0 = time.time()
    res = O.ss_dgc(wl.a, wl.w(), wl.t, wl.degree, wl.sigma, wl.lo, wl.hi, points=points)
    rec = {
        "about": "oracle SS-DGC (FP64) on the 64^3 Anderson workload, strided sweep points",
        "workload": wl.name, "n": wl.a.n, "nnz": wl.a.nnz, "nv": wl.nv, "degree": wl.degree, "nt": wl.nt,
        "sigma_hat": wl.sigma_hat, "lo": wl.lo, "hi": wl.hi, "sigma": wl.sigma, "seed": wl.seed,
        "points": points.tolist(), "dos": res["dos"].tolist(), "r1": res["r1"].tolist(),
        "r2": res["r2"].tolist(), "seconds": time.time() - t0,
    }
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), out), "w") as fh:
        json.dump(rec, fh, indent=1)
    print("wrote", out, "in", round(rec["seconds"], 1), "s")


if __name__ == "__main__":
    main()
