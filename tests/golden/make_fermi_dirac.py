"""Write the oracle's Fermi-Dirac traces on a clean periodic 10^3 lattice (the trace
experiment of Section 6, on a matrix whose spectrum has a closed form):

    python tests/golden/make_fermi_dirac.py

f(x) = 1 / (1 + exp(beta (x - mu))), beta = 10, mu = -1 (A's units); sigma^ = 0.005,
M = 2000, N_t = 400 midpoints, window width sigma~ = 0.016; one Gaussian block of
100 columns (seed 3) serves SS-DGC and DGC with N_v = 100, RESS-DGC with N_v = 100,
and RESS-DGC with N_v = 52, N~_v = 48 (the first 52 columns as W, the rest as W~).
The exact trace sums f over the closed-form eigenvalues -2 (cos 2 pi a/10 + cos 2 pi b/10
+ cos 2 pi c/10).  Calls only the oracle (and the input generators).  Run from the
repository root.
"""
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import ssm_oracle as O  # noqa: E402
from paper_1504_07690_amd import workloads as WL  # noqa: E402

OUT = "fermi_dirac_lattice10.json"
L, NV, M, SIGMA_HAT, NT, SEED = 10, 100, 2000, 0.005, 400, 3
NV_LOW = 52  # RESS-DGC with the hybrid correction: W = columns 0..51, W~ = columns 52..99
BETA, MU = 10.0, -1.0


def fermi_dirac(x):
    return 1.0 / (1.0 + np.exp(BETA * (np.asarray(x) - MU)))


def closed_form_eigenvalues(nx):
    c = np.cos(2.0 * math.pi * np.arange(nx) / nx)
    return np.sort(-2.0 * (c[:, None, None] + c[None, :, None] + c[None, None, :]).ravel())


def main():
    a = WL.anderson_3d(L, np.zeros(L ** 3))
    lo, hi = WL.interval(a)
    hw = 0.5 * (hi - lo)
    sigma = SIGMA_HAT * hw
    t = 0.5 * (lo + hi) + hw * WL.midpoint_grid(NT)
    wt = O.trace_weights(fermi_dirac, a.n, lo, hi, NT, sigma)
    w = WL.gaussian_block(a.n, NV, seed=SEED)
    t0 = time.time()
    ss = O.ss_dgc(a, w, t, M, sigma, lo, hi)["dos"]
    dgc = O.dgc_dos(a, w, t, M, sigma, lo, hi)
    ress = O.ress_dgc(a, w, None, t, M, sigma, lo, hi)["dos"]
    hybrid = O.ress_dgc(a, w[:, :NV_LOW], w[:, NV_LOW:], t, M, sigma, lo, hi)["dos"]
    rec = {
        "about": "oracle Fermi-Dirac traces (FP64) on the clean periodic 10^3 lattice",
        "n": a.n, "nnz": a.nnz, "lo": lo, "hi": hi, "sigma": sigma, "sigma_hat": SIGMA_HAT, "degree": M,
        "nt": NT, "nv": NV, "nv_low": NV_LOW, "seed": SEED, "beta": BETA, "mu": MU,
        "exact": float(fermi_dirac(closed_form_eigenvalues(L)).sum()),
        "ss_dgc": float(wt @ ss), "dgc": float(wt @ dgc), "ress_dgc": float(wt @ ress),
        "ress_dgc_hybrid_52_48": float(wt @ hybrid), "seconds": time.time() - t0,
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), OUT)
    with open(path, "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps(rec, indent=1))


if __name__ == "__main__":
    main()
