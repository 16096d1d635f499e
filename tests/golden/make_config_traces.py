"""Write the oracle's traces for the trace functions of two workloads, on small versions
of their matrices (whose spectra a dense eigensolver still gives):

    python tests/golden/make_config_traces.py

* exp(-beta A), beta = 1, on a 12^3 27-point stencil with lognormal(0, 1) edge weights
  (the 128^3 workload's generator), by the exact real-line deconvolution, cut below the
  Gershgorin lower bound;
* log(A) on a 12^3 Anderson lattice (disorder uniform in [-2, 2]) shifted so that its
  Gershgorin lower bound is 0.1 (the shifted SPD workload's construction), with f floored
  at half that bound (f(max(x, 0.05))), by Algorithm 8's windowed deconvolution.

Each case: the oracle's SS-DGC DOS on a Gaussian block (seed 7), the weights, the trace,
and the exact trace over the dense eigenvalues.  Calls only the oracle (and the input
generators).  Run from the repository root.
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

OUT = "config_traces_small.json"
SEED = 7


def stencil_case():
    return WL.stencil27_lognormal(12, np.random.default_rng(5))


def spd_case():
    a = WL.anderson_3d(12, np.random.default_rng(4).uniform(-2.0, 2.0, 12 ** 3))
    g_lo, _ = WL.gershgorin(a)
    return a.shifted(0.1 - g_lo)


CASES = {
    "exp_stencil27": dict(build=stencil_case, nv=96, degree=2000, nt=400, sigma_hat=0.005, beta=1.0),
    "log_shifted_spd": dict(build=spd_case, nv=96, degree=1500, nt=400, sigma_hat=1.0 / 150, floor=0.05),
}


def main():
    rec = {"about": "oracle traces (FP64) of the workloads' trace functions on small matrices", "seed": SEED}
    for name, c in CASES.items():
        t0 = time.time()
        a = c["build"]()
        lo, hi = WL.interval(a)
        hw = 0.5 * (hi - lo)
        sigma = c["sigma_hat"] * hw
        nt = c["nt"]
        t = 0.5 * (lo + hi) + hw * WL.midpoint_grid(nt)
        lam = np.linalg.eigvalsh(a.to_dense())
        spec_lo = None
        if "beta" in c:
            spec_lo, _ = WL.gershgorin(a)  # a lower bound of the spectrum: weights below it vanish
            wts = O.trace_weights_exp(c["beta"], a.n, lo, hi, nt, sigma, spec_lo=spec_lo)
            exact = float(np.exp(-c["beta"] * lam).sum())
        else:
            fl = c["floor"]
            wts = O.trace_weights(lambda x: np.log(np.maximum(x, fl)), a.n, lo, hi, nt, sigma)
            exact = float(np.log(lam).sum())
        w = WL.gaussian_block(a.n, c["nv"], seed=SEED)
        dos = O.ss_dgc(a, w, t, c["degree"], sigma, lo, hi)["dos"]
        rec[name] = {"n": a.n, "nnz": a.nnz, "lo": lo, "hi": hi, "sigma": sigma, "nt": nt, "nv": c["nv"],
                     "degree": c["degree"], "beta": c.get("beta"), "floor": c.get("floor"), "spec_lo": spec_lo,
                     "trace": float(wts @ dos), "trace_exact_dos": float(wts @ O.exact_dos(lam, t, sigma)),
                     "exact": exact, "seconds": time.time() - t0}
        print(name, rec[name], flush=True)
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), OUT), "w") as fh:
        json.dump(rec, fh, indent=1)


if __name__ == "__main__":
    main()
