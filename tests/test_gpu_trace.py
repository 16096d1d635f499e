"""Tr f(A) (Algorithm 8) through the C ABI against the FP64 oracle.

The device DOS with the library's weights (ssm_trace_weights, ssm_trace) is
compared with the oracle's DOS and the oracle's weights on the same W.  The
smearing is sigma^ = 0.005, inside the range where the deconvolution of §5 is
well posed for the paper's window width 0.016.  Gates: 1e-6 relative for the
FP64 path; 1e-3 relative for the mixed paths (their DOS L1 gate).  The exact
Tr f from a dense eigen-decomposition is printed for context only.
"""
import numpy as np
import pytest
import torch

from oracle import ssm_oracle as O
from paper_1504_07690_amd import workloads as WL

pytestmark = pytest.mark.gpu
DEV = "cuda:0"

FUNCS = {
    "exp(-x/2)": lambda x: np.exp(-0.5 * x),
    "x": lambda x: x,
    "x^2": lambda x: x * x,
}


@pytest.fixture(scope="module")
def S():
    from paper_1504_07690_amd import ssm
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return ssm


@pytest.fixture(scope="module")
def case():
    rng = np.random.default_rng(11)
    a = WL.laplacian_2d_dirichlet(16, rng.uniform(-1, 1, 256))
    wl = WL.make_workload(1, a=a, nv=16, degree=2000, nt=500, sigma_hat=0.005)
    w = wl.w()
    dos = O.ss_dgc(a, w, wl.t, wl.degree, wl.sigma, wl.lo, wl.hi)["dos"]
    ref = {}
    lam = np.linalg.eigvalsh(a.to_dense())
    for name, f in FUNCS.items():
        wt = O.trace_weights(f, a.n, wl.lo, wl.hi, wl.nt, wl.sigma)
        ref[name] = (float(wt @ dos), float(np.sum(f(lam))))
    return wl, w, ref


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-6), ("fp32", 1e-3), ("bf16x3", 1e-3)])
def test_trace_matches_oracle(S, case, precision, tol):
    wl, w, ref = case
    dt = torch.float64 if precision == "fp64" else torch.float32
    csr = S.DeviceCSR.from_csr(wl.a, dtype=dt, device=DEV)
    wd = torch.tensor(w if precision == "fp64" else w.astype(np.float32), dtype=dt, device=DEV)
    ctx = S.SSM(csr, lo=wl.lo, hi=wl.hi, sigma=wl.sigma, nv=wl.nv, degree=wl.degree, t=wl.t,
                precision=precision, seed=wl.seed, w=wd, device=DEV)
    ctx.dos()
    for name, f in FUNCS.items():
        wt = S.trace_weights(f, lo=wl.lo, hi=wl.hi, nt=wl.nt, n=wl.a.n, sigma=wl.sigma)
        tr = ctx.trace(wt)
        tr_oracle, tr_exact = ref[name]
        rel = abs(tr - tr_oracle) / abs(tr_oracle)
        print(f"{precision} Tr {name}: device {tr:.12e} oracle {tr_oracle:.12e} rel {rel:.2e} "
              f"(exact {tr_exact:.6e})")
        assert rel <= tol, name
    ctx.close()
