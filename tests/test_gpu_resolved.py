"""The reduced-precision paths where N_v exceeds the numerical rank of g(t_i I - A).

In the workloads' own regime every sweep point is under-sampled: the kept ranks sit at
N_v and the estimate at its ceiling of about N_v g_max, which hides the sweep's rounding.
Here the 32 x 32 random Laplacian of the small workload runs with N_v = 120, M = 1000 and
sigma = 0.01 in the rescaled variable, so that the numerical rank (at most about 100) is
below N_v and Algorithm 5 resolves the regularised DOS (Section 3.2).  Sweep points cover
the whole interval, the spectrum's edges and the empty margins included.

Each path runs end to end through the C ABI on the oracle's W and is compared with the
oracle's FP64 SS-DGC on the same W (relative L1 gate 1e-3 for the reduced-precision paths,
1e-9 of the largest value for FP64) and with the exact regularised DOS from a dense
eigen-decomposition; the kept ranks r1 are printed.  The reduced-precision paths run with
the rounding floor of Algorithm 4's truncation (their default) and, for the record, without.
"""
import numpy as np
import pytest
import torch

from oracle import ssm_oracle as O
from paper_1504_07690_amd import workloads as WL

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def case():
    from paper_1504_07690_amd import ssm as S
    a = WL.make_matrix(1)
    wl = WL.make_workload(1, a=a, nv=120, degree=1000, nt=64, sigma_hat=0.01)
    w = wl.w()
    ref = O.ss_dgc(a, w, wl.t, wl.degree, wl.sigma, wl.lo, wl.hi)
    exact = O.exact_dos(np.linalg.eigvalsh(a.to_dense()), wl.t, wl.sigma)
    return S, wl, w, ref, exact


def _l1(x, r):
    return float(np.abs(x - r).sum() / np.abs(r).sum())


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3"])
def test_rank_resolved_paths(case, precision):
    S, wl, w, ref, exact = case
    dt = torch.float64 if precision == "fp64" else torch.float32
    csr = S.DeviceCSR.from_csr(wl.a, dtype=dt, device=DEV)
    wd = torch.tensor(w, dtype=dt, device=DEV)
    ctx = S.SSM(csr, lo=wl.lo, hi=wl.hi, sigma=wl.sigma, nv=wl.nv, degree=wl.degree, t=wl.t, precision=precision,
                w=wd, device=DEV)
    dos, r1, r2 = ctx.dos()
    gmax = O.range_bound(wl.sigma, wl.a.n)
    # Algorithm 4 on the device's Gram matrices, with the floors it used
    from test_gpu_configs import _floors
    v = ctx.views()
    fl = _floors(wl, ctx, v, wl.t)
    kw, kz = v["k_w"].cpu().numpy(), v["k_z"].cpu().numpy()
    alg4 = np.array([O.geneig_trace(kw[i], kz[i], gmax, s_floor=fl[i])[0] for i in range(wl.nt)])
    assert np.abs(dos - alg4).max() <= 1e-9 * gmax
    ctx.close()
    if precision != "fp64":  # the same path without the rounding floor, for the record
        ctx = S.SSM(csr, lo=wl.lo, hi=wl.hi, sigma=wl.sigma, nv=wl.nv, degree=wl.degree, t=wl.t,
                    precision=precision, w=wd, floor_scale=-1.0, device=DEV)
        d_nf, r1_nf, _ = ctx.dos()
        ctx.close()
        print(f"{precision} without the rounding floor: L1 vs oracle {_l1(d_nf, ref['dos']):.2e}, vs exact "
              f"{_l1(d_nf, exact):.2e}")
    inside = ref["dos"] > 1e-3 * ref["dos"].max()
    print(f"{precision}: L1 vs oracle {_l1(dos, ref['dos']):.2e}, vs exact {_l1(dos, exact):.2e} "
          f"(oracle vs exact {_l1(ref['dos'], exact):.2e}); r1 inside the spectrum "
          f"{r1[inside].min()}..{r1[inside].max()}, outside {r1[~inside].min()}..{r1[~inside].max()} "
          f"(oracle {ref['r1'][inside].min()}..{ref['r1'][inside].max()}); "
          f"max error outside {np.abs(dos - ref['dos'])[~inside].max() / gmax:.2e} g_max")
    assert np.all(r1[inside] < wl.nv)  # rank-resolved: the tau test drops directions
    if precision == "fp64":
        assert np.abs(dos - ref["dos"]).max() <= 1e-9 * ref["dos"].max()
        assert np.array_equal(r1[inside], ref["r1"][inside])
    else:
        assert _l1(dos, ref["dos"]) <= 1e-3
    assert _l1(ref["dos"], exact) <= 1e-3
