"""RESS-DGC (Algorithm 7, with the hybrid correction of Algorithm 6) through the C ABI
against the oracle.

The device runs the recurrence on V = [W W~] to degree M/2 + 1 and takes every moment
X_l = V^T T_l(A~) V (l <= M) from Gram matrices of consecutive blocks; the oracle runs
Algorithm 7 as printed (M steps, X_W = W^T V_c at each).  Both are FP64.  Gates, from the
oracle's own agreement with SS-DGC at degree M/2 (Theorem 4) and a host model of the
device's arithmetic:
* where the oracle's estimate exceeds 1e-2 of its maximum: 1e-9 of the maximum;
* above 1e-4 of the maximum: 1e-6;
* everywhere: 1e-3 (at the spectrum's edges both sides are rounding noise of
  Algorithm 4 on a nearly null pencil).
Moments to 1e-11 of max |X_0|; Proposition 1's coefficients to 1e-13.
"""
import numpy as np
import pytest
import torch

from oracle import ssm_oracle as O
from paper_1504_07690_amd import workloads as WL

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def S():
    from paper_1504_07690_amd import ssm
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return ssm


def _ctx(S, wl, v, nv, nvh, budget=0, t=None, precision="fp64"):
    dt = torch.float64 if precision == "fp64" else torch.float32
    csr = S.DeviceCSR.from_csr(wl.a, dtype=dt, device=DEV)
    wd = torch.tensor(v, dtype=dt, device=DEV)
    ctx = S.SSM(csr, lo=wl.lo, hi=wl.hi, sigma=wl.sigma, nv=nv, degree=wl.degree, t=wl.t if t is None else t,
                precision=precision, seed=wl.seed, w=wd, budget=budget, method="ress", nv_hybrid=nvh, device=DEV)
    return csr, wd, ctx


def _moments(a, v, degree, lo, hi):
    x = np.zeros((degree + 1, v.shape[1], v.shape[1]))
    for l, v_c in O.chebyshev_blocks(a, v, degree, lo, hi):
        x[l] = v.T @ v_c
    return x


def _check(dos, ref, label):
    top = np.abs(ref).max()
    d = np.abs(dos - ref)
    bulk, mid = ref > 1e-2 * top, ref > 1e-4 * top
    print(f"{label}: max err bulk {d[bulk].max() / top:.2e}, resolved {d[mid].max() / top:.2e}, "
          f"all {d.max() / top:.2e} (of max)")
    assert d[bulk].max() <= 1e-9 * top
    assert d[mid].max() <= 1e-6 * top
    assert d.max() <= 1e-3 * top


@pytest.fixture(scope="module")
def cfg1():
    return WL.make_workload(1)


@pytest.mark.parametrize("nv,nvh", [(40, 0), (20, 20), (12, 8)])
def test_ress_matches_oracle(S, cfg1, nv, nvh):
    wl = cfg1
    v = WL.gaussian_block(wl.a.n, nv + nvh, seed=5)
    ref = O.ress_dgc(wl.a, v[:, :nv], v[:, nv:] if nvh else None, wl.t, wl.degree, wl.sigma, wl.lo, wl.hi)
    csr, wd, ctx = _ctx(S, wl, v, nv, nvh)
    dos, r1, r2 = ctx.dos()
    views = ctx.views()
    st = ctx.stats()
    x = views["moments"].cpu().numpy()
    nu = views["coeff_sq"].cpu().numpy()
    ctx.close()
    _check(dos, ref["dos"], f"RESS-DGC N_v={nv} N~_v={nvh}")
    keep = ref["dos"] > 1e-2 * ref["dos"].max()
    assert np.array_equal(r1[keep], ref["r1"][keep])
    assert st["spmm_launches"] == wl.degree // 2 + 1
    xr = _moments(wl.a, v, wl.degree, wl.lo, wl.hi)
    assert np.abs(x - xr).max() <= 1e-11 * np.abs(xr[0]).max()
    mu = ref["mu"][: wl.degree // 2 + 1]
    assert np.all(np.abs(nu - ref["nu"]) <= 1e-13 * (np.abs(mu).sum(axis=0) ** 2)[None, :])


def test_ress_small_workspace_ring_wraps(S, cfg1):
    """A budget that leaves a ring of a few slots: pairs are formed round by round and one
    pair per wrap spans the ring's last and first slots; the estimate is unchanged."""
    wl = cfg1
    nv, nvh = 20, 20
    v = WL.gaussian_block(wl.a.n, nv + nvh, seed=6)
    csr, wd, ctx = _ctx(S, wl, v, nv, nvh)
    full, _, _ = ctx.dos()
    ctx.close()
    e = wl.a.n * (nv + nvh) * 8
    budget = S.workspace_size(csr, lo=wl.lo, hi=wl.hi, sigma=wl.sigma, nv=nv, degree=wl.degree, nt=wl.nt,
                              precision="fp64", method="ress", nv_hybrid=nvh) - (wl.degree // 2 - 6) * e
    csr, wd, ctx = _ctx(S, wl, v, nv, nvh, budget=budget)
    st = ctx.stats()
    small, _, _ = ctx.dos()
    ctx.close()
    assert 3 <= st["chunk"] < wl.degree // 2, st
    assert np.abs(small - full).max() <= 1e-12 * np.abs(full).max()


@pytest.mark.parametrize("degree,nv,nvh", [(2, 8, 4), (4, 8, 0), (64, 12, 8), (130, 4, 4)])
def test_ress_degrees_and_ragged_block(S, degree, nv, nvh):
    rng = np.random.default_rng(degree)
    n = 397
    import scipy.sparse as sp
    m = (rng.random((n, n)) < 0.02) * rng.standard_normal((n, n))
    m = np.triu(m, 1)
    m = sp.csr_matrix(m + m.T + np.diag(rng.uniform(-2, 2, n)))
    m.sort_indices()
    a = WL.CSR(n, m.indptr.astype(np.int32), m.indices.astype(np.int32), m.data.astype(np.float64))
    wl = WL.make_workload(1, a=a, nv=nv, degree=degree, nt=37, sigma_hat=0.2)
    v = WL.gaussian_block(n, nv + nvh, seed=degree)
    ref = O.ress_dgc(a, v[:, :nv], v[:, nv:] if nvh else None, wl.t, degree, wl.sigma, wl.lo, wl.hi)
    csr, wd, ctx = _ctx(S, wl, v, nv, nvh)
    dos, _, _ = ctx.dos()
    x = ctx.views()["moments"].cpu().numpy()
    ctx.close()
    xr = _moments(a, v, degree, wl.lo, wl.hi)
    assert np.abs(x - xr).max() <= 1e-11 * np.abs(xr[0]).max()
    _check(dos, ref["dos"], f"ragged M={degree} N_v={nv} N~_v={nvh}")


@pytest.mark.parametrize("nv,nvh", [(64, 16), (96, 32), (128, 0), (160, 96)])
def test_ress_large_blocks(S, nv, nvh):
    """N_v' above 96 (tiled pair Gram) and N_v above 96 (Algorithm 4 in global scratch)."""
    rng = np.random.default_rng(nv + nvh)
    a = WL.laplacian_2d_dirichlet(24, rng.uniform(-1, 1, 576))
    wl = WL.make_workload(1, a=a, nv=nv, degree=160, nt=40, sigma_hat=0.05)
    v = WL.gaussian_block(a.n, nv + nvh, seed=nv)
    ref = O.ress_dgc(a, v[:, :nv], v[:, nv:] if nvh else None, wl.t, wl.degree, wl.sigma, wl.lo, wl.hi)
    csr, wd, ctx = _ctx(S, wl, v, nv, nvh)
    dos, _, _ = ctx.dos()
    ctx.close()
    _check(dos, ref["dos"], f"large N_v={nv} N~_v={nvh}")


def test_ress_errors(S, cfg1):
    from paper_1504_07690_amd import _abi as A
    wl = cfg1
    csr = S.DeviceCSR.from_csr(wl.a, dtype=torch.float32, device=DEV)
    with pytest.raises(A.SSMError) as ei:
        S.SSM(csr, lo=wl.lo, hi=wl.hi, sigma=wl.sigma, nv=8, degree=20, t=wl.t, precision="bf16x3",
              method="ress", device=DEV)
    assert ei.value.status == A.SSM_ERR_UNSUPPORTED
    v = WL.gaussian_block(wl.a.n, 8, seed=1)
    wl2 = WL.make_workload(1, nv=8, degree=20, nt=10)
    csr, wd, ctx = _ctx(S, wl2, v, 8, 0)
    ctx.dos()
    with pytest.raises(A.SSMError) as ei:
        ctx.backward(np.ones(wl2.nt))
    assert ei.value.status == A.SSM_ERR_UNSUPPORTED
    ctx.close()


def test_ress_hybrid_under_sampled_regime(S, cfg1):
    """Section 4: with N_v + N~_v below the numerical rank, SS-DGC on all the vectors is
    biased low (it can keep at most N_v' eigenvalues per point), while RESS-DGC with half
    of them spent on the hybrid correction is unbiased.  Against the exact DOS of the
    degree-M/2 filter the hybrid estimate is the closer one."""
    a = cfg1.a
    lo, hi = WL.interval(a)
    hw = 0.5 * (hi - lo)
    wl = WL.make_workload(1, a=a, nv=20, degree=2000, nt=40, sigma_hat=0.05)
    t = 0.5 * (lo + hi) + hw * np.linspace(-0.8, 0.8, 40)
    lam = np.linalg.eigvalsh(a.to_dense())
    ref = O.exact_dos(lam, t, wl.sigma)
    v = WL.gaussian_block(a.n, 40, seed=21)
    csr, wd, ctx = _ctx(S, wl, v, 20, 20, t=t)
    hybrid, _, _ = ctx.dos()
    ctx.close()
    csr = S.DeviceCSR.from_csr(a, dtype=torch.float64, device=DEV)
    ctx = S.SSM(csr, lo=lo, hi=hi, sigma=wl.sigma, nv=40, degree=1000, t=t, precision="fp64",
                w=torch.tensor(v, dtype=torch.float64, device=DEV), device=DEV)
    ss, r1, _ = ctx.dos()
    ctx.close()
    e_h = np.abs(hybrid - ref).sum() / np.abs(ref).sum()
    e_s = np.abs(ss - ref).sum() / np.abs(ref).sum()
    print(f"L1 vs exact DOS: RESS-DGC 20+20 {e_h:.3e}, SS-DGC 40 {e_s:.3e}; SS-DGC r1 max {r1.max()}")
    assert e_h < e_s


def _l1(x, r):
    return float(np.abs(x - r).sum() / np.abs(r).sum())


@pytest.mark.parametrize("nv,nvh", [(40, 0), (20, 20), (12, 8)])
def test_ress_fp32_recurrence(S, cfg1, nv, nvh):
    """RESS-DGC with an FP32 recurrence and pair Gram matrices of FP32 blocks (products and
    sums in FP64), against the oracle's FP64 Algorithm 7 on the same (FP32-rounded) V:
    relative L1 within 1e-3, the gate of the reduced-precision paths.  Its floor of
    Algorithm 4's truncation is 2^-18 of the sum of moments (the FP32 moments' rounding)."""
    wl = cfg1
    v = WL.gaussian_block(wl.a.n, nv + nvh, seed=5).astype(np.float32).astype(np.float64)
    ref = O.ress_dgc(wl.a, v[:, :nv], v[:, nv:] if nvh else None, wl.t, wl.degree, wl.sigma, wl.lo, wl.hi)
    csr, wd, ctx = _ctx(S, wl, v, nv, nvh, precision="fp32")
    dos, r1, r2 = ctx.dos()
    x = ctx.views()["moments"].cpu().numpy()
    ctx.close()
    xr = _moments(wl.a, v, wl.degree, wl.lo, wl.hi)
    xerr = np.abs(x - xr).max() / np.abs(xr[0]).max()
    print(f"RESS-DGC FP32 N_v={nv} N~_v={nvh}: DOS L1 vs the FP64 oracle {_l1(dos, ref['dos']):.2e}, "
          f"max error {np.abs(dos - ref['dos']).max() / ref['dos'].max():.2e} of the maximum; moments "
          f"{xerr:.2e} of max|X_0|")
    assert _l1(dos, ref["dos"]) <= 1e-3
    assert xerr <= 1e-5


def test_ress_fp32_rank_resolved(S):
    """N_v = 120 above the numerical rank of the 32 x 32 workload's filter (M = 1000,
    sigma^ = 0.01, 64 points over the whole interval): the FP64 and FP32 RESS-DGC paths
    against the oracle's Algorithm 7 and against the exact DOS of the degree-M/2 filter."""
    a = WL.make_matrix(1)
    wl = WL.make_workload(1, a=a, nv=120, degree=1000, nt=64, sigma_hat=0.01)
    v = WL.gaussian_block(a.n, 120, seed=7).astype(np.float32).astype(np.float64)
    ref = O.ress_dgc(a, v, None, wl.t, wl.degree, wl.sigma, wl.lo, wl.hi)
    exact = O.exact_dos(np.linalg.eigvalsh(a.to_dense()), wl.t, wl.sigma)
    out = {}
    for precision in ("fp64", "fp32"):
        csr, wd, ctx = _ctx(S, wl, v, 120, 0, precision=precision)
        out[precision] = ctx.dos()
        ctx.close()
    for precision, (dos, r1, r2) in out.items():
        print(f"RESS-DGC {precision} N_v=120: L1 vs oracle {_l1(dos, ref['dos']):.2e}, vs exact "
              f"{_l1(dos, exact):.2e} (oracle vs exact {_l1(ref['dos'], exact):.2e}); r1 {r1.min()}..{r1.max()}")
    _check(out["fp64"][0], ref["dos"], "RESS-DGC FP64 N_v=120")
    assert _l1(out["fp32"][0], ref["dos"]) <= 1e-3
    assert _l1(ref["dos"], exact) <= 1e-3
