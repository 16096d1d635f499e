"""The DGC estimate of Algorithm 2 formed during the SS-DGC recurrence, through the C ABI.

The device takes the moments from inner products of consecutive Chebyshev blocks
(N_v zeta_{2s} = 2 <Y_s, Y_s> - N_v zeta_0, N_v zeta_{2s+1} = 2 <Y_{s+1}, Y_s> - N_v
zeta_1); the oracle takes zeta_l = Tr[W^T T_l(A~) W]/N_v directly, block by block.
Gates: FP64 1e-9 of the largest value (rounding order only: the two forms agree to
1e-14 in FP64 on the host); the FP32 recurrence 1e-5 of the largest value (the same
forms with an FP32 recurrence agree to 1e-7 on the host, 100x margin).  The moments
obey |zeta_l| <= zeta_0 at any size (|T_l| <= 1 on [-1, 1]).
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


def _moments(a, w, degree, lo, hi):
    zeta = np.zeros(degree + 1)
    for l, v_c in O.chebyshev_blocks(a, w, degree, lo, hi):
        zeta[l] = np.sum(w * v_c) / w.shape[1]
    return zeta


def _ctx(S, wl, precision, budget=0, dgc=True, t=None):
    dt = torch.float64 if precision == "fp64" else torch.float32
    csr = S.DeviceCSR.from_csr(wl.a, dtype=dt, device=DEV)
    w = torch.tensor(wl.w(), dtype=dt, device=DEV)
    ctx = S.SSM(csr, lo=wl.lo, hi=wl.hi, sigma=wl.sigma, nv=wl.nv, degree=wl.degree,
                t=wl.t if t is None else t, precision=precision, seed=wl.seed, w=w, budget=budget, dgc=dgc,
                device=DEV)
    return csr, w, ctx


@pytest.fixture(scope="module")
def cfg1_dgc():
    wl = WL.make_workload(1)
    w = wl.w()
    return wl, O.dgc_dos(wl.a, w, wl.t, wl.degree, wl.sigma, wl.lo, wl.hi), \
        _moments(wl.a, w, wl.degree, wl.lo, wl.hi)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-9), ("fp32", 1e-5), ("bf16x3", 1e-5)])
def test_dgc_matches_oracle(S, cfg1_dgc, precision, tol):
    wl, ref, zeta_ref = cfg1_dgc
    csr, w, ctx = _ctx(S, wl, precision)
    ctx.dos()
    dgc, zeta = ctx.dgc()
    ctx.close()
    err = np.abs(dgc - ref).max() / np.abs(ref).max()
    zerr = np.abs(zeta - zeta_ref).max() / zeta_ref[0]
    print(f"{precision}: DGC max err {err:.2e} of max, moments {zerr:.2e} of zeta_0")
    assert err <= tol
    assert zerr <= tol
    assert np.all(np.abs(zeta) <= zeta[0] * (1 + 1e-6))


def test_dgc_leaves_ssm_unchanged_and_survives_small_plans(S, cfg1_dgc):
    """The moments ride on the recurrence of pass 0: the SS-DGC estimate is the same with
    or without them, and a budget that forces several passes and a ring of blocks (the
    moments of 101 steps reduced in groups) gives the same DGC estimate."""
    wl, ref, _ = cfg1_dgc
    csr, w, ctx = _ctx(S, wl, "fp64", dgc=False)
    plain, _, _ = ctx.dos()
    ctx.close()
    csr, w, ctx = _ctx(S, wl, "fp64")
    with_dgc, _, _ = ctx.dos()
    full, _ = ctx.dgc()
    ctx.close()
    assert np.abs(with_dgc - plain).max() <= 1e-12 * plain.max()
    csr, w, ctx = _ctx(S, wl, "fp64", budget=110 * 1024 * 1024)
    st = ctx.stats()
    ctx.dos()
    small, _ = ctx.dgc()
    ctx.close()
    assert st["passes"] > 1 or st["chunk"] < wl.degree + 1, st
    assert np.abs(small - full).max() <= 1e-12 * np.abs(full).max()
    assert np.abs(small - ref).max() <= 1e-9 * np.abs(ref).max()


@pytest.mark.parametrize("degree", [1, 2, 3, 64, 129])
def test_dgc_degrees_and_ragged_block(S, degree):
    """M = 1 (zeta_0, zeta_1 from the first step alone), even and odd M, and a block
    whose row count is not a multiple of a workgroup's rows (N = 397, N_v = 12)."""
    rng = np.random.default_rng(degree)
    n = 397
    import scipy.sparse as sp
    m = (rng.random((n, n)) < 0.02) * rng.standard_normal((n, n))
    m = np.triu(m, 1)
    m = sp.csr_matrix(m + m.T + np.diag(rng.uniform(-2, 2, n)))
    m.sort_indices()
    a = WL.CSR(n, m.indptr.astype(np.int32), m.indices.astype(np.int32), m.data.astype(np.float64))
    wl = WL.make_workload(1, a=a, nv=12, degree=degree, nt=37, sigma_hat=0.2)
    ref = O.dgc_dos(a, wl.w(), wl.t, degree, wl.sigma, wl.lo, wl.hi)
    zeta_ref = _moments(a, wl.w(), degree, wl.lo, wl.hi)
    for precision, tol in (("fp64", 1e-9), ("fp32", 1e-5)):
        csr, w, ctx = _ctx(S, wl, precision)
        ctx.dos()
        dgc, zeta = ctx.dgc()
        ctx.close()
        assert zeta.shape == (degree + 1,)
        assert np.abs(zeta - zeta_ref).max() <= tol * zeta_ref[0], precision
        assert np.abs(dgc - ref).max() <= tol * np.abs(ref).max(), precision


def test_dgc_state_errors(S):
    from paper_1504_07690_amd import _abi as A
    wl = WL.make_workload(1, nv=8, degree=16, nt=8)
    csr, w, ctx = _ctx(S, wl, "fp64", dgc=False)
    with pytest.raises(A.SSMError) as ei:
        ctx.dgc()
    assert ei.value.status == A.SSM_ERR_STATE
    ctx.close()
    csr, w, ctx = _ctx(S, wl, "fp64")
    with pytest.raises(A.SSMError) as ei:
        ctx.dgc()  # before ssm_dos
    assert ei.value.status == A.SSM_ERR_STATE
    ctx.dos()
    ctx.dgc()
    ctx.close()


def test_ssm_beats_dgc_on_device(S):
    """Section 3.2: with N_v above the numerical rank of g(tI - A) the SS-DGC estimate is
    far closer to the exact regularised DOS than DGC on the same W, both from one
    recurrence on the device."""
    a = WL.make_matrix(1)
    lo, hi = WL.interval(a)
    hw = 0.5 * (hi - lo)
    wl = WL.make_workload(1, a=a, nv=120, degree=1000, nt=12, sigma_hat=0.01)
    t = 0.5 * (lo + hi) + hw * np.linspace(-0.6, 0.6, 12)
    ref = O.exact_dos(np.linalg.eigvalsh(a.to_dense()), t, wl.sigma)
    csr, w, ctx = _ctx(S, wl, "fp64", t=t)
    ssm, _, _ = ctx.dos()
    dgc, _ = ctx.dgc()
    ctx.close()
    e_ssm = np.abs(ssm - ref).sum() / np.abs(ref).sum()
    e_dgc = np.abs(dgc - ref).sum() / np.abs(ref).sum()
    print(f"L1 error vs the exact DOS: SS-DGC {e_ssm:.2e}, DGC {e_dgc:.2e}")
    assert e_ssm < 1e-3
    assert e_ssm < 0.05 * e_dgc
