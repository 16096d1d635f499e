"""Pins of the CPU oracle against facts the paper and the mathematics fix.

None of these tests compares the oracle with itself: each one checks it
against a printed value, a closed form, a theorem, or a dense
eigen-decomposition of a small matrix.
"""
import math

import numpy as np
import pytest
import scipy.special as sps

from oracle import ssm_oracle as O
from paper_1504_07690_amd import workloads as WL


# ----------------------------------------------------------------------------
# Inputs: Philox known answers, Gaussian moments, closed-form spectra
# ----------------------------------------------------------------------------
def test_philox_known_answers(golden):
    for ctr, key, want in golden["philox4x32_10_kat"]["vectors"]:
        c = [np.array([int(x, 16)], dtype=np.uint64) for x in ctr]
        got = WL.philox4x32_10(c, [int(x, 16) for x in key])
        assert ["%08x" % int(g[0]) for g in got] == want


def test_gaussian_block_moments():
    w = WL.gaussian_block(4096, 64, seed=123)
    assert abs(w.mean()) < 5e-3
    assert abs(w.var() - 1.0) < 1e-2
    # fourth moment 3 and independence of columns (off-diagonal of W^T W / n small)
    assert abs(np.mean(w ** 4) - 3.0) < 0.05
    g = w.T @ w / w.shape[0]
    assert np.abs(g - np.diag(np.diag(g))).max() < 0.08
    # columns do not depend on nv (same counter per (row, group))
    w2 = WL.gaussian_block(16, 20, seed=123)
    assert np.array_equal(w2, WL.gaussian_block(4096, 64, seed=123)[:16, :20])


def test_laplacian_closed_form_spectrum():
    a = WL.laplacian_2d_dirichlet(16)
    ev = np.linalg.eigvalsh(a.to_dense())
    assert np.allclose(ev, WL.laplace2d_dirichlet_eigenvalues(16), atol=1e-12)
    cfg1 = WL.make_matrix(1)
    assert cfg1.n == 1024 and cfg1.nnz == 4992


def test_anderson_zero_disorder_closed_form():
    a = WL.anderson_3d(6, None)
    ev = np.sort(np.linalg.eigvalsh(a.to_dense()))
    k = 2 * np.pi * np.arange(6) / 6
    ref = np.sort((-2 * (np.cos(k)[:, None, None] + np.cos(k)[None, :, None]
                         + np.cos(k)[None, None, :])).ravel())
    assert np.allclose(ev, ref, atol=1e-12)


# ----------------------------------------------------------------------------
# Section 2: Gaussian, exact DOS
# ----------------------------------------------------------------------------
def test_printed_range_bound(golden):
    ex = golden["g_max_example"]
    g = O.range_bound(ex["sigma"], ex["n"])
    assert abs(g - ex["value"]) < 0.5 * 10 ** (-3)  # printed to one digit: 0.008
    assert ex["spurious_xi"] > g                    # the printed spurious value lies outside


def test_exact_dos_unit_mass_and_closed_form():
    nx = 32
    lam = WL.laplace2d_dirichlet_eigenvalues(nx)
    n = lam.size
    lo, hi = -1.0, 9.0
    t = np.linspace(lo, hi, 4001)
    sigma = 0.1
    phi = O.exact_dos(lam, t, sigma)
    mass = np.trapezoid(phi, t)
    assert abs(mass - 1.0) < 1e-10
    # one eigenvalue: the Gaussian itself, value 1/(N sqrt(2 pi) sigma) at the centre
    assert np.isclose(O.exact_dos([0.3], [0.3], 0.2, n=7)[0], 1.0 / (7 * math.sqrt(2 * math.pi) * 0.2))


# ----------------------------------------------------------------------------
# Algorithm 1
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("sigma_hat,degree,n,lo,hi", [
    (0.05, 200, 1024, -1.0, 9.0),
    (0.01, 1000, 262144, -7.3, 5.1),
    (0.2, 40, 10, -1.0, 1.0),
])
def test_coefficients_bessel_at_centre(sigma_hat, degree, n, lo, hi):
    """At t = c0: g(-hw cos theta) = K exp(-z) exp(-z cos 2 theta), z = 1/(4 sigma^2),
    so by Jacobi-Anger mu_2m = (2 - delta_m0) K (-1)^m e^{-z} I_m(z), odd mu = 0."""
    c0, hw = 0.5 * (lo + hi), 0.5 * (hi - lo)
    sigma = sigma_hat * hw
    mu = O.dgc_coefficients([c0], degree, sigma, n, lo, hi)[:, 0]
    big_k = 1.0 / (n * math.sqrt(2 * math.pi) * sigma)
    z = 1.0 / (4 * sigma_hat ** 2)
    m = np.arange(0, degree // 2 + 1)
    ref_even = (2.0 - (m == 0)) * big_k * (-1.0) ** m * sps.ive(m, z)
    scale = big_k
    assert np.abs(mu[0::2] - ref_even).max() < 1e-13 * scale
    assert np.abs(mu[1::2]).max() < 1e-13 * scale


def test_coefficients_reconstruct_gaussian():
    """sum_l mu_l T_l(s) ~= g(t - x(s)); error below Theorem 2's bound and ~1e-12 g_max."""
    n, lo, hi = 1000, -2.0, 8.0
    hw = 0.5 * (hi - lo)
    for sigma_hat, degree in ((0.05, 200), (0.02, 500)):
        sigma = sigma_hat * hw
        t = np.array([-1.5, 0.0, 3.0, 7.9])
        mu = O.dgc_coefficients(t, degree, sigma, n, lo, hi)
        s = np.cos(np.linspace(0, math.pi, 3001))
        for i, ti in enumerate(t):
            err = np.abs(O.chebyshev_eval(mu[:, i], s) - O.g_sigma(ti - (0.5 * (lo + hi) + hw * s), sigma, n))
            gmax = O.range_bound(sigma, n)
            assert err.max() < 1e-12 * gmax
            # Theorem 2's bound on E_M in the rescaled variable, alpha = M sigma^;
            # |g| on the ellipse carries the prefactor g_max (the proof's bound
            # omits 1/sqrt(2 pi sigma^2); it is kept here).
            al = degree * sigma_hat
            bound = 2.0 * gmax * math.exp(0.5 * al * al) / (al * sigma_hat) * (1 + al * sigma_hat) ** (-degree)
            assert err.max() <= bound + 1e-14 * gmax


def test_coefficients_truncation_error_decays():
    """Dropping degree loses accuracy as Theorem 2 predicts (M ~ 1/sigma)."""
    n, lo, hi = 100, -1.0, 1.0
    sigma = 0.05
    t = [0.3]
    s = np.linspace(-1, 1, 2001)
    errs = []
    for degree in (20, 40, 80, 160):
        mu = O.dgc_coefficients(t, degree, sigma, n, lo, hi)
        errs.append(np.abs(O.chebyshev_eval(mu[:, 0], s) - O.g_sigma(0.3 - s, sigma, n)).max())
    assert errs[0] > errs[1] > errs[2] > errs[3]
    assert errs[3] < 1e-10 * O.range_bound(sigma, n)


# ----------------------------------------------------------------------------
# The recurrence
# ----------------------------------------------------------------------------
def _small_sym(n=60, seed=0):
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((n, n)) * (rng.random((n, n)) < 0.1)
    a = a + a.T + np.diag(rng.uniform(-3, 3, n))
    return a


def test_recurrence_matches_dense_chebyshev():
    a = _small_sym()
    lam, q = np.linalg.eigh(a)
    lo, hi = lam[0] - 0.7, lam[-1] + 1.3
    lt = (2 * lam - (lo + hi)) / (hi - lo)
    w = WL.gaussian_block(a.shape[0], 7, seed=5)
    for l, v in O.chebyshev_blocks(a, w, 50, lo, hi):
        ref = q @ (np.cos(l * np.arccos(lt))[:, None] * (q.T @ w))
        assert np.abs(v - ref).max() < 1e-11 * np.abs(w).max(), l


def test_recurrence_product_identity_and_bound():
    a = WL.make_matrix(1)
    lo, hi = WL.interval(a)
    w = WL.gaussian_block(a.n, 8, seed=9)
    ys = [v.copy() for _, v in O.chebyshev_blocks(a, w, 40, lo, hi)]
    x = [w.T @ y for y in ys]
    nw = np.linalg.norm(w)
    for j in (3, 11, 20):
        for k in (0, 5, 20):
            lhs = ys[j].T @ ys[k]
            rhs = 0.5 * (x[j + k] + x[abs(j - k)])
            assert np.abs(lhs - rhs).max() < 1e-10 * nw * nw
    assert max(np.linalg.norm(y) for y in ys) <= nw * (1 + 1e-12)


# ----------------------------------------------------------------------------
# Algorithm 4 and Theorem 3
# ----------------------------------------------------------------------------
def _low_rank_psd(n, r, seed, scale=1.0):
    rng = np.random.default_rng(seed)
    u, _ = np.linalg.qr(rng.standard_normal((n, r)))
    s = scale * rng.uniform(0.1, 1.0, r)
    return u, s


def test_theorem3_exact_low_rank():
    n, r, nv = 200, 10, 24
    u, s = _low_rank_psd(n, r, 1)
    p = (u * s) @ u.T
    w = WL.gaussian_block(n, nv, seed=3)
    z = p @ w
    k_w, k_z = O.gram(w, z)
    tr, r1, r2, parts = O.geneig_trace(k_w, k_z, g_max=10.0, tau=1e-10, return_parts=True)
    assert r1 == r and r2 == r
    assert abs(tr - s.sum()) < 1e-10 * s.sum()
    kept = np.sort(parts["xi"][(parts["xi"] >= 0) & (parts["xi"] <= 10.0)])
    assert np.allclose(kept, np.sort(s), rtol=1e-9)


def test_range_filter_drops_out_of_range_value():
    """A generalized eigenvalue above 1/(N sqrt(2 pi sigma^2)) is discarded (Section 3.2)."""
    n, r, nv = 200, 6, 20
    u, s = _low_rank_psd(n, r, 2, scale=0.005)
    s[0] = 0.033                           # the paper's spurious value, above g_max = 0.008
    p = (u * s) @ u.T
    w = WL.gaussian_block(n, nv, seed=4)
    k_w, k_z = O.gram(w, p @ w)
    g_max = O.range_bound(0.05, 1000)
    tr, r1, r2 = O.geneig_trace(k_w, k_z, g_max=g_max, tau=1e-10)
    assert r1 == r and r2 == r - 1
    assert abs(tr - s[1:].sum()) < 1e-9 * s.sum()


def test_truncation_keeps_nothing_for_nonpositive_kw():
    k = -np.eye(5)
    assert O.geneig_trace(k, np.eye(5), g_max=1.0) == (0.0, 0, 0)


def test_truncation_threshold_inclusive():
    k_w = np.diag([1.0, 1e-7, 0.99e-7, -1.0])
    k_z = np.diag([0.5, 0.5e-7, 0.5e-7, 1.0])
    tr, r1, r2 = O.geneig_trace(k_w, k_z, g_max=1.0, tau=1e-7)
    assert r1 == 2 and r2 == 2 and abs(tr - 1.0) < 1e-12


# ----------------------------------------------------------------------------
# Algorithm 5 end to end
# ----------------------------------------------------------------------------
def test_identity_probe_reproduces_exact_dos():
    """With W = I_N, K_W = g^M(tI-A) and K_Z = K_W^2, so Algorithm 4 returns the sum
    of the kept eigenvalues of g^M(tI-A): the exact regularised DOS up to the
    Chebyshev truncation (Theorem 2) and the tau-dropped Gaussian tail."""
    rng = np.random.default_rng(11)
    a = WL.laplacian_2d_dirichlet(16, rng.uniform(-1, 1, 256))
    lo, hi = WL.interval(a)
    hw = 0.5 * (hi - lo)
    lam = np.linalg.eigvalsh(a.to_dense())
    sigma = 0.05 * hw
    t = 0.5 * (lo + hi) + hw * WL.midpoint_grid(40)
    out = O.ss_dgc(a, np.eye(a.n), t, 200, sigma, lo, hi)
    ref = O.exact_dos(lam, t, sigma)
    gmax = O.range_bound(sigma, a.n)
    assert np.abs(out["dos"] - ref).max() < 1e-6 * ref.max()
    # the dropped tail is below tau * max per eigenvalue: count it
    assert np.all(out["dos"] <= ref + 1e-9 * gmax)


def test_dgc_identity_probe_reproduces_exact_dos():
    """Algorithm 2 with W = sqrt(N) I_N (N_v = N, W W^T = N_v I, the case in which the
    Hutchinson average of Theorem 1 has no variance): zeta_l = Tr T_l(A~) exactly, so the
    DGC estimate is the Chebyshev expansion of the regularised DOS itself, equal to it up
    to the truncation of Theorem 2."""
    rng = np.random.default_rng(12)
    a = WL.laplacian_2d_dirichlet(14, rng.uniform(-1, 1, 196))
    lo, hi = WL.interval(a)
    hw = 0.5 * (hi - lo)
    lam = np.linalg.eigvalsh(a.to_dense())
    sigma = 0.05 * hw
    t = 0.5 * (lo + hi) + hw * WL.midpoint_grid(40)
    ref = O.exact_dos(lam, t, sigma)
    probe = np.sqrt(a.n) * np.eye(a.n)
    out = O.dgc_dos(a, probe, t, 200, sigma, lo, hi)
    assert np.abs(out - ref).max() < 1e-8 * ref.max()
    # a truncated expansion is visibly worse: the degree matters
    coarse = O.dgc_dos(a, probe, t, 20, sigma, lo, hi)
    assert np.abs(coarse - ref).max() > 1e-3 * ref.max()


@pytest.mark.slow
def test_ssm_beats_dgc_when_sampled_enough():
    """Section 3.2 / Fig. 6: once N_v exceeds the numerical rank of g(tI - A),
    SS-DGC is far more accurate than the Hutchinson-type DGC with the same W."""
    a = WL.make_matrix(1)
    lo, hi = WL.interval(a)
    hw = 0.5 * (hi - lo)
    sigma = 0.01 * hw
    degree, nv = 1000, 120
    lam = np.linalg.eigvalsh(a.to_dense())
    t = 0.5 * (lo + hi) + hw * np.linspace(-0.6, 0.6, 12)
    w = WL.gaussian_block(a.n, nv, seed=77)
    ssm = O.ss_dgc(a, w, t, degree, sigma, lo, hi)["dos"]
    dgc = O.dgc_dos(a, w, t, degree, sigma, lo, hi)
    ref = O.exact_dos(lam, t, sigma)
    e_ssm = np.abs(ssm - ref).sum() / np.abs(ref).sum()
    e_dgc = np.abs(dgc - ref).sum() / np.abs(ref).sum()
    assert e_ssm < 1e-3
    assert e_ssm < 0.05 * e_dgc


# ----------------------------------------------------------------------------
# Section 4: RESS-DGC
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("half,nt", [(0, 1), (1, 2), (5, 3), (40, 4)])
def test_square_coefficients_product_identity(half, nt):
    """Proposition 1 against the closed form from T_p T_q = (T_{p+q} + T_{|p-q|})/2:
    nu_l = 1/2 sum_{p+q=l} mu_p mu_q + 1/2 sum_{|p-q|=l} mu_p mu_q, and the squared series
    at points of [-1, 1]."""
    rng = np.random.default_rng(half + 7)
    mu = rng.standard_normal((half + 1, nt)) / (1.0 + np.arange(half + 1))[:, None]
    degree = 2 * half
    nu = O.square_coefficients(mu, degree)
    ref = np.zeros((degree + 1, nt))
    for p in range(half + 1):
        for q in range(half + 1):
            ref[p + q] += 0.5 * mu[p] * mu[q]
            ref[abs(p - q)] += 0.5 * mu[p] * mu[q]
    scale = np.abs(mu).sum(axis=0) ** 2
    assert np.all(np.abs(nu - ref) <= 1e-14 * scale)
    x = np.cos(rng.uniform(0, np.pi, 9))[:, None]
    assert np.all(np.abs(O.chebyshev_eval(nu, x) - O.chebyshev_eval(mu, x) ** 2) <= 1e-13 * scale)


def _ress_case(nx=14, nv=16, degree=200, nt=30, sigma_hat=0.05, seed=3):
    rng = np.random.default_rng(seed)
    a = WL.laplacian_2d_dirichlet(nx, rng.uniform(-1, 1, nx * nx))
    lo, hi = WL.interval(a)
    hw = 0.5 * (hi - lo)
    t = 0.5 * (lo + hi) + hw * WL.midpoint_grid(nt)
    return a, lo, hi, sigma_hat * hw, t, WL.gaussian_block(a.n, nv, seed=seed), degree


def test_ress_equals_ss_dgc_at_half_degree():
    """Theorem 4 with N~_v = 0: K_W = W^* Z and K_Z = Z^* Z for Z = g^{M/2}(tI - A) W,
    so RESS-DGC at degree M is SS-DGC at degree M/2 with the same (truncated) mu.
    In the bulk (above 1e-2 of the maximum) the two agree to rounding.  Towards the
    spectrum's edges both carry rounding noise of different origin (K_Z as a sum of
    moments that cancel, against Z^* Z of a noisy Z), amplified by Algorithm 4's
    S~^{-1/2}, and agree only to that level."""
    a, lo, hi, sigma, t, w, m = _ress_case()
    ress = O.ress_dgc(a, w, None, t, m, sigma, lo, hi)
    ss = O.ss_dgc(a, w, t, m // 2, sigma, lo, hi, mu=ress["mu"][: m // 2 + 1], keep=True)
    top = ss["dos"].max()
    resolved = ss["dos"] > 1e-4 * top
    assert resolved.sum() >= 20
    diff = np.abs(ress["dos"] - ss["dos"])
    assert diff[ss["dos"] > 0.5 * top].max() <= 1e-13 * top
    assert diff[ss["dos"] > 1e-2 * top].max() <= 1e-8 * top
    assert diff[resolved].max() <= 1e-7 * top
    assert np.abs(ress["dos"] - ss["dos"]).max() <= 1e-4 * top
    assert np.array_equal(ress["r1"][resolved], ss["r1"][resolved])
    kz = ss["k_z"]
    assert np.abs(ress["k_z"] - kz).max() <= 1e-11 * np.abs(kz).max()


def test_ress_hybrid_identity_probe_gives_exact_trace():
    """Algorithm 6 with W~ = sqrt(N) I_N (no Hutchinson variance): the correction is
    Tr g^{M/2}(tI - A) - Tr Xi~ exactly, so the estimate is the exact regularised DOS up
    to the degree-M/2 truncation, whatever W (here N_v = 8, far below the rank).  At the
    spectrum's edges Tr Xi~ carries the rounding noise of the moment form of K_Z."""
    a, lo, hi, sigma, t, w, m = _ress_case(nv=8, degree=400, nt=25, sigma_hat=0.05)
    probe = np.sqrt(a.n) * np.eye(a.n)
    out = O.ress_dgc(a, w, probe, t, m, sigma, lo, hi)
    ref = O.exact_dos(np.linalg.eigvalsh(a.to_dense()), t, sigma)
    resolved = ref > 1e-4 * ref.max()
    assert resolved.sum() >= 20
    assert np.abs(out["dos"] - ref)[resolved].max() < 1e-8 * ref.max()
    assert np.abs(out["dos"] - ref).max() < 1e-4 * ref.max()
    plain = O.ress_dgc(a, w, None, t, m, sigma, lo, hi)["dos"]
    assert np.abs(plain - ref).max() > 1e-2 * ref.max()  # N_v = 8 alone misses mass


def test_ress_floor_silences_points_outside_the_spectrum():
    """Sweep points outside the spectrum of a clean 8^3 lattice, where g(tI - A) is below
    1e-12 of its maximum: K_W and K_Z are rounding noise there, and without the rounding
    floor of the truncation the pencil reports a fifth of the maximum; with it, nothing."""
    a = WL.anderson_3d(8, np.zeros(512))
    lam = np.linalg.eigvalsh(a.to_dense())
    lo, hi = WL.interval(a)
    hw = 0.5 * (hi - lo)
    sigma = 0.01 * hw
    t = 0.5 * (lo + hi) + hw * WL.midpoint_grid(60)
    ref = O.exact_dos(lam, t, sigma)
    out = ref < 1e-12 * ref.max()
    assert out.sum() >= 2
    w = WL.gaussian_block(a.n, 40, seed=4)
    with_floor = O.ress_dgc(a, w, None, t, 600, sigma, lo, hi)["dos"]
    without = O.ress_dgc(a, w, None, t, 600, sigma, lo, hi, eta=0.0)["dos"]
    assert np.abs(with_floor[out]).max() <= 1e-9 * ref.max()
    assert np.abs(without[out]).max() > 1e-2 * ref.max()


@pytest.mark.parametrize("which", ["stencil8", "lap16"])
def test_rounding_floor_covers_fp32_sweep_error(which):
    """The rounding floor of Algorithm 4's truncation against a sweep carried out in FP32
    arithmetic (float32 coefficients and blocks, float32 matrix product) on two small
    matrices whose interval leaves 20 sigma of empty margin.  Pins of the floor's formula:
    - at the points where the exact regularised DOS is below 1e-12 of its maximum, the
      floor at eta = 2^-22 lies between 1 and 10 times the measured error
      ||K_W(FP32 Z) - K_W(FP64 Z)||_2 (a factor of N, N_v or ||W||_F off would miss by far);
    - there the FP32 estimate without the floor reports rounding (far above the FP64
      estimate's 1e-13 of the maximum) and with it exactly 0;
    - at the resolved points the floor stays below 1e-5 of max s, and the relative L1
      against the FP64 estimate does not grow."""
    if which == "stencil8":
        a, nv = WL.stencil27_lognormal(8, np.random.default_rng(5)), 48
    else:
        a, nv = WL.laplacian_2d_dirichlet(16, np.random.default_rng(3).uniform(-1, 1, 256)), 32
    m, nt = 2000, 128
    wl = WL.make_workload(1, a=a, nv=nv, degree=m, nt=nt, sigma_hat=0.005)
    w = wl.w()
    n = a.n
    mu = O.dgc_coefficients(wl.t, m, wl.sigma, n, wl.lo, wl.hi)
    ys = np.array([v for _, v in O.chebyshev_blocks(a, w, m, wl.lo, wl.hi)]).reshape(m + 1, -1)
    z64 = (mu.T @ ys).reshape(nt, n, nv)
    z32 = (mu.astype(np.float32).T @ ys.astype(np.float32)).astype(np.float64).reshape(nt, n, nv)
    gmax = O.range_bound(wl.sigma, n)
    ex = O.exact_dos(np.linalg.eigvalsh(a.to_dense()), wl.t, wl.sigma)
    empty = ex < 1e-12 * ex.max()
    assert empty.sum() >= 20
    fl = O.rounding_floor(mu, w, 2.0 ** -22)
    d64, d0, df, noise, smax = (np.zeros(nt) for _ in range(5))
    for i in range(nt):
        k64, k32 = O.gram(w, z64[i]), O.gram(w, z32[i])
        noise[i] = np.linalg.norm(k32[0] - k64[0], 2)
        smax[i] = np.linalg.eigvalsh(k64[0]).max()
        d64[i] = O.geneig_trace(*k64, gmax)[0]
        d0[i] = O.geneig_trace(*k32, gmax)[0]
        df[i] = O.geneig_trace(*k32, gmax, s_floor=fl[i])[0]
    ratio = fl[empty] / noise[empty]
    assert ratio.min() >= 1.0 and ratio.max() <= 10.0, (ratio.min(), ratio.max())
    assert d64[empty].max() <= 1e-13 * d64.max()
    assert d0[empty].max() >= 1e-8 * d64.max()
    assert np.all(df[empty] == 0.0)
    resolved = d64 > 1e-2 * d64.max()
    assert np.all(fl[resolved] <= 1e-5 * smax[resolved])
    l1 = lambda x: np.abs(x - d64).sum() / np.abs(d64).sum()
    assert l1(df) <= l1(d0) <= 1e-5


def test_ress_correction_vanishes_when_sampled_enough():
    """With N_v above the numerical rank the low-rank part is exact (Theorem 3), so the
    hybrid correction is at rounding level and both estimates agree."""
    a, lo, hi, sigma, t, w, m = _ress_case(nv=150, degree=400, nt=12, sigma_hat=0.05)
    wt = WL.gaussian_block(a.n, 8, seed=99)
    with_c = O.ress_dgc(a, w, wt, t, m, sigma, lo, hi)["dos"]
    plain = O.ress_dgc(a, w, None, t, m, sigma, lo, hi)["dos"]
    resolved = plain > 1e-4 * plain.max()
    assert np.abs(with_c - plain)[resolved].max() <= 1e-6 * plain.max()


# ----------------------------------------------------------------------------
# Algorithm 8
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("name", ["x", "x2", "exp"])
def test_trace_weights_exact_dos(name):
    """With the exact phi_sigma, sum_i w_i phi_sigma(t_i) reproduces Tr f(A)
    (Eq. traceconv): Tr A = sum a_ii, Tr A^2 = sum a_ij^2, and exp from the spectrum."""
    a = WL.make_matrix(1)
    dense = a.to_dense()
    lo, hi = WL.interval(a)
    hw = 0.5 * (hi - lo)
    lam = np.linalg.eigvalsh(dense)
    # sigma^ = 0.005: the window's Fourier transform (width sigma~ = 0.016) decays
    # faster than the Gaussian's, the condition Section 5 places on f.
    nt = 1000
    sigma = 0.005 * hw
    t = 0.5 * (lo + hi) + hw * WL.midpoint_grid(nt)
    phi = O.exact_dos(lam, t, sigma)
    f, ref = {
        "x": (lambda x: x, np.trace(dense)),
        "x2": (lambda x: x * x, np.sum(dense * dense)),
        "exp": (lambda x: np.exp(-0.5 * x), np.exp(-0.5 * lam).sum()),
    }[name]
    w = O.trace_weights(f, a.n, lo, hi, nt, sigma)
    assert abs(w @ phi - ref) < 1e-12 * abs(ref)


@pytest.mark.parametrize("beta", [0.0, 0.3, 1.0])
def test_trace_weights_exp_exact_dos(beta):
    """The real-line deconvolution for exp(-beta x): applied to the exact regularised DOS of
    a 27-point lognormal stencil it returns sum_j exp(-beta lambda_j) (beta = 0: N, the
    DOS's unit mass), the midpoint rule on Gaussian integrands being exact to rounding once
    the step is below sigma."""
    a = WL.stencil27_lognormal(8, np.random.default_rng(5))
    lam = np.linalg.eigvalsh(a.to_dense())
    lo, hi = WL.interval(a)
    sigma = 0.005 * 0.5 * (hi - lo)
    nt = 2000
    t = lo + (hi - lo) / nt * (np.arange(nt) + 0.5)
    w = O.trace_weights_exp(beta, a.n, lo, hi, nt, sigma)
    exact = np.exp(-beta * lam).sum()
    assert abs(w @ O.exact_dos(lam, t, sigma) - exact) <= 1e-12 * exact
    # cut below a lower bound of the spectrum (here the Gershgorin one): still exact
    g_lo, _ = WL.gershgorin(a)
    wc = O.trace_weights_exp(beta, a.n, lo, hi, nt, sigma, spec_lo=g_lo)
    assert np.count_nonzero(wc) < nt
    assert abs(wc @ O.exact_dos(lam, t, sigma) - exact) <= 1e-12 * exact
    # a grid too coarse for sigma loses it: the step matters
    coarse = O.trace_weights_exp(beta, a.n, lo, hi, 150, 0.02 * 0.5 * (hi - lo))
    tc = lo + (hi - lo) / 150 * (np.arange(150) + 0.5)
    if beta > 0:
        assert abs(coarse @ O.exact_dos(lam, tc, 0.02 * 0.5 * (hi - lo)) - exact) > 1e-6 * exact


def test_trace_weights_gaussian_semigroup():
    """h a Gaussian of width s > sigma: the deconvolved f~ is the Gaussian of width
    sqrt(s^2 - sigma^2) (Eq. deconvolv), checked on the grid."""
    lo, hi, nt = -1.0, 1.0, 512
    sigma, s = 0.02, 0.05
    f = lambda x: np.exp(-x * x / (2 * s * s)) / math.sqrt(2 * math.pi * s * s)
    w = O.trace_weights(f, 1, lo, hi, nt, sigma)
    t = WL.midpoint_grid(nt)
    f_tilde = w / (2.0 / nt)
    r = math.sqrt(s * s - sigma * sigma)
    ref = np.exp(-t * t / (2 * r * r)) / math.sqrt(2 * math.pi * r * r)
    # rounding noise in h^ is amplified by at most 1/eta = 1e10 at the cutoff
    assert np.abs(f_tilde - ref).max() < 1e-6 * ref.max()


# ----------------------------------------------------------------------------
# Gradient reference: central differences of the oracle
# ----------------------------------------------------------------------------
def _sym_direction(a, seed):
    """A symmetric perturbation of the stored values (the (r, c) and (c, r) entries equal)."""
    rng = np.random.default_rng(seed)
    d = rng.standard_normal(a.nnz)
    m = sp_csr(a, d)
    m = 0.5 * (m + m.T)
    m = m.tocsr()
    m.sort_indices()
    return np.asarray(m[np.repeat(np.arange(a.n), np.diff(a.row_ptr)), a.col_idx]).ravel()


def sp_csr(a, vals):
    import scipy.sparse as sp
    return sp.csr_matrix((vals, a.col_idx, a.row_ptr), shape=(a.n, a.n))


@pytest.mark.slow
def test_oracle_trace_gradient_matches_fprime():
    """With W = I the SS-DGC trace of f is Tr f(A) up to the expansion, truncation and
    deconvolution errors, so its derivative along a symmetric direction E is
    Tr(f'(A) E): central differences of the oracle against the dense eigen-decomposition."""
    rng = np.random.default_rng(4)
    a = WL.laplacian_2d_dirichlet(8, rng.uniform(-1, 1, 64))
    lo, hi = WL.interval(a)
    hw = 0.5 * (hi - lo)
    nt, degree, sigma = 900, 1200, 0.005 * hw
    t = 0.5 * (lo + hi) + hw * WL.midpoint_grid(nt)
    f = lambda x: np.exp(-0.5 * x)
    w = O.trace_weights(f, a.n, lo, hi, nt, sigma)
    e = _sym_direction(a, 1)
    h = 1e-5

    def tr(vals):
        b = WL.CSR(a.n, a.row_ptr, a.col_idx, vals)
        return w @ O.ss_dgc(b, np.eye(a.n), t, degree, sigma, lo, hi)["dos"]

    fd = (tr(a.values + h * e) - tr(a.values - h * e)) / (2 * h)
    lam, q = np.linalg.eigh(a.to_dense())
    fprime = (q * (-0.5 * np.exp(-0.5 * lam))) @ q.T
    exact = np.sum(fprime * sp_csr(a, e).toarray())
    assert abs(fd - exact) <= 1e-6 * abs(exact)
