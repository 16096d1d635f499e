"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Stage by stage on seeded inputs whose sizes span several tiles with ragged
tails, then end to end.  Tolerances:
* FP64 stages: rounding-order differences only (1e-12 .. 1e-13 relative);
* FP32 recurrence/sweep: FP32 rounding, and the DOS within 1e-3 relative L1
  of the FP64 oracle (the DOS tolerance of the method's mixed-precision mode);
* Gram, Algorithm 4: FP64 throughout, compared on identical inputs.
"""
import math

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


def _rng(seed):
    return np.random.default_rng(seed)


def _rand_sym_csr(n, density, seed):
    rng = _rng(seed)
    m = (rng.random((n, n)) < density) * rng.standard_normal((n, n))
    m = np.triu(m, 1)
    m = m + m.T + np.diag(rng.uniform(-2, 2, n))
    import scipy.sparse as sp
    c = sp.csr_matrix(m)
    c.sort_indices()
    return WL.CSR(n, c.indptr.astype(np.int32), c.indices.astype(np.int32), c.data.astype(np.float64))


def bf16_round(x):
    """float32 -> bfloat16 -> float32 with round-to-nearest-even (finite inputs)."""
    b = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32)


# ----------------------------------------------------------------------------
# W
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("n,nv", [(1001, 36), (5, 4), (3000, 80)])
def test_gaussian_block_matches_input_generator(S, dtype, n, nv):
    w = torch.empty(n, nv, dtype=dtype, device=DEV)
    S.gaussian_block(0xABCDEF0123, w)
    ref = WL.gaussian_block(n, nv, 0xABCDEF0123)
    got = w.cpu().numpy().astype(np.float64)
    if dtype == torch.float64:
        assert np.abs(got - ref).max() <= 1e-14 * max(1.0, np.abs(ref).max())
    else:
        assert np.abs(got - ref.astype(np.float32)).max() <= 2 ** -22 * np.abs(ref).max()


# ----------------------------------------------------------------------------
# Algorithm 1
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("lo,hi,n,sigma_hat,degree,nt", [
    (-0.999, 8.998, 1024, 0.05, 200, 200),      # the 32x32 workload's interval
    (-8.9, 8.9, 262144, 0.01, 1000, 97),         # the 64^3 Anderson workload's scale
    (-1.0, 1.0, 10, 0.3, 3, 5),
    (0.0, 40.0, 2097152, 0.005, 4000, 33),       # largest degree the build supports
])
def test_coefficients(S, lo, hi, n, sigma_hat, degree, nt):
    hw = 0.5 * (hi - lo)
    sigma = sigma_hat * hw
    t = 0.5 * (lo + hi) + hw * WL.midpoint_grid(nt)
    td = torch.tensor(t, dtype=torch.float64, device=DEV)
    c = torch.empty(degree + 1, nt, dtype=torch.float64, device=DEV)
    c32 = torch.empty(degree + 1, nt, dtype=torch.float32, device=DEV)
    S.coefficients(lo, hi, sigma, n, td, degree, c, c32)
    ref = O.dgc_coefficients(t, degree, sigma, n, lo, hi)
    gmax = O.range_bound(sigma, n)
    assert np.abs(c.cpu().numpy() - ref).max() <= 1e-12 * gmax
    assert np.array_equal(c32.cpu().numpy(), c.cpu().numpy().astype(np.float32))


# ----------------------------------------------------------------------------
# The recurrence
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("which", ["cfg1", "ragged"])
def test_chebyshev(S, precision, which):
    if which == "cfg1":
        a = WL.make_matrix(1)
        nv, degree = 8, 60
    else:
        a = _rand_sym_csr(777, 0.01, 3)
        nv, degree = 12, 45
    lo, hi = WL.interval(a)
    dt = torch.float64 if precision == "fp64" else torch.float32
    w = WL.gaussian_block(a.n, nv, 17)
    if dt == torch.float32:
        w = w.astype(np.float32).astype(np.float64)
    csr = S.DeviceCSR.from_csr(a, dtype=dt, device=DEV)
    wd = torch.tensor(w, dtype=dt, device=DEV)
    y = torch.empty(degree + 1, a.n, nv, dtype=dt, device=DEV)
    S.chebyshev(csr, lo, hi, precision, wd, y)
    got = y.cpu().numpy().astype(np.float64)
    tol = 1e-12 if precision == "fp64" else 2e-5
    scale = np.abs(w).max()
    for l, v in O.chebyshev_blocks(a, w, degree, lo, hi):
        assert np.abs(got[l] - v).max() <= tol * scale * max(1, l), l


# ----------------------------------------------------------------------------
# The sweep
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16"])
@pytest.mark.parametrize("kc,ntb,ldc,n,nv", [(37, 45, 48, 250, 12), (16, 128, 128, 64, 8), (1, 3, 4, 33, 4),
                                               (70, 200, 200, 130, 40)])
def test_sweep(S, precision, kc, ntb, ldc, n, nv):
    rng = _rng(kc * 1000 + ntb)
    dt = torch.float64 if precision == "fp64" else torch.float32
    c = rng.standard_normal((kc, ldc))
    y = rng.standard_normal((kc, n, nv))
    z0 = rng.standard_normal((ntb, n, nv))
    if dt == torch.float32:
        c, y, z0 = (x.astype(np.float32).astype(np.float64) for x in (c, y, z0))
    cd = torch.tensor(c, dtype=dt, device=DEV)
    yd = torch.tensor(y, dtype=dt, device=DEV)
    zd = torch.tensor(z0, dtype=dt, device=DEV)
    ci, yi = (c, y) if precision != "bf16" else (bf16_round(c).astype(np.float64), bf16_round(y).astype(np.float64))
    ref = O.sweep(ci[:, :ntb], iter(yi))
    mag = O.sweep(np.abs(ci[:, :ntb]), iter(np.abs(yi)))
    tol = (kc + 2) * (2.0 ** -53 if precision == "fp64" else 2.0 ** -24)
    S.sweep(precision, cd, yd, zd, accumulate=False)
    assert np.all(np.abs(zd.cpu().numpy() - ref) <= tol * mag + 1e-300)
    zd = torch.tensor(z0, dtype=dt, device=DEV)
    S.sweep(precision, cd, yd, zd, accumulate=True)
    assert np.all(np.abs(zd.cpu().numpy() - (ref + z0)) <= tol * (mag + np.abs(z0)) + 1e-300)


def bf16_from_f64(x):
    """double -> bfloat16 (8 significant bits), one rounding, ties to even."""
    m, e = np.frexp(np.asarray(x, dtype=np.float64))
    return np.ldexp(np.rint(m * 256.0) / 256.0, e)


def bf16_split(x):
    """hi = bf16(x), lo = bf16(x - hi) for float32 x (both round to nearest even)."""
    x = np.asarray(x, dtype=np.float32)
    hi = bf16_round(x)
    lo = bf16_round((x - hi).astype(np.float32))
    return hi.astype(np.float64), lo.astype(np.float64)


@pytest.mark.parametrize("kc,ntb,m1,n,nv", [(37, 45, 37, 250, 12), (16, 300, 40, 64, 8), (1, 3, 8, 33, 4),
                                            (70, 257, 1001, 130, 40)])
def test_sweep_split_bf16(S, kc, ntb, m1, n, nv):
    """bf16x3 sweep: the oracle's sweep applied to the split operands
    (Chi Yhi + Chi Ylo + Clo Yhi), against the device's split tables and kernel."""
    rng = _rng(kc * 7 + ntb)
    ldc = (ntb + 3) // 4 * 4
    ldk = (m1 + 7) // 8 * 8
    c = rng.standard_normal((m1, ldc))
    y = rng.standard_normal((kc, n, nv)).astype(np.float32).astype(np.float64)
    z0 = rng.standard_normal((ntb, n, nv)).astype(np.float32).astype(np.float64)
    cd = torch.tensor(c, device=DEV)
    chi, clo = S.split_coefficients(cd, ntb, ldk)
    # the tables against their definition
    hi = bf16_from_f64(c[:, :ntb])
    lo = bf16_from_f64(c[:, :ntb] - hi)
    assert np.array_equal(chi.float().cpu().numpy()[:, :m1].T, hi)
    assert np.array_equal(clo.float().cpu().numpy()[:, :m1].T, lo)
    assert not chi.float().cpu().numpy()[:, m1:].any()
    yhi, ylo = bf16_split(y)
    mu_h, mu_l = hi[:kc], lo[:kc]
    ref = O.sweep(mu_h, iter(yhi)) + O.sweep(mu_h, iter(ylo)) + O.sweep(mu_l, iter(yhi))
    mag = O.sweep(np.abs(mu_h), iter(np.abs(y))) + O.sweep(np.abs(mu_l), iter(np.abs(y)))
    tol = (3 * kc + 2) * 2.0 ** -24
    yd = torch.tensor(y, dtype=torch.float32, device=DEV)
    zd = torch.tensor(z0, dtype=torch.float32, device=DEV)
    S.sweep_split(chi, clo, yd, zd, kc=kc, accumulate=False)
    assert np.all(np.abs(zd.cpu().numpy() - ref) <= tol * mag + 1e-300)
    zd = torch.tensor(z0, dtype=torch.float32, device=DEV)
    S.sweep_split(chi, clo, yd, zd, kc=kc, accumulate=True)
    assert np.all(np.abs(zd.cpu().numpy() - (ref + z0)) <= tol * (mag + np.abs(z0)) + 1e-300)
    # against the unsplit product: about 16 significant bits
    full = O.sweep(c[:kc, :ntb], iter(y))
    fmag = O.sweep(np.abs(c[:kc, :ntb]), iter(np.abs(y)))
    assert np.all(np.abs(zd.cpu().numpy() - z0 - full) <= 2.0 ** -14 * fmag + 1e-300)


@pytest.mark.parametrize("kc,ntb,n,nv,k3", [(70, 257, 130, 40, 20), (70, 257, 130, 40, 33), (45, 20, 64, 8, 0),
                                              (16, 5, 33, 4, 1), (100, 9, 40, 8, 64)])
def test_sweep_split_tail_single_product(S, kc, ntb, n, nv, k3):
    """bf16x3 sweep with the single product Chi Yhi past the first k3 degrees (k3 rounded
    up to a multiple of 32) and the three products before."""
    rng = _rng(kc + 3 * ntb + k3)
    ldc = (ntb + 3) // 4 * 4
    m1 = kc
    ldk = (m1 + 7) // 8 * 8
    c = rng.standard_normal((m1, ldc))
    y = rng.standard_normal((kc, n, nv)).astype(np.float32).astype(np.float64)
    cd = torch.tensor(c, device=DEV)
    chi, clo = S.split_coefficients(cd, ntb, ldk)
    hi = bf16_from_f64(c[:, :ntb])
    lo = bf16_from_f64(c[:, :ntb] - hi)
    yhi, ylo = bf16_split(y)
    k3r = min(kc, -(-k3 // 32) * 32)
    three = (np.arange(kc) < k3r).astype(np.float64)[:, None]  # per degree
    mu_h, mu_l = hi[:kc], lo[:kc] * three
    ref = O.sweep(mu_h, iter(yhi)) + O.sweep(mu_h * three, iter(ylo)) + O.sweep(mu_l, iter(yhi))
    mag = O.sweep(np.abs(mu_h), iter(np.abs(y))) + O.sweep(np.abs(mu_l), iter(np.abs(y)))
    tol = (3 * kc + 2) * 2.0 ** -24
    yd = torch.tensor(y, dtype=torch.float32, device=DEV)
    zd = torch.zeros(ntb, n, nv, dtype=torch.float32, device=DEV)
    S.sweep_split(chi, clo, yd, zd, kc=kc, k3=k3)
    assert np.all(np.abs(zd.cpu().numpy() - ref) <= tol * mag + 1e-300)


# ----------------------------------------------------------------------------
# Gram
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("n,nv,ntb,nseg", [(1000, 40, 5, 1), (1000, 80, 3, 3), (97, 8, 2, 1), (4000, 96, 4, 5),
                                           (33, 4, 1, 1), (2048, 64, 2, 7), (3000, 128, 2, 3), (1500, 256, 2, 2),
                                           (501, 200, 1, 1)])
def test_gram(S, precision, n, nv, ntb, nseg):
    """The stage call on independent W and Z, where W^T Z is not symmetric: the matrix the
    call documents (the upper 16 x 16 blocks of W^T Z, mirrored, diagonal blocks
    averaged with their transposes) and K_Z = Z^T Z."""
    rng = _rng(n + nv)
    dt = torch.float64 if precision == "fp64" else torch.float32
    w = rng.standard_normal((n, nv))
    z = rng.standard_normal((ntb, n, nv))
    if dt == torch.float32:
        w, z = w.astype(np.float32).astype(np.float64), z.astype(np.float32).astype(np.float64)
    kw = torch.empty(ntb, nv, nv, dtype=torch.float64, device=DEV)
    kz = torch.empty_like(kw)
    S.gram(precision, torch.tensor(w, dtype=dt, device=DEV), torch.tensor(z, dtype=dt, device=DEV), kw, kz, nseg)
    from gram_completion import upper_completion
    for i in range(ntb):
        _, rz = O.gram(w, z[i])
        _, mz = O.gram(np.abs(w), np.abs(z[i]))
        rw = upper_completion(w.T @ z[i])    # W^T Z is not symmetric for independent inputs
        mw = upper_completion(np.abs(w).T @ np.abs(z[i]))
        tol = (n + 4) * 2.0 ** -53          # FP64 sums of exact products
        assert np.all(np.abs(kw[i].cpu().numpy() - rw) <= tol * mw)
        assert np.all(np.abs(kz[i].cpu().numpy() - rz) <= tol * mz)
        assert np.array_equal(kz[i].cpu().numpy(), kz[i].cpu().numpy().T)
        assert np.array_equal(kw[i].cpu().numpy(), kw[i].cpu().numpy().T)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("n,nv,ntb,nseg", [(1000, 40, 3, 1), (2048, 80, 2, 3), (1500, 128, 2, 2), (700, 256, 1, 1)])
def test_gram_against_oracle_symmetrised(S, precision, n, nv, ntb, nseg):
    """Gram matrices on the method's path, where W^T Z is symmetric in exact arithmetic
    (Z_i = B_i W with B_i symmetric, as g(t_i I - A) is): against the oracle's
    K_W = (W^T Z + Z^T W)/2 and K_Z = Z^T Z, up to the FP64 sums and half the asymmetry
    |W^T Z - Z^T W| / 2 that the rounding of Z leaves (the kernel forms the upper blocks of
    W^T Z only)."""
    rng = _rng(3 * n + nv)
    dt = torch.float64 if precision == "fp64" else torch.float32
    w = rng.standard_normal((n, nv))
    z = np.empty((ntb, n, nv))
    for i in range(ntb):
        b = rng.standard_normal((n, n)) / np.sqrt(n)
        z[i] = (b + b.T) @ w
    if dt == torch.float32:
        w, z = w.astype(np.float32).astype(np.float64), z.astype(np.float32).astype(np.float64)
    kw = torch.empty(ntb, nv, nv, dtype=torch.float64, device=DEV)
    kz = torch.empty_like(kw)
    S.gram(precision, torch.tensor(w, dtype=dt, device=DEV), torch.tensor(z, dtype=dt, device=DEV), kw, kz, nseg)
    tol = (n + 4) * 2.0 ** -53
    for i in range(ntb):
        rw, rz = O.gram(w, z[i])
        mw, mz = O.gram(np.abs(w), np.abs(z[i]))
        asym = 0.5 * np.abs(w.T @ z[i] - z[i].T @ w)
        assert asym.max() <= (1e-13 if precision == "fp64" else 1e-5) * np.abs(rw).max()
        assert np.all(np.abs(kw[i].cpu().numpy() - rw) <= tol * mw + asym + 1e-300)
        assert np.all(np.abs(kz[i].cpu().numpy() - rz) <= tol * mz + 1e-300)


# ----------------------------------------------------------------------------
# Algorithm 4
# ----------------------------------------------------------------------------
def _geneig_cases():
    cases = []
    rng = _rng(5)
    # Theorem 3 pencils: exact low rank PSD P, W Gaussian
    for (n, r, nv) in ((300, 10, 24), (300, 40, 44), (500, 3, 8), (400, 90, 96), (200, 30, 32), (600, 100, 128),
                       (800, 50, 256), (400, 150, 200)):
        u, _ = np.linalg.qr(rng.standard_normal((n, r)))
        s = rng.uniform(0.001, 0.01, r)
        w = rng.standard_normal((n, nv))
        z = (u * s) @ (u.T @ w)
        kw, kz = O.gram(w, z)
        cases.append((kw, kz, 0.008))
    # one generalised eigenvalue above the range bound (dropped)
    u, _ = np.linalg.qr(rng.standard_normal((200, 6)))
    s = np.array([0.033, 0.001, 0.002, 0.003, 0.004, 0.005])
    w = rng.standard_normal((200, 16))
    kw, kz = O.gram(w, (u * s) @ (u.T @ w))
    cases.append((kw, kz, 0.008))
    # degenerate: negative definite K_W (nothing kept), zero matrices
    cases.append((-np.eye(8), np.eye(8), 0.01))
    cases.append((np.zeros((4, 4)), np.zeros((4, 4)), 0.01))
    # the same above N_v = 48 (the tridiagonal path), and: K_W = I (every eigenvalue equal, T
    # already diagonal, no QL iteration) with K_Z diagonal, some entries above the range
    # bound; a rank-32 K_W of 64 columns (32 duplicated: a cluster of zero eigenvalues)
    cases.append((-np.eye(64), np.eye(64), 0.01))
    cases.append((np.zeros((64, 64)), np.zeros((64, 64)), 0.01))
    cases.append((np.eye(64), np.diag(rng.uniform(0.0, 0.02, 64)), 0.01))
    w = rng.standard_normal((300, 32))
    w = np.concatenate([w, w], axis=1)
    u, _ = np.linalg.qr(rng.standard_normal((300, 20)))
    kw, kz = O.gram(w, (u * rng.uniform(0.001, 0.01, 20)) @ (u.T @ w))
    cases.append((kw, kz, 0.008))
    return cases


@pytest.mark.parametrize("case", range(len(_geneig_cases())))
def test_geneig_synthetic(S, case):
    kw, kz, gmax = _geneig_cases()[case]
    nv = kw.shape[0]
    dos = torch.empty(1, dtype=torch.float64, device=DEV)
    ranks = torch.empty(2, dtype=torch.int32, device=DEV)
    S.geneig_trace(torch.tensor(kw[None], device=DEV), torch.tensor(kz[None], device=DEV), gmax, 1e-7, 1e-3, dos,
                   ranks)
    ref, r1, r2 = O.geneig_trace(kw, kz, gmax, 1e-7, 1e-3)
    assert abs(dos.item() - ref) <= 1e-10 * gmax
    assert ranks.cpu().tolist() == [r1, r2]


def test_geneig_workload_pencils(S):
    """Pencils of the real problem: the oracle's K_W, K_Z of the 32x32 workload."""
    wl = WL.make_workload(1)
    pts = np.arange(0, wl.nt, 7)
    res = O.ss_dgc(wl.a, wl.w(), wl.t, wl.degree, wl.sigma, wl.lo, wl.hi, points=pts, keep=True)
    gmax = O.range_bound(wl.sigma, wl.a.n)
    dos = torch.empty(pts.size, dtype=torch.float64, device=DEV)
    ranks = torch.empty(2 * pts.size, dtype=torch.int32, device=DEV)
    S.geneig_trace(torch.tensor(res["k_w"], device=DEV), torch.tensor(res["k_z"], device=DEV), gmax, 1e-7, 1e-3,
                   dos, ranks)
    assert np.abs(dos.cpu().numpy() - res["dos"]).max() <= 1e-9 * gmax
    rk = ranks.cpu().numpy()
    assert np.array_equal(rk[: pts.size], res["r1"]) and np.array_equal(rk[pts.size:], res["r2"])


def _theorem3_pencils(rng, count, n, r, nv):
    """K_W, K_Z of Theorem 3 pencils: exact low-rank PSD P (rank r), W Gaussian."""
    kws, kzs = [], []
    for _ in range(count):
        u, _ = np.linalg.qr(rng.standard_normal((n, r)))
        s = rng.uniform(0.001, 0.01, r)
        w = rng.standard_normal((n, nv))
        kw, kz = O.gram(w, (u * s) @ (u.T @ w))
        kws.append(kw)
        kzs.append(kz)
    return np.array(kws), np.array(kzs)


@pytest.mark.parametrize("nv", [49, 77, 131, 250])
def test_geneig_tridiagonal_path_odd_sizes(S, nv):
    """N_v not a multiple of 8 on the tridiagonal path: the last 8-entry block of each row
    in the reflector steps is partial, and the last 64-row group of U is partial (for
    77, 131 and 250); three Theorem 3 pencils against the oracle."""
    kw, kz = _theorem3_pencils(_rng(13 + nv), 3, 2 * nv + 50, nv // 3, nv)
    dos = torch.empty(3, dtype=torch.float64, device=DEV)
    ranks = torch.empty(6, dtype=torch.int32, device=DEV)
    S.geneig_trace(torch.tensor(kw, device=DEV), torch.tensor(kz, device=DEV), 0.008, 1e-7, 1e-3, dos, ranks)
    d, rk = dos.cpu().numpy(), ranks.cpu().numpy()
    for i in range(3):
        ref, r1, r2 = O.geneig_trace(kw[i], kz[i], 0.008, 1e-7, 1e-3)
        assert abs(d[i] - ref) <= 1e-10 * 0.008, i
        assert [rk[i], rk[3 + i]] == [r1, r2], i


def test_geneig_tridiagonal_path_redoes_a_stopped_point(S):
    """Above N_v = 48 a point whose QL stops (here: NaN in K_W, so no block ever splits)
    is redone by the Jacobi kernel, and only that point: its outputs are written (by
    Jacobi, which stops at once on a NaN norm and proceeds from the unrotated diagonal),
    the others match the oracle."""
    kw, kz = _theorem3_pencils(_rng(11), 3, 400, 60, 160)
    kw[1, 5, 7] = np.nan
    dos = torch.full((3,), 12345.0, dtype=torch.float64, device=DEV)
    ranks = torch.full((6,), -7, dtype=torch.int32, device=DEV)
    S.geneig_trace(torch.tensor(kw, device=DEV), torch.tensor(kz, device=DEV), 0.008, 1e-7, 1e-3, dos, ranks)
    d, rk = dos.cpu().numpy(), ranks.cpu().numpy()
    assert d[1] != 12345.0 and rk[1] != -7 and rk[4] != -7
    for i in (0, 2):
        ref, r1, r2 = O.geneig_trace(kw[i], kz[i], 0.008, 1e-7, 1e-3)
        assert abs(d[i] - ref) <= 1e-10 * 0.008
        assert [rk[i], rk[3 + i]] == [r1, r2]


def test_geneig_tridiagonal_path_launch_groups(S):
    """2100 points at N_v = 136: two launch groups of the tridiagonal path (2048 points
    each) through one scratch; points on both sides of the boundary against the oracle."""
    ntb, nv = 2100, 136
    rng = _rng(12)
    base_w, base_z = _theorem3_pencils(rng, 4, 300, 40, nv)
    # every point a distinct pencil: the four bases scaled, so each point's answer is known
    scale = 1.0 + 0.25 * (np.arange(ntb) % 7)
    kw = torch.tensor(base_w[np.arange(ntb) % 4] * scale[:, None, None], device=DEV)
    kz = torch.tensor(base_z[np.arange(ntb) % 4] * scale[:, None, None], device=DEV)
    dos = torch.empty(ntb, dtype=torch.float64, device=DEV)
    ranks = torch.empty(2 * ntb, dtype=torch.int32, device=DEV)
    S.geneig_trace(kw, kz, 0.008, 1e-7, 1e-3, dos, ranks)
    d, rk = dos.cpu().numpy(), ranks.cpu().numpy()
    for i in (0, 1, 2046, 2047, 2048, 2049, 2099):
        ref, r1, r2 = O.geneig_trace(kw[i].cpu().numpy(), kz[i].cpu().numpy(), 0.008, 1e-7, 1e-3)
        assert abs(d[i] - ref) <= 1e-10 * 0.008, i
        assert [rk[i], rk[ntb + i]] == [r1, r2], i
    # a pencil scaled by c has the same generalised eigenvalues: points agree with their base
    for i in range(ntb):
        assert abs(d[i] - d[i % 28]) <= 1e-10 * 0.008, i


# ----------------------------------------------------------------------------
# End to end (Algorithm 5 through ssm_create / ssm_dos)
# ----------------------------------------------------------------------------
def _run(S, wl, precision, budget=0, w=None, t=None):
    dt = torch.float64 if precision == "fp64" else torch.float32
    csr = S.DeviceCSR.from_csr(wl.a, dtype=dt, device=DEV)
    wd = None if w is None else torch.tensor(w, dtype=dt, device=DEV)
    ctx = S.SSM(csr, lo=wl.lo, hi=wl.hi, sigma=wl.sigma, nv=wl.nv, degree=wl.degree,
                t=wl.t if t is None else t, precision=precision, seed=wl.seed, w=wd, budget=budget, device=DEV)
    dos, r1, r2 = ctx.dos()
    st = ctx.stats()
    ctx.close()
    return dos, r1, r2, st


def _l1(a, b):
    return np.abs(a - b).sum() / np.abs(b).sum()


@pytest.fixture(scope="module")
def cfg1_oracle():
    wl = WL.make_workload(1)
    return wl, O.ss_dgc(wl.a, wl.w(), wl.t, wl.degree, wl.sigma, wl.lo, wl.hi)


def test_end_to_end_cfg1_fp64(S, cfg1_oracle):
    wl, ref = cfg1_oracle
    dos, r1, r2, st = _run(S, wl, "fp64")
    assert np.abs(dos - ref["dos"]).max() <= 1e-9 * ref["dos"].max()
    assert np.mean(r1 == ref["r1"]) >= 0.99 and np.mean(r2 == ref["r2"]) >= 0.99
    assert st["passes"] == 1 and st["spmm_launches"] == wl.degree


@pytest.mark.parametrize("precision,bound", [("fp32", 1e-3), ("bf16x3", 1e-3), ("bf16", 2e-2)])
def test_end_to_end_cfg1_mixed(S, cfg1_oracle, precision, bound):
    """FP32 meets the 1e-3 L1 gate.  Plain BF16 sweep inputs (8-bit mantissa) do not:
    their error is held to the bound measured for that mode, and the mode is
    reported, not used at the fixed-L1 comparison."""
    wl, ref = cfg1_oracle
    dos, r1, r2, _ = _run(S, wl, precision)
    l1 = _l1(dos, ref["dos"])
    print(f"cfg1 {precision}: DOS relative L1 vs FP64 oracle = {l1:.3e}")
    assert l1 <= bound


def test_end_to_end_identical_w_input(S, cfg1_oracle):
    """W passed in (the shared generator's) gives the same DOS as W drawn on the device."""
    wl, ref = cfg1_oracle
    dos, *_ = _run(S, wl, "fp64", w=wl.w())
    assert np.abs(dos - ref["dos"]).max() <= 1e-9 * ref["dos"].max()


def test_end_to_end_small_workspace_plans(S, cfg1_oracle):
    """A budget that forces several recurrence passes and a ring of Chebyshev blocks
    gives the single-pass result."""
    wl, ref = cfg1_oracle
    full, *_ = _run(S, wl, "fp64")
    budget = 110 * 1024 * 1024
    dos, _, _, st = _run(S, wl, "fp64", budget=budget)
    print("plan under budget:", st["passes"], "passes, chunk", st["chunk"], "batch", st["batch"])
    assert st["passes"] > 1 or st["chunk"] < wl.degree + 1
    assert np.abs(dos - full).max() <= 1e-11 * full.max()


def test_end_to_end_small_workspace_split(S, cfg1_oracle):
    """The split-BF16 path under budgets that force several sweep-point passes or a ring of
    Chebyshev blocks: its sweep launches then start inside the coefficient tables (a later
    pass's rows of the 128-byte-row tables, a later chunk's degrees) and accumulate into Z.
    Each estimate meets the 1e-3 L1 gate against the oracle and stays within 1e-4 of the
    maximum of the single-pass split-BF16 estimate (the chunked FP32 sums round differently)."""
    from paper_1504_07690_amd._abi import SSMError
    wl, ref = cfg1_oracle
    full, *_ = _run(S, wl, "bf16x3")
    csr = S.DeviceCSR.from_csr(wl.a, dtype=torch.float32, device=DEV)
    need = S.workspace_size(csr, lo=wl.lo, hi=wl.hi, sigma=wl.sigma, nv=wl.nv, degree=wl.degree, nt=wl.nt,
                            precision="bf16x3")
    plans = []
    for frac in (0.6, 0.35, 0.2):
        try:
            dos, _, _, st = _run(S, wl, "bf16x3", budget=int(frac * need))
        except SSMError as err:
            print(f"budget {frac} of {need} bytes: no plan ({err})")
            continue
        print(f"budget {frac}: {st['passes']} passes, chunk {st['chunk']}, batch {st['batch']}")
        plans.append((st["passes"], st["chunk"]))
        assert _l1(dos, ref["dos"]) <= 1e-3
        assert np.abs(dos - full).max() <= 1e-4 * full.max()
    assert any(p > 1 for p, _ in plans) and any(c < wl.degree + 1 for _, c in plans), plans


def test_end_to_end_ragged_anderson(S):
    """16^3 Anderson lattice: ragged tiles in every kernel (N = 4096, N_v = 20, N_t = 101)."""
    a = WL.anderson_3d(16, _rng(8).uniform(-2, 2, 16 ** 3))
    wl = WL.make_workload(2, a=a, nv=20, degree=300, nt=101, sigma_hat=0.03)
    ref = O.ss_dgc(wl.a, wl.w(), wl.t, wl.degree, wl.sigma, wl.lo, wl.hi)
    d64, *_ = _run(S, wl, "fp64")
    assert np.abs(d64 - ref["dos"]).max() <= 1e-9 * ref["dos"].max()
    d32, *_ = _run(S, wl, "fp32")
    assert _l1(d32, ref["dos"]) <= 1e-3
    dx3, *_ = _run(S, wl, "bf16x3")
    assert _l1(dx3, ref["dos"]) <= 1e-3


def test_identity_probe_exact_dos(S):
    """W = I_N (N_v = N = 64, an 8x8 Dirichlet Laplacian): the estimate is the exact
    regularised DOS from the dense eigenvalues (Theorem 3 with P = g(tI - A))."""
    a = WL.laplacian_2d_dirichlet(8, _rng(2).uniform(-1, 1, 64))
    wl = WL.make_workload(1, a=a, nv=64, degree=200, nt=50, sigma_hat=0.05)
    lam = np.linalg.eigvalsh(a.to_dense())
    dos, *_ = _run(S, wl, "fp64", w=np.eye(64))
    ref = O.exact_dos(lam, wl.t, wl.sigma)
    assert np.abs(dos - ref).max() <= 1e-6 * ref.max()


def test_bounds_error(S):
    from paper_1504_07690_amd._abi import SSMError, SSM_ERR_BOUNDS, SSM_ERR_NONFINITE
    wl = WL.make_workload(1)
    wl.hi = wl.lo + 0.5 * (wl.hi - wl.lo)    # interval misses the upper half of the spectrum
    with pytest.raises(SSMError) as ei:
        _run(S, wl, "fp64")
    assert ei.value.status in (SSM_ERR_BOUNDS, SSM_ERR_NONFINITE)


def test_nan_values_reported(S):
    from paper_1504_07690_amd._abi import SSMError, SSM_ERR_NONFINITE
    wl = WL.make_workload(1)
    vals = wl.a.values.copy()
    vals[10] = np.nan
    wl.a = WL.CSR(wl.a.n, wl.a.row_ptr, wl.a.col_idx, vals)
    with pytest.raises(SSMError) as ei:
        _run(S, wl, "fp32")
    assert ei.value.status == SSM_ERR_NONFINITE


@pytest.mark.parametrize("nx,nv,degree,nt", [(24, 128, 120, 24), (32, 256, 80, 16)])
def test_end_to_end_large_nv(S, nx, nv, degree, nt):
    """N_v above 96 (the Jacobi matrices in global scratch, the tiled Gram): FP64 against
    the oracle to 1e-9 of g_max, FP32 within 1e-3 relative L1."""
    rng = _rng(nx + nv)
    a = WL.laplacian_2d_dirichlet(nx, rng.uniform(-1, 1, nx * nx))
    wl = WL.make_workload(1, a=a, nv=nv, degree=degree, nt=nt, sigma_hat=0.05)
    ref = O.ss_dgc(a, wl.w(), wl.t, wl.degree, wl.sigma, wl.lo, wl.hi)
    gmax = O.range_bound(wl.sigma, a.n)
    dos, r1, r2, _ = _run(S, wl, "fp64", w=wl.w())
    assert np.abs(dos - ref["dos"]).max() <= 1e-9 * gmax
    assert np.array_equal(r1, ref["r1"]) and np.array_equal(r2, ref["r2"])
    dos32, *_ = _run(S, wl, "fp32", w=wl.w().astype(np.float32))
    print(f"nv={nv}: fp32 L1 {_l1(dos32, ref['dos']):.2e}")
    assert _l1(dos32, ref["dos"]) <= 1e-3


@pytest.mark.parametrize("which,precision,nv", [
    ("anderson16", "fp32", 20), ("anderson24", "fp64", 12), ("stencil12", "fp32", 20), ("stencil20", "bf16x3", 20),
    ("stencil12", "fp32", 256), ("stencil20", "bf16x3", 256), ("anderson16", "fp64", 128), ("stencil08", "fp32", 256),
    ("stencil10", "fp32", 256)])
def test_lattice_row_order_changes_nothing(S, which, precision, nv):
    """The recurrence's tiled visiting order of a lattice's rows (tiles of 16, 8, 4 or 2
    points of the x-y plane through every z), with the CSR entries through the scalar cache
    where a row fills a wave (N_v = 256 in FP32, 128 in FP64): every block and the DOS bit
    for bit equal to the plain row order's.  Where the tiles hold multiples of 8 points and
    rows fill waves, the lattice context takes the box-stencil kernel, which sums a point's
    terms in box order: there the blocks agree to the rounding of that order (FP32 1e-5,
    FP64 1e-13 of the block's largest entry, over 60 steps) and the DOS to 1e-5 (1e-12)."""
    nx = int(which[-2:])
    rng = _rng(nx)
    a = WL.anderson_3d(nx, rng.uniform(-2, 2, nx ** 3)) if which.startswith("anderson") else \
        WL.stencil27_lognormal(nx, rng)
    wl = WL.make_workload(2, a=a, nv=nv, degree=60, nt=24, sigma_hat=0.05)
    dt = torch.float64 if precision == "fp64" else torch.float32
    out = []
    for lattice in (None, (nx, nx, nx)):
        csr = S.DeviceCSR.from_csr(a, dtype=dt, device=DEV)
        ctx = S.SSM(csr, lo=wl.lo, hi=wl.hi, sigma=wl.sigma, nv=wl.nv, degree=wl.degree, t=wl.t,
                    precision=precision, seed=wl.seed, lattice=lattice, device=DEV)
        dos, r1, r2 = ctx.dos()
        out.append((dos, ctx.views()["y"].clone(), ctx.stats()["box_stencil"]))
        ctx.close()
    box = out[1][2]
    assert out[0][2] == 0
    assert box == (nv * (8 if precision == "fp64" else 4) % 1024 == 0 and nx % 8 == 0), box
    if not box:
        assert torch.equal(out[0][1], out[1][1])
        assert np.array_equal(out[0][0], out[1][0])
        return
    y0, y1 = out[0][1].double(), out[1][1].double()
    tol_y, tol_d = (1e-13, 1e-12) if precision == "fp64" else (1e-5, 1e-5)
    dy = ((y1 - y0).abs().amax(dim=(1, 2)) / y0.abs().amax(dim=(1, 2))).max().item()
    dd = np.abs(out[1][0] - out[0][0]).max() / np.abs(out[0][0]).max()
    print(f"{which} {precision} N_v={nv}: box kernel, blocks {dy:.2e}, DOS {dd:.2e} of the largest")
    assert dy <= tol_y and dd <= tol_d


@pytest.mark.parametrize("which,precision,nv", [("stencil16", "fp32", 256), ("anderson16", "fp64", 128),
                                                ("stencil08", "fp64", 256)])
def test_box_stencil_recurrence_against_oracle(S, which, precision, nv):
    """The box-stencil kernel of the recurrence (8 points of a lattice row per wave, every
    neighbourhood line gathered once, wrapped rows included) against the oracle's
    recurrence (Algorithm 5 steps 9-10): every block of 30 steps on the same W within the
    chebyshev test's bounds (FP32 2e-5, FP64 1e-12 of max|W| per step)."""
    nx = int(which[-2:])
    rng = _rng(nx + 1)
    a = WL.anderson_3d(nx, rng.uniform(-2, 2, nx ** 3)) if which.startswith("anderson") else \
        WL.stencil27_lognormal(nx, rng)
    degree = 30
    wl = WL.make_workload(2, a=a, nv=nv, degree=degree, nt=8, sigma_hat=0.05)
    dt = torch.float64 if precision == "fp64" else torch.float32
    w = wl.w()
    if precision == "fp32":
        w = w.astype(np.float32).astype(np.float64)
    csr = S.DeviceCSR.from_csr(a, dtype=dt, device=DEV)
    ctx = S.SSM(csr, lo=wl.lo, hi=wl.hi, sigma=wl.sigma, nv=nv, degree=degree, t=wl.t, precision=precision,
                w=torch.tensor(w, dtype=dt, device=DEV), lattice=(nx, nx, nx), device=DEV)
    assert ctx.stats()["box_stencil"] == 1
    ctx.dos()
    got = ctx.views()["y"].double().cpu().numpy()
    ctx.close()
    tol = 1e-12 if precision == "fp64" else 2e-5
    scale = np.abs(w).max()
    worst = 0.0
    for l, v in O.chebyshev_blocks(a, w, degree, wl.lo, wl.hi):
        err = np.abs(got[l] - v).max()
        worst = max(worst, err / (scale * max(1, l)))
        assert err <= tol * scale * max(1, l), l
    print(f"{which} {precision} N_v={nv}: worst block error {worst:.2e} of max|W| per step")


@pytest.mark.parametrize("plan", [None, (304, 48), (104, 0), (104, 32)])
def test_split_sweep_context_tables(S, plan):
    """The context's split-BF16 sweep reads its coefficient tables in 16-degree blocks of all
    N_t rows: rows of Z against the oracle's sweep (Algorithm 5 steps 6-8) of the device's
    own blocks, on a ragged case (N_t = 300 points over two 256-point tiles, M + 1 = 101
    degrees, N N_v not a multiple of 256), with every block resident, with a ring of 48
    blocks (launches starting at degrees 48 and 96 that add into Z), and with batches of 104
    points (launches starting at rows 104 and 208), alone and with a ring of 32."""
    from test_gpu_configs import _assert_z_rows
    a = WL.anderson_3d(13, _rng(31).uniform(-2, 2, 13 ** 3))
    wl = WL.make_workload(2, a=a, nv=20, degree=100, nt=300, sigma_hat=0.03)
    n, nv, m = wl.a.n, wl.nv, wl.degree
    rows = np.sort(_rng(32).choice(n, 7, replace=False))
    rows_t = torch.as_tensor(rows, device=DEV)
    mu = O.dgc_coefficients(wl.t, m, wl.sigma, n, wl.lo, wl.hi)
    csr = S.DeviceCSR.from_csr(wl.a, dtype=torch.float32, device=DEV)
    kw = dict(lo=wl.lo, hi=wl.hi, sigma=wl.sigma, nv=nv, degree=m, t=wl.t, precision="bf16x3", seed=wl.seed,
              device=DEV)
    ctx = S.SSM(csr, **kw)  # every block resident: the device's Y_0..Y_M
    ctx.dos()
    yr = ctx.views()["y"][:, rows_t, :].double().cpu().numpy()
    ctx.close()
    ctx = S.SSM(csr, plan=plan, **kw)
    ctx.dos()
    st = ctx.stats()
    v = ctx.views()
    p0, nb = v["first_point_of_last_batch"], v["batch"]
    nb = min(nb, wl.nt - p0)
    z = v["z"][:nb, rows_t, :].double().cpu().numpy()
    ctx.close()
    print(f"plan {plan}: {st['passes']} passes, chunk {st['chunk']}, {st['sweep_launches']} sweep launches, "
          f"k3 {st['split_k3']}; rows of Z of points {p0}..{p0 + nb - 1}")
    if plan is not None:
        assert st["passes"] > 1 or st["chunk"] < m + 1
    _assert_z_rows(z, mu[:, p0:p0 + nb], yr, "bf16x3", st["split_k3"])
