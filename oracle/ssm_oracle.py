"""CPU reference of the spectrum sweeping method (SS-DGC) in float64.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this module.  The HIP library never
calls it and shares no code with it.

Paper: L. Lin, "Randomized estimation of spectral densities of large matrices
made accurate" (arXiv:1504.07690).  Every function follows one passage of the
paper, in its order and notation; numpy/scipy routines serve only as library
primitives (FFT, dense symmetric eigensolver, sparse matrix times block, erf).

Units.  The paper assumes spec(A) in (-1, 1).  For a general matrix it applies
the affine map A~ = (2A - (lo+hi)I)/(hi-lo) (Section 2).  Here A, the sweep
points t and the smearing sigma stay in A's units; the Chebyshev expansion is
taken in the rescaled variable, i.e. the expanded function is
s -> g_sigma(t - x(s)) with x(s) = c0 + hw*s, c0 = (lo+hi)/2, hw = (hi-lo)/2.

Readings where the paper is silent (each also listed in the design notes):
* N_theta of Algorithm 1: 2*N_theta is the least power of two >= 4(M+1).
* Algorithm 5 applies A once more after the last accumulation (l = M); that
  product is never used and is not computed.
* W^* Z is symmetric in exact arithmetic (Section 3.1); it is symmetrised as
  (W^T Z + Z^T W)/2 before the eigen-decomposition of Algorithm 4.
* Algorithm 4, step 2 keeps s_j >= tau * max_i s_i (inclusive); if
  max_i s_i <= 0 nothing is kept and the estimate is 0.
* Algorithm 4, step 4 keeps xi in [0, (1 + rho) / (N sqrt(2 pi sigma^2))]
  (closed interval, relative slack rho, default 1e-3).
* Algorithm 7 takes mu_l (l <= M/2) from Algorithm 1 run at degree M (the
  run's N_theta) and sets the rest to 0; M must be even (Proposition 1).
* Algorithm 7's truncation also drops eigenvalues of K_W below the rounding
  level of its moment sum, 1e-12 sum_l |mu_l(t_i)| max|X_W,l| (see ress_dgc).
* A sweep in limited precision leaves an error in W^T Z; Algorithm 4's truncation
  then also drops eigenvalues of K_W below that error (rounding_floor).  The
  oracle itself is FP64 and takes no floor unless one is passed in.
* Algorithm 8 deconvolves with the unit-mass Gaussian (N times g_sigma),
  periodically on [-1, 1] in the rescaled variable, dropping wavenumbers k
  with exp(-(sigma^ pi k)^2 / 2) < eta (eta = 1e-10).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp
import scipy.special as sps


# ----------------------------------------------------------------------------
# Section 2: Gaussian regularisation and the exact regularised DOS
# ----------------------------------------------------------------------------
def g_sigma(s, sigma: float, n: int):
    """Eq. (gaussian): g_sigma(s) = exp(-s^2 / (2 sigma^2)) / (N sqrt(2 pi sigma^2))."""
    s = np.asarray(s, dtype=np.float64)
    return np.exp(-s * s / (2.0 * sigma * sigma)) / (n * math.sqrt(2.0 * math.pi * sigma * sigma))


def exact_dos(eigenvalues, t, sigma: float, n: int | None = None):
    """phi_sigma(t) = sum_i g_sigma(t - lambda_i) (Section 2), from eigenvalues."""
    lam = np.asarray(eigenvalues, dtype=np.float64)
    n = lam.size if n is None else n
    t = np.atleast_1d(np.asarray(t, dtype=np.float64))
    out = np.empty(t.shape)
    for k in range(0, t.size, 256):
        out[k:k + 256] = g_sigma(t[k:k + 256, None] - lam[None, :], sigma, n).sum(axis=1)
    return out


def range_bound(sigma: float, n: int) -> float:
    """Largest value of g_sigma: 1 / (N sqrt(2 pi sigma^2)) (Section 3.2)."""
    return 1.0 / (n * math.sqrt(2.0 * math.pi * sigma * sigma))


# ----------------------------------------------------------------------------
# Algorithm 1: Delta-Gauss-Chebyshev coefficients
# ----------------------------------------------------------------------------
def n_theta_for(degree: int) -> int:
    """N_theta > M (Algorithm 1); taken so that 2 N_theta = 2^ceil(log2(4(M+1)))."""
    two_nt = 1
    while two_nt < 4 * (degree + 1):
        two_nt *= 2
    return two_nt // 2


def dgc_coefficients(t, degree: int, sigma: float, n: int, lo: float, hi: float,
                     n_theta: int | None = None) -> np.ndarray:
    """mu_l(t_i), l = 0..M, for every sweep point (Algorithm 1, Eq. mucoef2).

    theta_j = j pi / N_theta (j < 2 N_theta); g_j = g_sigma(t - x(cos theta_j));
    g^ = DFT(g); mu_l = (2 - delta_l0) / (2 N_theta) Re g^_l.
    Returns an array of shape (M + 1, N_t).
    """
    t = np.atleast_1d(np.asarray(t, dtype=np.float64))
    n_theta = n_theta_for(degree) if n_theta is None else n_theta
    assert n_theta > degree
    c0, hw = 0.5 * (lo + hi), 0.5 * (hi - lo)
    theta = np.arange(2 * n_theta) * math.pi / n_theta
    x = c0 + hw * np.cos(theta)
    g = g_sigma(t[None, :] - x[:, None], sigma, n)          # (2 N_theta, N_t)
    ghat = np.fft.fft(g, axis=0)                             # sum_j e^{-i 2 pi j l / 2N_theta} g_j
    mu = ghat[: degree + 1].real / (2 * n_theta)
    mu[1:] *= 2.0
    return mu


def chebyshev_eval(mu: np.ndarray, s) -> np.ndarray:
    """sum_l mu_l T_l(s) by the three-term recurrence (Eq. gcheb) at scalar points s."""
    s = np.asarray(s, dtype=np.float64)
    t_prev, t_cur = np.ones_like(s), s.copy()
    out = mu[0] * t_prev
    if mu.shape[0] > 1:
        out = out + mu[1] * t_cur
    for l in range(2, mu.shape[0]):
        t_prev, t_cur = t_cur, 2.0 * s * t_cur - t_prev
        out = out + mu[l] * t_cur
    return out


# ----------------------------------------------------------------------------
# The three-term recurrence of Algorithms 2 and 5 on one block W
# ----------------------------------------------------------------------------
def _as_scipy(a):
    if sp.issparse(a):
        return a.tocsr()
    if hasattr(a, "to_scipy"):
        return a.to_scipy()
    return sp.csr_matrix(np.asarray(a, dtype=np.float64))


def chebyshev_blocks(a, w: np.ndarray, degree: int, lo: float, hi: float):
    """Yield (l, V_c) with V_c = T_l(A~) W for l = 0..M (Algorithm 5, steps 3-11).

    V_m, V_c <- 0, W; after the accumulations of step l:
    V_p <- (2 - delta_l0) A~ V_c - V_m; V_m <- V_c; V_c <- V_p,
    where A~ = (2A - (lo+hi) I)/(hi - lo) (Section 2).  The product that would
    follow the last accumulation (l = M) is not computed.
    """
    a = _as_scipy(a)
    alpha = 2.0 / (hi - lo)
    beta = -(hi + lo) / (hi - lo)
    v_m = np.zeros_like(w, dtype=np.float64)
    v_c = np.asarray(w, dtype=np.float64).copy()
    for l in range(degree + 1):
        yield l, v_c
        if l == degree:
            break
        a_vc = alpha * (a @ v_c) + beta * v_c
        v_p = (2.0 if l > 0 else 1.0) * a_vc - v_m
        v_m, v_c = v_c, v_p


# ----------------------------------------------------------------------------
# Algorithm 2: DGC (Hutchinson-type) estimate, for comparison
# ----------------------------------------------------------------------------
def dgc_dos(a, w, t, degree, sigma, lo, hi):
    """zeta_l = Tr[W^* T_l(A~) W] / N_v; phi~(t_i) = sum_l mu_l(t_i) zeta_l (Algorithm 2)."""
    n, nv = w.shape
    mu = dgc_coefficients(t, degree, sigma, n, lo, hi)
    zeta = np.zeros(degree + 1)
    for l, v_c in chebyshev_blocks(a, w, degree, lo, hi):
        zeta[l] = np.sum(w * v_c) / nv
    return mu.T @ zeta


# ----------------------------------------------------------------------------
# Algorithm 4: generalised eigenvalue problem, truncated
# ----------------------------------------------------------------------------
def geneig_trace(k_w: np.ndarray, k_z: np.ndarray, g_max: float, tau: float = 1e-7,
                 rho: float = 1e-3, return_parts: bool = False, s_floor: float = 0.0):
    """Tr Xi~ for the pencil (Z^*Z, W^*Z) of one sweep point (Algorithm 4).

    1. W^*Z = U S U^*.
    2. keep s_j >= tau max_i s_i  (S~, U~), and s_j >= s_floor (0 unless given).
    3. eig of S~^{-1/2} U~^* Z^*Z U~ S~^{-1/2}  -> xi.
    4. keep xi in [0, (1 + rho) g_max].
    Returns the sum of kept xi and the two kept counts (r1, r2); with
    ``return_parts`` also a dict with s, xi and C~ = U~ S~^{-1/2} Q~ (Q~: the
    eigenvectors of step 3 whose xi pass step 4), so that C~^* K_W C~ = I and
    C~^* K_Z C~ = Xi~.
    """
    k_w = 0.5 * (k_w + k_w.T)
    s, u = np.linalg.eigh(k_w)
    smax = s.max() if s.size else 0.0
    if not smax > 0.0:
        out = (0.0, 0, 0)
        return out + ({"s": s, "xi": np.zeros(0), "c": np.zeros((k_w.shape[0], 0))},) if return_parts else out
    keep = (s >= tau * smax) & (s >= s_floor)
    if not keep.any():
        out = (0.0, 0, 0)
        return out + ({"s": s, "xi": np.zeros(0), "c": np.zeros((k_w.shape[0], 0))},) if return_parts else out
    u_t = u[:, keep] / np.sqrt(s[keep])[None, :]
    b = u_t.T @ k_z @ u_t
    xi, q = np.linalg.eigh(0.5 * (b + b.T))
    in_range = (xi >= 0.0) & (xi <= (1.0 + rho) * g_max)
    out = (float(xi[in_range].sum()), int(keep.sum()), int(in_range.sum()))
    return out + ({"s": s, "xi": xi, "c": u_t @ q[:, in_range]},) if return_parts else out


def sweep(mu: np.ndarray, blocks) -> np.ndarray:
    """Z(t_i) = sum_l mu_l(t_i) V_l accumulated block by block (Algorithm 5, steps 6-8).

    ``mu`` has shape (L, N_t) and ``blocks`` yields the L blocks V_l in order."""
    z = None
    for l, v in enumerate(blocks):
        if z is None:
            z = np.zeros((mu.shape[1],) + v.shape)
        for i in range(mu.shape[1]):
            z[i] += mu[l, i] * v
    return z


def gram(w: np.ndarray, z: np.ndarray):
    """K_W = (W^T Z + Z^T W)/2 and K_Z = Z^T Z for one sweep point (Eq. tracelr)."""
    wz = w.T @ z
    return 0.5 * (wz + wz.T), z.T @ z


def rounding_floor(mu: np.ndarray, w: np.ndarray, eta: float) -> np.ndarray:
    """Rounding floor of Algorithm 4's truncation for a sweep in limited precision
    (a reading; the paper works in exact arithmetic): per sweep point,
    eta * ||mu(t_i)||_2 * ||W||_F^2 / sqrt(N N_v), with ||mu(t_i)||_2 over l = 0..M.

    When every term mu_l T_l(A~) W of the sweep carries a relative rounding of about eta,
    Z(t_i) carries an error of rms size eta ||mu(t_i)||_2 per entry (the blocks' entries
    are O(1): ||T_l(A~) W||_F <= ||W||_F), and W^T Z(t_i) one of spectral norm about
    eta ||mu(t_i)||_2 ||W||_F^2 / sqrt(N N_v).  Eigenvalues of K_W below that are rounding;
    step 2 of Algorithm 4 drops them with s_floor = this value.  ``mu`` has shape
    (M + 1, N_t)."""
    n, nv = w.shape
    return eta * np.sqrt((np.asarray(mu) ** 2).sum(axis=0)) * float(np.sum(w * w)) / math.sqrt(n * nv)


# ----------------------------------------------------------------------------
# Algorithm 5: SS-DGC
# ----------------------------------------------------------------------------
def ss_dgc(a, w, t, degree: int, sigma: float, lo: float, hi: float, tau: float = 1e-7,
           rho: float = 1e-3, points=None, keep=False, mu=None):
    """Spectrum sweeping estimate of phi_sigma at the sweep points (Algorithm 5).

    ``points`` selects a subset of the sweep points (the points are
    independent once the T_l(A~) W are known).  Returns a dict with the DOS
    estimate ``dos`` (A's units), the kept counts ``r1``, ``r2`` and, if
    ``keep``, the blocks Z(t_i) and the Gram matrices.
    """
    w = np.asarray(w, dtype=np.float64)
    n, nv = w.shape
    t = np.atleast_1d(np.asarray(t, dtype=np.float64))
    sel = np.arange(t.size) if points is None else np.asarray(points)
    if mu is None:
        mu = dgc_coefficients(t[sel], degree, sigma, n, lo, hi)          # step 1
    else:
        mu = np.asarray(mu)[:, sel]
    z = sweep(mu, (v for _, v in chebyshev_blocks(a, w, degree, lo, hi)))   # steps 3-11
    g_max = range_bound(sigma, n)
    dos = np.zeros(sel.size)
    r1 = np.zeros(sel.size, dtype=np.int64)
    r2 = np.zeros(sel.size, dtype=np.int64)
    kws, kzs = [], []
    for i in range(sel.size):                                            # steps 12-14
        k_w, k_z = gram(w, z[i])
        dos[i], r1[i], r2[i] = geneig_trace(k_w, k_z, g_max, tau, rho)
        if keep:
            kws.append(k_w)
            kzs.append(k_z)
    out = {"dos": dos, "r1": r1, "r2": r2, "mu": mu, "points": sel}
    if keep:
        out.update(z=z, k_w=np.array(kws), k_z=np.array(kzs))
    return out


# ----------------------------------------------------------------------------
# Section 4: RESS-DGC (Proposition 1, Theorem 4, Algorithms 6 and 7)
# ----------------------------------------------------------------------------
def square_coefficients(mu_half: np.ndarray, degree: int, n_theta: int | None = None) -> np.ndarray:
    """nu_l(t_i), l = 0..M, with (sum_{k<=M/2} mu_k T_k)^2 = sum_{l<=M} nu_l T_l
    (Proposition 1), by the quadrature of Algorithm 1 applied to the squared series:
    p_j = sum_k mu_k T_k(cos theta_j), nu_l = (2 - delta_l0)/(2 N_theta) Re DFT(p^2)_l.
    The quadrature is exact for N_theta > M (the integrand has degree <= 2M in
    cos theta).  ``mu_half`` has shape (M/2 + 1, N_t); returns (M + 1, N_t).
    """
    n_theta = n_theta_for(degree) if n_theta is None else n_theta
    assert n_theta > degree
    theta = np.arange(2 * n_theta) * math.pi / n_theta
    p = chebyshev_eval(np.asarray(mu_half, dtype=np.float64), np.cos(theta)[:, None])   # (2 N_theta, N_t)
    phat = np.fft.fft(p * p, axis=0)
    nu = phat[: degree + 1].real / (2 * n_theta)
    nu[1:] *= 2.0
    return nu


RESS_FLOOR = 1e-12  # eta of the rounding floor of Algorithm 7's truncation (see ress_dgc)


def ress_dgc(a, w, w_tilde, t, degree: int, sigma: float, lo: float, hi: float, tau: float = 1e-7,
             rho: float = 1e-3, eta: float = RESS_FLOOR):
    """RESS-DGC estimate of phi_sigma at the sweep points (Algorithm 7).

    1. mu_l(t_i) by Algorithm 1 at degree M, set to 0 for l > M/2;
    2. nu_l(t_i), l <= M, of the squared degree-M/2 series (Proposition 1);
    3-15. one recurrence on W (N x N_v) and one on W~ (N x N~_v, may have no
       columns); at every degree l: X_W = W^* V_c, X_C = W~^* V_c, X_W~ = W~^* V~_c, and
       K_W += mu_l X_W, K_Z += nu_l X_W, K_C += mu_l X_C, K_W~ += mu_l X_W~ per point;
    16-18. per point, Algorithm 4 on (K_Z, K_W) gives Xi~ and C~, and
       phi~ = Tr Xi~ + (Tr K_W~ - Tr[K_C C~ C~^* K_C^*]) / N~_v  (the last term only
       when N~_v > 0; Algorithm 6).
    Truncation floor: K_W is a sum of moments that cancel to almost nothing where
    g^{M/2}(t_i I - A) W is small, so its rounding is about u sum_l |mu_l(t_i)| max|X_W,l|,
    and so is K_Z's, independently.  Step 2 of Algorithm 4 therefore also drops s_j below
    eta sum_l |mu_l(t_i)| max|X_W,l| (eta = 1e-12): below that the pencil's eigenvalues
    are rounding and land anywhere, in range included.
    Returns a dict with ``dos``, ``r1``, ``r2`` and the accumulated matrices.
    """
    assert degree % 2 == 0, "Proposition 1 needs an even degree"
    w = np.asarray(w, dtype=np.float64)
    w_tilde = np.zeros((w.shape[0], 0)) if w_tilde is None else np.asarray(w_tilde, dtype=np.float64)
    n, nv = w.shape
    nvt = w_tilde.shape[1]
    t = np.atleast_1d(np.asarray(t, dtype=np.float64))
    nt = t.size
    half = degree // 2
    mu = dgc_coefficients(t, degree, sigma, n, lo, hi)                    # step 1
    mu[half + 1:] = 0.0
    nu = square_coefficients(mu[: half + 1], degree)                       # step 2
    k_w = np.zeros((nt, nv, nv))
    k_z = np.zeros((nt, nv, nv))
    k_c = np.zeros((nt, nvt, nv))
    k_wt = np.zeros((nt, nvt, nvt))
    xmax = np.zeros(degree + 1)
    blocks_t = chebyshev_blocks(a, w_tilde, degree, lo, hi) if nvt else None
    for l, v_c in chebyshev_blocks(a, w, degree, lo, hi):                  # steps 6-15
        x_w = w.T @ v_c
        xmax[l] = np.abs(x_w).max()
        k_w += mu[l][:, None, None] * x_w[None]
        k_z += nu[l][:, None, None] * x_w[None]
        if nvt:
            _, vt_c = next(blocks_t)
            k_c += mu[l][:, None, None] * (w_tilde.T @ v_c)[None]
            k_wt += mu[l][:, None, None] * (w_tilde.T @ vt_c)[None]
    g_max = range_bound(sigma, n)
    floor = eta * (np.abs(mu) * xmax[:, None]).sum(axis=0)
    dos = np.zeros(nt)
    r1 = np.zeros(nt, dtype=np.int64)
    r2 = np.zeros(nt, dtype=np.int64)
    for i in range(nt):                                                    # steps 16-18
        tr, r1[i], r2[i], parts = geneig_trace(k_w[i], k_z[i], g_max, tau, rho, return_parts=True,
                                               s_floor=floor[i])
        if nvt:
            kcc = k_c[i] @ parts["c"]
            tr += (np.trace(k_wt[i]) - np.sum(kcc * kcc)) / nvt
        dos[i] = tr
    return {"dos": dos, "r1": r1, "r2": r2, "mu": mu, "nu": nu, "k_w": k_w, "k_z": k_z, "k_c": k_c,
            "k_wt": k_wt, "floor": floor}


# ----------------------------------------------------------------------------
# Section 5, Algorithm 8: trace of a matrix function from the DOS
# ----------------------------------------------------------------------------
def window(t, a: float, sigma_tilde: float):
    """pi(t) of Eq. (pifunc): 1 on (-a, a), smoothly 0 near +-1."""
    t = np.asarray(t, dtype=np.float64)
    return 0.5 * (sps.erf((1.0 + a - 2.0 * t) / sigma_tilde)
                  - sps.erf((-1.0 - a - 2.0 * t) / sigma_tilde))


def periodic_extension(f, t_hat, lo: float, hi: float, a: float, sigma_tilde: float):
    """h(t) = f(t) pi(t) + c (1 - pi(t)) (Eq. hform), in the rescaled variable.

    c is taken as (f(x(-a)) + f(x(a)))/2: the paper notes the constant is
    arbitrary, and f need not be defined at the ends of [lo, hi].  f is only
    evaluated where pi(t) > 1e-300.
    """
    c0, hw = 0.5 * (lo + hi), 0.5 * (hi - lo)
    pi_t = window(t_hat, a, sigma_tilde)
    c = 0.5 * (f(c0 - hw * a) + f(c0 + hw * a))
    h = np.full(t_hat.shape, c, dtype=np.float64)
    m = pi_t > 1e-300
    h[m] = f(c0 + hw * t_hat[m]) * pi_t[m] + c * (1.0 - pi_t[m])
    return h


def trace_weights(f, n: int, lo: float, hi: float, nt: int, sigma: float, a: float = 0.9,
                  sigma_tilde: float = 0.016, eta: float = 1e-10):
    """Weights w_i with Tr f(A) ~= sum_i w_i phi~(t_i) (Algorithm 8).

    Grid: the nt midpoints t^_i of [-1, 1] (rescaled), t_i = c0 + hw t^_i.
    f~ solves (f~ * G) = h periodically on [-1, 1], G the unit-mass Gaussian
    of width sigma^ = sigma/hw (the deconvolution of Eq. deconvolv by Fourier
    transform); Tr f(A) ~= N dt^ sum_i f~(t^_i) phi^(t^_i), and phi^ = hw phi
    in A's units, so w_i = N dt^ hw f~_i.
    """
    hw = 0.5 * (hi - lo)
    sh = sigma / hw
    t_hat = -1.0 + (2.0 * np.arange(nt) + 1.0) / nt
    h = periodic_extension(f, t_hat, lo, hi, a, sigma_tilde)
    k = np.fft.fftfreq(nt, d=1.0 / nt)                  # integer wavenumbers, period 2
    gk = np.exp(-0.5 * (sh * math.pi * k) ** 2)
    k_c = math.floor(math.sqrt(2.0 * math.log(1.0 / eta)) / (math.pi * sh))
    hk = np.fft.fft(h)
    fk = np.where(np.abs(k) <= k_c, hk / gk, 0.0)
    f_tilde = np.fft.ifft(fk).real
    return n * (2.0 / nt) * hw * f_tilde


def trace_weights_exp(beta: float, n: int, lo: float, hi: float, nt: int, sigma: float,
                      spec_lo: float = -math.inf):
    """Weights w_i with Tr exp(-beta A) ~= sum_i w_i phi~(t_i), by the exact real-line
    deconvolution of Eq. (deconvolv): G * e^{-beta s} = e^{beta^2 sigma^2 / 2} e^{-beta s} for
    the unit-mass Gaussian G of width sigma, so f~(s) = e^{-beta^2 sigma^2 / 2} e^{-beta s},
    and w_i = N dt f~(t_i) on the nt midpoints of [lo, hi] (dt = (hi - lo)/nt, A's units).
    No periodic extension or window: the exponential grows without bound off the spectrum,
    and its periodic extension would not decay in Fourier space.  The sum is the midpoint
    rule for sum_j (f~ * G)(lambda_j) = sum_j e^{-beta lambda_j}; it needs the grid to cover
    each lambda_j - beta sigma^2 (the tilted Gaussian's centre) by several sigma.
    Given a lower bound spec_lo of the spectrum, the weights below spec_lo - beta sigma^2 -
    10 sigma are 0: the regularised DOS there is below e^{-50} of its values in exact
    arithmetic, and for beta > 0 the weights grow like e^{-beta t}, so they would only
    amplify the estimate's rounding."""
    dt = (hi - lo) / nt
    t = lo + dt * (np.arange(nt) + 0.5)
    w = n * dt * np.exp(-0.5 * (beta * sigma) ** 2 - beta * t)
    return np.where(t >= spec_lo - beta * sigma * sigma - 10.0 * sigma, w, 0.0)
