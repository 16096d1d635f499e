"""Seeded synthetic inputs shared by the library's tests, its benchmark and the CPU oracle.

This module holds no step of the spectrum sweeping method itself. It only builds
what the method takes as input:

* sparse real symmetric matrices in CSR form (int32 ``row_ptr``/``col_idx``,
  float64 ``values``), of the kinds the paper's experiments use: finite
  difference operators with a potential (Section 6, model problem) and sparse
  graph Laplacians (the University of Florida matrices of Section 6 are not
  available here and are stood in for by random graphs);
* the Gaussian random block W of Section 2 (entries i.i.d. N(0,1)), drawn from a
  counter-based generator, Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11,
  "Parallel random numbers: as easy as 1, 2, 3"), mapped to normals by the
  Box-Muller transform;
* a spectral interval [lo, hi] that encloses the spectrum (Section 2 assumes
  one is known; here it comes from Gershgorin discs, widened so that the
  spectrum sits in (-a, a) after rescaling, as Algorithm 8 requires);
* a uniform midpoint grid of sweep points.

The HIP library implements its own Philox kernel; the two are compared in the
tests, and the same W drawn here can be handed to both sides.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# ----------------------------------------------------------------------------
# Philox4x32-10 and Box-Muller
# ----------------------------------------------------------------------------
PHILOX_M0 = 0xD2511F53
PHILOX_M1 = 0xCD9E8D57
PHILOX_W0 = 0x9E3779B9
PHILOX_W1 = 0xBB67AE85
_MASK32 = np.uint64(0xFFFFFFFF)


def philox4x32_10(ctr, key):
    """Philox4x32 with 10 rounds on a batch of counters.

    ``ctr`` is a sequence of four uint32 arrays (same shape), ``key`` a pair of
    ints.  Returns four uint32 arrays.  Definition from Salmon et al. (SC'11):
    each round multiplies words 0 and 2 by the two Philox constants, and the
    new state is (hi(w2*M1) ^ c1 ^ k0, lo(w2*M1), hi(w0*M0) ^ c3 ^ k1,
    lo(w0*M0)); the key is bumped by the two Weyl constants between rounds.
    """
    c0, c1, c2, c3 = (np.asarray(c, dtype=np.uint64) & _MASK32 for c in ctr)
    k0 = np.uint64(int(key[0]) & 0xFFFFFFFF)
    k1 = np.uint64(int(key[1]) & 0xFFFFFFFF)
    m0 = np.uint64(PHILOX_M0)
    m1 = np.uint64(PHILOX_M1)
    s32 = np.uint64(32)
    for r in range(10):
        if r:
            k0 = (k0 + np.uint64(PHILOX_W0)) & _MASK32
            k1 = (k1 + np.uint64(PHILOX_W1)) & _MASK32
        p0 = m0 * c0
        p1 = m1 * c2
        c0, c1, c2, c3 = ((p1 >> s32) ^ c1 ^ k0, p1 & _MASK32,
                          (p0 >> s32) ^ c3 ^ k1, p0 & _MASK32)
    return tuple(x.astype(np.uint32) for x in (c0, c1, c2, c3))


def gaussian_block(n: int, nv: int, seed: int, dtype=np.float64) -> np.ndarray:
    """The random block W (n x nv, row-major), entries N(0,1).

    Element (r, j), with j = 4g + m, is normal number m of the Philox block
    with counter (g, 0, r mod 2^32, r div 2^32) and key (seed mod 2^32,
    seed div 2^32).  Normals 0,1 come from words (x0, x1) and normals 2,3 from
    (x2, x3) by Box-Muller with u = (x_even + 1) 2^-32 in (0, 1] and
    v = x_odd 2^-32 in [0, 1): radius sqrt(-2 ln u), angles cos/sin(2 pi v).
    """
    ng = (nv + 3) // 4
    rows = np.repeat(np.arange(n, dtype=np.uint64), ng)
    grp = np.tile(np.arange(ng, dtype=np.uint64), n)
    x0, x1, x2, x3 = philox4x32_10(
        (grp, np.zeros_like(grp), rows & _MASK32, rows >> np.uint64(32)),
        (seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF))
    out = np.empty((n * ng, 4), dtype=np.float64)
    for (a, b), cols in (((x0, x1), (0, 1)), ((x2, x3), (2, 3))):
        u = (a.astype(np.float64) + 1.0) * 2.0 ** -32
        v = b.astype(np.float64) * 2.0 ** -32
        rad = np.sqrt(-2.0 * np.log(u))
        out[:, cols[0]] = rad * np.cos(2.0 * np.pi * v)
        out[:, cols[1]] = rad * np.sin(2.0 * np.pi * v)
    w = out.reshape(n, ng * 4)[:, :nv]
    return np.ascontiguousarray(w, dtype=dtype)


# ----------------------------------------------------------------------------
# CSR matrices
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class CSR:
    """Real symmetric sparse matrix: sorted column indices within each row."""
    n: int
    row_ptr: np.ndarray  # int32 (n+1)
    col_idx: np.ndarray  # int32 (nnz)
    values: np.ndarray   # float64 (nnz)

    @property
    def nnz(self) -> int:
        return int(self.col_idx.shape[0])

    def to_scipy(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.values, self.col_idx, self.row_ptr),
                             shape=(self.n, self.n))

    def to_dense(self) -> np.ndarray:
        return self.to_scipy().toarray()

    def shifted(self, c: float) -> "CSR":
        """A + cI (every row must store its diagonal)."""
        vals = self.values.copy()
        for r in range(self.n):
            lo, hi = self.row_ptr[r], self.row_ptr[r + 1]
            d = np.nonzero(self.col_idx[lo:hi] == r)[0]
            assert d.size == 1, "diagonal entry missing"
            vals[lo + d[0]] += c
        return CSR(self.n, self.row_ptr, self.col_idx, vals)


def _from_coo(n, rows, cols, vals) -> CSR:
    import scipy.sparse as sp
    m = sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr()
    m.sum_duplicates()
    m.sort_indices()
    return CSR(n, m.indptr.astype(np.int32), m.indices.astype(np.int32),
               m.data.astype(np.float64))


def laplacian_2d_dirichlet(nx: int, potential: np.ndarray | None = None) -> CSR:
    """5-point Dirichlet Laplacian on an nx x nx grid (4 on the diagonal, -1 to
    each of the up-to-4 neighbours), plus diag(potential)."""
    n = nx * nx
    idx = np.arange(n).reshape(nx, nx)
    rows = [idx.ravel()]
    cols = [idx.ravel()]
    vals = [np.full(n, 4.0) + (0.0 if potential is None else potential)]
    for a, b in ((idx[:-1, :], idx[1:, :]), (idx[:, :-1], idx[:, 1:])):
        a, b = a.ravel(), b.ravel()
        rows += [a, b]
        cols += [b, a]
        vals += [np.full(a.size, -1.0), np.full(a.size, -1.0)]
    return _from_coo(n, np.concatenate(rows), np.concatenate(cols), np.concatenate(vals))


def anderson_3d(nx: int, disorder: np.ndarray | None, hopping: float = -1.0) -> CSR:
    """3D 7-point periodic lattice: A_ii = disorder_i, A_ij = hopping for the six
    nearest neighbours (Anderson model)."""
    n = nx ** 3
    i = np.arange(n)
    x, y, z = i % nx, (i // nx) % nx, i // (nx * nx)
    rows = [i]
    cols = [i]
    vals = [np.zeros(n) if disorder is None else np.asarray(disorder, dtype=np.float64)]
    for dx, dy, dz in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
        j = ((x + dx) % nx) + ((y + dy) % nx) * nx + ((z + dz) % nx) * nx * nx
        rows.append(i)
        cols.append(j)
        vals.append(np.full(n, hopping))
    return _from_coo(n, np.concatenate(rows), np.concatenate(cols), np.concatenate(vals))


def er_graph_laplacian(n: int, mean_degree: int, rng: np.random.Generator) -> CSR:
    """Weighted Laplacian L = D - W of an Erdos-Renyi G(n, m) graph with
    m = mean_degree * n / 2 draws of (i, j), i != j; repeated pairs keep their
    first weight; weights uniform in (0, 1]."""
    m = mean_degree * n // 2
    i = rng.integers(0, n, size=m, dtype=np.int64)
    j = rng.integers(0, n, size=m, dtype=np.int64)
    w = 1.0 - rng.random(m)
    keep = i != j
    i, j, w = i[keep], j[keep], w[keep]
    a, b = np.minimum(i, j), np.maximum(i, j)
    key = a * n + b
    _, first = np.unique(key, return_index=True)
    a, b, w = a[first], b[first], w[first]
    deg = np.bincount(a, weights=w, minlength=n) + np.bincount(b, weights=w, minlength=n)
    rows = np.concatenate([a, b, np.arange(n)])
    cols = np.concatenate([b, a, np.arange(n)])
    vals = np.concatenate([-w, -w, deg])
    return _from_coo(n, rows, cols, vals)


def stencil27_lognormal(nx: int, rng: np.random.Generator) -> CSR:
    """Weighted graph Laplacian of the periodic 26-neighbour lattice (27-point
    stencil) with i.i.d. symmetric edge weights exp(N(0,1))."""
    n = nx ** 3
    i = np.arange(n, dtype=np.int64)
    x, y, z = i % nx, (i // nx) % nx, i // (nx * nx)
    offs = [(dx, dy, dz) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)
            if (dx, dy, dz) > (0, 0, 0)]
    rows, cols, vals = [], [], []
    deg = np.zeros(n)
    for dx, dy, dz in offs:  # 13 "forward" directions, each edge drawn once
        j = ((x + dx) % nx) + ((y + dy) % nx) * nx + ((z + dz) % nx) * nx * nx
        w = np.exp(rng.standard_normal(n))
        rows += [i, j]
        cols += [j, i]
        vals += [-w, -w]
        deg += w
        np.add.at(deg, j, w)
    rows.append(i)
    cols.append(i)
    vals.append(deg)
    return _from_coo(n, np.concatenate(rows), np.concatenate(cols), np.concatenate(vals))


def gershgorin(a: CSR) -> tuple[float, float]:
    """Union of Gershgorin discs of a real symmetric CSR matrix."""
    rows = np.repeat(np.arange(a.n), np.diff(a.row_ptr))
    diag = np.zeros(a.n)
    is_d = a.col_idx == rows
    diag[rows[is_d]] = a.values[is_d]
    rad = np.bincount(rows[~is_d], weights=np.abs(a.values[~is_d]), minlength=a.n)
    return float(np.min(diag - rad)), float(np.max(diag + rad))


# ----------------------------------------------------------------------------
# Workload descriptions
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class Workload:
    """A matrix plus the method's parameters, in A's units.

    ``sigma_hat`` is the smearing in the rescaled [-1, 1] variable and
    ``sigma = sigma_hat * hw`` the same smearing in A's units; the sweep points
    are the midpoints t_i = c0 + hw * (-1 + (2i+1)/nt)."""
    name: str
    a: CSR
    nv: int
    degree: int
    nt: int
    sigma_hat: float
    lo: float
    hi: float
    seed: int
    lattice: tuple | None = None  # (nx, ny, nz) when row x + nx (y + ny z) is lattice point (x, y, z)

    @property
    def c0(self) -> float:
        return 0.5 * (self.lo + self.hi)

    @property
    def hw(self) -> float:
        return 0.5 * (self.hi - self.lo)

    @property
    def sigma(self) -> float:
        return self.sigma_hat * self.hw

    @property
    def t(self) -> np.ndarray:
        return self.c0 + self.hw * midpoint_grid(self.nt)

    @property
    def dt(self) -> float:
        return 2.0 * self.hw / self.nt

    def w(self, dtype=np.float64) -> np.ndarray:
        return gaussian_block(self.a.n, self.nv, self.seed, dtype)


def midpoint_grid(nt: int) -> np.ndarray:
    """nt midpoints of a uniform partition of [-1, 1]."""
    return -1.0 + (2.0 * np.arange(nt) + 1.0) / nt


def interval(a: CSR, inner: float = 0.9) -> tuple[float, float]:
    """[lo, hi] such that the Gershgorin enclosure maps into [-inner, inner]."""
    g_lo, g_hi = gershgorin(a)
    c0 = 0.5 * (g_lo + g_hi)
    hw = 0.5 * (g_hi - g_lo) / inner
    return c0 - hw, c0 + hw


W_SEED = 0x5EED_0001


def make_matrix(cfg: int) -> CSR:
    """The synthetic matrix of workload ``cfg`` (numpy PCG64 seeded 1000+cfg)."""
    rng = np.random.Generator(np.random.PCG64(1000 + cfg))
    if cfg == 1:
        return laplacian_2d_dirichlet(32, rng.uniform(-1.0, 1.0, size=32 * 32))
    if cfg == 2:
        return anderson_3d(64, rng.uniform(-2.0, 2.0, size=64 ** 3))
    if cfg == 3:
        return er_graph_laplacian(1 << 20, 16, rng)
    if cfg == 4:
        a = make_matrix(2)
        g_lo, _ = gershgorin(a)
        return a.shifted(0.1 - g_lo)
    if cfg == 5:
        return stencil27_lognormal(128, rng)
    raise ValueError(f"no workload {cfg}")


_PARAMS = {  # nv, M, nt, sigma_hat
    1: (40, 200, 200, 0.05),
    2: (80, 1000, 1000, 0.01),
    3: (128, 2000, 2000, 0.005),
    4: (80, 1500, 1500, 10.0 / 1500),
    5: (256, 4000, 4000, 0.005),
}

NAMES = {
    1: "laplace2d_32x32_dirichlet_potential",
    2: "anderson3d_64cube_W4",
    3: "er_graph_laplacian_2p20_deg16",
    4: "anderson3d_64cube_W4_shifted_spd",
    5: "stencil27_128cube_lognormal",
}


LATTICES = {2: (64, 64, 64), 4: (64, 64, 64), 5: (128, 128, 128)}
LATTICE_N = {k: v[0] * v[1] * v[2] for k, v in LATTICES.items()}


def make_workload(cfg: int, a: CSR | None = None, **override) -> Workload:
    """Workload ``cfg`` with optional parameter overrides (nv, degree, nt,
    sigma_hat, seed)."""
    a = make_matrix(cfg) if a is None else a
    nv, m, nt, sh = _PARAMS[cfg]
    lo, hi = interval(a)
    kw = dict(name=NAMES[cfg], a=a, nv=nv, degree=m, nt=nt, sigma_hat=sh,
              lo=lo, hi=hi, seed=W_SEED, lattice=LATTICES.get(cfg) if a.n == LATTICE_N.get(cfg) else None)
    kw.update(override)
    return Workload(**kw)


def laplace2d_dirichlet_eigenvalues(nx: int) -> np.ndarray:
    """Closed-form spectrum of the nx x nx 5-point Dirichlet Laplacian:
    4 - 2 cos(i pi/(nx+1)) - 2 cos(j pi/(nx+1)), i, j = 1..nx."""
    th = np.arange(1, nx + 1) * math.pi / (nx + 1)
    return np.sort((4.0 - 2.0 * np.cos(th)[:, None] - 2.0 * np.cos(th)[None, :]).ravel())
