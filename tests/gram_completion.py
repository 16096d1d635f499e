"""The library's K_W from a computed W^T Z (its Gram kernel forms the upper 16 x 16 blocks
only): entry (r, c) of block (a, b), a < b, is (W^T Z)[r][c] and is mirrored to (c, r);
diagonal blocks are averaged with their transpose.  Equal to (W^T Z + Z^T W)/2 whenever
W^T Z is symmetric, as it is in exact arithmetic on the method's path."""
import numpy as np


def upper_completion(m: np.ndarray) -> np.ndarray:
    nv = m.shape[0]
    blk = np.arange(nv) // 16
    out = np.where(blk[:, None] < blk[None, :], m, m.T)
    return np.where(blk[:, None] == blk[None, :], 0.5 * (m + m.T), out)


def entry(wp, wq, zp, zq, p: int, q: int) -> float:
    """K_W[p][q] from columns p and q of W and of Z (float64 vectors)."""
    bp, bq = p // 16, q // 16
    if bp < bq:
        return float(wp @ zq)
    if bp > bq:
        return float(wq @ zp)
    return 0.5 * float(wp @ zq + wq @ zp)
