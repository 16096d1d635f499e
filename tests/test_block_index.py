"""The 2 x 2 rotation-block index of the Jacobi kernel (geneig.hip): a lane with linear index
idx takes block (j, k), j <= k, of the npairs x npairs upper triangle numbered row by row.
The kernel inverts row j's start j P - j (j - 1) / 2 with a float square root and corrects
by one step; this checks that arithmetic (float32 rounding, as on the device) against the
row walk for every index and every pair count the kernel supports (N_v <= 256)."""
import numpy as np


def _walk(p, idx):
    j, rem = 0, idx
    while rem >= p - j:
        rem -= p - j
        j += 1
    return j, j + rem


def _closed_form(p, idx):
    p2 = 2 * p + 1
    disc = (p2 * p2 - 8 * idx).astype(np.float32)
    j = ((np.float32(p2) - np.sqrt(disc)) * np.float32(0.5)).astype(np.int64)
    j = np.clip(j, 0, p - 1)
    start = j * p - j * (j - 1) // 2
    j = np.where(start > idx, j - 1, j)
    nxt = (j + 1) * p - (j + 1) * j // 2
    j = np.where(nxt <= idx, j + 1, j)
    return j, j + (idx - (j * p - j * (j - 1) // 2))


def test_block_index_matches_row_walk():
    for p in range(1, 129):
        idx = np.arange(p * (p + 1) // 2, dtype=np.int64)
        j, k = _closed_form(p, idx)
        ref = np.array([_walk(p, int(i)) for i in idx])
        assert np.array_equal(j, ref[:, 0]) and np.array_equal(k, ref[:, 1]), p
