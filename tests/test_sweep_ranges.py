"""Load ranges of the split-BF16 sweep's Y operand (sweep_gemm.hip), on the host.

Lane t of a wave reads two floats at column c = 2 t of the tile's 256 columns (clamped to
the last pair of the block when the tile is ragged), for 8 consecutive degrees kb .. kb+7.
Where 28 e + 1024 < 2^31 the 8 loads share one buffer resource based at degree kb, with
record count (rows - 1) 4 e + min(4 (e - q0), 1024), rows = the degrees of the 8 below kc;
degree j sits at byte offset 4 j e past the lane's.  A raw buffer load returns zeros unless
it lies inside the records.  This checks, for every lane and degree:
* a degree below kc reads its own row at the lane's column, entirely inside the records;
* a degree at or past kc starts past the records (reads zero);
* every byte inside the records lies within the kc rows of the block;
* every offset fits in 31 bits.
"""
import numpy as np
import pytest


def _ranges(e, kc, q0):
    t = np.arange(128)
    c2 = 2 * t
    boff = np.where(q0 + c2 < e, c2, e - 2 - q0) * 4
    last = min((e - q0) * 4, 1024)
    j = np.arange(8)
    for kb in range(0, kc + 24, 8):
        rows = min(kc - kb, 8) if kb < kc else 0
        base = (kb if kb < kc else 0) * e + q0  # floats from the block's start
        nrec = (rows - 1) * e * 4 + last if rows else 0
        off = boff[:, None] + (j * e * 4)[None, :]
        yield kb, rows, base, nrec, off, boff


@pytest.mark.parametrize("e", [4, 12, 100, 252, 256, 260, 1000, 1024, 4096 + 8, 262144 * 80])
@pytest.mark.parametrize("kc", [1, 5, 8, 9, 33, 288, 1001])
def test_shared_resource_ranges(e, kc):
    assert 28 * e + 1024 < 2 ** 31
    ntiles = (e + 255) // 256
    for q0 in sorted({0, 256 * (ntiles - 1)}):
        for kb, rows, base, nrec, off, boff in _ranges(e, kc, q0):
            assert nrec < 2 ** 31 and off.max() < 2 ** 31
            valid = np.arange(8)[None, :] < rows
            assert np.all(off[:, :rows] + 8 <= nrec)
            assert np.all(off[:, rows:] >= nrec)
            row, col = np.divmod(base + off // 4, e)
            assert np.all(np.where(valid, row == kb + np.arange(8)[None, :], True))
            assert np.all(np.where(valid, col == q0 + boff[:, None] // 4, True))
            inside = off < nrec
            assert np.all(np.where(inside, base * 4 + off + 8 <= kc * e * 4, True))

