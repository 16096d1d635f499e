"""ssm_gram_noalloc, the Gram stage call for callers that cannot allocate device memory
(its partial sums go to the library's static device array), against ssm_gram with a
caller scratch buffer on the same inputs: the same kernels and the same fixed-order sums,
so the results must be identical.  Two calls in a row, the second with a smaller input
(fewer rows, columns, points and segments), each checked; and the size limit."""
import numpy as np
import pytest
import torch

from paper_1504_07690_amd import _abi as A

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def S():
    from paper_1504_07690_amd import ssm
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return ssm


def _inputs(precision, n, nv, ntb, seed):
    rng = np.random.default_rng(seed)
    dt = torch.float64 if precision == "fp64" else torch.float32
    w = torch.tensor(rng.standard_normal((n, nv)), dtype=dt, device=DEV)
    z = torch.tensor(rng.standard_normal((ntb, n, nv)), dtype=dt, device=DEV)
    return w, z


CALLS = [("fp64", 4000, 96, 8, 5), ("fp32", 1500, 40, 3, 2)]  # the second call is smaller


def test_gram_noalloc_matches_gram(S):
    for j, (precision, n, nv, ntb, nseg) in enumerate(CALLS):
        print(f"call {j}: {precision} n={n} nv={nv} ntb={ntb} nseg={nseg}", flush=True)
        w, z = _inputs(precision, n, nv, ntb, 10 + j)
        kw = torch.empty(ntb, nv, nv, dtype=torch.float64, device=DEV)
        kz = torch.empty_like(kw)
        S.gram(precision, w, z, kw, kz, nseg)
        kw2 = torch.full_like(kw, float("nan"))
        kz2 = torch.full_like(kz, float("nan"))
        S.gram_noalloc(precision, w, z, kw2, kz2, nseg)
        torch.cuda.synchronize()
        assert torch.equal(kw2, kw) and torch.equal(kz2, kz), j


def test_gram_noalloc_size_limit(S):
    """Partial sums beyond the static array are refused before any device work."""
    w, z = _inputs("fp32", 64, 256, 1, 3)
    kw = torch.empty(1, 256, 256, dtype=torch.float64, device=DEV)
    kz = torch.empty_like(kw)
    # 4 nseg ntb 2 nv^2 doubles: nseg = 9, ntb = 1, nv = 256 -> 37.7 MB > 32 MiB
    st = A.lib.ssm_gram_noalloc(1, 64, 256, 1, w.data_ptr(), z.data_ptr(), kw.data_ptr(), kz.data_ptr(), 9, None)
    assert st == A.SSM_ERR_UNSUPPORTED
    S.gram_noalloc("fp32", w, z, kw, kz, 7)  # 29.4 MB fits
