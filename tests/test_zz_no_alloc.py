"""The allocation-free sigma entry point (static per-GPU scratch) against figaro_sigma.

Both run the same kernels; the outputs must agree bit for bit.  Two calls in a row, the
second with a smaller n, on each route (bidiagonal route for n <= 128, block Jacobi
above), show that the shared scratch keeps no state that a later call depends on.
"""
import ctypes

import numpy as np
import pytest

import paper_2503_23385_amd as fg

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def upper(n, seed):
    rng = np.random.default_rng(seed)
    return np.triu(rng.standard_normal((n, n)))


@pytest.mark.parametrize("sizes", [(512, 300), (300, 130), (128, 40), (100, 7)])
def test_noalloc_matches_sigma(sizes):
    d = dev()
    for k, n in enumerate(sizes):
        print(f"[noalloc] n={n} call {k}", flush=True)
        M = upper(n, 1000 + n)
        R = torch.from_numpy(M).to(d)
        ref = fg.sigma(R)
        out = torch.full((n,), float("nan"), dtype=torch.float64, device=d)
        fg.sigma_noalloc(R, out=out)
        torch.cuda.synchronize()
        a, b = out.cpu().numpy(), ref.cpu().numpy()
        assert np.all(np.isfinite(a))
        assert np.array_equal(a, b), (n, np.abs(a - b).max())
        lap = np.linalg.svd(M, compute_uv=False)
        assert np.linalg.norm(a - lap) / np.linalg.norm(lap) <= 1e-12


def test_noalloc_rejects_sizes_beyond_the_scratch():
    d = dev()
    R = torch.zeros((513, 513), dtype=torch.float64, device=d)
    S = torch.zeros(513, dtype=torch.float64, device=d)
    rc = fg.lib().figaro_sigma_noalloc(ctypes.c_void_p(R.data_ptr()), 513, 513, ctypes.c_void_p(S.data_ptr()), None)
    assert rc == fg.FIGARO_EINVAL
    assert b"static scratch" in fg.lib().figaro_last_error()
