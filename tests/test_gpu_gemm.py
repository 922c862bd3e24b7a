"""GPU unit test of the library's grouped fp64 and fp32 MFMA GEMM against numpy."""
import numpy as np
import pytest

from gpu_util import say

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _colmajor(x):
    return torch.tensor(np.asfortranarray(x), device="cuda:0").t().contiguous().t()


@pytest.mark.parametrize("m,n,k,ta,tb", [(16, 16, 4, 0, 0), (64, 64, 16, 0, 0), (70, 33, 45, 0, 0),
                                         (130, 7, 200, 0, 0), (50, 60, 70, 1, 0), (50, 60, 70, 0, 1),
                                         (50, 60, 70, 1, 1), (1, 1, 1, 0, 0),
                                         # few tiles, long K: split-K with a second reduction pass
                                         (130, 7, 2000, 0, 0), (200, 16, 3584, 1, 0), (64, 16, 1000, 0, 1),
                                         # N <= 16, neither operand transposed: the skinny path
                                         (56, 16, 196, 0, 0), (200, 16, 3584, 0, 0), (33, 3, 9, 0, 0)])
def test_gemm_matches_numpy(m, n, k, ta, tb):
    import paper_2503_17535_amd as hp
    say(f"[case] gemm {m}x{n}x{k} ta={ta} tb={tb}")
    g = np.random.default_rng(m * 1000 + n * 10 + k)
    A = g.normal(size=(k, m) if ta else (m, k))
    B = g.normal(size=(n, k) if tb else (k, n))
    C = g.normal(size=(m, n))
    ref = 0.7 * (A.T if ta else A) @ (B.T if tb else B) - 0.3 * C
    Cd = _colmajor(C)
    hp.debug_gemm(_colmajor(A), _colmajor(B), Cd, alpha=0.7, beta=-0.3, trans_a=bool(ta), trans_b=bool(tb))
    torch.cuda.synchronize()
    np.testing.assert_allclose(Cd.cpu().numpy(), ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())


@pytest.mark.parametrize("m,n,k,ta,tb", [(16, 16, 4, 0, 0), (70, 33, 45, 0, 0), (130, 7, 200, 0, 0),
                                         (50, 60, 70, 1, 0), (50, 60, 70, 1, 1), (130, 7, 2000, 0, 0),
                                         (56, 16, 196, 0, 0)])
def test_gemm_f32_matches_numpy(m, n, k, ta, tb):
    # fp32 products with fp32 accumulation: error bound ~ k * 2^-24 * |A||B|
    import paper_2503_17535_amd as hp
    say(f"[case] gemm f32 {m}x{n}x{k} ta={ta} tb={tb}")
    g = np.random.default_rng(m * 1000 + n * 10 + k + 7)
    A = g.normal(size=(k, m) if ta else (m, k)).astype(np.float32)
    B = g.normal(size=(n, k) if tb else (k, n)).astype(np.float32)
    C = g.normal(size=(m, n)).astype(np.float32)
    A64, B64, C64 = A.astype(np.float64), B.astype(np.float64), C.astype(np.float64)
    ref = 0.7 * (A64.T if ta else A64) @ (B64.T if tb else B64) - 0.3 * C64
    Cd = _colmajor(C)
    hp.debug_gemm(_colmajor(A), _colmajor(B), Cd, alpha=0.7, beta=-0.3, trans_a=bool(ta), trans_b=bool(tb))
    torch.cuda.synchronize()
    scale = 0.7 * np.abs(A64).max() * np.abs(B64).max() * k + 0.3 * np.abs(C64).max()
    assert np.abs(Cd.cpu().numpy() - ref).max() < 4 * k * 2.0 ** -24 * scale
