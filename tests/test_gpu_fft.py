"""Block FFT over the lattice index (Lemma 2.2, eq. (DiagMLcirc); the
Proposition on block-circulant diagonalisation) against the oracle's explicit
O(L^2) sums, for the LDS FFT (7-smooth extents by Stockham passes, other chain
lengths by Bluestein's chirp-z form) and the direct-DFT fallback of lattices
the LDS buffer cannot hold.

Bound: every output column (one entry (mu, nu) of one matrix over all k) is
compared relative to the largest input of that column,
    |X - X_ref| <= 2e-14 sqrt(L1 L2 L3) max_k |A_k[mu, nu]|,
which holds entry by entry even when columns differ by many orders of
magnitude (each column is scaled to unit maximum before two are packed into
one complex line).
"""
import math

import numpy as np
import pytest

import oracle
from paper_1408_3839_amd import tl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.fail("no HIP device visible: the GPU tests need an MI355X")
    tl.load()


def _gpu_fft(A):
    b, L1, L2, L3, m0, _ = A.shape
    inp = torch.from_numpy(np.ascontiguousarray(A)).cuda()
    out = torch.full(A.shape + (2,), float("nan"), dtype=torch.float64, device="cuda")
    wsb = tl.tl_block_fft_workspace_bytes(L1, L2, L3, m0, b)
    ws = torch.empty(max(1, wsb), dtype=torch.uint8, device="cuda")
    print(f"tl_block_fft L=({L1},{L2},{L3}) m0={m0} batch={b} ws={wsb}", flush=True)
    tl.tl_block_fft(inp, L1, L2, L3, m0, b, out, ws, wsb)
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    return o[..., 0] + 1j * o[..., 1]


def _reference(Ab):
    L1, L2, L3 = Ab.shape[:3]
    return oracle.block_dft_1level(Ab) if L2 == L3 == 1 else oracle.block_dft(Ab)


def _check(A, got):
    P = int(np.prod(A.shape[1:4]))
    for b in range(A.shape[0]):
        ref = _reference(A[b])
        colmax = np.abs(A[b]).max(axis=(0, 1, 2))          # [m0][m0]
        err = np.abs(got[b] - ref).max(axis=(0, 1, 2))
        bound = 2e-14 * math.sqrt(P) * colmax
        assert np.all(np.isfinite(got[b]))
        assert np.all(err <= bound), (float((err / np.maximum(bound, 1e-300)).max()))


def _random(shape, seed, spread=0.0):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal(shape)
    if spread:
        m0 = shape[-1]
        A *= np.exp(rng.uniform(-spread, spread, (m0, m0)))
    return A


# 7-smooth lengths (Stockham), chain lengths with other prime factors
# (Bluestein: 37, 61, 509 and 2039 prime, 2 * 211), and whole 3-level lattices
@pytest.mark.parametrize("shape", [
    (2, 512, 1, 1, 4), (2, 210, 1, 1, 3), (2, 2048, 1, 1, 1), (2, 37, 1, 1, 13),
    (2, 61, 1, 1, 8), (2, 509, 1, 1, 4), (2, 422, 1, 1, 2), (1, 2039, 1, 1, 2),
    (2, 8, 8, 8, 10), (2, 5, 6, 7, 2), (2, 3, 4, 5, 3), (2, 1, 6, 1, 4), (2, 2, 1, 9, 1),
    (1, 16, 16, 16, 1), (3, 1, 1, 1, 5), (2, 1, 1, 2, 3),
])
def test_lds_fft_parity(shape):
    b, L1, L2, L3, m0 = shape
    # no workspace but the Bluestein tables (at most L + 4096 complex values)
    assert tl.tl_block_fft_workspace_bytes(L1, L2, L3, m0, b) <= 16 * (L1 + 4096) + 256
    A = _random((b, L1, L2, L3, m0, m0), seed=sum(shape))
    _check(A, _gpu_fft(A))


@pytest.mark.parametrize("shape", [(2, 64, 1, 1, 8), (2, 8, 8, 8, 5), (2, 509, 1, 1, 3)])
def test_fft_columns_of_very_different_size(shape):
    """Entries spanning e^(+-25) within one block: each column keeps its own
    relative accuracy (power-of-two scaling before the packing)."""
    b, L1, L2, L3, m0 = shape
    A = _random((b, L1, L2, L3, m0, m0), seed=7 + sum(shape), spread=25.0)
    _check(A, _gpu_fft(A))


@pytest.mark.parametrize("shape", [(2, 11, 3, 1, 4), (1, 4099, 1, 1, 1), (1, 13, 1, 17, 2)])
def test_direct_dft_fallback_parity(shape):
    """Lattices the LDS FFT does not take: several axes with a prime factor
    above 7, or one chain longer than 2048 of non-7-smooth length."""
    b, L1, L2, L3, m0 = shape
    A = _random((b, L1, L2, L3, m0, m0), seed=3 + sum(shape))
    _check(A, _gpu_fft(A))


def test_fft_hermitian_blocks_of_symmetric_columns():
    """A block column with A_{-k} = A_k^T (the generating blocks of a symmetric
    block circulant) transforms to Hermitian blocks."""
    rng = np.random.default_rng(5)
    L, m0 = 509, 4
    A = rng.standard_normal((L, m0, m0))
    for k in range(1, L):
        A[L - k] = A[k].T if k < L - k else A[L - k]
    A[0] = 0.5 * (A[0] + A[0].T)
    got = _gpu_fft(A[None, :, None, None])[0, :, 0, 0]
    herm = np.abs(got - np.conj(np.swapaxes(got, -1, -2))).max()
    assert herm <= 1e-13 * np.abs(A).max() * math.sqrt(L)
