"""The allocation-free assembly entry point against the ordinary one.

tl_assemble_core_hamiltonian_block_noalloc runs the same kernels as
tl_assemble_core_hamiltonian_block with the scratch taken from a static device
array instead of a caller workspace, so H and S must be bitwise equal.  Two
calls follow each other on the same device, the second with a smaller system,
so the second runs on scratch that still holds the first call's values.
"""
import numpy as np
import pytest

from paper_1408_3839_amd import tl, workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.fail("no HIP device visible: the GPU tests need an MI355X")
    tl.load()


def _inputs(sys):
    h = tl.SystemHandle(sys)
    sz = tl.tl_query_sizes(h)
    f64 = dict(dtype=torch.float64, device="cuda:0")
    G = torch.empty(sz["basis_elems"], **f64)
    AG = torch.empty_like(G)
    SG = torch.empty_like(G)
    P = torch.empty(sz["pot_elems"], **f64)
    pws = tl.tl_potential_workspace_bytes(h)
    pw = torch.empty(max(1, pws), dtype=torch.uint8, device="cuda:0")
    tl.tl_build_basis(h, G, AG, SG)
    tl.tl_lattice_sum_potential(h, P, pw, pws)
    return h, sz, (G, AG, SG, P)


def _both(sys, prec, n_slices=0):
    """(H, S) from the ordinary call and from the allocation-free call."""
    h, sz, (G, AG, SG, P) = _inputs(sys)
    f64 = dict(dtype=torch.float64, device="cuda:0")
    wsb = tl.tl_assemble_workspace_bytes(h, prec, n_slices)
    ws = torch.empty(max(1, wsb), dtype=torch.uint8, device="cuda:0")
    H0 = torch.empty(sz["block_elems"], **f64)
    S0 = torch.empty_like(H0)
    tl.tl_assemble_core_hamiltonian_block(h, G, AG, SG, P, prec, n_slices, H0, S0, ws, wsb)
    H1 = torch.full_like(H0, float("nan"))
    S1 = torch.full_like(H0, float("nan"))
    tl.tl_assemble_core_hamiltonian_block_noalloc(h, G, AG, SG, P, prec, n_slices, H1, S1)
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in (H0, S0, H1, S1)]


def _bitwise(a, b):
    assert a.shape == b.shape
    assert np.array_equal(a.view(np.uint64), b.view(np.uint64))


@pytest.mark.parametrize("prec", [tl.TL_FP64, tl.TL_SPLIT_BF16, tl.TL_FP32])
def test_noalloc_two_calls_second_smaller(prec):
    big = wl.config(2)
    small = wl.tiny_periodic(L=(5, 1, 1), m0=5, c=7, h=0.25, R=9, alpha_range=(0.3, 4.0))
    for sys in (big, small):
        H0, S0, H1, S1 = _both(sys, prec)
        assert np.all(np.isfinite(H1)) and np.all(np.isfinite(S1))
        _bitwise(H0, H1)
        _bitwise(S0, S1)


@pytest.mark.parametrize("prec", [tl.TL_FP64, tl.TL_SPLIT_FP16])
def test_noalloc_open_chain_then_periodic(prec):
    chain = wl.box_chain_system("box12", 12, 1.5, [1.0, 2.0], 0.1, [400, 64, 72], 5,
                                (0.3, 4.0), 10, seed=21)
    for sys in (chain, wl.config(1)):
        H0, S0, H1, S1 = _both(sys, prec)
        assert np.all(np.isfinite(H1))
        _bitwise(H0, H1)
        _bitwise(S0, S1)
