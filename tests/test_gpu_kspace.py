"""Fourier-side combination (tl_assemble_kblocks): the k-blocks from the 1D
DFTs of the contraction factors against the oracle's explicit block DFT of
its real-space block column, against the GPU block-FFT route, and the
k-block eigenvalues."""
import numpy as np
import pytest
import scipy.linalg as sla

import oracle
from paper_1408_3839_amd import workloads as wl

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

CASES = {
    "c1": lambda: wl.config(1),
    "c5": lambda: wl.config(5),
    "tiny_3d": lambda: wl.tiny_periodic(L=(3, 2, 2), m0=4, c=4, h=0.5, R=6, K=(1, 1, 1),
                                        sites=((0, 0, 0), (0.5, 0.5, -0.5)), Z=(1.0, 2.0)),
    "tiny_432": lambda: wl.tiny_periodic(L=(4, 3, 2), m0=3, c=4, h=0.5, R=6, K=(2, 1, 1)),
    "tiny_L5_c7": lambda: wl.tiny_periodic(L=(5, 1, 1), m0=5, c=7, h=0.25, R=9,
                                           alpha_range=(0.3, 4.0)),
    "tiny_1L4": lambda: wl.tiny_periodic(L=(1, 4, 1), m0=2, c=6, h=0.5, R=6, K=(0, 2, 0)),
    # (T+2)(L1+L2+L3) = 42 * 130: the two-kernel form (factor DFTs in the workspace)
    "chain128_R40": lambda: wl.tiny_periodic(L=(128, 1, 1), m0=2, c=4, h=0.5, R=40),
}
_ref = {}


def _oracle(name):
    if name not in _ref:
        s = CASES[name]()
        H, S, _ = oracle.core_hamiltonian_blocks(s)
        dft = oracle.block_dft_1level if s.L[1] == s.L[2] == 1 else oracle.block_dft
        _ref[name] = (s, dft(H), dft(S))
    return _ref[name]


def _run(s, route, precision="fp64", n_slices=0):
    from paper_1408_3839_amd.pipeline import PeriodicPipeline
    pl = PeriodicPipeline(s, precision=precision, n_slices=n_slices, route=route)
    pl.run()
    torch.cuda.synchronize()
    hs = pl.HSbar.cpu().numpy()
    Hb = (hs[0, :, 0] + 1j * hs[0, :, 1]).reshape(*pl.L, pl.m0, pl.m0)
    Sb = (hs[1, :, 0] + 1j * hs[1, :, 1]).reshape(*pl.L, pl.m0, pl.m0)
    return pl, Hb, Sb


@pytest.mark.parametrize("name", list(CASES))
def test_kspace_blocks_match_oracle(name):
    s, Hr, Sr = _oracle(name)
    pl, Hb, Sb = _run(s, "kspace")
    eh = np.abs(Hb - Hr).max() / np.abs(Hr).max()
    es = np.abs(Sb - Sr).max() / np.abs(Sr).max()
    _, Hf, Sf = _run(s, "block_fft")
    df = max(np.abs(Hb - Hf).max() / np.abs(Hf).max(), np.abs(Sb - Sf).max() / np.abs(Sf).max())
    # Hermitian k-blocks (to rounding: the two triangles are separate sums)
    herm = np.abs(Hb - np.conj(np.swapaxes(Hb, -1, -2))).max() / np.abs(Hb).max()
    print(f"\n{name}: k-space vs oracle {eh:.2e} / {es:.2e}, vs block-FFT route {df:.2e}, "
          f"Hermitian defect {herm:.2e}")
    assert eh <= 1e-12 and es <= 1e-12
    assert df <= 1e-12 and herm <= 1e-13


@pytest.mark.parametrize("name", ["c1", "c5", "tiny_3d"])
def test_kspace_eigenvalues(name):
    """Eigenvalues of the k-space route against LAPACK on the oracle's
    k-blocks, within the first-order bound of the block error."""
    s, Hr, Sr = _oracle(name)
    pl, Hb, Sb = _run(s, "kspace")
    ev = pl.evals.cpu().numpy().reshape(-1, s.m0)
    assert np.all(pl.info.cpu().numpy() == 0)
    Hr2, Sr2 = Hr.reshape(-1, s.m0, s.m0), Sr.reshape(-1, s.m0, s.m0)
    dH = np.abs(Hb.reshape(Hr2.shape) - Hr2).max()
    dS = np.abs(Sb.reshape(Sr2.shape) - Sr2).max()
    worst = 0.0
    for j in range(Hr2.shape[0]):
        lam, U = sla.eigh(Hr2[j], Sr2[j])
        un = np.sum(np.abs(U) ** 2, axis=0)
        nh, ns = np.linalg.norm(Hr2[j], 2), np.linalg.norm(Sr2[j], 2)
        tol = (s.m0 * (dH + np.abs(lam) * dS) + 256 * 2.0 ** -52 * (nh + np.abs(lam) * ns)) * un
        d = np.abs(ev[j] - lam)
        assert np.all(d <= 4 * tol + 1e-12 * np.maximum(1, np.abs(lam))), (j, d, tol)
        worst = max(worst, float(d.max()))
    print(f"\n{name}: max |d lambda| = {worst:.3e} Ha")


@pytest.mark.parametrize("mode", [("split_fp16", 5), ("split_bf16", 6), ("fp32", 0)],
                         ids=lambda m: f"{m[0]}-{m[1]}")
def test_kspace_reduced_precision(mode):
    """The k-space route over the reduced-precision contractions equals the
    block-FFT route over the same contractions (same factors, different
    order of the DFT and the products)."""
    prec, ns = mode
    s = wl.config(5)
    _, Hk, Sk = _run(s, "kspace", prec, ns)
    _, Hf, Sf = _run(s, "block_fft", prec, ns)
    d = max(np.abs(Hk - Hf).max() / np.abs(Hf).max(), np.abs(Sk - Sf).max() / np.abs(Sf).max())
    print(f"\nc5 {prec} s={ns}: k-space vs block-FFT route {d:.2e}")
    assert d <= 1e-12


def test_kspace_route_graph_replay():
    """The k-space route captured in one HIP graph (basis and potential,
    contraction, reduction, fused factor DFTs and combination, k-block
    eigensolves) and replayed three times with eager work and
    synchronisations between the replays: every replay equals the eager run
    bit for bit."""
    from paper_1408_3839_amd.pipeline import PeriodicPipeline
    pl = PeriodicPipeline(wl.config(5), route="kspace")
    pl.run()
    torch.cuda.synchronize()
    ref = (pl.HSbar.clone(), pl.evals.clone(), pl.info.clone())
    pl.capture()
    for rep in range(3):
        pl.HSbar.fill_(float("nan"))
        pl.evals.fill_(float("nan"))
        torch.cuda.synchronize()
        pl.replay()
        torch.cuda.synchronize()
        assert torch.equal(pl.HSbar, ref[0]) and torch.equal(pl.evals, ref[1]), rep
        assert torch.equal(pl.info, ref[2]), rep
        pl.run()
        torch.cuda.synchronize()
