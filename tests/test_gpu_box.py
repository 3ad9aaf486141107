"""Open-boundary chain (box mode): full H and S against the oracle's
entry-by-entry matrices."""
import numpy as np
import pytest

import oracle
from paper_1408_3839_amd import workloads as wl

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _small_box():
    return wl.box_chain_system("box12", 12, 1.5, [1.0, 2.0], 0.1, [400, 64, 72], 5, (0.3, 4.0),
                               10, seed=21)


def test_box_small_full_matrices():
    from paper_1408_3839_amd.pipeline import BoxPipeline
    s = _small_box()
    bp = BoxPipeline(s)
    bp.run()
    torch.cuda.synchronize()
    H = bp.H.cpu().numpy()
    S = bp.S.cpu().numpy()
    Hr, Sr = oracle.full_matrices(s)
    eh = np.abs(H - Hr).max() / np.abs(Hr).max()
    es = np.abs(S - Sr).max() / np.abs(Sr).max()
    print(f"box12: max|dH|/max|H| = {eh:.3e}, max|dS|/max|S| = {es:.3e}")
    assert np.array_equal(H, H.T) and np.array_equal(S, S.T)
    assert eh <= 1e-12 and es <= 1e-12


def test_box_chain_256_sampled_entries():
    """The 256-site chain (N_b = 2048, 8500 x 256 x 256 grid, R = 32): a
    sample of rows and columns (near the diagonal, far off it, both ends of
    the chain) against the oracle's entries."""
    from paper_1408_3839_amd.pipeline import BoxPipeline
    s = wl.config(3)
    bp = BoxPipeline(s)
    bp.run()
    torch.cuda.synchronize()
    H = bp.H
    S = bp.S
    assert torch.equal(H, H.T) and torch.equal(S, S.T)
    assert torch.isfinite(H).all() and torch.isfinite(S).all()
    rng = np.random.default_rng(3)
    rows = np.unique(np.concatenate([np.arange(0, 16), np.arange(1000, 1016), np.arange(2032, 2048),
                                     rng.integers(0, 2048, 16)]))
    cols = np.unique(np.concatenate([rows, rng.integers(0, 2048, 24)]))
    Hr, Sr = oracle.full_matrices(s, rows=rows, cols=cols)
    Hg = H.cpu().numpy()[np.ix_(rows, cols)]
    Sg = S.cpu().numpy()[np.ix_(rows, cols)]
    eh = np.abs(Hg - Hr).max() / np.abs(Hr).max()
    es = np.abs(Sg - Sr).max() / np.abs(Sr).max()
    print(f"chain256: max|dH|/max|H| = {eh:.3e}, max|dS|/max|S| = {es:.3e}")
    assert eh <= 1e-12 and es <= 1e-12


def test_box_chain_graph_replay():
    """The whole open-chain path (basis, potential, full H and S, lowest-k
    eigenpairs) captured once and replayed three times, with eager work and
    synchronisations between the replays: every replay equals the eager
    result bit for bit."""
    from paper_1408_3839_amd.pipeline import BoxPipeline
    s = _small_box()
    bp = BoxPipeline(s, k=16)
    bp.run()
    torch.cuda.synchronize()
    ref = [t.clone() for t in (bp.H, bp.S, bp.eig.evals, bp.eig.evecs, bp.eig.info)]
    bp.capture()
    for rep in range(3):
        for t in (bp.H, bp.S, bp.eig.evals, bp.eig.evecs):
            t.fill_(float("nan"))
        torch.cuda.synchronize()
        bp.replay()
        torch.cuda.synchronize()
        got = (bp.H, bp.S, bp.eig.evals, bp.eig.evecs, bp.eig.info)
        for a, b in zip(ref, got):
            assert torch.equal(a, b), rep
        x = torch.randn(1024, device="cuda") @ torch.randn(1024, device="cuda")  # eager work
        torch.cuda.synchronize()
        del x
