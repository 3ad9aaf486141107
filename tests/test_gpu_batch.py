"""The batched path (one launch per stage for a ragged batch) against the
single-system path and the FP64 oracle."""
import numpy as np
import pytest
import scipy.linalg as sla

import oracle
from paper_1408_3839_amd import workloads as wl

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _same_evals(a, b):
    """Batch and single launches bisect with different point schedules: the
    eigenvalues agree to the bisection tolerance (a few ulps of the spectrum's
    scale), not bit for bit."""
    a, b = a.cpu().numpy(), b.cpu().numpy()
    assert np.array_equal(np.isnan(a), np.isnan(b))
    ok = ~np.isnan(a)
    scale = np.max(np.abs(a[ok]), initial=1.0)
    return bool(np.all(np.abs(a[ok] - b[ok]) <= 64 * 2.0 ** -52 * max(1.0, scale)))


def _ragged():
    out = []
    specs = [(6, 3, 8), (9, 5, 7), (4, 1, 6), (13, 8, 10), (7, 13, 9), (16, 4, 12)]
    for i, (L, m0, c) in enumerate(specs):
        out.append(wl.tiny_periodic(L=(L, 1, 1), m0=m0, c=c, h=0.25, R=10, seed=50 + i,
                                    alpha_range=(0.3, 5.0)))
    return out


@pytest.mark.parametrize("precision,slices", [("fp64", 0), ("split_bf16", 6), ("fp32", 0)])
def test_batch_equals_single(precision, slices):
    from paper_1408_3839_amd.pipeline import BatchPipeline, PeriodicPipeline
    systems = _ragged()
    bp = BatchPipeline(systems, precision=precision, n_slices=slices)
    bp.run()
    torch.cuda.synchronize()
    for s, v in zip(systems, bp.views):
        sp = PeriodicPipeline(s, precision=precision, n_slices=slices)
        sp.run()
        torch.cuda.synchronize()
        assert torch.equal(v["H"], sp.H), s.name
        assert torch.equal(v["S"], sp.S), s.name
        assert _same_evals(v["evals"], sp.evals), s.name
        assert torch.equal(v["info"], sp.info), s.name


@pytest.mark.parametrize("lengths", [(11, 13), (8, 9)], ids=["bluestein_only", "smooth_only"])
def test_batch_single_kind_fft(lengths):
    """Batches whose chain lengths all take one of the two transform kernels
    (Bluestein, or Stockham for 7-smooth lengths): the other launch is
    skipped and the stage events go with the one that runs."""
    from paper_1408_3839_amd import tl
    from paper_1408_3839_amd.pipeline import BatchPipeline, PeriodicPipeline
    systems = [wl.tiny_periodic(L=(L, 1, 1), m0=m0, c=6, h=0.25, R=8, seed=70 + i,
                                alpha_range=(0.3, 5.0))
               for i, (L, m0) in enumerate(zip(lengths, (3, 5)))]
    bp = BatchPipeline(systems)
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    e1.record(stream)
    tl.tl_set_stage_events(tl.TL_STAGE_FFT, e0.cuda_event, e1.cuda_event)
    try:
        bp.run()
    finally:
        tl.tl_set_stage_events(tl.TL_STAGE_FFT, None, None)
    torch.cuda.synchronize()
    assert e0.elapsed_time(e1) > 0.0
    for s, v in zip(systems, bp.views):
        sp = PeriodicPipeline(s)
        sp.run()
        torch.cuda.synchronize()
        assert torch.equal(v["H"], sp.H), s.name
        assert _same_evals(v["evals"], sp.evals), s.name
        Hr, Sr, _ = oracle.core_hamiltonian_blocks(s)
        Hb = oracle.block_dft(Hr).reshape(-1, s.m0, s.m0)
        Sb = oracle.block_dft(Sr).reshape(-1, s.m0, s.m0)
        ev = v["evals"].cpu().numpy()
        for j in range(Hb.shape[0]):
            lam, U = sla.eigh(Hb[j], Sb[j])
            un = np.sum(np.abs(U) ** 2, axis=0)
            tol = 1e-10 * np.maximum(1, np.abs(lam)) + 256 * 2.0 ** -52 * (
                np.linalg.norm(Hb[j], 2) + np.abs(lam) * np.linalg.norm(Sb[j], 2)) * un
            assert np.all(np.abs(ev[j] - lam) <= tol), (s.name, j)


def test_batch_parity_with_oracle():
    from paper_1408_3839_amd.pipeline import BatchPipeline
    systems = _ragged()
    bp = BatchPipeline(systems)
    bp.run()
    torch.cuda.synchronize()
    for s, v in zip(systems, bp.views):
        Hr, Sr, scale = oracle.core_hamiltonian_blocks(s)
        H = v["H"].cpu().numpy()
        assert np.all(np.abs(H - Hr) <= 1e-10 * scale + 1e-290), s.name
        Hb = oracle.block_dft(Hr).reshape(-1, s.m0, s.m0)
        Sb = oracle.block_dft(Sr).reshape(-1, s.m0, s.m0)
        ev = v["evals"].cpu().numpy()
        for j in range(Hb.shape[0]):
            lam, U = sla.eigh(Hb[j], Sb[j])
            un = np.sum(np.abs(U) ** 2, axis=0)
            tol = 1e-10 * np.maximum(1, np.abs(lam)) + 256 * 2.0 ** -52 * (
                np.linalg.norm(Hb[j], 2) + np.abs(lam) * np.linalg.norm(Sb[j], 2)) * un
            assert np.all(np.abs(ev[j] - lam) <= tol), (s.name, j)


def test_batch_graph_replay():
    from paper_1408_3839_amd.pipeline import BatchPipeline
    bp = BatchPipeline(_ragged())
    bp.run()
    torch.cuda.synchronize()
    ref = bp.buf["evals"].clone()
    refH = bp.buf["HS"].clone()
    bp.capture()
    for rep in range(3):
        bp.buf["evals"].fill_(0.0)
        bp.buf["HS"].fill_(0.0)
        torch.cuda.synchronize()
        bp.replay()
        torch.cuda.synchronize()
        assert torch.equal(bp.buf["evals"], ref) and torch.equal(bp.buf["HS"], refH), rep
        bp.run()
        torch.cuda.synchronize()


def test_ragged_64_chain_batch():
    """The 64-instance ragged batch (L in [16, 512], m0 in {4, 8, 13}): every
    instance equals its single-system run on a sample, the smallest ones match
    the oracle, and every k-block is solved or flagged."""
    from paper_1408_3839_amd.pipeline import BatchPipeline, PeriodicPipeline
    systems = wl.batch(64)
    bp = BatchPipeline(systems)
    bp.run()
    torch.cuda.synchronize()
    info = bp.buf["info"].cpu().numpy()
    assert np.all(info >= 0)
    # every flagged k-block has a numerically singular Sbar_j (smallest
    # eigenvalue within rounding of zero), every clearly definite one is solved
    hsbar = bp.buf["HSbar"].cpu().numpy()
    eps = 2.0 ** -52
    off = ok_ = 0
    flagged = 0
    for s, v in zip(systems, bp.views):
        L, m0 = int(s.L[0]), s.m0
        be = L * m0 * m0
        Sb = hsbar[2 * (off + be):2 * (off + 2 * be)].reshape(L, m0, m0, 2)
        Sb = Sb[..., 0] + 1j * Sb[..., 1]
        inf = v["info"].cpu().numpy()
        for j in range(L):
            w = np.linalg.eigvalsh(0.5 * (Sb[j] + Sb[j].conj().T))
            tiny = 64 * m0 * eps * np.abs(w).max()
            if inf[j] > 0:
                flagged += 1
                assert w[0] <= tiny, (s.name, j, w[0], tiny)
            elif w[0] > 1e3 * tiny:
                ok_ += 1
            if w[0] > 1e3 * tiny:
                assert inf[j] == 0, (s.name, j)
        off += 2 * be
    print(f"\nragged batch: {int(np.sum(info > 0))} of {info.size} k-blocks flagged "
          f"(Sbar_j not numerically definite), {ok_} clearly definite and solved")
    assert flagged == int(np.sum(info > 0))
    order = np.argsort([int(s.L[0]) for s in systems])
    for i in list(order[:3]) + [int(order[-1])]:
        s, v = systems[i], bp.views[i]
        sp = PeriodicPipeline(s)
        sp.run()
        torch.cuda.synchronize()
        assert torch.equal(v["H"], sp.H) and _same_evals(v["evals"], sp.evals), s.name
    for i in order[:2]:
        s, v = systems[i], bp.views[i]
        Hr, Sr, scale = oracle.core_hamiltonian_blocks(s)
        assert np.all(np.abs(v["H"].cpu().numpy() - Hr) <= 1e-10 * scale + 1e-290), s.name


def test_autotune_picks_and_caches(tmp_path):
    """The autotuner times every (tile edge, tiling target) pair, keeps the
    fastest in its cache, answers the next call from the cache, and the tuned
    batch still matches the oracle; both tile edges give the same H bit for
    bit up to the summation order inside a tile (checked against the oracle)."""
    from paper_1408_3839_amd import autotune
    from paper_1408_3839_amd.pipeline import BatchPipeline
    systems = _ragged()
    cache = str(tmp_path / "tuning.json")
    cands = (128, 512, 2048)
    best, times = autotune.tune_batch(systems, candidates=cands, reps=2, cache_path=cache)
    assert set(times) == {f"{e}x{c}" for e in (64, 32) for c in cands}
    assert f"{best[1]}x{best[0]}" == min(times, key=times.get)
    assert all(t > 0 for t in times.values())
    best2, times2 = autotune.tune_batch(systems, candidates=cands, reps=2, cache_path=cache)
    assert best2 == best and times2 == times
    for edge in (64, 32):
        bp = BatchPipeline(systems, want_blocks=best[0], tile_edge=edge)
        bp.run()
        torch.cuda.synchronize()
        for s, v in zip(systems[:2], bp.views[:2]):
            Hr, Sr, scale = oracle.core_hamiltonian_blocks(s)
            assert np.all(np.abs(v["H"].cpu().numpy() - Hr) <= 1e-10 * scale + 1e-290)
    # the split modes have one tile shape: only the tiling target is timed
    _, ts = autotune.tune_batch(systems, precision="split_fp16", n_slices=5, candidates=cands,
                                reps=1, cache_path=None)
    assert set(ts) == {f"64x{c}" for c in cands}
