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


def _per_entry(A, Ar, scale, dr, dc):
    """|A - Ar| per entry against its no-cancellation scale, with the floor of
    the support cutoff: the dropped products are below exp(-46) ~ 1e-20 of
    either function's peak, so an entry moves by at most ~1e-18 of the
    geometric mean of the two functions' own diagonal scales.  A value <= 1e-10
    means |dA| <= 1e-10 scale + 1e-18 sqrt(scale_ff scale_gg)."""
    floor = 1e-8 * np.sqrt(np.outer(dr, dc))
    return np.abs(A - Ar) / (scale + floor)


def test_box_small_full_matrices():
    from paper_1408_3839_amd.pipeline import BoxPipeline
    s = _small_box()
    bp = BoxPipeline(s)
    bp.run()
    torch.cuda.synchronize()
    H = bp.H.cpu().numpy()
    S = bp.S.cpu().numpy()
    Hr, Sr = oracle.full_matrices(s)
    Ha, Sa = oracle.full_matrices(s, absolute=True)
    eh = np.abs(H - Hr).max() / np.abs(Hr).max()
    es = np.abs(S - Sr).max() / np.abs(Sr).max()
    ph = _per_entry(H, Hr, Ha, np.diag(Ha), np.diag(Ha))
    ps = _per_entry(S, Sr, Sa, np.diag(Sa), np.diag(Sa))
    print(f"box12: max|dH|/max|H| = {eh:.3e}, max|dS|/max|S| = {es:.3e}; per entry "
          f"{ph.max():.3e} / {ps.max():.3e}")
    assert np.array_equal(H, H.T) and np.array_equal(S, S.T)
    assert eh <= 1e-12 and es <= 1e-12
    assert ph.max() <= 1e-10 and ps.max() <= 1e-10


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
    Ha, Sa = oracle.full_matrices(s, rows=rows, cols=cols, absolute=True)
    both = np.union1d(rows, cols)
    Hd, Sd = oracle.full_matrices(s, rows=both, cols=both, absolute=True)
    pos = {f: i for i, f in enumerate(both)}
    ir, ic = [pos[f] for f in rows], [pos[f] for f in cols]
    Hg = H.cpu().numpy()[np.ix_(rows, cols)]
    Sg = S.cpu().numpy()[np.ix_(rows, cols)]
    eh = np.abs(Hg - Hr).max() / np.abs(Hr).max()
    es = np.abs(Sg - Sr).max() / np.abs(Sr).max()
    ph = _per_entry(Hg, Hr, Ha, np.diag(Hd)[ir], np.diag(Hd)[ic])
    ps = _per_entry(Sg, Sr, Sa, np.diag(Sd)[ir], np.diag(Sd)[ic])
    print(f"chain256: max|dH|/max|H| = {eh:.3e}, max|dS|/max|S| = {es:.3e}; per entry "
          f"{ph.max():.3e} / {ps.max():.3e}")
    for name, p_, A, Ar, Aa in (("H", ph, Hg, Hr, Ha), ("S", ps, Sg, Sr, Sa)):
        r_, c_ = np.unravel_index(np.argmax(p_), p_.shape)
        print(f"  worst {name}: f={rows[r_]} f'={cols[c_]} gpu={A[r_, c_]:.6e} oracle={Ar[r_, c_]:.6e} "
              f"scale={Aa[r_, c_]:.3e} max scale={Aa.max():.3e}")
    assert eh <= 1e-12 and es <= 1e-12
    assert ph.max() <= 1e-10 and ps.max() <= 1e-10


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


# (precision, slices, bound on max|dH| / max|H| and max|dS| / max|S|)
SPLIT_MODES = [("split_fp16", 3, 3e-7), ("split_fp16", 4, 1e-9), ("split_fp16", 5, 3e-12),
               ("split_fp16", 6, 1e-14), ("split_bf16", 4, 1e-8), ("split_bf16", 6, 1e-13),
               ("split_bf16", 7, 1e-14)]


@pytest.mark.parametrize("mode", SPLIT_MODES, ids=lambda m: f"{m[0]}-{m[1]}")
def test_box_small_split(mode):
    """Split-precision x contraction of the 12-site chain: every entry of H
    and S against the oracle, within a bound that shrinks as 2^(-beta s);
    H and S exactly symmetric."""
    from paper_1408_3839_amd.pipeline import BoxPipeline
    prec, ns, bound = mode
    s = _small_box()
    bp = BoxPipeline(s, precision=prec, n_slices=ns)
    bp.run()
    torch.cuda.synchronize()
    H = bp.H.cpu().numpy()
    S = bp.S.cpu().numpy()
    Hr, Sr = oracle.full_matrices(s)
    eh = np.abs(H - Hr).max() / np.abs(Hr).max()
    es = np.abs(S - Sr).max() / np.abs(Sr).max()
    print(f"box12 {prec} s={ns}: max|dH|/max|H| = {eh:.3e}, max|dS|/max|S| = {es:.3e}")
    assert np.array_equal(H, H.T) and np.array_equal(S, S.T)
    assert eh <= bound and es <= bound


@pytest.mark.parametrize("mode", [("split_fp16", 5), ("split_bf16", 6)],
                         ids=lambda m: f"{m[0]}-{m[1]}")
def test_box_chain_256_split_entries(mode):
    """The 256-site chain with the split x contraction: the sampled entries
    against the oracle, and every entry against the FP64 path."""
    from paper_1408_3839_amd.pipeline import BoxPipeline
    prec, ns = mode
    s = wl.config(3)
    bp = BoxPipeline(s, precision=prec, n_slices=ns)
    bp.run()
    b64 = BoxPipeline(s)
    b64.run()
    torch.cuda.synchronize()
    assert torch.equal(bp.H, bp.H.T) and torch.equal(bp.S, bp.S.T)
    dh = float((bp.H - b64.H).abs().max() / b64.H.abs().max())
    ds = float((bp.S - b64.S).abs().max() / b64.S.abs().max())
    rng = np.random.default_rng(5)
    rows = np.unique(np.concatenate([np.arange(0, 8), np.arange(1020, 1028), np.arange(2040, 2048),
                                     rng.integers(0, 2048, 8)]))
    cols = np.unique(np.concatenate([rows, rng.integers(0, 2048, 16)]))
    Hr, Sr = oracle.full_matrices(s, rows=rows, cols=cols)
    Hg = bp.H.cpu().numpy()[np.ix_(rows, cols)]
    Sg = bp.S.cpu().numpy()[np.ix_(rows, cols)]
    eh = np.abs(Hg - Hr).max() / np.abs(Hr).max()
    es = np.abs(Sg - Sr).max() / np.abs(Sr).max()
    print(f"chain256 {prec} s={ns}: vs FP64 path {dh:.3e} / {ds:.3e}; "
          f"sampled vs oracle {eh:.3e} / {es:.3e}")
    assert dh <= 1e-12 and ds <= 1e-12
    assert eh <= 1e-12 and es <= 1e-12


def test_chain_orbital_factors():
    """The open chain's orbitals as rank-m0 canonical tensors
    (tl_chain_orbital_factors): the lowest 4 orbitals of a 12-cell chain at
    sampled grid nodes against the oracle's expansion over every function of
    the same GPU eigenvector, and their FEM norm from the factors equal to 1
    (the eigenvectors are S-normalised)."""
    from paper_1408_3839_amd.pipeline import BoxPipeline
    s = wl.box_chain_system("c12", 12, 1.8, [1.0, 3.0], 0.0625, [600, 96, 96], 8, (0.1, 30.0),
                            16, seed=3)
    bp = BoxPipeline(s, k=4)
    bp.run()
    fac = bp.orbital_factors()
    torch.cuda.synchronize()
    F = fac.cpu().numpy()
    U = bp.eig.evecs.cpu().numpy()
    m0 = s.m0
    n = [int(v) for v in s.n]
    offs = np.cumsum([0] + [m0 * n[d] for d in range(3)])
    rng = np.random.default_rng(3)
    nodes = [(int(rng.integers(200, 400)), int(rng.integers(30, 66)), int(rng.integers(30, 66)))
             for _ in range(60)]
    for r in range(4):
        phi = [F[r, offs[d]:offs[d + 1]].reshape(m0, n[d]) for d in range(3)]
        got = np.array([np.sum(phi[0][:, a] * phi[1][:, b] * phi[2][:, c]) for a, b, c in nodes])
        ref = oracle.chain_orbital(s, U[r], nodes)
        err = np.abs(got - ref).max() / np.abs(ref).max()
        gram = np.ones((m0, m0))
        for d in range(3):
            gram *= phi[d] @ oracle.fem_mass(phi[d], False, s.h).T
        norm = gram.sum()
        print(f"\norbital {r}: max |dpsi| / max|psi| = {err:.2e}, FEM norm - 1 = {abs(norm - 1):.2e}")
        assert err <= 1e-12
        assert abs(norm - 1.0) <= 1e-8
