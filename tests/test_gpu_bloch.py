"""Bloch eigenvectors (tl_bloch_vectors, eq. (eigvecA)): the full-lattice
eigenvectors built on the GPU from the k-block eigenvectors against the
oracle's Kronecker-product form applied to the same k-block vectors, and as
eigenvectors of the full pencil assembled by the oracle."""
import numpy as np
import pytest

import oracle
from paper_1408_3839_amd import workloads as wl

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

CASES = {
    "c1": lambda: wl.config(1),
    "tiny_3d": lambda: wl.tiny_periodic(L=(3, 2, 2), m0=4, c=4, h=0.5, R=6, K=(1, 1, 1),
                                        sites=((0, 0, 0), (0.5, 0.5, -0.5)), Z=(1.0, 2.0)),
    "tiny_432": lambda: wl.tiny_periodic(L=(4, 3, 2), m0=3, c=4, h=0.5, R=6, K=(2, 1, 1)),
    "tiny_L5_c7": lambda: wl.tiny_periodic(L=(5, 1, 1), m0=5, c=7, h=0.25, R=9,
                                           alpha_range=(0.3, 4.0)),
}


def _run(s):
    from paper_1408_3839_amd.pipeline import PeriodicPipeline
    pl = PeriodicPipeline(s, with_evecs=True)
    pl.run()
    torch.cuda.synchronize()
    return pl


def _cx(t):
    a = t.cpu().numpy()
    return a[..., 0] + 1j * a[..., 1]


@pytest.mark.parametrize("name", list(CASES))
def test_bloch_vectors_all_states(name):
    s = CASES[name]()
    pl = _run(s)
    nc, m0 = pl.nblocks, pl.m0
    states = np.arange(nc * m0)
    U = _cx(pl.bloch_vectors(states)).reshape(len(states), nc * m0)
    u = _cx(pl.evecs)
    ref = oracle.bloch_vectors(u, pl.L, states)
    d = np.abs(U - ref).max() / np.abs(ref).max()
    # eigenvectors of the full pencil (oracle matrices), S-orthonormal across k
    Hf, Sf = oracle.full_matrices(s)
    lam = pl.evals.cpu().numpy().ravel()
    Ut = U.T
    R = Hf @ Ut - (Sf @ Ut) * lam[None, :]
    scale = np.linalg.norm(Hf, 2) + np.abs(lam) * np.linalg.norm(Sf, 2)
    res = np.linalg.norm(R, axis=0) / (scale * np.linalg.norm(Ut, axis=0))
    G = Ut.conj().T @ Sf @ Ut
    print(f"\n{name}: vs oracle form {d:.2e}, max residual {res.max():.2e}, "
          f"max |U^H S U - I| {np.abs(G - np.eye(len(states))).max():.2e}")
    assert d <= 1e-14
    assert res.max() <= 1e-10
    assert np.abs(G - np.eye(len(states))).max() <= 1e-8


def test_bloch_vectors_subset_and_invalid_state():
    """A chosen subset in any order (here c2's lowest band at every k-point,
    reversed, and one band of one k-point twice), checked against the
    block-circulant matrices of the oracle's generating blocks; an index
    outside the lattice's states gives a NaN row."""
    s = wl.config(2)
    pl = _run(s)
    nc, m0 = pl.nblocks, pl.m0
    states = list(reversed([j * m0 for j in range(nc)])) + [5 * m0 + 3, 5 * m0 + 3, nc * m0, -1]
    U = _cx(pl.bloch_vectors(states)).reshape(len(states), nc * m0)
    assert np.all(np.isnan(U[-2:]))
    U = U[:-2]
    ref = oracle.bloch_vectors(_cx(pl.evecs), pl.L, states[:-2])
    assert np.abs(U - ref).max() <= 1e-14 * np.abs(ref).max()
    H, S, _ = oracle.core_hamiltonian_blocks(s)
    Hf, Sf = oracle.bcirc_full(H), oracle.bcirc_full(S)
    lam = pl.evals.cpu().numpy().ravel()[states[:-2]]
    Ut = U.T
    R = Hf @ Ut - (Sf @ Ut) * lam[None, :]
    scale = np.linalg.norm(Hf, 2) + np.abs(lam) * np.linalg.norm(Sf, 2)
    res = np.linalg.norm(R, axis=0) / (scale * np.linalg.norm(Ut, axis=0))
    print(f"\nc2 lowest band: max residual {res.max():.2e}")
    assert res.max() <= 1e-10
