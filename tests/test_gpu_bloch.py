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


def test_kblock_eigenvectors_c2_vs_oracle():
    """The k-block eigenvectors of the (64,1,1) chain (Jacobi route) against
    LAPACK on the oracle's k-blocks: the residual in the oracle's pencil, and
    the S-metric angle to LAPACK's vector for every eigenvalue separated from
    its neighbours (relative gap >= 1e-6) and of first-order condition <= 1e6.
    The angle is held to the Davis-Kahan bound of the two vectors' errors in
    the equivalent standard problem C = S^-1/2 H S^-1/2: the GPU vector's
    residual r in the oracle's pencil, |r| / sqrt(lambda_min(S)), plus LAPACK's
    own backward error, 64 eps (|H| / lambda_min(S) + |lambda|), over the gap."""
    import scipy.linalg as sla
    s = wl.config(2)
    pl = _run(s)
    m0 = s.m0
    H, S, _ = oracle.core_hamiltonian_blocks(s)
    Hb = oracle.block_dft_1level(H).reshape(-1, m0, m0)
    Sb = oracle.block_dft_1level(S).reshape(-1, m0, m0)
    u = _cx(pl.evecs)
    ev = pl.evals.cpu().numpy()
    worst_res = worst_ang = worst_ratio = 0.0
    n_cmp = 0
    for j in range(Hb.shape[0]):
        lam, V = sla.eigh(Hb[j], Sb[j])
        R = Hb[j] @ u[j] - (Sb[j] @ u[j]) * ev[j][None, :]
        scale = np.linalg.norm(Hb[j], 2) + np.abs(ev[j]) * np.linalg.norm(Sb[j], 2)
        res = np.linalg.norm(R, axis=0) / (scale * np.linalg.norm(u[j], axis=0))
        worst_res = max(worst_res, float(res.max()))
        cond = scale * np.sum(np.abs(V) ** 2, axis=0)
        smin = np.linalg.eigvalsh(Sb[j])[0]
        for m in range(m0):
            gap = min([abs(lam[q] - ev[j][m]) for q in range(m0) if q != m] or [np.inf])
            if cond[m] > 1e6 or gap < 1e-6 * max(1.0, abs(lam[m])):
                continue
            # sin of the angle in the S inner product: the S-norm of the part
            # of the (S-normalised) GPU vector orthogonal to LAPACK's
            un = u[j][:, m] / np.sqrt(np.real(np.vdot(u[j][:, m], Sb[j] @ u[j][:, m])))
            w = un - V[:, m] * np.vdot(V[:, m], Sb[j] @ un)
            ang = float(np.sqrt(abs(np.real(np.vdot(w, Sb[j] @ w)))))
            eps = 2.0 ** -52
            bound = (np.linalg.norm(R[:, m]) / np.sqrt(smin)
                     + 64 * eps * (np.linalg.norm(Hb[j], 2) / smin + abs(lam[m]))) / gap
            worst_ang = max(worst_ang, ang)
            if ang / (bound + 1e-15) > worst_ratio:
                info = (j, m, lam[m], gap, cond[m], smin, ang, bound,
                        np.linalg.norm(R[:, m]), np.linalg.norm(Hb[j], 2))
            worst_ratio = max(worst_ratio, ang / (bound + 1e-15))
            n_cmp += 1
    print(f"\nc2 k-block eigenvectors: max residual {worst_res:.2e}, max angle {worst_ang:.2e} "
          f"(at most {worst_ratio:.2f} x its Davis-Kahan bound) over {n_cmp} well-separated, "
          f"well-conditioned eigenvectors")
    print("  worst (j, m, lambda, gap, cond, lambda_min(S), angle, bound, |r|, |H|):", info)
    assert worst_res <= 1e-10
    assert n_cmp >= 400 and worst_ratio <= 2.0


@pytest.mark.parametrize("name", list(CASES))
def test_bloch_orbital_factors(name):
    """The orbital of a Bloch state on the grid as a rank-m0 canonical tensor
    (tl_bloch_orbital_factors): its values at sampled grid nodes against the
    oracle's expansion over all cells of the oracle's Bloch vector of the same
    k-block eigenvector, and its FEM norm psi^H (S_1 x S_2 x S_3) psi = 1;
    out-of-range states give NaN."""
    s = CASES[name]()
    pl = _run(s)
    L = [int(v) for v in s.L]
    m0, nc = s.m0, int(np.prod(L))
    states = [0, m0 + 1, nc * m0 - 1, -1, nc * m0]
    coef, fac = pl.orbital_factors(states)
    torch.cuda.synchronize()
    w, F = _cx(coef), _cx(fac)
    assert np.all(np.isnan(w[3:])) and np.all(np.isnan(F[3:]))
    u = _cx(pl.evecs)
    U = oracle.bloch_vectors(u, L, states[:3])
    n = [int(v) for v in s.n]
    offs = np.cumsum([0] + [m0 * n[d] for d in range(3)])
    rng = np.random.default_rng(5)
    nodes = [tuple(int(rng.integers(0, n[d])) for d in range(3)) for _ in range(150)]
    for r in range(3):
        phi = [F[r, offs[d]:offs[d + 1]].reshape(m0, n[d]) for d in range(3)]
        got = np.array([np.sum(w[r] * phi[0][:, a] * phi[1][:, b] * phi[2][:, c])
                        for a, b, c in nodes])
        ref = oracle.bloch_orbital(s, U[r], nodes)
        err = np.abs(got - ref).max() / np.abs(ref).max()
        # FEM norm from the factors: sum_(mu,nu) conj(w_mu) w_nu prod_d phi_mu^H S_d phi_nu
        gram = np.ones((m0, m0), complex)
        for d in range(3):
            Sphi = oracle.fem_mass(phi[d], bool(s.periodic[d]), s.h)
            gram *= phi[d].conj() @ Sphi.T
        norm = np.vdot(w[r], gram @ w[r])
        print(f"\n{name} state {states[r]}: max |dpsi| / max|psi| = {err:.2e}, "
              f"FEM norm - 1 = {abs(norm - 1):.2e}")
        assert err <= 1e-12
        assert abs(norm - 1.0) <= 1e-9
