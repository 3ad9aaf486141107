"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Every step is run on the GPU from the same seeded inputs as the oracle and
compared element by element:
  basis samples and FEM images      |d| <= 1e-14 * row max
  potential vectors                 |d| <= 1e-13 * row max
  H, S generating blocks            |d| <= 1e-10 * entry scale (no-cancellation magnitude)
  block DFT                         |d| <= 1e-13 * L * max|A|
  k-block eigenvalues               first-order perturbation bound (see _eig_tol)
"""
import math

import numpy as np
import pytest
import scipy.linalg as sla

import oracle
from paper_1408_3839_amd import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.fail("no HIP device visible: the GPU tests need an MI355X")
    from paper_1408_3839_amd import tl
    tl.load()


def _systems():
    return {
        "tiny_L4_m3": lambda: wl.tiny_periodic(L=(4, 1, 1), m0=3, c=8, h=0.25, R=10),
        "tiny_L5_c7_m5": lambda: wl.tiny_periodic(L=(5, 1, 1), m0=5, c=7, h=0.25, R=9,
                                                  alpha_range=(0.3, 4.0)),
        "tiny_3d_2site": lambda: wl.tiny_periodic(L=(3, 2, 2), m0=4, c=4, h=0.5, R=6,
                                                  K=(1, 1, 1), sites=((0, 0, 0), (0.5, 0.5, -0.5)),
                                                  Z=(1.0, 2.0)),
        "m0_1": lambda: wl.tiny_periodic(L=(6, 1, 1), m0=1, c=6, h=0.3, R=8),
        "m0_13": lambda: wl.tiny_periodic(L=(4, 1, 1), m0=13, c=8, h=0.25, R=8,
                                          alpha_range=(0.3, 5.0)),
        "c1": lambda: wl.config(1),
        "c2": lambda: wl.config(2),
        "c5": lambda: wl.config(5),
    }


SYSTEMS = _systems()
NAMES = list(SYSTEMS)


def _pipeline(sys, **kw):
    from paper_1408_3839_amd.pipeline import PeriodicPipeline
    return PeriodicPipeline(sys, **kw)


def _split_dims(flat, sizes_rows, n):
    out, off = [], 0
    for d in range(3):
        k = int(sizes_rows[d]) * int(n[d])
        out.append(flat[off:off + k].reshape(int(sizes_rows[d]), int(n[d])))
        off += k
    return out


@pytest.mark.parametrize("name", NAMES)
def test_basis_parity(name):
    sys = SYSTEMS[name]()
    pl = _pipeline(sys)
    pl.build_basis()
    torch.cuda.synchronize()
    rows = pl.sizes["basis_rows"]
    G = _split_dims(pl.G.cpu().numpy(), rows, sys.n)
    AG = _split_dims(pl.AG.cpu().numpy(), rows, sys.n)
    SG = _split_dims(pl.SG.cpu().numpy(), rows, sys.n)
    for d in range(3):
        g = oracle.cell0_basis(sys, d)
        per = bool(sys.periodic[d])
        gmax = np.abs(g).max(axis=1, keepdims=True)
        # the stencils cancel: their rounding scale is |g|/h and |g| h
        for got, ref, scale in ((G[d], g, gmax),
                                (AG[d], oracle.fem_stiffness(g, per, sys.h), 4 * gmax / sys.h),
                                (SG[d], oracle.fem_mass(g, per, sys.h), gmax * sys.h)):
            assert np.all(np.abs(got - ref) <= 1e-14 * scale), (name, d)


@pytest.mark.parametrize("name", NAMES)
def test_potential_parity(name):
    sys = SYSTEMS[name]()
    pl = _pipeline(sys)
    pl.lattice_sum_potential()
    torch.cuda.synchronize()
    T = pl.sizes["pot_terms"]
    P = _split_dims(pl.P.cpu().numpy(), [T, T, T], sys.n)
    ref = oracle.potential_vectors(sys)
    for d in range(3):
        scale = np.abs(ref[d]).max(axis=1, keepdims=True)
        err = np.abs(P[d] - ref[d])
        assert np.all(err <= 1e-13 * scale), (name, d, float((err / scale).max()))


LONG_WINDOWS = {
    # windows of 201 and 601 images: the wide Gaussians (t (K+1) c h <= sqrt(750))
    # take the lane-run recurrence, the narrower ones the per-image path
    "L200_c4": lambda: wl.tiny_periodic(L=(200, 1, 1), m0=2, c=4, h=0.5, R=12),
    "L600_c3_2site": lambda: wl.tiny_periodic(L=(600, 1, 1), m0=2, c=3, h=0.5, R=12,
                                              sites=((0, 0, 0), (0.5, 0, 0)), Z=(1.0, 2.0)),
}


@pytest.mark.parametrize("name", list(LONG_WINDOWS))
def test_potential_parity_long_window(name):
    """Lattice sums over long image windows (the image-run recurrence for
    Gaussians that reach every image) against the oracle's direct sums."""
    sys = LONG_WINDOWS[name]()
    K, D = int(sys.K[0]), int(sys.cell_nodes[0]) * sys.h
    assert (2 * K + 64) // 64 >= 4
    assert any(t * sys.h < 0.5 and (t * (K + 1) * D) ** 2 <= 750.0 for t in sys.t_q)
    pl = _pipeline(sys)
    pl.lattice_sum_potential()
    torch.cuda.synchronize()
    T = pl.sizes["pot_terms"]
    P = _split_dims(pl.P.cpu().numpy(), [T, T, T], sys.n)
    ref = oracle.potential_vectors(sys)
    for d in range(3):
        scale = np.abs(ref[d]).max(axis=1, keepdims=True)
        err = np.abs(P[d] - ref[d])
        assert np.all(err <= 1e-13 * scale), (name, d, float((err / scale).max()))


@pytest.mark.parametrize("name", NAMES + ["box12"])
def test_basis_and_potential_one_call(name):
    """The combined call (one launch for periodic m0 <= 8, two otherwise)
    writes exactly what the two separate calls write."""
    from paper_1408_3839_amd import tl
    if name == "box12":
        from paper_1408_3839_amd.pipeline import BoxPipeline
        pl = BoxPipeline(wl.box_chain_system("box12", 12, 1.5, [1.0, 2.0], 0.1, [400, 64, 72],
                                             5, (0.3, 4.0), 10, seed=12))
    else:
        pl = _pipeline(SYSTEMS[name]())
    tl.tl_build_basis(pl.handle, pl.G, pl.AG, pl.SG)
    tl.tl_lattice_sum_potential(pl.handle, pl.P, pl.pot_ws, pl.pot_ws_bytes)
    ref = [t.clone() for t in (pl.G, pl.AG, pl.SG, pl.P)]
    for t in (pl.G, pl.AG, pl.SG, pl.P):
        t.fill_(float("nan"))
    tl.tl_build_basis_and_potential(pl.handle, pl.G, pl.AG, pl.SG, pl.P, pl.pot_ws,
                                    pl.pot_ws_bytes)
    torch.cuda.synchronize()
    for got, want in zip((pl.G, pl.AG, pl.SG, pl.P), ref):
        assert torch.equal(got, want), name


@pytest.mark.parametrize("name", NAMES)
def test_assembly_parity(name):
    sys = SYSTEMS[name]()
    pl = _pipeline(sys)
    pl.build_basis()
    pl.lattice_sum_potential()
    pl.assemble()
    torch.cuda.synchronize()
    H = pl.H.cpu().numpy()
    S = pl.S.cpu().numpy()
    Hr, Sr, scale = oracle.core_hamiltonian_blocks(sys)
    # entries whose every product underflows are exactly 0 on both sides
    assert np.all(H[scale == 0] == 0) and np.all(S[scale == 0] == 0)
    # FP64 MFMA flushes denormal products: entries below 1e-290 are compared
    # absolutely, everything else relative to its no-cancellation magnitude
    eh = np.abs(H - Hr) / np.where(scale > 0, scale, 1.0)
    es = np.abs(S - Sr) / np.maximum(np.abs(Sr), 1e-300)
    bad = (np.abs(H - Hr) > 1e-10 * scale + 1e-290)
    w = np.unravel_index(np.argmax(eh), eh.shape)
    assert not bad.any(), (name, float(eh.max()), w, float(Hr[w]), float(H[w]), float(scale[w]))
    assert np.all(np.abs(S - Sr) <= 1e-10 * np.abs(Sr) + 1e-14 * np.abs(Sr).max()), \
        (name, float(es.max()))


def _gpu_dft(A):
    from paper_1408_3839_amd import tl
    L1, L2, L3, m0 = A.shape[1], A.shape[2], A.shape[3], A.shape[4]
    b = A.shape[0]
    inp = torch.from_numpy(np.ascontiguousarray(A)).cuda()
    out = torch.empty(A.shape + (2,), dtype=torch.float64, device="cuda")
    wsb = tl.tl_block_fft_workspace_bytes(L1, L2, L3, m0, b)
    ws = torch.empty(max(1, wsb), dtype=torch.uint8, device="cuda")
    tl.tl_block_fft(inp, L1, L2, L3, m0, b, out, ws, wsb)
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    return o[..., 0] + 1j * o[..., 1]


@pytest.mark.parametrize("shape", [(1, 1, 1, 3), (7, 1, 1, 2), (64, 1, 1, 8), (8, 8, 8, 3),
                                   (3, 4, 5, 2), (1, 6, 1, 4), (2, 1, 9, 1), (37, 1, 1, 13)])
def test_block_fft_parity(shape):
    rng = np.random.default_rng(sum(shape))
    L1, L2, L3, m0 = shape
    A = rng.standard_normal((2, L1, L2, L3, m0, m0))
    got = _gpu_dft(A)
    for b in range(2):
        ref = oracle.block_dft_1level(A[b]) if L2 == L3 == 1 else oracle.block_dft(A[b])
        tol = 1e-13 * L1 * L2 * L3 * np.abs(A[b]).max()
        assert np.abs(got[b] - ref).max() <= tol


def _random_pencils(rng, count, m, cond=1e3):
    H = np.zeros((count, m, m), complex)
    S = np.zeros((count, m, m), complex)
    for j in range(count):
        X = rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m))
        H[j] = (X + X.conj().T) / 2
        Q, _ = np.linalg.qr(rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m)))
        d = np.exp(np.linspace(0, -math.log(cond), m))
        S[j] = (Q * d) @ Q.conj().T
        S[j] = (S[j] + S[j].conj().T) / 2
    return H, S


def _run_heigh(H, S, evecs=True):
    from paper_1408_3839_amd import tl
    count, m = H.shape[0], H.shape[1]
    Ht = torch.from_numpy(np.stack([H.real, H.imag], -1).copy()).cuda()
    St = None if S is None else torch.from_numpy(np.stack([S.real, S.imag], -1).copy()).cuda()
    ev = torch.empty(count, m, dtype=torch.float64, device="cuda")
    vec = torch.empty(count, m, m, 2, dtype=torch.float64, device="cuda") if evecs else None
    info = torch.empty(count, dtype=torch.int32, device="cuda")
    tl.tl_batched_heigh(Ht, St, count, m, ev, vec, info)
    torch.cuda.synchronize()
    V = None
    if evecs:
        v = vec.cpu().numpy()
        V = v[..., 0] + 1j * v[..., 1]
    return ev.cpu().numpy(), V, info.cpu().numpy()


def _eig_tol(Hj, Sj, lam_ref, U_ref, c=256.0):
    """First-order perturbation bound for each eigenvalue of the pencil:
    |d lambda_i| <= c eps (|H| + |lambda_i| |S|) |u_i|^2 with u_i^H S u_i = 1,
    plus 1e-10 relative (the FP64 parity target)."""
    eps = 2.0 ** -52
    nh = np.linalg.norm(Hj, 2)
    ns = np.linalg.norm(Sj, 2)
    un = np.sum(np.abs(U_ref) ** 2, axis=0)
    return 1e-10 * np.maximum(1.0, np.abs(lam_ref)) + c * eps * (nh + np.abs(lam_ref) * ns) * un


@pytest.mark.parametrize("evecs", [False, True], ids=["evals-only", "with-evecs"])
def test_heigh_ill_conditioned_block_vs_50_digits(evecs):
    """The k = 0 block of the (64,1,1) chain (kappa(Sbar) ~ 7e13), as the
    FP64 oracle forms it, through both eigensolver routes (Householder +
    Sturm without eigenvectors, Jacobi with them): errors against the
    eigenvalues of the same pencil in 50-digit arithmetic, next to LAPACK's
    (Sec. 4.2 eq. (HF-FSpace-Block))."""
    from mp_pencil import mp_generalized_eigvals
    from test_conditioning_cpu import c2_kblocks
    Hb, Sb = c2_kblocks()
    H0, S0 = Hb[:1], Sb[:1]
    ref = mp_generalized_eigvals(H0[0], S0[0])
    lam, U = sla.eigh(H0[0], S0[0])
    ev, _, info = _run_heigh(H0, S0, evecs=evecs)
    assert info[0] == 0
    err_gpu = np.abs(ev[0] - ref)
    err_lap = np.abs(lam - ref)
    eps = 2.0 ** -52
    cond = (np.linalg.norm(H0[0], 2) + np.abs(ref) * np.linalg.norm(S0[0], 2)) * \
        np.sum(np.abs(U) ** 2, axis=0)
    print(f"\nk = 0 block ({'eigenvalues only' if not evecs else 'with eigenvectors'}):")
    for i in range(len(ref)):
        print(f"  lambda {ref[i]: .12f}  GPU error {err_gpu[i]:.2e}  LAPACK error "
              f"{err_lap[i]:.2e}  condition {cond[i]:.2e}")
    print(f"  max error: GPU {err_gpu.max():.2e}, LAPACK {err_lap.max():.2e}")
    # both within the first-order bound of their rounding; the well
    # conditioned eigenvalues to 1e-10
    assert np.all(err_gpu <= 256 * eps * cond + 1e-10)
    ok = cond <= 1e6
    assert np.all(err_gpu[ok] <= 1e-10)


@pytest.mark.parametrize("m", [1, 2, 3, 7, 8, 9, 13, 16, 17, 31, 32])
def test_heigh_random_pencils(m):
    rng = np.random.default_rng(100 + m)
    H, S = _random_pencils(rng, 37, m)
    ev, V, info = _run_heigh(H, S)
    assert np.all(info == 0)
    for j in range(H.shape[0]):
        lam, U = sla.eigh(H[j], S[j])
        assert np.all(np.abs(ev[j] - lam) <= _eig_tol(H[j], S[j], lam, U)), (m, j)
        # residual and S-normalisation of the returned vectors
        R = H[j] @ V[j] - (S[j] @ V[j]) * ev[j][None, :]
        scale = np.linalg.norm(H[j], 2) + np.abs(ev[j]) * np.linalg.norm(S[j], 2)
        assert np.all(np.linalg.norm(R, axis=0) <= 1e-11 * scale * np.linalg.norm(V[j], axis=0))
        G = V[j].conj().T @ S[j] @ V[j]
        assert np.abs(G - np.eye(m)).max() < 1e-9


def test_heigh_standard_problem_and_not_definite():
    rng = np.random.default_rng(7)
    H, S = _random_pencils(rng, 6, 5)
    ev, _, info = _run_heigh(H, None, evecs=False)
    assert np.all(info == 0)
    for j in range(6):
        assert np.abs(ev[j] - np.linalg.eigvalsh(H[j])).max() < 1e-12 * np.abs(H[j]).max() * 5
    S[2] = -np.eye(5)               # not positive definite at the first pivot
    S[4][3, 3] = -1.0 - np.abs(S[4]).sum()
    ev, _, info = _run_heigh(H, S, evecs=True)
    assert info[2] == 1 and np.all(np.isnan(ev[2]))
    assert info[4] > 0 and np.all(np.isnan(ev[4]))
    for j in (0, 1, 3, 5):
        assert info[j] == 0
        lam, U = sla.eigh(H[j], S[j])
        assert np.all(np.abs(ev[j] - lam) <= _eig_tol(H[j], S[j], lam, U))


@pytest.mark.parametrize("name", NAMES)
def test_end_to_end_eigenvalues(name):
    """Whole path on the GPU (basis, potential, assembly, block FFT, k-block
    eigensolves) against the oracle's LAPACK eigenvalues of its own blocks."""
    sys = SYSTEMS[name]()
    pl = _pipeline(sys)
    pl.run()
    torch.cuda.synchronize()
    ev = pl.evals.cpu().numpy()
    info = pl.info.cpu().numpy()
    assert np.all(info == 0)
    Hr, Sr, _ = oracle.core_hamiltonian_blocks(sys)
    Hb = oracle.block_dft(Hr)
    Sb = oracle.block_dft(Sr)
    m0 = sys.m0
    Hf = Hb.reshape(-1, m0, m0)
    Sf = Sb.reshape(-1, m0, m0)
    for j in range(Hf.shape[0]):
        lam, U = sla.eigh(Hf[j], Sf[j])
        tol = _eig_tol(Hf[j], Sf[j], lam, U)
        assert np.all(np.abs(ev[j] - lam) <= tol), (name, j, ev[j] - lam, tol)


def test_graph_replay_matches_eager():
    """The whole path captured in a HIP graph: every replay, with eager work
    and synchronisations in between, reproduces the eager result bit for bit."""
    sys = wl.config(2)
    pl = _pipeline(sys)
    pl.run()
    torch.cuda.synchronize()
    H0 = pl.H.clone()
    ev0 = pl.evals.clone()
    pl.capture()
    for rep in range(3):
        pl.HS.fill_(0.0)
        pl.evals.fill_(0.0)
        torch.cuda.synchronize()
        pl.replay()
        torch.cuda.synchronize()
        assert torch.equal(pl.H, H0), rep
        assert torch.equal(pl.evals, ev0), rep
        pl.run()            # eager work between replays
        torch.cuda.synchronize()
        assert torch.equal(pl.evals, ev0), rep


@pytest.mark.parametrize("m", [1, 2, 3, 4, 5, 7, 8, 9, 10, 12, 13, 15, 16])
@pytest.mark.parametrize("standard", [False, True])
def test_heigh_eigenvalues_only(m, standard):
    """Without eigenvectors, m0 <= 16 blocks take the Householder-tridiagonal +
    Sturm-bisection route (one wave for m0 <= 8, 256 threads above);
    eigenvalues against LAPACK within the first-order bound, ascending,
    info = 0."""
    rng = np.random.default_rng(300 + m + 50 * standard)
    H, S = _random_pencils(rng, 41, m)
    if standard:
        S = None
    ev, _, info = _run_heigh(H, S, evecs=False)
    assert np.all(info == 0)
    for j in range(H.shape[0]):
        Sj = np.eye(m) if standard else S[j]
        lam, U = sla.eigh(H[j], Sj)
        assert np.all(np.abs(ev[j] - lam) <= _eig_tol(H[j], Sj, lam, U)), (m, j, ev[j] - lam)
        assert np.all(np.diff(ev[j]) >= 0)


@pytest.mark.parametrize("m", [8, 16])
def test_heigh_eigenvalues_only_degenerate_and_reduced(m):
    """Exactly repeated eigenvalues and an already diagonal block (every
    reflector is the identity) on the eigenvalue-only route."""
    H = np.zeros((3, m, m), complex)
    H[0] = np.diag(np.resize([1.0, 1.0, 1.0, 2.0, 2.0, -3.0, 0.5, 0.5], m))
    Q, _ = np.linalg.qr(np.random.default_rng(4).standard_normal((m, m))
                        + 1j * np.random.default_rng(5).standard_normal((m, m)))
    H[1] = Q @ H[0] @ Q.conj().T
    H[1] = (H[1] + H[1].conj().T) / 2
    H[2] = np.diag(np.arange(m, dtype=float)) + np.diag(np.full(m - 1, 0.25), 1) + np.diag(np.full(m - 1, 0.25), -1)
    ev, _, info = _run_heigh(H, None, evecs=False)
    assert np.all(info == 0)
    S = np.broadcast_to(np.eye(m), H.shape).astype(complex)
    S[1][0, 0] = 0.0  # not definite at the first pivot: reported, the others unaffected
    ev2, _, info2 = _run_heigh(H, S, evecs=False)
    assert info2[1] == 1 and np.all(np.isnan(ev2[1])) and info2[0] == 0 and info2[2] == 0
    for j in range(3):
        lam = np.linalg.eigvalsh(H[j])
        assert np.abs(ev[j] - lam).max() <= 64 * 2.0 ** -52 * np.abs(lam).max(), (j, ev[j] - lam)
