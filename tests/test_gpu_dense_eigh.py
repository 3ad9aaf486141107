"""Dense lowest-k generalized eigensolver (open-boundary chain) against the
oracle's LAPACK-based eigh, closed forms and invariants."""
import os

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

EPS = 2.0 ** -52
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "box_chain_256_lowest64.txt")


def _run(H, S, k, evecs=True):
    from paper_1408_3839_amd.pipeline import DenseEigh
    N = H.shape[0]
    de = DenseEigh(N, k, with_evecs=evecs)
    Hd = torch.from_numpy(np.ascontiguousarray(H)).cuda()
    Sd = torch.from_numpy(np.ascontiguousarray(S)).cuda()
    de.run(Hd, Sd)
    torch.cuda.synchronize()
    U = de.evecs.cpu().numpy().T if evecs else None
    return de.evals.cpu().numpy(), U, int(de.info.cpu().item())


def _eig_tol(H, S, lam, U, c=256.0):
    """First-order bound per eigenvalue: c eps (|H| + |lambda| |S|) |u|^2,
    u^T S u = 1, plus 1e-12 relative."""
    nh, ns = np.linalg.norm(H, 2), np.linalg.norm(S, 2)
    un = np.sum(U * U, axis=0)
    return 1e-12 * np.maximum(1.0, np.abs(lam)) + c * EPS * (nh + np.abs(lam) * ns) * un


def _check_vectors(H, S, lam, U, res_tol=1e-11, orth_tol=1e-9):
    R = H @ U - (S @ U) * lam[None, :]
    scale = np.linalg.norm(H, 2) + np.abs(lam) * np.linalg.norm(S, 2)
    res = np.linalg.norm(R, axis=0) / (scale * np.linalg.norm(U, axis=0))
    assert res.max() <= res_tol, res.max()
    G = U.T @ S @ U
    assert np.abs(G - np.eye(U.shape[1])).max() <= orth_tol, np.abs(G - np.eye(U.shape[1])).max()


def _random_pencil(rng, n, cond_shift=0.5):
    A = rng.standard_normal((n, n))
    H = A + A.T
    B = rng.standard_normal((n, n))
    S = B @ B.T / n + cond_shift * np.eye(n)
    return H, S


@pytest.mark.parametrize("N,k", [(1, 1), (2, 1), (2, 2), (3, 3), (5, 4), (64, 64), (65, 7),
                                 (150, 12), (300, 64), (257, 33)])
def test_random_pencils(N, k):
    rng = np.random.default_rng(1000 + N + k)
    H, S = _random_pencil(rng, N)
    ev, U, info = _run(H, S, k)
    assert info == 0
    w, v = oracle.lowest_generalized_eigs(H, S, k)
    assert np.all(np.abs(ev - w) <= _eig_tol(H, S, w, v)), np.abs(ev - w).max()
    assert np.all(np.diff(ev) >= 0)
    _check_vectors(H, S, ev, U)


def test_eigenvalues_only():
    rng = np.random.default_rng(5)
    H, S = _random_pencil(rng, 200)
    ev, U, info = _run(H, S, 20, evecs=False)
    assert info == 0 and U is None
    w, v = oracle.lowest_generalized_eigs(H, S, 20)
    assert np.all(np.abs(ev - w) <= _eig_tol(H, S, w, v))


def test_fem_laplacian_closed_form():
    """Linear-FEM Dirichlet Laplacian pencil: lambda_j =
    (6/h^2)(1 - cos t_j)/(2 + cos t_j), t_j = j pi/(n+1)."""
    n, h, k = 700, 0.02, 64
    K = (np.diag(np.full(n, 2.0)) - np.diag(np.ones(n - 1), 1) - np.diag(np.ones(n - 1), -1)) / h
    M = (np.diag(np.full(n, 4.0)) + np.diag(np.ones(n - 1), 1) + np.diag(np.ones(n - 1), -1)) * h / 6
    t = np.arange(1, k + 1) * np.pi / (n + 1)
    lam = 6.0 / h ** 2 * (1 - np.cos(t)) / (2 + np.cos(t))
    ev, U, info = _run(K, M, k)
    assert info == 0
    i = np.arange(1, n + 1)[:, None]
    Uref = np.sin(i * t[None, :])
    Uref /= np.sqrt(np.sum(Uref * (M @ Uref), axis=0))[None, :]
    assert np.all(np.abs(ev - lam) <= _eig_tol(K, M, lam, Uref)), np.abs(ev / lam - 1).max()
    _check_vectors(K, M, ev, U)


def test_diagonal_pencil():
    """Diagonal H and S: the eigenvalues are the sorted ratios h_ii / s_ii."""
    rng = np.random.default_rng(9)
    n = 130
    h = rng.uniform(-5, 5, n)
    s = rng.uniform(0.5, 2.0, n)
    ev, U, info = _run(np.diag(h), np.diag(s), 16)
    assert info == 0
    ref = np.sort(h / s)[:16]
    assert np.allclose(ev, ref, rtol=0, atol=1e-13 * np.abs(h / s).max())


def test_not_positive_definite_reports_pivot():
    """S with a negative eigenvalue in its leading 70 x 70 block: info > 0
    names the first failing pivot, the call completes, outputs stay finite."""
    n = 100
    S = np.eye(n)
    S[69, 69] = -1.0
    H = np.diag(np.arange(n, dtype=np.float64))
    ev, U, info = _run(H, S, 5)
    assert info == 70
    assert np.all(np.isfinite(ev)) and np.all(np.isfinite(U))


def test_repeat_calls_same_result():
    rng = np.random.default_rng(12)
    H, S = _random_pencil(rng, 180)
    a = _run(H, S, 10)
    b = _run(H, S, 10)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_box_chain_256_lowest64():
    """The 256-site chain (N_b = 2048): GPU assembly then the GPU
    eigensolver; eigenvalues against the oracle's (stored by
    tests/golden/make_box_chain_eigs.py) within the first-order bound."""
    from paper_1408_3839_amd import workloads as wl
    from paper_1408_3839_amd.pipeline import BoxPipeline
    rows = [l.split() for l in open(GOLDEN) if not l.startswith("#")]
    meta = {l.split()[1]: float(l.split()[2]) for l in open(GOLDEN) if l.startswith("# norm2")}
    w = np.array([float(r[1]) for r in rows])
    un = np.array([float(r[2]) for r in rows])
    bp = BoxPipeline(wl.config(3), k=64)
    bp.run()
    torch.cuda.synchronize()
    assert int(bp.eig.info.item()) == 0
    ev = bp.eig.evals.cpu().numpy()
    tol = 1e-12 * np.abs(w) + 256 * EPS * (meta["norm2_H"] + np.abs(w) * meta["norm2_S"]) * un
    err = np.abs(ev - w)
    print(f"box chain: max |d lambda| = {err.max():.3e}, max tol = {tol.max():.3e}")
    assert np.all(err <= tol)
    H = bp.H.cpu().numpy()
    S = bp.S.cpu().numpy()
    U = bp.eig.evecs.cpu().numpy().T
    R = H @ U - (S @ U) * ev[None, :]
    scale = meta["norm2_H"] + np.abs(ev) * meta["norm2_S"]
    res = np.linalg.norm(R, axis=0) / (scale * np.linalg.norm(U, axis=0))
    G = U.T @ S @ U
    print(f"box chain: max residual {res.max():.3e}, max |U^T S U - I| "
          f"{np.abs(G - np.eye(64)).max():.3e}")
    assert res.max() <= 1e-10
    assert np.abs(G - np.eye(64)).max() <= 1e-8


def test_box_chain_256_lowest64_split_fp16():
    """The 256-site chain assembled with the split-FP16 x contraction (five
    slices), then the FP64 eigensolver: the lowest 64 eigenvalues against the
    oracle's within 1e-6 Ha, and within the first-order bound of the measured
    matrix perturbation (against the FP64 path) plus the eigensolver's own."""
    from paper_1408_3839_amd import workloads as wl
    from paper_1408_3839_amd.pipeline import BoxPipeline
    rows = [l.split() for l in open(GOLDEN) if not l.startswith("#")]
    meta = {l.split()[1]: float(l.split()[2]) for l in open(GOLDEN) if l.startswith("# norm2")}
    w = np.array([float(r[1]) for r in rows])
    un = np.array([float(r[2]) for r in rows])
    bp = BoxPipeline(wl.config(3), k=64, precision="split_fp16", n_slices=5)
    bp.run()
    b64 = BoxPipeline(wl.config(3))
    b64.assemble()
    torch.cuda.synchronize()
    assert int(bp.eig.info.item()) == 0
    ev = bp.eig.evals.cpu().numpy()
    dH = np.linalg.norm((bp.H - b64.H).cpu().numpy())  # Frobenius >= 2-norm
    dS = np.linalg.norm((bp.S - b64.S).cpu().numpy())
    tol = (1e-12 * np.abs(w) + 256 * EPS * (meta["norm2_H"] + np.abs(w) * meta["norm2_S"]) * un
           + 2 * (dH + np.abs(w) * dS) * un)
    err = np.abs(ev - w)
    print(f"box chain split-fp16 x5: max |d lambda| = {err.max():.3e} Ha, max tol = "
          f"{tol.max():.3e}; |dH|_F = {dH:.3e}, |dS|_F = {dS:.3e}")
    assert np.all(err <= tol)
    assert err.max() <= 1e-6
