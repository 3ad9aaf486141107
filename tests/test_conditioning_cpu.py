"""The ill-conditioned k-block of the periodic (64,1,1) chain.

The random exponents make some mass-matrix blocks Sbar_j nearly singular:
at k = 0 the chain's diffuse functions have almost no Bloch norm and
kappa(Sbar_0) ~ 7e13.  Which FP64 solver is closer to the exact eigenvalues of
the FP64 pencil (taken as exact input) is decided against 50-digit arithmetic
(Sec. 4.2 eq. (HF-FSpace-Block)); the GPU route is compared in
test_gpu_parity.py::test_heigh_ill_conditioned_block_vs_50_digits.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import oracle
from mp_pencil import mp_generalized_eigvals
from paper_1408_3839_amd import workloads as wl


def c2_kblocks():
    s = wl.config(2)
    H, S, _ = oracle.core_hamiltonian_blocks(s)
    m0 = s.m0
    return (oracle.block_dft_1level(H).reshape(-1, m0, m0),
            oracle.block_dft_1level(S).reshape(-1, m0, m0))


def test_mp_pencil_solver_pins():
    """The 50-digit solver itself: a 2 x 2 pencil with closed-form
    eigenvalues, and agreement with LAPACK on a well-conditioned pencil."""
    # H = [[a, b], [b, c]], S = diag(s1, s2): det(H - l S) = 0
    a, b, c, s1, s2 = 2.0, 0.5, -1.0, 1.0, 4.0
    A = s1 * s2
    B = -(a * s2 + c * s1)
    C = a * c - b * b
    disc = np.sqrt(B * B - 4 * A * C)
    exact = np.sort([(-B - disc) / (2 * A), (-B + disc) / (2 * A)])
    got = mp_generalized_eigvals(np.array([[a, b], [b, c]]), np.diag([s1, s2]))
    assert np.abs(got - exact).max() <= 1e-15
    rng = np.random.default_rng(3)
    X = rng.standard_normal((6, 6)) + 1j * rng.standard_normal((6, 6))
    Hm = X + X.conj().T
    Y = rng.standard_normal((6, 6)) + 1j * rng.standard_normal((6, 6))
    Sm = Y @ Y.conj().T + 6 * np.eye(6)
    ref = mp_generalized_eigvals(Hm, Sm)
    assert np.abs(ref - sla.eigh(Hm, Sm, eigvals_only=True)).max() <= 1e-13


def test_c2_ill_conditioned_block_lapack_vs_50_digits():
    Hb, Sb = c2_kblocks()
    kappa = np.array([np.linalg.cond(Sb[j]) for j in range(Sb.shape[0])])
    j = int(np.argmax(kappa))
    assert j == 0 and kappa[j] > 1e13
    ref = mp_generalized_eigvals(Hb[j], Sb[j])
    lam, U = sla.eigh(Hb[j], Sb[j])
    err = np.abs(lam - ref)
    eps = 2.0 ** -52
    cond = (np.linalg.norm(Hb[j], 2) + np.abs(ref) * np.linalg.norm(Sb[j], 2)) * \
        np.sum(np.abs(U) ** 2, axis=0)
    print(f"\nk = 0 block, kappa(Sbar) = {kappa[j]:.2e}")
    for i in range(len(ref)):
        print(f"  lambda {ref[i]: .15f}  LAPACK error {err[i]:.2e}  condition {cond[i]:.2e}")
    # LAPACK stays within its first-order bound, far below the 1e-6 Ha target
    assert np.all(err <= 64 * eps * cond + 1e-12)
    assert err.max() <= 1e-8
