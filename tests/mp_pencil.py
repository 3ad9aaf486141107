"""Reference eigenvalues of a small Hermitian-definite pencil in 50-digit
arithmetic (mpmath): the FP64 matrices are taken as exact inputs (their
Hermitian parts, (A + A^H)/2, formed in 50 digits), S = L L^H by Cholesky,
C = L^-1 H L^-H, eigenvalues of C.  Used to decide which FP64
solver is closer on ill-conditioned k-blocks (Sec. 4.2 eq. (HF-FSpace-Block)).
Test infrastructure only."""
from __future__ import annotations

import numpy as np


def mp_generalized_eigvals(H: np.ndarray, S: np.ndarray, dps: int = 50) -> np.ndarray:
    import mpmath
    mp = mpmath.mp
    old = mp.dps
    mp.dps = dps
    try:
        n = H.shape[0]
        cplx = np.iscomplexobj(H) or np.iscomplexobj(S)
        conv = (lambda z: mpmath.mpc(float(z.real), float(z.imag))) if cplx else \
            (lambda z: mpmath.mpf(float(z)))
        Hm = mpmath.matrix(n, n)
        Sm = mpmath.matrix(n, n)
        for i in range(n):
            for j in range(n):
                Hm[i, j] = conv(H[i, j])
                Sm[i, j] = conv(S[i, j])
        Hm = (Hm + (Hm.H if cplx else Hm.T)) / 2
        Sm = (Sm + (Sm.H if cplx else Sm.T)) / 2
        Lc = mpmath.cholesky(Sm)
        Li = mpmath.inverse(Lc)
        LiH = Li.H if cplx else Li.T
        C = Li * Hm * LiH
        C = (C + (C.H if cplx else C.T)) / 2
        ev = mp.eighe(C, eigvals_only=True) if cplx else mp.eigsy(C, eigvals_only=True)
        return np.array(sorted(float(v.real if cplx else v) for v in ev))
    finally:
        mp.dps = old
