"""Closed-form one-electron integrals over Cartesian Gaussians (l <= 1 per
dimension), written from the Obara-Saika recurrences (Obara & Saika, J. Chem.
Phys. 84, 3963 (1986); Helgaker, Jorgensen & Olsen, Molecular
Electronic-Structure Theory, ch. 9).  They pin the grid-based oracle: its FEM
overlap / kinetic entries and its sinc-tensor nuclear attraction must converge
to these values as h -> 0.  Independent of the oracle and of the GPU library.
"""
from __future__ import annotations

import functools
import math

import numpy as np
from scipy import special


def overlap_1d(i: int, j: int, a: float, A: float, b: float, B: float) -> float:
    """int (x-A)^i (x-B)^j exp(-a(x-A)^2 - b(x-B)^2) dx (unnormalised)."""
    p = a + b
    P = (a * A + b * B) / p
    XPA, XPB = P - A, P - B
    S00 = math.sqrt(math.pi / p) * math.exp(-a * b / p * (A - B) ** 2)

    @functools.lru_cache(maxsize=None)
    def S(ii, jj):
        if ii < 0 or jj < 0:
            return 0.0
        if ii == 0 and jj == 0:
            return S00
        if ii > 0:
            return XPA * S(ii - 1, jj) + ((ii - 1) * S(ii - 2, jj) + jj * S(ii - 1, jj - 1)) / (2 * p)
        return XPB * S(ii, jj - 1) + (ii * S(ii - 1, jj - 1) + (jj - 1) * S(ii, jj - 2)) / (2 * p)

    return S(i, j)


def dd_1d(i: int, j: int, a: float, A: float, b: float, B: float) -> float:
    """int d/dx[(x-A)^i e^{-a(x-A)^2}] d/dx[(x-B)^j e^{-b(x-B)^2}] dx."""
    def S(ii, jj):
        if ii < 0 or jj < 0:
            return 0.0
        return overlap_1d(ii, jj, a, A, b, B)
    return (i * j * S(i - 1, j - 1) - 2 * b * i * S(i - 1, j + 1)
            - 2 * a * j * S(i + 1, j - 1) + 4 * a * b * S(i + 1, j + 1))


def boys(m: int, T: float) -> float:
    """F_m(T) = int_0^1 t^{2m} exp(-T t^2) dt = Gamma(m+1/2) P(m+1/2, T) / (2 T^{m+1/2})
    (P the regularised lower incomplete gamma); Taylor series for tiny T."""
    if T < 1e-10:
        return 1.0 / (2 * m + 1) - T / (2 * m + 3)
    return special.gamma(m + 0.5) * special.gammainc(m + 0.5, T) / (2.0 * T ** (m + 0.5))


def nuclear_attraction(la, a, A, lb, b, B, C) -> float:
    """int g_a(r) g_b(r) / |r - C| d^3r for unnormalised Cartesian Gaussians
    (x-A)^la exp(-a|r-A|^2), by the Obara-Saika vertical recurrence."""
    A = np.asarray(A, float)
    B = np.asarray(B, float)
    C = np.asarray(C, float)
    p = a + b
    P = (a * A + b * B) / p
    KAB = math.exp(-a * b / p * float(np.sum((A - B) ** 2)))
    T = p * float(np.sum((P - C) ** 2))
    pref = 2 * math.pi / p * KAB

    @functools.lru_cache(maxsize=None)
    def theta(ta, tb, m):
        if min(ta) < 0 or min(tb) < 0:
            return 0.0
        if sum(ta) == 0 and sum(tb) == 0:
            return pref * boys(m, T)
        if sum(ta) > 0:
            i = next(k for k in range(3) if ta[k] > 0)
            am = tuple(v - (k == i) for k, v in enumerate(ta))
            amm = tuple(v - 2 * (k == i) for k, v in enumerate(ta))
            bm = tuple(v - (k == i) for k, v in enumerate(tb))
            out = (P[i] - A[i]) * theta(am, tb, m) - (P[i] - C[i]) * theta(am, tb, m + 1)
            out += am[i] / (2 * p) * (theta(amm, tb, m) - theta(amm, tb, m + 1))
            out += tb[i] / (2 * p) * (theta(am, bm, m) - theta(am, bm, m + 1))
            return out
        i = next(k for k in range(3) if tb[k] > 0)
        bm = tuple(v - (k == i) for k, v in enumerate(tb))
        bmm = tuple(v - 2 * (k == i) for k, v in enumerate(tb))
        am = tuple(v - (k == i) for k, v in enumerate(ta))
        out = (P[i] - B[i]) * theta(ta, bm, m) - (P[i] - C[i]) * theta(ta, bm, m + 1)
        out += bm[i] / (2 * p) * (theta(ta, bmm, m) - theta(ta, bmm, m + 1))
        out += ta[i] / (2 * p) * (theta(am, bm, m) - theta(am, bm, m + 1))
        return out

    return theta(tuple(int(v) for v in la), tuple(int(v) for v in lb), 0)


def molecule_integrals(sys):
    """Closed-form S, T, V (no periodic images) for the unit-cell basis of a
    single-cell system with every dimension open: returns (S, T, V) where
    H = T - V and V = sum_nu Z_nu int g g / |r - a_nu|."""
    m0 = sys.m0
    S = np.zeros((m0, m0))
    T = np.zeros((m0, m0))
    V = np.zeros((m0, m0))
    for mu in range(m0):
        for nu in range(m0):
            a, b = float(sys.fn_alpha[mu]), float(sys.fn_alpha[nu])
            A, B = sys.fn_center[mu], sys.fn_center[nu]
            la, lb = sys.fn_l[mu], sys.fn_l[nu]
            norm = float(np.prod(sys.fn_coef[mu]) * np.prod(sys.fn_coef[nu]))
            s1 = [overlap_1d(int(la[d]), int(lb[d]), a, A[d], b, B[d]) for d in range(3)]
            t1 = [dd_1d(int(la[d]), int(lb[d]), a, A[d], b, B[d]) for d in range(3)]
            S[mu, nu] = norm * s1[0] * s1[1] * s1[2]
            T[mu, nu] = 0.5 * norm * (t1[0] * s1[1] * s1[2] + s1[0] * t1[1] * s1[2]
                                      + s1[0] * s1[1] * t1[2])
            v = 0.0
            for k in range(sys.nuc_Z.shape[0]):
                v += sys.nuc_Z[k] * nuclear_attraction(la, a, A, lb, b, B, sys.nuc_pos[k])
            V[mu, nu] = norm * v
    return S, T, V
