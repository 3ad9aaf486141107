"""Seeded synthetic workloads for the lattice core-Hamiltonian path.

This module only *describes* problems: lattice geometry, grid, nuclei, the
Gaussian basis of one unit cell and the exponential-sum table (t_q, w_q) that
approximates the Newton kernel.  It contains none of the arithmetic of the
method itself (no sampling, no lattice sum, no contraction, no transform, no
eigensolve); the GPU library and the CPU oracle each implement that on their
own and both read the same `System` objects built here.

Conventions (shared input data, both sides read them the same way):

* Dimension l in {0,1,2} is x, y, z.  `periodic[l]` selects a torus of
  `L[l]` cells of length `a[l]` (nodes x_i = i*h, i = 0..n-1, n = L*a/h) or an
  open box with homogeneous Dirichlet conditions (nodes x_i = x0 + i*h).
* Periodic mode: `nuc_pos`/`nuc_Z` are the sites of the unit cell (positions
  relative to the cell origin, cell k has origin k*a); `K[l]` is the image
  range -K..K of the lattice sum restricted to the central cell.
* Box mode: `nuc_pos`/`nuc_Z` list every nucleus of the system and
  `cell_origin` lists the origin of every cell that carries a copy of the
  unit-cell basis.
* Basis function mu of a cell: centre `cell origin + fn_center[mu]`, 1D
  factors coef[mu][l] * (x - A_l)^l_mu,l * exp(-alpha_mu (x - A_l)^2).
  `fn_coef[mu][l]` is the L2(R) normalisation of that 1D factor (basis-set
  data, like the coefficients of a basis-set file).
* Newton kernel: 1/rho ~ sum_q w_q exp(-t_q^2 rho^2) (sinc quadrature of the
  Laplace-Gauss transform, Sec. 3.2, eq. (sinc_general)).  The paper leaves
  the nodes open; the table here is a log-trapezoid rule whose offset and
  step are fitted once per (R, rho range) by a deterministic grid search.
"""
from __future__ import annotations

import dataclasses
import functools
import math
from typing import List, Optional

import numpy as np


@dataclasses.dataclass
class System:
    name: str
    mode: str                      # "periodic" | "box"
    L: np.ndarray                  # int[3] cells per dimension
    periodic: np.ndarray           # int[3] 1 = torus, 0 = Dirichlet box
    n: np.ndarray                  # int[3] grid nodes per dimension
    h: float                       # grid step (bohr), same in every dimension
    x0: np.ndarray                 # float[3] coordinate of node 0
    a: np.ndarray                  # float[3] lattice constant (bohr)
    cell_nodes: np.ndarray         # int[3] a/h in periodic dims, 0 elsewhere
    K: np.ndarray                  # int[3] lattice-sum image range (periodic dims)
    nuc_pos: np.ndarray            # float[M][3]
    nuc_Z: np.ndarray              # float[M]
    cell_origin: Optional[np.ndarray]  # float[ncell][3] (box mode only)
    fn_center: np.ndarray          # float[m0][3] offset of each function in its cell
    fn_l: np.ndarray               # int[m0][3] Cartesian powers (0 or 1)
    fn_alpha: np.ndarray           # float[m0]
    fn_coef: np.ndarray            # float[m0][3]
    R: int                         # sinc-quadrature terms
    t_q: np.ndarray                # float[R]
    w_q: np.ndarray                # float[R]
    quad_max_rel_err: float        # max |rho*sum_q w_q e^{-t_q^2 rho^2} - 1| on the fit range
    quad_rho: tuple                # (rho_min, rho_max) of the fit
    seed: int = 0

    @property
    def m0(self) -> int:
        return int(self.fn_alpha.shape[0])

    @property
    def ncells(self) -> int:
        return int(np.prod(self.L))

    def describe(self) -> dict:
        return {
            "name": self.name, "mode": self.mode, "L": [int(v) for v in self.L],
            "n": [int(v) for v in self.n], "h": self.h, "m0": self.m0, "R": self.R,
            "M": int(self.nuc_Z.shape[0]), "K": [int(v) for v in self.K],
            "seed": self.seed,
        }


# ---------------------------------------------------------------------------
# basis-set data


def gaussian_1d_norm(alpha: float, l: int) -> float:
    """L2(R) normalisation of x^l exp(-alpha x^2), l in {0, 1}."""
    base = (2.0 * alpha / math.pi) ** 0.25
    if l == 0:
        return base
    if l == 1:
        return base * math.sqrt(4.0 * alpha)
    raise ValueError("only l in {0,1} per dimension")


def cartesian_shells(m0: int) -> List[tuple]:
    """Composition of the unit-cell basis: min(4, m0) s-functions, then
    p-functions cycling x, y, z (8 = 4s + px py pz px, 10 = 4s + 2 p-shells,
    13 = 4s + 3 p-shells)."""
    out = []
    for j in range(m0):
        if j < min(4, m0):
            out.append((0, 0, 0))
        else:
            d = (j - 4) % 3
            out.append(tuple(1 if e == d else 0 for e in range(3)))
    return out


def _basis(m0: int, rng: np.random.Generator, alpha_lo: float, alpha_hi: float,
           site_offsets: np.ndarray):
    alphas = np.exp(rng.uniform(math.log(alpha_lo), math.log(alpha_hi), size=m0))
    ls = np.array(cartesian_shells(m0), dtype=np.int64)
    M0 = site_offsets.shape[0]
    centers = np.array([site_offsets[j % M0] for j in range(m0)], dtype=np.float64)
    coef = np.array([[gaussian_1d_norm(float(alphas[j]), int(ls[j][d])) for d in range(3)]
                     for j in range(m0)], dtype=np.float64)
    return centers, ls, alphas.astype(np.float64), coef


# ---------------------------------------------------------------------------
# exponential-sum table for 1/rho


def _quad_table(R: int, u0: float, hq: float):
    u = u0 + hq * np.arange(R, dtype=np.float64)
    t = np.exp(u)
    w = (2.0 / math.sqrt(math.pi)) * hq * t
    return t, w


def _quad_err(R, u0, hq, rho):
    t, w = _quad_table(R, u0, hq)
    f = np.exp(-np.square(np.outer(rho, t))) @ w
    return float(np.max(np.abs(rho * f - 1.0)))


@functools.lru_cache(maxsize=64)
def sinc_quadrature(R: int, rho_min: float, rho_max: float):
    """Log-trapezoid rule t_q = exp(u0 + q*hq), w_q = 2/sqrt(pi) * hq * t_q for
    1/rho = 2/sqrt(pi) int_R exp(-rho^2 e^{2u}) e^u du, with (u0, hq) chosen by
    a coarse-to-fine grid search that minimises the max relative error on
    [rho_min, rho_max].  Returns (t, w, max_rel_err)."""
    rho = np.exp(np.linspace(math.log(rho_min), math.log(rho_max), 600))
    span = math.log(rho_max / rho_min)
    best = (math.inf, 0.0, 0.0)
    hq_lo, hq_hi = 0.15, max(0.3, 3.0 * (span + 8.0) / max(R - 1, 1))
    u_lo, u_hi = -math.log(rho_max) - 8.0, -math.log(rho_max) + 2.0
    for _ in range(4):
        for hq in np.linspace(hq_lo, hq_hi, 33):
            for u0 in np.linspace(u_lo, u_hi, 33):
                e = _quad_err(R, float(u0), float(hq), rho)
                if e < best[0]:
                    best = (e, float(u0), float(hq))
        dh = (hq_hi - hq_lo) / 8.0
        du = (u_hi - u_lo) / 8.0
        hq_lo, hq_hi = max(0.02, best[2] - dh), best[2] + dh
        u_lo, u_hi = best[1] - du, best[1] + du
    t, w = _quad_table(R, best[1], best[2])
    return t, w, best[0]


# ---------------------------------------------------------------------------
# system builders


def _finish(name, mode, L, periodic, n, h, x0, a, K, nuc_pos, nuc_Z, cell_origin,
            centers, ls, alphas, coef, R, rho_min, rho_max, seed) -> System:
    t, w, err = sinc_quadrature(int(R), float(rho_min), float(rho_max))
    cell_nodes = np.array([int(round(a[d] / h)) if periodic[d] else 0 for d in range(3)],
                          dtype=np.int64)
    return System(
        name=name, mode=mode, L=np.asarray(L, dtype=np.int64),
        periodic=np.asarray(periodic, dtype=np.int64), n=np.asarray(n, dtype=np.int64),
        h=float(h), x0=np.asarray(x0, dtype=np.float64), a=np.asarray(a, dtype=np.float64),
        cell_nodes=cell_nodes, K=np.asarray(K, dtype=np.int64),
        nuc_pos=np.asarray(nuc_pos, dtype=np.float64).reshape(-1, 3),
        nuc_Z=np.asarray(nuc_Z, dtype=np.float64).reshape(-1),
        cell_origin=None if cell_origin is None else np.asarray(cell_origin, dtype=np.float64),
        fn_center=centers, fn_l=ls, fn_alpha=alphas, fn_coef=coef,
        R=int(R), t_q=t, w_q=w, quad_max_rel_err=err, quad_rho=(rho_min, rho_max), seed=seed)


def periodic_system(name: str, L, a, h: float, box_len, sites, Z, m0: int,
                    alpha_range, R: int, seed: int, K=None,
                    periodic=None, quad_rho=None) -> System:
    """Periodic (torus) lattice in the dims with L > 1 (or as given by
    `periodic`), open Dirichlet box of length box_len[l] in the others."""
    L = np.asarray(L, dtype=np.int64)
    if periodic is None:
        periodic = (L > 1).astype(np.int64)
    a = np.asarray(a, dtype=np.float64)
    n = np.zeros(3, dtype=np.int64)
    x0 = np.zeros(3)
    for d in range(3):
        if periodic[d]:
            c = a[d] / h
            if abs(c - round(c)) > 1e-9:
                raise ValueError("a/h must be an integer in periodic dims")
            n[d] = int(L[d] * round(c))
        else:
            n[d] = int(round(box_len[d] / h))
            x0[d] = -0.5 * (n[d] - 1) * h
    if K is None:
        K = [int(L[d] // 2) if periodic[d] else 0 for d in range(3)]
    sites = np.asarray(sites, dtype=np.float64).reshape(-1, 3)
    rng = np.random.default_rng(seed)
    centers, ls, alphas, coef = _basis(m0, rng, alpha_range[0], alpha_range[1], sites)
    # fit range of the kernel: half a cell up to the farthest node-image distance
    ext = np.array([(K[d] + 0.5) * a[d] + np.max(np.abs(sites[:, d])) if periodic[d]
                    else 0.5 * n[d] * h + np.max(np.abs(sites[:, d])) for d in range(3)])
    rho_max = float(np.sqrt(np.sum(ext ** 2)))
    rho_min = 0.5 * h
    if quad_rho is not None:      # one table shared by a family of systems
        rho_min, rho_max = quad_rho
    return _finish(name, "periodic", L, periodic, n, h, x0, a, K, sites, Z, None,
                   centers, ls, alphas, coef, R, rho_min, rho_max, seed)


def box_chain_system(name: str, ncell: int, spacing: float, Z_pattern, h: float,
                     n, m0: int, alpha_range, R: int, seed: int) -> System:
    """Open-boundary chain of `ncell` sites along x at (k - (ncell-1)/2)*spacing,
    charges cycling through Z_pattern, one basis copy per site."""
    n = np.asarray(n, dtype=np.int64)
    x0 = -0.5 * (n - 1) * h
    xs = (np.arange(ncell) - 0.5 * (ncell - 1)) * spacing
    nuc = np.stack([xs, np.zeros(ncell), np.zeros(ncell)], axis=1)
    Z = np.array([Z_pattern[k % len(Z_pattern)] for k in range(ncell)], dtype=np.float64)
    rng = np.random.default_rng(seed)
    centers, ls, alphas, coef = _basis(m0, rng, alpha_range[0], alpha_range[1],
                                       np.zeros((1, 3)))
    ext = 0.5 * n * h
    rho_max = float(np.sqrt(np.sum(ext ** 2))) + 0.5 * ncell * spacing
    return _finish(name, "box", [ncell, 1, 1], [0, 0, 0], n, h, x0,
                   [spacing, 0.0, 0.0], [0, 0, 0], nuc, Z, nuc.copy(),
                   centers, ls, alphas, coef, R, 0.5 * h, rho_max, seed)


# ---------------------------------------------------------------------------
# the five workload families


def config(cid: int, instance: int = 0) -> System:
    """Concrete synthetic inputs for the five workloads (c1..c5)."""
    if cid == 1:   # periodic (8,1,1) chain, m0=4 s, R=20, 128^3 grid
        return periodic_system("c1_chain8_m4", [8, 1, 1], [2.0, 0, 0], 0.125,
                               [0, 16.0, 16.0], [[0, 0, 0]], [1.0], 4, (0.1, 20.0),
                               20, seed=1)
    if cid == 2:   # periodic (64,1,1) chain, m0=8 s+p, R=24, 2048x256x256
        return periodic_system("c2_chain64_m8", [64, 1, 1], [2.0, 0, 0], 0.0625,
                               [0, 16.0, 16.0], [[0, 0, 0]], [1.0], 8, (0.1, 30.0),
                               24, seed=2)
    if cid == 3:   # open box (256,1,1), Z in {1,3}, m0=8, R=32, 8500x256x256
        return box_chain_system("c3_box256_m8", 256, 1.8, [1.0, 3.0], 0.0625,
                                [8500, 256, 256], 8, (0.1, 30.0), 32, seed=3)
    if cid == 4:   # one instance of the ragged batch
        return batch_instance(instance)
    if cid == 5:   # periodic (8,8,8), 2-site cell, m0=10, R=32
        return periodic_system("c5_cubic8_m10", [8, 8, 8], [3.0, 3.0, 3.0], 0.1,
                               [0, 0, 0], [[0, 0, 0], [0.7, 0.7, 0.7]], [1.0, 2.0], 10,
                               (0.1, 30.0), 32, seed=5)
    raise ValueError(cid)


def batch_instance(i: int) -> System:
    """Instance i of the ragged periodic batch: L ~ U{16..512}, m0 in {4,8,13},
    spacing ~ U[1.6,2.4] rounded to a multiple of h = 0.0625."""
    rng = np.random.default_rng(4000 + i)
    L = int(rng.integers(16, 513))
    m0 = int(rng.choice([4, 8, 13]))
    h = 0.0625
    a = round(float(rng.uniform(1.6, 2.4)) / h) * h
    # one exponential-sum table for the whole batch: distances up to the
    # largest chain ((256 + 1/2) * 2.4 bohr) plus the transverse box
    return periodic_system(f"c4_inst{i}_L{L}_m{m0}", [L, 1, 1], [a, 0, 0], h,
                           [0, 16.0, 16.0], [[0, 0, 0]], [1.0], m0, (0.1, 30.0), 24,
                           seed=4000 + i, quad_rho=(0.5 * h, 640.0))


def batch(count: int = 64) -> List[System]:
    return [batch_instance(i) for i in range(count)]


def tiny_periodic(L=(4, 1, 1), m0=3, c=8, h=0.25, box=6.0, R=12, seed=11,
                  sites=((0, 0, 0),), Z=(1.0,), alpha_range=(0.3, 3.0), K=None) -> System:
    """Small periodic systems for brute-force and invariant checks."""
    L = np.asarray(L)
    a = [c * h if L[d] > 1 else 0.0 for d in range(3)]
    return periodic_system(f"tiny_L{'x'.join(str(int(v)) for v in L)}_m{m0}", L, a, h,
                           [box, box, box], sites, Z, m0, alpha_range, R, seed=seed, K=K)
