"""Plain FP64 CPU oracle for the lattice core-Hamiltonian path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, links or runs
this package: only the tests, the smoke check of the entry module and the
CPU-baseline leg of the benchmark do.  It shares no code with the HIP library.

Every function writes out what the paper defines, in the paper's order, with
numpy/scipy primitives (a dot product, a matmul, erf/erfc, a LAPACK eigensolver)
as the only library steps.  Notation follows the paper: a lattice L=(L1,L2,L3)
of unit cells, m0 Gaussian basis functions per cell, canonical rank-R Newton
kernel, generating blocks A_k of a symmetric 3-level block-circulant matrix.

Readings where the paper is silent (each also listed in the design notes):
* one node set per dimension serves the potential cells (piecewise constant,
  Sec. 3.2) and the hat-function FEM (Sec. 3.4);
* cell-average projection of each Gaussian factor of the kernel;
* lattice sum over images -K..K restricted to the central cell and replicated
  with the lattice period (Sec. 4.1, eq. (EwaldSumP) with a symmetric range);
* FEM mass matrix <S g, g> in the mass matrix (Sec. 4.1, eq. (BC-mass));
* generating blocks are the first block column, A_k = <g_(.,k) | op | g_(.,0)>,
  and the transform is Abar_j = sum_k omega^(jk) A_k, omega = exp(-2 pi i/L)
  (Appendix, Proposition on block-circulant diagonalisation).
"""
from __future__ import annotations

import math
from typing import Dict, List, Sequence, Tuple

import numpy as np
from scipy import linalg as sla
from scipy import special

# Gaussian factors are summed over every periodic image within this exponent
# (exp(-46) ~ 1e-20 relative to the peak, below FP64 resolution).
GAUSS_TAIL_EXPONENT = 46.0


# ---------------------------------------------------------------------------
# grids and basis sampling (Sec. 3.4, eq. (Gaus pwl): nodal values g(x_i))


def node_coords(sys, d: int) -> np.ndarray:
    """Nodes x_i = x0 + i*h of dimension d (torus dims start at 0)."""
    return sys.x0[d] + sys.h * np.arange(int(sys.n[d]), dtype=np.float64)


def gaussian_factor(x: np.ndarray, A: float, l: int, alpha: float, coef: float) -> np.ndarray:
    """coef * (x-A)^l * exp(-alpha (x-A)^2), the 1D factor of a Cartesian GTO."""
    r = x - A
    return coef * (r ** l) * np.exp(-alpha * r * r)


def sample_factor(sys, d: int, A: float, l: int, alpha: float, coef: float) -> np.ndarray:
    """Nodal samples of one 1D factor; on a torus the factor is periodised by
    summing its images A + j*P, P = L*a, over every image that can reach the
    interval within the Gaussian tail cutoff."""
    x = node_coords(sys, d)
    if not sys.periodic[d]:
        return gaussian_factor(x, A, l, alpha, coef)
    P = sys.L[d] * sys.a[d]
    rcut = math.sqrt(GAUSS_TAIL_EXPONENT / alpha)
    J = int(math.ceil(rcut / P)) + 1
    g = np.zeros_like(x)
    for j in range(-J, J + 1):
        g += gaussian_factor(x, A + j * P, l, alpha, coef)
    return g


def cell0_basis(sys, d: int) -> np.ndarray:
    """G[mu][i]: samples of the m0 unit-cell functions (cell 0 / origin 0)."""
    return np.stack([sample_factor(sys, d, float(sys.fn_center[mu][d]), int(sys.fn_l[mu][d]),
                                   float(sys.fn_alpha[mu]), float(sys.fn_coef[mu][d]))
                     for mu in range(sys.m0)])


def fem_stiffness(g: np.ndarray, periodic: bool, h: float) -> np.ndarray:
    """A g with A = (1/h) tridiag(-1, 2, -1) (Sec. 3.4); circulant on a torus,
    homogeneous Dirichlet (zero outside the nodes) in a box."""
    left = np.roll(g, 1, axis=-1)
    right = np.roll(g, -1, axis=-1)
    if not periodic:
        left[..., 0] = 0.0
        right[..., -1] = 0.0
    return (2.0 * g - left - right) / h


def fem_mass(g: np.ndarray, periodic: bool, h: float) -> np.ndarray:
    """S g with S = (h/6) tridiag(1, 4, 1) (Sec. 3.4)."""
    left = np.roll(g, 1, axis=-1)
    right = np.roll(g, -1, axis=-1)
    if not periodic:
        left[..., 0] = 0.0
        right[..., -1] = 0.0
    return (4.0 * g + left + right) * (h / 6.0)


# ---------------------------------------------------------------------------
# canonical Newton kernel and the lattice sum (Sec. 3.2, Sec. 4.1)


def cell_gaussian_integral(t: float, x: np.ndarray, h: float, A: float) -> np.ndarray:
    """b(x_i) = int_{x_i-h/2}^{x_i+h/2} exp(-t^2 (y-A)^2) dy: projection of one
    Gaussian factor of the exponential sum onto the piecewise-constant cell of
    node x_i (eq. (galten) with 1/|x| replaced by its sinc expansion).
    For t*h >= 1/2 the closed form (sqrt(pi)/2t)(erf(v) - erf(u)) is taken on
    the side where the difference does not cancel (erfc for both arguments
    positive or both negative); for t*h < 1/2, where any erf difference
    cancels, the integrand is smooth on the cell and an 8-point
    Gauss-Legendre rule integrates it to full precision."""
    x = np.asarray(x, dtype=np.float64)
    if t * h < 0.5:
        gx, gw = special.roots_legendre(8)
        y = x[:, None] + 0.5 * h * gx[None, :] - A
        return 0.5 * h * (np.exp(-(t * t) * y * y) @ gw)
    u = t * (x - 0.5 * h - A)
    v = t * (x + 0.5 * h - A)
    out = np.empty_like(u)
    pos = u >= 0.0
    neg = v <= 0.0
    mid = ~(pos | neg)
    out[pos] = special.erfc(u[pos]) - special.erfc(v[pos])
    out[neg] = special.erfc(-v[neg]) - special.erfc(-u[neg])
    out[mid] = special.erf(v[mid]) + special.erf(-u[mid])
    return out * (math.sqrt(math.pi) / (2.0 * t))


def potential_groups(sys) -> List[List[int]]:
    """Nuclei that share their (y, z) position share the y and z factors of the
    kernel, so their x factors add up (rank stays R per group)."""
    groups: Dict[Tuple[float, float], List[int]] = {}
    for nu in range(sys.nuc_Z.shape[0]):
        key = (float(sys.nuc_pos[nu][1]), float(sys.nuc_pos[nu][2]))
        groups.setdefault(key, []).append(nu)
    return list(groups.values())


def central_cell_nodes(sys, d: int) -> np.ndarray:
    """Representative of every torus node in the central cell window
    [-floor(c/2), c - floor(c/2)) around the origin, in node units."""
    c = int(sys.cell_nodes[d])
    i = np.arange(int(sys.n[d]))
    return ((i + c // 2) % c) - c // 2


def lattice_summed_factor(sys, d: int, t: float, A: float) -> np.ndarray:
    """One canonical factor of the lattice-summed kernel on dimension d.
    Torus: sum over images A + k*a, k = -K..K, evaluated on the central cell and
    replicated with period a (eq. (EwaldSumP), restricted then replicated).
    Box: the single factor centred at A."""
    if not sys.periodic[d]:
        return cell_gaussian_integral(t, node_coords(sys, d), sys.h, A)
    r = central_cell_nodes(sys, d).astype(np.float64) * sys.h
    K = int(sys.K[d])
    acc = np.zeros_like(r)
    for k in range(-K, K + 1):
        acc += cell_gaussian_integral(t, r, sys.h, A + k * sys.a[d])
    return acc


def potential_vectors(sys) -> List[np.ndarray]:
    """P^(d)[term][i] for d = 0,1,2 with term = group*R + q.  The weight w_q and
    the charges Z_nu sit in the x factor, so that
    v(x) ~ sum_term prod_d P^(d)[term](x_d)  (eq. (EwaldTensorGl))."""
    groups = potential_groups(sys)
    out = [[], [], []]
    for grp in groups:
        y0 = float(sys.nuc_pos[grp[0]][1])
        z0 = float(sys.nuc_pos[grp[0]][2])
        for q in range(sys.R):
            t = float(sys.t_q[q])
            vx = np.zeros(int(sys.n[0]))
            for nu in grp:
                vx += sys.nuc_Z[nu] * lattice_summed_factor(sys, 0, t, float(sys.nuc_pos[nu][0]))
            out[0].append(sys.w_q[q] * vx)
            out[1].append(lattice_summed_factor(sys, 1, t, y0))
            out[2].append(lattice_summed_factor(sys, 2, t, z0))
    return [np.stack(v) for v in out]


# ---------------------------------------------------------------------------
# Galerkin entries: products of 1D inner products (Lemma 3.1 proof, Sec. 3.4)


def shift_contractions(sys, d: int, G: np.ndarray, P: np.ndarray, absolute: bool = False):
    """1D inner products on dimension d for every shift s of the left function
    by s cells (s = 0..L_d-1 on a torus, s = 0 in a box):
      C[t][mu][nu][s] = sum_i g_mu(x_i - s a) p_t(x_i) g_nu(x_i)
      D[mu][nu][s]    = <A (shifted g_mu), g_nu>,  M[mu][nu][s] = <S (shifted g_mu), g_nu>.
    absolute=True returns the same sums over absolute values of every product
    (|A| and |S| stencils), the magnitude the sums have without cancellation."""
    per = bool(sys.periodic[d])
    nshift = int(sys.L[d]) if per else 1
    c = int(sys.cell_nodes[d])
    T = P.shape[0]
    m0 = G.shape[0]
    C = np.zeros((T, m0, m0, nshift))
    D = np.zeros((m0, m0, nshift))
    M = np.zeros((m0, m0, nshift))
    if absolute:
        G, P = np.abs(G), np.abs(P)
    for s in range(nshift):
        Gs = np.roll(G, s * c, axis=1)          # Gs[mu][i] = g_mu(x_{i - s c})
        for t in range(T):
            C[t, :, :, s] = (Gs * P[t]) @ G.T
        if absolute:
            # (1/h)(2|g_i| + |g_i-1| + |g_i+1|) = 4|g|/h - A|g|
            D[:, :, s] = (4.0 * Gs / sys.h - fem_stiffness(Gs, per, sys.h)) @ G.T
            M[:, :, s] = fem_mass(Gs, per, sys.h) @ G.T
        else:
            D[:, :, s] = fem_stiffness(Gs, per, sys.h) @ G.T
            M[:, :, s] = fem_mass(Gs, per, sys.h) @ G.T
    return C, D, M


def core_hamiltonian_blocks(sys, return_parts: bool = False):
    """Generating blocks of the periodic core Hamiltonian and mass matrix:
    H[k1][k2][k3][mu][nu] = <g_(mu,k) | -1/2 Lap - v_c | g_(nu,0)>,
    S[k1][k2][k3][mu][nu] = <g_(mu,k) | g_(nu,0)> (FEM mass), with
      V_k = sum_t prod_d C^(d)[t][:,:,k_d]
      T_k = 1/2 (D1 M2 M3 + M1 D2 M3 + M1 M2 D3),  S_k = M1 M2 M3,  H_k = T_k - V_k.
    Also returns `scale`, the entry magnitude without any cancellation: the
    same formula with every 1D sum taken over absolute values of its products
    (|A| = (1/h) tridiag(1,2,1)), used by the parity norm."""
    assert sys.mode == "periodic"
    P = potential_vectors(sys)
    parts, absparts = [], []
    for d in range(3):
        G = cell0_basis(sys, d)
        parts.append(shift_contractions(sys, d, G, P[d]))
        absparts.append(shift_contractions(sys, d, G, P[d], absolute=True))
    L = [int(v) for v in sys.L]
    m0 = sys.m0
    H = np.zeros((L[0], L[1], L[2], m0, m0))
    S = np.zeros_like(H)
    scale = np.zeros_like(H)
    (C1, D1, M1), (C2, D2, M2), (C3, D3, M3) = parts
    (A1, E1, N1), (A2, E2, N2), (A3, E3, N3) = absparts
    for k1 in range(L[0]):
        for k2 in range(L[1]):
            for k3 in range(L[2]):
                V = np.sum(C1[:, :, :, k1] * C2[:, :, :, k2] * C3[:, :, :, k3], axis=0)
                t1 = D1[:, :, k1] * M2[:, :, k2] * M3[:, :, k3]
                t2 = M1[:, :, k1] * D2[:, :, k2] * M3[:, :, k3]
                t3 = M1[:, :, k1] * M2[:, :, k2] * D3[:, :, k3]
                T = 0.5 * (t1 + t2 + t3)
                H[k1, k2, k3] = T - V
                S[k1, k2, k3] = M1[:, :, k1] * M2[:, :, k2] * M3[:, :, k3]
                Va = np.sum(A1[:, :, :, k1] * A2[:, :, :, k2] * A3[:, :, :, k3], axis=0)
                Ta = 0.5 * (E1[:, :, k1] * N2[:, :, k2] * N3[:, :, k3]
                            + N1[:, :, k1] * E2[:, :, k2] * N3[:, :, k3]
                            + N1[:, :, k1] * N2[:, :, k2] * E3[:, :, k3])
                scale[k1, k2, k3] = Ta + Va
    if return_parts:
        return H, S, scale, {"P": P, "parts": parts}
    return H, S, scale


# ---------------------------------------------------------------------------
# explicit supercell / box matrices (no shift structure used)


def _all_function_samples(sys, d: int, origins: np.ndarray) -> np.ndarray:
    """Samples of every basis function of every cell on dimension d, each one
    evaluated at its own centre (cell origin + offset)."""
    rows = []
    for o in origins:
        for mu in range(sys.m0):
            rows.append(sample_factor(sys, d, float(o[d] + sys.fn_center[mu][d]),
                                      int(sys.fn_l[mu][d]), float(sys.fn_alpha[mu]),
                                      float(sys.fn_coef[mu][d])))
    return np.stack(rows)


def cell_origins(sys) -> np.ndarray:
    if sys.mode == "box":
        return np.asarray(sys.cell_origin)
    L = [int(v) for v in sys.L]
    out = []
    for k1 in range(L[0]):
        for k2 in range(L[1]):
            for k3 in range(L[2]):
                out.append([k1 * sys.a[0], k2 * sys.a[1], k3 * sys.a[2]])
    return np.array(out, dtype=np.float64)


def full_matrices(sys, rows: Sequence[int] = None, cols: Sequence[int] = None,
                  absolute: bool = False):
    """H and S over all N_b = ncells*m0 functions (cell-major, function-minor),
    every entry from the 1D inner products of explicitly sampled functions:
    H_fg = 1/2 sum_d <A_d g_f, g_g> prod_{e!=d} <S_e g_f, g_g> - sum_t prod_d <g_f p_t g_g>.
    Optional `rows`/`cols` restrict the computation to a sub-block.
    absolute=True returns the entry scales instead (the same formula, every 1D
    sum over absolute values of its products, |A| = (1/h) tridiag(1,2,1), the
    terms of H added in magnitude), as core_hamiltonian_blocks' `scale`."""
    origins = cell_origins(sys)
    P = potential_vectors(sys)
    Nb = origins.shape[0] * sys.m0
    rows = np.arange(Nb) if rows is None else np.asarray(rows)
    cols = np.arange(Nb) if cols is None else np.asarray(cols)
    Cs, Ds, Ms = [], [], []
    for d in range(3):
        Gall = _all_function_samples(sys, d, origins)
        per = bool(sys.periodic[d])
        Gr, Gc = Gall[rows], Gall[cols]
        Pd = P[d]
        if absolute:
            Gr, Gc, Pd = np.abs(Gr), np.abs(Gc), np.abs(Pd)
        Cs.append(np.stack([(Gr * Pd[t]) @ Gc.T for t in range(Pd.shape[0])]))
        if absolute:
            Ds.append((4.0 * Gr / sys.h - fem_stiffness(Gr, per, sys.h)) @ Gc.T)
        else:
            Ds.append(fem_stiffness(Gr, per, sys.h) @ Gc.T)
        Ms.append(fem_mass(Gr, per, sys.h) @ Gc.T)
    V = np.sum(Cs[0] * Cs[1] * Cs[2], axis=0)
    T = 0.5 * (Ds[0] * Ms[1] * Ms[2] + Ms[0] * Ds[1] * Ms[2] + Ms[0] * Ms[1] * Ds[2])
    if absolute:
        return T + V, Ms[0] * Ms[1] * Ms[2]
    return T - V, Ms[0] * Ms[1] * Ms[2]


# ---------------------------------------------------------------------------
# block-circulant structure and its Fourier block-diagonalisation (Sec. 2, App.)


def bcirc_full(blocks: np.ndarray) -> np.ndarray:
    """Assemble the 3-level block-circulant matrix whose first block column is
    blocks[k1][k2][k3]: block (k, m) = A_{(k - m) mod L} (Definition 2.1)."""
    L1, L2, L3, m0, _ = blocks.shape
    idx = [(k1, k2, k3) for k1 in range(L1) for k2 in range(L2) for k3 in range(L3)]
    N = len(idx) * m0
    A = np.zeros((N, N), dtype=blocks.dtype)
    for bi, k in enumerate(idx):
        for bj, m in enumerate(idx):
            d = ((k[0] - m[0]) % L1, (k[1] - m[1]) % L2, (k[2] - m[2]) % L3)
            A[bi * m0:(bi + 1) * m0, bj * m0:(bj + 1) * m0] = blocks[d]
    return A


def btoepl_full(blocks: np.ndarray) -> np.ndarray:
    """The symmetric one-level block Toeplitz matrix of the Appendix, eq.
    (block_SToepl): block (r, c) = A_(r-c) for r >= c and A_(c-r)^T for
    r < c.  blocks: [L][m0][m0]."""
    L, m0, _ = blocks.shape
    A = np.zeros((L * m0, L * m0), dtype=blocks.dtype)
    for r in range(L):
        for c in range(L):
            B = blocks[r - c] if r >= c else blocks[c - r].T
            A[r * m0:(r + 1) * m0, c * m0:(c + 1) * m0] = B
    return A


def btoepl_multilevel_full(B: np.ndarray, L: Sequence[int]) -> np.ndarray:
    """The multilevel block Toeplitz matrix over L1 x L2 x L3 cells (the
    recursive Definition of the d-level class, without its symmetry
    constraint): block (r, c) = B[r - c + L - 1] for cells r, c flattened as
    [r1][r2][r3].  B: [2L1-1][2L2-1][2L3-1][m0][m0]."""
    L1, L2, L3 = (int(v) for v in L)
    m0 = B.shape[-1]
    cells = [(a, b, c) for a in range(L1) for b in range(L2) for c in range(L3)]
    A = np.zeros((len(cells) * m0, len(cells) * m0), dtype=B.dtype)
    for i, r in enumerate(cells):
        for j, c in enumerate(cells):
            A[i * m0:(i + 1) * m0, j * m0:(j + 1) * m0] = \
                B[r[0] - c[0] + L1 - 1, r[1] - c[1] + L2 - 1, r[2] - c[2] + L3 - 1]
    return A


def block_dft(blocks: np.ndarray) -> np.ndarray:
    """Abar_j = sum_k omega_1^(j1 k1) omega_2^(j2 k2) omega_3^(j3 k3) A_k with
    omega_l = exp(-2 pi i / L_l), by explicit O(|L|^2) sums (Proposition on
    block-circulant diagonalisation; three levels via F_L1 x F_L2 x F_L3).
    Exponents are reduced modulo L before the complex exponential."""
    L1, L2, L3, m0, _ = blocks.shape
    out = np.zeros(blocks.shape, dtype=np.complex128)
    for j1 in range(L1):
        for j2 in range(L2):
            for j3 in range(L3):
                acc = np.zeros((m0, m0), dtype=np.complex128)
                for k1 in range(L1):
                    for k2 in range(L2):
                        for k3 in range(L3):
                            ph = ((j1 * k1) % L1) / L1 + ((j2 * k2) % L2) / L2 \
                                + ((j3 * k3) % L3) / L3
                            acc += np.exp(-2j * math.pi * ph) * blocks[k1, k2, k3]
                out[j1, j2, j3] = acc
    return out


def block_dft_1level(blocks: np.ndarray) -> np.ndarray:
    """Same transform for (L,1,1) lattices, one level, as a plain double loop
    written with a phase matrix (used for long chains)."""
    L = blocks.shape[0]
    j = np.arange(L)
    ph = np.outer(j, j) % L
    W = np.exp(-2j * math.pi * ph / L)
    flat = blocks.reshape(L, -1)
    return (W @ flat).reshape(blocks.shape).astype(np.complex128)


def kblock_eigvals(Hbar: np.ndarray, Sbar: np.ndarray = None) -> np.ndarray:
    """Ascending eigenvalues of every k-block pencil (Hbar_j - lambda Sbar_j),
    eq. (HF-FSpace-Block), by LAPACK's generalized Hermitian solver."""
    shp = Hbar.shape[:-2]
    m0 = Hbar.shape[-1]
    Hf = Hbar.reshape(-1, m0, m0)
    Sf = None if Sbar is None else Sbar.reshape(-1, m0, m0)
    ev = np.zeros((Hf.shape[0], m0))
    for j in range(Hf.shape[0]):
        if Sf is None:
            ev[j] = sla.eigh(Hf[j], eigvals_only=True)
        else:
            ev[j] = sla.eigh(Hf[j], Sf[j], eigvals_only=True)
    return ev.reshape(shp + (m0,))


def unitary_dft(L: int) -> np.ndarray:
    """F_L = L^(-1/2) [omega^(jk)], omega = exp(-2 pi i / L) (Sec. 2, the
    Fourier matrix that diagonalises the cyclic shift)."""
    j = np.arange(L)
    return np.exp(-2j * math.pi * (np.outer(j, j) % L) / L) / math.sqrt(L)


def bloch_vectors(u: np.ndarray, L: Sequence[int], states: Sequence[int]) -> np.ndarray:
    """Eigenvectors of the block-circulant pencil from those of its k-blocks,
    eq. (eigvecA): U_(j,m) = (F^* x I_m0) Ubar_(j,m), Ubar_(j,m) =
    E_[j] vec[u_(0,m), ..., u_(L-1,m)], i.e. u_(j,m) in block j and zeros
    elsewhere; three levels with F = F_L1 x F_L2 x F_L3 (Kronecker products,
    written out as dense matrices).
    u: [L1 L2 L3][m0][m0] complex, column m = eigenvector m of block j;
    states: flat indices j m0 + m.  Returns [len(states)][L1 L2 L3 m0]."""
    L1, L2, L3 = (int(v) for v in L)
    m0 = u.shape[-1]
    nc = L1 * L2 * L3
    F = np.kron(np.kron(unitary_dft(L1), unitary_dft(L2)), unitary_dft(L3))
    W = np.kron(F.conj().T, np.eye(m0))
    out = np.zeros((len(states), nc * m0), dtype=np.complex128)
    for r, st in enumerate(states):
        j, m = divmod(int(st), m0)
        Ubar = np.zeros(nc * m0, dtype=np.complex128)
        Ubar[j * m0:(j + 1) * m0] = u.reshape(nc, m0, m0)[j][:, m]
        out[r] = W @ Ubar
    return out


def bloch_orbital(sys, U: np.ndarray, nodes: Sequence[Sequence[int]]) -> np.ndarray:
    """Values of the orbital with full-lattice coefficients U ([L1 L2 L3 m0],
    e.g. a row of bloch_vectors) at grid nodes (i0, i1, i2):
      psi(x_i) = sum_c sum_mu U[c][mu] prod_d g_mu^d(x_(i_d) - c_d a_d),
    the Galerkin expansion over the replicated basis (eq. (eigvecA) for the
    coefficients, Sec. 3.4 for the nodal samples); on a torus the shifted
    periodised sample of cell 0 is read c_d * cell_nodes_d nodes back."""
    L = [int(v) for v in sys.L]
    m0 = sys.m0
    G = [cell0_basis(sys, d) for d in range(3)]
    cn = [int(sys.n[d]) // L[d] for d in range(3)]
    out = np.zeros(len(nodes), dtype=np.complex128)
    for r, node in enumerate(nodes):
        v = 0.0 + 0.0j
        for c1 in range(L[0]):
            for c2 in range(L[1]):
                for c3 in range(L[2]):
                    c = (c1 * L[1] + c2) * L[2] + c3
                    for mu in range(m0):
                        g = 1.0
                        for d, cd in enumerate((c1, c2, c3)):
                            g *= G[d][mu][(int(node[d]) - cd * cn[d]) % int(sys.n[d])]
                        v += U[c * m0 + mu] * g
        out[r] = v
    return out


def chain_orbital(sys, U: np.ndarray, nodes: Sequence[Sequence[int]]) -> np.ndarray:
    """Values of the orbital with coefficients U over all N_b functions of an
    open chain (cell-major, function-minor) at grid nodes (i0, i1, i2):
    psi(x_i) = sum_f U[f] prod_d g_f^d(x_(i_d)), every function sampled at its
    own centre (Sec. 3.4; the coefficients of the full eigensolver)."""
    X = [_all_function_samples(sys, d, cell_origins(sys)) for d in range(3)]
    return np.array([np.sum(U * X[0][:, a] * X[1][:, b] * X[2][:, c]) for a, b, c in nodes])


def lowest_generalized_eigs(H: np.ndarray, S: np.ndarray, k: int):
    """Lowest k eigenpairs of the symmetric-definite pencil (H, S)."""
    w, v = sla.eigh(H, S, subset_by_index=[0, k - 1])
    return w, v
