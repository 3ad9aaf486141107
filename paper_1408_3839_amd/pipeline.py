"""Device buffers and call sequence for the periodic path (plumbing only).

Allocates the arrays that the C ABI exchanges (torch tensors on the GPU) and
runs the five calls in order on one stream:

    tl_build_basis -> tl_lattice_sum_potential -> tl_assemble_core_hamiltonian_block
    -> tl_block_fft (H and S as a batch of two) -> tl_batched_heigh
"""
from __future__ import annotations

import torch

from . import tl


class PeriodicPipeline:
    def __init__(self, sys, precision: str = "fp64", n_slices: int = 0,
                 device: str = "cuda:0", with_evecs: bool = False, route: str = "block_fft"):
        """route: "block_fft" (block column, then the 3-level block FFT) or
        "kspace" (tl_assemble_kblocks: the DFT taken factor by factor, no
        block column)."""
        if sys.mode != "periodic":
            raise ValueError("PeriodicPipeline needs a periodic-mode system")
        if route not in ("block_fft", "kspace"):
            raise ValueError(f"unknown route {route!r}")
        self.route = route
        tl.load()
        self.sys = sys
        self.handle = tl.SystemHandle(sys)
        self.prec = tl.PRECISIONS[precision]
        self.n_slices = int(n_slices)
        self.device = torch.device(device)
        sz = tl.tl_query_sizes(self.handle)
        self.sizes = sz
        f64 = dict(dtype=torch.float64, device=self.device)
        self.G = torch.empty(sz["basis_elems"], **f64)
        self.AG = torch.empty(sz["basis_elems"], **f64)
        self.SG = torch.empty(sz["basis_elems"], **f64)
        self.P = torch.empty(sz["pot_elems"], **f64)
        self.pot_ws_bytes = tl.tl_potential_workspace_bytes(self.handle)
        self.pot_ws = torch.empty(max(1, self.pot_ws_bytes), dtype=torch.uint8, device=self.device)
        self.asm_ws_bytes = tl.tl_assemble_workspace_bytes(self.handle, self.prec, self.n_slices)
        self.asm_ws = torch.empty(max(1, self.asm_ws_bytes), dtype=torch.uint8, device=self.device)
        L = [int(v) for v in sys.L]
        self.L = L
        self.m0 = sys.m0
        self.nblocks = L[0] * L[1] * L[2]
        self.HS = torch.empty(2, sz["block_elems"], **f64)          # H and S block columns
        self.HSbar = torch.empty(2, sz["block_elems"], 2, **f64)    # their transforms
        self.fft_ws_bytes = tl.tl_block_fft_workspace_bytes(L[0], L[1], L[2], self.m0, 2)
        self.fft_ws = torch.empty(max(1, self.fft_ws_bytes), dtype=torch.uint8, device=self.device)
        if route == "kspace":
            self.kws_bytes = tl.tl_assemble_kblocks_workspace_bytes(self.handle, self.prec,
                                                                    self.n_slices)
            self.kws = torch.empty(max(1, self.kws_bytes), dtype=torch.uint8, device=self.device)
        self.evals = torch.empty(self.nblocks, self.m0, **f64)
        self.evecs = torch.empty(self.nblocks, self.m0, self.m0, 2, **f64) if with_evecs else None
        self.info = torch.empty(self.nblocks, dtype=torch.int32, device=self.device)

    @property
    def H(self):
        return self.HS[0].view(*self.L, self.m0, self.m0)

    @property
    def S(self):
        return self.HS[1].view(*self.L, self.m0, self.m0)

    def build_basis(self, stream=None):
        tl.tl_build_basis(self.handle, self.G, self.AG, self.SG, stream)

    def lattice_sum_potential(self, stream=None):
        tl.tl_lattice_sum_potential(self.handle, self.P, self.pot_ws, self.pot_ws_bytes, stream)

    def assemble(self, stream=None):
        tl.tl_assemble_core_hamiltonian_block(self.handle, self.G, self.AG, self.SG, self.P,
                                              self.prec, self.n_slices, self.HS[0], self.HS[1],
                                              self.asm_ws, self.asm_ws_bytes, stream)

    def assemble_kblocks(self, stream=None):
        tl.tl_assemble_kblocks(self.handle, self.G, self.AG, self.SG, self.P, self.prec,
                               self.n_slices, self.HSbar[0], self.HSbar[1], self.kws,
                               self.kws_bytes, stream)

    def block_fft(self, stream=None):
        L = self.L
        tl.tl_block_fft(self.HS, L[0], L[1], L[2], self.m0, 2, self.HSbar, self.fft_ws,
                        self.fft_ws_bytes, stream)

    def heigh(self, stream=None):
        tl.tl_batched_heigh(self.HSbar[0], self.HSbar[1], self.nblocks, self.m0, self.evals,
                            self.evecs, self.info, stream)

    def bloch_vectors(self, states, stream=None):
        """Full-lattice eigenvectors of the given flat states j*m0 + m (needs
        with_evecs): [len(states)][L1 L2 L3][m0] complex (last axis re, im)."""
        if self.evecs is None:
            raise ValueError("bloch_vectors needs a pipeline built with with_evecs=True")
        st = torch.as_tensor(states, dtype=torch.int32).to(self.device)
        out = torch.empty(st.numel(), self.nblocks, self.m0, 2, dtype=torch.float64,
                          device=self.device)
        L = self.L
        tl.tl_bloch_vectors(self.evecs, L[0], L[1], L[2], self.m0, st, st.numel(), out, stream)
        return out

    def orbital_factors(self, states, stream=None):
        """Rank-m0 canonical form of the orbitals of the given flat states on
        the grid (needs with_evecs and the basis samples):
        (coef [n][m0][2], factors [n][basis_elems][2]), dim d of the factors
        at offset sum_(e<d) m0 n_e."""
        if self.evecs is None:
            raise ValueError("orbital_factors needs a pipeline built with with_evecs=True")
        st = torch.as_tensor(states, dtype=torch.int32).to(self.device)
        coef = torch.empty(st.numel(), self.m0, 2, dtype=torch.float64, device=self.device)
        fac = torch.empty(st.numel(), self.G.numel(), 2, dtype=torch.float64, device=self.device)
        tl.tl_bloch_orbital_factors(self.handle, self.G, self.evecs, st, st.numel(), coef, fac,
                                    stream)
        return coef, fac

    def basis_and_potential(self, stream=None):
        tl.tl_build_basis_and_potential(self.handle, self.G, self.AG, self.SG, self.P,
                                        self.pot_ws, self.pot_ws_bytes, stream)

    def run(self, stream=None):
        self.basis_and_potential(stream)
        if self.route == "kspace":
            self.assemble_kblocks(stream)
        else:
            self.assemble(stream)
            self.block_fft(stream)
        self.heigh(stream)
        return self.evals

    def capture(self):
        """Capture one whole run() into a HIP graph (every launch of the path,
        no allocation, no memset); replay() then re-executes all of it."""
        side = torch.cuda.Stream(device=self.device)
        side.wait_stream(torch.cuda.current_stream(self.device))
        with torch.cuda.stream(side):
            self.run()
        torch.cuda.current_stream(self.device).wait_stream(side)
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self.run()
        return self.graph

    def replay(self):
        self.graph.replay()
        return self.evals


class BatchPipeline:
    """Buffers and descriptor for a ragged batch of periodic (L,1,1) lattices;
    run() enqueues the whole chain with one launch per stage."""

    def __init__(self, systems, precision: str = "fp64", n_slices: int = 0,
                 want_blocks: int = 0, device: str = "cuda:0", tile_edge: int = 64):
        import numpy as np
        tl.load()
        self.systems = list(systems)
        self.sarr = tl.SystemArray(self.systems)
        self.device = torch.device(device)
        self.plan = tl.tl_batch_plan_create(self.sarr, tl.PRECISIONS[precision], n_slices,
                                            want_blocks)
        self.plan.tile_edge = int(tile_edge)
        p = self.plan
        f64 = dict(dtype=torch.float64, device=self.device)
        self.buf = {
            "G": torch.empty(max(1, p.basis_elems), **f64),
            "AG": torch.empty(max(1, p.basis_elems), **f64),
            "SG": torch.empty(max(1, p.basis_elems), **f64),
            "P": torch.empty(max(1, p.pot_elems), **f64),
            "HS": torch.empty(max(1, p.hs_elems), **f64),
            "HSbar": torch.empty(max(1, 2 * p.hs_elems), **f64),
            "evals": torch.empty(max(1, p.eval_elems), **f64),
            "info": torch.empty(max(1, p.kblocks), dtype=torch.int32, device=self.device),
            "ws": torch.empty(max(1, p.ws_bytes), dtype=torch.uint8, device=self.device),
        }
        self.host_desc = np.zeros(p.desc_bytes, dtype=np.uint8)
        tl.tl_batch_write_descriptor(self.sarr, p, self.buf, self.host_desc)
        self.desc = torch.from_numpy(self.host_desc).to(self.device)
        torch.cuda.synchronize(self.device)
        # per-instance views
        self.views = []
        oh = oe = ok = 0
        for s in self.systems:
            L, m0 = int(s.L[0]), s.m0
            be = L * m0 * m0
            self.views.append({
                "H": self.buf["HS"][oh:oh + be].view(L, 1, 1, m0, m0),
                "S": self.buf["HS"][oh + be:oh + 2 * be].view(L, 1, 1, m0, m0),
                "evals": self.buf["evals"][oe:oe + L * m0].view(L, m0),
                "info": self.buf["info"][ok:ok + L],
            })
            oh += 2 * be
            oe += L * m0
            ok += L

    def run(self, stream=None):
        tl.tl_batch_run(self.plan, self.host_desc, self.desc, stream)

    def capture(self):
        side = torch.cuda.Stream(device=self.device)
        side.wait_stream(torch.cuda.current_stream(self.device))
        with torch.cuda.stream(side):
            self.run()
        torch.cuda.current_stream(self.device).wait_stream(side)
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self.run()
        return self.graph

    def replay(self):
        self.graph.replay()


class DenseEigh:
    """Workspace and outputs of the dense lowest-k generalized eigensolver."""

    def __init__(self, N: int, k: int, with_evecs: bool = True, device: str = "cuda:0"):
        tl.load()
        self.N, self.k = int(N), int(k)
        self.device = torch.device(device)
        self.ws_bytes = tl.tl_dense_gen_eigh_workspace_bytes(N, k)
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
        self.evals = torch.empty(k, dtype=torch.float64, device=self.device)
        self.evecs = (torch.empty(k, N, dtype=torch.float64, device=self.device)
                      if with_evecs else None)
        self.info = torch.empty(1, dtype=torch.int32, device=self.device)

    def run(self, H, S, stream=None):
        tl.tl_dense_gen_eigh_lowest(H, S, self.N, self.k, self.evals, self.evecs, self.info,
                                    self.ws, self.ws_bytes, stream)
        return self.evals


class BoxPipeline:
    """Buffers and calls for an open-boundary chain: basis, potential, the
    full N_b x N_b core Hamiltonian and mass matrix, and (k > 0) the lowest k
    generalized eigenpairs."""

    def __init__(self, sys, k: int = 0, with_evecs: bool = True, device: str = "cuda:0",
                 precision: str = "fp64", n_slices: int = 0):
        if sys.mode != "box":
            raise ValueError("BoxPipeline needs a box-mode system")
        tl.load()
        self.sys = sys
        self.prec = tl.PRECISIONS[precision]
        self.n_slices = int(n_slices)
        self.handle = tl.SystemHandle(sys)
        self.device = torch.device(device)
        sz = tl.tl_query_sizes(self.handle)
        self.sizes = sz
        f64 = dict(dtype=torch.float64, device=self.device)
        self.G = torch.empty(sz["basis_elems"], **f64)
        self.AG = torch.empty(sz["basis_elems"], **f64)
        self.SG = torch.empty(sz["basis_elems"], **f64)
        self.P = torch.empty(sz["pot_elems"], **f64)
        self.pot_ws_bytes = tl.tl_potential_workspace_bytes(self.handle)
        self.pot_ws = torch.empty(max(1, self.pot_ws_bytes), dtype=torch.uint8, device=self.device)
        self.asm_ws_bytes = tl.tl_assemble_workspace_bytes(self.handle, self.prec, self.n_slices)
        self.asm_ws = torch.empty(max(1, self.asm_ws_bytes), dtype=torch.uint8, device=self.device)
        self.Nb = int(sz["basis_rows"][0])
        self.H = torch.empty(self.Nb, self.Nb, **f64)
        self.S = torch.empty(self.Nb, self.Nb, **f64)
        self.eig = DenseEigh(self.Nb, k, with_evecs, device) if k > 0 else None

    def assemble(self, stream=None):
        tl.tl_build_basis_and_potential(self.handle, self.G, self.AG, self.SG, self.P,
                                        self.pot_ws, self.pot_ws_bytes, stream)
        tl.tl_assemble_core_hamiltonian_block(self.handle, self.G, self.AG, self.SG, self.P,
                                              self.prec, self.n_slices, self.H, self.S, self.asm_ws,
                                              self.asm_ws_bytes, stream)

    def run(self, stream=None):
        self.assemble(stream)
        if self.eig is not None:
            self.eig.run(self.H, self.S, stream)

    def orbital_factors(self, stream=None):
        """Rank-m0 canonical factors of the k computed orbitals on the grid
        (needs the eigenvectors): [k][m0 (n0 + n1 + n2)], dim d at offset
        m0 sum_(e<d) n_e."""
        if self.eig is None or self.eig.evecs is None:
            raise ValueError("orbital_factors needs the eigenvectors (k > 0, with_evecs)")
        n = [int(v) for v in self.sys.n]
        fac = torch.empty(self.eig.k, self.sys.m0 * sum(n), dtype=torch.float64,
                          device=self.device)
        tl.tl_chain_orbital_factors(self.handle, self.G, self.eig.evecs, self.eig.k, fac, stream)
        return fac

    def capture(self):
        """Capture one whole run() (assembly and eigensolve) into a HIP graph."""
        side = torch.cuda.Stream(device=self.device)
        side.wait_stream(torch.cuda.current_stream(self.device))
        with torch.cuda.stream(side):
            self.run()
        torch.cuda.current_stream(self.device).wait_stream(side)
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self.run()
        return self.graph

    def replay(self):
        self.graph.replay()
