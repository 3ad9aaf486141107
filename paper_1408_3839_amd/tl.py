"""ctypes binding of libtl.so: the C ABI declared in include/tl.h, one Python
function per entry point with the same name.  Argument marshalling only:
torch tensors provide device memory (data_ptr) and streams; every step of the
computation runs in the library's HIP kernels.  There is no fallback: if the
library or a GPU is missing, the calls raise.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtl.so")

TL_OK, TL_EINVAL, TL_EUNSUPPORTED, TL_EHIP, TL_EWORKSPACE = 0, -1, -2, -3, -4
TL_FP64, TL_FP32, TL_SPLIT_BF16, TL_SPLIT_FP16 = 0, 1, 2, 3
TL_MODE_PERIODIC, TL_MODE_BOX = 0, 1
TL_STAGE_CONTRACTION, TL_STAGE_LATTICE_SUM, TL_STAGE_FFT = 0, 1, 2
PRECISIONS = {"fp64": TL_FP64, "fp32": TL_FP32, "split_bf16": TL_SPLIT_BF16,
              "split_fp16": TL_SPLIT_FP16}

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)


class TlSystem(ctypes.Structure):
    _fields_ = [
        ("mode", ctypes.c_int),
        ("L", ctypes.c_int * 3),
        ("periodic", ctypes.c_int * 3),
        ("n", ctypes.c_int * 3),
        ("cell_nodes", ctypes.c_int * 3),
        ("K", ctypes.c_int * 3),
        ("h", ctypes.c_double),
        ("x0", ctypes.c_double * 3),
        ("a", ctypes.c_double * 3),
        ("box_origin0", ctypes.c_double),
        ("n_nuc", ctypes.c_int),
        ("nuc_pos", _dp),
        ("nuc_Z", _dp),
        ("m0", ctypes.c_int),
        ("fn_center", _dp),
        ("fn_l", _ip),
        ("fn_alpha", _dp),
        ("fn_coef", _dp),
        ("R", ctypes.c_int),
        ("t_q", _dp),
        ("w_q", _dp),
    ]


class TlSizes(ctypes.Structure):
    _fields_ = [
        ("basis_rows", ctypes.c_int64 * 3),
        ("basis_elems", ctypes.c_int64),
        ("pot_terms", ctypes.c_int64),
        ("pot_elems", ctypes.c_int64),
        ("block_elems", ctypes.c_int64),
    ]


TL_MAX_BATCH = 512


class TlBatchPlan(ctypes.Structure):
    _fields_ = [
        ("count", ctypes.c_int), ("precision", ctypes.c_int), ("n_slices", ctypes.c_int),
        ("want_blocks", ctypes.c_int), ("max_m0", ctypes.c_int), ("max_len", ctypes.c_int),
        ("basis_elems", ctypes.c_int64), ("pot_elems", ctypes.c_int64),
        ("hs_elems", ctypes.c_int64), ("eval_elems", ctypes.c_int64), ("kblocks", ctypes.c_int64),
        ("ws_bytes", ctypes.c_size_t), ("desc_bytes", ctypes.c_size_t),
        ("tile_edge", ctypes.c_int),
    ]


class TlBatchBuffers(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in
                ("G", "AG", "SG", "P", "HS", "HSbar", "evals", "info", "ws")]


# name -> (restype, argtypes) of every exported symbol of include/tl.h
SIGNATURES = {
    "tl_version": (ctypes.c_char_p, []),
    "tl_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "tl_last_error": (ctypes.c_char_p, []),
    "tl_query_sizes": (ctypes.c_int, [ctypes.POINTER(TlSystem), ctypes.POINTER(TlSizes)]),
    "tl_potential_workspace_bytes": (ctypes.c_int, [ctypes.POINTER(TlSystem),
                                                    ctypes.POINTER(ctypes.c_size_t)]),
    "tl_assemble_workspace_bytes": (ctypes.c_int, [ctypes.POINTER(TlSystem), ctypes.c_int,
                                                   ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)]),
    "tl_block_fft_workspace_bytes": (ctypes.c_int, [ctypes.c_int] * 5
                                     + [ctypes.POINTER(ctypes.c_size_t)]),
    "tl_build_basis": (ctypes.c_int, [ctypes.POINTER(TlSystem), ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "tl_lattice_sum_potential": (ctypes.c_int, [ctypes.POINTER(TlSystem), ctypes.c_void_p,
                                                ctypes.c_void_p, ctypes.c_size_t,
                                                ctypes.c_void_p]),
    "tl_build_basis_and_potential": (ctypes.c_int, [ctypes.POINTER(TlSystem)]
                                     + [ctypes.c_void_p] * 5
                                     + [ctypes.c_size_t, ctypes.c_void_p]),
    "tl_assemble_core_hamiltonian_block": (
        ctypes.c_int, [ctypes.POINTER(TlSystem), ctypes.c_void_p, ctypes.c_void_p,
                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                       ctypes.c_void_p]),
    "tl_assemble_core_hamiltonian_block_noalloc": (
        ctypes.c_int, [ctypes.POINTER(TlSystem), ctypes.c_void_p, ctypes.c_void_p,
                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "tl_assemble_kblocks_workspace_bytes": (
        ctypes.c_int, [ctypes.POINTER(TlSystem), ctypes.c_int, ctypes.c_int,
                       ctypes.POINTER(ctypes.c_size_t)]),
    "tl_assemble_kblocks": (
        ctypes.c_int, [ctypes.POINTER(TlSystem), ctypes.c_void_p, ctypes.c_void_p,
                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                       ctypes.c_void_p]),
    "tl_set_contraction_events": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "tl_set_stage_events": (ctypes.c_int, [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]),
    "tl_block_fft": (ctypes.c_int, [ctypes.c_void_p] + [ctypes.c_int] * 5
                     + [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "tl_batched_heigh": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                        ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_void_p]),
    "tl_bloch_vectors": (ctypes.c_int, [ctypes.c_void_p] + [ctypes.c_int] * 4
                         + [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]),
    "tl_bloch_orbital_factors": (ctypes.c_int, [ctypes.POINTER(TlSystem)] + [ctypes.c_void_p] * 3
                                 + [ctypes.c_int] + [ctypes.c_void_p] * 3),
    "tl_chain_orbital_factors": (ctypes.c_int, [ctypes.POINTER(TlSystem)] + [ctypes.c_void_p] * 2
                                 + [ctypes.c_int] + [ctypes.c_void_p] * 2),
    "tl_btoepl_workspace_bytes": (ctypes.c_int, [ctypes.c_int] * 3
                                  + [ctypes.POINTER(ctypes.c_size_t)]),
    "tl_btoepl_setup": (ctypes.c_int, [ctypes.c_void_p] + [ctypes.c_int] * 3
                        + [ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "tl_btoepl_matvec": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p] + [ctypes.c_int] * 3
                         + [ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "tl_btoepl_power": (ctypes.c_int, [ctypes.c_int] * 3 + [ctypes.c_void_p] * 4
                        + [ctypes.c_size_t, ctypes.c_void_p]),
    "tl_btoepl3_workspace_bytes": (ctypes.c_int, [ctypes.c_int] * 5
                                   + [ctypes.POINTER(ctypes.c_size_t)]),
    "tl_btoepl3_setup": (ctypes.c_int, [ctypes.c_void_p] + [ctypes.c_int] * 5
                         + [ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "tl_btoepl3_matvec": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p] + [ctypes.c_int] * 5
                          + [ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "tl_btoepl3_power": (ctypes.c_int, [ctypes.c_int] * 5 + [ctypes.c_void_p] * 4
                         + [ctypes.c_size_t, ctypes.c_void_p]),
    "tl_btoepl_lowest_workspace_bytes": (ctypes.c_int, [ctypes.c_int] * 3
                                         + [ctypes.POINTER(ctypes.c_size_t)]),
    "tl_btoepl_lowest": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p] + [ctypes.c_int] * 5
                         + [ctypes.c_double, ctypes.c_double] + [ctypes.c_void_p] * 4
                         + [ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                            ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "tl_btoepl3_lowest_workspace_bytes": (ctypes.c_int, [ctypes.c_int] * 5
                                          + [ctypes.POINTER(ctypes.c_size_t)]),
    "tl_btoepl3_lowest": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p] + [ctypes.c_int] * 7
                          + [ctypes.c_double, ctypes.c_double] + [ctypes.c_void_p] * 4
                          + [ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                             ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "tl_dense_gen_eigh_workspace_bytes": (ctypes.c_int, [ctypes.c_int, ctypes.c_int,
                                                         ctypes.POINTER(ctypes.c_size_t)]),
    "tl_set_dense_eigh_events": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "tl_dense_gen_eigh_lowest": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                                ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                                ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                                ctypes.c_void_p]),
    "tl_batch_plan_create": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                            ctypes.c_int, ctypes.c_int,
                                            ctypes.POINTER(TlBatchPlan)]),
    "tl_batch_write_descriptor": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int,
                                                 ctypes.POINTER(TlBatchPlan),
                                                 ctypes.POINTER(TlBatchBuffers), ctypes.c_void_p,
                                                 ctypes.c_size_t]),
    "tl_batch_run": (ctypes.c_int, [ctypes.POINTER(TlBatchPlan), ctypes.c_void_p,
                                    ctypes.c_void_p, ctypes.c_void_p]),
}

_lib = None


class TlError(RuntimeError):
    pass


def load(path: str = LIB_PATH):
    """Load libtl.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise TlError(f"{path} not found: build it with `python -m paper_1408_3839_amd.build`")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(status: int, what: str):
    if status != TL_OK:
        lib = load()
        raise TlError(f"{what}: {lib.tl_status_string(status).decode()} "
                      f"({lib.tl_last_error().decode()})")


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def _stream(stream) -> Optional[int]:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


class SystemHandle:
    """A TlSystem plus the host arrays it points into (kept alive together)."""

    def __init__(self, sys):
        self.sys = sys
        self.arrays = []
        s = TlSystem()
        s.mode = TL_MODE_BOX if sys.mode == "box" else TL_MODE_PERIODIC
        for d in range(3):
            s.L[d] = int(sys.L[d])
            s.periodic[d] = int(sys.periodic[d])
            s.n[d] = int(sys.n[d])
            s.cell_nodes[d] = int(sys.cell_nodes[d])
            s.K[d] = int(sys.K[d])
            s.x0[d] = float(sys.x0[d])
            s.a[d] = float(sys.a[d])
        s.h = float(sys.h)
        s.box_origin0 = float(sys.cell_origin[0][0]) if sys.mode == "box" else 0.0
        s.n_nuc = int(sys.nuc_Z.shape[0])
        s.nuc_pos = self._d(sys.nuc_pos)
        s.nuc_Z = self._d(sys.nuc_Z)
        s.m0 = int(sys.m0)
        s.fn_center = self._d(sys.fn_center)
        s.fn_l = self._i(sys.fn_l)
        s.fn_alpha = self._d(sys.fn_alpha)
        s.fn_coef = self._d(sys.fn_coef)
        s.R = int(sys.R)
        s.t_q = self._d(sys.t_q)
        s.w_q = self._d(sys.w_q)
        self.struct = s

    def _d(self, a):
        a = np.ascontiguousarray(a, dtype=np.float64)
        self.arrays.append(a)
        return a.ctypes.data_as(_dp)

    def _i(self, a):
        a = np.ascontiguousarray(a, dtype=np.int32)
        self.arrays.append(a)
        return a.ctypes.data_as(_ip)

    @property
    def ref(self):
        return ctypes.byref(self.struct)


def _handle(sys) -> SystemHandle:
    return sys if isinstance(sys, SystemHandle) else SystemHandle(sys)


# ---------------------------------------------------------------- entry points


def tl_version() -> str:
    return load().tl_version().decode()


def tl_query_sizes(sys) -> dict:
    h = _handle(sys)
    out = TlSizes()
    _check(load().tl_query_sizes(h.ref, ctypes.byref(out)), "tl_query_sizes")
    return {"basis_rows": list(out.basis_rows), "basis_elems": out.basis_elems,
            "pot_terms": out.pot_terms, "pot_elems": out.pot_elems,
            "block_elems": out.block_elems}


def tl_potential_workspace_bytes(sys) -> int:
    h = _handle(sys)
    v = ctypes.c_size_t()
    _check(load().tl_potential_workspace_bytes(h.ref, ctypes.byref(v)),
           "tl_potential_workspace_bytes")
    return v.value


def tl_assemble_workspace_bytes(sys, precision=TL_FP64, n_slices=0) -> int:
    h = _handle(sys)
    v = ctypes.c_size_t()
    _check(load().tl_assemble_workspace_bytes(h.ref, int(precision), int(n_slices),
                                              ctypes.byref(v)), "tl_assemble_workspace_bytes")
    return v.value


def tl_assemble_kblocks_workspace_bytes(sys, precision=TL_FP64, n_slices=0) -> int:
    h = _handle(sys)
    v = ctypes.c_size_t()
    _check(load().tl_assemble_kblocks_workspace_bytes(h.ref, int(precision), int(n_slices),
                                                      ctypes.byref(v)),
           "tl_assemble_kblocks_workspace_bytes")
    return v.value


def tl_block_fft_workspace_bytes(L1, L2, L3, m0, batch) -> int:
    v = ctypes.c_size_t()
    _check(load().tl_block_fft_workspace_bytes(int(L1), int(L2), int(L3), int(m0), int(batch),
                                               ctypes.byref(v)), "tl_block_fft_workspace_bytes")
    return v.value


def tl_build_basis(sys, G, AG, SG, stream=None):
    h = _handle(sys)
    _check(load().tl_build_basis(h.ref, _ptr(G), _ptr(AG), _ptr(SG), _stream(stream)),
           "tl_build_basis")


def tl_lattice_sum_potential(sys, P, ws, ws_bytes, stream=None):
    h = _handle(sys)
    _check(load().tl_lattice_sum_potential(h.ref, _ptr(P), _ptr(ws), int(ws_bytes),
                                           _stream(stream)), "tl_lattice_sum_potential")


def tl_build_basis_and_potential(sys, G, AG, SG, P, ws, ws_bytes, stream=None):
    h = _handle(sys)
    _check(load().tl_build_basis_and_potential(h.ref, _ptr(G), _ptr(AG), _ptr(SG), _ptr(P),
                                               _ptr(ws), int(ws_bytes), _stream(stream)),
           "tl_build_basis_and_potential")


def tl_assemble_core_hamiltonian_block(sys, G, AG, SG, P, precision, n_slices, H, S, ws,
                                       ws_bytes, stream=None):
    h = _handle(sys)
    _check(load().tl_assemble_core_hamiltonian_block(
        h.ref, _ptr(G), _ptr(AG), _ptr(SG), _ptr(P), int(precision), int(n_slices), _ptr(H),
        _ptr(S), _ptr(ws), int(ws_bytes), _stream(stream)), "tl_assemble_core_hamiltonian_block")


def tl_assemble_kblocks(sys, G, AG, SG, P, precision, n_slices, Hk, Sk, ws, ws_bytes,
                        stream=None):
    h = _handle(sys)
    _check(load().tl_assemble_kblocks(
        h.ref, _ptr(G), _ptr(AG), _ptr(SG), _ptr(P), int(precision), int(n_slices), _ptr(Hk),
        _ptr(Sk), _ptr(ws), int(ws_bytes), _stream(stream)), "tl_assemble_kblocks")


def tl_assemble_core_hamiltonian_block_noalloc(sys, G, AG, SG, P, precision, n_slices, H, S,
                                               stream=None):
    h = _handle(sys)
    _check(load().tl_assemble_core_hamiltonian_block_noalloc(
        h.ref, _ptr(G), _ptr(AG), _ptr(SG), _ptr(P), int(precision), int(n_slices), _ptr(H),
        _ptr(S), _stream(stream)), "tl_assemble_core_hamiltonian_block_noalloc")


def tl_set_contraction_events(start_event, stop_event):
    """start_event/stop_event: raw hipEvent_t handles (int) or None."""
    _check(load().tl_set_contraction_events(start_event, stop_event),
           "tl_set_contraction_events")


def tl_set_stage_events(stage, start_event, stop_event):
    """Profiling events (raw hipEvent_t handles or None) attached to one
    stage's kernel launch (TL_STAGE_*)."""
    _check(load().tl_set_stage_events(int(stage), start_event, stop_event),
           "tl_set_stage_events")


def tl_block_fft(inp, L1, L2, L3, m0, batch, out, ws=None, ws_bytes=0, stream=None):
    _check(load().tl_block_fft(_ptr(inp), int(L1), int(L2), int(L3), int(m0), int(batch),
                               _ptr(out), _ptr(ws), int(ws_bytes), _stream(stream)),
           "tl_block_fft")


def tl_batched_heigh(H, S, count, m0, evals, evecs, info, stream=None):
    _check(load().tl_batched_heigh(_ptr(H), _ptr(S), int(count), int(m0), _ptr(evals),
                                   _ptr(evecs), _ptr(info), _stream(stream)), "tl_batched_heigh")


def tl_bloch_vectors(evecs, L1, L2, L3, m0, states, n_states, out, stream=None):
    _check(load().tl_bloch_vectors(_ptr(evecs), int(L1), int(L2), int(L3), int(m0), _ptr(states),
                                   int(n_states), _ptr(out), _stream(stream)), "tl_bloch_vectors")


def tl_bloch_orbital_factors(sys, G, evecs, states, n_states, coef, factors, stream=None):
    h = _handle(sys)
    _check(load().tl_bloch_orbital_factors(h.ref, _ptr(G), _ptr(evecs), _ptr(states),
                                           int(n_states), _ptr(coef), _ptr(factors),
                                           _stream(stream)), "tl_bloch_orbital_factors")


def tl_chain_orbital_factors(sys, G, evecs, n_states, factors, stream=None):
    h = _handle(sys)
    _check(load().tl_chain_orbital_factors(h.ref, _ptr(G), _ptr(evecs), int(n_states),
                                           _ptr(factors), _stream(stream)),
           "tl_chain_orbital_factors")


def tl_btoepl_workspace_bytes(L, m0, nvec) -> int:
    v = ctypes.c_size_t()
    _check(load().tl_btoepl_workspace_bytes(int(L), int(m0), int(nvec), ctypes.byref(v)),
           "tl_btoepl_workspace_bytes")
    return v.value


def tl_btoepl_setup(A, L, m0, nvec, ws, ws_bytes, stream=None):
    _check(load().tl_btoepl_setup(_ptr(A), int(L), int(m0), int(nvec), _ptr(ws), int(ws_bytes),
                                  _stream(stream)), "tl_btoepl_setup")


def tl_btoepl_matvec(X, Y, L, m0, nvec, ws, ws_bytes, stream=None):
    _check(load().tl_btoepl_matvec(_ptr(X), _ptr(Y), int(L), int(m0), int(nvec), _ptr(ws),
                                   int(ws_bytes), _stream(stream)), "tl_btoepl_matvec")


def tl_btoepl_power(L, m0, iters, x, y, lam, ws, ws_bytes, stream=None):
    _check(load().tl_btoepl_power(int(L), int(m0), int(iters), _ptr(x), _ptr(y), _ptr(lam),
                                  _ptr(ws), int(ws_bytes), _stream(stream)), "tl_btoepl_power")


def tl_btoepl3_workspace_bytes(L1, L2, L3, m0, nvec) -> int:
    v = ctypes.c_size_t()
    _check(load().tl_btoepl3_workspace_bytes(int(L1), int(L2), int(L3), int(m0), int(nvec),
                                             ctypes.byref(v)), "tl_btoepl3_workspace_bytes")
    return v.value


def tl_btoepl3_setup(B, L1, L2, L3, m0, nvec, ws, ws_bytes, stream=None):
    _check(load().tl_btoepl3_setup(_ptr(B), int(L1), int(L2), int(L3), int(m0), int(nvec),
                                   _ptr(ws), int(ws_bytes), _stream(stream)), "tl_btoepl3_setup")


def tl_btoepl3_matvec(X, Y, L1, L2, L3, m0, nvec, ws, ws_bytes, stream=None):
    _check(load().tl_btoepl3_matvec(_ptr(X), _ptr(Y), int(L1), int(L2), int(L3), int(m0),
                                    int(nvec), _ptr(ws), int(ws_bytes), _stream(stream)),
           "tl_btoepl3_matvec")


def tl_btoepl3_power(L1, L2, L3, m0, iters, x, y, lam, ws, ws_bytes, stream=None):
    _check(load().tl_btoepl3_power(int(L1), int(L2), int(L3), int(m0), int(iters), _ptr(x),
                                   _ptr(y), _ptr(lam), _ptr(ws), int(ws_bytes), _stream(stream)),
           "tl_btoepl3_power")


def tl_btoepl_lowest_workspace_bytes(L, m0, nb) -> int:
    v = ctypes.c_size_t()
    _check(load().tl_btoepl_lowest_workspace_bytes(int(L), int(m0), int(nb), ctypes.byref(v)),
           "tl_btoepl_lowest_workspace_bytes")
    return v.value


def tl_btoepl_lowest(H, S, L, m0, nev, nb, max_iter, tol, shift, x0, evals, evecs, resid, ws,
                     ws_bytes, stream=None):
    """Returns (iterations, converged count)."""
    it, nc = ctypes.c_int(), ctypes.c_int()
    _check(load().tl_btoepl_lowest(_ptr(H), _ptr(S), int(L), int(m0), int(nev), int(nb),
                                   int(max_iter), float(tol), float(shift), _ptr(x0), _ptr(evals),
                                   _ptr(evecs), _ptr(resid), ctypes.byref(it), ctypes.byref(nc),
                                   _ptr(ws), int(ws_bytes), _stream(stream)), "tl_btoepl_lowest")
    return it.value, nc.value


def tl_btoepl3_lowest_workspace_bytes(L1, L2, L3, m0, nb) -> int:
    v = ctypes.c_size_t()
    _check(load().tl_btoepl3_lowest_workspace_bytes(int(L1), int(L2), int(L3), int(m0), int(nb),
                                                    ctypes.byref(v)),
           "tl_btoepl3_lowest_workspace_bytes")
    return v.value


def tl_btoepl3_lowest(H, S, L1, L2, L3, m0, nev, nb, max_iter, tol, shift, x0, evals, evecs,
                      resid, ws, ws_bytes, stream=None):
    """Returns (iterations, converged count)."""
    it, nc = ctypes.c_int(), ctypes.c_int()
    _check(load().tl_btoepl3_lowest(_ptr(H), _ptr(S), int(L1), int(L2), int(L3), int(m0),
                                    int(nev), int(nb), int(max_iter), float(tol), float(shift),
                                    _ptr(x0), _ptr(evals), _ptr(evecs), _ptr(resid),
                                    ctypes.byref(it), ctypes.byref(nc), _ptr(ws), int(ws_bytes),
                                    _stream(stream)), "tl_btoepl3_lowest")
    return it.value, nc.value


def tl_dense_gen_eigh_workspace_bytes(N, k) -> int:
    v = ctypes.c_size_t()
    _check(load().tl_dense_gen_eigh_workspace_bytes(int(N), int(k), ctypes.byref(v)),
           "tl_dense_gen_eigh_workspace_bytes")
    return v.value


def tl_set_dense_eigh_events(events=None):
    """events: six raw hipEvent_t handles (ints), or None to switch off."""
    if events is None:
        _check(load().tl_set_dense_eigh_events(None, 0), "tl_set_dense_eigh_events")
        return
    arr = (ctypes.c_void_p * len(events))(*events)
    _check(load().tl_set_dense_eigh_events(arr, len(events)), "tl_set_dense_eigh_events")


def tl_dense_gen_eigh_lowest(H, S, N, k, evals, evecs, info, ws, ws_bytes, stream=None):
    _check(load().tl_dense_gen_eigh_lowest(_ptr(H), _ptr(S), int(N), int(k), _ptr(evals),
                                           _ptr(evecs), _ptr(info), _ptr(ws), int(ws_bytes),
                                           _stream(stream)), "tl_dense_gen_eigh_lowest")


class SystemArray:
    """A contiguous C array of TlSystem for the batched entry points."""

    def __init__(self, systems):
        self.handles = [SystemHandle(s) for s in systems]
        self.array = (TlSystem * len(systems))(*[h.struct for h in self.handles])

    @property
    def ptr(self):
        return ctypes.cast(self.array, ctypes.c_void_p)

    def __len__(self):
        return len(self.handles)


def tl_batch_plan_create(systems, precision=TL_FP64, n_slices=0, want_blocks=0) -> TlBatchPlan:
    arr = systems if isinstance(systems, SystemArray) else SystemArray(systems)
    plan = TlBatchPlan()
    _check(load().tl_batch_plan_create(arr.ptr, len(arr), int(precision), int(n_slices),
                                       int(want_blocks), ctypes.byref(plan)),
           "tl_batch_plan_create")
    return plan


def tl_batch_write_descriptor(systems, plan, buffers: dict, host_desc) -> None:
    """buffers: name -> device tensor (G AG SG P HS HSbar evals info ws);
    host_desc: writable host buffer (numpy uint8 array) of plan.desc_bytes."""
    arr = systems if isinstance(systems, SystemArray) else SystemArray(systems)
    b = TlBatchBuffers(*[_ptr(buffers[n]) for n in
                         ("G", "AG", "SG", "P", "HS", "HSbar", "evals", "info", "ws")])
    _check(load().tl_batch_write_descriptor(arr.ptr, len(arr), ctypes.byref(plan),
                                            ctypes.byref(b), host_desc.ctypes.data,
                                            host_desc.nbytes), "tl_batch_write_descriptor")


def tl_batch_run(plan, host_desc, desc_dev, stream=None) -> None:
    _check(load().tl_batch_run(ctypes.byref(plan), host_desc.ctypes.data, _ptr(desc_dev),
                               _stream(stream)), "tl_batch_run")
