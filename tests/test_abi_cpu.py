"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every entry point declared in include/tl.h, reports the documented sizes and
rejects invalid arguments before enqueuing anything."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1408_3839_amd import tl, workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "tl.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(tl_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    lib = tl.load()
    names = _declared()
    assert "tl_batched_heigh" in names and len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n
        assert n in tl.SIGNATURES, n


def test_version_and_status_strings():
    assert "gfx950" in tl.tl_version()
    lib = tl.load()
    assert lib.tl_status_string(tl.TL_EWORKSPACE).decode() == "workspace too small"


@pytest.mark.parametrize("cid", [1, 2, 3, 5])
def test_sizes(cid):
    s = wl.config(cid)
    z = tl.tl_query_sizes(s)
    groups = len({(float(p[1]), float(p[2])) for p in s.nuc_pos})
    assert z["pot_terms"] == s.R * groups
    rows = [s.m0 * (s.ncells if (s.mode == "box" and d == 0) else 1) for d in range(3)]
    assert z["basis_rows"] == rows
    assert z["basis_elems"] == sum(rows[d] * int(s.n[d]) for d in range(3))
    assert z["pot_elems"] == z["pot_terms"] * int(np.sum(s.n))
    nb = s.ncells * s.m0
    assert z["block_elems"] == (nb * nb if s.mode == "box" else s.ncells * s.m0 * s.m0)


def _expect(status_fn, code, *args):
    with pytest.raises(tl.TlError) as ei:
        status_fn(*args)
    assert tl.load().tl_status_string(code).decode() in str(ei.value)
    return str(ei.value)


def test_invalid_systems_rejected():
    base = wl.config(1)
    cases = []
    s = wl.config(1); s.h = 0.0; cases.append((s, "grid step"))
    s = wl.config(1); s.fn_alpha = s.fn_alpha.copy(); s.fn_alpha[0] = -1.0; cases.append((s, "fn_alpha"))
    s = wl.config(1); s.a = s.a.copy(); s.a[0] = 2.03; cases.append((s, "a[0]/h"))
    s = wl.config(1); s.n = s.n.copy(); s.n[0] = 127; cases.append((s, "n[0]"))
    s = wl.config(1); s.nuc_pos = s.nuc_pos + np.array([0.01, 0, 0]); cases.append((s, "multiples of h"))
    s = wl.config(1); s.fn_l = s.fn_l.copy(); s.fn_l[0][0] = 2; cases.append((s, "fn_l"))
    s = wl.config(1); s.t_q = s.t_q.copy(); s.t_q[3] = np.nan; cases.append((s, "quadrature"))
    for sys, frag in cases:
        msg = _expect(tl.tl_query_sizes, tl.TL_EINVAL, sys)
        assert frag in msg, (frag, msg)
    s = wl.tiny_periodic(m0=3)
    s.fn_alpha = np.ones(33); s.fn_l = np.zeros((33, 3), int); s.fn_center = np.zeros((33, 3))
    s.fn_coef = np.ones((33, 3))
    assert "m0" in _expect(tl.tl_query_sizes, tl.TL_EINVAL, s)
    assert base.R <= 64


def test_null_outputs_and_small_workspaces_rejected():
    s = wl.config(1)
    _expect(tl.tl_build_basis, tl.TL_EINVAL, s, 0, 0, 0, 0)
    _expect(tl.tl_lattice_sum_potential, tl.TL_EINVAL, s, 0, 0, 0, 0)
    _expect(tl.tl_assemble_core_hamiltonian_block, tl.TL_EWORKSPACE, s, 8, 8, 8, 8,
            tl.TL_FP64, 0, 8, 8, 0, 0, 0)
    _expect(tl.tl_assemble_core_hamiltonian_block, tl.TL_EINVAL, s, 8, 8, 8, 8, 7, 0, 8, 8,
            0, 0, 0)
    _expect(tl.tl_block_fft, tl.TL_EINVAL, 8, 0, 1, 1, 4, 1, 8, 0, 0, 0)
    # lattices the LDS FFT cannot hold (a non-7-smooth extent on one of several
    # axes) take the per-axis direct DFT, which needs a workspace
    _expect(tl.tl_block_fft, tl.TL_EWORKSPACE, 8, 11, 3, 1, 4, 1, 8, 0, 0, 0)
    _expect(tl.tl_batched_heigh, tl.TL_EINVAL, 8, 0, 4, 0, 8, 0, 8, 0)
    _expect(tl.tl_batched_heigh, tl.TL_EINVAL, 8, 0, 4, 33, 8, 0, 8, 0)
    _expect(tl.tl_batched_heigh, tl.TL_EINVAL, 0, 0, 4, 4, 8, 0, 8, 0)
    _expect(tl.tl_build_basis_and_potential, tl.TL_EINVAL, s, 8, 8, 8, 0, 0, 0, 0)


def test_workspace_queries():
    for cid in (1, 2, 5):
        s = wl.config(cid)
        assert tl.tl_potential_workspace_bytes(s) == 0
        assert tl.tl_assemble_workspace_bytes(s) % 256 == 0
    # whole lattices in LDS: 7-smooth lattices of up to 4096 cells need no
    # workspace; other chain lengths up to 2048 (Bluestein) keep the chirp
    # c(k), k < L, and the filter's transform (M = 4096 points) there
    assert tl.tl_block_fft_workspace_bytes(64, 1, 1, 8, 2) == 0
    assert tl.tl_block_fft_workspace_bytes(8, 8, 8, 10, 2) == 0
    assert tl.tl_block_fft_workspace_bytes(2039, 1, 1, 4, 2) == 384 * 256   # 16 (2039 + 4096)
    assert tl.tl_block_fft_workspace_bytes(37, 1, 1, 4, 2) == 7 * 256      # 16 (37 + 75)
    assert tl.tl_block_fft_workspace_bytes(4099, 1, 1, 4, 2) == 0      # one axis: no workspace
    assert tl.tl_block_fft_workspace_bytes(11, 3, 1, 4, 2) == 8 * 2 * 33 * 16 * 2
    assert tl.tl_block_fft_workspace_bytes(16, 16, 32, 2, 1) == 8 * 2 * 8192 * 4


def test_box_mode_queries_and_rejections():
    s = wl.config(3)
    z = tl.tl_query_sizes(s)
    nb = z["basis_rows"][0]
    assert nb == 2048
    wb = tl.tl_assemble_workspace_bytes(s)
    assert wb > 0 and wb % 256 == 0
    # the open-boundary assembly runs in FP64 or a split mode, with a valid
    # slice count; the checks precede any launch
    _expect(tl.tl_assemble_core_hamiltonian_block, tl.TL_EUNSUPPORTED, s, 8, 8, 8, 8,
            tl.TL_FP32, 0, 8, 8, 8, wb, 0)
    _expect(tl.tl_assemble_core_hamiltonian_block, tl.TL_EINVAL, s, 8, 8, 8, 8,
            tl.TL_SPLIT_FP16, 7, 8, 8, 8, wb, 0)
    _expect(tl.tl_assemble_core_hamiltonian_block, tl.TL_EINVAL, s, 8, 8, 8, 8,
            tl.TL_SPLIT_BF16, 1, 8, 8, 8, wb, 0)
    # workspace: the transverse contraction, the factor tables and the
    # weighted potentials Q[mu][nu] (m0^2 n_x doubles)
    assert wb >= 8 * 8 * 8 * 8500
    assert tl.tl_assemble_workspace_bytes(s, tl.TL_SPLIT_FP16, 5) == wb
    _expect(tl.tl_assemble_core_hamiltonian_block, tl.TL_EWORKSPACE, s, 8, 8, 8, 8,
            tl.TL_FP64, 0, 8, 8, 8, wb - 256, 0)


def test_dense_eigh_validation():
    b = tl.tl_dense_gen_eigh_workspace_bytes(2048, 64)
    assert b >= 4 * 2048 * 2048 * 8 and b % 256 == 0
    assert tl.tl_dense_gen_eigh_workspace_bytes(1, 1) > 0
    for N, k in [(0, 1), (10, 0), (10, 11), (200, 65), (7681, 1)]:
        with pytest.raises(tl.TlError):
            tl.tl_dense_gen_eigh_workspace_bytes(N, k)
    _expect(tl.tl_dense_gen_eigh_lowest, tl.TL_EINVAL, 8, 8, 100, 101, 8, 8, 8, 8, 1 << 30, 0)
    _expect(tl.tl_dense_gen_eigh_lowest, tl.TL_EINVAL, 0, 8, 100, 10, 8, 8, 8, 8, 1 << 30, 0)
    _expect(tl.tl_dense_gen_eigh_lowest, tl.TL_EWORKSPACE, 8, 8, 100, 10, 8, 8, 8, 8, 1024, 0)


def test_noalloc_assembly_rejects_oversize_before_enqueue():
    """The allocation-free assembly refuses, on the host, a system whose
    scratch exceeds its static 32 MiB (no device memory is touched: the
    pointers below are never dereferenced)."""
    big = wl.tiny_periodic(L=(512, 1, 1), m0=32, c=64, h=0.25, R=64)
    hb = tl.SystemHandle(big)
    assert tl.tl_assemble_workspace_bytes(hb, tl.TL_SPLIT_BF16, 8) > 32 << 20
    fake = 1 << 40
    msg = _expect(tl.tl_assemble_core_hamiltonian_block_noalloc, tl.TL_EUNSUPPORTED, hb,
                  fake, fake, fake, fake, tl.TL_SPLIT_BF16, 8, fake, fake, 0)
    assert "static scratch" in msg


def test_kblocks_queries_and_rejections():
    s = wl.config(5)
    b = tl.tl_assemble_kblocks_workspace_bytes(s)
    base = tl.tl_assemble_workspace_bytes(s)
    # (T + 2)(L1 + L2 + L3) = 66 * 24 factors fit the fused kernel's LDS
    assert b == base
    c2 = wl.config(2)
    assert tl.tl_assemble_kblocks_workspace_bytes(c2) == tl.tl_assemble_workspace_bytes(c2)
    # 42 * 130 factors do not: (T + 2) m0^2 L complex values per transformed dim
    big = wl.tiny_periodic(L=(128, 1, 1), m0=2, c=4, h=0.5, R=40)
    assert tl.tl_assemble_kblocks_workspace_bytes(big) == \
        tl.tl_assemble_workspace_bytes(big) + 42 * 4 * 128 * 16
    with pytest.raises(tl.TlError):
        tl.tl_assemble_kblocks_workspace_bytes(wl.config(3))   # box mode
    _expect(tl.tl_assemble_kblocks, tl.TL_EUNSUPPORTED, wl.config(3), 8, 8, 8, 8, tl.TL_FP64, 0,
            8, 8, 8, 1 << 30, 0)
    _expect(tl.tl_assemble_kblocks, tl.TL_EWORKSPACE, s, 8, 8, 8, 8, tl.TL_FP64, 0, 8, 8, 8,
            b - 256, 0)
    _expect(tl.tl_assemble_kblocks, tl.TL_EINVAL, s, 8, 8, 8, 8, tl.TL_SPLIT_FP16, 9, 8, 8, 8,
            b, 0)


def test_bloch_vectors_validation():
    _expect(tl.tl_bloch_vectors, tl.TL_EINVAL, 8, 0, 1, 1, 4, 8, 3, 8, 0)
    _expect(tl.tl_bloch_vectors, tl.TL_EINVAL, 8, 4, 1, 1, 33, 8, 3, 8, 0)
    _expect(tl.tl_bloch_vectors, tl.TL_EINVAL, 8, 4, 1, 1, 4, 8, -1, 8, 0)
    _expect(tl.tl_bloch_vectors, tl.TL_EINVAL, 0, 4, 1, 1, 4, 8, 3, 8, 0)
    tl.tl_bloch_vectors(0, 4, 1, 1, 4, 0, 0, 0, 0)  # no states: nothing to do, no launch


def test_batch_plan_tile_edge():
    """The plan carries the FP64 tile edge (64 by default); a descriptor is
    only written for 64 or 32 (host check, before any device address is
    used)."""
    systems = [wl.tiny_periodic(L=(4, 1, 1)), wl.tiny_periodic(L=(5, 1, 1), m0=2)]
    plan = tl.tl_batch_plan_create(systems)
    assert plan.tile_edge == 64
    plan.tile_edge = 48
    fake = {n: 8 for n in ("G", "AG", "SG", "P", "HS", "HSbar", "evals", "info", "ws")}
    host = np.zeros(plan.desc_bytes, dtype=np.uint8)
    with pytest.raises(tl.TlError) as ei:
        tl.tl_batch_write_descriptor(systems, plan, fake, host)
    assert "tile_edge" in str(ei.value)


def test_btoepl_sizes_and_validation():
    b = tl.tl_btoepl_workspace_bytes(256, 8, 64)
    # k-blocks 2L m0^2 complex; padded X, its transform, [R; I] and their transforms
    assert b >= 8 * (2 * 512 * 64 + 512 * 512 + 2 * 512 * 512 + 2 * 512 * 512 + 4 * 512 * 512)
    with pytest.raises(tl.TlError):
        tl.tl_btoepl_workspace_bytes(0, 8, 1)
    with pytest.raises(tl.TlError):
        tl.tl_btoepl_workspace_bytes(2049, 8, 1)
    with pytest.raises(tl.TlError):
        tl.tl_btoepl_workspace_bytes(16, 33, 1)
    with pytest.raises(tl.TlError):
        tl.tl_btoepl_workspace_bytes(16, 4, 0)
    _expect(tl.tl_btoepl_matvec, tl.TL_EINVAL, 8, 8, 16, 4, 2, 8, 8, 0)   # workspace too small
    _expect(tl.tl_btoepl_power, tl.TL_EINVAL, 16, 4, 0, 8, 8, 8, 8, 1 << 30, 0)


def test_bloch_orbital_factors_validation():
    box = wl.config(3)
    _expect(lambda: tl.tl_bloch_orbital_factors(box, 8, 8, 8, 1, 8, 8, 0), tl.TL_EUNSUPPORTED)
    per = wl.config(1)
    _expect(lambda: tl.tl_bloch_orbital_factors(per, None, 8, 8, 1, 8, 8, 0), tl.TL_EINVAL)
    _expect(lambda: tl.tl_bloch_orbital_factors(per, 8, 8, 8, -1, 8, 8, 0), tl.TL_EINVAL)
    tl.tl_bloch_orbital_factors(per, None, None, None, 0, None, None, 0)  # nothing to do
    _expect(lambda: tl.tl_chain_orbital_factors(per, 8, 8, 1, 8, 0), tl.TL_EUNSUPPORTED)
    _expect(lambda: tl.tl_chain_orbital_factors(box, None, 8, 1, 8, 0), tl.TL_EINVAL)
    tl.tl_chain_orbital_factors(box, None, None, 0, None, 0)


def test_btoepl3_sizes_and_validation():
    b = tl.tl_btoepl3_workspace_bytes(4, 3, 2, 2, 3)
    # embedded k-blocks, padded X, its transform, [R; I] and their transforms
    P, Ev = 8 * 4 * 3 * 2, 2 * 3
    assert b >= 8 * (2 * P * 4 + P * Ev + 2 * P * Ev + 2 * P * Ev + 4 * P * Ev)
    assert tl.tl_btoepl3_workspace_bytes(37, 1, 1, 2, 1) > 0  # Bluestein on one level
    with pytest.raises(tl.TlError):
        tl.tl_btoepl3_workspace_bytes(9, 8, 8, 1, 1)  # 4608 embedded cells
    with pytest.raises(tl.TlError):
        tl.tl_btoepl3_workspace_bytes(0, 1, 1, 1, 1)
    _expect(lambda: tl.tl_btoepl3_workspace_bytes(11, 2, 1, 1, 1), tl.TL_EUNSUPPORTED)
    _expect(lambda: tl.tl_btoepl3_matvec(8, 8, 4, 3, 2, 2, 3, 8, 8, 0), tl.TL_EWORKSPACE)


def test_btoepl3_lowest_sizes_and_validation():
    assert tl.tl_btoepl3_lowest_workspace_bytes(4, 4, 3, 2, 6) > 0
    with pytest.raises(tl.TlError):
        tl.tl_btoepl3_lowest_workspace_bytes(9, 8, 8, 1, 4)  # 4608 embedded cells
    with pytest.raises(tl.TlError):
        tl.tl_btoepl3_lowest_workspace_bytes(4, 4, 3, 2, 22)
    for bad in [dict(nev=7), dict(nb=22), dict(L1=1, L2=1, L3=1), dict(tol=0.0), dict(L2=0)]:
        a = dict(L1=4, L2=4, L3=3, nev=4, nb=6, tol=1e-9)
        a.update(bad)
        _expect(lambda: tl.tl_btoepl3_lowest(8, 8, a["L1"], a["L2"], a["L3"], 2, a["nev"], a["nb"],
                                             10, a["tol"], 0.0, None, 8, None, None, 8, 8, 0),
                tl.TL_EINVAL)


def test_btoepl_lowest_sizes_and_validation():
    b = tl.tl_btoepl_lowest_workspace_bytes(256, 4, 12)
    # two embedded operators, 15 blocks of N nb vectors, the preconditioner's k-blocks
    assert b >= 2 * tl.tl_btoepl_workspace_bytes(256, 4, 12) + 8 * 15 * 1024 * 12
    with pytest.raises(tl.TlError):
        tl.tl_btoepl_lowest_workspace_bytes(256, 4, 22)
    with pytest.raises(tl.TlError):
        tl.tl_btoepl_lowest_workspace_bytes(2049, 4, 8)
    args = dict(H=8, S=8, L=64, m0=4, nev=4, nb=8, max_iter=10, tol=1e-9, shift=0.0, x0=None,
                evals=8, evecs=None, resid=None, ws=8, ws_bytes=8, stream=0)

    def call(**kw):
        a = dict(args, **kw)
        return tl.tl_btoepl_lowest(a["H"], a["S"], a["L"], a["m0"], a["nev"], a["nb"],
                                   a["max_iter"], a["tol"], a["shift"], a["x0"], a["evals"],
                                   a["evecs"], a["resid"], a["ws"], a["ws_bytes"], a["stream"])
    for bad in [dict(nev=9), dict(nev=0), dict(nb=22), dict(L=5, m0=1), dict(max_iter=0),
                dict(tol=0.0), dict(H=None), dict(evals=None)]:
        _expect(lambda: call(**bad), tl.TL_EINVAL)
    _expect(call, tl.TL_EWORKSPACE)  # 8 bytes of workspace
