"""The C-ABI library loads, exports every declared symbol, and its host-side
logic (validation, layout) behaves; no device calls (runs without a GPU)."""
import ctypes
import os
import re
import subprocess
import tempfile

import pytest

import workloads as W
from paper_2110_03732_amd import grmhd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    txt = open(os.path.join(ROOT, "include", "grmhd.h")).read()
    return sorted(set(re.findall(r"\b(gr_[a-zA-Z0-9_]+)\s*\(", txt)))


def test_header_and_binding_agree():
    assert declared_symbols() == sorted(grmhd.EXPORTED)


def test_library_exports_every_declared_symbol():
    L = grmhd.lib()
    for name in declared_symbols():
        assert hasattr(L, name), name
    assert grmhd.gr_abi_version() == 6


def test_validation_rejects_bad_grids():
    s = W.blast_wave(16)
    g = grmhd.grid_of(s)
    assert grmhd.gr_validate(g) == 0
    for field, bad in [("ndim", 4), ("ng", 2), ("recon", 7), ("imex", 3), ("gamma_ad", 1.0), ("newton_maxit", 0),
                       ("rho_atm", 0.0), ("atm_factor", 0.5)]:
        g2 = grmhd.grid_of(s)
        setattr(g2, field, bad)
        assert grmhd.gr_validate(g2) == grmhd.GR_EINVAL, field
    g2 = grmhd.grid_of(s)
    g2.xi = 0.1
    assert grmhd.gr_validate(g2) == 0  # mean-field dynamo supported
    g2.xi = float("nan")
    assert grmhd.gr_validate(g2) == grmhd.GR_EINVAL
    g2 = grmhd.grid_of(s)
    g2.frozen_matter = 2
    assert grmhd.gr_validate(g2) == grmhd.GR_EINVAL
    g2 = grmhd.grid_of(s)
    g2.glm = 1
    assert grmhd.gr_validate(g2) == 0  # GLM cleaning supported
    g2.kappa_B = -1.0
    assert grmhd.gr_validate(g2) == grmhd.GR_EINVAL
    g2.kappa_B = 1.0
    g2.xi = 0.1
    assert grmhd.gr_validate(g2) == grmhd.GR_EUNSUPPORTED  # GLM with the dynamo term
    g2.xi = 0.0
    g2.uct = 1
    assert grmhd.gr_validate(g2) == grmhd.GR_EUNSUPPORTED  # GLM has no edge EMF
    g2.uct = 0
    g2.glm = 2
    assert grmhd.gr_validate(g2) == grmhd.GR_EINVAL
    g2 = grmhd.grid_of(s)
    g2.uct = 1
    assert grmhd.gr_validate(g2) == 0  # ideal-MHD edge EMF supported
    g2.uct = 2
    assert grmhd.gr_validate(g2) == grmhd.GR_EINVAL
    g2 = grmhd.grid_of(s)
    g2.bc[0][0] = W.PERIODIC  # periodic on one side only
    assert grmhd.gr_validate(g2) == grmhd.GR_EINVAL
    g2 = grmhd.grid_of(s)
    g2.n[0] = 2
    g2.bc[0][0] = g2.bc[0][1] = W.PERIODIC  # fewer cells than ghosts
    assert grmhd.gr_validate(g2) == grmhd.GR_EINVAL
    assert grmhd.gr_workspace_bytes(g2) == 0
    assert grmhd.gr_field_stride(g2) == 0 and grmhd.gr_row_stride(g2) == 0 and grmhd.gr_field_origin(g2) == 0


def test_validation_size_limits():
    """a field must stay below 2^32 bytes (32-bit offsets: at most 5e8 points
    with padded rows) and the padded z extent is a launch-grid dimension
    (<= 65535)"""
    s = W.tov_star(16)
    g = grmhd.grid_of(s)
    for n, ok in [((780, 780, 780), True), ((800, 800, 800), False), ((4, 4, 65529), True), ((4, 4, 65530), False)]:
        g.n[0], g.n[1], g.n[2] = n
        pts = (n[0] + 2 * g.ng + 15) // 16 * 16 * (n[1] + 2 * g.ng) * (n[2] + 2 * g.ng) + (16 - g.ng % 16) % 16
        assert (pts <= 5e8 and n[2] + 2 * g.ng <= 65535) == ok
        assert (grmhd.gr_validate(g) == 0) == ok, n
    g.n[0] = g.n[1] = g.n[2] = 0
    assert grmhd.gr_validate(g) == grmhd.GR_EINVAL  # empty grid


@pytest.mark.parametrize("make", [lambda: W.shock_tube(400), lambda: W.blast_wave(512), lambda: W.tov_star(32),
                                  lambda: W.glm_monopole(24, ndim=3), lambda: W.glm_wave(64)])
def test_layout(make):
    s = make()
    g = grmhd.grid_of(s)
    fs = grmhd.gr_field_stride(g)
    assert fs >= s.shape[0] * s.shape[1] * s.shape[2] and fs % 32 == 0
    # padded rows: whole 128-byte lines, the first interior point of every
    # row on a line boundary, everything inside the field
    Nz, Ny, Nx = s.shape
    P, o = grmhd.gr_row_stride(g), grmhd.gr_field_origin(g)
    assert P % 16 == 0 and Nx <= P < Nx + 16
    assert 0 <= o < 16 and (o + s.ng) % 16 == 0
    assert o + P * Ny * Nz <= fs
    wb = grmhd.gr_workspace_bytes(g)
    nst = 2 if s.imex == W.SSP2 else 4
    # stage prims + E (+ Psi, Phi with GLM), stage faces, stored L (+ q_B,
    # q_Psi, q_Phi components with GLM), stored R
    fields = [(0, 10), (1, 3), (2, 13), (3, 3)] if s.glm else [(0, 8), (1, 3), (2, 11), (3, 3)]
    offs = set()
    for kind, nf in fields:
        for st in range(nst):
            for f in range(nf):
                o = grmhd.gr_workspace_offset(g, kind, st, f)
                assert o % 256 == 0 and o + 8 * fs <= wb
                offs.add(o)
        with pytest.raises(grmhd.GrError):
            grmhd.gr_workspace_offset(g, kind, 0, nf)
    assert len(offs) == nst * sum(nf for _, nf in fields)  # no two fields share storage
    with pytest.raises(grmhd.GrError):
        grmhd.gr_workspace_offset(g, 0, nst, 0)


def test_strerror():
    L = grmhd.lib()
    assert L.gr_strerror(0) == b"ok"
    assert L.gr_strerror(-2) == b"workspace too small"
    assert ctypes.sizeof(grmhd.gr_grid) > 0


def test_batch_create_rejects_bad_arguments():
    """host-side checks of gr_batch_create, made before any device call"""
    s1, s2 = W.shock_tube(64), W.blast_wave(16)  # IMEX-SSP2 and IMEX-SSP3
    g1, g2 = grmhd.grid_of(s1), grmhd.grid_of(s2)
    fake = 1 << 20

    def state(g):
        st = grmhd.gr_state()
        st.q = st.face = st.prim = st.work = fake
        st.work_bytes = grmhd.gr_workspace_bytes(g)
        return st

    h = ctypes.c_void_p()
    L = grmhd.lib()
    ga = (grmhd.gr_grid * 2)(g1, g2)
    sa = (grmhd.gr_state * 2)(state(g1), state(g2))
    da = (ctypes.c_double * 2)(1e-3, 1e-3)
    assert L.gr_batch_create(ctypes.byref(h), ga, sa, da, 0, None, None) == grmhd.GR_EINVAL
    assert L.gr_batch_create(ctypes.byref(h), ga, sa, da, 2, None, None) == grmhd.GR_EUNSUPPORTED
    bad = (ctypes.c_double * 2)(1e-3, 0.0)
    g2b = grmhd.grid_of(W.blast_wave(16, imex=W.SSP2))
    ga2 = (grmhd.gr_grid * 2)(g1, g2b)
    sa2 = (grmhd.gr_state * 2)(state(g1), state(g2b))
    assert L.gr_batch_create(ctypes.byref(h), ga2, sa2, bad, 2, None, None) == grmhd.GR_EINVAL
    small = state(g1)
    small.work_bytes = 8
    sa3 = (grmhd.gr_state * 1)(small)
    assert L.gr_batch_create(ctypes.byref(h), ga, sa3, da, 1, None, None) == grmhd.GR_ENOMEM
    assert h.value is None
    assert L.gr_batch_destroy(None) == grmhd.GR_OK


def test_header_is_plain_c():
    """include/grmhd.h compiles as C99 with warnings as errors (the boundary
    needs no C++ or PyTorch type)"""
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "t.c")
        with open(src, "w") as f:
            f.write('#include "grmhd.h"\nint main(void) { gr_grid g; (void)g; return gr_abi_version() > 0 ? 0 : 1; }\n')
        subprocess.check_call(["gcc", "-std=c99", "-Wall", "-Wextra", "-Werror", "-fsyntax-only",
                               "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"),
                               "-I", os.path.join(rocm, "include"), src])
