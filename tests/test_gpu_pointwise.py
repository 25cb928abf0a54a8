"""Point-wise parity of the fused implicit solve (pass 0, Sec 2.4) and of the
recovery with E and B given (gr_con2prim, Sec 2.6) over the grid of the
oracle's own pins: W in {1, 1.01, 2, 10, 100}, sigma in {0, 1, 1e2, 1e4},
p/rho in {1e-6 .. 1e2}, eta~ in {1e-8 .. 1e8}, flat and with a constant
metric.

Bound per cell: both sides solve for the same unique root; each is within
its stopping tolerance of it, and the root itself is conditioned by the
cancellation in p = (w~/W - rho)/Gamma_1, where tau + D carries the rest mass,
kinetic and field energies: the relative error of the primitives may reach
eps (tau + D)/p.  The test allows 1e-12 max(1, (tau + D)/p) relative (u~
relative to max(1, |u~|)), the bound the oracle's own round trip meets, and
1e-12 max(1, (tau + D)/p) of max(|E|, |B|) for the electric field.
"""
import ctypes

import numpy as np
import pytest

import oracle
import workloads as W
from parity import say

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch


def _cond(s, q, p):
    """(tau + D)/p per interior cell, from the oracle's conserved variables
    and pressure"""
    sl = s.interior
    ps6 = 1.0 if not s.metric else s.psi[sl] ** 6
    tD = (q[4][sl] + q[0][sl]) / ps6
    return np.maximum(1.0, tD / np.maximum(p, 1e-300))


def _bmag(s):
    """|B| of every interior cell (contravariant components, orthonormal
    magnitude), from the initial face fields"""
    sl = s.interior
    f = s.face
    ps6 = 1.0 if not s.metric else s.psi ** 6
    B = []
    for d in range(3):
        if s.active(d):
            up = np.roll(f[d], -1, axis=2 - d)
            B.append((0.5 * (f[d] + up) / ps6)[sl])
        else:
            B.append((f[d] / ps6)[sl])
    ps4 = 1.0 if not s.metric else s.psi[sl] ** 4
    return np.sqrt(ps4 * (B[0] ** 2 + B[1] ** 2 + B[2] ** 2))


def _emag(s, E):
    ps4 = 1.0 if not s.metric else s.psi[s.interior] ** 4
    return np.sqrt(ps4 * (E[0] ** 2 + E[1] ** 2 + E[2] ** 2))


def _rel(got, want, sc):
    return np.abs(got - want) / sc


METRICS = {"flat": None, "alpha0.8_psi1.3": (0.8, 1.3)}


@pytest.mark.parametrize("met", sorted(METRICS))
def test_pin_grid_con2prim(met):
    _torch()
    from paper_2110_03732_amd import grmhd
    s = W.pin_grid_states(seed=4, metric=METRICS[met])
    say("pin grid con2prim %s: %d cells" % (met, s.ncells))
    run = grmhd.Run(s, device="cuda:0")
    run.con2prim()
    got = run.prims()
    ref = oracle.OracleState(s)
    cond = _cond(s, ref.q, s.prim[4][s.interior])
    nf = oracle.lib().or_c2p_grid(ctypes.byref(ref.grid), oracle._pp(ref.q), oracle._pp(ref.face),
                                  oracle._pp(ref.prim), oracle._p(ref.psi))
    assert nf == 0 and run.fail_count() == 0
    sl = s.interior
    worst = 0.0
    for v in range(5):
        a, b, t = got[v][sl], ref.prim[v][sl], s.prim[v][sl]
        sc = np.abs(b) if v in (0, 4) else np.maximum(1.0, np.abs(b))
        e = _rel(a, b, sc) / cond
        e0 = _rel(a, t, np.abs(t) if v in (0, 4) else np.maximum(1.0, np.abs(t))) / cond
        worst = max(worst, e.max(), e0.max())
        assert e.max() <= 1e-12, (v, e.max(), int(e.argmax()))
        assert e0.max() <= 1e-12, (v, e0.max(), int(e0.argmax()))
    say("  worst relative error / condition %.1e" % worst)


ETATS = [1e-8, 1e-4, 1.0, 1e4, 1e8]


def _cell_B(s):
    """contravariant cell-centred B of every interior cell (3, ...)"""
    sl = s.interior
    ps6 = 1.0 if not s.metric else s.psi ** 6
    out = []
    for d in range(3):
        f = s.face[d]
        if s.active(d):
            f = 0.5 * (f + np.roll(f, -1, axis=2 - d))
        out.append((f / ps6)[sl])
    return np.stack(out)


def _manufactured_Es(s, etat):
    """E* that eq. im_E (xi = 0) maps onto the state's own E for this eta~:
    E* = E + (W/eta~) [E + v x B - (E . v) v] with the metric gamma_ij =
    psi^4 delta_ij (v x B = eps^{ijk} v_j B_k, (E . v) = gamma_ij E^i v^j)"""
    sl = s.interior
    psi = 1.0 if not s.metric else s.psi[sl]
    g = psi ** 4
    u = np.stack([s.prim[1 + d][sl] for d in range(3)])
    Wl = np.sqrt(1.0 + g * (u ** 2).sum(0))
    v = u / Wl
    B = _cell_B(s)
    E = np.stack([s.E[d][sl] for d in range(3)])
    vxB = np.cross((v * g).reshape(3, -1).T, (B * g).reshape(3, -1).T).T.reshape(E.shape) / psi ** 6
    Ev = g * (E * v).sum(0)
    return E + (Wl / etat) * (E + vxB - Ev * v)


def _set_qE(s, run, ref, Es):
    """write q_E = psi^6 E* into the interior cells of both states"""
    sl = s.interior
    ps6 = 1.0 if not s.metric else s.psi[sl] ** 6
    qd = run.q.view(run.nq, run.fs)
    Nz, Ny, Nx = s.shape
    k, j, i = np.meshgrid(np.arange(Nz)[sl[0]], np.arange(Ny)[sl[1]], np.arange(Nx)[sl[2]], indexing="ij")
    idx = run.torch.as_tensor((run.origin + i + run.pitch * (j + Ny * k)).ravel(), device=qd.device)
    for d in range(3):
        val = (ps6 * Es[d]).ravel()
        qd[5 + d].index_copy_(0, idx, run.torch.as_tensor(val, dtype=run.torch.float64, device=qd.device))
        ref.q[5 + d][sl] = ps6 * Es[d]
    run.torch.cuda.synchronize()


@pytest.mark.parametrize("met", sorted(METRICS))
@pytest.mark.parametrize("etat", ETATS)
def test_pin_grid_implicit_stage(met, etat):
    """pass 0 of IMEX-SSP2 is the fused implicit E + u~ solve alone; with q_E
    set to the manufactured E* of each cell the solve must return the cell's
    own primitives and E (the oracle's manufactured-root pin, extended to the
    whole pin grid); eta~ = eta/(alpha a_00 dt)"""
    _torch()
    from paper_2110_03732_amd import grmhd
    s = W.pin_grid_states(seed=6, metric=METRICS[met])
    alpha = 1.0 if s.metric == 0 else METRICS[met][0]
    dt = 0.01
    _, A, _, _ = oracle.tableau(W.SSP2)
    s.eta = etat * alpha * A[0, 0] * dt
    say("pin grid implicit stage %s eta~ %.0e: %d cells" % (met, etat, s.ncells))
    run = grmhd.Run(s, device="cuda:0")
    ref = oracle.OracleState(s)
    _set_qE(s, run, ref, _manufactured_Es(s, etat))
    q0 = [a.copy() for a in ref.q]
    run.stage(0, dt)
    stage, _ = ref.step(dt, dump_stage=0)
    sl = s.interior
    gstage = [run.work_field(0, 0, f)[sl] for f in range(8)]
    rstage = [stage[f][sl] for f in range(8)]
    truth = [s.prim[v][sl] for v in range(5)] + [s.E[d][sl] for d in range(3)]
    cond = _cond(s, q0, truth[4])
    em = np.maximum(np.maximum(_emag(s, truth[5:8]), _bmag(s)), 1e-300)
    worst = worst_t = 0.0
    for f in range(8):
        a, b, c = gstage[f], rstage[f], truth[f]
        if f in (0, 4):
            sc = np.abs(c)
        elif f < 4:
            sc = np.maximum(1.0, np.abs(c))
        else:
            sc = em
        e = _rel(a, b, sc) / cond
        et = np.maximum(_rel(a, c, sc), _rel(b, c, sc)) / cond
        worst, worst_t = max(worst, e.max()), max(worst_t, et.max())
        assert e.max() <= 1e-12, (f, e.max(), int(e.argmax()))
        assert et.max() <= 1e-11, (f, et.max(), int(et.argmax()))
    say("  worst relative error / condition: device-oracle %.1e, against the root %.1e" % (worst, worst_t))
    assert run.fail_count() == 0


@pytest.mark.parametrize("imex", [W.SSP2, W.SSP3])
@pytest.mark.parametrize("wmax", [10.0, 100.0])
@pytest.mark.parametrize("eta", [3e-11, 3e-7, 3e-3, 3e1])
def test_stage_one_implicit_parity(imex, wmax, eta):
    """pass 0 is the point-wise fused implicit solve only (no spatial
    operator), on random states up to W = wmax; eta spans eta~ from about
    1e-8 to 1e4 (dt = 0.01, a_00 = 0.29 / 0.24)"""
    _torch()
    from paper_2110_03732_amd import grmhd
    say("case random_states: implicit stage, imex %d, W <= %g, eta %g" % (imex, wmax, eta))
    s = W.random_states((10, 9, 8), seed=5, wmax=wmax)
    s.imex = imex
    s.eta = eta
    run = grmhd.Run(s, device="cuda:0")
    dt = 0.01
    run.stage(0, dt)
    ref = oracle.OracleState(s)
    q0 = [a.copy() for a in ref.q]
    stage, _ = ref.step(dt, dump_stage=0)
    sl = s.interior
    rstage = [stage[f][sl] for f in range(8)]
    cond = _cond(s, q0, rstage[4])
    em = np.maximum(np.maximum(_emag(s, rstage[5:8]), _bmag(s)), 1e-300)
    worst = 0.0
    for f in range(8):
        g = run.work_field(0, 0, f)[sl]
        r = rstage[f]
        if f in (0, 4):
            sc = np.abs(r)
        elif f < 4:
            sc = np.maximum(1.0, np.abs(r))
        else:
            sc = em
        e = np.abs(g - r) / sc / cond
        worst = max(worst, e.max())
        assert e.max() <= 1e-12, (f, e.max())
    fo = rstage[0] == s.rho_atm
    assert np.array_equal(run.work_field(0, 0, 0)[sl] == s.rho_atm, fo)
    say("  worst relative error / condition %.1e, fallbacks %d" % (worst, int(fo.sum())))
    assert run.fail_count() == int(fo.sum())
