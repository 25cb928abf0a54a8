"""Pins of the oracle's ideal-MHD upwind constrained transport (App. A):
the edge electric field from reconstructed transport velocities and face
fields.  Pins: exactness on a uniform flow through a linear divergence-free
field (the CT face update then equals -(v . grad) B, the exact induction
equation, for every reconstruction; the resistive UCT of Sec 3.2 gives the
same); free streaming of a uniform state; div B at round-off and periodic face
totals conserved; agreement with the resistive UCT in the ideal limit
converging with resolution on a smooth field; mirror symmetry of the blast
wave; B^x bit-constant in 1-D; the constant-metric rescaling test (in
test_oracle_spatial.py) covers the metric factors."""
import ctypes
import math

import numpy as np
import pytest

import oracle
import workloads as W
from oracle import _p, _pp


def _run(s, steps, dt=None):
    st = oracle.OracleState(s)
    dt = st.dt() if dt is None else dt
    for _ in range(steps):
        st.step(dt)
    return st


def _linear_field_setup(ndim, recon, uct):
    n = {2: 10, 3: 8}[ndim]
    ng = 3 if recon == W.PPM else 2
    s = W._blank(W.Setup("linear_B", ndim, (n, n, n), ng, (0, 0, 0), (1.0, 0.8, 0.9), W._bc(ndim, W.PERIODIC),
                         5.0 / 3.0, recon, W.SSP2, eta=1e-3, uct=uct))
    v = np.array([0.31, -0.22, 0.17 if ndim == 3 else 0.0])
    B0 = np.array([0.4, -0.3, 0.25])
    sl = {"s1": 0.7, "s2": -0.45, "s3": 0.35, "s4": -0.6, "s5": 0.5 if ndim == 3 else 0.0,
          "s6": -0.25 if ndim == 3 else 0.0}

    def Bfield(x, y, z):
        return (B0[0] + sl["s1"] * y + sl["s5"] * z, B0[1] + sl["s2"] * x + sl["s6"] * z,
                B0[2] + sl["s3"] * x + sl["s4"] * y)

    X, Y, Z = s.mesh()
    Wl = 1.0 / math.sqrt(1.0 - v @ v)
    prim = [np.full(s.shape, 1.2), np.full(s.shape, Wl * v[0]), np.full(s.shape, Wl * v[1]),
            np.full(s.shape, Wl * v[2]), np.full(s.shape, 0.7)]
    Bc = Bfield(X, Y, Z)
    E = [np.ascontiguousarray(-(v[1] * Bc[2] - v[2] * Bc[1])), np.ascontiguousarray(-(v[2] * Bc[0] - v[0] * Bc[2])),
         np.ascontiguousarray(-(v[0] * Bc[1] - v[1] * Bc[0]))]
    face = []
    for d in range(3):
        pos = [X, Y, Z]
        if s.active(d):
            pos[d] = pos[d] - 0.5 * s.dx(d)
        face.append(np.ascontiguousarray(Bfield(*pos)[d]))
    exact = (-(v[1] * sl["s1"] + v[2] * sl["s5"]), -(v[0] * sl["s2"] + v[2] * sl["s6"]),
             -(v[0] * sl["s3"] + v[1] * sl["s4"]))
    return s, prim, E, face, exact


@pytest.mark.parametrize("ndim", [2, 3])
@pytest.mark.parametrize("recon", [W.MINMOD, W.MC, W.PPM])
def test_linear_field_face_update_exact(ndim, recon):
    """uniform v, linear div-free B, E = -v x B: every reconstruction is exact,
    so the face update rate equals -(v . grad) B to round-off in both UCT
    forms (a swapped velocity component, face or sign breaks it)"""
    out = {}
    for uct in (0, 1):
        s, prim, E, face, exact = _linear_field_setup(ndim, recon, uct)
        g = oracle.grid_of(s)
        Lc = [np.zeros(s.shape) for _ in range(8)]
        Lf = [np.zeros(s.shape) for _ in range(3)]
        oracle.lib().or_explicit_L(ctypes.byref(g), _pp(prim), _pp(E), _pp(face), _p(None), _p(None), _pp(Lc),
                                   _pp(Lf))
        sl = s.interior
        for d in range(3):
            got = Lf[d][sl]
            assert np.abs(got - exact[d]).max() <= 2e-13, (uct, d, np.abs(got - exact[d]).max())
        out[uct] = Lf
    for d in range(3):
        assert np.abs(out[0][d][s.interior] - out[1][d][s.interior]).max() <= 2e-13


@pytest.mark.parametrize("ndim", [1, 2, 3])
def test_ideal_uct_free_stream(ndim):
    n = {1: 12, 2: 8, 3: 6}[ndim]
    s = W._blank(W.Setup("uniform", ndim, (n, n, n), 3, (0, 0, 0), (1, 1, 1), W._bc(ndim, W.PERIODIC), 5.0 / 3.0,
                         W.PPM, W.SSP3, eta=1e-3, uct=1))
    v = np.array([0.3, -0.2, 0.1])
    B = np.array([0.4, 0.7, -0.5])
    Wl = 1 / math.sqrt(1 - v @ v)
    s.prim[0] = 1.3
    s.prim[1:4] = (Wl * v)[:, None, None, None]
    s.prim[4] = 0.6
    s.E[:] = (-np.cross(v, B))[:, None, None, None]
    s.face = np.zeros((3,) + s.shape)
    s.face[:] = B[:, None, None, None]
    st = _run(s, 2)
    for d in range(3):
        assert np.abs(st.face[d][s.interior] - B[d]).max() <= 1e-14
    for vv in range(5):
        ref = s.prim[vv][s.interior]
        assert np.abs(st.prim[vv][s.interior] - ref).max() <= 1e-13 * max(1, np.abs(ref).max())


def test_ideal_uct_div_b_and_periodic_totals():
    s = W.loop_advection(32, 16)
    s.uct = 1
    st = oracle.OracleState(s)
    dt = st.dt()
    tot0 = [st.face[d][s.interior].sum() for d in range(3)]
    for _ in range(30):
        st.step(dt)
    assert st.divB()[2] <= 1e-12
    for d in range(3):
        assert abs(st.face[d][s.interior].sum() - tot0[d]) <= 1e-13 * s.ncells * max(1e-3, abs(tot0[d]))
    for make in (lambda: W.blast_wave(32), lambda: W.tov_star(16)):
        s = make()
        s.uct = 1
        st = _run(s, 2)
        assert st.divB()[2] <= 1e-12
        assert st.nfail == 0


def _smooth_field(n, uct):
    """periodic [0, 1]^2, rho = p = 1, uniform v = (0.3, 0.15), weak smooth
    field from A_z = A0 sin(2 pi x) sin(2 pi y) / (2 pi), E = -v x B, eta =
    1e-6 (the ideal limit)"""
    s = W._blank(W.Setup("smooth_field", 2, (n, n, 1), 2, (0, 0, 0), (1, 1, 1), W._bc(2, W.PERIODIC), 4.0 / 3.0,
                         W.MC, W.SSP2, eta=1e-6, rho_atm=1e-12, p_atm=1e-14, uct=uct))
    A0 = 1e-2
    vx, vy = 0.3, 0.15
    Wl = 1.0 / math.sqrt(1 - vx * vx - vy * vy)
    s.prim[0] = 1.0
    s.prim[1] = Wl * vx
    s.prim[2] = Wl * vy
    s.prim[4] = 1.0
    X, Y, _ = s.mesh()
    k = 2 * math.pi
    Bx = A0 * np.sin(k * X) * np.cos(k * Y)
    By = -A0 * np.cos(k * X) * np.sin(k * Y)
    s.E[2] = -(vx * By - vy * Bx)
    s.A = np.zeros((3,) + s.edge_shape)
    Xe, Ye, _ = s.edge_mesh(2)
    s.A[2] = A0 * np.sin(k * Xe) * np.sin(k * Ye) / k
    return s


def test_ideal_limit_agrees_with_resistive_uct():
    """at eta = 1e-6 the two edge EMFs are two discretisations of the same
    ideal induction equation: their difference after t = 0.25 shrinks with
    resolution (observed rate >= 1.5)"""
    diffs = []
    for n in (16, 32, 64):
        res = {}
        for uct in (0, 1):
            s = _smooth_field(n, uct)
            st = oracle.OracleState(s)
            dt = st.dt()
            nst = int(round(0.25 / dt))
            dt = 0.25 / nst
            for _ in range(nst):
                st.step(dt)
            assert st.nfail == 0
            res[uct] = np.stack([st.face[d][s.interior] for d in range(2)])
        scale = np.abs(res[0]).mean()
        diffs.append(np.abs(res[1] - res[0]).mean() / scale)
    rates = [math.log2(diffs[i] / diffs[i + 1]) for i in range(2)]
    assert min(rates) >= 1.5, (diffs, rates)
    assert diffs[-1] <= 1e-2


def test_ideal_uct_blast_wave_mirror_symmetry():
    """the left and right transport velocities enter the edge EMF
    symmetrically: the blast wave, given a radial outflow so that the
    reconstructed velocities differ across every face, keeps its mirror
    symmetry in x and in y (pressure and density compared)"""
    s = W.blast_wave(32)
    s.uct = 1
    X, Y, _ = s.mesh()
    r2 = X ** 2 + Y ** 2
    s.prim[1] = 0.4 * X * np.exp(-r2)
    s.prim[2] = 0.4 * Y * np.exp(-r2)
    st = _run(s, 4)
    p = st.prim[4][s.interior][0]
    rho = st.prim[0][s.interior][0]
    assert np.abs(p - p[:, ::-1]).max() <= 1e-13 * p.max()
    assert np.abs(p - p[::-1, :]).max() <= 1e-13 * p.max()
    assert np.abs(rho - rho[:, ::-1]).max() <= 1e-13 * rho.max()
    assert st.nfail == 0


def test_ideal_uct_1d_normal_field_bit_constant():
    s = W.shock_tube(64)
    s.uct = 1
    st = _run(s, 20)
    assert np.all(st.face[0][s.interior] == 0.5)
    assert st.nfail == 0
