"""Pins of the oracle's spatial operator, constrained transport and whole
step (no GPU): invariants, symmetries, closed forms and the paper's tables."""
import ctypes
import math

import numpy as np
import pytest

import oracle
import workloads as W
from oracle import _p, _pp


def run(s, steps, dt=None):
    st = oracle.OracleState(s)
    dt = st.dt() if dt is None else dt
    for _ in range(steps):
        st.step(dt)
    return st


def interior(s, a):
    return a[s.interior]


# --------------------------------------------------------------------------
@pytest.mark.parametrize("ndim", [1, 2, 3])
@pytest.mark.parametrize("recon,imex", [(W.MC, W.SSP2), (W.PPM, W.SSP3)])
def test_free_stream(ndim, recon, imex):
    """a uniform state with E = -v x B is an exact steady solution"""
    n = {1: 12, 2: 8, 3: 6}[ndim]
    s = W._blank(W.Setup("uniform", ndim, (n, n, n), 3 if recon == W.PPM else 2, (0, 0, 0), (1, 1, 1),
                         W._bc(ndim, W.PERIODIC), 5.0 / 3.0, recon, imex, eta=1e-3))
    v = np.array([0.3, -0.2, 0.1])
    B = np.array([0.4, 0.7, -0.5])
    Wl = 1 / math.sqrt(1 - v @ v)
    s.prim[0] = 1.3
    s.prim[1:4] = (Wl * v)[:, None, None, None]
    s.prim[4] = 0.6
    s.E[:] = (-np.cross(v, B))[:, None, None, None]
    s.face = np.zeros((3,) + s.shape)
    s.face[:] = B[:, None, None, None]
    st = run(s, 2)
    for vv in range(5):
        ref = s.prim[vv][s.interior]
        assert np.abs(interior(s, st.prim[vv]) - ref).max() <= 1e-13 * max(1, np.abs(ref).max())
    for d in range(3):
        assert np.abs(interior(s, st.face[d]) - B[d]).max() <= 1e-14
    assert st.nfail == 0


def _embed(s1, ndim, axis, ntrans=4):
    """embed a 1-D x problem along `axis` of a periodic ndim grid, rotating
    vector components cyclically (x -> axis)"""
    n = s1.n[0]
    shape_n = [ntrans, ntrans, ntrans]
    shape_n[axis] = n
    lo = [0.0, 0.0, 0.0]
    hi = [1.0, 1.0, 1.0]
    lo[axis], hi[axis] = s1.lo[0], s1.hi[0]
    bc = [(W.PERIODIC, W.PERIODIC)] * 3
    bc[axis] = s1.bc[0]
    s = W._blank(W.Setup("embed", ndim, tuple(shape_n), s1.ng, tuple(lo), tuple(hi), tuple(bc), s1.gamma_ad,
                         s1.recon, s1.imex, eta=s1.eta, rho_atm=s1.rho_atm, p_atm=s1.p_atm))
    perm = [(axis + c) % 3 for c in range(3)]  # old component c -> new component perm[c]

    def spread(a1):
        line = a1[0, 0, :]  # along x in the 1-D setup
        out = np.zeros(s.shape)
        idx = [None, None, None]
        idx[2 - axis] = slice(None)
        sh = [1, 1, 1]
        sh[2 - axis] = len(line)
        out[...] = line.reshape(sh)
        return out

    s.prim[0] = spread(s1.prim[0])
    s.prim[4] = spread(s1.prim[4])
    s.face = np.zeros((3,) + s.shape)
    for c in range(3):
        s.prim[1 + perm[c]] = spread(s1.prim[1 + c])
        s.E[perm[c]] = spread(s1.E[c])
        s.face[perm[c]] = spread(s1.face[c])
    return s, perm


@pytest.mark.parametrize("ndim,axis", [(2, 0), (2, 1), (3, 0), (3, 1), (3, 2)])
def test_direction_consistency(ndim, axis):
    """the 1-D shock tube embedded along any axis of a 2-D / 3-D grid (vector
    components rotated cyclically) evolves exactly like the 1-D run: this pins
    every directional code path, the upwind EMF's reduction to the 1-D HLL
    flux of B, and the CT update"""
    if ndim == 2 and axis == 2:
        pytest.skip()
    s1 = W.shock_tube(48)
    st1 = run(s1, 6)
    s, perm = _embed(W.shock_tube(48), ndim, axis)
    st = run(s, 6, dt=oracle.OracleState(s1).dt())
    line1 = {v: interior(s1, st1.prim[v])[0, 0, :] for v in range(5)}
    for v, vn in [(0, 0), (4, 4)] + [(1 + c, 1 + perm[c]) for c in range(3)]:
        a = interior(s, st.prim[vn])
        a = np.moveaxis(a, 2 - axis, -1)
        assert np.abs(a - line1[v]).max() <= 1e-13, (v, np.abs(a - line1[v]).max())
    for c in range(3):
        ref = interior(s1, st1.face[c])[0, 0, :]
        a = np.moveaxis(interior(s, st.face[perm[c]]), 2 - axis, -1)
        assert np.abs(a - ref).max() <= 1e-13


def test_shock_tube_normal_field_bit_constant():
    s = W.shock_tube(64)
    st = run(s, 20)
    assert np.all(interior(s, st.face[0]) == 0.5)


def test_blast_wave_mirror_symmetry():
    s = W.blast_wave(32, steps=4)
    st = run(s, 4)
    p = interior(s, st.prim[4])[0]
    rho = interior(s, st.prim[0])[0]
    assert np.abs(p - p[:, ::-1]).max() <= 1e-13
    assert np.abs(p - p[::-1, :]).max() <= 1e-13
    assert np.abs(rho - rho[:, ::-1]).max() <= 1e-13 * rho.max()
    assert st.nfail == 0


def test_ct_keeps_div_b_and_periodic_totals():
    """loop advection, periodic: discrete div B stays at round-off and the
    totals of q_D, q_S, q_tau and of every face field are conserved"""
    s = W.loop_advection(32, 16)
    st = oracle.OracleState(s)
    dt = st.dt()
    d0 = st.divB()
    tot0 = [interior(s, a).sum() for a in st.q[:5] + st.face]
    for _ in range(100):
        st.step(dt)
    d1 = st.divB()
    assert d0[2] <= 1e-12 and d1[2] <= 1e-12
    tot1 = [interior(s, a).sum() for a in st.q[:5] + st.face]
    scale = [max(abs(t), 1.0) for t in tot0]
    for a, b, sc in zip(tot0, tot1, scale):
        assert abs(a - b) <= 1e-13 * sc * s.ncells
    assert st.nfail == 0


def test_star_div_b_round_off():
    s = W.tov_star(16)
    st = run(s, 2)
    assert st.divB()[2] <= 1e-12
    assert st.nfail == 0


# --------------------------------------------------------------------------
@pytest.mark.parametrize("uct,frozen", [(0, 0), (1, 0), (0, 1)])
def test_constant_metric_is_a_rescaled_flat_run(uct, frozen):
    """constant lapse alpha and conformal factor psi: the conformally flat run
    equals a flat run on a domain psi^2 larger with time step alpha dt and
    orthonormal components psi^2 (u~, E, B) (face field q_B = psi^4 B_flat);
    for the resistive (Sec 3.2) and the ideal-MHD (App. A) edge EMFs, and
    with the matter frozen (E from eq. im_E at the fixed velocity).  The
    electric field has a divergence, so the Gauss-law charge current is
    exercised as well"""
    alpha, psi = 0.8, 1.1
    sA = W.blast_wave(16, recon=W.MC, imex=W.SSP2, steps=3)
    sA.uct = uct
    sA.frozen_matter = frozen
    sA.eta = 1e-2
    sA.metric = 1
    sA.alpha = np.full(sA.shape, alpha)
    sA.psi = np.full(sA.shape, psi)
    # give it velocity and electric field so that every term is exercised
    X, Y, _ = sA.mesh()
    sA.prim[1] = 0.3 * np.exp(-(X ** 2 + Y ** 2))
    sA.prim[2] = -0.2 * np.exp(-(X ** 2 + Y ** 2))
    sA.E[2] = 0.05 * np.exp(-(X ** 2 + Y ** 2))
    sA.E[0] = 0.04 * np.exp(-((X - 0.5) ** 2 + Y ** 2))
    stA = oracle.OracleState(sA)
    dtA = 0.02
    sB = W.blast_wave(16, recon=W.MC, imex=W.SSP2, steps=3)
    sB.uct = uct
    sB.frozen_matter = frozen
    sB.eta = 1e-2
    sB.lo = (-6 * psi ** 2, -6 * psi ** 2, 0)
    sB.hi = (6 * psi ** 2, 6 * psi ** 2, 1)
    sB.prim = sA.prim.copy()
    sB.prim[1:4] *= psi ** 2
    sB.E = sA.E * psi ** 2
    sB.A = None
    sB.face = np.stack(stA.face) / psi ** 4
    stB = oracle.OracleState(sB)
    for _ in range(3):
        stA.step(dtA)
        stB.step(alpha * dtA)
    sl = sA.interior
    for v in (0, 4):
        a, b = stA.prim[v][sl], stB.prim[v][sl]
        assert np.abs(a - b).max() <= 1e-12 * np.abs(b).max()
    for v in (1, 2, 3):
        a, b = stA.prim[v][sl] * psi ** 2, stB.prim[v][sl]
        assert np.abs(a - b).max() <= 1e-12 * max(1e-3, np.abs(b).max())
    EA, EB = stA.E(), stB.E()
    assert np.abs(EA[:, sl[0], sl[1], sl[2]] * psi ** 2 - EB[:, sl[0], sl[1], sl[2]]).max() <= 1e-12
    for d in range(3):
        assert np.abs(stA.face[d][sl] / psi ** 4 - stB.face[d][sl]).max() <= 1e-12


def _explicit_L(s, faces=False):
    st = oracle.OracleState(s)
    cells = [st.prim[v] for v in range(5)] + [np.ascontiguousarray(st.q[5 + v] / s.psi ** 6) for v in range(3)]
    oracle.lib().or_ghost_fill(ctypes.byref(st.grid), _pp(cells), 8, _pp(st.face))
    Lc = [np.zeros(s.shape) for _ in range(8)]
    Lf = [np.zeros(s.shape) for _ in range(3)]
    oracle.lib().or_explicit_L(ctypes.byref(st.grid), _pp(cells[:5]), _pp(cells[5:]), _pp(st.face), _p(st.alpha),
                               _p(st.psi), _pp(Lc), _pp(Lf))
    return (Lc, Lf) if faces else Lc


@pytest.mark.parametrize("side", ["a", "b"])
def test_edge_speed_is_that_of_the_faster_face(side):
    """Sec 3.2 (vi): an edge's speed in each direction is the larger of the
    speeds of the two faces of that direction beside it.  A fluid at rest with
    E = 0 and a face field that jumps across the other direction, in a lapse
    growing across it (side a: q_B^y jumping across x = 0, lapse growing in
    y; side b: q_B^x jumping across y = 0, lapse growing in x): the EMF of a
    z-edge is then one dissipation term alone, so the face update of that
    field along each row (column) of faces equals, bit for bit, that of a
    constant lapse equal to the lapse of the cell above (to the right), the
    faster face"""
    n = 12
    d, t = (1, 0) if side == "a" else (0, 1)  # field direction, jump direction

    def setup(alpha_of):
        s = W.density_wave(n, ndim=2, amp=0.0, v=0.0)
        s.bc = ((W.OUTFLOW, W.OUTFLOW),) * 3
        s.lo, s.hi = (-1.0, -1.0, 0.0), (1.0, 1.0, 1.0)
        M = s.mesh()
        s.metric = 1
        s.alpha = alpha_of(M[d])
        s.psi = np.ones(s.shape)
        s.prim[0], s.prim[4] = 1.0, 0.1
        for i in range(3):
            s.E[i] = 0.0
        s.A = None
        s.face = np.zeros((3,) + s.shape)
        s.face[d] = np.where(M[t] > 0.0, 0.1, -0.1)  # a function of the other coordinate only
        return s

    def lapse(x):
        return 1.0 + 0.15 * (x + 1.0)

    s = setup(lapse)
    _, Lf = _explicit_L(s, faces=True)
    g = s.g(d)
    xc = s.mesh()[d][0, :, :]
    changed = 0
    for j in range(g + 1, g + n):  # faces between cells j - 1 and j along d
        up = lapse(xc[j, g] if d == 1 else xc[g, j])
        _, Lf_c = _explicit_L(setup(lambda x: np.full(x.shape, up)), faces=True)
        if d == 1:
            mine, ref = Lf[1][:, j, g:g + n], Lf_c[1][:, j, g:g + n]
        else:
            mine, ref = Lf[0][:, g:g + n, j], Lf_c[0][:, g:g + n, j]
        assert np.array_equal(mine, ref), j
        changed += int(np.abs(mine).max() > 0.0)
    assert changed == n - 1


def test_tov_hydrostatic_residual_converges():
    """Cowling star at t=0: the gravity sources (Sec 2.1, beta = 0, K = 0)
    balance the pressure gradient, so L(q) in the interior is truncation error
    that shrinks with resolution; a dropped or mis-signed source term leaves
    an O(1) residual"""
    res = []
    for n in (24, 48):
        s = W.tov_star(n, b_max=0.0)
        Lc = _explicit_L(s)
        X, Y, Z = s.mesh()
        r = np.sqrt(X ** 2 + Y ** 2 + Z ** 2)
        m = r < 4.0
        LS = np.sqrt(Lc[1] ** 2 + Lc[2] ** 2 + Lc[3] ** 2)
        res.append(LS[m].mean())
    rate = math.log2(res[0] / res[1])
    assert rate >= 1.3, res
    assert res[1] < 5e-6


def test_uniform_pressure_in_a_conformal_factor_is_an_equilibrium():
    """a uniform fluid at rest in a conformally flat metric with unit lapse
    and psi linear in x: the divergence of the momentum flux psi^6 p equals
    the metric source (1/2) sqrt(gamma) S^jk d_x gamma_jk = 6 psi^5 p d_x psi
    (Sec 2.1), so L vanishes up to truncation error, which falls at second
    order (faces take the mean of the two cells' psi)"""
    res = []
    for n in (32, 64, 128):
        s = W.density_wave(n, ndim=1, amp=0.0, v=0.0)
        s.bc = ((W.OUTFLOW, W.OUTFLOW),) * 3
        s.lo, s.hi = (-1.0, 0.0, 0.0), (1.0, 1.0, 1.0)
        X = s.mesh()[0]
        s.metric = 1
        s.alpha = np.ones(s.shape)
        s.psi = 1.0 + 0.2 * X
        s.prim[0], s.prim[4] = 1.0, 0.1
        for i in range(3):
            s.E[i] = 0.0
        s.A = None
        s.face = np.zeros((3,) + s.shape)
        Lc = _explicit_L(s)
        res.append(np.abs(Lc[1][s.interior]).max())
    rates = [math.log2(res[i] / res[i + 1]) for i in range(2)]
    assert min(rates) >= 1.8, (res, rates)
    assert res[-1] < 1e-5, res


# --------------------------------------------------------------------------
# smooth-wave convergence and the paper's convergence tables
def test_density_wave_second_order():
    errs = []
    for n in (32, 64, 128):
        s = W.density_wave(n, ndim=1)
        st = oracle.OracleState(s)
        dt = st.dt()
        nst = int(round(0.5 / dt))
        dt = 0.5 / nst
        for _ in range(nst):
            st.step(dt)
        errs.append(np.abs(interior(s, st.prim[0]) - interior(s, W.density_wave_exact(s, 0.5))).mean())
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(rates) >= 1.9, rates


def test_telegraph_period_closed_form(golden):
    assert W.telegraph_params()["T"] == pytest.approx(golden["telegraph"]["T"], rel=1e-15)


def test_telegraph_matches_paper_table(golden):
    T = golden["telegraph"]["T"]
    tab = dict(zip(golden["telegraph"]["N"], golden["telegraph"]["L1"]))
    errs = {}
    for n in (32, 64):
        s = W.telegraph(n)
        st = oracle.OracleState(s)
        dt = st.dt()
        nst = int(math.ceil(T / dt - 1e-12))
        dt = T / nst
        for _ in range(nst):
            st.step(dt)
        X, Y, _ = s.mesh()
        Bz, _, _ = W.telegraph_fields(X, Y, T)
        errs[n] = np.abs(interior(s, st.face[2]) - interior(s, Bz)).mean()
        assert st.nfail == 0
        assert errs[n] == pytest.approx(tab[n], rel=0.15)
    assert 1.5 <= math.log2(errs[32] / errs[64]) <= 2.3


def _cs_run(n):
    s = W.current_sheet(n)
    st = oracle.OracleState(s)
    dt = st.dt()
    nst = int(math.ceil(9.0 / dt - 1e-9))
    dt = 9.0 / nst
    for _ in range(nst):
        st.step(dt)
    return interior(s, st.face[1]).ravel()


@pytest.mark.slow
def test_current_sheet_matches_paper_table(golden):
    """delta_N of B^y at t=10 against a finer run (N=512 here, 8192 in the
    paper, whose own error is below 4% of delta_128), MC + HLL + SSP2"""
    tab = dict(zip(golden["current_sheet"]["N"], golden["current_sheet"]["delta"]))
    tab[64] = 1.646e-3  # printed 1.646E-4: a typo (see the golden file)
    ref = _cs_run(512)
    d = {}
    for n in (64, 128):
        by = _cs_run(n)
        refc = ref.reshape(n, 512 // n).mean(1)
        d[n] = np.abs(by - refc).sum() / n / by.max()
        assert d[n] == pytest.approx(tab[n], rel=0.2), (n, d[n])
    assert 2.2 <= math.log2(d[64] / d[128]) <= 3.0


def test_current_sheet_tracks_erf():
    """the erf profile (exact for p -> infinity) is followed closely at p = 5000"""
    s = W.current_sheet(128)
    st = oracle.OracleState(s)
    dt = st.dt()
    nst = int(math.ceil(1.0 / dt - 1e-9))
    for _ in range(nst):
        st.step(1.0 / nst)
    X, _, _ = s.mesh()
    ex = W.current_sheet_exact(interior(s, X).ravel(), 2.0)
    assert np.abs(interior(s, st.face[1]).ravel() - ex).mean() < 1e-3


@pytest.mark.parametrize("n,rel", [(32, 0.15), (64, 0.25)])
def test_charged_vortex_matches_paper_table(golden, n, rel):
    """pins the non-stiff current rho_e v (Gauss-law charge) and fixed boundaries"""
    tab = dict(zip(golden["charged_vortex"]["N"], golden["charged_vortex"]["L1"]))
    s = W.charged_vortex(n)
    st = oracle.OracleState(s)
    dt = st.dt()
    nst = int(math.ceil(10.0 / dt - 1e-12))
    dt = 10.0 / nst
    bz0 = st.face[2].copy()
    for _ in range(nst):
        st.step(dt)
    err = np.abs(interior(s, st.face[2]) - interior(s, bz0)).mean()
    assert err == pytest.approx(tab[n], rel=rel)
    assert st.nfail == 0


def test_gauss_charge_current_closed_form():
    """non-stiff current (Sec 2.4 split, Gauss-law charge of Sec 2.1): a heavy
    fluid moving along y through a charge density rho_e = d_x E^x (eta large,
    B = 0) drives dE^y/dt = -rho_e v^y at t = 0"""
    n = 64
    s = W._blank(W.Setup("charge", 1, (n, 1, 1), 2, (0, 0, 0), (1, 1, 1), W._bc(1, W.PERIODIC), 4.0 / 3.0, W.MC,
                         W.SSP2, eta=1e12))
    X, _, _ = s.mesh()
    vy = 0.1
    Wl = 1 / math.sqrt(1 - vy * vy)
    s.prim[0] = 1e12
    s.prim[2] = Wl * vy
    s.prim[4] = 1.0
    s.E[0] = 0.01 * np.sin(2 * math.pi * X)
    st = oracle.OracleState(s)
    dt = 1e-4
    E0 = st.E()
    st.step(dt)
    dEy = (st.E()[1] - E0[1])[s.interior] / dt
    rho_e = 0.01 * 2 * math.pi * np.cos(2 * math.pi * X)[s.interior]
    expect = -rho_e * vy
    # central-difference charge: relative error (2 pi dx)^2/6 ~ 2e-3
    assert np.abs(dEy - expect).max() <= 5e-3 * np.abs(expect).max()


def test_killing_energy_in_static_lapse():
    """static metric: alpha psi^6 (tau + D) obeys a conservation law (time-like
    Killing vector), which the tau source -psi^6 S^j d_j alpha (Sec 2.1 with
    beta = 0, K = 0) makes hold up to truncation error; without it the energy
    drifts at O(rho v d alpha)"""
    drift = []
    for n in (32, 64):
        s = W.density_wave(n, ndim=1, amp=0.0, v=0.3)
        s.metric = 1
        X, _, _ = s.mesh()
        s.alpha = 1.0 + 0.1 * np.sin(2 * math.pi * X)
        s.psi = np.ones(s.shape)
        st = oracle.OracleState(s)
        e0 = (s.alpha * (st.q[4] + st.q[0]))[s.interior].sum() / n
        dt = 0.4 / n
        for _ in range(int(round(0.1 / dt))):
            st.step(dt)
        e1 = (s.alpha * (st.q[4] + st.q[0]))[s.interior].sum() / n
        drift.append(abs(e1 - e0) / e0)
    assert drift[1] < drift[0] / 3
    assert drift[1] < 1e-5, drift


def test_div_b_norms_of_a_known_divergence():
    """face field q_B^x = x^2 + y, q_B^y = x y^2 on a 2-D grid: the face
    difference of a quadratic is its derivative at the cell centre, so the
    discrete divergence there is exactly 2x + 2xy; the three norms are the
    mean of its magnitude, the root mean square and the maximum over the
    interior cells"""
    s = W.density_wave(10, ndim=2, amp=0.0, v=0.0)
    s.lo, s.hi = (-1.0, -0.5, 0.0), (1.0, 1.5, 1.0)
    st = oracle.OracleState(s)
    X, Y, _ = s.mesh()
    hx, hy = s.dx(0), s.dx(1)
    st.face[0][...] = (X - 0.5 * hx) ** 2 + Y
    st.face[1][...] = X * (Y - 0.5 * hy) ** 2
    st.face[2][...] = 0.0
    sl = s.interior
    div = (2.0 * X + 2.0 * X * Y)[sl]
    got = st.divB()
    assert got[0] == pytest.approx(np.abs(div).mean(), rel=1e-12)
    assert got[1] == pytest.approx(math.sqrt((div ** 2).mean()), rel=1e-12)
    assert got[2] == pytest.approx(np.abs(div).max(), rel=1e-12)
