"""Pins of the oracle's rules that the paper states only in words or not at
all (no GPU): the conductivity of eq. sigma_D (Sec 5.11), the atmosphere and
failure fallback (Sec 2.4, last paragraph; reading R18), the ghost rules
(reading R17), the time step (Sec 2.5; reading R16) and the PPM
monotonicity constraints (reading R10).

Every expected value here comes from the stated rule evaluated by hand in
the test, or from a property that holds for the rule whatever its code:
a uniform cell at rest relaxes exactly as y' = -alpha y / eta under the
tableau (so the eta that the oracle used is read off the decay), ghost
points are copies of named interior points, the time step of a constant
metric equals a flat step on a rescaled grid, and a limited PPM parabola is
monotone and keeps the cell mean.
"""
import ctypes
import math

import numpy as np
import pytest

import oracle
import workloads as W


def _R(imex, z):
    _, A, _, w = oracle.tableau(imex)
    s = len(w)
    return 1 + z * w @ np.linalg.solve(np.eye(s) - z * A, np.ones(s))


def _uniform(ndim=1, rho=1.0, p=0.1, E=(0.3, -0.2, 0.1), alpha=1.0, psi=1.0, imex=W.SSP2):
    """uniform periodic box at rest, B = 0 (the spatial operator vanishes)"""
    s = W.density_wave(8, ndim=ndim, amp=0.0, v=0.0, imex=imex)
    s.prim[0] = rho
    s.prim[4] = p
    for i in range(3):
        s.E[i] = E[i]
    if alpha != 1.0 or psi != 1.0:
        s.metric = 1
        s.alpha = np.full(s.shape, alpha)
        s.psi = np.full(s.shape, psi)
    return s


# --------------------------------------------------------------------------
# eq. sigma_D: sigma_c = sigma_0 max(1 - D_atmo/D, 0)^2, eta = 1/sigma_c kept in
# [eta_min, eta_max]; D is the undensitised D = q_D / psi^6, D_atmo the
# atmosphere threshold atm_factor rho_atm (reading R23b)
def _eta_by_hand(D, sigma0, D_atmo, eta_min, eta_max):
    x = max(1.0 - D_atmo / D, 0.0)
    sig = sigma0 * x * x
    eta = math.inf if sig == 0.0 else 1.0 / sig
    return min(max(eta, eta_min), eta_max)


# (rho, sigma0): inside the clamp, at eta_max (sigma -> 0 near the
# threshold), at eta_min (large sigma_0)
ETA_CASES = [(1e-3, 1e6), (2e-6, 1e6), (4e-6, 1e6), (1.0000001e-6, 1e6), (1e-2, 1e8)]


@pytest.mark.parametrize("imex", [W.SSP2, W.SSP3])
@pytest.mark.parametrize("rho,sigma0", ETA_CASES)
def test_eta_of_D_from_relaxation(imex, rho, sigma0):
    """a cell at rest relaxes E by R(-alpha dt/eta)^n with eta from eq.
    sigma_D evaluated here; a constant metric psi = 1.2 makes q_D = psi^6 D
    differ from D, so the undensitised D is pinned"""
    alpha, psi = 0.8, 1.2
    rho_atm, atm_factor, eta_min, eta_max = 1e-10, 1e4, 1e-6, 1.0
    eta = _eta_by_hand(rho, sigma0, rho_atm * atm_factor, eta_min, eta_max)
    s = _uniform(rho=rho, p=0.1 * rho, alpha=alpha, psi=psi, imex=imex,
                 E=(0.3 * rho, -0.2 * rho, 0.1 * rho))
    s.eta_mode, s.sigma0, s.eta_min, s.eta_max = 1, sigma0, eta_min, eta_max
    s.rho_atm, s.atm_factor, s.p_atm = rho_atm, atm_factor, 1e-18
    dt = 0.7 * eta / alpha  # alpha dt / eta of order one: R is far from 0 and 1
    st = oracle.OracleState(s)
    sl = s.interior
    E0 = st.E()[:, sl[0], sl[1], sl[2]].copy()
    R = _R(imex, -alpha * dt / eta)
    for n in range(1, 4):
        st.step(dt)
        E = st.E()[:, sl[0], sl[1], sl[2]]
        assert np.abs(E - R ** n * E0).max() <= 1e-12 * np.abs(E0).max(), (n, eta)
    assert st.nfail == 0


def test_eta_max_below_threshold():
    """sigma_c = 0 at and below D_atmo: eta = eta_max there (uniform eta_mode 1
    cells just above the atmosphere threshold relax with eta_max)"""
    rho_atm, atm_factor = 1e-10, 1e4
    D = rho_atm * atm_factor * 1.0000000001  # sigma_0 x^2 ~ 1e-14: far below 1/eta_max
    assert _eta_by_hand(D, 1e6, rho_atm * atm_factor, 1e-6, 1.0) == 1.0
    s = _uniform(rho=D, p=1e-3 * D, E=(1e-7, 0.0, 0.0))
    s.eta_mode, s.sigma0, s.eta_min, s.eta_max = 1, 1e6, 1e-6, 1.0
    s.rho_atm, s.atm_factor, s.p_atm = rho_atm, atm_factor, 1e-20
    st = oracle.OracleState(s)
    dt = 0.3
    st.step(dt)
    sl = s.interior
    assert np.allclose(st.E()[0][sl], _R(W.SSP2, -dt / 1.0) * 1e-7, rtol=1e-12, atol=0)


# --------------------------------------------------------------------------
# atmosphere and failure fallback (reading R18): rho_atm, u~ = 0, p_atm; the
# electric field of a cell at rest, E = E*/(1 + alpha a_ii dt / eta) (the
# v = 0 solution of eq. im_E); failures are counted, atmosphere cells are not;
# the final recovery rewrites q_D, q_S, q_tau from the fallback state
@pytest.mark.parametrize("kind", ["atmosphere", "failure"])
@pytest.mark.parametrize("metric", [(1.0, 1.0), (0.8, 1.2)])
def test_fallback_state_field_and_count(kind, metric):
    alpha, psi = metric
    eta, dt, gam = 0.02, 0.01, 5.0 / 3.0
    E0 = np.array([0.3, -0.2, 0.1])
    s = _uniform(rho=1.0, p=0.1, E=E0, alpha=alpha, psi=psi)
    s.eta, s.rho_atm, s.p_atm, s.atm_factor = eta, 1e-6, 1e-9, 1.001
    if kind == "atmosphere":
        s.prim[0] = 0.9e-6  # below atm_factor rho_atm
        s.prim[4] = 1e-9
    st = oracle.OracleState(s)
    sl = s.interior
    if kind == "failure":
        st.q[4][sl] = -0.1 * psi ** 6  # tau < 0: no root
    n = s.ncells
    stage, _ = st.step(dt, dump_stage=0)
    _, A, _, _ = oracle.tableau(W.SSP2)
    # stage 0 of IMEX-SSP2 is implicit only: E* = E^n
    want_E = E0 / (1.0 + alpha * A[0, 0] * dt / eta)
    for i in range(3):
        assert np.allclose(stage[5 + i][sl], want_E[i], rtol=1e-14, atol=0)
    assert np.all(stage[0][sl] == s.rho_atm) and np.all(stage[4][sl] == s.p_atm)
    assert np.all(stage[1][sl] == 0.0) and np.all(stage[2][sl] == 0.0) and np.all(stage[3][sl] == 0.0)
    # counted: both implicit stages and the final recovery of every cell
    assert st.nfail == (3 * n if kind == "failure" else 0)
    # final recovery: the state is the fallback one, its q_D, q_S, q_tau
    # rewritten from it with the evolved E (B = 0)
    assert np.all(st.prim[0][sl] == s.rho_atm) and np.all(st.prim[4][sl] == s.p_atm)
    E = st.E()[:, sl[0], sl[1], sl[2]]
    g4 = psi ** 4
    U = 0.5 * g4 * (E ** 2).sum(0)
    ps6 = psi ** 6
    h = 1.0 + gam / (gam - 1.0) * s.p_atm / s.rho_atm
    assert np.allclose(st.q[0][sl], ps6 * s.rho_atm, rtol=1e-14, atol=0)
    assert np.allclose(st.q[4][sl] / ps6, s.rho_atm * h - s.p_atm - s.rho_atm + U, rtol=1e-12, atol=0)
    for i in range(3):
        assert np.all(st.q[1 + i][sl] == 0.0)  # E x B = 0 with B = 0


@pytest.mark.parametrize("metric", [(1.0, 1.0), (0.8, 1.2)])
def test_fallback_field_with_the_dynamo_term(metric):
    """the field of an atmosphere cell with the mean-field dynamo term
    (xi != 0, B != 0) is the v = 0 solution of eq. im_E: the general
    solve of eq. im_E (pinned against a direct 3x3 solve) at u~ = 0"""
    alpha, psi = metric
    eta, dt, xi = 0.02, 0.01, 0.3
    E0 = np.array([0.3, -0.2, 0.1])
    B0 = np.array([0.1, 0.05, -0.2])
    s = _uniform(rho=0.9e-6, p=1e-9, E=E0, alpha=alpha, psi=psi)
    s.eta, s.rho_atm, s.p_atm, s.atm_factor, s.xi = eta, 1e-6, 1e-9, 1.001, xi
    s.A = None
    s.face = np.stack([np.full(s.shape, psi ** 6 * B0[d]) for d in range(3)])
    st = oracle.OracleState(s)
    sl = s.interior
    stage, _ = st.step(dt, dump_stage=0)
    _, A, _, _ = oracle.tableau(W.SSP2)
    want = oracle.implicit_E(psi, eta / (alpha * A[0, 0] * dt), xi, np.zeros(3), E0, B0)
    assert np.abs(want - E0).max() > 1e-3  # the dynamo term and the relaxation both act
    for i in range(3):
        assert np.allclose(stage[5 + i][sl], want[i], rtol=1e-13, atol=1e-15)
    assert np.all(stage[0][sl] == s.rho_atm) and st.nfail == 0


def test_final_recovery_rewrites_conserved_variables():
    """or_c2p_grid (recovery with E and B known): a tau < 0 cell and a cell
    below the threshold get the fallback primitives and q_D, q_S, q_tau of the
    fallback state with their own E and B; only the first is counted"""
    s = W.random_states((6, 5, 4), seed=13)
    st = oracle.OracleState(s)
    g = s.ng
    bad, atm = (g + 1, g + 2, g + 3), (g + 4, g + 1, g + 2)  # (i, j, k)
    st.q[4][bad[2], bad[1], bad[0]] = -1.0
    st.q[0][atm[2], atm[1], atm[0]] = 0.5 * s.rho_atm
    nf = oracle.lib().or_c2p_grid(ctypes.byref(st.grid), oracle._pp(st.q), oracle._pp(st.face),
                                  oracle._pp(st.prim), None)
    assert nf == 1
    for (i, j, k) in (bad, atm):
        pr = np.array([st.prim[v][k, j, i] for v in range(5)])
        assert pr[0] == s.rho_atm and pr[4] == s.p_atm and np.all(pr[1:4] == 0.0)
        E = np.array([st.q[5 + v][k, j, i] for v in range(3)])
        B = np.array([0.5 * (st.face[0][k, j, i] + st.face[0][k, j, i + 1]),
                      0.5 * (st.face[1][k, j, i] + st.face[1][k, j + 1, i]),
                      0.5 * (st.face[2][k, j, i] + st.face[2][k + 1, j, i])])
        # flat metric: S = E x B, tau = rho h W^2 - p + (E^2 + B^2)/2 - D at rest
        h = 1.0 + s.gamma_ad / (s.gamma_ad - 1.0) * s.p_atm / s.rho_atm
        want = [s.rho_atm, *np.cross(E, B), s.rho_atm * h - s.p_atm + 0.5 * (E @ E + B @ B) - s.rho_atm]
        got = [st.q[v][k, j, i] for v in range(5)]
        assert np.allclose(got, want, rtol=1e-13, atol=1e-15)


# --------------------------------------------------------------------------
# ghost rules (reading R17): outflow = copy of the nearest interior point,
# periodic = the image, fixed = untouched; the normal face array d keeps its
# evolved faces g .. g + n and its ghosts copy the nearest evolved face
def _pad(a, g, mode):
    return np.pad(a, g, mode="edge" if mode == W.OUTFLOW else "wrap")


@pytest.mark.parametrize("bc", [W.OUTFLOW, W.PERIODIC])
@pytest.mark.parametrize("shape", [(7, 1, 1), (6, 5, 1), (5, 4, 3)])
def test_ghost_fill_rules(bc, shape):
    ndim = sum(1 for n in shape if n > 1) if shape != (7, 1, 1) else 1
    g = 3
    s = W._blank(W.Setup("ghosts", ndim, shape, g, (0, 0, 0), (1, 1, 1), W._bc(ndim, bc), 5 / 3, W.PPM, W.SSP2))
    rng = np.random.default_rng(3)
    cells = [np.ascontiguousarray(rng.normal(size=s.shape)) for _ in range(8)]
    faces = [np.ascontiguousarray(rng.normal(size=s.shape)) for _ in range(3)]
    c0 = [c.copy() for c in cells]
    f0 = [f.copy() for f in faces]
    grid = oracle.grid_of(s)
    oracle.lib().or_ghost_fill(ctypes.byref(grid), oracle._pp(cells), 8, oracle._pp(faces))
    act = [s.active(d) for d in range(3)]
    pads = tuple((g, g) if act[d] else (0, 0) for d in (2, 1, 0))
    inner = s.interior
    for v in range(8):
        want = np.pad(c0[v][inner], pads, mode="edge" if bc == W.OUTFLOW else "wrap")
        assert np.array_equal(cells[v], want), v
    for fd in range(3):
        # transverse directions: like a cell array; along fd: the evolved
        # faces g .. g + n (one more than the cells)
        ext = list(inner)
        ax = 2 - fd
        if act[fd]:
            ext[ax] = slice(g, g + s.n[fd] + 1)
        evolved = f0[fd][tuple(ext)]
        if bc == W.OUTFLOW:
            p = list(pads)
            if act[fd]:
                p[ax] = (g, g - 1)
            want = np.pad(evolved, tuple(p), mode="edge")
        else:
            # periodic: face g + n is the image of face g; ghosts wrap the n distinct faces
            ev = evolved
            if act[fd]:
                ev = np.take(evolved, range(s.n[fd]), axis=ax)
            p = list(pads)
            if act[fd]:
                p[ax] = (g, g)
            want = np.pad(ev, tuple(p), mode="wrap")
            if act[fd]:
                # the evolved top face g + n itself is not overwritten
                idx = [slice(None)] * 3
                idx[ax] = g + s.n[fd]
                want[tuple(idx)] = np.pad(np.take(evolved, [s.n[fd]], axis=ax),
                                          tuple(q if a != ax else (0, 0) for a, q in enumerate(p)),
                                          mode="wrap").squeeze(axis=ax)
        assert np.array_equal(faces[fd], want), fd


def test_ghost_fill_fixed_untouched():
    s = W._blank(W.Setup("ghosts", 2, (5, 4, 1), 2, (0, 0, 0), (1, 1, 1), W._bc(2, W.FIXED), 5 / 3, W.MC, W.SSP2))
    rng = np.random.default_rng(4)
    cells = [np.ascontiguousarray(rng.normal(size=s.shape)) for _ in range(8)]
    faces = [np.ascontiguousarray(rng.normal(size=s.shape)) for _ in range(3)]
    c0 = [c.copy() for c in cells]
    f0 = [f.copy() for f in faces]
    oracle.lib().or_ghost_fill(ctypes.byref(oracle.grid_of(s)), oracle._pp(cells), 8, oracle._pp(faces))
    assert all(np.array_equal(a, b) for a, b in zip(cells + faces, c0 + f0))


def test_outflow_boundary_faces_are_evolved():
    """faces on the domain boundary are evolved by CT, not copied: a uniform
    flow through a linear field changes the boundary faces at the same rate
    as the interior ones (-(v . grad) B), and div B stays at round-off"""
    s = W._blank(W.Setup("lin", 2, (12, 10, 1), 2, (-1, -1, 0), (1, 1, 1), W._bc(2, W.OUTFLOW), 5 / 3, W.MC,
                         W.SSP2, eta=1e-6))
    vx = 0.3
    Wl = 1 / math.sqrt(1 - vx * vx)
    s.prim[0], s.prim[4], s.prim[1] = 1.0, 1.0, Wl * vx
    # B^y = b x (linear in x), E = -v x B: E^z = v B^y
    X, _, _ = s.mesh()
    b = 0.05
    s.face = np.zeros((3,) + s.shape)
    s.face[1] = b * X
    s.E[2] = vx * b * X
    st = oracle.OracleState(s)
    f0 = st.face[1].copy()
    dt = 0.2 * st.dt()
    st.step(dt)
    g = s.ng
    # dB^y/dt = -d_x E^z = -v b everywhere, also on the faces of the boundary rows j = g and j = g + n
    rate = (st.face[1] - f0)[g:g + 1, g:g + s.n[1] + 1, g:g + s.n[0]] / dt
    assert np.allclose(rate, -vx * b, rtol=1e-9, atol=0)
    assert st.divB()[2] <= 1e-13


# --------------------------------------------------------------------------
# time step (Sec 2.5 speeds alpha sqrt(gamma^dd) = alpha / psi^2, reading R16)
def test_cfl_dt_flat_closed_form():
    s = W.blast_wave(512, eta=1e-6)
    assert oracle.OracleState.dt(_light(s)) == pytest.approx(4.6875e-3, rel=1e-15)  # 0.4 * (12 / 512) / 2
    s1 = W.shock_tube(400)
    assert oracle.OracleState.dt(_light(s1)) == pytest.approx(1e-3, rel=1e-15)  # 0.4 * 2.5e-3


class _light:
    """enough of OracleState for dt(): the grid and the metric arrays"""

    def __init__(self, s):
        self.grid = oracle.grid_of(s)
        self.alpha = np.ascontiguousarray(s.alpha) if s.metric else None
        self.psi = np.ascontiguousarray(s.psi) if s.metric else None


@pytest.mark.parametrize("ndim", [1, 2, 3])
def test_cfl_dt_constant_metric_is_rescaled_flat_step(ndim):
    """with constant alpha and psi the light cone spans psi^-2 alpha dt per
    coordinate time: the step equals the flat step on a psi^2-larger grid
    divided by alpha"""
    alpha, psi = 0.7, 1.3
    n = (8, 6 if ndim > 1 else 1, 5 if ndim > 2 else 1)
    mk = lambda lo, hi: W._blank(W.Setup("c", ndim, n, 2, lo, hi, W._bc(ndim, W.OUTFLOW), 2.0, W.MC, W.SSP2))
    s = mk((0, 0, 0), (1.0, 0.75, 0.5))
    s.metric = 1
    s.alpha = np.full(s.shape, alpha)
    s.psi = np.full(s.shape, psi)
    f = mk((0, 0, 0), (psi ** 2, 0.75 * psi ** 2, 0.5 * psi ** 2))
    assert _light(s).grid.metric == 1
    dt_m = oracle.OracleState.dt(_light(s))
    dt_f = oracle.OracleState.dt(_light(f))
    assert dt_m == pytest.approx(dt_f / alpha, rel=1e-14)
    # and the flat step sums the inverse spacings of the active directions
    dxs = [1.0 / 8, 0.75 / 6, 0.5 / 5][:ndim]
    assert oracle.OracleState.dt(_light(mk((0, 0, 0), (1.0, 0.75, 0.5)))) == pytest.approx(
        0.4 / sum(1 / d for d in dxs), rel=1e-14)


def test_cfl_dt_takes_the_fastest_cell():
    """a non-uniform lapse: the step is set by the cell with the largest
    alpha / psi^2 (interior cells only; ghosts are ignored)"""
    s = W._blank(W.Setup("c", 2, (6, 6, 1), 2, (0, 0, 0), (1, 1, 1), W._bc(2, W.OUTFLOW), 2.0, W.MC, W.SSP2))
    s.metric = 1
    s.alpha = np.full(s.shape, 0.5)
    s.psi = np.full(s.shape, 1.0)
    s.alpha[0, 4, 5] = 0.9  # interior cell
    s.alpha[0, 0, 0] = 5.0  # ghost cell: ignored
    dt = oracle.OracleState.dt(_light(s))
    assert dt == pytest.approx(0.4 / (0.9 * 6 + 0.9 * 6), rel=1e-14)


# --------------------------------------------------------------------------
# PPM monotonicity constraints (reading R10): the limited parabola of a cell,
# a(x) = aL + x (dA + a6 (1 - x)) on x in [0, 1] with dA = aR - aL and
# a6 = 6 (a - (aL + aR)/2), keeps the cell mean a, is monotone on the cell, and
# is flat at a local extremum; a smooth monotone profile is left unchanged
def _cell_lr(w7):
    """(aL, aR) of the middle cell of w7 (cells c-3..c+3) from the face form"""
    _, aL = oracle.recon(W.PPM, np.ascontiguousarray(w7[0:6]))
    aR, _ = oracle.recon(W.PPM, np.ascontiguousarray(w7[1:7]))
    return aL, aR


def test_ppm_limited_parabola_is_monotone_and_conservative():
    rng = np.random.default_rng(21)
    x = np.linspace(0.0, 1.0, 201)
    n_lim = 0
    for trial in range(3000):
        w = rng.normal(size=7) if trial % 3 else np.cumsum(rng.random(7)) * rng.choice([-1, 1])
        a = w[3]
        aL, aR = _cell_lr(w)
        if (w[4] - a) * (a - w[2]) <= 0.0:
            # local extremum: flat
            assert aL == a and aR == a
            continue
        dA, a6 = aR - aL, 6.0 * (a - 0.5 * (aL + aR))
        prof = aL + x * (dA + a6 * (1.0 - x))
        # cell mean of the parabola: aL + dA/2 + a6/6 = a
        assert aL + 0.5 * dA + a6 / 6.0 == pytest.approx(a, abs=1e-12 * (1 + abs(a)))
        d = np.diff(prof)
        tol = 1e-12 * (1 + np.abs(w).max())
        assert np.all(d >= -tol) or np.all(d <= tol), (trial, w, aL, aR)
        # the values stay within the range of the cell and its neighbours' interfaces
        assert min(aL, aR) - tol <= a <= max(aL, aR) + tol
        n_lim += 1
    assert n_lim > 1000


def test_ppm_smooth_monotone_profile_unchanged():
    """on a smooth monotone profile neither constraint fires: the face values
    are the fourth-order interface values 7/12 (a0 + a1) - 1/12 (a-1 + a2)"""
    xs = np.arange(8) * 0.1
    w = np.exp(xs)  # cell values of a smooth increasing profile (mild curvature)
    aL, aR = _cell_lr(w[0:7])
    iface = lambda am1, a0, a1, a2: 7.0 / 12.0 * (a0 + a1) - 1.0 / 12.0 * (am1 + a2)
    assert aL == pytest.approx(iface(w[1], w[2], w[3], w[4]), rel=1e-15)
    assert aR == pytest.approx(iface(w[2], w[3], w[4], w[5]), rel=1e-15)


def test_ppm_steep_side_is_limited():
    """a parabola whose extremum would fall inside the cell is steepened
    toward the far side: aL = 3a - 2aR (or aR = 3a - 2aL), which moves the
    extremum to the cell edge (the derivative vanishes there)"""
    rng = np.random.default_rng(5)
    hits = 0
    for _ in range(5000):
        w = np.cumsum(rng.random(7) ** 3) * rng.choice([-1, 1])
        a = w[3]
        aL, aR = _cell_lr(w)
        dA, a6 = aR - aL, 6.0 * (a - 0.5 * (aL + aR))
        if abs(a6) < 1e-12 * (1 + abs(a)) or abs(dA) < 1e-14:
            continue
        # derivative of the parabola at the edges: dA + a6 (1 - 2x)
        d0, d1 = dA + a6, dA - a6
        if abs(d0) <= 1e-9 * abs(dA) or abs(d1) <= 1e-9 * abs(dA):
            hits += 1
    assert hits > 50
