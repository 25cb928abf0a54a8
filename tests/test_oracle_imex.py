"""Pins of the oracle's time integrator (Sec 2.3) and reconstructions (no GPU)."""
import math

import numpy as np
import pytest

import oracle
import workloads as W


# --------------------------------------------------------------------------
# tableaux
def test_ssp2_tableau_is_the_printed_one(golden):
    At, A, wt, w = oracle.tableau(W.SSP2)
    g = 1 - 1 / math.sqrt(2)
    ref = golden["imex_ssp2"]
    assert np.array_equal(At, np.array(ref["At"], dtype=float))
    assert np.allclose(A, [[g, 0], [1 - 2 * g, g]], rtol=0, atol=1e-16)
    assert np.array_equal(wt, ref["wt"]) and np.array_equal(w, ref["w"])


def _order_conditions(At, A, wt, w, order):
    ct = At.sum(1)
    c = A.sum(1)
    res = []
    for b in (wt, w):
        res.append(b.sum() - 1)
        for cc in (ct, c):
            res.append(b @ cc - 0.5)
    if order >= 3:
        for b in (wt, w):
            for c1 in (ct, c):
                for c2 in (ct, c):
                    res.append(b @ (c1 * c2) - 1 / 3)
            for M in (At, A):
                for cc in (ct, c):
                    res.append(b @ M @ cc - 1 / 6)
    return np.abs(res).max()


def test_ssp2_order_conditions_and_l_stability():
    At, A, wt, w = oracle.tableau(W.SSP2)
    assert _order_conditions(At, A, wt, w, 2) < 1e-15
    # L-stability: R(z) = 1 + z w^T (I - zA)^-1 1 -> 1 - w^T A^-1 1 = 0 as z -> -inf
    assert abs(1 - w @ np.linalg.solve(A, np.ones(2))) < 1e-14


def test_ssp3_order_conditions():
    """every third-order explicit, implicit and coupling condition of the
    cited IMEX-SSP3(4,3,3) tableau (not printed in the paper)"""
    At, A, wt, w = oracle.tableau(W.SSP3)
    assert _order_conditions(At, A, wt, w, 3) < 2e-14
    assert np.all(np.triu(At) == 0)          # explicit
    assert np.all(np.triu(A, 1) == 0)        # diagonally implicit


def _R(A, w, z):
    s = len(w)
    return 1 + z * w @ np.linalg.solve(np.eye(s) - z * A, np.ones(s))


def _uniform_relax(imex, eta, alpha=1.0, psi=1.0, ndim=1):
    """uniform periodic box at rest, B = 0, E0 != 0: the spatial operator vanishes
    and E obeys dE/dt = -alpha E / eta (Sec 2.2 with v = 0)"""
    s = W.density_wave(8, ndim=ndim, amp=0.0, v=0.0, imex=imex)
    s.eta = eta
    s.E[0] = 0.3
    s.E[1] = -0.2
    s.E[2] = 0.1
    if alpha != 1.0 or psi != 1.0:
        s.metric = 1
        s.alpha = np.full(s.shape, alpha)
        s.psi = np.full(s.shape, psi)
    return s


@pytest.mark.parametrize("imex", [W.SSP2, W.SSP3])
@pytest.mark.parametrize("eta", [1e-6, 1.0])
@pytest.mark.parametrize("metric", [(1.0, 1.0), (0.7, 1.2)])
def test_stiff_relaxation_amplification(imex, eta, metric):
    alpha, psi = metric
    s = _uniform_relax(imex, eta, alpha, psi)
    st = oracle.OracleState(s)
    dt = 0.05
    _, A, _, w = oracle.tableau(imex)
    R = _R(A, w, -alpha * dt / eta)
    sl = s.interior
    E0 = st.E()[:, sl[0], sl[1], sl[2]].copy()
    tau0 = st.q[4][sl] / psi ** 6
    for n in range(1, 6):
        st.step(dt)
        E = st.E()[:, sl[0], sl[1], sl[2]]
        assert np.abs(E - R ** n * E0).max() <= 1e-13 * np.abs(E0).max() + 1e-300
        # tau is untouched (no flux, no source): p = (Gamma-1)(tau0 - E^2/2)
        E2 = psi ** 4 * (E ** 2).sum(0)
        p = st.prim[4][sl]
        assert np.abs(p - (s.gamma_ad - 1) * (tau0 - 0.5 * E2)).max() <= 1e-13
    assert st.nfail == 0


@pytest.mark.parametrize("imex,order", [(W.SSP2, 2), (W.SSP3, 3)])
def test_relaxation_time_order(imex, order):
    """E(T) against exp(-T/eta) for eta = 1 (non-stiff): the IMEX step has its order"""
    errs = []
    for dt in (0.1, 0.05):
        s = _uniform_relax(imex, 1.0)
        st = oracle.OracleState(s)
        for _ in range(int(round(1.0 / dt))):
            st.step(dt)
        sl = s.interior
        errs.append(abs(st.E()[0][sl].mean() - 0.3 * math.exp(-1.0)))
    rate = math.log2(errs[0] / errs[1])
    assert rate == pytest.approx(order, abs=0.15)


# --------------------------------------------------------------------------
# reconstructions (one variable, face between w[2] and w[3])
@pytest.mark.parametrize("kind", [W.MINMOD, W.MC, W.PPM])
def test_recon_exact_on_linear_data(kind):
    w = 0.3 + 0.7 * np.arange(6)
    L, R = oracle.recon(kind, w)
    assert L == pytest.approx(0.5 * (w[2] + w[3]), abs=1e-14)
    assert R == pytest.approx(0.5 * (w[2] + w[3]), abs=1e-14)


def test_ppm_interface_exact_on_cubic_data():
    x = np.arange(6) - 2.5  # face at x = 0
    w_cell = lambda a, b: (b ** 4 - a ** 4) / 4 + 0.5 * (b ** 3 - a ** 3) / 3  # cell averages of x^3 + 0.5 x^2
    avg = np.array([w_cell(xi - 0.5, xi + 0.5) for xi in x])
    # the interface value is exact for cubics; a smooth monotone profile keeps it
    L, R = oracle.recon(W.PPM, avg)
    assert L == pytest.approx(0.0, abs=1e-13) and R == pytest.approx(0.0, abs=1e-13)


@pytest.mark.parametrize("kind", [W.MINMOD, W.MC, W.PPM])
def test_recon_reflection_symmetry_and_bounds(kind):
    rng = np.random.default_rng(kind + 1)
    for _ in range(200):
        w = rng.normal(size=6)
        L, R = oracle.recon(kind, w)
        L2, R2 = oracle.recon(kind, w[::-1].copy())
        assert L == pytest.approx(R2, abs=1e-14) and R == pytest.approx(L2, abs=1e-14)
        # the left state lies between the cell value and its right neighbour's
        # range of the stencil cells it came from (no new extrema)
        assert min(w[1:4]) - 1e-14 <= L <= max(w[1:4]) + 1e-14
        assert min(w[2:5]) - 1e-14 <= R <= max(w[2:5]) + 1e-14


@pytest.mark.parametrize("kind", [W.MINMOD, W.MC, W.PPM])
def test_recon_flat_at_extremum(kind):
    w = np.array([0.0, 1.0, 3.0, 1.0, 0.0, -1.0])  # w[2] is a local maximum
    L, _ = oracle.recon(kind, w)
    assert L == 3.0
