"""Pins of the oracle's point-wise pieces (no GPU).

Each check is fixed by the mathematics, not by re-typing the oracle's formula:
round trips, a direct linear solve of the implicit equation, finite
differences, manufactured roots and closed-form limits.
"""
import itertools
import math

import numpy as np
import pytest

import oracle

GAM = 5.0 / 3.0


def crossg(psi, a, b):
    """epsilon^{ijk} a_j b_k for contravariant a, b in gamma_ij = psi^4 delta_ij"""
    g = psi ** 4
    return np.cross(a * g, b * g) / psi ** 6


def unit(rng):
    d = rng.normal(size=3)
    return d / np.linalg.norm(d)


# --------------------------------------------------------------------------
# Sec 2.1 / 2.6: prim -> cons -> prim round trip
@pytest.mark.parametrize("psi", [1.0, 1.3])
def test_prim_cons_round_trip(psi):
    rng = np.random.default_rng(11)
    worst = 0.0
    for W, sig, pr in itertools.product([1.0, 1.01, 2.0, 10.0, 100.0], [0.0, 1.0, 1e2, 1e4],
                                        [1e-6, 1e-2, 1.0, 1e2]):
        rho = 0.7
        p = pr * rho
        ut = math.sqrt(W * W - 1) * unit(rng) / psi ** 2
        b = math.sqrt(sig * rho)
        B = b * unit(rng) / psi ** 2
        E = 0.9 * rng.random() * b * unit(rng) / psi ** 2
        prim = np.array([rho, *ut, p])
        q = oracle.prim2cons(GAM, psi, prim, E, B)
        r, back = oracle.c2p(GAM, psi, q, E, B)
        assert r == 0
        tau = q[4] / psi ** 6
        D = q[0] / psi ** 6
        # cancellation bound: the thermal part is a fraction p/(tau+D) of the energy
        cond = max(1.0, (tau + D) / p)
        e_rho = abs(back[0] - rho) / rho
        e_u = np.abs(back[1:4] - ut).max() / max(1.0, np.abs(ut).max())
        e_p = abs(back[4] - p) / p
        assert e_rho <= 1e-12 * cond, (W, sig, pr, e_rho)
        assert e_u <= 1e-12 * cond, (W, sig, pr, e_u)
        assert e_p <= 1e-12 * cond, (W, sig, pr, e_p)
        worst = max(worst, e_p / cond)
    assert worst < 1e-12


def test_c2p_cold_gas_p_zero():
    """p = 0 exactly (cold gas) is a valid root at the lower end of the bracket"""
    prim = np.array([1e12, 0, 0, 0, 0.0])
    E = np.array([0.3, -0.1, 0.0])
    B = np.array([0.0, 0.0, 0.7])
    q = oracle.prim2cons(4 / 3, 1.0, prim, E, B)
    r, back = oracle.c2p(4 / 3, 1.0, q, E, B)
    assert r == 0
    assert back[0] == pytest.approx(1e12, rel=1e-14)
    assert abs(back[4]) <= 1e-3  # round-off of tau + D ~ 1e12 is 1e-4


def test_c2p_reports_unphysical_state():
    """tau below the rest-mass + field energy has no root with p >= 0"""
    q = np.array([1.0, 0.0, 0.0, 0.0, -0.1, 0, 0, 0])
    r, _ = oracle.c2p(GAM, 1.0, q, np.zeros(3), np.zeros(3))
    assert r == 1


# --------------------------------------------------------------------------
# Sec 2.4, eq. im_E: the A_0..A_5 form equals a direct solve of the implicit
# equation E = E* - (W/eta~){[E + v x B - (E.v) v] - xi [B - v x E - (B.v) v]}
@pytest.mark.parametrize("xi", [0.0, 0.3, -0.7])
@pytest.mark.parametrize("psi", [1.0, 1.2])
@pytest.mark.parametrize("etat", [1e-3, 0.4, 1e3])
def test_im_E_coefficients_match_direct_solve(xi, psi, etat):
    rng = np.random.default_rng(int(100 * etat + 7 * psi + 13 * xi + 50))
    for _ in range(5):
        ut = rng.normal(size=3)
        Es = rng.normal(size=3)
        B = rng.normal(size=3)
        E = oracle.implicit_E(psi, etat, xi, ut, Es, B)
        g = psi ** 4
        W = math.sqrt(1 + g * ut @ ut)
        v = ut / W

        def resid(Ev):
            Ed = g * Ev @ v
            Bd = g * B @ v
            return Ev - Es + (W / etat) * ((Ev + crossg(psi, v, B) - Ed * v) - xi * (B - crossg(psi, v, Ev) - Bd * v))

        r0 = resid(np.zeros(3))
        M = np.stack([resid(e) - r0 for e in np.eye(3)], axis=1)
        Ed = np.linalg.solve(M, -r0)
        assert np.abs(E - Ed).max() <= 1e-12 * max(1.0, np.abs(Ed).max())


@pytest.mark.parametrize("xi", [0.0, 0.3])
@pytest.mark.parametrize("psi", [1.0, 1.15])
def test_jacobian_matches_finite_differences(xi, psi):
    rng = np.random.default_rng(5)
    for _ in range(4):
        q = np.array([1.3, *(0.4 * rng.normal(size=3)), 2.0, *(0.3 * rng.normal(size=3))])
        B = 0.5 * rng.normal(size=3)
        ut = 0.5 * rng.normal(size=3)
        etat = 10 ** rng.uniform(-2, 2)
        _, J = oracle.implicit_residual(GAM, psi, q, B, etat, xi, ut)
        h = 1e-6
        Jfd = np.zeros((3, 3))
        for j in range(3):
            e = np.zeros(3)
            e[j] = h
            fp, _ = oracle.implicit_residual(GAM, psi, q, B, etat, xi, ut + e)
            fm, _ = oracle.implicit_residual(GAM, psi, q, B, etat, xi, ut - e)
            Jfd[:, j] = (fp - fm) / (2 * h)
        assert np.abs(J - Jfd).max() <= 1e-7 * np.abs(J).max()


def manufactured(rng, psi, etat, sig_max=10.0):
    rho = 10 ** rng.uniform(-1, 1)
    p = rho * 10 ** rng.uniform(-2, 1)
    W = 1 + 9 * rng.random() ** 2
    ut = math.sqrt(W * W - 1) * unit(rng) / psi ** 2
    b = math.sqrt(10 ** rng.uniform(-2, math.log10(sig_max)) * rho)
    B = b * unit(rng) / psi ** 2
    Et = 0.5 * b * rng.random() * unit(rng) / psi ** 2
    prim = np.array([rho, *ut, p])
    q = oracle.prim2cons(GAM, psi, prim, Et, B)
    v = ut / W
    g = psi ** 4
    # the E* that the implicit step maps onto E_true (eq. im_E with xi = 0)
    Es = Et + (W / etat) * (Et + crossg(psi, v, B) - g * (Et @ v) * v)
    q[5:] = psi ** 6 * Es
    return prim, Et, B, q


@pytest.mark.parametrize("etat", [1e-8, 1e-4, 1.0, 1e4, 1e8])
def test_implicit_manufactured_root(etat):
    rng = np.random.default_rng(int(-math.log10(etat) * 10 + 100))
    for _ in range(40):
        psi = 1.0 + 0.2 * rng.random()
        prim, Et, B, q = manufactured(rng, psi, etat)
        r, got, E, it = oracle.implicit(GAM, psi, q, B, etat, 0.0, prim[1:4] * 0.95)
        assert r == 0
        assert got[0] == pytest.approx(prim[0], rel=1e-10)
        assert np.abs(got[1:4] - prim[1:4]).max() <= 1e-10 * (1 + np.abs(prim[1:4]).max())
        assert got[4] == pytest.approx(prim[4], rel=1e-9)
        assert np.abs(E - Et).max() <= 1e-9 * max(np.abs(Et).max(), np.abs(B).max())
        assert it <= 20


@pytest.mark.parametrize("psi", [1.0, 1.3])
@pytest.mark.parametrize("etat", [1e-8, 1e-4, 1.0, 1e4, 1e8])
def test_implicit_manufactured_root_pin_grid(etat, psi):
    """manufactured roots over the whole pin grid: W in {1 .. 100}, sigma in
    {0 .. 1e4}, p/rho in {1e-6 .. 1e2}, |E| < |B|; the solve returns the state
    within 1e-12 of the cancellation bound max(1, (tau + D)/p)"""
    rng = np.random.default_rng(int(-math.log10(etat) * 10 + 200 + 7 * psi))
    for W, sig, pr in itertools.product([1.0, 1.01, 2.0, 10.0, 100.0], [0.0, 1.0, 1e2, 1e4],
                                        [1e-6, 1e-2, 1.0, 1e2]):
        rho = 0.7
        p = pr * rho
        ut = math.sqrt(W * W - 1) * unit(rng) / psi ** 2
        b = math.sqrt(sig * rho)
        B = b * unit(rng) / psi ** 2
        Et = 0.9 * rng.random() * b * unit(rng) / psi ** 2
        prim = np.array([rho, *ut, p])
        q = oracle.prim2cons(GAM, psi, prim, Et, B)
        v = ut / W
        Es = Et + (W / etat) * (Et + crossg(psi, v, B) - psi ** 4 * (Et @ v) * v)
        q[5:] = psi ** 6 * Es
        r, got, E, it = oracle.implicit(GAM, psi, q, B, etat, 0.0, prim[1:4])
        assert r == 0, (W, sig, pr)
        cond = max(1.0, (q[4] + q[0]) / psi ** 6 / p)
        assert abs(got[0] - rho) / rho <= 1e-12 * cond, (W, sig, pr)
        assert np.abs(got[1:4] - ut).max() / max(1.0, np.abs(ut).max()) <= 1e-12 * cond, (W, sig, pr)
        assert abs(got[4] - p) / p <= 1e-12 * cond, (W, sig, pr)
        em = max(np.abs(Et).max(), np.abs(B).max(), 1e-300)
        assert np.abs(E - Et).max() / em <= 1e-12 * cond, (W, sig, pr)


def test_implicit_root_is_unique_from_several_starts():
    rng = np.random.default_rng(9)
    for _ in range(30):
        psi = 1.0
        etat = 10 ** rng.uniform(-3, 3)
        prim, Et, B, q = manufactured(rng, psi, etat, sig_max=1.0)
        roots = []
        for guess in [np.zeros(3), prim[1:4], 0.5 * prim[1:4], 0.3 * rng.normal(size=3)]:
            r, got, E, _ = oracle.implicit(GAM, psi, q, B, etat, 0.0, guess)
            if r == 0:
                roots.append(got)
        assert roots
        for g in roots:
            assert np.abs(g - roots[0]).max() <= 1e-9 * (1 + np.abs(roots[0]).max())


def test_implicit_v_zero_closed_form():
    """fluid at rest (S = E x B): E = eta~ E*/(1 + eta~), independent of B"""
    for etat in [1e-6, 0.3, 5.0]:
        E0 = np.array([0.2, -0.4, 0.1])
        B = np.array([0.3, 0.5, -0.2])
        prim = np.array([1.0, 0, 0, 0, 0.5])
        Etrue = etat * E0 / (1 + etat)
        q = oracle.prim2cons(GAM, 1.0, prim, Etrue, B)
        q[5:] = E0
        r, got, E, _ = oracle.implicit(GAM, 1.0, q, B, etat, 0.0, np.zeros(3))
        assert r == 0
        assert np.abs(E - Etrue).max() <= 1e-13
        assert np.abs(got[1:4]).max() <= 1e-13
        assert got[4] == pytest.approx(0.5, rel=1e-12)


def test_implicit_large_eta_reduces_to_c2p():
    """eta~ -> infinity: E -> E*, and the fused solve is the plain recovery"""
    rng = np.random.default_rng(3)
    for _ in range(10):
        prim, Et, B, q = manufactured(rng, 1.0, 1e14)
        r, got, E, _ = oracle.implicit(GAM, 1.0, q, B, 1e14, 0.0, prim[1:4])
        r2, ref = oracle.c2p(GAM, 1.0, q, q[5:], B)
        assert r == 0 and r2 == 0
        assert np.abs(got - ref).max() <= 1e-9 * (1 + np.abs(ref).max())
        assert np.abs(E - q[5:]).max() <= 1e-11 * (1 + np.abs(E).max())


def test_implicit_small_eta_ideal_limit():
    """eta~ -> 0: E -> -v x B with an error O(eta~)"""
    rng = np.random.default_rng(4)
    prim, Et, B, q = manufactured(rng, 1.0, 1.0)
    errs = []
    for etat in [1e-4, 1e-6]:
        r, got, E, _ = oracle.implicit(GAM, 1.0, q, B, etat, 0.0, prim[1:4])
        assert r == 0
        W = math.sqrt(1 + got[1:4] @ got[1:4])
        v = got[1:4] / W
        errs.append(np.abs(E + np.cross(v, B)).max())
    assert errs[1] < errs[0] * 0.05
    assert errs[1] < 1e-4


# --------------------------------------------------------------------------
# mean-field dynamo (xi != 0, eq. ohms_law): manufactured roots of the fused
# solve from the implicit Ohm's-law equation written out directly
@pytest.mark.parametrize("xi", [0.2, -0.5])
@pytest.mark.parametrize("etat", [1e-3, 1.0, 1e3])
def test_implicit_manufactured_root_dynamo(xi, etat):
    rng = np.random.default_rng(int(1000 * abs(xi) + 10 * math.log10(etat) + 77))
    for _ in range(20):
        psi = 1.0 + 0.2 * rng.random()
        g = psi ** 4
        rho = 10 ** rng.uniform(-1, 1)
        p = rho * 10 ** rng.uniform(-2, 1)
        W = 1 + 3 * rng.random() ** 2
        ut = math.sqrt(W * W - 1) * unit(rng) / psi ** 2
        b = math.sqrt(10 ** rng.uniform(-2, 0) * rho)
        B = b * unit(rng) / psi ** 2
        Et = 0.5 * b * rng.random() * unit(rng) / psi ** 2
        prim = np.array([rho, *ut, p])
        q = oracle.prim2cons(GAM, psi, prim, Et, B)
        v = ut / W
        Es = Et + (W / etat) * ((Et + crossg(psi, v, B) - g * (Et @ v) * v)
                                - xi * (B - crossg(psi, v, Et) - g * (B @ v) * v))
        q[5:] = psi ** 6 * Es
        r, got, E, it = oracle.implicit(GAM, psi, q, B, etat, xi, prim[1:4] * 0.97)
        assert r == 0
        assert got[0] == pytest.approx(prim[0], rel=1e-10)
        assert np.abs(got[1:4] - prim[1:4]).max() <= 1e-10 * (1 + np.abs(prim[1:4]).max())
        assert got[4] == pytest.approx(prim[4], rel=1e-9)
        assert np.abs(E - Et).max() <= 1e-9 * max(np.abs(Et).max(), np.abs(B).max())


def test_implicit_v_zero_closed_form_dynamo():
    """fluid at rest: (1 + eta~) E = eta~ E* + xi B"""
    for etat, xi in [(1e-4, 0.5), (0.3, -0.2), (5.0, 0.9)]:
        E0 = np.array([0.2, -0.4, 0.1])
        B = np.array([0.3, 0.5, -0.2])
        prim = np.array([1.0, 0, 0, 0, 0.5])
        Etrue = (etat * E0 + xi * B) / (1 + etat)
        q = oracle.prim2cons(GAM, 1.0, prim, Etrue, B)
        q[5:] = E0
        r, got, E, _ = oracle.implicit(GAM, 1.0, q, B, etat, xi, np.zeros(3))
        assert r == 0
        assert np.abs(E - Etrue).max() <= 1e-13
        assert np.abs(got[1:4]).max() <= 1e-12
