"""Mean-field dynamo (xi != 0) in the oracle: the 1-D steady dynamo test of
Sec 5.7 with the matter frozen.  Pins: the growth rates printed in the paper
(0.385 for k = 1, none for k = 5) and the closed-form dispersion relation of
Maxwell's equations with the Ohm's law of a fluid at rest, which the printed
numbers satisfy with eta = 0.1 (reading in the golden fixture)."""
import numpy as np
import pytest

import oracle
import workloads as W


def _growth(k, n=128, t_end=6.0, t_fit=(2.0, 6.0)):
    s = W.steady_dynamo(n, k=k)
    st = oracle.OracleState(s)
    dt = st.dt()
    prim0 = [a.copy() for a in st.prim]
    q0 = [a.copy() for a in st.q]
    t, ts, amp = 0.0, [], []
    while t < t_end:
        st.step(dt)
        t += dt
        ts.append(t)
        amp.append(np.abs(st.face[1][s.interior]).max())
    ts, amp = np.array(ts), np.array(amp)
    m = (ts > t_fit[0]) & (ts < t_fit[1])
    g = np.polyfit(ts[m], np.log(amp[m]), 1)[0]
    return g, amp, st, prim0, q0, s


def test_printed_growth_k1(golden):
    ref = golden["steady_dynamo"]
    g, _, _, _, _, _ = _growth(1)
    assert abs(g - ref["growth"][0]) <= 0.002
    assert abs(g - W.dynamo_growth_rate(1)) <= 1e-3 * W.dynamo_growth_rate(1)


def test_closed_form_growth_k2():
    g, _, _, _, _, _ = _growth(2)
    assert abs(g - W.dynamo_growth_rate(2)) <= 1e-3 * W.dynamo_growth_rate(2)


def test_k5_neutral(golden):
    """k = 5: resistivity and dynamo cancel; only the scheme's dissipation of
    a 25-cell wavelength remains"""
    assert W.dynamo_growth_rate(5) == pytest.approx(golden["steady_dynamo"]["growth"][1], abs=1e-12)
    g, amp, _, _, _, _ = _growth(5)
    assert abs(g) <= 0.05
    assert 0.8 * amp[0] <= amp[-1] <= 1.01 * amp[0]


def test_fastest_growth_printed(golden):
    ks = np.linspace(0.5, 5.0, 901)
    gmax = max(W.dynamo_growth_rate(k) for k in ks)
    assert abs(gmax - golden["steady_dynamo"]["fastest_growth"]) <= 0.005


def test_frozen_matter_keeps_the_fluid():
    _, _, st, prim0, q0, s = _growth(1, n=32, t_end=0.5, t_fit=(0.0, 0.5))
    sl = s.interior
    for v in range(5):
        assert np.array_equal(st.prim[v][sl], prim0[v][sl])
    for v in range(5):
        assert np.array_equal(st.q[v][sl], q0[v][sl])
    assert max(np.abs(st.q[5 + i][sl]).max() for i in range(3)) > 0.0
