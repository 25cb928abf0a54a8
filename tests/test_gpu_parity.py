"""Parity of the HIP library (through the C ABI) with the CPU oracle.

Tolerance (FP64 both sides, different operation order), per primitive, E
and face field over interior cells, each normalised by the field's own scale
(tests/parity.py): relative L1 <= 1e-10 and element-wise <= 1e-9 after one
step, relative L1 <= 1e-8 and element-wise <= 1e-7 after 100 steps;
|div B|_inf <= 1e-12.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W
from parity import check, device_E, oracle_E, say, state_errors

pytestmark = pytest.mark.gpu

ONE = (1e-10, 1e-9)    # relative L1, element-wise after one step
HUNDRED = (1e-8, 1e-7)  # after 100 steps


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch


def gpu_run(s):
    from paper_2110_03732_amd import grmhd
    return grmhd.Run(s, device="cuda:0")


CASES = {
    "shock_tube_400_minmod_ssp2": lambda: W.shock_tube(400),
    "shock_tube_37_ppm_ssp3": lambda: W.shock_tube(37, recon=W.PPM, imex=W.SSP3),
    "blast_48_ppm_ssp3_stiff": lambda: W.blast_wave(48, eta=1e-6),
    "blast_48_ppm_ssp3_eta1e-2": lambda: W.blast_wave(48, eta=1e-2),
    "blast_37x23_mc_ssp2": lambda: _ragged_blast(),
    "loop_periodic_40x20": lambda: W.loop_advection(40, 20),
    "telegraph_32_p0": lambda: W.telegraph(32),
    "charged_vortex_32_fixed": lambda: W.charged_vortex(32),
    "star_24_cowling": lambda: W.tov_star(24),
    "star_13x11x9_ragged": lambda: _ragged_star(),
    # the star on its equatorial plane and on the x axis (metric with
    # inactive directions: planar and line EMF tiles, one-row x/y tiles)
    "star_2d_40_cowling": lambda: _star_slice(40, 2),
    "star_2d_33_mc_ssp2_cowling": lambda: _star_slice(33, 2, recon=W.MC, imex=W.SSP2),
    "star_1d_150_cowling": lambda: _star_slice(150, 1),
    "star_1d_97_minmod_ssp2_cowling": lambda: _star_slice(97, 1, recon=W.MINMOD, imex=W.SSP2),
    "dynamo_k1_frozen_xi0.5": lambda: W.steady_dynamo(64, k=1),
    "blast_48_ppm_ssp3_xi0.05": lambda: _with(W.blast_wave(48, eta=1e-2), xi=0.05),
    # degenerate and minimal shapes: one-cell-thick active directions, periodic
    # grids as small as the ghost width, fixed boundaries
    "box_3d_12x9x1_outflow_mc": lambda: _smooth_box(3, (12, 9, 1), W.OUTFLOW),
    "box_3d_1x10x8_outflow_ppm_ssp3": lambda: _smooth_box(3, (1, 10, 8), W.OUTFLOW, W.PPM, W.SSP3),
    "box_2d_1x16_outflow_mc": lambda: _smooth_box(2, (1, 16, 1), W.OUTFLOW),
    "box_1d_3_periodic_ppm": lambda: _smooth_box(1, (3, 1, 1), W.PERIODIC, W.PPM),
    "box_3d_3x3x3_periodic_ppm_ssp3": lambda: _smooth_box(3, (3, 3, 3), W.PERIODIC, W.PPM, W.SSP3),
    "box_2d_5x4_fixed_minmod": lambda: _smooth_box(2, (5, 4, 1), W.FIXED, W.MINMOD),
    # a different boundary rule along each direction of a ragged 3-D grid
    "box_3d_37x15x18_mixed_bc_ppm_ssp3": lambda: _mixed_box(W.PPM, W.SSP3),
    "box_3d_37x15x18_mixed_bc_mc_ssp2": lambda: _mixed_box(W.MC, W.SSP2),
    # ideal-MHD edge EMF (App. A)
    "shock_tube_400_minmod_ssp2_uct_ideal": lambda: _with(W.shock_tube(400), uct=1),
    "blast_48_ppm_ssp3_stiff_uct_ideal": lambda: _with(W.blast_wave(48, eta=1e-6), uct=1),
    "blast_48_ppm_ssp3_eta1e-2_uct_ideal": lambda: _with(W.blast_wave(48, eta=1e-2), uct=1),
    "blast_37x23_mc_ssp2_uct_ideal": lambda: _with(_ragged_blast(), uct=1),
    "loop_periodic_40x20_uct_ideal": lambda: _with(W.loop_advection(40, 20), uct=1),
    "star_24_cowling_uct_ideal": lambda: _with(W.tov_star(24), uct=1),
    "star_13x11x9_ragged_uct_ideal": lambda: _with(_ragged_star(), uct=1),
    "star_2d_40_cowling_uct_ideal": lambda: _with(_star_slice(40, 2), uct=1),
    "star_1d_150_cowling_uct_ideal": lambda: _with(_star_slice(150, 1), uct=1),
}


def _star_slice(n, ndim, **kw):
    """the Cowling star on z = 0 (ndim 2) or on the x axis (ndim 1), with a
    small velocity inside the star"""
    s = W.tov_star(n, ndim=ndim, **kw)
    X, Y, _ = s.mesh()
    w = s.prim[0] / s.prim[0].max()
    s.prim[1] = 0.01 * np.sin(X / 3) * w
    if ndim >= 2:
        s.prim[2] = -0.008 * np.sin(Y / 2.5) * w
    return s


def _smooth_box(ndim, n, bc, recon=W.MC, imex=W.SSP2):
    """degenerate and minimal shapes: a smooth bump of density and pressure,
    a swirl, a uniform field with E = -v x B, on [-1, 1]^ndim"""
    ng = 3 if recon == W.PPM else 2
    s = W._blank(W.Setup("box", ndim, n, ng, (-1, -1, -1), (1, 1, 1), W._bc(ndim, bc), 5.0 / 3.0, recon, imex,
                         eta=1e-2))
    X, Y, Z = s.mesh()
    r2 = sum(a * a for a, d in zip((X, Y, Z), range(3)) if s.active(d))
    g = np.exp(-2.0 * r2)
    s.prim[0] = 1.0 + 0.3 * g
    s.prim[4] = 0.5 + 0.2 * g
    v = [0.2 * g * (Y if ndim > 1 else 1.0), -0.15 * g * X, 0.1 * g]
    Wl = 1.0 / np.sqrt(1.0 - v[0] ** 2 - v[1] ** 2 - v[2] ** 2)
    B = (0.3, 0.2, 0.1)
    for i in range(3):
        s.prim[1 + i] = Wl * v[i]
    s.E[0] = -(v[1] * B[2] - v[2] * B[1])
    s.E[1] = -(v[2] * B[0] - v[0] * B[2])
    s.E[2] = -(v[0] * B[1] - v[1] * B[0])
    s.face = np.zeros((3,) + s.shape)
    for i in range(3):
        s.face[i] = B[i]
    return s


def _mixed_box(recon, imex, glm=False):
    """the smooth box on a ragged 3-D grid spanning several tiles of every
    kernel, with a different boundary rule along each direction: periodic in
    x, outflow in y, fixed in z (GLM: cell-centred q_B and the two cleaning
    fields in place of the face fields and the edge EMF)"""
    s = _smooth_box(3, (37, 15, 18), W.PERIODIC, recon, imex)
    s.bc = ((W.PERIODIC, W.PERIODIC), (W.OUTFLOW, W.OUTFLOW), (W.FIXED, W.FIXED))
    s.name = "box_mixed"
    if glm:
        s.glm, s.kappa_E, s.kappa_B = 1, 1.0, 2.0
    return s


def _with(s, **kw):
    for k, v in kw.items():
        setattr(s, k, v)
    return s


def _ragged_blast():
    s = W.blast_wave(37, eta=1e-3, recon=W.MC, imex=W.SSP2)
    s2 = W._blank(W.Setup("blast_ragged", 2, (37, 23, 1), 2, (-6, -4, 0), (6, 4, 1), W._bc(2, W.OUTFLOW), 4 / 3, W.MC,
                          W.SSP2, eta=1e-3, rho_atm=1e-14))
    X, Y, _ = s2.mesh()
    s2.prim[0] = 0.01
    s2.prim[4] = np.where(X ** 2 + Y ** 2 < 1, 1.0, 1e-3)
    s2.A = np.zeros((3,) + s2.edge_shape)
    _, Ye, _ = s2.edge_mesh(2)
    s2.A[2] = 0.1 * Ye
    del s
    return s2


def _ragged_star():
    W.tov_star(8)
    # a ragged box inside the star (same initial-data recipe)
    s2 = W._blank(W.Setup("star_ragged", 3, (13, 11, 9), 3, (-6.5, -5.5, -4.5), (6.5, 5.5, 4.5),
                          W._bc(3, W.OUTFLOW), 2.0, W.PPM, W.SSP3, eta_mode=1, eta=1e-6, sigma0=1e6, eta_min=1e-6,
                          eta_max=1.0, rho_atm=1e-10, p_atm=1e-18, metric=1, atm_factor=1e4))
    T = W._TOV_CACHE[("tov",)]
    X, Y, Z = s2.mesh()
    r = np.sqrt(X ** 2 + Y ** 2 + Z ** 2)
    rho = T["rho"](r)
    s2.prim[0] = np.where(rho > 1e-10, rho, 1e-10)
    s2.prim[4] = np.where(rho > 1e-10, np.maximum(100 * rho ** 2, 1e-18), 1e-18)
    s2.prim[1] = 0.01 * np.sin(X / 3) * s2.prim[0] / s2.prim[0].max()
    s2.alpha = T["alpha"](r)
    s2.psi = T["psi"](r)
    s2.A = np.zeros((3,) + s2.edge_shape)
    Xe, Ye, Ze = s2.edge_mesh(0)
    s2.A[0] = -1e-5 * Ye * np.exp(-(Xe ** 2 + Ye ** 2 + Ze ** 2) / 8)
    Xe, Ye, Ze = s2.edge_mesh(1)
    s2.A[1] = 1e-5 * Xe * np.exp(-(Xe ** 2 + Ye ** 2 + Ze ** 2) / 8)
    return s2


@pytest.mark.parametrize("name", sorted(CASES))
def test_one_step_parity(name):
    _torch()
    say("case %s: one step" % name)
    s = CASES[name]()
    run = gpu_run(s)
    ref = oracle.OracleState(s)
    dt = ref.dt()
    assert run.dt() == pytest.approx(dt, rel=1e-14)
    run.step(dt)
    ref.step(dt)
    check(s, run, ref, *ONE)
    d = run.divB()
    assert d[2] <= 1e-12
    assert run.fail_count() == ref.nfail


@pytest.mark.parametrize("name", ["shock_tube_400_minmod_ssp2", "blast_48_ppm_ssp3_eta1e-2", "star_24_cowling",
                                  "dynamo_k1_frozen_xi0.5", "blast_48_ppm_ssp3_eta1e-2_uct_ideal",
                                  "star_24_cowling_uct_ideal", "loop_periodic_40x20", "star_2d_40_cowling",
                                  "star_1d_150_cowling", "box_3d_37x15x18_mixed_bc_ppm_ssp3"])
def test_hundred_steps_parity(name):
    _torch()
    say("case %s: 100 steps" % name)
    s = CASES[name]()
    run = gpu_run(s)
    ref = oracle.OracleState(s)
    dt = ref.dt()
    for _ in range(100):
        run.step(dt)
        ref.step(dt)
    check(s, run, ref, *HUNDRED)
    d = run.divB()
    assert d[2] <= 1e-12
    assert run.fail_count() == ref.nfail


def test_con2prim_round_trip_and_parity():
    _torch()
    say("case random_states: con2prim")
    s = W.random_states((10, 9, 8), seed=3)
    run = gpu_run(s)
    run.con2prim()
    got = run.prims()
    ref = oracle.OracleState(s)
    import ctypes
    nf = oracle.lib().or_c2p_grid(ctypes.byref(ref.grid), oracle._pp(ref.q), oracle._pp(ref.face), oracle._pp(ref.prim),
                                  None)
    assert nf == 0 and run.fail_count() == 0
    sl = s.interior
    for v in range(5):
        sc = np.abs(s.prim[v][sl]).max() if v in (0, 4) else 1.0
        assert np.abs(got[v][sl] - ref.prim[v][sl]).max() <= 1e-10 * sc
        assert np.abs(got[v][sl] - s.prim[v][sl]).max() <= 1e-10 * sc


def test_explicit_operator_parity():
    """the stored L of stage 0 (pass 1 of SSP2) against the oracle's L"""
    _torch()
    say("case blast 40^2: explicit operator")
    s = W.blast_wave(40, eta=1e-2, recon=W.MC, imex=W.SSP2)
    X, Y, _ = s.mesh()
    s.prim[1] = 0.2 * np.exp(-(X ** 2 + Y ** 2) / 4)
    s.E[2] = 0.01 * np.exp(-(X ** 2 + Y ** 2) / 4)
    run = gpu_run(s)
    ref = oracle.OracleState(s)
    dt = ref.dt()
    run.stage(0, dt)
    run.stage(1, dt)
    _, L = ref.step(dt, dump_stage=0, with_L=True)
    sl = s.interior
    for f in range(11):
        g = run.work_field(2, 0, f)[sl]
        r = L[f][sl]
        sc = max(np.abs(r).max(), 1e-12)
        assert np.abs(g - r).max() <= 1e-9 * sc, (f, np.abs(g - r).max(), sc)


def test_divb_norm_and_dt_match_oracle():
    _torch()
    s = W.loop_advection(40, 20)
    run = gpu_run(s)
    ref = oracle.OracleState(s)
    d_gpu, d_ref = run.divB(), ref.divB()
    assert np.all(d_gpu <= 1e-12) and np.all(d_ref <= 1e-12)
    # a field with a planted divergence (not from a potential): norms agree
    s2 = W.random_states((7, 6, 5), seed=2)
    run2 = gpu_run(s2)
    ref2 = oracle.OracleState(s2)
    assert np.allclose(run2.divB(), ref2.divB(), rtol=1e-12, atol=0)
    s3 = W.tov_star(20)
    assert gpu_run(s3).dt() == pytest.approx(oracle.OracleState(s3).dt(), rel=1e-14)


def test_failure_fallback_counted():
    """host-forced unphysical cells (tau < 0) fall back to the atmosphere and are counted"""
    torch = _torch()
    s = W.random_states((8, 8, 8), seed=7)
    run = gpu_run(s)
    q = run.q.view(8, run.fs)
    pts = [(s.g(0) + 1, s.g(1) + 2, s.g(2) + 3), (s.g(0) + 4, s.g(1) + 5, s.g(2) + 1)]
    for i, j, k in pts:
        q[4, run.offset(i, j, k)] = -1.0
    torch.cuda.synchronize()
    run.con2prim()
    assert run.fail_count() == 2
    p = run.prims()
    for i, j, k in pts:
        c = p[:, k, j, i]
        assert c[0] == s.rho_atm and c[4] == s.p_atm and np.all(c[1:4] == 0.0)


def test_bitwise_deterministic():
    _torch()
    outs = []
    for _ in range(2):
        s = W.blast_wave(48, eta=1e-6)
        run = gpu_run(s)
        dt = run.dt()
        for _ in range(3):
            run.step(dt)
        outs.append((run.prims(), run.faces(), run.cons()))
    for a, b in zip(outs[0], outs[1]):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("name", ["tov_star_128_ppm_ssp3", "blast_512_ppm_ssp3_stiff", "shock_tube_400_10steps"])
def test_full_size_parity(name):
    """the benchmark workloads at their full sizes and launch configuration:
    the 128^3 star and the 512^2 blast wave one step, the 400-cell shock tube
    ten steps, element by element against the oracle"""
    _torch()
    say("full-size case %s" % name)
    if name.startswith("tov"):
        s, nsteps = W.tov_star(128), 1
    elif name.startswith("blast"):
        s, nsteps = W.blast_wave(512, eta=1e-6), 1
    else:
        s, nsteps = W.shock_tube(400), 10
    run = gpu_run(s)
    ref = oracle.OracleState(s)
    dt = ref.dt()
    for _ in range(nsteps):
        run.step(dt)
        ref.step(dt)
    check(s, run, ref, *ONE)
    assert run.divB()[2] <= 1e-12
    assert run.fail_count() == ref.nfail


@pytest.mark.parametrize("name", ["tov_star_128_ppm_ssp3", "blast_512_ppm_ssp3_stiff", "loop_512x256_periodic"])
def test_full_size_hundred_steps_invariants(name):
    """100 steps of the benchmark workloads at full size (the 128^3 star: the
    benchmark's own step): properties that hold at any size, against no
    oracle: div B at round-off (CT), no recovery failures, finite states; on
    the periodic loop the totals of q_D, q_tau and every face field kept"""
    _torch()
    say("full-size 100 steps %s" % name)
    if name.startswith("tov"):
        s = W.tov_star(128)
    elif name.startswith("blast"):
        s = W.blast_wave(512, eta=1e-6)
    else:
        s = W.loop_advection(512, 256)
    run = gpu_run(s)
    dt = run.dt()
    sl = s.interior
    tot0 = None
    if name.startswith("loop"):
        q, f = run.cons(), run.faces()
        tot0 = [q[0][sl].sum(), q[4][sl].sum()] + [f[d][sl].sum() for d in range(3)]
    for _ in range(100):
        run.step(dt)
    assert run.divB()[2] <= 1e-12
    assert run.fail_count() == 0
    p = run.prims()
    assert np.all(np.isfinite(p[:, sl[0], sl[1], sl[2]]))
    if tot0 is not None:
        q, f = run.cons(), run.faces()
        tot1 = [q[0][sl].sum(), q[4][sl].sum()] + [f[d][sl].sum() for d in range(3)]
        for a, b in zip(tot0, tot1):
            assert abs(a - b) <= 1e-13 * s.ncells * max(abs(a), 1e-3)


@pytest.mark.timeout(900)
@pytest.mark.parametrize("name", ["blast_512_ppm_ssp3_eta1e-6", "blast_512_ppm_ssp3_eta1e-2", "tov_star_64_ppm_ssp3"])
def test_full_size_hundred_steps_parity(name):
    """100 steps of the 512^2 blast wave (both resistivities of its
    configuration) and of the star at 64^3 (4 z-phase tiles, 8 x/y tiles per
    row, every EMF tile form), element by element against the oracle"""
    _torch()
    say("full-size 100 steps vs oracle %s" % name)
    if name.startswith("blast"):
        s = W.blast_wave(512, eta=1e-6 if name.endswith("1e-6") else 1e-2)
    else:
        s = W.tov_star(64)
    run = gpu_run(s)
    ref = oracle.OracleState(s)
    dt = ref.dt()
    for k in range(100):
        run.step(dt)
        ref.step(dt)
        if k % 25 == 24:
            say("  step %d" % (k + 1))
    check(s, run, ref, *HUNDRED)
    assert run.divB()[2] <= 1e-12
    assert run.fail_count() == ref.nfail


@pytest.mark.timeout(600)
def test_full_size_star_twenty_steps_parity():
    """20 steps of the 128^3 star, the benchmark's own step and launch
    configuration (at 2^21 cells every pass runs its EMF and face-update
    launches on the library's second stream), element by element against the
    oracle at the multi-step bar"""
    _torch()
    s = W.tov_star(128)
    say("128^3 star, 20 steps vs oracle")
    run = gpu_run(s)
    ref = oracle.OracleState(s)
    dt = ref.dt()
    for k in range(20):
        run.step(dt)
        ref.step(dt)
        if k % 5 == 4:
            say("  step %d" % (k + 1))
    check(s, run, ref, *HUNDRED)
    assert run.divB()[2] <= 1e-12
    assert run.fail_count() == ref.nfail


def test_shock_tube_to_t04_parity():
    """the 400-cell shock tube of its configuration run to t = 0.4 (400
    steps of dt = 1e-3) against the oracle"""
    _torch()
    s = W.shock_tube(400)
    say("shock tube 400 cells to t = 0.4")
    run = gpu_run(s)
    ref = oracle.OracleState(s)
    dt = ref.dt()
    assert dt == pytest.approx(1e-3, rel=1e-15)
    for _ in range(400):
        run.step(dt)
        ref.step(dt)
    assert run.t == pytest.approx(0.4, rel=1e-12)
    check(s, run, ref, *HUNDRED)
    assert run.divB()[2] <= 1e-12
    assert run.fail_count() == ref.nfail
