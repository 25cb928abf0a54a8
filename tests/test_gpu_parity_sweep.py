"""A seeded sweep of small problems through the HIP library and the oracle:
every combination the kernels distinguish (dimension, reconstruction, IMEX
tableau, metric, boundary rule, EMF form, dynamo term, resistivity from ideal
to diffusive) drawn from splitmix64, two steps each, primitives, E and faces
within relative L1 1e-10 and element-wise 1e-9 of each field's scale, div B
at round-off.  A second sweep draws ragged 3-D boxes with a boundary rule of
their own along each direction."""
import math

import numpy as np
import pytest

import oracle
import workloads as W
from parity import check

pytestmark = pytest.mark.gpu

RECONS = (W.MINMOD, W.MC, W.PPM)
IMEXES = (W.SSP2, W.SSP3)


def _case(i):
    u = 0.5 * (W.uniform_pm1(20261203, i, 12) + 1.0)  # 12 draws in [0, 1)
    kind = int(u[0] * 4)
    recon = RECONS[int(u[1] * 3)]
    imex = IMEXES[int(u[2] * 2)]
    eta = math.exp(math.log(1e-6) + u[3] * (math.log(1.0) - math.log(1e-6)))
    uct = int(u[4] < 0.3)
    xi = 0.05 if u[5] < 0.2 else 0.0
    if kind == 0:
        n = 64 + int(u[6] * 200)
        s = W.shock_tube(n, seed=i, eta=eta, recon=recon, imex=imex, rho_r=0.125 + 0.5 * u[7],
                         p_r=0.1 + 0.5 * u[8], by_l=u[9] - 0.5)
    elif kind == 1:
        n = 24 + int(u[6] * 24)
        s = W.blast_wave(n, eta=eta, seed=i, recon=recon, imex=imex, bx=0.2 * u[7], p_in=0.1 + u[8])
        X, Y, _ = s.mesh()
        s.prim[1] = 0.3 * (u[9] - 0.5) * np.exp(-(X ** 2 + Y ** 2) / 4)
    elif kind == 2:
        s = W.loop_advection(16 + 2 * int(u[6] * 16), 8 + 2 * int(u[7] * 8), eta=eta, recon=recon, imex=imex,
                             vx=0.4 * (u[8] - 0.5), vy=0.4 * (u[9] - 0.5))
    else:
        s = W.tov_star(12 + int(u[6] * 10), imex=imex)  # PPM, as the star workload
    s.uct = uct
    s.xi = xi
    return s


@pytest.mark.parametrize("i", range(48))
def test_sweep(i):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2110_03732_amd import grmhd
    s = _case(i)
    print("sweep %d: %s ndim %d n %s recon %d imex %d metric %d uct %d xi %g eta %.2e" % (
        i, s.name, s.ndim, s.n, s.recon, s.imex, s.metric, s.uct, s.xi, s.eta), flush=True)
    run = grmhd.Run(s, device="cuda:0")
    ref = oracle.OracleState(s)
    dt = ref.dt()
    for _ in range(2):
        run.step(dt)
        ref.step(dt)
    check(s, run, ref, 1e-10, 1e-9, tag="sweep %d" % i)
    assert run.divB()[2] <= 1e-12
    assert run.fail_count() == ref.nfail


BCS = (W.OUTFLOW, W.PERIODIC, W.FIXED)


def _box_case(i):
    """a ragged 3-D box (the smooth bump, swirl and uniform field of the
    parity cases) with its own boundary rule along each direction and a
    random reconstruction, tableau, resistivity, EMF form and dynamo term"""
    from test_gpu_parity import _smooth_box
    u = 0.5 * (W.uniform_pm1(20261204, i, 12) + 1.0)
    recon = RECONS[int(u[0] * 3)]
    imex = IMEXES[int(u[1] * 2)]
    n = (5 + int(u[2] * 17), 5 + int(u[3] * 13), 5 + int(u[4] * 15))
    s = _smooth_box(3, n, W.OUTFLOW, recon, imex)
    s.bc = tuple((BCS[int(u[5 + d] * 3)],) * 2 for d in range(3))
    s.eta = math.exp(math.log(1e-6) + u[8] * (math.log(1.0) - math.log(1e-6)))
    s.uct = int(u[9] < 0.3)
    s.xi = 0.05 if u[10] < 0.25 else 0.0
    s.name = "box_sweep"
    return s


@pytest.mark.parametrize("i", range(16))
def test_sweep_3d_boxes(i):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2110_03732_amd import grmhd
    s = _box_case(i)
    print("box sweep %d: n %s bc %s recon %d imex %d uct %d xi %g eta %.2e" % (
        i, s.n, [b[0] for b in s.bc], s.recon, s.imex, s.uct, s.xi, s.eta), flush=True)
    run = grmhd.Run(s, device="cuda:0")
    ref = oracle.OracleState(s)
    dt = ref.dt()
    for _ in range(2):
        run.step(dt)
        ref.step(dt)
    check(s, run, ref, 1e-10, 1e-9, tag="box sweep %d" % i)
    assert run.divB()[2] <= 1e-12
    assert run.fail_count() == ref.nfail


def test_sweep_3d_boxes_batched():
    """the 16 boxes of the box sweep advanced two steps inside two batches
    (one per IMEX tableau, replayed graphs), each against the oracle at the
    same bars"""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2110_03732_amd import grmhd
    cases = [_box_case(i) for i in range(16)]
    for imex in IMEXES:
        setups = [s for s in cases if s.imex == imex]
        print("batched box sweep: imex %d, %d runs" % (imex, len(setups)), flush=True)
        runs = [grmhd.Run(s, device="cuda:0") for s in setups]
        dts = [r.dt() for r in runs]
        b = grmhd.Batch(runs, dts)
        b.run(2)
        torch.cuda.synchronize()
        for s, r, dt in zip(setups, runs, dts):
            ref = oracle.OracleState(s)
            assert dt == pytest.approx(ref.dt(), rel=1e-14)
            for _ in range(2):
                ref.step(dt)
            check(s, r, ref, 1e-10, 1e-9, tag="batched box n %s bc %s" % (s.n, [x[0] for x in s.bc]))
            assert r.divB()[2] <= 1e-12
            assert r.fail_count() == ref.nfail
        b.close()
