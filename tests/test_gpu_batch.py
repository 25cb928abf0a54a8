"""Batched runs (gr_batch_*) through the C ABI.

A run advanced inside a batch must give the result of the same run advanced
alone with gr_step.  The batched and the single-grid kernels are two
compilations of the same source; their instruction selection may differ by an
ulp in a few places, which can move a Newton stopping decision, so the
comparison allows 1e-13 of each field's scale.  Two batches holding the same
run compute it with the same kernels: that comparison is exact.  The batch
mixes dimensions, reconstructions, sizes, resistivities and (with the star)
the metric, and the dynamo term; one run is checked against the CPU oracle as
well.
"""
import os
import sys

import numpy as np
import pytest

import oracle
import workloads as W
from parity import device_E, oracle_E, state_errors
from test_gpu_parity import _mixed_box

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _mix(imex):
    """small runs of every kind the kernels distinguish"""
    prm = W.batch_mix_params(6, seed=3, n1=(100, 700), n2=(40, 90))
    setups = [W.make_run_setup(p, imex=imex) for p in prm]
    setups.append(W.tov_star(20, imex=imex))
    # the metric on a plane and on a line (planar and line EMF tiles)
    setups.append(W.tov_star(24, ndim=2, imex=imex))
    setups.append(W.tov_star(90, ndim=1, imex=imex))
    setups.append(W.current_sheet(96, recon=W.MC, imex=imex))
    # the mean-field dynamo instances: frozen matter, and a moving fluid
    setups.append(W.steady_dynamo(64, imex=imex))
    b = W.blast_wave(32, eta=1e-2, imex=imex)
    b.xi = 0.05
    setups.append(b)
    return setups


def _same(a, b):
    for x, y, what in ((a.prims(), b.prims(), "prim"), (a.faces(), b.faces(), "face"), (a.cons(), b.cons(), "cons")):
        assert np.array_equal(x, y), what


def _close(a, b, tol=1e-13):
    for x, y, what in ((a.prims(), b.prims(), "prim"), (a.faces(), b.faces(), "face"), (a.cons(), b.cons(), "cons")):
        for f in range(x.shape[0]):
            sc = max(np.abs(y[f]).max(), 1e-300)
            assert np.abs(x[f] - y[f]).max() <= tol * sc, (what, f)


@pytest.mark.parametrize("imex", [W.SSP2, W.SSP3])
def test_batch_equals_single_runs(imex):
    torch = _torch()
    from paper_2110_03732_amd import grmhd
    setups = _mix(imex)
    say("batch of %d runs, imex %d" % (len(setups), imex))
    alone = [grmhd.Run(s, device="cuda:0") for s in setups]
    mixed = [grmhd.Run(s, device="cuda:0") for s in setups]
    dts = [r.dt() for r in alone]
    nsteps = 4
    for r, dt in zip(alone, dts):
        for _ in range(nsteps):
            r.step(dt)
    b = grmhd.Batch(mixed, dts)
    for _ in range(nsteps):
        b.step()
    torch.cuda.synchronize()
    for r1, r2, s in zip(alone, mixed, setups):
        _close(r1, r2)
        assert r1.fail_count() == r2.fail_count()
    b.close()


def test_batch_result_independent_of_company():
    """a run in a batch of one and the same run inside a mixed batch: the same
    kernels, so the same bits"""
    torch = _torch()
    from paper_2110_03732_amd import grmhd
    setups = _mix(W.SSP3)
    say("batch of one vs mixed batch")
    mixed = [grmhd.Run(s, device="cuda:0") for s in setups]
    dts = [r.dt() for r in mixed]
    b = grmhd.Batch(mixed, dts)
    for _ in range(6):
        b.step()
    for i, s in enumerate(setups):
        r1 = grmhd.Run(s, device="cuda:0")
        b1 = grmhd.Batch([r1], [dts[i]])
        for _ in range(6):
            b1.step()
        torch.cuda.synchronize()
        _same(r1, mixed[i])
        b1.close()
    b.close()


def test_batch_update_membership():
    """runs leave and join a batch through gr_batch_update (no rebuild of the
    batch): each run ends bit for bit where the same run ends in a batch of
    one stepped the same number of times"""
    torch = _torch()
    from paper_2110_03732_amd import grmhd
    setups = _mix(W.SSP3)[:6]
    say("batch membership updates, %d runs" % len(setups))
    runs = [grmhd.Run(s, device="cuda:0") for s in setups]
    dts = [r.dt() for r in runs]
    counts = [0] * len(runs)
    b = grmhd.Batch(runs[:3], dts[:3])
    plan = [([0, 1, 2], 2), ([1, 2, 3, 4], 3), ([0, 5], 1), ([0, 1, 2, 3, 4, 5], 2), ([4], 1)]
    for k, (members, nsteps) in enumerate(plan):
        if k > 0:
            b.update([runs[i] for i in members], [dts[i] for i in members])
        for _ in range(nsteps):
            b.step()
        for i in members:
            counts[i] += nsteps
    torch.cuda.synchronize()
    for i, s in enumerate(setups):
        r1 = grmhd.Run(s, device="cuda:0")
        b1 = grmhd.Batch([r1], [dts[i]])
        for _ in range(counts[i]):
            b1.step()
        torch.cuda.synchronize()
        _same(r1, runs[i])
        assert r1.fail_count() == runs[i].fail_count()
        b1.close()
    b.close()


def test_batch_graph_replays_equal_eager():
    """graph replays, with eager work and synchronisations between them, give
    the eager steps' results after every replay"""
    torch = _torch()
    from paper_2110_03732_amd import grmhd
    setups = _mix(W.SSP3)
    say("graph replay, %d runs" % len(setups))
    ra = [grmhd.Run(s, device="cuda:0") for s in setups]
    rb = [grmhd.Run(s, device="cuda:0") for s in setups]
    dts = [r.dt() for r in ra]
    ba = grmhd.Batch(ra, dts)
    bb = grmhd.Batch(rb, dts)
    for rep in range(3):
        ba.step()
        ba.step()
        bb.run(2)
        junk = torch.ones(1 << 20, dtype=torch.float64, device="cuda:0") * 3.0  # eager work in between
        torch.cuda.synchronize()
        assert float(junk.sum()) == 3.0 * (1 << 20)
        for x, y in zip(ra, rb):
            _same(x, y)
    ba.close()
    bb.close()


def test_batch_run_matches_oracle():
    """every kind of run the batched kernels distinguish -- 1-D/2-D SSP2
    runs, and the SSP3 mix: the 3-D star with its metric, the star on a plane
    and a line, the current sheet, the dynamo (frozen and moving), plus GLM
    and ideal-MHD UCT runs and 3-D boxes with a different boundary rule along
    each direction -- advanced three steps by graph replay inside
    batches, element by element against the oracle (relative L1 1e-10,
    element-wise 1e-9 of each field's scale, as the one-step parity tests)"""
    torch = _torch()
    from paper_2110_03732_amd import grmhd
    groups = [[W.blast_wave(48, eta=1e-2, imex=W.SSP2), W.shock_tube(300, eta=1e-3)]]
    mix3 = _mix(W.SSP3)
    ideal = W.blast_wave(40, eta=1e-6, imex=W.SSP3)
    ideal.uct = 1
    # a different boundary rule along each direction, face fields and GLM
    mix3 += [ideal, W.glm_monopole(33, kappa=5.0, ndim=2, imex=W.SSP3), _mixed_box(W.PPM, W.SSP3),
             _mixed_box(W.PPM, W.SSP3, glm=True)]
    groups.append(mix3)
    for setups in groups:
        say("batch vs oracle: %d runs" % len(setups))
        runs = [grmhd.Run(s, device="cuda:0") for s in setups]
        dts = [r.dt() for r in runs]
        b = grmhd.Batch(runs, dts)
        b.run(3)
        torch.cuda.synchronize()
        for s, r, dt in zip(setups, runs, dts):
            ref = oracle.OracleState(s)
            for _ in range(3):
                ref.step(dt)
            errs = state_errors(s, r.prims(), ref.prim, device_E(r), oracle_E(ref), r.faces(), ref.face)
            bad = [e for e in errs if not (e[1] <= 1e-10 and e[2] <= 1e-9)]
            assert not bad, (s.name, bad)
            assert r.fail_count() == ref.nfail, s.name
        b.close()


def test_batch_autotuner_cache(tmp_path):
    """the tuner writes one decision per class of runs, picks allowed tiles,
    and a second batch reads the cache instead of timing again"""
    torch = _torch()
    from paper_2110_03732_amd import grmhd
    setups = _mix(W.SSP3)
    runs = [grmhd.Run(s, device="cuda:0") for s in setups]
    dts = [r.dt() for r in runs]
    cache = str(tmp_path / "tiles.txt")
    b = grmhd.Batch(runs, dts, tune_cache=cache)
    lines = open(cache).read().split("\n")
    lines = [l for l in lines if l.strip()]
    classes = {(s.recon, s.metric, s.ndim) for s in setups}
    assert len([l for l in lines if l.startswith("xy")]) == len(classes)
    assert len([l for l in lines if l.startswith("cz")]) == len({c for c in classes if c[2] == 3})
    for i, s in enumerate(setups):
        xy, cz = b.tiles(i)
        if s.ndim == 1:
            assert xy.endswith("x1")
        else:
            assert not xy.endswith("x1")
    # tuning launches leave no trace in the results or the failure counters
    ref = [grmhd.Run(s, device="cuda:0") for s in setups]
    bref = grmhd.Batch(ref, dts)  # default tiles, no tuning launches
    b.step()
    bref.step()
    torch.cuda.synchronize()
    for x, y in zip(runs, ref):
        _same(x, y)
        assert x.fail_count() == y.fail_count()
    bref.close()
    before = open(cache).read()
    b2 = grmhd.Batch([grmhd.Run(s, device="cuda:0") for s in setups], dts, tune_cache=cache)
    assert open(cache).read() == before
    for i in range(len(setups)):
        assert b2.tiles(i) == b.tiles(i)
    b.close()
    b2.close()


def test_batch_with_side_stream_fork():
    """a batch holding at least 2^20 cells runs the EMF and face-update
    launches of each pass on the batch's second stream beside the x/y
    sweeps: its runs equal the same runs advanced alone (each below 2^20
    cells, so launched on one stream) to 1e-13 of each field's scale with the
    same failure counts, graph replays equal eager steps bit for bit, and the
    star matches the oracle"""
    torch = _torch()
    from paper_2110_03732_amd import grmhd
    setups = [W.blast_wave(768, eta=1e-6), W.tov_star(64), W.blast_wave(512, eta=1e-2)]
    assert sum(s.ncells for s in setups) >= 1 << 20
    assert all(s.ncells < 1 << 20 for s in setups)
    say("forked batch: %s" % [s.ncells for s in setups])
    ra = [grmhd.Run(s, device="cuda:0") for s in setups]
    rb = [grmhd.Run(s, device="cuda:0") for s in setups]
    alone = [grmhd.Run(s, device="cuda:0") for s in setups]
    dts = [r.dt() for r in ra]
    ba = grmhd.Batch(ra, dts)
    bb = grmhd.Batch(rb, dts)
    for _ in range(3):
        ba.step()
    bb.run(3)
    for r, dt in zip(alone, dts):
        for _ in range(3):
            r.step(dt)
    torch.cuda.synchronize()
    for x, y, z in zip(ra, rb, alone):
        _same(x, y)
        _close(x, z)
        assert x.fail_count() == z.fail_count()
    s = setups[1]
    ref = oracle.OracleState(s)
    for _ in range(3):
        ref.step(dts[1])
    r = ra[1]
    errs = state_errors(s, r.prims(), ref.prim, device_E(r), oracle_E(ref), r.faces(), ref.face)
    bad = [e for e in errs if not (e[1] <= 1e-10 and e[2] <= 1e-9)]
    assert not bad, bad
    assert r.fail_count() == ref.nfail
    # a membership update that takes the batch below 2^20 cells (its passes
    # then launch on one stream), then back above it
    small = [ra[0], ra[1]]
    assert sum(x.setup.ncells for x in small) < 1 << 20
    ba.update(small, dts[:2])
    ba.step()
    ba.update(ra, dts)
    ba.step()
    for i, z in enumerate(alone):
        for _ in range(2 if i < 2 else 1):
            z.step(dts[i])
    torch.cuda.synchronize()
    for x, z in zip(ra, alone):
        _close(x, z)
        assert x.fail_count() == z.fail_count()
    ba.close()
    bb.close()


def test_batch_forks_only_in_graph():
    """a batch of 2^18 to 2^20 cells forks its EMF and face-update launches
    only when captured (gr_batch_run), not in eager steps: the two give the
    same runs bit for bit"""
    torch = _torch()
    from paper_2110_03732_amd import grmhd
    setups = [W.blast_wave(512, eta=1e-2), W.tov_star(48)]
    assert 1 << 18 <= sum(s.ncells for s in setups) < 1 << 20
    say("batch forked in graph only: %s" % [s.ncells for s in setups])
    ra = [grmhd.Run(s, device="cuda:0") for s in setups]
    rb = [grmhd.Run(s, device="cuda:0") for s in setups]
    dts = [r.dt() for r in ra]
    ba = grmhd.Batch(ra, dts)
    bb = grmhd.Batch(rb, dts)
    for _ in range(3):
        ba.step()
    bb.run(3)
    torch.cuda.synchronize()
    for x, y in zip(ra, rb):
        _same(x, y)
        assert x.fail_count() == y.fail_count()
    ba.close()
    bb.close()


def test_batch_set_dt_and_tiles():
    """gr_batch_set_dt gives every run a new time step: the steps after it
    equal, bit for bit, those of a batch given the same steps by
    gr_batch_update (eager, and as a graph captured again after the change),
    and the runs advanced alone to 1e-13; gr_batch_tiles names the tiles of
    every run"""
    import re
    torch = _torch()
    from paper_2110_03732_amd import grmhd
    setups = [W.blast_wave(48, eta=1e-2), W.shock_tube(200, imex=W.SSP3), W.tov_star(20)]
    say("set_dt batch: %s" % [s.ncells for s in setups])
    ra, rb, rc, alone = ([grmhd.Run(s, device="cuda:0") for s in setups] for _ in range(4))
    dt1 = [r.dt() for r in ra]
    dt2 = [0.5 * d for d in dt1]
    ba, bb, bc = grmhd.Batch(ra, dt1), grmhd.Batch(rb, dt1), grmhd.Batch(rc, dt1)
    ba.run(2)
    bb.run(2)
    bc.step()
    bc.step()
    ba.set_dt(dt2)
    bb.update(rb, dt2)
    bc.set_dt(dt2)
    ba.run(2)
    for _ in range(2):
        bb.step()
        bc.step()
    for r, d1, d2 in zip(alone, dt1, dt2):
        for dt in (d1, d1, d2, d2):
            r.step(dt)
    torch.cuda.synchronize()
    for x, y, z, w in zip(ra, rb, rc, alone):
        _same(x, y)
        _same(z, y)
        _close(x, w)
        assert x.fail_count() == w.fail_count()
        assert abs(x.t - w.t) <= 1e-15 * w.t
    for i in range(len(setups)):
        for name in ba.tiles(i):
            assert re.fullmatch(r"\d+x\d+", name), name
    with pytest.raises(ValueError):
        ba.set_dt(dt2[:2])
    with pytest.raises(grmhd.GrError):  # GR_EINVAL: a step that is not positive
        ba.set_dt([dt2[0], 0.0, dt2[2]])
    assert ba.dts == dt2
    for b in (ba, bb, bc):
        b.close()
