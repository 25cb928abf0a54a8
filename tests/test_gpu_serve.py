"""Continuous-batching request loop: every request's result is the same
alone and in the mix, under an HBM budget small enough that requests queue,
join and leave the batch at different times.  Alone = the request served by
itself (the same batched kernels: exact) and the request stepped through the
single-grid path (separately compiled kernels: within 1e-13 of each field's
scale).  Every served result is also compared with the CPU oracle run for
the same steps (relative L1 <= 1e-10 and element-wise <= 1e-9 of each
field's scale, as the one-step parity tests; the requests take 2-9 steps)."""
import sys

import numpy as np
import pytest

import oracle
import workloads as W
from parity import state_errors

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch


def test_served_equals_alone():
    torch = _torch()
    from paper_2110_03732_amd import grmhd, serve
    trace = W.served_trace(10, rate=400.0, seed=11, blast=(24, 56), star=(14, 22), steps=(2, 9))
    payloads = {r["rid"]: W.make_run_setup(r, imex=W.SSP3) for r in trace}
    biggest = max(serve.run_bytes(grmhd.grid_of(s)) for s in payloads.values())
    budget = 3 * biggest
    print("trace of %d requests, budget %d bytes" % (len(trace), budget), flush=True)
    srv = serve.Server(budget, chunk=3, keep=True)
    recs, summary = srv.serve(trace, lambda r: payloads[r["rid"]])
    assert summary["requests"] == len(trace)
    assert summary["peak_resident_bytes"] <= budget
    assert summary["p50_latency_s"] is not None and summary["p99_latency_s"] >= summary["p50_latency_s"]
    assert len({r["admit"] for r in recs}) > 1  # requests joined at different times
    for rec in recs:
        req = trace[rec["rid"]]
        s = payloads[rec["rid"]]
        solo = serve.Server(budget, chunk=3, keep=True)
        one, _ = solo.serve([dict(req, arrival=0.0)], lambda r: payloads[r["rid"]])
        assert np.array_equal(one[0]["prims"], rec["prims"]), rec["rid"]
        assert np.array_equal(one[0]["faces"], rec["faces"]), rec["rid"]
        assert one[0]["fails"] == rec["fails"]
        run = grmhd.Run(s, device="cuda:0")
        dt = run.dt()
        for _ in range(req["steps"]):
            run.step(dt)
        torch.cuda.synchronize()
        for got, want in ((run.prims(), rec["prims"]), (run.faces(), rec["faces"])):
            for f in range(got.shape[0]):
                assert np.abs(got[f] - want[f]).max() <= 1e-13 * max(np.abs(want[f]).max(), 1e-300), rec["rid"]
        assert run.fail_count() == rec["fails"]
        assert rec["latency"] > 0.0 and rec["done"] >= rec["admit"] >= rec["arrival"] - 1e-9
        # the served result against the oracle
        ref = oracle.OracleState(s)
        for _ in range(req["steps"]):
            ref.step(dt)
        ps6 = 1.0 if not s.metric else s.psi ** 6
        Eg = rec["cons"][5:8] / ps6
        Er = np.stack([ref.q[5 + i] / ps6 for i in range(3)])
        errs = state_errors(s, rec["prims"], ref.prim, Eg, Er, rec["faces"], ref.face)
        bad = [e for e in errs if not (e[1] <= 1e-10 and e[2] <= 1e-9)]
        assert not bad, (rec["rid"], bad)
        assert rec["fails"] == ref.nfail


def test_serve_edge_cases():
    """an empty trace, a request of zero steps (finishes with its initial
    state), a request larger than the whole budget (refused)"""
    _torch()
    from paper_2110_03732_amd import grmhd, serve
    srv = serve.Server(1 << 30, chunk=2, keep=True)
    recs, summary = srv.serve([], lambda r: None)
    assert recs == [] and summary["requests"] == 0 and summary["p50_latency_s"] is None
    s = W.blast_wave(24, eta=1e-2, imex=W.SSP2)
    req = {"rid": 0, "arrival": 0.0, "steps": 0}
    recs, summary = srv.serve([req], lambda r: s)
    assert summary["requests"] == 1 and recs[0]["fails"] == 0
    ref = grmhd.Run(s, device="cuda:0")
    assert np.array_equal(recs[0]["prims"], ref.prims()) and np.array_equal(recs[0]["faces"], ref.faces())
    tiny = serve.Server(1024, chunk=2)
    with pytest.raises(ValueError):
        tiny.serve([dict(req, steps=3)], lambda r: s)
