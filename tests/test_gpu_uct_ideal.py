"""The ideal-MHD edge EMF (App. A) in batches: runs with the resistive and
the ideal-MHD EMF share one batch, each within 1e-13 of its single-grid
result (separately compiled kernels); one-step and 100-step parity with the
oracle is in test_gpu_parity.py (the *_uct_ideal cases)."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch


def _with(s, **kw):
    for k, v in kw.items():
        setattr(s, k, v)
    return s


def test_uct_ideal_in_batch_matches_plain():
    torch = _torch()
    from paper_2110_03732_amd import grmhd
    print("batch of resistive and ideal-MHD edge EMFs", flush=True)
    setups = [_with(W.blast_wave(40, eta=1e-2, imex=W.SSP2), uct=1), W.blast_wave(32, eta=1e-2, imex=W.SSP2),
              _with(W.shock_tube(300), uct=1), _with(W.loop_advection(48, 24), uct=1), W.shock_tube(200)]
    runs = [grmhd.Run(s, device="cuda:0") for s in setups]
    dts = [r.dt() for r in runs]
    b = grmhd.Batch(runs, dts)
    b.run(5)
    torch.cuda.synchronize()
    for s, r, dt in zip(setups, runs, dts):
        p = grmhd.Run(s, device="cuda:0")
        for _ in range(5):
            p.step(dt)
        for got, want in ((r.prims(), p.prims()), (r.faces(), p.faces()), (r.cons(), p.cons())):
            for f in range(got.shape[0]):
                assert np.abs(got[f] - want[f]).max() <= 1e-13 * max(np.abs(want[f]).max(), 1e-300), (s.name, f)
        assert r.divB()[2] <= 1e-12
    b.close()
