"""The allocation-free divergence norm (gr_divB_norm_noalloc) against
gr_divB_norm through the C ABI: the same three norms, bit for bit, on two
calls in a row -- a 3-D star, then a smaller 2-D blast wave (the shared
device array keeps the first call's partials; the second must not see them)
-- with the state's workspace pointer cleared for the allocation-free call."""
import ctypes

import numpy as np
import pytest

import workloads as W
from parity import say

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch


def _norms(run, fn, torch, state):
    out = torch.full((3,), -1.0, dtype=torch.float64, device=run.q.device)
    fn(run.grid, state, out.data_ptr(), run.stream.cuda_stream)
    run.stream.synchronize()
    return out.cpu().numpy()


def test_divb_norm_noalloc_matches_workspace_form():
    torch = _torch()
    from paper_2110_03732_amd import grmhd
    cases = [W.tov_star(40), W.blast_wave(48, eta=1e-2)]
    cases[1].face = np.zeros((3,) + cases[1].shape)
    cases[1].face[0] = 1e-3 * W.uniform_pm1(5, 1, int(np.prod(cases[1].shape))).reshape(cases[1].shape)
    for k, s in enumerate(cases):
        say("no-alloc div B norm, call %d: %s %s" % (k, s.name, s.n))
        run = grmhd.Run(s, device="cuda:0")
        if k == 0:
            for _ in range(2):
                run.step(run.dt())
        want = _norms(run, grmhd.gr_divB_norm, torch, run.state)
        bare = grmhd.gr_state()
        ctypes.memmove(ctypes.addressof(bare), ctypes.addressof(run.state), ctypes.sizeof(bare))
        bare.work = None
        bare.work_bytes = 0
        got = _norms(run, grmhd.gr_divB_norm_noalloc, torch, bare)
        say("  workspace %s, allocation-free %s" % (want, got))
        assert np.all(want >= 0.0)
        assert np.array_equal(got, want)
        if k == 1:
            assert want[2] > 1e-6  # the planted divergence is seen
