"""A whole step (gr_step) captured into a HIP graph from a caller's stream.

The capture holds every launch of the step; on a grid of 2^18 cells or more
it also holds the fork of the EMF and face-update launches to the library's
second stream and the join back (eager steps fork from 2^20 cells, so the
512^2 plane compares a forked graph with a one-stream eager step).  Each
replay must give the eager step's result bit for bit (the same kernels on the
same inputs), also with eager work and synchronisations between the replays.
"""
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("name", ["tov_star_104_forked", "blast_512_forked_in_graph", "blast_64_one_stream",
                                  "shock_tube_400_one_stream"])
def test_captured_step_replays_equal_eager(name):
    torch = _torch()
    from paper_2110_03732_amd import grmhd
    if name.startswith("tov"):
        s = W.tov_star(104)
        assert s.ncells >= 1 << 20
    elif name.startswith("blast_512"):
        s = W.blast_wave(512, eta=1e-2)
        assert 1 << 18 <= s.ncells < 1 << 20
    elif name.startswith("blast"):
        s = W.blast_wave(64, eta=1e-2)
    else:
        s = W.shock_tube(400)
    say("captured step %s (%d cells)" % (name, s.ncells))
    eager = grmhd.Run(s, device="cuda:0")
    graphed = grmhd.Run(s, device="cuda:0")
    dt = eager.dt()
    g = torch.cuda.CUDAGraph()
    cap = torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=cap):
        grmhd.gr_step(graphed.grid, graphed.state, dt, cap.cuda_stream)
    torch.cuda.synchronize()
    for rep in range(4):
        eager.step(dt)
        g.replay()
        junk = torch.ones(1 << 20, dtype=torch.float64, device="cuda:0") * 3.0  # eager work in between
        torch.cuda.synchronize()
        assert float(junk.sum()) == 3.0 * (1 << 20)
        for x, y, what in ((eager.prims(), graphed.prims(), "prim"), (eager.faces(), graphed.faces(), "face"),
                           (eager.cons(), graphed.cons(), "cons")):
            assert np.array_equal(x, y), (rep, what)
        assert eager.fail_count() == graphed.fail_count()
