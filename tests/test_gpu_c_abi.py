"""The library driven from plain C (tests/c_abi/abi_smoke.c: hipMalloc, the C
ABI, no PyTorch): the 400-cell shock tube to t = 0.4 runs without error, and
its final primitives are bit-identical to the same run through the Python
binding (same library, same kernels, same inputs)."""
import math
import os
import subprocess
import tempfile

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EXE = os.path.join(ROOT, "tests", "c_abi", "abi_smoke")


def _setup():
    """the C program's problem, built the same way"""
    s = W._blank(W.Setup("c_abi_shock_tube", 1, (400, 1, 1), 2, (-0.5, 0, 0), (0.5, 1, 1), W._bc(1, W.OUTFLOW), 2.0,
                         W.MINMOD, W.SSP2, eta=1e-3, rho_atm=1e-14, p_atm=1e-14))
    X, _, _ = s.mesh()
    left = X < 0.0
    s.prim[0] = np.where(left, 1.0, 0.125)
    s.prim[4] = np.where(left, 1.0, 0.1)
    s.face = np.zeros((3,) + s.shape)
    s.face[0] = 0.5
    s.face[1] = np.where(left, 0.5, -0.5)
    return s


def test_c_program_matches_python_binding():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    assert os.path.exists(EXE), "tests/c_abi/abi_smoke is not built (run __graft_entry__.build())"
    from paper_2110_03732_amd import grmhd
    with tempfile.TemporaryDirectory() as d:
        out = os.path.join(d, "prims.bin")
        r = subprocess.run([EXE, out], capture_output=True, text=True, timeout=120)
        print(r.stdout, r.stderr, flush=True)
        assert r.returncode == 0, r.stderr
        got = np.fromfile(out, dtype=np.float64).reshape(5, 400)
    s = _setup()
    run = grmhd.Run(s, device="cuda:0")
    dt = run.dt()
    nsteps = int(0.4 / dt + 0.5)
    for _ in range(nsteps):
        run.step(dt)
    want = run.prims()[:, 0, 0, s.g(0):s.g(0) + 400]
    assert np.array_equal(got, want)
    assert math.isclose(float(want[0].max()), 1.0, rel_tol=0.05) and want[0].min() > 0.1
