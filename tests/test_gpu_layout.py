"""The padded device layout of the C ABI: the points between rows (and
before the origin, after the last row) are neither read nor written by any
call.  Padding of the caller's q, face, prim and metric fields is set to NaN
after initialisation; after a few steps, a recovery, the reductions and the
elliptic cleaning it is still NaN (never written) and every result equals,
bit for bit, that of a run with zero padding (never read)."""
import math

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch


def _pad_mask(run):
    """True on the padding points of one device field of fs doubles"""
    Nz, Ny, Nx = run.setup.shape
    m = np.ones(run.fs, dtype=bool)
    for r in range(Ny * Nz):
        a = run.origin + r * run.pitch
        m[a: a + Nx] = False
    return m


CASES = {
    "star_3d_20": lambda: W.tov_star(20),
    "blast_2d_37": lambda: W.blast_wave(37, eta=1e-2, imex=W.SSP2),
    "shock_tube_1d_101_ppm": lambda: W.shock_tube(101, recon=W.PPM, imex=W.SSP3),
    "glm_monopole_2d_33": lambda: W.glm_monopole(33, kappa=5.0, ndim=2),
    "star_3d_17_uct_ideal": lambda: _with(W.tov_star(17), uct=1),
}


def _with(s, **kw):
    for k, v in kw.items():
        setattr(s, k, v)
    return s


@pytest.mark.parametrize("name", sorted(CASES))
def test_padding_never_read_or_written(name):
    torch = _torch()
    from paper_2110_03732_amd import grmhd
    print("layout case %s" % name, flush=True)
    s = CASES[name]()
    clean = grmhd.Run(s, device="cuda:0")
    dirty = grmhd.Run(s, device="cuda:0")
    mask = torch.from_numpy(_pad_mask(dirty)).to(dirty.q.device)
    fields = [(dirty.q, dirty.nq), (dirty.face, 3), (dirty.prim, 5)]
    if dirty.metric is not None:
        fields.append((dirty.metric, 2))
    torch.cuda.synchronize()
    for t, nf in fields:
        v = t.view(nf, dirty.fs)
        v[:, mask] = float("nan")
    torch.cuda.synchronize()
    dt = clean.dt()
    assert dirty.dt() == dt
    for _ in range(3):
        clean.step(dt)
        dirty.step(dt)
    clean.con2prim()
    dirty.con2prim()
    if not s.glm:
        assert np.array_equal(clean.clean_divB(2)[1], dirty.clean_divB(2)[1])
    assert np.array_equal(clean.divB(), dirty.divB())
    assert clean.fail_count() == dirty.fail_count()
    for a, b in ((clean.prims(), dirty.prims()), (clean.cons(), dirty.cons()), (clean.faces(), dirty.faces())):
        assert np.array_equal(a, b)
        assert np.all(np.isfinite(b))
    torch.cuda.synchronize()
    for t, nf in fields:
        pad = t.view(nf, dirty.fs)[:, mask].cpu().numpy()
        assert np.all(np.isnan(pad)), "padding written"
    assert math.isfinite(dt)
