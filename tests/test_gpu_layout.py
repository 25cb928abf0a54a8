"""The padded device layout of the C ABI, and the paired point-wise passes
of a whole step.  Layout: the points between rows (and before the origin,
after the last row) are neither read nor written by any call.  Padding of the
caller's q, face, prim and metric fields is set to NaN after initialisation;
after a few steps, a recovery, the reductions and the elliptic cleaning it is
still NaN (never written) and every result equals, bit for bit, that of a run
with zero padding (never read)."""
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


PAIR_CASES = {
    "star_3d_24": lambda: W.tov_star(24),
    "blast_2d_40_ssp3_stiff": lambda: W.blast_wave(40, eta=1e-6),
    "shock_tube_1d_200_ssp3": lambda: W.shock_tube(200, imex=W.SSP3),
    "dynamo_xi_ssp3": lambda: _with(W.blast_wave(32, eta=1e-2), xi=0.05),
    "star_2d_33_ssp3": lambda: W.tov_star(33, ndim=2),
}


@pytest.mark.parametrize("name", sorted(PAIR_CASES))
def test_whole_step_equals_stage_by_stage(name):
    """gr_step runs the two point-wise passes of IMEX-SSP3(4,3,3) (stages 0
    and 1) as one launch; the result equals the stage-by-stage calls (same
    arithmetic, compiled in another instance: 1e-13 of each field's scale)
    with the same failure count"""
    torch = _torch()
    from paper_2110_03732_amd import grmhd
    print("pair case %s" % name, flush=True)
    s = PAIR_CASES[name]()
    assert s.imex == W.SSP3
    a = grmhd.Run(s, device="cuda:0")
    b = grmhd.Run(s, device="cuda:0")
    dt = a.dt()
    for _ in range(3):
        a.step(dt)
        for p in range(5):
            b.stage(p, dt)
    torch.cuda.synchronize()
    for x, y in ((a.prims(), b.prims()), (a.cons(), b.cons()), (a.faces(), b.faces())):
        for f in range(x.shape[0]):
            sc = max(np.abs(y[f]).max(), 1e-300)
            assert np.abs(x[f] - y[f]).max() <= 1e-13 * sc, f
    assert a.fail_count() == b.fail_count()


def test_batch_step_pairs_the_point_wise_passes():
    """one step of a batch holding one IMEX-SSP3 star: pass 0 (with pass 1
    inside it) launches the cell pass only, passes 2-4 launch the x/y sweeps,
    three EMF directions, face update and cell pass: 19 launches (20 with the
    passes run one by one); a GLM run is never paired"""
    _torch()
    from paper_2110_03732_amd import grmhd
    s = W.tov_star(16)
    run = grmhd.Run(s, device="cuda:0")
    b = grmhd.Batch([run], [run.dt()])
    assert b.stats()[0] == 19
    b.close()
    g = W.glm_monopole(16, kappa=1.0, ndim=3, imex=W.SSP3)
    rg = grmhd.Run(g, device="cuda:0")
    bg = grmhd.Batch([rg], [rg.dt()])
    # GLM: no EMF and face launches; passes 0 and 1 one by one
    assert bg.stats()[0] == 1 + 1 + 3 * 2
    bg.close()


GHOST_CASES = {
    "blast_2d_37_outflow_mc": lambda: W.blast_wave(37, eta=1e-2, recon=W.MC, imex=W.SSP2),
    "loop_2d_40x20_periodic": lambda: W.loop_advection(40, 20),
    "star_3d_20_outflow": lambda: W.tov_star(20),
    "star_3d_17_uct_ideal": lambda: _with(W.tov_star(17), uct=1),
    "shock_tube_1d_101_ppm_ssp3": lambda: W.shock_tube(101, recon=W.PPM, imex=W.SSP3),
    "glm_monopole_2d_33": lambda: W.glm_monopole(33, kappa=5.0, ndim=2),
    "dynamo_1d_periodic": lambda: W.steady_dynamo(64, k=1),
    # periodic as small as the ghost width, a one-cell-thick active
    # direction, ragged tiles in every direction
    "box_3d_3x3x3_periodic_ppm_ssp3": lambda: _parity_case("box_3d_3x3x3_periodic_ppm_ssp3"),
    "box_3d_12x9x1_outflow_mc": lambda: _parity_case("box_3d_12x9x1_outflow_mc"),
    "star_13x11x9_ragged": lambda: _parity_case("star_13x11x9_ragged"),
}


def _parity_case(name):
    import test_gpu_parity
    return test_gpu_parity.CASES[name]()


def _ghost_mask(run, face_dir=None):
    """True on the ghost points of one device field (points of the padded box
    outside the interior; for the face field of normal face_dir the
    boundary faces g + n along it are evolved, not ghosts)"""
    s = run.setup
    Nz, Ny, Nx = s.shape
    g = s.ng
    lo, hi = [0, 0, 0], [Nx, Ny, Nz]
    for d in range(3):
        if s.active(d):
            n = (Nx, Ny, Nz)[d] - 2 * g
            lo[d], hi[d] = g, g + n + (1 if d == face_dir else 0)
    m = np.zeros(run.fs, dtype=bool)
    z, y, x = np.meshgrid(np.arange(Nz), np.arange(Ny), np.arange(Nx), indexing="ij")
    ghost = ~((x >= lo[0]) & (x < hi[0]) & (y >= lo[1]) & (y < hi[1]) & (z >= lo[2]) & (z < hi[2]))
    idx = run.origin + x + run.pitch * (y + Ny * z)
    m[idx[ghost]] = True
    return m


@pytest.mark.parametrize("name", sorted(GHOST_CASES))
def test_ghost_points_never_read_or_written(name):
    """outflow and periodic grids: every ghost point of the state (q, faces,
    primitives) and of the workspace stage blocks set to NaN after
    initialisation; three steps and the cleaning give the clean run's results
    bit for bit (no kernel reads a ghost point of a stage field: the
    boundary maps give every such read its interior point; the one ghost
    layer of the stage E the cell pass reads is written in the pass before
    it is read), and the state's ghost points are still NaN"""
    torch = _torch()
    from paper_2110_03732_amd import grmhd
    print("ghost case %s" % name, flush=True)
    s = GHOST_CASES[name]()
    assert all(b != W.FIXED for side in s.bc for b in side)
    clean = grmhd.Run(s, device="cuda:0")
    dirty = grmhd.Run(s, device="cuda:0")
    dev = dirty.q.device
    cell = torch.from_numpy(_ghost_mask(dirty)).to(dev)
    face = [torch.from_numpy(_ghost_mask(dirty, None if s.glm else d)).to(dev) for d in range(3)]
    torch.cuda.synchronize()
    state = [(dirty.q.view(dirty.nq, dirty.fs), [cell] * dirty.nq), (dirty.prim.view(5, dirty.fs), [cell] * 5),
             (dirty.face.view(3, dirty.fs), face)]
    for t, masks in state:
        for f, m in enumerate(masks):
            t[f][m] = float("nan")
    nstage = 4 if s.imex == W.SSP3 else 2
    for j in range(nstage):
        for f in range(10 if s.glm else 8):
            off = grmhd.gr_workspace_offset(dirty.grid, 0, j, f) // 8
            dirty.work[off: off + dirty.fs][cell] = float("nan")
        for d in range(3):
            off = grmhd.gr_workspace_offset(dirty.grid, 1, j, d) // 8
            dirty.work[off: off + dirty.fs][face[d]] = float("nan")
    torch.cuda.synchronize()
    dt = clean.dt()
    assert dirty.dt() == dt
    for _ in range(3):
        clean.step(dt)
        dirty.step(dt)
    if not s.glm:
        assert np.array_equal(clean.clean_divB(2)[1], dirty.clean_divB(2)[1])
    assert np.array_equal(clean.divB(), dirty.divB())
    assert clean.fail_count() == dirty.fail_count()
    sl = s.interior
    for a, b in ((clean.prims(), dirty.prims()), (clean.cons(), dirty.cons())):
        assert np.array_equal(a[(slice(None),) + sl], b[(slice(None),) + sl])
    # faces compared on the device layout: every evolved face
    torch.cuda.synchronize()
    for d in range(3):
        keep = ~face[d].cpu().numpy() & ~_pad_mask(dirty)
        a = clean.face.view(3, clean.fs)[d].cpu().numpy()[keep]
        b = dirty.face.view(3, dirty.fs)[d].cpu().numpy()[keep]
        assert np.array_equal(a, b), d
        assert np.all(np.isnan(dirty.face.view(3, dirty.fs)[d].cpu().numpy()[face[d].cpu().numpy()])), "ghost face written"
    for t, nf in ((dirty.q, dirty.nq), (dirty.prim, 5)):
        g = t.view(nf, dirty.fs)[:, cell].cpu().numpy()
        assert np.all(np.isnan(g)), "ghost point of the state written"
