"""Pins of the oracle's elliptic divergence cleaning (Sec 3.3): a pure
gradient is removed completely, a curl is left alone, the result is
divergence-free to round-off, the correction is an orthogonal projection
(Pythagoras in the face inner product, idempotent), and the edge
circulations (the discrete curl) do not change."""
import numpy as np
import pytest

import workloads as W
from oracle import clean as C


def _setups():
    return [
        ("1d_outflow", W.shock_tube(40)),
        ("2d_outflow", W.blast_wave(24)),
        ("2d_ragged_outflow", W.Setup("r", 2, (19, 13, 1), 2, (0, 0, 0), (1.9, 1.0, 1), W._bc(2, W.OUTFLOW), 2.0,
                                      W.MC, W.SSP2)),
        ("2d_periodic", W.loop_advection(20, 10)),
        ("3d_outflow", W.Setup("c", 3, (9, 8, 7), 2, (0, 0, 0), (0.9, 0.8, 0.7), W._bc(3, W.OUTFLOW), 2.0, W.MC,
                               W.SSP2)),
    ]


def _random_faces(s, seed):
    rng = np.random.default_rng(seed)
    f = np.zeros((3,) + s.shape)
    for d in range(3):
        f[d] = rng.normal(size=s.shape)
    return f


def _mask(s):
    """face points the cleaning acts on: faces g .. g+n of active d, interior
    in the other directions"""
    m = np.zeros((3,) + s.shape, dtype=bool)
    for d in range(3):
        sl = [slice(s.g(2), s.g(2) + s.nn(2)), slice(s.g(1), s.g(1) + s.nn(1)), slice(s.g(0), s.g(0) + s.nn(0))]
        if s.active(d):
            sl[2 - d] = slice(s.g(d), s.g(d) + s.nn(d) + 1)
        m[d][tuple(sl)] = True
    return m


@pytest.mark.parametrize("name,s", _setups())
def test_pure_gradient_is_removed(name, s):
    rng = np.random.default_rng(3)
    phi = rng.normal(size=(s.nn(2), s.nn(1), s.nn(0)))
    f = C.gradient_faces(s, phi)
    f2, phi2 = C.clean(s, f)
    scale = np.abs(f).max()
    assert np.abs(f2[_mask(s)]).max() <= 1e-11 * scale
    per = all(s.bc[d][0] == W.PERIODIC for d in range(s.ndim))
    if per:
        phi2 = phi2 - phi2.mean() + phi.mean()
    assert np.abs(phi2 - phi).max() <= 1e-10 * np.abs(phi).max()


@pytest.mark.parametrize("name,s", _setups())
def test_divergence_free_after_and_projection(name, s):
    f = _random_faces(s, 5)
    if all(s.bc[d][0] == W.PERIODIC for d in range(s.ndim)):
        # periodic images: the last face of a periodic direction is the first one
        for d in range(s.ndim):
            ax = 2 - d
            a = np.moveaxis(f[d], ax, 0)
            a[s.g(d) + s.nn(d)] = a[s.g(d)]
    m = _mask(s)
    div0 = np.abs(C.divergence(s, f)).max()
    f2, _ = C.clean(s, f)
    assert np.abs(C.divergence(s, f2)).max() <= 1e-12 * div0
    g = f - f2
    # orthogonal projection: |f|^2 = |f2|^2 + |g|^2 with the face weights
    # dx_d of the inner product sum_f q_B^d(f) p_B^d(f) V_cell; the two
    # boundary faces of a direction carry half the cell weight each
    w = np.zeros_like(f)
    for d in range(3):
        w[d][m[d]] = 1.0
        if s.active(d):
            ax = 2 - d
            wd = np.moveaxis(w[d], ax, 0)
            if s.bc[d][0] != W.PERIODIC:
                wd[s.g(d)] *= 0.5
                wd[s.g(d) + s.nn(d)] *= 0.5
            else:
                wd[s.g(d) + s.nn(d)] = 0.0  # the periodic image face counts once
    n2 = lambda a: float((w * a * a).sum())
    assert n2(f) == pytest.approx(n2(f2) + n2(g), rel=1e-12)
    f3, _ = C.clean(s, f2)
    assert np.abs(f3 - f2)[m].max() <= 1e-12 * np.abs(f2[m]).max()


def test_curl_is_left_alone_and_circulation_kept():
    s = W.Setup("c", 3, (9, 8, 7), 2, (0, 0, 0), (0.9, 0.8, 0.7), W._bc(3, W.OUTFLOW), 2.0, W.MC, W.SSP2)
    rng = np.random.default_rng(11)
    dx = [s.dx(d) for d in range(3)]
    # faces = discrete curl of a random edge potential (divergence-free)
    A = [rng.normal(size=s.shape) for _ in range(3)]
    f = np.zeros((3,) + s.shape)
    for d in range(3):
        m1, m2 = (d + 1) % 3, (d + 2) % 3
        f[d] = (np.roll(A[m2], -1, axis=2 - m1) - A[m2]) / dx[m1] - (np.roll(A[m1], -1, axis=2 - m2) - A[m1]) / dx[m2]
    m = _mask(s)
    f = np.where(m, f, 0.0)
    # only the faces inside the mask are kept: the curl is then exact on the
    # interior cells whose faces all lie in it
    div0 = np.abs(C.divergence(s, f)).max()
    assert div0 <= 1e-10 * np.abs(f).max()
    f2, phi = C.clean(s, f)
    assert np.abs(f2 - f)[m].max() <= 1e-9 * np.abs(f).max()
    # random faces: the circulation around every interior z-edge is unchanged
    g = _random_faces(s, 2)
    g = np.where(m, g, 0.0)
    g2, _ = C.clean(s, g)
    sl = (slice(s.g(2), s.g(2) + s.nn(2)), slice(s.g(1) + 1, s.g(1) + s.nn(1)), slice(s.g(0) + 1, s.g(0) + s.nn(0)))

    def circ(h):  # d_x B^y - d_y B^x at interior z-edges
        bx, by = h[0], h[1]
        return (by - np.roll(by, 1, axis=2)) / dx[0] - (bx - np.roll(bx, 1, axis=1)) / dx[1]
    assert np.abs(circ(g2)[sl] - circ(g)[sl]).max() <= 1e-10 * np.abs(circ(g)[sl]).max()
