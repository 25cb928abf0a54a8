"""Elliptic divergence cleaning of the face fields (Sec 3.3, eq. poisson and
eq. update_bfield), the plain definition written out with numpy/scipy.

TEST INFRASTRUCTURE ONLY, like the rest of `oracle/`: only the test-suite
and the benchmark's CPU leg may import it.

Discrete form on the staggered mesh (interior cells c, active directions d):
  div(c)  = sum_d (q_B^d(c + e_d) - q_B^d(c)) / dx_d
  L Phi(c) = sum_d (Phi(c + e_d) - 2 Phi(c) + Phi(c - e_d)) / dx_d^2
  q_B^d(f) <- q_B^d(f) - (Phi(c) - Phi(c - e_d)) / dx_d   on every d-face f
              of the interior, both boundary faces included,
with Phi outside the domain equal to -Phi of the boundary cell (Phi = 0 on
the boundary face: the paper states no boundary rule for Phi; with this one
every divergence is removable) or the periodic image.  L Phi = div is solved
by a sparse direct solve; with every direction periodic the constant null
space is fixed by Phi = 0 in the first cell (the system is consistent: the
periodic divergence sums to zero).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

PERIODIC = 1


def _geom(s):
    act = [s.active(d) for d in range(3)]
    n = [s.nn(d) for d in range(3)]
    g = [s.g(d) for d in range(3)]
    dx = [s.dx(d) if act[d] else 1.0 for d in range(3)]
    per = [act[d] and s.bc[d][0] == PERIODIC for d in range(3)]
    return act, n, g, dx, per


def _interior(faces, s):
    sl = s.interior
    return sl


def divergence(s, faces):
    """div(c) on the interior cells, shape (nz, ny, nx)"""
    act, n, g, dx, _ = _geom(s)
    out = np.zeros((n[2], n[1], n[0]))
    for d in range(3):
        if not act[d]:
            continue
        lo = [slice(g[2], g[2] + n[2]), slice(g[1], g[1] + n[1]), slice(g[0], g[0] + n[0])]
        hi = list(lo)
        ax = 2 - d
        hi[ax] = slice(g[d] + 1, g[d] + n[d] + 1)
        out += (faces[d][tuple(hi)] - faces[d][tuple(lo)]) / dx[d]
    return out


def laplacian(s):
    """sparse L on the interior cells (row index i + nx (j + ny k))"""
    act, n, g, dx, per = _geom(s)
    N = n[0] * n[1] * n[2]
    idx = np.arange(N).reshape(n[2], n[1], n[0])
    rows, cols, vals = [], [], []
    diag = np.zeros(N)
    for d in range(3):
        if not act[d]:
            continue
        h2 = 1.0 / dx[d] ** 2
        ax = 2 - d
        diag -= 2.0 * h2
        for sgn in (+1, -1):
            nb = np.roll(idx, -sgn, axis=ax)  # neighbour c + sgn e_d (wrapped)
            pos = np.arange(n[d])
            inside = (pos + sgn >= 0) & (pos + sgn < n[d])
            shape = [1, 1, 1]
            shape[ax] = n[d]
            inside = np.broadcast_to(inside.reshape(shape), idx.shape)
            if per[d]:
                rows.append(idx.ravel())
                cols.append(nb.ravel())
                vals.append(np.full(N, h2))
            else:
                rows.append(idx[inside])
                cols.append(nb[inside])
                vals.append(np.full(int(inside.sum()), h2))
                diag[idx[~inside]] -= h2  # Phi(outside) = -Phi(c)
    rows.append(np.arange(N))
    cols.append(np.arange(N))
    vals.append(diag)
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(N, N))


def solve_phi(s, faces):
    act, n, g, dx, per = _geom(s)
    L = laplacian(s).tolil()
    b = divergence(s, faces).ravel().copy()
    if all(per[d] for d in range(3) if act[d]):
        L[0, :] = 0.0
        L[0, 0] = 1.0
        b[0] = 0.0
    return spla.spsolve(L.tocsc(), b).reshape(n[2], n[1], n[0])


def gradient_faces(s, phi):
    """(Phi(c) - Phi(c - e_d)) / dx_d on every d-face of the interior (padded
    face arrays, zero elsewhere)"""
    act, n, g, dx, per = _geom(s)
    out = np.zeros((3,) + s.shape)
    for d in range(3):
        if not act[d]:
            continue
        ax = 2 - d
        # Phi on cells -1 .. n along d with the boundary rule
        lo_pad = np.take(phi, [n[d] - 1], axis=ax) if per[d] else -np.take(phi, [0], axis=ax)
        hi_pad = np.take(phi, [0], axis=ax) if per[d] else -np.take(phi, [n[d] - 1], axis=ax)
        ext = np.concatenate([lo_pad, phi, hi_pad], axis=ax)
        grad = np.diff(ext, axis=ax) / dx[d]  # faces 0 .. n along d
        sl = [slice(g[2], g[2] + n[2]), slice(g[1], g[1] + n[1]), slice(g[0], g[0] + n[0])]
        sl[ax] = slice(g[d], g[d] + n[d] + 1)
        out[d][tuple(sl)] = grad
    return out


def clean(s, faces):
    """returns (cleaned faces, Phi)"""
    phi = solve_phi(s, faces)
    return faces - gradient_faces(s, phi), phi
