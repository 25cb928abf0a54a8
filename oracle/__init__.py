"""ctypes wrapper of the plain-C CPU oracle (oracle/oracle.c).

TEST INFRASTRUCTURE ONLY: the HIP library is tested against the oracle.  Only
the test-suite, the smoke check and the CPU-baseline leg of the benchmark may
import this module.  It shares no code with the GPU path; the only common
input is the seeded initial data of the `workloads` module.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SRC_PATH = os.path.join(_HERE, "oracle.c")
# the planted-mistake tests point the wrapper at a modified copy of the
# source; its library is built beside that copy
if os.environ.get("GR_ORACLE_SRC"):
    SRC_PATH = os.path.abspath(os.environ["GR_ORACLE_SRC"])
    LIB_PATH = os.path.join(os.path.dirname(SRC_PATH), "liboracle.so")


def build(force=False):
    """gcc -O2 -ffp-contract=off -fopenmp -> oracle/liboracle.so"""
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC_PATH):
        tmp = LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", "-Wall",
                               "-o", tmp, SRC_PATH, "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


class OrGrid(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int), ("n", ctypes.c_int * 3), ("ng", ctypes.c_int),
                ("lo", ctypes.c_double * 3), ("hi", ctypes.c_double * 3), ("bc", (ctypes.c_int * 2) * 3),
                ("gamma_ad", ctypes.c_double), ("recon", ctypes.c_int), ("imex", ctypes.c_int),
                ("cfl", ctypes.c_double), ("eta_mode", ctypes.c_int), ("eta", ctypes.c_double),
                ("sigma0", ctypes.c_double), ("eta_min", ctypes.c_double), ("eta_max", ctypes.c_double),
                ("rho_atm", ctypes.c_double), ("p_atm", ctypes.c_double), ("metric", ctypes.c_int),
                ("newton_tol", ctypes.c_double), ("newton_maxit", ctypes.c_int), ("xi", ctypes.c_double),
                ("atm_factor", ctypes.c_double), ("frozen_matter", ctypes.c_int), ("glm", ctypes.c_int),
                ("kappa_E", ctypes.c_double), ("kappa_B", ctypes.c_double), ("uct", ctypes.c_int)]


_lib = None
_D = ctypes.POINTER(ctypes.c_double)
_DD = ctypes.POINTER(_D)


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(LIB_PATH)
        G = ctypes.POINTER(OrGrid)
        L.or_prim2cons.argtypes = [ctypes.c_double, ctypes.c_double, _D, _D, _D, _D]
        L.or_flux.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double, _D, _D, _D, _D]
        L.or_flux_B.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, _D, _D]
        L.or_c2p.argtypes = [ctypes.c_double, ctypes.c_double, _D, _D, _D, _D]
        L.or_c2p.restype = ctypes.c_int
        L.or_implicit_E.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double, _D, _D, _D, _D]
        L.or_implicit_residual.argtypes = [ctypes.c_double, ctypes.c_double, _D, _D, ctypes.c_double,
                                           ctypes.c_double, _D, _D, _D]
        L.or_implicit.argtypes = [ctypes.c_double, ctypes.c_double, _D, _D, ctypes.c_double, ctypes.c_double, _D,
                                  ctypes.c_double, ctypes.c_int, _D, _D, ctypes.POINTER(ctypes.c_int)]
        L.or_implicit.restype = ctypes.c_int
        L.or_recon.argtypes = [ctypes.c_int, _D, _D, _D]
        L.or_tableau.argtypes = [ctypes.c_int, _D, _D, _D, _D]
        L.or_tableau.restype = ctypes.c_int
        L.or_ghost_fill.argtypes = [G, _DD, ctypes.c_int, _DD]
        L.or_explicit_L.argtypes = [G, _DD, _DD, _DD, _D, _D, _DD, _DD]
        L.or_step.argtypes = [G, _DD, _DD, _DD, _D, _D, ctypes.c_double, ctypes.c_int, _DD, _DD]
        L.or_step.restype = ctypes.c_long
        L.or_c2p_grid.argtypes = [G, _DD, _DD, _DD, _D]
        L.or_c2p_grid.restype = ctypes.c_long
        L.or_init.argtypes = [G, _DD, _DD, _DD, _D, _DD, _DD, _DD]
        L.or_cfl_dt.argtypes = [G, _D, _D]
        L.or_cfl_dt.restype = ctypes.c_double
        L.or_divB.argtypes = [G, _DD, _D]
        L.or_step_glm.argtypes = [G, _DD, _DD, _DD, _D, _D, ctypes.c_double]
        L.or_step_glm.restype = ctypes.c_long
        L.or_explicit_L_glm.argtypes = [G, _DD, _D, _D, _DD]
        L.or_divB_glm.argtypes = [G, _DD, _D]
        L.or_threads.argtypes = [ctypes.c_int]
        L.or_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_D)


def _pp(arrs):
    if arrs is None:
        return None
    ptrs = (_D * len(arrs))(*[_p(a) for a in arrs])
    return ctypes.cast(ptrs, _DD)


def grid_of(s) -> OrGrid:
    g = OrGrid()
    g.ndim = s.ndim
    for d in range(3):
        g.n[d] = s.nn(d)
        g.lo[d] = s.lo[d]
        g.hi[d] = s.hi[d]
        g.bc[d][0] = s.bc[d][0]
        g.bc[d][1] = s.bc[d][1]
    g.ng = s.ng
    g.gamma_ad = s.gamma_ad
    g.recon = s.recon
    g.imex = s.imex
    g.cfl = s.cfl
    g.eta_mode = s.eta_mode
    g.eta = s.eta
    g.sigma0 = s.sigma0
    g.eta_min = s.eta_min
    g.eta_max = s.eta_max
    g.rho_atm = s.rho_atm
    g.p_atm = s.p_atm
    g.metric = s.metric
    g.newton_tol = s.newton_tol
    g.newton_maxit = s.newton_maxit
    g.xi = s.xi
    g.atm_factor = s.atm_factor
    g.frozen_matter = s.frozen_matter
    g.glm = s.glm
    g.kappa_E = s.kappa_E
    g.kappa_B = s.kappa_B
    g.uct = s.uct
    return g


class OracleState:
    """q (8; 10 with GLM: + q_Psi, q_Phi), face (3: face-centred q_B, or
    cell-centred q_B with GLM), prim (5) numpy arrays of padded cell shape"""

    def __init__(self, s):
        self.setup = s
        self.grid = grid_of(s)
        shp = s.shape
        self.q = [np.zeros(shp) for _ in range(10 if s.glm else 8)]
        self.face = [np.zeros(shp) for _ in range(3)]
        self.prim = [np.zeros(shp) for _ in range(5)]
        self.alpha = np.ascontiguousarray(s.alpha) if s.metric else None
        self.psi = np.ascontiguousarray(s.psi) if s.metric else None
        self.t = 0.0
        self.nfail = 0
        prim_in = [np.ascontiguousarray(s.prim[v]) for v in range(5)]
        E_in = [np.ascontiguousarray(s.E[v]) for v in range(3)]
        A = [np.ascontiguousarray(s.A[v]) for v in range(3)] if s.A is not None else None
        lib().or_init(ctypes.byref(self.grid), _pp(prim_in), _pp(E_in), _pp(A), _p(self.psi), _pp(self.q),
                      _pp(self.face), _pp(self.prim))
        if s.face is not None:
            for d in range(3):
                self.face[d] += s.face[d]
            # conserved variables must see the added face field
            self._recons(prim_in, E_in)
        if s.glm:
            self.face = cell_centred_qB(s, self.face)

    def _recons(self, prim_in, E_in):
        s = self.setup
        q = np.zeros(8)
        sl = s.interior
        g = [s.g(d) for d in range(3)]
        act = [s.active(d) for d in range(3)]
        for k in range(sl[0].start, sl[0].stop):
            for j in range(sl[1].start, sl[1].stop):
                for i in range(sl[2].start, sl[2].stop):
                    ps = 1.0 if self.psi is None else self.psi[k, j, i]
                    B = np.zeros(3)
                    idx = (k, j, i)
                    for d in range(3):
                        if not act[d]:
                            B[d] = self.face[d][idx] / ps ** 6
                        else:
                            ip = list(idx)
                            ip[2 - d] += 1
                            B[d] = 0.5 * (self.face[d][idx] + self.face[d][tuple(ip)]) / ps ** 6
                    pr = np.array([prim_in[v][idx] for v in range(5)])
                    E = np.array([E_in[v][idx] for v in range(3)])
                    prim2cons(s.gamma_ad, ps, pr, E, B, q)
                    for v in range(8):
                        self.q[v][idx] = q[v]
        del g

    def step(self, dt, dump_stage=-1, with_L=False):
        stage = L = None
        if dump_stage >= 0:
            stage = [np.zeros(self.setup.shape) for _ in range(8)]
            if with_L:
                L = [np.zeros(self.setup.shape) for _ in range(11)]
        if self.setup.glm:
            nf = lib().or_step_glm(ctypes.byref(self.grid), _pp(self.q), _pp(self.face), _pp(self.prim),
                                   _p(self.alpha), _p(self.psi), dt)
            self.nfail += nf
            self.t += dt
            return nf
        nf = lib().or_step(ctypes.byref(self.grid), _pp(self.q), _pp(self.face), _pp(self.prim), _p(self.alpha),
                           _p(self.psi), dt, max(dump_stage, 0), _pp(stage), _pp(L))
        self.nfail += nf
        self.t += dt
        return (stage, L) if dump_stage >= 0 else nf

    def dt(self):
        return lib().or_cfl_dt(ctypes.byref(self.grid), _p(self.alpha), _p(self.psi))

    def divB(self):
        out = np.zeros(3)
        if self.setup.glm:
            lib().or_divB_glm(ctypes.byref(self.grid), _pp(self.face), _p(out))
        else:
            lib().or_divB(ctypes.byref(self.grid), _pp(self.face), _p(out))
        return out

    def prims(self):
        return np.stack(self.prim)

    def E(self):
        ps6 = 1.0 if self.psi is None else self.psi ** 6
        return np.stack([self.q[5 + v] / ps6 for v in range(3)])


def cell_centred_qB(s, face):
    """GLM initial data: cell-centred q_B^d = mean of the two d-faces of the
    cell (the face value along an inactive direction or at the array end)"""
    out = []
    for d in range(3):
        f = face[d]
        if not s.active(d):
            out.append(f.copy())
            continue
        ax = 2 - d
        up = np.concatenate([np.take(f, range(1, f.shape[ax]), axis=ax), np.take(f, [f.shape[ax] - 1], axis=ax)],
                            axis=ax)
        out.append(np.ascontiguousarray(0.5 * (f + up)))
    return out


# ---------------------------------------------------------------------------
# point-wise entry points
def prim2cons(gam, psi, prim, E, B, out=None):
    out = np.zeros(8) if out is None else out
    lib().or_prim2cons(gam, psi, _p(np.ascontiguousarray(prim, dtype=float)),
                       _p(np.ascontiguousarray(E, dtype=float)), _p(np.ascontiguousarray(B, dtype=float)), _p(out))
    return out


def flux(d, gam, alpha, psi, prim, E, B):
    out = np.zeros(8)
    lib().or_flux(d, gam, alpha, psi, _p(np.ascontiguousarray(prim, dtype=float)),
                  _p(np.ascontiguousarray(E, dtype=float)), _p(np.ascontiguousarray(B, dtype=float)), _p(out))
    return out


def flux_B(d, alpha, psi, E):
    out = np.zeros(3)
    lib().or_flux_B(d, alpha, psi, _p(np.ascontiguousarray(E, dtype=float)), _p(out))
    return out


def c2p(gam, psi, q, E, B):
    out = np.zeros(5)
    r = lib().or_c2p(gam, psi, _p(np.ascontiguousarray(q, dtype=float)), _p(np.ascontiguousarray(E, dtype=float)),
                     _p(np.ascontiguousarray(B, dtype=float)), _p(out))
    return r, out


def implicit_E(psi, etat, xi, ut, Es, B):
    out = np.zeros(3)
    lib().or_implicit_E(psi, etat, xi, _p(np.ascontiguousarray(ut, dtype=float)),
                        _p(np.ascontiguousarray(Es, dtype=float)), _p(np.ascontiguousarray(B, dtype=float)), _p(out))
    return out


def implicit_residual(gam, psi, q, B, etat, xi, ut):
    f = np.zeros(3)
    J = np.zeros(9)
    lib().or_implicit_residual(gam, psi, _p(np.ascontiguousarray(q, dtype=float)),
                               _p(np.ascontiguousarray(B, dtype=float)), etat, xi,
                               _p(np.ascontiguousarray(ut, dtype=float)), _p(f), _p(J))
    return f, J.reshape(3, 3)


def implicit(gam, psi, q, B, etat, xi, guess, tol=1e-13, maxit=60):
    prim = np.zeros(5)
    E = np.zeros(3)
    it = ctypes.c_int(0)
    r = lib().or_implicit(gam, psi, _p(np.ascontiguousarray(q, dtype=float)), _p(np.ascontiguousarray(B, dtype=float)),
                          etat, xi, _p(np.ascontiguousarray(guess, dtype=float)), tol, maxit, _p(prim), _p(E),
                          ctypes.byref(it))
    return r, prim, E, it.value


def recon(kind, w):
    L = ctypes.c_double(0)
    R = ctypes.c_double(0)
    lib().or_recon(kind, _p(np.ascontiguousarray(w, dtype=float)), ctypes.byref(L), ctypes.byref(R))
    return L.value, R.value


def tableau(imex):
    At = np.zeros(16)
    A = np.zeros(16)
    wt = np.zeros(4)
    w = np.zeros(4)
    s = lib().or_tableau(imex, _p(At), _p(A), _p(wt), _p(w))
    return At.reshape(4, 4)[:s, :s], A.reshape(4, 4)[:s, :s], wt[:s], w[:s]


def threads(n=0):
    """OpenMP threads of the oracle: n > 0 sets them; returns the count in use"""
    return lib().or_threads(int(n))


def run(s, steps=None, dt=None):
    st = OracleState(s)
    dt = st.dt() if dt is None else dt
    for _ in range(s.steps if steps is None else steps):
        st.step(dt)
    return st
