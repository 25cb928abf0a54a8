"""Seeded synthetic inputs for the resistive-GRMHD IMEX stage.

This module is shared by the HIP library's callers (tests, bench, serving)
and by the CPU oracle's tests.  It holds no arithmetic of the numerical
method: it only lays out grids and evaluates initial data (analytic profiles,
a TOV equilibrium integrated here, edge vector potentials, seeded noise).
The discrete curl of the vector potential and the primitive -> conserved map
are done independently by each side.

Array conventions (both sides rely on them):
  * a cell array has shape (Nz, Ny, Nx) with N_d = n_d + 2 g_d (g_d = 0 for an
    inactive direction), x fastest; flat index i + Nx (j + Ny k);
  * face array d at index (i,j,k) sits half a cell below the cell centre in
    direction d (same shape as a cell array);
  * edge array A_k at index (i,j,k) sits half a cell below the cell centre in
    the two directions other than k; it is one point longer than a cell array
    in every active direction;
  * primitives are (rho, u~^x, u~^y, u~^z, p) with u~^i = W v^i, E^i and B^i are
    contravariant components, face fields are densitised (psi^6 B^d).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

OUTFLOW, PERIODIC, FIXED = 0, 1, 2
MINMOD, MC, PPM = 0, 1, 2
SSP2, SSP3 = 0, 1


@dataclasses.dataclass
class Setup:
    name: str
    ndim: int
    n: tuple
    ng: int
    lo: tuple
    hi: tuple
    bc: tuple                      # ((x_lo, x_hi), (y_lo, y_hi), (z_lo, z_hi))
    gamma_ad: float
    recon: int
    imex: int
    cfl: float = 0.4
    eta_mode: int = 0
    eta: float = 1e-3
    sigma0: float = 0.0
    eta_min: float = 0.0
    eta_max: float = 1.0
    rho_atm: float = 1e-14
    p_atm: float = 1e-14
    metric: int = 0
    newton_tol: float = 1e-13
    newton_maxit: int = 60
    xi: float = 0.0
    atm_factor: float = 1.001
    frozen_matter: int = 0
    glm: int = 0               # 1: cell-centred B with GLM cleaning (Sec 3.1)
    kappa_E: float = 1.0
    kappa_B: float = 1.0
    uct: int = 0               # 0 resistive upwind CT (Sec 3.2), 1 ideal-MHD form (App. A)
    steps: int = 1
    # initial data (padded arrays, see module docstring)
    prim: Optional[np.ndarray] = None      # (5, Nz, Ny, Nx)
    E: Optional[np.ndarray] = None         # (3, Nz, Ny, Nx)
    A: Optional[np.ndarray] = None         # (3, Nz+1?, Ny+1?, Nx+1?) or None
    face: Optional[np.ndarray] = None      # (3, Nz, Ny, Nx) densitised face values added to curl A, or None
    alpha: Optional[np.ndarray] = None     # (Nz, Ny, Nx) or None (flat)
    psi: Optional[np.ndarray] = None

    # --- geometry helpers -------------------------------------------------
    def active(self, d):
        return d < self.ndim

    def g(self, d):
        return self.ng if self.active(d) else 0

    def nn(self, d):
        return self.n[d] if self.active(d) else 1

    def N(self, d):
        return self.nn(d) + 2 * self.g(d)

    @property
    def shape(self):
        return (self.N(2), self.N(1), self.N(0))

    @property
    def edge_shape(self):
        return tuple(self.N(d) + (1 if self.active(d) else 0) for d in (2, 1, 0))

    def dx(self, d):
        return (self.hi[d] - self.lo[d]) / self.n[d] if self.active(d) else 1.0

    def centres(self, d):
        """cell-centre coordinates along d for every padded index"""
        if not self.active(d):
            return np.zeros(1)
        i = np.arange(self.N(d))
        return self.lo[d] + (i - self.g(d) + 0.5) * self.dx(d)

    def lower_faces(self, d, extra=0):
        """coordinates half a cell below the centres (edge / face positions)"""
        if not self.active(d):
            return np.zeros(1)
        i = np.arange(self.N(d) + extra)
        return self.lo[d] + (i - self.g(d)) * self.dx(d)

    def mesh(self):
        """cell-centre coordinates broadcast to (Nz, Ny, Nx)"""
        x, y, z = self.centres(0), self.centres(1), self.centres(2)
        Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
        return X, Y, Z

    def edge_mesh(self, k):
        """coordinates of edge array A_k (edge_shape)"""
        cs = []
        for d in range(3):
            ext = 1 if self.active(d) else 0
            if d == k:
                if self.active(d):
                    c = np.concatenate([self.centres(d), [self.centres(d)[-1] + self.dx(d)]])
                else:
                    c = np.zeros(1)
            else:
                c = self.lower_faces(d, ext)
            cs.append(c)
        Z, Y, X = np.meshgrid(cs[2], cs[1], cs[0], indexing="ij")
        return X, Y, Z

    @property
    def interior(self):
        return tuple(slice(self.g(d), self.g(d) + self.nn(d)) for d in (2, 1, 0))

    @property
    def ncells(self):
        return self.nn(0) * self.nn(1) * self.nn(2)

    def dt(self):
        """max-diffusivity CFL step; the speeds depend on the metric only"""
        if self.metric:
            a = self.alpha[self.interior]
            p = self.psi[self.interior]
            s = sum(a / p ** 2 / self.dx(d) for d in range(self.ndim))
            return self.cfl / float(s.max())
        return self.cfl / sum(1.0 / self.dx(d) for d in range(self.ndim))


# ----------------------------------------------------------------------------
# counter-based noise: splitmix64 of (seed, stream, index) -> U[-1, 1)


def splitmix64(x: np.ndarray) -> np.ndarray:
    x = np.asarray(x, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = x + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


def uniform_pm1(seed: int, stream: int, count: int) -> np.ndarray:
    """count values in [-1, 1) from splitmix64((seed << 40) ^ (stream << 32) ^ i)"""
    base = ((seed & 0xFFFFFF) << 40) ^ ((stream & 0xFF) << 32)
    idx = np.arange(count, dtype=np.uint64) ^ np.uint64(base)
    z = splitmix64(idx)
    u = (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)
    return 2.0 * u - 1.0


def _blank(s: Setup):
    s.prim = np.zeros((5,) + s.shape)
    s.E = np.zeros((3,) + s.shape)
    s.face = None
    s.A = None
    return s


def _bc(ndim, kind):
    return tuple((kind, kind) if d < ndim else (OUTFLOW, OUTFLOW) for d in range(3))


# ----------------------------------------------------------------------------
# workloads of the benchmark configurations
def shock_tube(n=400, seed=1, eta=1e-3, recon=MINMOD, imex=SSP2, noise=1e-6, rho_l=1.0, rho_r=0.125, p_l=1.0,
               p_r=0.1, by_l=0.5, bx=0.5):
    """1-D relativistic resistive shock tube (Balsara-1 type), Gamma = 2.
    left (rho, p, Bx, By) = (1, 1, 0.5, 0.5), right (0.125, 0.1, 0.5, -0.5)
    by default; By on the right is -By on the left."""
    s = _blank(Setup("shock_tube", 1, (n, 1, 1), 3 if recon == PPM else 2, (-0.5, 0, 0), (0.5, 1, 1),
                     _bc(1, OUTFLOW), 2.0, recon, imex, eta=eta, rho_atm=1e-12, p_atm=1e-14,
                     steps=int(round(0.4 / (0.4 * 1.0 / n)))))
    X, _, _ = s.mesh()
    left = X < 0.0
    u = uniform_pm1(seed, 0, int(np.prod(s.shape))).reshape(s.shape)
    s.prim[0] = np.where(left, rho_l, rho_r) * (1.0 + noise * u)
    s.prim[4] = np.where(left, p_l, p_r)
    face = np.zeros((3,) + s.shape)
    face[0] = bx
    face[1] = np.where(left, by_l, -by_l)
    s.face = face
    return s


def blast_wave(n=512, eta=1e-6, seed=1, recon=PPM, imex=SSP3, steps=100, bx=0.1, p_in=1.0, p_out=1e-3,
               rho=0.01):
    """2-D resistive cylindrical blast wave on [-6, 6]^2, Gamma = 4/3,
    B^x = bx from A_z = bx * y on the edges."""
    s = _blank(Setup("blast_wave", 2, (n, n, 1), 3 if recon == PPM else 2, (-6, -6, 0), (6, 6, 1),
                     _bc(2, OUTFLOW), 4.0 / 3.0, recon, imex, eta=eta, rho_atm=1e-12 * rho, p_atm=1e-14,
                     steps=steps))
    X, Y, _ = s.mesh()
    r = np.sqrt(X ** 2 + Y ** 2)
    s.prim[0] = rho
    s.prim[4] = np.where(r < 1.0, p_in, p_out)
    s.A = np.zeros((3,) + s.edge_shape)
    _, Ye, _ = s.edge_mesh(2)
    s.A[2] = bx * Ye
    return s


def tov_profile(K=100.0, Gamma=2.0, rho_c=1.28e-3, nr=20000):
    """Static spherical star (TOV) in isotropic coordinates.  Integrates
    m, p, nu in the areal radius with RK4, then maps to the isotropic radius.
    Returns a dict of callables of the isotropic radius for rho, p, alpha, psi
    and the total mass M and isotropic surface radius R_iso."""
    def eos_e(p):
        rho = (max(p, 0.0) / K) ** (1.0 / Gamma)
        return rho + p / (Gamma - 1.0)

    def rhs(r, y):
        # y = (m, p, nu, ln(rbar / r)); the last one is regular at the centre
        m, p, nu, lnq = y
        if p <= 0:
            return np.zeros(4)
        e = eos_e(p)
        dpdr = -(e + p) * (m + 4 * math.pi * r ** 3 * p) / (r * (r - 2 * m))
        dm = 4 * math.pi * r ** 2 * e
        dnu = 2 * (m + 4 * math.pi * r ** 3 * p) / (r * (r - 2 * m))
        dlnq = (1.0 / math.sqrt(1 - 2 * m / r) - 1.0) / r
        return np.array([dm, dpdr, dnu, dlnq])

    p_c = K * rho_c ** Gamma
    r = 1e-6
    y = np.array([4.0 / 3.0 * math.pi * r ** 3 * eos_e(p_c), p_c, 0.0, 0.0])
    h = 20.0 / nr
    rs, ys = [r], [y.copy()]
    while y[1] > 0 and r < 50:
        k1 = rhs(r, y)
        k2 = rhs(r + h / 2, y + h / 2 * k1)
        k3 = rhs(r + h / 2, y + h / 2 * k2)
        k4 = rhs(r + h, y + h * k3)
        yn = y + h / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
        if yn[1] <= 0:
            # surface: linear interpolation of p to zero
            f = y[1] / (y[1] - yn[1])
            r = r + f * h
            y = y + f * (yn - y)
            y[1] = 0.0
            rs.append(r)
            ys.append(y.copy())
            break
        r += h
        y = yn
        rs.append(r)
        ys.append(y.copy())
    rs = np.array(rs)
    ys = np.array(ys)
    R, M = rs[-1], ys[-1, 0]
    # isotropic radius: ln(rbar/r) + const, matched to the exterior at the surface
    Rbar = 0.5 * (R - M + math.sqrt(R * R - 2 * M * R))
    lnq = ys[:, 3] - ys[-1, 3] + math.log(Rbar / R)
    rbar = rs * np.exp(lnq)
    psi_in = np.exp(-0.5 * lnq)
    nu_in = ys[:, 2] - ys[-1, 2] + math.log(1 - 2 * M / R)
    alpha_in = np.exp(0.5 * nu_in)
    p_in = ys[:, 1]
    rho_in = (np.maximum(p_in, 0) / K) ** (1.0 / Gamma)
    rbar[0] = 0.0

    def f_in(tab):
        return lambda x: np.interp(x, rbar, tab)

    def psi(x):
        x = np.asarray(x, dtype=float)
        return np.where(x < Rbar, f_in(psi_in)(x), 1.0 + M / (2 * np.maximum(x, 1e-300)))

    def alpha(x):
        x = np.asarray(x, dtype=float)
        out = (1 - M / (2 * np.maximum(x, 1e-300))) / (1 + M / (2 * np.maximum(x, 1e-300)))
        return np.where(x < Rbar, f_in(alpha_in)(x), out)

    def rho(x):
        x = np.asarray(x, dtype=float)
        return np.where(x < Rbar, f_in(rho_in)(x), 0.0)

    def p(x):
        x = np.asarray(x, dtype=float)
        return np.where(x < Rbar, f_in(p_in)(x), 0.0)

    return dict(rho=rho, p=p, alpha=alpha, psi=psi, M=M, R=Rbar, p_c=p_c, K=K, Gamma=Gamma)


_TOV_CACHE = {}


def tov_star(n=128, ext=12.0, b_max=1e-4, rho_atm=1e-10, steps=200, recon=PPM, imex=SSP3, sigma0=1e6,
             eta_in=1e-6, eta_out=1.0, atm_factor=1e4, ndim=3):
    """3-D magnetised polytropic star (K = 100, Gamma = 2, rho_c = 1.28e-3) in
    a static conformally flat metric, poloidal field from
    A_phi = A_b varpi^2 max(p - 0.04 p_c, 0)^2 scaled so max|B| = b_max,
    atmosphere rho_atm, eta from sigma(D) clamped to [eta_in, eta_out].
    ndim 2 / 1: the same star on its equatorial plane z = 0 / on the x axis
    (the inactive coordinates are 0), n cells per active direction."""
    key = ("tov",)
    if key not in _TOV_CACHE:
        _TOV_CACHE[key] = tov_profile()
    T = _TOV_CACHE[key]
    K, G = T["K"], T["Gamma"]
    shape = tuple(n if d < ndim else 1 for d in range(3))
    s = _blank(Setup("tov_star" if ndim == 3 else "tov_star_%dd" % ndim, ndim, shape, 3 if recon == PPM else 2,
                     (-ext,) * 3, (ext,) * 3, _bc(ndim, OUTFLOW), 2.0, recon, imex, eta_mode=1, eta=eta_in,
                     sigma0=sigma0,
                     eta_min=eta_in, eta_max=eta_out, rho_atm=rho_atm, p_atm=K * rho_atm ** G, metric=1,
                     steps=steps, atm_factor=atm_factor))
    X, Y, Z = s.mesh()
    r = np.sqrt(X ** 2 + Y ** 2 + Z ** 2)
    rho = T["rho"](r)
    p = T["p"](r)
    inside = rho > rho_atm
    s.prim[0] = np.where(inside, rho, rho_atm)
    s.prim[4] = np.where(inside, np.maximum(K * rho ** G, s.p_atm), s.p_atm)
    s.alpha = T["alpha"](r)
    s.psi = T["psi"](r)
    pcut = 0.04 * T["p_c"]

    def fpot(rr):
        return np.maximum(T["p"](rr) - pcut, 0.0) ** 2

    # normalisation of A_b from the analytic curl of the continuous potential
    hh = 1e-4
    f = fpot(r)
    fp = (fpot(r + hh) - fpot(r - hh)) / (2 * hh)
    rr = np.maximum(r, 1e-12)
    bx = -X * Z * fp / rr
    by = -Y * Z * fp / rr
    bz = 2 * f + (X ** 2 + Y ** 2) * fp / rr
    bmag = np.sqrt(bx ** 2 + by ** 2 + bz ** 2) / s.psi ** 6
    bnorm = float(bmag[s.interior].max())
    A_b = b_max / bnorm if bnorm > 0 else 0.0
    s.A = np.zeros((3,) + s.edge_shape)
    Xe, Ye, Ze = s.edge_mesh(0)
    s.A[0] = -Ye * A_b * fpot(np.sqrt(Xe ** 2 + Ye ** 2 + Ze ** 2))
    Xe, Ye, Ze = s.edge_mesh(1)
    s.A[1] = Xe * A_b * fpot(np.sqrt(Xe ** 2 + Ye ** 2 + Ze ** 2))
    return s


# ----------------------------------------------------------------------------
# test problems of the paper's Sec 5
def current_sheet(n=256, eta=0.01, t0=1.0, p=5000.0, recon=MC, imex=SSP2, gamma=4.0 / 3.0):
    """Self-similar current sheet: B^y = erf(x / (2 sqrt(eta t))) at t = t0,
    E^z = sqrt(eta/(pi t)) exp(-x^2/(4 eta t)), rho = 1, p = 5000, [-1.5, 1.5]."""
    s = _blank(Setup("current_sheet", 1, (n, 1, 1), 3 if recon == PPM else 2, (-1.5, 0, 0), (1.5, 1, 1),
                     _bc(1, OUTFLOW), gamma, recon, imex, eta=eta, rho_atm=1e-12, p_atm=1e-14))
    X, _, _ = s.mesh()
    s.prim[0] = 1.0
    s.prim[4] = p
    s.E[2] = np.sqrt(eta / (math.pi * t0)) * np.exp(-X ** 2 / (4 * eta * t0))
    face = np.zeros((3,) + s.shape)
    from scipy.special import erf
    face[1] = erf(X / (2 * np.sqrt(eta * t0)))
    s.face = face
    return s


def current_sheet_exact(x, t, eta=0.01):
    from scipy.special import erf
    return erf(x / (2 * np.sqrt(eta * t)))


def telegraph_params(sigma=1.0, Lx=1.0, Ly=0.5):
    kx = 2 * math.pi / Lx
    tana = Lx / Ly
    k = kx * math.sqrt(1 + tana ** 2)
    mu = math.sqrt(k * k - sigma * sigma / 4.0)
    return dict(k=k, mu=mu, T=2 * math.pi / mu, alpha=math.atan(tana), kvec=(kx, kx * tana))


def telegraph_fields(X, Y, t, sigma=1.0, B1=1.0):
    P = telegraph_params(sigma)
    phase = P["kvec"][0] * X + P["kvec"][1] * Y - P["mu"] * t
    damp = B1 * math.exp(-sigma / 2 * t)
    Bz = damp * np.cos(phase)
    Ey_r = damp * (P["mu"] / P["k"] * np.cos(phase) + sigma / (2 * P["k"]) * np.sin(phase))
    a = P["alpha"]
    return Bz, -math.sin(a) * Ey_r, math.cos(a) * Ey_r


def telegraph(n=64, sigma=1.0, recon=MC, imex=SSP2):
    """2-D telegraph-equation wave, periodic 1 x 0.5, rho = 1e12, p = 0, v = 0."""
    s = _blank(Setup("telegraph", 2, (n, n // 2, 1), 3 if recon == PPM else 2, (0, 0, 0), (1.0, 0.5, 1),
                     _bc(2, PERIODIC), 4.0 / 3.0, recon, imex, eta=1.0 / sigma, rho_atm=1e-3, p_atm=0.0))
    X, Y, _ = s.mesh()
    Bz, Ex, Ey = telegraph_fields(X, Y, 0.0, sigma)
    s.prim[0] = 1e12
    s.prim[4] = 0.0
    s.E[0] = Ex
    s.E[1] = Ey
    face = np.zeros((3,) + s.shape)
    face[2] = Bz
    s.face = face
    return s


def charged_vortex(n=64, q0=0.7, p0=0.1, rho=1.0, gamma=4.0 / 3.0, eta=1e-3, recon=MC, imex=SSP2):
    """Stationary charged vortex on [-10, 10]^2 with fixed boundary values."""
    s = _blank(Setup("charged_vortex", 2, (n, n, 1), 3 if recon == PPM else 2, (-10, -10, 0), (10, 10, 1),
                     _bc(2, FIXED), gamma, recon, imex, eta=eta, rho_atm=1e-12, p_atm=1e-14))
    X, Y, _ = s.mesh()
    R2 = X ** 2 + Y ** 2
    R = np.sqrt(R2)
    ER = q0 / 2 * R / (R2 + 1)
    root = np.sqrt((R2 + 1) ** 2 - q0 ** 2 / 4)
    Bz = root / (R2 + 1)
    vphi = -q0 / 2 * R / root
    g1 = (gamma - 1) / gamma
    p = -rho * g1 + (p0 + rho * g1) * ((4 * R2 + 4 - q0 ** 2) / ((R2 + 1) * (4 - q0 ** 2))) ** (
        gamma / (2 * (gamma - 1)))
    Rs = np.maximum(R, 1e-300)
    cx, cy = X / Rs, Y / Rs
    vx, vy = -vphi * cy, vphi * cx
    W = 1.0 / np.sqrt(1 - vx ** 2 - vy ** 2)
    s.prim[0] = rho
    s.prim[1] = W * vx
    s.prim[2] = W * vy
    s.prim[4] = p
    s.E[0] = ER * cx
    s.E[1] = ER * cy
    face = np.zeros((3,) + s.shape)
    face[2] = Bz
    s.face = face
    return s


def loop_advection(nx=64, ny=32, A0=1e-3, Rl=0.3, eta=1e-6, recon=MC, imex=SSP2, vx=0.2, vy=0.1):
    """Field-loop advection, periodic [-1, 1] x [-0.5, 0.5], rho = p = 1."""
    s = _blank(Setup("loop_advection", 2, (nx, ny, 1), 3 if recon == PPM else 2, (-1, -0.5, 0), (1, 0.5, 1),
                     _bc(2, PERIODIC), 4.0 / 3.0, recon, imex, eta=eta, rho_atm=1e-12, p_atm=1e-14))
    X, Y, _ = s.mesh()
    W = 1.0 / math.sqrt(1 - vx * vx - vy * vy)
    s.prim[0] = 1.0
    s.prim[1] = W * vx
    s.prim[2] = W * vy
    s.prim[4] = 1.0
    r = np.sqrt(X ** 2 + Y ** 2)
    rs = np.maximum(r, 1e-300)
    inside = r < Rl
    Bx = np.where(inside, -A0 * Y / rs, 0.0)
    By = np.where(inside, A0 * X / rs, 0.0)
    s.E[2] = -(vx * By - vy * Bx)
    s.A = np.zeros((3,) + s.edge_shape)
    Xe, Ye, _ = s.edge_mesh(2)
    re = np.sqrt(Xe ** 2 + Ye ** 2)
    s.A[2] = np.where(re < Rl, A0 * (Rl - re), 0.0)
    return s


def density_wave(n=64, ndim=1, amp=0.2, v=0.5, recon=MC, imex=SSP2, gamma=5.0 / 3.0):
    """Periodic sinusoidal density wave advected at uniform velocity and pressure."""
    dims = (n, n if ndim > 1 else 1, 1)
    s = _blank(Setup("density_wave", ndim, dims, 3 if recon == PPM else 2, (0, 0, 0), (1, 1, 1),
                     _bc(ndim, PERIODIC), gamma, recon, imex, eta=1.0, rho_atm=1e-12, p_atm=1e-14))
    X, Y, _ = s.mesh()
    phase = X + (Y if ndim > 1 else 0.0)
    s.prim[0] = 1.0 + amp * np.sin(2 * math.pi * phase)
    vv = np.array([v, v if ndim > 1 else 0.0, 0.0]) / (math.sqrt(2) if ndim > 1 else 1.0)
    W = 1.0 / math.sqrt(1 - float(vv @ vv))
    for d in range(3):
        s.prim[1 + d] = W * vv[d]
    s.prim[4] = 1.0
    return s


def density_wave_exact(s: Setup, t):
    X, Y, _ = s.mesh()
    vv = np.array([0.5, 0.5 if s.ndim > 1 else 0.0]) / (math.sqrt(2) if s.ndim > 1 else 1.0)
    phase = (X - vv[0] * t) + ((Y - vv[1] * t) if s.ndim > 1 else 0.0)
    return 1.0 + 0.2 * np.sin(2 * math.pi * phase)


def random_states(shape3, seed=1, wmax=10.0, sigma_max=10.0, emax_frac=0.5, rho_range=(0.1, 10.0),
                  ndim=3):
    """Random smooth-free cell states for point-wise checks (prim, E, face arrays)."""
    s = _blank(Setup("random_states", ndim, shape3, 2, (0, 0, 0), (1, 1, 1), _bc(ndim, OUTFLOW), 5.0 / 3.0,
                     MINMOD, SSP2, eta=1e-3))
    cnt = int(np.prod(s.shape))

    def U(stream):
        return uniform_pm1(seed, stream, cnt).reshape(s.shape)

    lr0, lr1 = math.log(rho_range[0]), math.log(rho_range[1])
    rho = np.exp(lr0 + (lr1 - lr0) * 0.5 * (U(1) + 1))
    p = rho * np.exp(math.log(1e-3) + math.log(1e3 / 1e-3) * 0.5 * (U(2) + 1))
    W = 1.0 + (wmax - 1.0) * (0.5 * (U(3) + 1)) ** 2
    ux, uy, uz = U(4), U(5), U(6)
    nrm = np.sqrt(ux ** 2 + uy ** 2 + uz ** 2) + 1e-300
    umag = np.sqrt(W ** 2 - 1)
    s.prim[0] = rho
    s.prim[1] = umag * ux / nrm
    s.prim[2] = umag * uy / nrm
    s.prim[3] = umag * uz / nrm
    s.prim[4] = p
    bmag = np.sqrt(sigma_max * rho * 0.5 * (U(7) + 1))
    face = np.zeros((3,) + s.shape)
    for d in range(3):
        face[d] = bmag * U(8 + d) / math.sqrt(3)
    for d in range(3):
        s.E[d] = emax_frac * bmag * U(11 + d) / math.sqrt(3)
    s.face = face
    return s


def pin_grid_states(seed=1, metric=None, reps=2, efrac=0.9):
    """Point-wise cases over the grid of the oracle's own pins: W in {1, 1.01,
    2, 10, 100}, magnetisation sigma = B^2/rho in {0, 1, 1e2, 1e4}, p/rho in
    {1e-6, 1e-2, 1, 1e2}, each combination `reps` times with seeded
    directions of u~, B and E (|E| = efrac |B| times a seeded factor in
    [0, 1)); rho = 0.7.  A 1-D row of cells (B^y, B^z cell values; the x-face
    values chosen so that the mean of a cell's two faces is its B^x).
    metric = (alpha, psi): a constant lapse and conformal factor (components
    scaled by psi^-2 so that W and sigma hold in the orthonormal frame)."""
    Ws = [1.0, 1.01, 2.0, 10.0, 100.0]
    sigs = [0.0, 1.0, 1e2, 1e4]
    prs = [1e-6, 1e-2, 1.0, 1e2]
    combos = [(w, sg, pr) for w in Ws for sg in sigs for pr in prs] * reps
    n = len(combos)
    s = _blank(Setup("pin_grid", 1, (n, 1, 1), 2, (0, 0, 0), (1, 1, 1), _bc(1, OUTFLOW), 5.0 / 3.0, MINMOD, SSP2,
                     eta=1e-3, rho_atm=1e-12, p_atm=1e-20))
    g = s.ng
    dirs = [uniform_pm1(seed, 20 + k, 3 * n).reshape(n, 3) for k in range(3)]
    fac = 0.5 * (uniform_pm1(seed, 23, n) + 1.0)
    ps2 = 1.0 if metric is None else metric[1] ** 2
    rho = 0.7
    bc = np.zeros((n, 3))
    for c, (w, sg, pr) in enumerate(combos):
        i = g + c
        du = dirs[0][c] / (np.linalg.norm(dirs[0][c]) + 1e-300)
        db = dirs[1][c] / (np.linalg.norm(dirs[1][c]) + 1e-300)
        de = dirs[2][c] / (np.linalg.norm(dirs[2][c]) + 1e-300)
        s.prim[0][0, 0, i] = rho
        s.prim[4][0, 0, i] = pr * rho
        um = math.sqrt(w * w - 1.0)
        for d in range(3):
            s.prim[1 + d][0, 0, i] = um * du[d] / ps2
        b = math.sqrt(sg * rho)
        bc[c] = b * db / ps2
        for d in range(3):
            s.E[d][0, 0, i] = efrac * fac[c] * b * de[d] / ps2
    # ghosts: copies of the first / last cell
    for v in range(5):
        s.prim[v][0, 0, :g] = s.prim[v][0, 0, g]
        s.prim[v][0, 0, g + n:] = s.prim[v][0, 0, g + n - 1]
    for d in range(3):
        s.E[d][0, 0, :g] = s.E[d][0, 0, g]
        s.E[d][0, 0, g + n:] = s.E[d][0, 0, g + n - 1]
    pf = 1.0 if metric is None else metric[1] ** 6
    face = np.zeros((3,) + s.shape)
    fx = np.zeros(s.shape[2])
    fx[:g + 1] = bc[0, 0] * pf
    for c in range(n):
        fx[g + c + 1] = 2.0 * bc[c, 0] * pf - fx[g + c]
    fx[g + n + 1:] = fx[g + n]
    face[0][0, 0, :] = fx
    for d in (1, 2):
        col = np.concatenate([np.full(g, bc[0, d]), bc[:, d], np.full(g, bc[-1, d])]) * pf
        face[d][0, 0, :] = col
    s.face = face
    if metric is not None:
        s.metric = 1
        s.alpha = np.full(s.shape, metric[0])
        s.psi = np.full(s.shape, metric[1])
    return s


def steady_dynamo(n=128, k=1, eta=0.1, xi=0.5, rho=1e-14, p=1e-14, recon=MC, imex=SSP2, gamma=4.0 / 3.0):
    """1-D steady mean-field dynamo (Sec 5.7): periodic x in [-pi, pi], fluid
    at rest with the matter frozen, B^y = 0.1 sin(kx), B^z = -0.1 cos(kx),
    E = 0, xi = 0.5.  eta = 0.1 is the reading under which the printed growth
    rates hold (0.385 for k = 1, none for k = 5, 0.59 at the fastest k)."""
    s = _blank(Setup("steady_dynamo", 1, (n, 1, 1), 3 if recon == PPM else 2, (-math.pi, 0, 0), (math.pi, 1, 1),
                     _bc(1, PERIODIC), gamma, recon, imex, eta=eta, rho_atm=1e-3 * rho, p_atm=1e-3 * p, xi=xi,
                     frozen_matter=1))
    X, _, _ = s.mesh()
    s.prim[0] = rho
    s.prim[4] = p
    face = np.zeros((3,) + s.shape)
    face[1] = 0.1 * np.sin(k * X)
    face[2] = -0.1 * np.cos(k * X)
    s.face = face
    return s


def glm_wave(n=128, k=1, kappa=1.0, b=1e-3, rho=1.0, p=1.0, recon=MC, imex=SSP2):
    """1-D periodic x in [-pi, pi], fluid at rest and frozen, B^x = b sin(kx)
    (a pure divergence), E = 0, GLM with kappa_B = kappa_E = kappa.  The
    (B^x, Phi) pair obeys B'' + kappa B' + k^2 B = 0 (Sec 3.1 with v = 0)."""
    s = _blank(Setup("glm_wave", 1, (n, 1, 1), 3 if recon == PPM else 2, (-math.pi, 0, 0), (math.pi, 1, 1),
                     _bc(1, PERIODIC), 5.0 / 3.0, recon, imex, eta=1e-3, rho_atm=1e-6 * rho, p_atm=1e-6 * p,
                     frozen_matter=1, glm=1, kappa_E=kappa, kappa_B=kappa))
    X, _, _ = s.mesh()
    s.prim[0] = rho
    s.prim[4] = p
    face = np.zeros((3,) + s.shape)
    # the cell-centred field is the mean of the two faces: these face values
    # make it exactly b sin(k x_cell)
    dx = s.dx(0)
    face[0] = b * np.sin(k * (X - 0.5 * dx)) / math.cos(0.5 * k * dx)
    s.face = face
    return s


def glm_monopole(n=64, kappa=1.0, R=0.2, ndim=3, ext=2.0, recon=MC, imex=SSP2):
    """Gaussian magnetic monopole (Sec 5.1): B^x = exp(-r^2/R^2) - exp(-1) for
    r < R, uniform rho = 1, eps = 0.1 (p = (Gamma - 1) rho eps), v = 0,
    Gamma = 5/3, eta = 1e-16, GLM with kappa_E = kappa_B = kappa, domain
    [-ext, ext]^ndim, outflow."""
    nn = (n, n if ndim > 1 else 1, n if ndim > 2 else 1)
    lo = tuple(-ext if d < ndim else 0.0 for d in range(3))
    hi = tuple(ext if d < ndim else 1.0 for d in range(3))
    s = _blank(Setup("glm_monopole", ndim, nn, 3 if recon == PPM else 2, lo, hi, _bc(ndim, OUTFLOW), 5.0 / 3.0,
                     recon, imex, eta=1e-16, rho_atm=1e-8, p_atm=1e-10, glm=1, kappa_E=kappa, kappa_B=kappa))
    s.prim[0] = 1.0
    s.prim[4] = (5.0 / 3.0 - 1.0) * 0.1
    # faces: B^x at the x-faces from the profile at face positions
    X, Y, Z = s.mesh()
    Xf = (X - 0.5 * s.dx(0), Y, Z)
    r2 = sum(a ** 2 for a in Xf[:ndim])
    face = np.zeros((3,) + s.shape)
    face[0] = np.where(r2 < R * R, np.exp(-r2 / (R * R)) - math.exp(-1.0), 0.0)
    s.face = face
    return s


def dynamo_growth_rate(k, eta=0.1, xi=0.5):
    """growing root of g^2 + g/eta + k^2 - k xi/eta = 0: Maxwell's equations
    with the Ohm's law J = (E - xi B)/eta of a fluid at rest, for the
    force-free mode curl B = -k B of the initial field"""
    b = 1.0 / eta
    c = k * k - k * xi / eta
    return 0.5 * (-b + math.sqrt(b * b - 4.0 * c))


# ---------------------------------------------------------------------------
# many-run workloads: a batch of independent runs and a served request trace
def _u01(seed, stream, count):
    return 0.5 * (uniform_pm1(seed, stream, count) + 1.0)


def _log_uniform(u, lo, hi):
    return np.exp(np.log(lo) + u * (np.log(hi) - np.log(lo)))


def batch_mix_params(nruns=256, seed=1, n1=(128, 4096), n2=(64, 256), eta=(1e-6, 1.0)):
    """Parameters of a mix of independent runs: kind ~ Bernoulli(1/2); 1-D
    shock tubes with N ~ U{n1}, rho_L ~ U[0.125, 1], rho_R ~ U[0.125, rho_L],
    p_L ~ U[0.1, 1], p_R ~ U[0.1, p_L], By_L ~ U[-0.5, 0.5], Bx = 0.5, minmod;
    2-D blast waves with side ~ U{n2}, p_in ~ logU[1e-2, 1], p_out = 1e-3,
    Bx ~ U[0, 0.1], PPM; eta ~ logU[eta]; IMEX-SSP2(2,2,2) for all.  Every
    draw comes from the counter-based generator (stream 100 + k)."""
    u = [_u01(seed, 100 + k, nruns) for k in range(8)]
    out = []
    for i in range(nruns):
        e = float(_log_uniform(u[1][i], *eta))
        if u[0][i] < 0.5:
            n = int(n1[0] + min(int(u[2][i] * (n1[1] - n1[0] + 1)), n1[1] - n1[0]))
            rho_l = 0.125 + u[3][i] * (1.0 - 0.125)
            rho_r = 0.125 + u[4][i] * (rho_l - 0.125)
            p_l = 0.1 + u[5][i] * 0.9
            p_r = 0.1 + u[6][i] * (p_l - 0.1)
            by_l = -0.5 + u[7][i]
            out.append(dict(kind="shock_tube", n=n, eta=e, rho_l=rho_l, rho_r=rho_r, p_l=p_l, p_r=p_r,
                            by_l=by_l, seed=seed + i))
        else:
            n = int(n2[0] + min(int(u[2][i] * (n2[1] - n2[0] + 1)), n2[1] - n2[0]))
            p_in = float(_log_uniform(u[3][i], 1e-2, 1.0))
            bx = 0.1 * u[4][i]
            out.append(dict(kind="blast_wave", n=n, eta=e, p_in=p_in, bx=bx, seed=seed + i))
    return out


def make_run_setup(prm, imex=SSP2):
    """Setup of one entry of batch_mix_params / served_trace"""
    k = prm["kind"]
    if k == "shock_tube":
        return shock_tube(prm["n"], seed=prm["seed"], eta=prm["eta"], recon=MINMOD, imex=imex, rho_l=prm["rho_l"],
                          rho_r=prm["rho_r"], p_l=prm["p_l"], p_r=prm["p_r"], by_l=prm["by_l"])
    if k == "blast_wave":
        return blast_wave(prm["n"], eta=prm["eta"], seed=prm["seed"], recon=PPM, imex=imex,
                          p_in=prm.get("p_in", 1.0), bx=prm.get("bx", 0.1))
    if k == "tov_star":
        return tov_star(prm["n"], imex=imex, eta_in=prm["eta"])
    raise ValueError(k)


def served_trace(nreq=2000, rate=200.0, seed=7, blast=(64, 512), star=(32, 96), steps=(10, 500), eta=(1e-6, 1.0)):
    """Poisson request stream: exponential inter-arrival times of mean 1/rate;
    half 2-D blast waves (side ~ U{blast}, PPM + SSP3) and half 3-D stars
    (side ~ U{star}, PPM + SSP3, eta ~ logU[eta] inside the star); steps ~
    U{steps}."""
    u = [_u01(seed, 200 + k, nreq) for k in range(5)]
    t = np.cumsum(-np.log(1.0 - u[0]) / rate)
    out = []
    for i in range(nreq):
        e = float(_log_uniform(u[2][i], *eta))
        ns = int(steps[0] + min(int(u[3][i] * (steps[1] - steps[0] + 1)), steps[1] - steps[0]))
        if u[1][i] < 0.5:
            n = int(blast[0] + min(int(u[4][i] * (blast[1] - blast[0] + 1)), blast[1] - blast[0]))
            prm = dict(kind="blast_wave", n=n, eta=e, seed=seed + i)
        else:
            n = int(star[0] + min(int(u[4][i] * (star[1] - star[0] + 1)), star[1] - star[0]))
            prm = dict(kind="tov_star", n=n, eta=e, seed=seed + i)
        prm.update(rid=i, arrival=float(t[i]), steps=ns)
        out.append(prm)
    return out
