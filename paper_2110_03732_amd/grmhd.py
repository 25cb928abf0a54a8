"""Thin ctypes binding of the C ABI in include/grmhd.h (libgrmhd.so).

Function names are those of the C ABI.  PyTorch is used only for device
memory and streams: every step of the method runs in the library's HIP
kernels.  Loading fails loudly when the built library is missing.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgrmhd.so")

GR_OK, GR_EINVAL, GR_ENOMEM, GR_EHIP, GR_EUNSUPPORTED = 0, -1, -2, -3, -4
EXPORTED = ["gr_abi_version", "gr_strerror", "gr_validate", "gr_field_stride", "gr_row_stride", "gr_field_origin",
            "gr_workspace_bytes",
            "gr_workspace_offset", "gr_init_state", "gr_imex_stage", "gr_step", "gr_con2prim", "gr_divB_norm",
            "gr_cfl_dt", "gr_fail_count", "gr_timing_start", "gr_timing_read", "gr_kernel_class_name",
            "gr_clean_divB", "gr_batch_create", "gr_batch_update", "gr_batch_set_dt", "gr_batch_step", "gr_batch_run",
            "gr_batch_stats", "gr_batch_tiles", "gr_tile_name", "gr_batch_destroy", "gr_stream_read", "gr_stream_copy",
            "gr_divB_norm_noalloc"]


class GrError(RuntimeError):
    pass


class gr_grid(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int), ("n", ctypes.c_int * 3), ("ng", ctypes.c_int),
                ("lo", ctypes.c_double * 3), ("hi", ctypes.c_double * 3), ("bc", (ctypes.c_int * 2) * 3),
                ("gamma_ad", ctypes.c_double), ("recon", ctypes.c_int), ("imex", ctypes.c_int),
                ("cfl", ctypes.c_double), ("eta_mode", ctypes.c_int), ("eta", ctypes.c_double),
                ("sigma0", ctypes.c_double), ("eta_min", ctypes.c_double), ("eta_max", ctypes.c_double),
                ("rho_atm", ctypes.c_double), ("p_atm", ctypes.c_double), ("metric", ctypes.c_int),
                ("newton_tol", ctypes.c_double), ("newton_maxit", ctypes.c_int), ("xi", ctypes.c_double),
                ("atm_factor", ctypes.c_double), ("frozen_matter", ctypes.c_int), ("glm", ctypes.c_int),
                ("kappa_E", ctypes.c_double), ("kappa_B", ctypes.c_double), ("uct", ctypes.c_int)]


class gr_state(ctypes.Structure):
    _fields_ = [("q", ctypes.c_void_p), ("face", ctypes.c_void_p), ("prim", ctypes.c_void_p),
                ("metric", ctypes.c_void_p), ("work", ctypes.c_void_p), ("work_bytes", ctypes.c_size_t)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise GrError("libgrmhd.so is not built (run __graft_entry__.build()): %s" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        G = ctypes.POINTER(gr_grid)
        S = ctypes.POINTER(gr_state)
        V = ctypes.c_void_p
        D = ctypes.POINTER(ctypes.c_double)
        L.gr_abi_version.restype = ctypes.c_int
        L.gr_strerror.restype = ctypes.c_char_p
        L.gr_strerror.argtypes = [ctypes.c_int]
        L.gr_validate.argtypes = [G]
        L.gr_field_stride.argtypes = [G]
        L.gr_field_stride.restype = ctypes.c_size_t
        L.gr_row_stride.argtypes = [G]
        L.gr_row_stride.restype = ctypes.c_size_t
        L.gr_field_origin.argtypes = [G]
        L.gr_field_origin.restype = ctypes.c_size_t
        L.gr_workspace_bytes.argtypes = [G]
        L.gr_workspace_bytes.restype = ctypes.c_size_t
        L.gr_workspace_offset.argtypes = [G, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)]
        L.gr_init_state.argtypes = [G, S, D, D, D, D, D, V]
        L.gr_imex_stage.argtypes = [G, S, ctypes.c_int, ctypes.c_double, V]
        L.gr_step.argtypes = [G, S, ctypes.c_double, V]
        L.gr_con2prim.argtypes = [G, S, V]
        L.gr_divB_norm.argtypes = [G, S, V, V]
        L.gr_divB_norm_noalloc.argtypes = [G, S, V, V]
        L.gr_clean_divB.argtypes = [G, S, ctypes.c_int, V, V]
        L.gr_clean_divB.restype = ctypes.c_int
        L.gr_cfl_dt.argtypes = [G, S, D, V]
        L.gr_fail_count.argtypes = [G, S, ctypes.POINTER(ctypes.c_ulonglong), V]
        L.gr_timing_start.argtypes = [ctypes.c_uint]
        L.gr_timing_read.argtypes = [ctypes.c_int, D, ctypes.POINTER(ctypes.c_long), D]
        L.gr_kernel_class_name.argtypes = [ctypes.c_int]
        L.gr_kernel_class_name.restype = ctypes.c_char_p
        PB = ctypes.POINTER(ctypes.c_void_p)
        L.gr_batch_create.argtypes = [PB, G, S, D, ctypes.c_int, ctypes.c_char_p, V]
        L.gr_batch_update.argtypes = [V, G, S, D, ctypes.c_int, V]
        L.gr_batch_set_dt.argtypes = [V, D, V]
        L.gr_batch_step.argtypes = [V, V]
        L.gr_batch_run.argtypes = [V, ctypes.c_int, V]
        L.gr_batch_stats.argtypes = [V, ctypes.POINTER(ctypes.c_int), D, ctypes.POINTER(ctypes.c_long)]
        L.gr_batch_tiles.argtypes = [V, ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
        L.gr_tile_name.argtypes = [ctypes.c_int, ctypes.c_int]
        L.gr_tile_name.restype = ctypes.c_char_p
        L.gr_batch_destroy.argtypes = [V]
        L.gr_stream_read.argtypes = [V, ctypes.c_size_t, V, V]
        L.gr_stream_copy.argtypes = [V, V, ctypes.c_size_t, V]
        for name in ("gr_batch_create", "gr_batch_update", "gr_batch_set_dt", "gr_batch_step", "gr_batch_run",
                     "gr_batch_stats", "gr_batch_tiles", "gr_batch_destroy", "gr_stream_read", "gr_stream_copy"):
            getattr(L, name).restype = ctypes.c_int
        for name in ("gr_timing_start", "gr_timing_read", "gr_validate", "gr_workspace_offset", "gr_init_state", "gr_imex_stage", "gr_step", "gr_con2prim",
                     "gr_divB_norm", "gr_divB_norm_noalloc", "gr_cfl_dt", "gr_fail_count"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _chk(r):
    if r != GR_OK:
        raise GrError("libgrmhd: %s (%d)" % (lib().gr_strerror(r).decode(), r))


# ---------------------------------------------------------------------------
# C-ABI wrappers (same names); argument marshalling only
def gr_abi_version():
    return lib().gr_abi_version()


def gr_validate(grid):
    return lib().gr_validate(ctypes.byref(grid))


def gr_field_stride(grid):
    return lib().gr_field_stride(ctypes.byref(grid))


def gr_row_stride(grid):
    return lib().gr_row_stride(ctypes.byref(grid))


def gr_field_origin(grid):
    return lib().gr_field_origin(ctypes.byref(grid))


def gr_workspace_bytes(grid):
    return lib().gr_workspace_bytes(ctypes.byref(grid))


def gr_workspace_offset(grid, kind, stage, field):
    off = ctypes.c_size_t(0)
    _chk(lib().gr_workspace_offset(ctypes.byref(grid), kind, stage, field, ctypes.byref(off)))
    return off.value


def _hp(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def gr_init_state(grid, state, prim_host, E_host, A_host, face_host, metric_host, stream):
    _chk(lib().gr_init_state(ctypes.byref(grid), ctypes.byref(state), _hp(prim_host), _hp(E_host), _hp(A_host),
                             _hp(face_host), _hp(metric_host), ctypes.c_void_p(stream)))


def gr_imex_stage(grid, state, p, dt, stream):
    _chk(lib().gr_imex_stage(ctypes.byref(grid), ctypes.byref(state), p, dt, ctypes.c_void_p(stream)))


def gr_step(grid, state, dt, stream):
    _chk(lib().gr_step(ctypes.byref(grid), ctypes.byref(state), dt, ctypes.c_void_p(stream)))


def gr_con2prim(grid, state, stream):
    _chk(lib().gr_con2prim(ctypes.byref(grid), ctypes.byref(state), ctypes.c_void_p(stream)))


def gr_divB_norm(grid, state, out3_dev_ptr, stream):
    _chk(lib().gr_divB_norm(ctypes.byref(grid), ctypes.byref(state), ctypes.c_void_p(out3_dev_ptr),
                            ctypes.c_void_p(stream)))


def gr_divB_norm_noalloc(grid, state, out3_dev_ptr, stream):
    _chk(lib().gr_divB_norm_noalloc(ctypes.byref(grid), ctypes.byref(state), ctypes.c_void_p(out3_dev_ptr),
                                    ctypes.c_void_p(stream)))


def gr_clean_divB(grid, state, vcycles, out6_dev_ptr, stream):
    _chk(lib().gr_clean_divB(ctypes.byref(grid), ctypes.byref(state), int(vcycles), ctypes.c_void_p(out6_dev_ptr),
                             ctypes.c_void_p(stream)))


def gr_cfl_dt(grid, state, stream):
    dt = ctypes.c_double(0.0)
    _chk(lib().gr_cfl_dt(ctypes.byref(grid), ctypes.byref(state), ctypes.byref(dt), ctypes.c_void_p(stream)))
    return dt.value


def gr_fail_count(grid, state, stream):
    c = ctypes.c_ulonglong(0)
    _chk(lib().gr_fail_count(ctypes.byref(grid), ctypes.byref(state), ctypes.byref(c), ctypes.c_void_p(stream)))
    return c.value


def gr_timing_start(mask):
    _chk(lib().gr_timing_start(mask))


def gr_timing_read(kernel_class):
    ms = ctypes.c_double(0.0)
    n = ctypes.c_long(0)
    by = ctypes.c_double(0.0)
    _chk(lib().gr_timing_read(kernel_class, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(by)))
    return ms.value, n.value, by.value


def gr_kernel_class_name(kernel_class):
    return lib().gr_kernel_class_name(kernel_class).decode()


def gr_batch_create(grids, states, dt, tune_cache, stream):
    n = len(grids)
    ga = (gr_grid * n)(*grids)
    sa = (gr_state * n)(*states)
    da = (ctypes.c_double * n)(*[float(x) for x in dt])
    h = ctypes.c_void_p()
    tc = None if tune_cache is None else tune_cache.encode()
    _chk(lib().gr_batch_create(ctypes.byref(h), ga, sa, da, n, tc, stream))
    return h


def gr_batch_update(batch, grids, states, dt, stream):
    n = len(grids)
    ga = (gr_grid * n)(*grids)
    sa = (gr_state * n)(*states)
    da = (ctypes.c_double * n)(*[float(x) for x in dt])
    _chk(lib().gr_batch_update(batch, ga, sa, da, n, stream))


def gr_stream_read(src_dev_ptr, nbytes, sink_dev_ptr, stream):
    _chk(lib().gr_stream_read(src_dev_ptr, nbytes, sink_dev_ptr, stream))


def gr_stream_copy(src_dev_ptr, dst_dev_ptr, nbytes, stream):
    _chk(lib().gr_stream_copy(src_dev_ptr, dst_dev_ptr, nbytes, stream))


def gr_batch_set_dt(batch, dt, stream):
    da = (ctypes.c_double * len(dt))(*[float(x) for x in dt])
    _chk(lib().gr_batch_set_dt(batch, da, stream))


def gr_batch_step(batch, stream):
    _chk(lib().gr_batch_step(batch, stream))


def gr_batch_run(batch, nsteps, stream):
    _chk(lib().gr_batch_run(batch, int(nsteps), stream))


def gr_batch_stats(batch):
    n = ctypes.c_int()
    by = ctypes.c_double()
    c = ctypes.c_long()
    _chk(lib().gr_batch_stats(batch, ctypes.byref(n), ctypes.byref(by), ctypes.byref(c)))
    return n.value, by.value, c.value


def gr_batch_tiles(batch, run):
    a = ctypes.c_int()
    b = ctypes.c_int()
    _chk(lib().gr_batch_tiles(batch, run, ctypes.byref(a), ctypes.byref(b)))
    return lib().gr_tile_name(0, a.value).decode(), lib().gr_tile_name(1, b.value).decode()


def gr_batch_destroy(batch):
    _chk(lib().gr_batch_destroy(batch))


# ---------------------------------------------------------------------------
def grid_of(s) -> gr_grid:
    """gr_grid of a workloads.Setup"""
    g = gr_grid()
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


class Run:
    """Device state of one run: torch tensors for the field blocks and the
    workspace, and the gr_grid / gr_state structs that point at them."""

    def __init__(self, setup, device="cuda", stream=None):
        import torch
        self.torch = torch
        self.setup = setup
        self.grid = grid_of(setup)
        r = gr_validate(self.grid)
        _chk(r)
        self.fs = gr_field_stride(self.grid)
        self.np = int(np.prod(setup.shape))
        self.pitch = gr_row_stride(self.grid)  # padded device rows
        self.origin = gr_field_origin(self.grid)
        dev = torch.device(device)
        self.nq = 10 if setup.glm else 8
        self.q = torch.zeros(self.nq * self.fs, dtype=torch.float64, device=dev)
        self.face = torch.zeros(3 * self.fs, dtype=torch.float64, device=dev)
        self.prim = torch.zeros(5 * self.fs, dtype=torch.float64, device=dev)
        self.metric = torch.zeros(2 * self.fs, dtype=torch.float64, device=dev) if setup.metric else None
        wb = gr_workspace_bytes(self.grid)
        self.work = torch.zeros((wb + 7) // 8, dtype=torch.float64, device=dev)
        self.state = gr_state()
        self.state.q = self.q.data_ptr()
        self.state.face = self.face.data_ptr()
        self.state.prim = self.prim.data_ptr()
        self.state.metric = self.metric.data_ptr() if self.metric is not None else None
        self.state.work = self.work.data_ptr()
        self.state.work_bytes = wb
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        s = setup
        prim = np.ascontiguousarray(s.prim.reshape(5, -1))
        E = np.ascontiguousarray(s.E.reshape(3, -1))
        A = np.ascontiguousarray(s.A.reshape(3, -1)) if s.A is not None else None
        face = np.ascontiguousarray(s.face.reshape(3, -1)) if s.face is not None else None
        met = np.ascontiguousarray(np.stack([s.alpha, s.psi]).reshape(2, -1)) if s.metric else None
        gr_init_state(self.grid, self.state, prim, E, A, face, met, self.stream.cuda_stream)
        self.t = 0.0

    # --- stepping ---------------------------------------------------------
    def dt(self):
        return gr_cfl_dt(self.grid, self.state, self.stream.cuda_stream)

    def step(self, dt):
        gr_step(self.grid, self.state, dt, self.stream.cuda_stream)
        self.t += dt

    def stage(self, p, dt):
        gr_imex_stage(self.grid, self.state, p, dt, self.stream.cuda_stream)

    def con2prim(self):
        gr_con2prim(self.grid, self.state, self.stream.cuda_stream)

    def divB(self):
        out = self.torch.zeros(3, dtype=self.torch.float64, device=self.q.device)
        gr_divB_norm(self.grid, self.state, out.data_ptr(), self.stream.cuda_stream)
        self.stream.synchronize()
        return out.cpu().numpy()

    def clean_divB(self, vcycles=10):
        """elliptic cleaning of the face fields; returns (L1, L2, Linf) of
        div q_B before and after"""
        out = self.torch.zeros(6, dtype=self.torch.float64, device=self.q.device)
        gr_clean_divB(self.grid, self.state, vcycles, out.data_ptr(), self.stream.cuda_stream)
        self.stream.synchronize()
        o = out.cpu().numpy()
        return o[:3], o[3:]

    def fail_count(self):
        return gr_fail_count(self.grid, self.state, self.stream.cuda_stream)

    # --- views (host copies) ------------------------------------------------
    def offset(self, i, j, k):
        """index of point (i, j, k) inside a device field (padded rows)"""
        Nz, Ny, Nx = self.setup.shape
        return self.origin + i + self.pitch * (j + Ny * k)

    def _unpad(self, a):
        """device field values (..., fs) -> compact (..., Nz, Ny, Nx)"""
        Nz, Ny, Nx = self.setup.shape
        lead = a.shape[:-1]
        a = a[..., self.origin: self.origin + self.pitch * Ny * Nz].reshape(lead + (Nz, Ny, self.pitch))
        return np.ascontiguousarray(a[..., :Nx])

    def _block(self, t, nf):
        self.stream.synchronize()
        return self._unpad(t.view(nf, self.fs).cpu().numpy())

    def prims(self):
        return self._block(self.prim, 5)

    def cons(self):
        return self._block(self.q, self.nq)

    def faces(self):
        return self._block(self.face, 3)

    def work_field(self, kind, stage, field):
        off = gr_workspace_offset(self.grid, kind, stage, field) // 8
        self.stream.synchronize()
        return self._unpad(self.work[off: off + self.fs].cpu().numpy())


class Batch:
    """Many independent Runs advanced together (gr_batch_*).  The runs keep
    their own device state; the batch holds the launch list of one step."""

    def __init__(self, runs, dts, tune_cache=None, stream=None):
        if not runs:
            raise ValueError("empty batch")
        self.runs = list(runs)
        self.dts = [float(x) for x in dts]
        self.stream = stream if stream is not None else runs[0].stream
        self.h = gr_batch_create([r.grid for r in self.runs], [r.state for r in self.runs], self.dts, tune_cache,
                                 self.stream.cuda_stream)

    def update(self, runs, dts):
        """replace the batch's runs (stream-ordered, no host synchronisation);
        the runs' state must stay alive while the batch may still use it"""
        if not runs:
            raise ValueError("empty batch")
        self.runs = list(runs)
        self.dts = [float(x) for x in dts]
        gr_batch_update(self.h, [r.grid for r in self.runs], [r.state for r in self.runs], self.dts,
                        self.stream.cuda_stream)

    def set_dt(self, dts):
        """new time steps for the batch's runs (stream-ordered)"""
        dts = [float(x) for x in dts]
        if len(dts) != len(self.runs):
            raise ValueError("one time step per run")
        gr_batch_set_dt(self.h, dts, self.stream.cuda_stream)
        self.dts = dts

    def step(self):
        gr_batch_step(self.h, self.stream.cuda_stream)
        for r, dt in zip(self.runs, self.dts):
            r.t += dt

    def run(self, nsteps):
        gr_batch_run(self.h, nsteps, self.stream.cuda_stream)
        for r, dt in zip(self.runs, self.dts):
            r.t += nsteps * dt

    def stats(self):
        return gr_batch_stats(self.h)

    def tiles(self, i):
        return gr_batch_tiles(self.h, i)

    def close(self):
        if self.h is not None:
            self.stream.synchronize()
            gr_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
