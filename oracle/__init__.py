"""ctypes wrapper of the CPU Yee oracle -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The GPU library never calls it.

Fields are numpy arrays of shape (6, nz+1, ny+1, nx+1) (x fastest), in
component order Ex, Ey, Ez, Hx, Hy, Hz; H is stored as eta0*H.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_fp = np.ctypeslib.ndpointer(dtype=np.float32, flags="C_CONTIGUOUS")
_u8 = np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS")
_ip = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_u16 = np.ctypeslib.ndpointer(dtype=np.uint16, flags="C_CONTIGUOUS")
_i = C.c_int
_l = C.c_long


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        L = C.CDLL(_LIB_PATH)
        L.orc_coefficients.argtypes = [_i, _dp, _dp, C.c_double, C.c_double, C.c_double, C.c_double, _dp, _dp]
        L.orc_h_half_f64.argtypes = [_i, _i, _i, _dp, _dp]
        L.orc_e_half_f64.argtypes = [_i, _i, _i, _dp, _u8, _dp]
        L.orc_h_half_f32.argtypes = [_i, _i, _i, _fp, _fp]
        L.orc_e_half_f32.argtypes = [_i, _i, _i, _fp, _u8, _fp]
        L.orc_run_f64.argtypes = [_i, _i, _i, _dp, _dp, _u8, _dp, _l, _i, _i, _ip, _dp, _i, _i, _ip, _dp]
        L.orc_run_f64.restype = _i
        L.orc_run_f32.argtypes = [_i, _i, _i, _fp, _fp, _u8, _fp, _l, _i, _i, _ip, _fp, _i, _i, _ip, _dp]
        L.orc_run_f32.restype = _i
        L.orc_run_q.argtypes = [_i, _i, _i, _i, _i, _fp, _fp, _u8, _fp, _l, _i, _i, _ip, _fp, _i, _i, _ip, _dp,
                                C.c_float, _ip, _fp, _ip]
        L.orc_run_q.restype = _i
        L.orc_quantize_bits.argtypes = [_i, _i, _fp, _u16]
        L.orc_choose_scales.argtypes = [_fp, C.c_float, _ip]
        L.orc_quantize_state.argtypes = [_i, _i, _i, _i, _i, C.c_float, _fp, _ip, _fp, _ip]
        L.orc_energy_f64.argtypes = [_i, _i, _i, _dp, _dp, _u8, _dp]
        L.orc_energy_f64.restype = C.c_double
        L.orc_energy_f32.argtypes = [_i, _i, _i, _fp, _dp, _u8, _fp]
        L.orc_energy_f32.restype = C.c_double
        L.orc_threads.restype = _i
        L.orc_set_threads.argtypes = [_i]
        L.orc_set_threads.restype = None
        L.orc_divergence_f64.argtypes = [_i, _i, _i, C.c_double, C.c_double, C.c_double, _dp, _u8, _dp, _dp, _dp]
        L.orc_graded_coefficients.argtypes = [_i, _dp, _dp, C.c_double, _i, _i, _i, _dp, _dp, _dp, _dp, _dp, _dp]
        L.orc_h_half_graded_f64.argtypes = [_i, _i, _i, _dp, _dp]
        L.orc_e_half_graded_f64.argtypes = [_i, _i, _i, _dp, _dp, _u8, _dp]
        L.orc_h_half_graded_f32.argtypes = [_i, _i, _i, _fp, _fp]
        L.orc_e_half_graded_f32.argtypes = [_i, _i, _i, _fp, _fp, _u8, _fp]
        L.orc_run_graded_f64.argtypes = [_i, _i, _i, _dp, _dp, _dp, _u8, _dp, _l, _i, _i, _ip, _dp, _i, _i, _ip,
                                         _dp]
        L.orc_run_graded_f64.restype = _i
        L.orc_run_graded_f32.argtypes = [_i, _i, _i, _fp, _fp, _fp, _u8, _fp, _l, _i, _i, _ip, _fp, _i, _i, _ip,
                                         _dp]
        L.orc_run_graded_f32.restype = _i
        L.orc_energy_graded_f64.argtypes = [_i, _i, _i, _dp, _dp, _dp, _dp, _dp, _u8, _dp]
        L.orc_energy_graded_f64.restype = C.c_double
        L.orc_divergence_graded_f64.argtypes = [_i, _i, _i, _dp, _dp, _dp, _dp, _u8, _dp, _dp, _dp]
        L.orc_energy_graded_f32.argtypes = [_i, _i, _i, _dp, _dp, _dp, _fp, _dp, _u8, _fp]
        L.orc_energy_graded_f32.restype = C.c_double
        L.orc_cpml_coefficients.argtypes = [_i, _dp, _dp, C.c_double, _i, _i, _i, _dp, _dp, _dp, _i, _i,
                                            C.c_double, C.c_double, C.c_double, _dp, _dp, _dp, _dp]
        L.orc_cpml_coefficients.restype = _i
        L.orc_run_cpml_f64.argtypes = [_i, _i, _i, _i, _dp, _dp, _dp, _dp, _u8, _dp, _dp, _l, _i, _i, _ip, _dp,
                                       _i, _i, _ip, _dp]
        L.orc_run_cpml_f64.restype = _i
        L.orc_run_cpml_f32.argtypes = [_i, _i, _i, _i, _fp, _fp, _fp, _fp, _u8, _fp, _fp, _l, _i, _i, _ip, _fp,
                                       _i, _i, _ip, _dp]
        L.orc_run_cpml_f32.restype = _i
        L.orc_run_q_graded.argtypes = [_i, _i, _i, _i, _i, _fp, _fp, _fp, _u8, _fp, _l, _i, _i, _ip, _fp, _i, _i,
                                       _ip, _dp, C.c_float, _ip, _fp, _ip]
        L.orc_run_q_graded.restype = _i
        _lib = L
    return _lib


def coefficients(eps_r, sigma, dt, dx, dy, dz):
    """(coef (n_mat, 4) = Ca, Cbx, Cby, Cbz; ch (3,)) in float64."""
    eps_r = np.ascontiguousarray(eps_r, dtype=np.float64)
    sigma = np.ascontiguousarray(sigma, dtype=np.float64)
    coef = np.zeros((len(eps_r), 4))
    ch = np.zeros(3)
    lib().orc_coefficients(len(eps_r), eps_r, sigma, dt, dx, dy, dz, coef, ch)
    return coef, ch


def graded_coefficients(eps_r, sigma, dt, dx, dy, dz):
    """Graded spacing (per-index primal cell sizes dx (nx,), dy (ny,), dz (nz,)):
    (cag (n_mat, 2) = Ca, G; hc and ec: x, y and z arrays concatenated,
    (nx+1)+(ny+1)+(nz+1) values) in float64."""
    eps_r = np.ascontiguousarray(eps_r, dtype=np.float64)
    sigma = np.ascontiguousarray(sigma, dtype=np.float64)
    dx, dy, dz = (np.ascontiguousarray(a, dtype=np.float64) for a in (dx, dy, dz))
    n = len(dx) + len(dy) + len(dz) + 3
    cag, hc, ec = np.zeros((len(eps_r), 2)), np.zeros(n), np.zeros(n)
    lib().orc_graded_coefficients(len(eps_r), eps_r, sigma, dt, len(dx), len(dy), len(dz), dx, dy, dz,
                                  cag, hc, ec)
    return cag, hc, ec


def cpml_coefficients(eps_r, sigma, dt, dx, dy, dz, thickness, order=3, sigma_factor=1.0, kappa_max=1.0,
                      alpha_max=0.0):
    """CPML layers of `thickness` cells on every face over per-index cell sizes:
    (cag (n_mat, 2), hc, ec with kappa folded in, cp ((nx+1)+(ny+1)+(nz+1), 6) =
    b_h, a_h, c dt / d, b_e, a_e, c dt / d') in float64."""
    eps_r = np.ascontiguousarray(eps_r, dtype=np.float64)
    sigma = np.ascontiguousarray(sigma, dtype=np.float64)
    dx, dy, dz = (np.ascontiguousarray(a, dtype=np.float64) for a in (dx, dy, dz))
    n = len(dx) + len(dy) + len(dz) + 3
    cag, hc, ec, cp = np.zeros((len(eps_r), 2)), np.zeros(n), np.zeros(n), np.zeros((n, 6))
    rc = lib().orc_cpml_coefficients(len(eps_r), eps_r, sigma, dt, len(dx), len(dy), len(dz), dx, dy, dz,
                                     thickness, order, sigma_factor, kappa_max, alpha_max, cag, hc, ec, cp)
    if rc:
        raise ValueError("CPML layers must leave an interior on every axis")
    return cag, hc, ec, cp


def zero_fields(nx, ny, nz, dtype=np.float64):
    return np.zeros((6, nz + 1, ny + 1, nx + 1), dtype=dtype)


def _points(pts):
    return np.ascontiguousarray(np.array(pts, dtype=np.int32).reshape(-1, 4))


class Problem:
    """A grid, its material table and per-cell indices, sources and probes."""

    def __init__(self, nx, ny, nz, dx, dy, dz, dt, eps_r, sigma, mat,
                 sources=(), waveforms=None, probes=(), spacing=None, cpml=None):
        self.nx, self.ny, self.nz = nx, ny, nz
        self.dx, self.dy, self.dz, self.dt = dx, dy, dz, dt
        self.eps_r = np.ascontiguousarray(eps_r, dtype=np.float64)
        self.sigma = np.ascontiguousarray(sigma, dtype=np.float64)
        self.mat = np.ascontiguousarray(mat, dtype=np.uint8).reshape(nz, ny, nx)
        self.coef64, self.ch64 = coefficients(self.eps_r, self.sigma, dt, dx, dy, dz)
        self.coef32 = self.coef64.astype(np.float32)
        self.ch32 = self.ch64.astype(np.float32)
        self.src = _points(sources)
        if waveforms is None or len(self.src) == 0:
            self.wave64 = np.zeros((max(len(self.src), 1), 1))
        else:
            self.wave64 = np.ascontiguousarray(np.asarray(waveforms, dtype=np.float64).reshape(len(self.src), -1))
        self.wave32 = self.wave64.astype(np.float32)
        self.probe = _points(probes)
        # graded spacing: per-index primal cell sizes (dx (nx,), dy (ny,), dz (nz,))
        self.graded = spacing is not None
        if self.graded:
            self.sx, self.sy, self.sz = (np.ascontiguousarray(a, dtype=np.float64) for a in spacing)
            assert (len(self.sx), len(self.sy), len(self.sz)) == (nx, ny, nz)
            self.cag64, self.hc64, self.ec64 = graded_coefficients(self.eps_r, self.sigma, dt,
                                                                   self.sx, self.sy, self.sz)
            self.cag32, self.hc32, self.ec32 = (a.astype(np.float32) for a in (self.cag64, self.hc64, self.ec64))
        # CPML layers (dict: thickness, order, sigma_factor, kappa_max, alpha_max) on top of
        # the graded update (uniform sizes become per-index arrays)
        self.cpml = dict(cpml) if cpml else None
        if self.cpml:
            if not self.graded:
                self.graded = True
                self.sx, self.sy, self.sz = np.full(nx, float(dx)), np.full(ny, float(dy)), np.full(nz, float(dz))
            self.cag64, self.hc64, self.ec64, self.cp64 = cpml_coefficients(
                self.eps_r, self.sigma, dt, self.sx, self.sy, self.sz, **self.cpml)
            self.cag32, self.hc32, self.ec32, self.cp32 = (a.astype(np.float32) for a in
                                                           (self.cag64, self.hc64, self.ec64, self.cp64))
            self.reset_psi()

    def reset_psi(self):
        """Zero the CPML auxiliary state of both modes (12 arrays over the node
        box each, allocated when a mode first runs)."""
        self._psi = {}

    def _psi_of(self, dtype):
        key = np.dtype(dtype).name
        if key not in self._psi:
            self._psi[key] = np.zeros((12, self.nz + 1, self.ny + 1, self.nx + 1), dtype)
        return self._psi[key]

    @property
    def psi64(self):
        return self._psi_of(np.float64)

    @property
    def psi32(self):
        return self._psi_of(np.float32)

    @classmethod
    def from_workload(cls, wl):
        return cls(wl.nx, wl.ny, wl.nz, wl.dx, wl.dy, wl.dz, wl.dt, wl.eps_r, wl.sigma, wl.mat,
                   wl.sources, wl.waveforms, wl.probes, spacing=getattr(wl, "spacing", None),
                   cpml=getattr(wl, "cpml", None))

    @property
    def a_max(self) -> float:
        return float(np.max(np.abs(self.wave32))) if len(self.src) else 0.0

    def run_f64(self, f, step0, n_steps):
        """Advance f (float64, in place); returns probes (n_steps, n_probe) float64."""
        assert f.dtype == np.float64 and f.flags.c_contiguous
        out = np.zeros((n_steps, max(len(self.probe), 1)))
        if self.cpml:
            rc = lib().orc_run_cpml_f64(self.nx, self.ny, self.nz, self.cpml["thickness"], self.hc64, self.cag64,
                                        self.ec64, self.cp64, self.mat, f, self.psi64, step0, n_steps,
                                        len(self.src), self.src, self.wave64, self.wave64.shape[1],
                                        len(self.probe), self.probe, out)
        elif self.graded:
            rc = lib().orc_run_graded_f64(self.nx, self.ny, self.nz, self.hc64, self.cag64, self.ec64, self.mat, f,
                                          step0, n_steps, len(self.src), self.src, self.wave64,
                                          self.wave64.shape[1], len(self.probe), self.probe, out)
        else:
            rc = lib().orc_run_f64(self.nx, self.ny, self.nz, self.ch64, self.coef64, self.mat, f, step0,
                                   n_steps, len(self.src), self.src, self.wave64, self.wave64.shape[1],
                                   len(self.probe), self.probe, out)
        if rc:
            raise ValueError("bad source or probe descriptor")
        return out[:, :len(self.probe)]

    def run_f32(self, f, step0, n_steps):
        assert f.dtype == np.float32 and f.flags.c_contiguous
        out = np.zeros((n_steps, max(len(self.probe), 1)))
        if self.cpml:
            rc = lib().orc_run_cpml_f32(self.nx, self.ny, self.nz, self.cpml["thickness"], self.hc32, self.cag32,
                                        self.ec32, self.cp32, self.mat, f, self.psi32, step0, n_steps,
                                        len(self.src), self.src, self.wave32, self.wave32.shape[1],
                                        len(self.probe), self.probe, out)
        elif self.graded:
            rc = lib().orc_run_graded_f32(self.nx, self.ny, self.nz, self.hc32, self.cag32, self.ec32, self.mat, f,
                                          step0, n_steps, len(self.src), self.src, self.wave32,
                                          self.wave32.shape[1], len(self.probe), self.probe, out)
        else:
            rc = lib().orc_run_f32(self.nx, self.ny, self.nz, self.ch32, self.coef32, self.mat, f, step0,
                                   n_steps, len(self.src), self.src, self.wave32, self.wave32.shape[1],
                                   len(self.probe), self.probe, out)
        if rc:
            raise ValueError("bad source or probe descriptor")
        return out[:, :len(self.probe)]

    def run_q(self, f, step0, n_steps, fmt, T, state):
        """Reduced-storage emulation.  state: dict with 'scales' (6 int32),
        'm_stored' (6 float32), 'flag' (1 int32), updated in place."""
        assert f.dtype == np.float32 and f.flags.c_contiguous
        assert not self.cpml, "reduced storage is emulated without CPML layers"
        out = np.zeros((n_steps, max(len(self.probe), 1)))
        if self.graded:
            rc = lib().orc_run_q_graded(self.nx, self.ny, self.nz, fmt, T, self.hc32, self.cag32, self.ec32, self.mat,
                                        f, step0, n_steps, len(self.src), self.src, self.wave32, self.wave32.shape[1],
                                        len(self.probe), self.probe, out, self.a_max,
                                        state["scales"], state["m_stored"], state["flag"])
        else:
            rc = lib().orc_run_q(self.nx, self.ny, self.nz, fmt, T, self.ch32, self.coef32, self.mat, f, step0,
                                 n_steps, len(self.src), self.src, self.wave32, self.wave32.shape[1],
                                 len(self.probe), self.probe, out, self.a_max,
                                 state["scales"], state["m_stored"], state["flag"])
        if rc:
            raise ValueError("bad source or probe descriptor")
        return out[:, :len(self.probe)]

    def quantize_upload(self, f, fmt):
        """Quantise freshly uploaded float32 fields; returns the q-mode state."""
        st = {"scales": np.zeros(6, np.int32), "m_stored": np.zeros(6, np.float32),
              "flag": np.zeros(1, np.int32)}
        lib().orc_quantize_state(self.nx, self.ny, self.nz, fmt, 1, self.a_max, f,
                                 st["scales"], st["m_stored"], st["flag"])
        return st

    def h_half_f64(self, f):
        if self.graded:
            lib().orc_h_half_graded_f64(self.nx, self.ny, self.nz, self.hc64, f)
        else:
            lib().orc_h_half_f64(self.nx, self.ny, self.nz, self.ch64, f)

    def e_half_f64(self, f):
        if self.graded:
            lib().orc_e_half_graded_f64(self.nx, self.ny, self.nz, self.cag64, self.ec64, self.mat, f)
        else:
            lib().orc_e_half_f64(self.nx, self.ny, self.nz, self.coef64, self.mat, f)

    def h_half_f32(self, f):
        if self.graded:
            lib().orc_h_half_graded_f32(self.nx, self.ny, self.nz, self.hc32, f)
        else:
            lib().orc_h_half_f32(self.nx, self.ny, self.nz, self.ch32, f)

    def e_half_f32(self, f):
        if self.graded:
            lib().orc_e_half_graded_f32(self.nx, self.ny, self.nz, self.cag32, self.ec32, self.mat, f)
        else:
            lib().orc_e_half_f32(self.nx, self.ny, self.nz, self.coef32, self.mat, f)

    def energy(self, f):
        """Discrete energy (FP64): in units of eps0*dx*dy*dz on uniform grids,
        of eps0 (volumes in m^3) on graded ones."""
        if self.graded:
            if f.dtype == np.float32:
                f = np.ascontiguousarray(f)
                return lib().orc_energy_graded_f32(self.nx, self.ny, self.nz, self.sx, self.sy, self.sz,
                                                   self.hc32, self.eps_r, self.mat, f)
            f = np.ascontiguousarray(f, dtype=np.float64)
            return lib().orc_energy_graded_f64(self.nx, self.ny, self.nz, self.sx, self.sy, self.sz, self.hc64,
                                               self.eps_r, self.mat, f)
        if f.dtype == np.float64:
            return lib().orc_energy_f64(self.nx, self.ny, self.nz, self.ch64, self.eps_r, self.mat, f)
        return lib().orc_energy_f32(self.nx, self.ny, self.nz, self.ch32, self.eps_r, self.mat, f)

    def divergence(self, f):
        """(div_e over the node box, div_h over cells) in float64."""
        f = np.ascontiguousarray(f, dtype=np.float64)
        de = np.zeros((self.nz + 1, self.ny + 1, self.nx + 1))
        dh = np.zeros((self.nz, self.ny, self.nx))
        if self.graded:
            lib().orc_divergence_graded_f64(self.nx, self.ny, self.nz, self.sx, self.sy, self.sz,
                                            self.eps_r, self.mat, f, de, dh)
        else:
            lib().orc_divergence_f64(self.nx, self.ny, self.nz, self.dx, self.dy, self.dz,
                                     self.eps_r, self.mat, f, de, dh)
        return de, dh


def quantize_bits(fmt, x):
    x = np.ascontiguousarray(x, dtype=np.float32).ravel()
    out = np.zeros(x.size, np.uint16)
    lib().orc_quantize_bits(fmt, x.size, x, out)
    return out


def choose_scales(m_prev, a_max):
    """Per-component scales from the previous stored maxima (6,) and A."""
    m = np.ascontiguousarray(m_prev, dtype=np.float32)
    out = np.zeros(6, np.int32)
    lib().orc_choose_scales(m, float(a_max), out)
    return out


def threads() -> int:
    """Threads the oracle's parallel loops use."""
    return int(lib().orc_threads())


def set_threads(n: int):
    """Threads for the parallel loops from now on (timing only)."""
    lib().orc_set_threads(int(n))
