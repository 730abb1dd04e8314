"""Python binding of the Yee FDTD C ABI (include/fdtd.h) -- marshalling only.

Every step of the solver runs in the HIP library libfdtd.so; this module
only converts arguments.  PyTorch provides device memory (the workspace is
a torch uint8 tensor) and the stream (torch's current stream).  There is no
fallback: if libfdtd.so is missing, loading it raises.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

from .workload import FP32, FP16, BF16  # noqa: F401  (re-exported storage codes)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfdtd.so")

OK, EINVAL, ENOMEM, EDEVICE, ECFL, ERANGE, ESTATE = 0, -1, -2, -3, -4, -5, -6
KERNEL_AUTO, KERNEL_PLAIN, KERNEL_FUSED = 0, 1, 2

_lib = None


class FdtdError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"fdtd error {code}: {msg}")
        self.code = code


class _Material(C.Structure):
    _fields_ = [("eps_r", C.c_double), ("mu_r", C.c_double), ("sigma", C.c_double)]


class _Diag(C.Structure):
    _fields_ = [("energy", C.c_double), ("div_e_max", C.c_double), ("div_e_sumsq", C.c_double),
                ("div_h_max", C.c_double), ("div_h_sumsq", C.c_double), ("max_abs", C.c_double * 6)]


def lib():
    """Load libfdtd.so (after torch, so the process uses one HIP runtime)."""
    global _lib
    if _lib is None:
        import torch  # noqa: F401  -- loads the HIP runtime the library binds to
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        vp, i, d, sz, ll = C.c_void_p, C.c_int, C.c_double, C.c_size_t, C.c_longlong
        L.fdtd_workspace_bytes.argtypes = [i, i, i, i]
        L.fdtd_workspace_bytes.restype = sz
        L.fdtd_create.argtypes = [C.POINTER(vp), i, i, i, d, d, d, d, C.POINTER(_Material), i, vp, i, vp, sz, vp]
        L.fdtd_set_kernel.argtypes = [vp, i, i]
        L.fdtd_set_tiling.argtypes = [vp, i, i]
        L.fdtd_set_zero_skip.argtypes = [vp, i]
        L.fdtd_set_poison.argtypes = [vp, i]
        L.fdtd_set_fields.argtypes = [vp, vp]
        L.fdtd_set_source.argtypes = [vp, i, i, i, i, vp, i, C.POINTER(i)]
        L.fdtd_set_probe.argtypes = [vp, i, i, i, i, C.POINTER(i)]
        L.fdtd_step.argtypes = [vp, i]
        L.fdtd_step_batch.argtypes = [C.POINTER(vp), i, C.POINTER(i)]
        L.fdtd_read_fields.argtypes = [vp, i, vp]
        L.fdtd_read_probes.argtypes = [vp, vp, ll, i]
        L.fdtd_set_energy_trace.argtypes = [vp, i]
        L.fdtd_reserve_steps.argtypes = [vp, ll]
        L.fdtd_read_energy.argtypes = [vp, vp, ll, i]
        L.fdtd_diagnostics.argtypes = [vp, C.POINTER(_Diag)]
        L.fdtd_diagnostics_noalloc.argtypes = [vp, C.POINTER(_Diag)]
        L.fdtd_set_stream.argtypes = [vp, vp]
        L.fdtd_steps_done.argtypes = [vp, C.POINTER(ll)]
        L.fdtd_time_block.argtypes = [vp, C.POINTER(i)]
        L.fdtd_tune_time_block.argtypes = [vp, i, C.POINTER(i), vp]
        L.fdtd_state_bytes.argtypes = [vp]
        L.fdtd_state_bytes.restype = sz
        L.fdtd_save_state.argtypes = [vp, vp, sz]
        L.fdtd_load_state.argtypes = [vp, vp, sz]
        L.fdtd_storage_state.argtypes = [vp, C.POINTER(i), C.POINTER(i)]
        L.fdtd_synchronize.argtypes = [vp]
        L.fdtd_destroy.argtypes = [vp]
        L.fdtd_destroy.restype = None
        L.fdtd_last_error.restype = C.c_char_p
        L.fdtd_coefficients.argtypes = [C.POINTER(_Material), i, d, d, d, d, vp, vp]
        L.fdtd_set_spacing.argtypes = [vp, vp, vp, vp]
        L.fdtd_graded_coefficients.argtypes = [C.POINTER(_Material), i, i, i, i, vp, vp, vp, d, vp, vp]
        L.fdtd_set_cpml.argtypes = [vp, i, i, d, d, d]
        L.fdtd_cpml_coefficients.argtypes = [C.POINTER(_Material), i, i, i, i, vp, vp, vp, d, i, i, d, d, d,
                                             vp, vp, vp]
        L.fdtd_live_nodes.argtypes = [C.POINTER(_Material), i, vp, i, i, i, vp, i, vp]
        L.fdtd_tile_stats.argtypes = [vp, C.POINTER(C.c_longlong), C.POINTER(C.c_longlong)]
        for name in ("fdtd_create", "fdtd_set_kernel", "fdtd_set_tiling", "fdtd_set_zero_skip", "fdtd_set_poison", "fdtd_set_fields", "fdtd_set_source", "fdtd_set_probe",
                     "fdtd_step", "fdtd_step_batch", "fdtd_read_fields", "fdtd_read_probes", "fdtd_diagnostics", "fdtd_diagnostics_noalloc",
                     "fdtd_steps_done", "fdtd_set_stream", "fdtd_set_energy_trace", "fdtd_read_energy", "fdtd_reserve_steps",
                     "fdtd_storage_state", "fdtd_synchronize", "fdtd_coefficients", "fdtd_set_spacing",
                     "fdtd_graded_coefficients", "fdtd_set_cpml", "fdtd_cpml_coefficients", "fdtd_save_state",
                     "fdtd_load_state", "fdtd_live_nodes", "fdtd_tile_stats", "fdtd_time_block",
                     "fdtd_tune_time_block"):
            getattr(L, name).restype = i
        _lib = L
    return _lib


def _diag_dict(d):
    return {"energy": d.energy, "div_e_max": d.div_e_max, "div_e_sumsq": d.div_e_sumsq,
            "div_h_max": d.div_h_max, "div_h_sumsq": d.div_h_sumsq, "max_abs": list(d.max_abs)}


def _check(rc):
    if rc != OK:
        raise FdtdError(rc, lib().fdtd_last_error().decode())


def _materials(eps_r, sigma, mu_r=None):
    eps_r = np.asarray(eps_r, dtype=np.float64).ravel()
    sigma = np.asarray(sigma, dtype=np.float64).ravel()
    mu_r = np.ones_like(eps_r) if mu_r is None else np.asarray(mu_r, dtype=np.float64).ravel()
    arr = (_Material * len(eps_r))()
    for m in range(len(eps_r)):
        arr[m].eps_r, arr[m].mu_r, arr[m].sigma = float(eps_r[m]), float(mu_r[m]), float(sigma[m])
    return arr, len(eps_r)


def coefficients(eps_r, sigma, dx, dy, dz, dt, mu_r=None):
    """The library's FP32 coefficient table (n_mat, 4) and ch (3,)."""
    arr, n = _materials(eps_r, sigma, mu_r)
    out = np.zeros((n, 4), np.float32)
    ch = np.zeros(3, np.float32)
    _check(lib().fdtd_coefficients(arr, n, dx, dy, dz, dt, out.ctypes.data, ch.ctypes.data))
    return out, ch


def _sizes(dx, dy, dz):
    return tuple(np.ascontiguousarray(a, dtype=np.float64).ravel() for a in (dx, dy, dz))


def graded_coefficients(eps_r, sigma, dx, dy, dz, dt, mu_r=None):
    """The library's FP32 graded-spacing tables: cag (n_mat, 2) = (Ca, G) and
    gc ((nx+1)+(ny+1)+(nz+1), 2) = (c dt / primal size, c dt / dual size)."""
    arr, n = _materials(eps_r, sigma, mu_r)
    dx, dy, dz = _sizes(dx, dy, dz)
    cag = np.zeros((n, 2), np.float32)
    gc = np.zeros((len(dx) + len(dy) + len(dz) + 3, 2), np.float32)
    _check(lib().fdtd_graded_coefficients(arr, n, len(dx), len(dy), len(dz), dx.ctypes.data, dy.ctypes.data,
                                          dz.ctypes.data, dt, cag.ctypes.data, gc.ctypes.data))
    return cag, gc


def cpml_coefficients(eps_r, sigma, dx, dy, dz, dt, thickness, order=3, sigma_factor=1.0, kappa_max=1.0,
                      alpha_max=0.0, mu_r=None):
    """The library's FP32 CPML tables: cag (n_mat, 2), gc (n_idx, 2) with kappa
    folded in, cp (n_idx, 6) = b_h, a_h, c dt / d, b_e, a_e, c dt / d'."""
    arr, n = _materials(eps_r, sigma, mu_r)
    dx, dy, dz = _sizes(dx, dy, dz)
    nidx = len(dx) + len(dy) + len(dz) + 3
    cag = np.zeros((n, 2), np.float32)
    gc = np.zeros((nidx, 2), np.float32)
    cp = np.zeros((nidx, 6), np.float32)
    _check(lib().fdtd_cpml_coefficients(arr, n, len(dx), len(dy), len(dz), dx.ctypes.data, dy.ctypes.data,
                                        dz.ctypes.data, dt, thickness, order, sigma_factor, kappa_max, alpha_max,
                                        cag.ctypes.data, gc.ctypes.data, cp.ctypes.data))
    return cag, gc, cp


def live_nodes(eps_r, sigma, mat, sources=(), mu_r=None):
    """The library's live-node map for all-zero stored values: (nz+1, ny+1,
    nx+1) uint8, 1 = live, for cell materials mat (nz, ny, nx) and sources
    given as (comp, i, j, k)."""
    arr, n = _materials(eps_r, sigma, mu_r)
    mat = np.ascontiguousarray(mat, dtype=np.uint8)
    nz, ny, nx = mat.shape
    src = np.ascontiguousarray(np.asarray(list(sources), dtype=np.int32).reshape(-1, 4))
    out = np.zeros((nz + 1, ny + 1, nx + 1), np.uint8)
    _check(lib().fdtd_live_nodes(arr, n, mat.ctypes.data, nx, ny, nz, src.ctypes.data, len(src), out.ctypes.data))
    return out


def step_batch(solvers, n_steps):
    """Advance solvers[i] by n_steps[i] steps in shared persistent launches."""
    n = len(solvers)
    hs = (C.c_void_p * max(n, 1))(*[s._h for s in solvers])
    ns = (C.c_int * max(n, 1))(*[int(k) for k in n_steps])
    _check(lib().fdtd_step_batch(hs, n, ns))


def workspace_bytes(nx, ny, nz, storage=FP32):
    return int(lib().fdtd_workspace_bytes(nx, ny, nz, storage))


class Solver:
    """One FDTD solve on the GPU.  Arrays use the (nz+1, ny+1, nx+1) node box."""

    def __init__(self, nx, ny, nz, dx, dy, dz, dt, eps_r, sigma, mat=None, storage=FP32,
                 kernel=KERNEL_AUTO, time_block=0, mu_r=None, torch_workspace=True, stream=None):
        import torch
        self.nx, self.ny, self.nz = nx, ny, nz
        self.storage = storage
        arr, n_mat = _materials(eps_r, sigma, mu_r)
        mat_ptr = None
        if mat is not None:
            self._mat = np.ascontiguousarray(mat, dtype=np.uint8).reshape(nz, ny, nx)
            mat_ptr = self._mat.ctypes.data
        self._ws = None
        ws_ptr, ws_bytes = None, 0
        if torch_workspace:
            ws_bytes = workspace_bytes(nx, ny, nz, storage)
            if ws_bytes == 0:
                raise FdtdError(EINVAL, "invalid dimensions or storage")
            self._ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
            ws_ptr = self._ws.data_ptr()
        if stream is None:
            stream = torch.cuda.current_stream()
        self._stream = stream
        h = C.c_void_p()
        _check(lib().fdtd_create(C.byref(h), nx, ny, nz, dx, dy, dz, dt, arr, n_mat, mat_ptr, storage,
                                 ws_ptr, ws_bytes, C.c_void_p(stream.cuda_stream)))
        self._h = h
        self.n_probes = 0
        self.set_kernel(kernel, time_block)

    @classmethod
    def from_workload(cls, wl, storage=None, kernel=KERNEL_AUTO, time_block=0, **kw):
        s = cls(wl.nx, wl.ny, wl.nz, wl.dx, wl.dy, wl.dz, wl.dt, wl.eps_r, wl.sigma, wl.mat,
                storage=wl.storage if storage is None else storage, kernel=kernel, time_block=time_block, **kw)
        for q, (c, i, j, k) in enumerate(wl.sources):
            s.add_source(c, i, j, k, wl.waveforms[q].astype(np.float32))
        for (c, i, j, k) in wl.probes:
            s.add_probe(c, i, j, k)
        if getattr(wl, "spacing", None) is not None:
            s.set_spacing(*wl.spacing)
        if getattr(wl, "cpml", None):
            s.set_cpml(**wl.cpml)
        if wl.init_fields is not None:
            s.set_fields(wl.init_fields.astype(np.float32))
        return s

    def set_kernel(self, kernel, time_block):
        _check(lib().fdtd_set_kernel(self._h, kernel, time_block))

    def set_spacing(self, dx, dy, dz):
        """Graded spacing: per-index cell sizes dx (nx,), dy (ny,), dz (nz,)."""
        dx, dy, dz = _sizes(dx, dy, dz)
        assert (len(dx), len(dy), len(dz)) == (self.nx, self.ny, self.nz)
        _check(lib().fdtd_set_spacing(self._h, dx.ctypes.data, dy.ctypes.data, dz.ctypes.data))

    def set_cpml(self, thickness, order=3, sigma_factor=1.0, kappa_max=1.0, alpha_max=0.0):
        """CPML absorbing layers of `thickness` cells on every face (0 removes them)."""
        _check(lib().fdtd_set_cpml(self._h, int(thickness), int(order), float(sigma_factor), float(kappa_max),
                                   float(alpha_max)))

    def set_zero_skip(self, enable: bool):
        """Skip fused-kernel tiles that can only compute +0 (default on)."""
        _check(lib().fdtd_set_zero_skip(self._h, 1 if enable else 0))

    def set_poison(self, enable: bool):
        """Debugging aid: NaN-fill each fused launch's output buffer first."""
        _check(lib().fdtd_set_poison(self._h, 1 if enable else 0))

    def set_tiling(self, variant=0, z_chunk=0):
        _check(lib().fdtd_set_tiling(self._h, variant, z_chunk))

    def set_fields(self, f: Optional[np.ndarray]):
        if f is None:
            _check(lib().fdtd_set_fields(self._h, None))
            return
        f = np.ascontiguousarray(f, dtype=np.float32)
        assert f.shape == (6, self.nz + 1, self.ny + 1, self.nx + 1)
        _check(lib().fdtd_set_fields(self._h, f.ctypes.data))

    def add_source(self, comp, i, j, k, waveform) -> int:
        w = np.ascontiguousarray(waveform, dtype=np.float32)
        sid = C.c_int()
        _check(lib().fdtd_set_source(self._h, comp, i, j, k, w.ctypes.data, len(w), C.byref(sid)))
        return sid.value

    def add_probe(self, comp, i, j, k) -> int:
        pid = C.c_int()
        _check(lib().fdtd_set_probe(self._h, comp, i, j, k, C.byref(pid)))
        self.n_probes = pid.value + 1
        return pid.value

    def step(self, n: int):
        _check(lib().fdtd_step(self._h, int(n)))

    def set_stream(self, stream):
        """Move the solver to a torch stream (after its pending work)."""
        _check(lib().fdtd_set_stream(self._h, C.c_void_p(stream.cuda_stream)))
        self._stream = stream

    def read_field(self, comp) -> np.ndarray:
        out = np.empty((self.nz + 1, self.ny + 1, self.nx + 1), np.float32)
        _check(lib().fdtd_read_fields(self._h, comp, out.ctypes.data))
        return out

    def read_fields(self) -> np.ndarray:
        return np.stack([self.read_field(c) for c in range(6)])

    def read_probes(self, first: int, n: int) -> np.ndarray:
        out = np.zeros((n, max(self.n_probes, 1)), np.float64)
        _check(lib().fdtd_read_probes(self._h, out.ctypes.data, first, n))
        return out[:, :self.n_probes]

    def reserve_steps(self, total_steps: int):
        """Allocate the probe rows (and energy records) of the first
        total_steps steps now, so that stepping up to there allocates nothing
        and never synchronises the stream."""
        _check(lib().fdtd_reserve_steps(self._h, int(total_steps)))

    def set_energy_trace(self, every: int):
        """Record the energy W^n of every state n = k * every a step starts from
        (0: off); before the first step."""
        _check(lib().fdtd_set_energy_trace(self._h, int(every)))

    def read_energy(self, first: int, n: int) -> np.ndarray:
        """Energy records first .. first+n-1 (record k: state k * every)."""
        out = np.empty(n, np.float64)
        _check(lib().fdtd_read_energy(self._h, out.ctypes.data, first, n))
        return out

    def diagnostics(self) -> dict:
        d = _Diag()
        _check(lib().fdtd_diagnostics(self._h, C.byref(d)))
        return _diag_dict(d)

    def diagnostics_noalloc(self) -> dict:
        """The same diagnostics through the entry point that allocates no
        device memory (a static per-GPU scratch array)."""
        d = _Diag()
        _check(lib().fdtd_diagnostics_noalloc(self._h, C.byref(d)))
        return _diag_dict(d)

    def tile_stats(self):
        """(workgroups dispatched, tiles of the full tiling) of the fused
        launches since creation."""
        a, b = C.c_longlong(), C.c_longlong()
        _check(lib().fdtd_tile_stats(self._h, C.byref(a), C.byref(b)))
        return a.value, b.value

    def save_state(self) -> np.ndarray:
        """The whole evolving state as an opaque byte array (checkpoint)."""
        buf = np.empty(int(lib().fdtd_state_bytes(self._h)), np.uint8)
        _check(lib().fdtd_save_state(self._h, buf.ctypes.data, buf.size))
        return buf

    def load_state(self, buf: np.ndarray):
        """Restore a state saved from a solver of the same configuration."""
        buf = np.ascontiguousarray(buf, dtype=np.uint8)
        _check(lib().fdtd_load_state(self._h, buf.ctypes.data, buf.size))

    def steps_done(self) -> int:
        n = C.c_longlong()
        _check(lib().fdtd_steps_done(self._h, C.byref(n)))
        return n.value

    @property
    def time_block(self) -> int:
        """Steps per launch of the next step call (1: the plain kernels)."""
        t = C.c_int()
        _check(lib().fdtd_time_block(self._h, C.byref(t)))
        return t.value

    def tune_time_block(self, n_steps: int):
        """Measure T = 3, 4, 5 over about n_steps steps each (the solver
        advances by them) and keep the fastest: (T, {T: ns per step})."""
        t = C.c_int()
        ns = (C.c_double * 3)()
        _check(lib().fdtd_tune_time_block(self._h, n_steps, C.byref(t), ns))
        return t.value, {T: ns[q] for q, T in enumerate((3, 4, 5))}

    def storage_state(self):
        sc = (C.c_int * 6)()
        sat = C.c_int()
        _check(lib().fdtd_storage_state(self._h, sc, C.byref(sat)))
        return list(sc), bool(sat.value)

    def synchronize(self):
        _check(lib().fdtd_synchronize(self._h))

    def close(self):
        if getattr(self, "_h", None):
            lib().fdtd_destroy(self._h)
            self._h = None
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
