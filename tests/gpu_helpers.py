"""Shared helpers of the GPU parity tests: run a workload through the HIP
library (via the C ABI binding) and through the CPU oracle."""
import numpy as np

import oracle
from paper_1301_4539_amd import fdtd, workload as W


def init32(wl):
    if wl.init_fields is None:
        return oracle.zero_fields(wl.nx, wl.ny, wl.nz, np.float32)
    return np.ascontiguousarray(wl.init_fields.astype(np.float32))


def pec_clean(wl, f):
    """The library forces tangential E on the walls (and unused box slots) to zero."""
    g = f.copy()
    nx, ny, nz = wl.nx, wl.ny, wl.nz
    m = W.interior_e_mask(nx, ny, nz)
    g[0:3][~m] = 0.0
    g[3, nz, :, :] = 0; g[3, :, ny, :] = 0
    g[4, nz, :, :] = 0; g[4, :, :, nx] = 0
    g[5, :, ny, :] = 0; g[5, :, :, nx] = 0
    return g


def gpu_run(wl, steps, kernel=fdtd.KERNEL_FUSED, T=1, storage=W.FP32, chunks=None, init=None):
    """Returns (fields (6,...) float32, probes (steps, n_probe) float64, solver diag dict)."""
    s = fdtd.Solver.from_workload(wl, storage=storage, kernel=kernel, time_block=T)
    try:
        if init is not None:
            s.set_fields(init)
        for n in (chunks or [steps]):
            s.step(n)
        s.synchronize()
        f = s.read_fields()
        p = s.read_probes(0, steps) if wl.probes else np.zeros((steps, 0))
        return f, p
    finally:
        s.close()


def oracle_f32(wl, steps, init=None):
    prob = oracle.Problem.from_workload(wl)
    f = pec_clean(wl, init32(wl) if init is None else init.astype(np.float32))
    p = prob.run_f32(f, 0, steps)
    return f, p


def oracle_f64(wl, steps):
    prob = oracle.Problem.from_workload(wl)
    f = wl.init_fields.copy() if wl.init_fields is not None else oracle.zero_fields(wl.nx, wl.ny, wl.nz)
    f = pec_clean(wl, f)
    p = prob.run_f64(f, 0, steps)
    return f, p


def oracle_q(wl, steps, fmt, T, init=None):
    prob = oracle.Problem.from_workload(wl)
    f = pec_clean(wl, init32(wl) if init is None else init.astype(np.float32))
    st = prob.quantize_upload(f, fmt)
    p = prob.run_q(f, 0, steps, fmt, T, st)
    return f, p, st


def first_mismatch(a, b):
    bad = np.argwhere(a != b)
    if len(bad) == 0:
        return None
    idx = tuple(bad[0])
    return f"{len(bad)} mismatches; first at {idx}: gpu={a[idx]!r} oracle={b[idx]!r}"
