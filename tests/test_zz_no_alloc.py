"""The diagnostics entry point that allocates no device memory
(fdtd_diagnostics_noalloc, a static per-GPU scratch array) against the
allocating one (fdtd_diagnostics): the same kernels in the same order, so
every value agrees bit for bit -- on two calls in a row, the second on a
smaller grid (the array keeps the first call's partials beyond the second's
count, which must not leak into it), then on the first grid again; a grid
whose partials exceed the array is rejected before any device work."""
import numpy as np
import pytest

from paper_1301_4539_amd import fdtd, workload as W

pytestmark = pytest.mark.gpu


def _solver(nx, ny, nz, storage, seed):
    wl = W.spheres(nx, ny, nz, 6, 12, seed=seed, n_sources=2, n_probes=4, rmin=2, rmax=8, name="noalloc",
                   storage=storage)
    s = fdtd.Solver.from_workload(wl, kernel=fdtd.KERNEL_FUSED, time_block=3)
    rng = np.random.default_rng(seed)
    s.set_fields(rng.standard_normal((6, nz + 1, ny + 1, nx + 1)).astype(np.float32))
    s.step(12)
    return s


def _same(a, b, what):
    for k in ("energy", "div_e_max", "div_e_sumsq", "div_h_max", "div_h_sumsq"):
        assert a[k] == b[k], f"{what}: {k} {a[k]!r} != {b[k]!r}"
    assert a["max_abs"] == b["max_abs"], f"{what}: max_abs"


def test_noalloc_diagnostics_equal_the_allocating_ones():
    print("noalloc diagnostics: 150x100x80 fp32, then 40x30x20 fp16, then again", flush=True)
    big = _solver(150, 100, 80, W.FP32, 31)
    small = _solver(40, 30, 20, W.FP16, 32)
    try:
        first = big.diagnostics_noalloc()
        _same(first, big.diagnostics(), "150x100x80 fp32")
        assert first["energy"] > 0
        second = small.diagnostics_noalloc()          # smaller input: fewer partials
        _same(second, small.diagnostics(), "40x30x20 fp16")
        big.step(3)
        _same(big.diagnostics_noalloc(), big.diagnostics(), "150x100x80 fp32 after 3 more steps")
    finally:
        big.close()
        small.close()


def test_noalloc_diagnostics_reject_grids_beyond_the_scratch():
    print("noalloc diagnostics: 1300x1300x8 rejected", flush=True)
    wl = W.spheres(1300, 1300, 8, 0, 1, seed=33, n_sources=0, n_probes=0, rmin=1, rmax=2, name="wide")
    s = fdtd.Solver.from_workload(wl)
    try:
        with pytest.raises(fdtd.FdtdError) as e:
            s.diagnostics_noalloc()
        assert e.value.code == fdtd.EINVAL
        assert s.diagnostics()["energy"] == 0.0        # the allocating entry point still serves it
    finally:
        s.close()
