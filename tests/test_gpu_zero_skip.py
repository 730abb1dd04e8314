"""Zero-tile skipping of the fused kernel: with skipping on, results are bit
for bit those with skipping off and those of the oracle -- from zero fields
with sources (tiles far from the sources skipped while the field spreads,
their probes recorded as 0), after fdtd_set_fields of a localized state,
with 16-bit storage, graded sizes, split steps and batched steps."""
import numpy as np
import pytest

import oracle
from paper_1301_4539_amd import fdtd, workload as W
from tests import gpu_helpers as G

pytestmark = pytest.mark.gpu


def spreading(n_steps=60, storage=W.FP32, seed=4270):
    """A 200x120x150 grid (many tiles of every shape) with one Ez source near
    a corner region and probes spread over the grid, so that most tiles stay
    zero for the first tens of steps."""
    wl = W.spheres(200, 120, 150, 10, n_steps, seed=seed, n_sources=1, n_probes=16, rmin=3, rmax=10,
                   name="spreading", storage=storage)
    wl.sources = [(W.EZ, 40, 30, 35)]
    wl.waveforms = np.random.default_rng(seed).standard_normal((1, n_steps))
    return wl


def _run(wl, steps, skip, T, storage=W.FP32, chunks=None, init=None, kernel=fdtd.KERNEL_FUSED):
    s = fdtd.Solver.from_workload(wl, storage=storage, kernel=kernel, time_block=T)
    try:
        s.set_zero_skip(skip)
        if init is not None:
            s.set_fields(init)
        for n in (chunks or [steps]):
            s.step(n)
        s.synchronize()
        return s.read_fields(), s.read_probes(0, steps)
    finally:
        s.close()


def _assert_same(a, b, what):
    msg = G.first_mismatch(a, b)
    assert msg is None, f"{what}: {msg}"


@pytest.mark.parametrize("T", [1, 2, 3, 4])
def test_skip_from_zero_bitexact(T):
    wl = spreading()
    print(f"zero skip T={T}, 60 steps from zero", flush=True)
    f1, p1 = _run(wl, 60, True, T, chunks=[7, 13, 40])
    f0, p0 = _run(wl, 60, False, T)
    _assert_same(f1, f0, "fields skip on/off")
    _assert_same(p1, p0, "probes skip on/off")
    fo, po = G.oracle_f32(wl, 60)
    _assert_same(f1, fo, "fields vs oracle")
    _assert_same(p1, po, "probes vs oracle")
    assert np.count_nonzero(f1) > 0 and np.count_nonzero(f1 == 0) > f1.size // 4   # still spreading


@pytest.mark.parametrize("fmt", [W.FP16, W.BF16])
def test_skip_reduced_storage_bitexact(fmt):
    wl = spreading(n_steps=45, storage=fmt, seed=4271)
    print(f"zero skip fmt={fmt} T=3, 45 steps", flush=True)
    f1, p1 = _run(wl, 45, True, 3, storage=fmt)
    f0, p0 = _run(wl, 45, False, 3, storage=fmt)
    _assert_same(f1, f0, "fields skip on/off")
    _assert_same(p1, p0, "probes skip on/off")
    fo, po, _ = G.oracle_q(wl, 45, fmt, 3)
    _assert_same(f1, fo, "fields vs emulation")


def test_skip_graded_bitexact():
    wl = spreading(n_steps=40, seed=4272)
    rng = np.random.default_rng(4272)
    wl.spacing = tuple(rng.uniform(0.5e-3, 1.5e-3, n) for n in (wl.nx, wl.ny, wl.nz))
    wl.dt = W.courant_dt_graded(*wl.spacing)
    print("zero skip graded T=3, 40 steps", flush=True)
    f1, p1 = _run(wl, 40, True, 3)
    f0, p0 = _run(wl, 40, False, 3)
    _assert_same(f1, f0, "fields skip on/off")
    _assert_same(p1, p0, "probes skip on/off")


def test_skip_after_localized_upload():
    """A state that is nonzero only in a small block (the box comes from the
    uploaded values) and no sources."""
    wl = spreading(n_steps=40, seed=4273)
    wl.sources, wl.waveforms = [], np.zeros((0, 40))
    init = np.zeros((6, wl.nz + 1, wl.ny + 1, wl.nx + 1), np.float32)
    rng = np.random.default_rng(4273)
    init[:, 100:112, 60:70, 150:170] = rng.standard_normal((6, 12, 10, 20))
    print("zero skip after a localized upload, 40 steps", flush=True)
    f1, p1 = _run(wl, 40, True, 4, init=init)
    f0, p0 = _run(wl, 40, False, 4, init=init)
    _assert_same(f1, f0, "fields skip on/off")
    _assert_same(p1, p0, "probes skip on/off")
    prob = oracle.Problem.from_workload(wl)
    fo = G.pec_clean(wl, init)
    po = prob.run_f32(fo, 0, 40)
    _assert_same(f1, fo, "fields vs oracle")
    _assert_same(p1, po, "probes vs oracle")


def test_skip_after_batched_and_plain_steps():
    """The box follows steps taken by fdtd_step_batch and by the plain kernel."""
    wl = spreading(n_steps=48, seed=4274)
    print("zero skip after batched and plain steps, 48 steps", flush=True)
    s = fdtd.Solver.from_workload(wl, kernel=fdtd.KERNEL_FUSED, time_block=4)
    try:
        fdtd.step_batch([s], [12])
        s.set_kernel(fdtd.KERNEL_PLAIN, 1)
        s.step(6)
        s.set_kernel(fdtd.KERNEL_FUSED, 4)
        s.step(30)
        f1, p1 = s.read_fields(), s.read_probes(0, 48)
    finally:
        s.close()
    f0, p0 = _run(wl, 48, False, 4)
    _assert_same(f1, f0, "fields")
    _assert_same(p1, p0, "probes")


def test_skip_with_conductor_from_zero():
    """Perfect-conductor cells (a slab and a sphere) with the field spreading
    from zero: skipping on equals off equals the oracle."""
    wl = spreading(n_steps=48, seed=4275)
    wl.eps_r = np.append(wl.eps_r, 1.0)
    wl.mu_r = np.append(wl.mu_r, 1.0)
    wl.sigma = np.append(wl.sigma, np.inf)
    k, j, i = np.meshgrid(*(np.arange(v) for v in (wl.nz, wl.ny, wl.nx)), indexing="ij")
    wl.mat[(i >= 150) | ((i + 0.5 - 60) ** 2 + (j + 0.5 - 40) ** 2 + (k + 0.5 - 50) ** 2 <= 100)] = 16
    print("zero skip with conductor cells, 48 steps", flush=True)
    f1, p1 = _run(wl, 48, True, 4)
    f0, p0 = _run(wl, 48, False, 4)
    _assert_same(f1, f0, "fields skip on/off")
    _assert_same(p1, p0, "probes skip on/off")
    fo, po = G.oracle_f32(wl, 48)
    _assert_same(f1, fo, "fields vs oracle")
    _assert_same(p1, po, "probes vs oracle")
