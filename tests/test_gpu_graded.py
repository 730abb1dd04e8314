"""GPU parity of graded (per-index) cell sizes: the HIP library against the
oracle's graded FP32 operation-order mode, bit for bit, for the plain kernel
and the fused kernel at every T and tile shape, and against the graded FP64
oracle in relative L2.  Also the rules of fdtd_set_spacing."""
import ctypes as C

import numpy as np
import pytest

import oracle
from paper_1301_4539_amd import fdtd, workload as W
from tests import gpu_helpers as G

pytestmark = pytest.mark.gpu


def graded_ragged(n_steps=40, seed=4243):
    """Several tiles in x and y, several z chunks and a ragged tail, with
    random cell sizes in [0.4, 2] mm on every axis (so neighbouring primal and
    dual sizes all differ) and random source waveforms."""
    wl = W.spheres(131, 75, 50, 12, n_steps, seed=seed, n_sources=3, n_probes=16, rmin=3, rmax=12,
                   name="graded_ragged")
    rng = np.random.default_rng(seed)
    wl.spacing = tuple(rng.uniform(0.4e-3, 2e-3, n) for n in (wl.nx, wl.ny, wl.nz))
    wl.dt = W.courant_dt_graded(*wl.spacing)
    wl.waveforms = rng.standard_normal(wl.waveforms.shape)
    wl.init_fields = rng.standard_normal((6, wl.nz + 1, wl.ny + 1, wl.nx + 1))   # every cell active
    return wl


def _assert_same(a, b, what):
    msg = G.first_mismatch(a, b)
    assert msg is None, f"{what}: {msg}"


def test_graded_plain_bitexact_and_fp64():
    wl = graded_ragged()
    print("graded plain, 131x75x50, 40 steps", flush=True)
    f, p = G.gpu_run(wl, 40, kernel=fdtd.KERNEL_PLAIN)
    fo, po = G.oracle_f32(wl, 40)
    _assert_same(f, fo, "fields")
    _assert_same(p, po, "probes")
    f64, _ = G.oracle_f64(wl, 40)
    err = W.rel_l2(f, f64)
    print(f"graded rel-L2 vs FP64 after 40 steps: {err:.3e}")
    assert err <= 1e-5


@pytest.mark.parametrize("T", [1, 2, 3, 4])
def test_graded_fused_bitexact(T):
    wl = graded_ragged()
    print(f"graded fused T={T}, 131x75x50, 40 steps in chunks 7+13+20", flush=True)
    f, p = G.gpu_run(wl, 40, kernel=fdtd.KERNEL_FUSED, T=T, chunks=[7, 13, 20])
    fo, po = G.oracle_f32(wl, 40)
    _assert_same(f, fo, "fields")
    _assert_same(p, po, "probes")


@pytest.mark.parametrize("variant", [1, 2, 3])
def test_graded_fused_tile_shapes_bitexact(variant):
    wl = graded_ragged(n_steps=24)
    fo, po = G.oracle_f32(wl, 24)
    for T in (3, 4):
        print(f"graded fused T={T} variant={variant}, z chunk 9", flush=True)
        s = fdtd.Solver.from_workload(wl, kernel=fdtd.KERNEL_FUSED, time_block=T)
        try:
            s.set_tiling(variant, 9)
            s.step(24)
            f = s.read_fields()
            p = s.read_probes(0, 24)
        finally:
            s.close()
        _assert_same(f, fo, f"fields T={T}")
        _assert_same(p, po, f"probes T={T}")


def test_graded_automatic_kernel_bitexact():
    wl = graded_ragged(n_steps=30, seed=4244)
    print("graded automatic kernel and T, 30 steps", flush=True)
    f, p = G.gpu_run(wl, 30, kernel=fdtd.KERNEL_AUTO, T=0)
    fo, po = G.oracle_f32(wl, 30)
    _assert_same(f, fo, "fields")
    _assert_same(p, po, "probes")


def test_graded256_full_size_bitexact():
    """The graded 256^3 workload at full size, fused kernel with the automatic
    T and tile shape (the configuration the benchmark times), 100 steps."""
    wl = W.graded256(n_steps=100)
    init = np.random.default_rng(256).standard_normal((6, wl.nz + 1, wl.ny + 1, wl.nx + 1), dtype=np.float32)
    print("graded256 full size, random initial fields, automatic T, 100 steps", flush=True)
    f, p = G.gpu_run(wl, 100, kernel=fdtd.KERNEL_AUTO, T=0, init=init)
    fo, po = G.oracle_f32(wl, 100, init=init)
    _assert_same(f, fo, "fields")
    _assert_same(p, po, "probes")
    assert np.abs(p).max() > 0


def test_graded_uniform_sizes_close_to_uniform_solver():
    """Equal sizes along each axis: the graded solver computes the uniform
    update with coefficients formed as G * (c dt / d) instead of one rounded
    Cb, so it agrees with the uniform solver to FP32 rounding, not bit for bit."""
    wl = W.spheres(64, 48, 40, 6, 50, seed=77, n_sources=1, n_probes=4, rmin=3, rmax=8, name="u")
    fu, _ = G.gpu_run(wl, 50, kernel=fdtd.KERNEL_FUSED, T=4)
    wl.spacing = (np.full(wl.nx, wl.dx), np.full(wl.ny, wl.dy), np.full(wl.nz, wl.dz))
    fg, _ = G.gpu_run(wl, 50, kernel=fdtd.KERNEL_FUSED, T=4)
    assert W.rel_l2(fg, fu) < 1e-5


def _solver(storage=W.FP32, nx=20, ny=16, nz=12):
    wl = W.spheres(nx, ny, nz, 2, 10, seed=5, n_sources=1, n_probes=2, rmin=2, rmax=4, name="e")
    return wl, fdtd.Solver.from_workload(wl, storage=storage)


def test_set_spacing_rules():
    wl, s = _solver()
    sizes = [np.full(n, 1e-3) for n in (wl.nx, wl.ny, wl.nz)]
    try:
        small = [a.copy() for a in sizes]
        small[1][3] = 0.2e-3                       # dt of 1 mm cells exceeds this cell's bound
        with pytest.raises(fdtd.FdtdError) as e:
            s.set_spacing(*small)
        assert e.value.code == fdtd.ECFL
        bad = [a.copy() for a in sizes]
        bad[2][0] = -1e-3
        with pytest.raises(fdtd.FdtdError) as e:
            s.set_spacing(*bad)
        assert e.value.code == fdtd.EINVAL
        s.set_spacing(*sizes)
        with pytest.raises(fdtd.FdtdError) as e:
            fdtd.step_batch([s], [2])
        assert e.value.code == fdtd.EINVAL
        s.step(2)
        with pytest.raises(fdtd.FdtdError) as e:
            s.set_spacing(*sizes)
        assert e.value.code == fdtd.ESTATE
    finally:
        s.close()
    wl, s16 = _solver(storage=W.FP16)
    try:   # 16-bit storage takes graded sizes too (on the fused kernels)
        s16.set_spacing(*[np.full(n, 1e-3) for n in (wl.nx, wl.ny, wl.nz)])
        with pytest.raises(fdtd.FdtdError) as e:
            s16.set_kernel(fdtd.KERNEL_PLAIN, 1)
        assert e.value.code == fdtd.EINVAL
        s16.step(3)
        s16.synchronize()
    finally:
        s16.close()


def test_graded_diagnostics_match_oracle():
    import oracle
    wl = graded_ragged(n_steps=25, seed=4250)
    wl.init_fields = None
    init = np.random.default_rng(5).standard_normal((6, wl.nz + 1, wl.ny + 1, wl.nx + 1)).astype(np.float32)
    print("graded diagnostics, 25 steps", flush=True)
    s = fdtd.Solver.from_workload(wl, kernel=fdtd.KERNEL_FUSED, time_block=3)
    try:
        s.set_fields(init)
        s.step(25)
        d = s.diagnostics()
        f = s.read_fields()
    finally:
        s.close()
    prob = oracle.Problem.from_workload(wl)
    w = prob.energy(f)
    de, dh = prob.divergence(f.astype(np.float64))
    assert abs(d["energy"] - w) <= 1e-12 * abs(w)
    assert abs(d["div_e_max"] - np.max(np.abs(de))) <= 1e-12 * np.max(np.abs(de))
    assert abs(d["div_h_max"] - np.max(np.abs(dh))) <= 1e-12 * np.max(np.abs(dh))
    assert abs(d["div_e_sumsq"] - np.sum(de * de)) <= 1e-10 * np.sum(de * de)
    assert abs(d["div_h_sumsq"] - np.sum(dh * dh)) <= 1e-10 * np.sum(dh * dh)
    for c in range(6):
        assert d["max_abs"][c] == float(np.max(np.abs(f[c])))


def test_graded_lossless_energy_conserved_on_gpu():
    """The volume-weighted energy of a lossless graded PEC box stays constant
    over 200 GPU steps (FP32 round-off)."""
    wl = graded_ragged(n_steps=200, seed=4251)
    wl.sigma[:] = 0.0
    wl.sources, wl.waveforms = [], np.zeros((0, 200))
    init = wl.init_fields.astype(np.float32)
    wl.init_fields = None
    s = fdtd.Solver.from_workload(wl, kernel=fdtd.KERNEL_FUSED, time_block=3)
    try:
        s.set_fields(init)
        w0 = s.diagnostics()["energy"]
        s.step(200)
        w1 = s.diagnostics()["energy"]
    finally:
        s.close()
    assert abs(w1 - w0) < 1e-5 * w0


@pytest.mark.parametrize("fmt,T", [(W.FP16, 3), (W.FP16, 1), (W.BF16, 3), (W.BF16, 4)])
def test_graded_reduced_storage_bitexact_with_emulation(fmt, T):
    wl = graded_ragged(n_steps=30, seed=4252)
    wl.storage = fmt
    wl.init_fields = None
    print(f"graded reduced storage fmt={fmt} T={T}, 30 steps in 11+19", flush=True)
    f, p = G.gpu_run(wl, 30, kernel=fdtd.KERNEL_FUSED, T=T, storage=fmt, chunks=[11, 19])
    prob = oracle.Problem.from_workload(wl)
    fo = oracle.zero_fields(wl.nx, wl.ny, wl.nz, np.float32)
    st = prob.quantize_upload(fo, fmt)
    po = np.concatenate([prob.run_q(fo, 0, 11, fmt, T, st), prob.run_q(fo, 11, 19, fmt, T, st)])
    _assert_same(f, fo, "fields")
    _assert_same(p, po, "probes")


def test_graded_fp16_diagnostics_match_oracle():
    wl = graded_ragged(n_steps=20, seed=4253)
    wl.storage = W.FP16
    init = wl.init_fields.astype(np.float32)
    wl.init_fields = None
    s = fdtd.Solver.from_workload(wl, kernel=fdtd.KERNEL_FUSED, time_block=3)
    try:
        s.set_fields(init)
        s.step(20)
        d = s.diagnostics()
        f = s.read_fields()
    finally:
        s.close()
    prob = oracle.Problem.from_workload(wl)
    w = prob.energy(f)
    assert abs(d["energy"] - w) <= 1e-12 * abs(w)
    for c in range(6):
        assert d["max_abs"][c] == float(np.max(np.abs(f[c])))
