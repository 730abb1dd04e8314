"""GPU parity: the HIP library against the CPU oracle, element by element.

FP32 storage: bit-exact with the oracle's FP32 operation-order mode, for the
plain kernel and the fused kernel at every time-block length T (tiling,
fusion and temporal blocking change the order in which values are computed,
never the operations that compute them -- the paper's Sec. 3.1 point).
Against the FP64 oracle: relative L2 <= 1e-5 after 100 steps of the 32^3
cavity.  Reduced storage: bit-exact with the oracle's emulation at the same T.
"""
import numpy as np
import pytest

from paper_1301_4539_amd import fdtd, workload as W
from tests import gpu_helpers as G

pytestmark = pytest.mark.gpu

TS = [1, 2, 3, 4]


def ragged(n_steps=40, storage=W.FP32):
    """Spans several tiles in x and y and several z chunks, with a ragged tail;
    seeded random source waveforms so the sources matter from the first step."""
    wl = W.spheres(131, 75, 50, 12, n_steps, seed=4242, n_sources=3, n_probes=16, rmin=3, rmax=12,
                   name="ragged", storage=storage)
    wl.waveforms = np.random.default_rng(17).standard_normal(wl.waveforms.shape)
    return wl


def _assert_same(a, b, what):
    msg = G.first_mismatch(a, b)
    assert msg is None, f"{what}: {msg}"


def test_cavity32_plain_bitexact_and_fp64():
    wl = W.cavity32()
    f, p = G.gpu_run(wl, 100, kernel=fdtd.KERNEL_PLAIN)
    fo, po = G.oracle_f32(wl, 100)
    _assert_same(f, fo, "fields")
    _assert_same(p, po, "probes")
    f64, _ = G.oracle_f64(wl, 100)
    err = W.rel_l2(f, f64)
    print(f"cavity32 rel-L2 vs FP64 after 100 steps: {err:.3e}")
    assert err <= 1e-5


@pytest.mark.parametrize("T", TS)
def test_cavity32_fused_bitexact(T):
    wl = W.cavity32()
    f, p = G.gpu_run(wl, 100, kernel=fdtd.KERNEL_FUSED, T=T)
    fo, po = G.oracle_f32(wl, 100)
    _assert_same(f, fo, "fields")
    _assert_same(p, po, "probes")


@pytest.mark.parametrize("T", TS)
def test_ragged_spheres_fused_bitexact(T):
    wl = ragged()
    f, p = G.gpu_run(wl, 40, kernel=fdtd.KERNEL_FUSED, T=T)
    fo, po = G.oracle_f32(wl, 40)
    _assert_same(f, fo, "fields")
    _assert_same(p, po, "probes")
    assert np.max(np.abs(fo[0:3])) > 0.1          # the sources really drove the fields


def test_ragged_spheres_plain_bitexact():
    wl = ragged()
    f, p = G.gpu_run(wl, 40, kernel=fdtd.KERNEL_PLAIN)
    fo, po = G.oracle_f32(wl, 40)
    _assert_same(f, fo, "fields")
    _assert_same(p, po, "probes")


@pytest.mark.parametrize("shape", [(2, 2, 2), (3, 2, 5), (70, 3, 2), (2, 40, 3), (5, 4, 130)])
@pytest.mark.parametrize("T", [1, 3])
def test_tiny_and_thin_grids_random_state(shape, T):
    nx, ny, nz = shape
    rng = np.random.default_rng(sum(shape) + T)
    wl = W.spheres(nx, ny, nz, 0, 12, seed=7, n_sources=0, n_probes=0, name="tiny")
    wl.mat = rng.integers(0, 16, size=(nz, ny, nx)).astype(np.uint8)
    init = rng.standard_normal((6, nz + 1, ny + 1, nx + 1)).astype(np.float32)
    f, _ = G.gpu_run(wl, 12, kernel=fdtd.KERNEL_FUSED, T=T, init=init)
    fo, _ = G.oracle_f32(wl, 12, init=init)
    _assert_same(f, fo, "fields")


@pytest.mark.parametrize("fmt", [W.FP16, W.BF16])
@pytest.mark.parametrize("T", TS)
def test_reduced_storage_bitexact_with_emulation(fmt, T):
    wl = ragged(n_steps=36, storage=fmt)
    f, p = G.gpu_run(wl, 36, kernel=fdtd.KERNEL_FUSED, T=T, storage=fmt)
    fo, po, st = G.oracle_q(wl, 36, fmt, T)
    _assert_same(f, fo, "fields")
    _assert_same(p, po, "probes")


@pytest.mark.parametrize("fmt,T", [(W.FP32, 4), (W.FP16, 3), (W.BF16, 3)])
def test_automatic_time_block(fmt, T):
    """Without an explicit T the solver uses the fastest form: 4 steps per
    pass for FP32 storage, 3 for 16-bit storage (the re-quantisation points
    of the 16-bit emulation pin which T ran)."""
    wl = ragged(n_steps=36, storage=fmt)
    s = fdtd.Solver.from_workload(wl)
    try:
        s.step(36)
        f, p = s.read_fields(), s.read_probes(0, 36)
    finally:
        s.close()
    if fmt == W.FP32:
        fo, po = G.oracle_f32(wl, 36)
    else:
        fo, po, _ = G.oracle_q(wl, 36, fmt, T)
    _assert_same(f, fo, "fields")
    _assert_same(p, po, "probes")


@pytest.mark.parametrize("fmt", [W.FP16, W.BF16])
def test_reduced_storage_upload_roundtrip(fmt):
    wl = W.cavity32()
    wl.storage = fmt
    s = fdtd.Solver.from_workload(wl, kernel=fdtd.KERNEL_FUSED, time_block=2)
    try:
        got = s.read_fields()
        scales, sat = s.storage_state()
    finally:
        s.close()
    import oracle
    prob = oracle.Problem.from_workload(wl)
    ref = G.pec_clean(wl, G.init32(wl))
    st = prob.quantize_upload(ref, fmt)
    assert list(st["scales"]) == scales and not sat
    _assert_same(got, ref, "uploaded fields")


def test_step_splitting_and_kernel_variants_identical():
    wl = ragged(n_steps=30)
    ref, pref = G.gpu_run(wl, 30, kernel=fdtd.KERNEL_PLAIN)
    for T, chunks in ((1, [30]), (2, [7, 1, 22]), (3, [30]), (4, [5, 5, 20]), (2, [1] * 30)):
        f, p = G.gpu_run(wl, 30, kernel=fdtd.KERNEL_FUSED, T=T, chunks=chunks)
        _assert_same(f, ref, f"T={T} chunks={chunks}")
        _assert_same(p, pref, f"probes T={T}")


@pytest.mark.parametrize("T", [3, 4])
def test_fp32_blocks_packed_from_the_current_step(T):
    """FP32 storage packs full T-step blocks from wherever a call starts (its
    results do not depend on where blocks fall): after 5 steps, 20 more run
    as ceil(20 / T) launches, not ending at absolute multiples of T, and the
    run at odd offsets stays bit-exact with the oracle."""
    wl = ragged(n_steps=37)
    one = fdtd.Solver.from_workload(wl, kernel=fdtd.KERNEL_FUSED, time_block=T)
    try:
        one.set_zero_skip(False)
        one.step(T)
        full_T = one.tile_stats()[1]          # tiles of one full-block launch
    finally:
        one.close()
    s = fdtd.Solver.from_workload(wl, kernel=fdtd.KERNEL_FUSED, time_block=T)
    try:
        s.set_zero_skip(False)
        s.step(5)
        before = s.tile_stats()[1]
        s.step(4 * T)
        assert s.tile_stats()[1] - before == 4 * full_T      # four full blocks from step 5
        s.step(37 - 5 - 4 * T)
        s.synchronize()
        f, p = s.read_fields(), s.read_probes(0, 37)
    finally:
        s.close()
    fo, po = G.oracle_f32(wl, 37)
    _assert_same(f, fo, f"fields T={T}")
    _assert_same(p, po, f"probes T={T}")


def test_probes_equal_field_reads():
    wl = ragged(n_steps=20)
    s = fdtd.Solver.from_workload(wl, kernel=fdtd.KERNEL_FUSED, time_block=3)
    try:
        for n in range(1, 21):
            s.step(1)
            row = s.read_probes(n - 1, 1)[0]
            for q, (c, i, j, k) in enumerate(wl.probes):
                assert row[q] == float(s.read_field(c)[k, j, i])
    finally:
        s.close()


def test_diagnostics_match_oracle():
    import oracle
    wl = ragged(n_steps=25)
    rng = np.random.default_rng(3)
    init = rng.standard_normal((6, wl.nz + 1, wl.ny + 1, wl.nx + 1)).astype(np.float32)
    s = fdtd.Solver.from_workload(wl, kernel=fdtd.KERNEL_FUSED, time_block=2)
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


def test_lossless_energy_conserved_on_gpu():
    """Energy of a lossless PEC box stays constant over 200 GPU steps (FP32 round-off)."""
    wl = W.spheres(60, 50, 40, 6, 200, seed=9, n_sources=0, n_probes=0, rmin=3, rmax=8)
    wl.sigma[:] = 0.0
    rng = np.random.default_rng(4)
    init = rng.standard_normal((6, wl.nz + 1, wl.ny + 1, wl.nx + 1)).astype(np.float32)
    s = fdtd.Solver.from_workload(wl, kernel=fdtd.KERNEL_FUSED, time_block=4)
    try:
        s.set_fields(init)
        w0 = s.diagnostics()["energy"]
        s.step(200)
        w1 = s.diagnostics()["energy"]
    finally:
        s.close()
    assert abs(w1 - w0) < 1e-5 * w0


@pytest.mark.parametrize("storage,T", [(W.FP32, 1), (W.FP32, 2), (W.FP32, 3), (W.FP32, 4), (W.FP16, 3), (W.BF16, 4)])
def test_poisoned_output_buffers_change_nothing(storage, T):
    """Race check: with every fused launch's output buffer filled with NaN
    first, the results are bit-identical -- each launch rewrites every value
    it owns and reads only its input buffer."""
    wl = ragged(n_steps=22, storage=storage)
    print(f"poison storage={storage} T={T}", flush=True)
    runs = []
    for poison in (False, True):
        s = fdtd.Solver.from_workload(wl, kernel=fdtd.KERNEL_FUSED, time_block=T)
        try:
            s.set_poison(poison)
            s.step(9)
            s.step(13)
            runs.append((s.read_fields(), s.read_probes(0, 22)))
        finally:
            s.close()
    assert np.all(np.isfinite(runs[1][0]))
    _assert_same(runs[1][0], runs[0][0], "fields")
    _assert_same(runs[1][1], runs[0][1], "probes")
