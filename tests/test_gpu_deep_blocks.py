"""GPU parity of the deeper time blocks, T = 5 and 6 steps per HBM pass (the
step gathering the paper's conclusion proposes beyond its two steps): FP32
storage bit for bit with the oracle's FP32 operation-order mode at every
tile shape, split steps and zero-tile skipping; FP16/BF16 storage bit for
bit with the oracle's emulation at the same T; and the rules that keep
batches and graded spacing at T <= 4."""
import numpy as np
import pytest

import oracle
from paper_1301_4539_amd import fdtd, workload as W
from tests import gpu_helpers as G

pytestmark = pytest.mark.gpu

DEEP = [5, 6]


def ragged(n_steps=40, storage=W.FP32, seed=4242):
    wl = W.spheres(131, 75, 50, 12, n_steps, seed=seed, n_sources=3, n_probes=16, rmin=3, rmax=12,
                   name="ragged", storage=storage)
    wl.waveforms = np.random.default_rng(17).standard_normal(wl.waveforms.shape)
    return wl


def _assert_same(a, b, what):
    msg = G.first_mismatch(a, b)
    assert msg is None, f"{what}: {msg}"


@pytest.mark.parametrize("T", DEEP)
def test_cavity32_deep_bitexact(T):
    wl = W.cavity32()
    print(f"cavity32 fused T={T}, 100 steps", flush=True)
    f, p = G.gpu_run(wl, 100, kernel=fdtd.KERNEL_FUSED, T=T)
    fo, po = G.oracle_f32(wl, 100)
    _assert_same(f, fo, "fields")
    _assert_same(p, po, "probes")


@pytest.mark.parametrize("T", DEEP)
@pytest.mark.parametrize("variant", [1, 2, 3])
def test_ragged_deep_every_shape_bitexact(T, variant):
    """Every tile shape, with z chunks of 9 planes (several chunks and a
    ragged last one) and steps split so that partial blocks run too."""
    wl = ragged(n_steps=40)
    fo, po = G.oracle_f32(wl, 40)
    print(f"ragged fused T={T} variant={variant}, 40 steps in 7+20+13", flush=True)
    s = fdtd.Solver.from_workload(wl, kernel=fdtd.KERNEL_FUSED, time_block=T)
    try:
        s.set_tiling(variant, 9 if variant == 1 else 0)
        for n in (7, 20, 13):
            s.step(n)
        f = s.read_fields()
        p = s.read_probes(0, 40)
    finally:
        s.close()
    _assert_same(f, fo, "fields")
    _assert_same(p, po, "probes")
    assert np.max(np.abs(fo[0:3])) > 0.1


@pytest.mark.parametrize("T", DEEP)
def test_deep_random_state_and_zero_skip(T):
    """From a random state (every tile active) and from zero fields with the
    zero-tile skip on and off: all equal the oracle."""
    wl = ragged(n_steps=30, seed=4301)
    init = np.random.default_rng(T).standard_normal((6, wl.nz + 1, wl.ny + 1, wl.nx + 1)).astype(np.float32)
    print(f"random state T={T}", flush=True)
    f, p = G.gpu_run(wl, 30, kernel=fdtd.KERNEL_FUSED, T=T, init=init)
    fo, po = G.oracle_f32(wl, 30, init=init)
    _assert_same(f, fo, "fields (random state)")
    _assert_same(p, po, "probes (random state)")
    fo, po = G.oracle_f32(wl, 30)
    for skip in (True, False):
        print(f"zero fields T={T} skip={skip}", flush=True)
        s = fdtd.Solver.from_workload(wl, kernel=fdtd.KERNEL_FUSED, time_block=T)
        try:
            s.set_zero_skip(skip)
            s.step(30)
            f = s.read_fields()
            p = s.read_probes(0, 30)
        finally:
            s.close()
        _assert_same(f, fo, f"fields skip={skip}")
        _assert_same(p, po, f"probes skip={skip}")


@pytest.mark.parametrize("fmt", [W.FP16, W.BF16])
@pytest.mark.parametrize("T", DEEP)
def test_deep_reduced_storage_bitexact_with_emulation(fmt, T):
    wl = ragged(n_steps=36, storage=fmt)
    print(f"reduced storage fmt={fmt} T={T}, 36 steps in 13+23", flush=True)
    f, p = G.gpu_run(wl, 36, kernel=fdtd.KERNEL_FUSED, T=T, storage=fmt, chunks=[13, 23])
    # blocks end at multiples of T and where a step call ends (the stored
    # state is re-encoded there): the emulation runs the same two calls
    prob = oracle.Problem.from_workload(wl)
    fo = G.pec_clean(wl, G.init32(wl))
    st = prob.quantize_upload(fo, fmt)
    po = np.concatenate([prob.run_q(fo, 0, 13, fmt, T, st), prob.run_q(fo, 13, 23, fmt, T, st)])
    _assert_same(f, fo, "fields")
    _assert_same(p, po, "probes")


@pytest.mark.parametrize("storage,T", [(W.FP32, 6), (W.FP16, 5)])
def test_deep_poisoned_output_buffers_change_nothing(storage, T):
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


def test_spheres256_full_size_deep_bitexact():
    """The benchmarked 256^3 dielectric grid at full size with T = 6 and its
    automatic shape and z chunks, from a random state, 24 steps."""
    wl = W.spheres256(n_steps=24)
    init = np.random.default_rng(2566).standard_normal((6, wl.nz + 1, wl.ny + 1, wl.nx + 1)).astype(np.float32)
    print("spheres256 full size, T=6, 24 steps", flush=True)
    f, p = G.gpu_run(wl, 24, kernel=fdtd.KERNEL_FUSED, T=6, init=init)
    fo, po = G.oracle_f32(wl, 24, init=init)
    _assert_same(f, fo, "fields")
    _assert_same(p, po, "probes")


def test_deep_block_rules():
    wl = W.spheres(20, 16, 12, 2, 10, seed=5, n_sources=1, n_probes=2, rmin=2, rmax=4, name="e")
    s = fdtd.Solver.from_workload(wl)
    try:
        with pytest.raises(fdtd.FdtdError) as e:
            s.set_kernel(fdtd.KERNEL_FUSED, 7)
        assert e.value.code == fdtd.EINVAL
        s.set_kernel(fdtd.KERNEL_FUSED, 5)
        with pytest.raises(fdtd.FdtdError) as e:      # batches run blocks of at most 4 steps
            fdtd.step_batch([s], [5])
        assert e.value.code == fdtd.EINVAL
        sizes = [np.full(n, 1e-3) for n in (wl.nx, wl.ny, wl.nz)]
        with pytest.raises(fdtd.FdtdError) as e:      # graded spacing too
            s.set_spacing(*sizes)
        assert e.value.code == fdtd.EINVAL
        s.set_kernel(fdtd.KERNEL_AUTO, 0)             # the automatic T takes graded sizes
        s.set_spacing(*sizes)
        with pytest.raises(fdtd.FdtdError) as e:
            s.set_kernel(fdtd.KERNEL_FUSED, 6)
        assert e.value.code == fdtd.EINVAL
        s.step(3)
        s.synchronize()
    finally:
        s.close()
