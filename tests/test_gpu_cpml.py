"""GPU parity of CPML absorbing layers: the HIP plain kernels and the fused
kernel (T = 1..3) with layers against the oracle's CPML FP32 operation-order
mode, bit for bit (fields and probes), on uniform and graded grids, split
steps, from zero with the zero-tile skip on and off and with NaN-poisoned
outputs, plain and fused steps interleaved, the 256^3 open-space workload at
full size; and the rules of fdtd_set_cpml."""
import functools

import numpy as np
import pytest

import oracle
from paper_1301_4539_amd import fdtd, workload as W
from tests import gpu_helpers as G

pytestmark = pytest.mark.gpu

LAYER = dict(thickness=6, order=3, sigma_factor=1.0, kappa_max=5.0, alpha_max=0.05)


def open_ragged(n_steps=40, seed=4245, graded=False, layer=LAYER):
    """Spans two 64-point blocks in x with a ragged tail, layers on every face,
    random materials, sources, initial fields (every cell and every psi active
    from the first step), optionally random cell sizes."""
    wl = W.spheres(71, 45, 38, 8, n_steps, seed=seed, n_sources=3, n_probes=16, rmin=3, rmax=9,
                   name="open_ragged")
    rng = np.random.default_rng(seed)
    if graded:
        wl.spacing = tuple(rng.uniform(0.5e-3, 1.5e-3, n) for n in (wl.nx, wl.ny, wl.nz))
        wl.dt = W.courant_dt_graded(*wl.spacing)
    wl.cpml = dict(layer)
    wl.waveforms = rng.standard_normal(wl.waveforms.shape)
    wl.init_fields = rng.standard_normal((6, wl.nz + 1, wl.ny + 1, wl.nx + 1))
    return wl


def _assert_same(a, b, what):
    msg = G.first_mismatch(a, b)
    assert msg is None, f"{what}: {msg}"


@pytest.mark.parametrize("graded", [False, True])
def test_cpml_bitexact(graded):
    wl = open_ragged(graded=graded)
    print(f"cpml 71x45x38 graded={graded}, 40 steps in chunks 7+13+20", flush=True)
    f, p = G.gpu_run(wl, 40, kernel=fdtd.KERNEL_PLAIN, chunks=[7, 13, 20])
    fo, po = G.oracle_f32(wl, 40)
    _assert_same(f, fo, "fields")
    _assert_same(p, po, "probes")
    f64, _ = G.oracle_f64(wl, 40)
    err = W.rel_l2(f, f64)
    print(f"cpml rel-L2 vs FP64 after 40 steps: {err:.3e}")
    assert err <= 1e-5


@pytest.mark.parametrize("graded", [False, True])
@pytest.mark.parametrize("T", [1, 2, 3])
def test_cpml_fused_bitexact(graded, T):
    """The fused kernel with layers (psi carried through the T levels in
    registers) against the oracle, in split calls that end mid-block."""
    wl = open_ragged(graded=graded)
    print(f"cpml fused T={T} 71x45x38 graded={graded}, 40 steps in chunks 7+13+20", flush=True)
    f, p = G.gpu_run(wl, 40, kernel=fdtd.KERNEL_FUSED, T=T, chunks=[7, 13, 20])
    fo, po = G.oracle_f32(wl, 40)
    _assert_same(f, fo, "fields")
    _assert_same(p, po, "probes")


@pytest.mark.parametrize("skip,poison", [(True, False), (False, False), (False, True)])
def test_cpml_fused_from_zero(skip, poison):
    """Source-driven from zero fields: the zero-tile skip leaves out tiles
    whose fields and psi are all +0; with every output buffer (fields and
    psi) NaN-filled before each launch, every owned value is still rewritten."""
    wl = open_ragged(n_steps=60, seed=4248)
    wl.init_fields = None
    print(f"cpml fused T=2 from zero, skip={skip} poison={poison}, 60 steps", flush=True)
    s = fdtd.Solver.from_workload(wl, kernel=fdtd.KERNEL_FUSED, time_block=2)
    try:
        s.set_zero_skip(skip)
        s.set_poison(poison)
        s.step(25)
        s.step(35)
        f, p = s.read_fields(), s.read_probes(0, 60)
    finally:
        s.close()
    fo, po = G.oracle_f32(wl, 60)
    _assert_same(f, fo, "fields")
    _assert_same(p, po, "probes")


def test_cpml_plain_and_fused_interleaved():
    """The plain kernels update psi in place, the fused one reads one copy and
    writes the other: switching between them mid-run keeps the state."""
    wl = open_ragged(n_steps=31, seed=4249, graded=True)
    print("cpml plain 9 + fused T=3 11 + plain 5 + fused T=2 6", flush=True)
    s = fdtd.Solver.from_workload(wl, kernel=fdtd.KERNEL_PLAIN, time_block=1)
    try:
        s.step(9)
        s.set_kernel(fdtd.KERNEL_FUSED, 3)
        s.step(11)
        s.set_kernel(fdtd.KERNEL_PLAIN, 1)
        s.step(5)
        s.set_kernel(fdtd.KERNEL_FUSED, 2)
        s.step(6)
        f, p = s.read_fields(), s.read_probes(0, 31)
    finally:
        s.close()
    fo, po = G.oracle_f32(wl, 31)
    _assert_same(f, fo, "fields")
    _assert_same(p, po, "probes")


def test_cpml_thin_layers_and_automatic_kernel():
    layer = dict(thickness=1, order=2, sigma_factor=0.8, kappa_max=2.0, alpha_max=0.0)
    wl = open_ragged(n_steps=30, seed=4246, layer=layer)
    print("cpml 1-cell layers, automatic kernel, 30 steps", flush=True)
    f, p = G.gpu_run(wl, 30, kernel=fdtd.KERNEL_AUTO, T=0)
    fo, po = G.oracle_f32(wl, 30)
    _assert_same(f, fo, "fields")
    _assert_same(p, po, "probes")


def test_cpml_state_cleared_by_set_fields():
    wl = open_ragged(n_steps=40, seed=4247)
    init = wl.init_fields.astype(np.float32)
    s = fdtd.Solver.from_workload(wl)
    try:
        s.step(20)
        s.set_fields(init)
        s.step(20)
        f = s.read_fields()
    finally:
        s.close()
    # the oracle starts from the same fields with zero psi, at step 20 (the
    # step counter, which indexes the source waveforms, is not reset)
    prob = oracle.Problem.from_workload(wl)
    fo = G.pec_clean(wl, init)
    prob.run_f32(fo, 20, 20)
    _assert_same(f, fo, "fields after set_fields")


@functools.lru_cache(maxsize=1)
def _open256_oracle():
    wl = W.open256(n_steps=100)
    init = np.random.default_rng(257).standard_normal((6, wl.nz + 1, wl.ny + 1, wl.nx + 1), dtype=np.float32)
    fo, po = G.oracle_f32(wl, 100, init=init)
    return wl, init, fo, po


@pytest.mark.parametrize("kernel", [fdtd.KERNEL_AUTO, fdtd.KERNEL_PLAIN])
def test_open256_full_size_bitexact(kernel):
    """The 256^3 open-space workload (10-cell layers) at full size, 100 steps
    from random fields, through the automatic kernel choice (the fused kernel
    at its default T, as the benchmark runs it) and the plain kernels."""
    wl, init, fo, po = _open256_oracle()
    print(f"open256 full size, random initial fields, 100 steps, kernel={kernel}", flush=True)
    f, p = G.gpu_run(wl, 100, kernel=kernel, T=0 if kernel == fdtd.KERNEL_AUTO else 1, init=init)
    _assert_same(f, fo, "fields")
    _assert_same(p, po, "probes")


def test_set_cpml_rules():
    wl = W.spheres(20, 16, 12, 2, 10, seed=5, n_sources=1, n_probes=2, rmin=2, rmax=4, name="e")
    s = fdtd.Solver.from_workload(wl)
    try:
        for bad in [dict(thickness=6), dict(thickness=2, order=0), dict(thickness=2, kappa_max=0.5)]:
            with pytest.raises(fdtd.FdtdError) as e:
                s.set_cpml(**bad)
            assert e.value.code == fdtd.EINVAL
        s.set_kernel(fdtd.KERNEL_FUSED, 4)
        with pytest.raises(fdtd.FdtdError) as e:     # layers run fused blocks of at most 3 steps
            s.set_cpml(3)
        assert e.value.code == fdtd.EINVAL
        s.set_kernel(fdtd.KERNEL_AUTO, 0)
        assert s.time_block == 4
        s.set_cpml(3)
        assert s.time_block == 2                     # the automatic T with layers
        with pytest.raises(fdtd.FdtdError) as e:
            s.set_kernel(fdtd.KERNEL_FUSED, 4)
        assert e.value.code == fdtd.EINVAL
        s.set_kernel(fdtd.KERNEL_PLAIN, 0)
        assert s.time_block == 1
        s.set_kernel(fdtd.KERNEL_FUSED, 2)
        assert s.time_block == 2
        for call in (lambda: s.diagnostics(), lambda: fdtd.step_batch([s], [2])):
            with pytest.raises(fdtd.FdtdError) as e:
                call()
            assert e.value.code == fdtd.EINVAL
        s.step(2)
        with pytest.raises(fdtd.FdtdError) as e:
            s.set_cpml(2)
        assert e.value.code == fdtd.ESTATE
    finally:
        s.close()
    s16 = fdtd.Solver.from_workload(wl, storage=W.FP16)
    try:
        with pytest.raises(fdtd.FdtdError) as e:
            s16.set_cpml(3)
        assert e.value.code == fdtd.EINVAL
    finally:
        s16.close()
